// Integer box algebra on a periodic index space (host only, internal).
#pragma once
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

struct IBox {
  int lo[3], hi[3];  // inclusive
  int size(int d) const { return hi[d] - lo[d] + 1; }
  bool empty() const { return hi[0] < lo[0] || hi[1] < lo[1] || hi[2] < lo[2]; }
  long long volume() const { return empty() ? 0 : (long long)size(0) * size(1) * size(2); }
};

inline IBox isect(const IBox& a, const IBox& b) {
  IBox r;
  for (int d = 0; d < 3; ++d) {
    r.lo[d] = std::max(a.lo[d], b.lo[d]);
    r.hi[d] = std::min(a.hi[d], b.hi[d]);
  }
  return r;
}

inline IBox grow(const IBox& a, int g) {
  IBox r = a;
  for (int d = 0; d < 3; ++d) {
    r.lo[d] -= g;
    r.hi[d] += g;
  }
  return r;
}

inline IBox shift(const IBox& a, int sx, int sy, int sz) {
  IBox r = a;
  const int s[3] = {sx, sy, sz};
  for (int d = 0; d < 3; ++d) {
    r.lo[d] += s[d];
    r.hi[d] += s[d];
  }
  return r;
}

// floor division by 2 (arithmetic shift), for cells one outside the domain too
inline IBox coarsen(const IBox& a) {
  IBox r;
  for (int d = 0; d < 3; ++d) {
    r.lo[d] = a.lo[d] >> 1;
    r.hi[d] = a.hi[d] >> 1;
  }
  return r;
}

inline IBox refine(const IBox& a) {
  IBox r;
  for (int d = 0; d < 3; ++d) {
    r.lo[d] = 2 * a.lo[d];
    r.hi[d] = 2 * a.hi[d] + 1;
  }
  return r;
}

// a \ b as disjoint boxes appended to out
inline void subtract(const IBox& a, const IBox& b, std::vector<IBox>& out) {
  const IBox i = isect(a, b);
  if (i.empty()) {
    out.push_back(a);
    return;
  }
  IBox r = a;
  for (int d = 0; d < 3; ++d) {
    if (r.lo[d] < i.lo[d]) {
      IBox p = r;
      p.hi[d] = i.lo[d] - 1;
      out.push_back(p);
      r.lo[d] = i.lo[d];
    }
    if (r.hi[d] > i.hi[d]) {
      IBox p = r;
      p.lo[d] = i.hi[d] + 1;
      out.push_back(p);
      r.hi[d] = i.hi[d];
    }
  }
}

// Visit marks of BoxBins::query, one set per thread (queries of one or several bins may
// run on several threads at once; every query takes a fresh mark).
struct BinStamps {
  std::vector<int> stamp;
  int cur = 0;
};
inline BinStamps& bin_stamps() {
  thread_local BinStamps s;
  return s;
}

// Uniform bins over [0, M)^3 listing the boxes that overlap each bin.
struct BoxBins {
  int M = 0, B = 32, nb = 0, nbox = 0;
  std::vector<std::vector<int>> bins;

  void build(const std::vector<IBox>& boxes, int M_) {
    M = M_;
    B = std::max(8, std::min(64, M));
    nb = (M + B - 1) / B;
    bins.assign((size_t)nb * nb * nb, {});
    nbox = (int)boxes.size();
    for (int i = 0; i < (int)boxes.size(); ++i) {
      const IBox& b = boxes[i];
      for (int z = b.lo[2] / B; z <= b.hi[2] / B; ++z)
        for (int y = b.lo[1] / B; y <= b.hi[1] / B; ++y)
          for (int x = b.lo[0] / B; x <= b.hi[0] / B; ++x) bins[((size_t)z * nb + y) * nb + x].push_back(i);
    }
  }

  // f(box) once for every box whose bins overlap q (q clipped to [0, M)^3)
  template <class F>
  void query(const IBox& q0, F f) const {
    IBox q = q0;
    for (int d = 0; d < 3; ++d) {
      q.lo[d] = std::max(q.lo[d], 0);
      q.hi[d] = std::min(q.hi[d], M - 1);
    }
    if (q.empty() || nb == 0) return;
    BinStamps& st = bin_stamps();
    if ((int)st.stamp.size() < nbox) st.stamp.resize(nbox, 0);
    if (++st.cur == 0x7fffffff) {
      std::fill(st.stamp.begin(), st.stamp.end(), 0);
      st.cur = 1;
    }
    const int mark = st.cur;
    int* stamp = st.stamp.data();
    for (int z = q.lo[2] / B; z <= q.hi[2] / B; ++z)
      for (int y = q.lo[1] / B; y <= q.hi[1] / B; ++y)
        for (int x = q.lo[0] / B; x <= q.hi[0] / B; ++x)
          for (int i : bins[((size_t)z * nb + y) * nb + x])
            if (stamp[i] != mark) {
              stamp[i] = mark;
              f(i);
            }
  }
};

// f(box, shift[3]) for every periodic image box + shift*M (shift in {-1,0,1}^3) that
// may overlap q, which may reach up to M cells outside [0, M)^3.
// Only shifts whose image of the domain meets q are visited.
template <class F>
inline void for_images(const IBox& q, int M, const BoxBins& bins, F f) {
  int s0[3], s1[3];
  for (int d = 0; d < 3; ++d) {
    s0[d] = q.lo[d] < 0 ? -1 : (q.lo[d] < M ? 0 : 1);
    s1[d] = q.hi[d] >= M ? 1 : (q.hi[d] >= 0 ? 0 : -1);
  }
  for (int sz = s0[2]; sz <= s1[2]; ++sz)
    for (int sy = s0[1]; sy <= s1[1]; ++sy)
      for (int sx = s0[0]; sx <= s1[0]; ++sx) {
        const int sh[3] = {sx, sy, sz};
        const IBox qs = shift(q, -sx * M, -sy * M, -sz * M);
        bins.query(qs, [&](int b) { f(b, sh); });
      }
}

inline long long covered_volume(const IBox& q, int M, const BoxBins& bins, const std::vector<IBox>& boxes) {
  long long v = 0;
  for_images(q, M, bins, [&](int b, const int sh[3]) {
    v += isect(q, shift(boxes[b], sh[0] * M, sh[1] * M, sh[2] * M)).volume();
  });
  return v;
}

// Berger-Rigoutsos clustering of the tags of a level into boxes of the next level
// (implemented in cluster.cpp).  `carried` (ncarried cells of the level above, index
// space 2M) adds the blocks met by their coarse parents grown by carry_grow + nbuf cells.
bool cluster_level(int M, const std::vector<IBox>& level_boxes, bool full_level, int bf, int max_box, int nbuf,
                   double efficiency, const int32_t* tags, long long ntag, std::vector<IBox>& out, std::string& err,
                   const int32_t* carried = nullptr, long long ncarried = 0, int carry_grow = 0);

// Bitsets of tagged blocks (bf/2 cells; bit x + nb (y + nb z); block_words(M, bf) 64-bit
// words for a level of M cells per axis, nb = M / (bf/2)):
long long block_words(int M, int bf);
// the same clustering from such a bitset;
bool cluster_bits(int M, const std::vector<IBox>& level_boxes, bool full_level, int bf, int max_box,
                  double efficiency, const uint64_t* bits, long long nwords, std::vector<IBox>& out,
                  std::string& err);
// OR into it the blocks met by cells grown by r (the cells' parents, from a level of 2M
// cells, when halve);
bool mark_list_blocks(int M, int bf, int r, bool halve, const int32_t* cells, long long n, uint64_t* bits,
                      long long nwords, std::string& err);
// OR into it eight octant bitsets (the same size, one after the other), each grown by one
// block towards its octant: bit 0 of the octant index +x (else -x), bit 1 +y, bit 2 +z.
bool dilate_octants(int M, int bf, const uint64_t* oct, uint64_t* bits, long long nwords, std::string& err);

// Local regrid (implemented in local_regrid.cpp), on the block grid of the finer level
// (blocks of bf cells).  local_tag_boxes: boxes to add to level l+1 (fine index, M_fine
// cells per axis) so that every tagged level-l cell with its n_error_buf buffer is
// refined, given the level's current boxes.  local_nest_boxes: boxes to add to level k
// (M_k cells per axis) so that the added level-(k+1) boxes keep a nesting gap of bf/2
// level-k cells.  Added blocks are merged into x runs of at most max_box cells, listed in
// (z, y, x) block order.
bool local_tag_boxes(int M_fine, const std::vector<IBox>& fine_boxes, int bf, int nbuf, int max_box,
                     const int32_t* tags, long long ntag, std::vector<IBox>& out, std::string& err);
bool local_nest_boxes(int M_k, const std::vector<IBox>& added_fine, const std::vector<IBox>& level_boxes, int bf,
                      int max_box, std::vector<IBox>& out, std::string& err);
