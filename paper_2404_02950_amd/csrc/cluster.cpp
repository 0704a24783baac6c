// Host clustering of tagged cells into the boxes of the next level (global regrid).
//
// Berger & Rigoutsos, "An algorithm for point clustering and grid generation", IEEE
// Trans. Systems, Man and Cybernetics 21 (1991): take the bounding box of the tagged
// points; accept it if the fraction of tagged points reaches the efficiency threshold;
// otherwise cut it at a hole of a signature (tag counts per slice), else at the
// strongest sign change of the signature's second difference, else in the middle of
// its longest side, and recurse on the two halves.
//
// Clustering runs on blocks of bf/2 cells of the tagged level (one fine blocking
// factor after refinement), so every produced box is blocking-factor aligned.  Tags are
// first grown by n_error_buf cells (periodically).  Blocks whose one-block neighbourhood
// is not inside the tagged level are dropped and may not lie inside an accepted box (a
// box holding one is cut further), which keeps the new level properly nested with a gap
// of one fine blocking factor.
//
// The recursion works on the list of tagged blocks (partitioned in place at each cut),
// so its cost follows the number of tagged blocks, not the size of the domain; the only
// whole-domain structures are two bitsets of one bit per block.
#include <stdint.h>

#include <algorithm>
#include <cstdlib>
#include <string>
#include <vector>

#include "sh_geom.h"

namespace {

struct Bits {
  int n = 0;
  std::vector<uint64_t> w;
  void init(int n_) {
    n = n_;
    w.assign(((size_t)n * n * n + 63) / 64, 0);
  }
  static size_t key(int n, int x, int y, int z) { return ((size_t)z * n + y) * n + x; }
  void set(int x, int y, int z) {
    const size_t k = key(n, x, y, z);
    w[k >> 6] |= 1ull << (k & 63);
  }
  bool get(int x, int y, int z) const {
    const size_t k = key(n, x, y, z);
    return (w[k >> 6] >> (k & 63)) & 1;
  }
  // bits k0..k1 (inclusive)
  void set_range(size_t k0, size_t k1) {
    const size_t w0 = k0 >> 6, w1 = k1 >> 6;
    const uint64_t m0 = ~0ull << (k0 & 63), m1 = ~0ull >> (63 - (k1 & 63));
    if (w0 == w1) {
      w[w0] |= m0 & m1;
      return;
    }
    w[w0] |= m0;
    for (size_t i = w0 + 1; i < w1; ++i) w[i] = ~0ull;
    w[w1] |= m1;
  }
  // x = lo..hi (periodic, fewer than n cells) of row (y, z)
  void set_x(int lo, int hi, int y, int z) {
    const size_t row = key(n, 0, y, z);
    if (lo >= 0 && hi < n) {
      set_range(row + lo, row + hi);
      return;
    }
    const int a = ((lo % n) + n) % n, b = ((hi % n) + n) % n;
    if (a <= b) {
      set_range(row + a, row + b);
    } else {
      set_range(row + a, row + n - 1);
      set_range(row, row + b);
    }
  }
};

int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
// periodic index (no division for indices within one period of [0, n))
int wrap(int a, int n) {
  if (a >= 0 && a < n) return a;
  if (a >= -n && a < 2 * n) return a < 0 ? a + n : a - n;
  return ((a % n) + n) % n;
}

struct Pt {
  int c[3];
};

struct Ctx {
  std::vector<Pt> pts;
  const Bits* cov = nullptr;  // blocks inside the tagged level (null: the whole domain)
  double eff = 0.7;
  std::vector<IBox> out;
  std::vector<long long> sig[3];
  std::vector<long long> lap;  // second differences of a signature (reused)
  std::vector<Pt> tmp;         // upper part during a cut (reused)
};

IBox bounding(const Pt* p, long long n) {
  IBox b;
  for (int d = 0; d < 3; ++d) {
    b.lo[d] = p[0].c[d];
    b.hi[d] = p[0].c[d];
  }
  for (long long i = 1; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      b.lo[d] = std::min(b.lo[d], p[i].c[d]);
      b.hi[d] = std::max(b.hi[d], p[i].c[d]);
    }
  return b;
}

// every block of the box has its one-block neighbourhood inside the level
bool clean(const Bits& cov, const IBox& b) {
  const int n = cov.n;
  for (int z = b.lo[2] - 1; z <= b.hi[2] + 1; ++z)
    for (int y = b.lo[1] - 1; y <= b.hi[1] + 1; ++y)
      for (int x = b.lo[0] - 1; x <= b.hi[0] + 1; ++x)
        if (!cov.get(wrap(x, n), wrap(y, n), wrap(z, n))) return false;
  return true;
}

void br(Ctx& C, long long first, long long count) {
  if (count == 0) return;
  Pt* p = C.pts.data() + first;
  const IBox box = bounding(p, count);
  const long long vol = box.volume();
  if (vol == 1 || ((double)count >= C.eff * (double)vol && (!C.cov || clean(*C.cov, box)))) {
    C.out.push_back(box);
    return;
  }
  // signatures: tagged blocks per slice along each direction
  for (int d = 0; d < 3; ++d) C.sig[d].assign(box.size(d), 0);
  for (long long i = 0; i < count; ++i)
    for (int d = 0; d < 3; ++d) ++C.sig[d][p[i].c[d] - box.lo[d]];
  int best_d = -1, best_cut = 0;
  // 1) a hole in a signature, the one nearest the middle of its side
  double best_dist = 1e30;
  for (int d = 0; d < 3; ++d) {
    const double mid = 0.5 * (box.lo[d] + box.hi[d]);
    for (int i = box.lo[d] + 1; i < box.hi[d]; ++i)
      if (C.sig[d][i - box.lo[d]] == 0 && std::abs(i - mid) < best_dist) {
        best_dist = std::abs(i - mid);
        best_d = d;
        best_cut = i;
      }
  }
  // 2) the strongest inflection of a signature (sign change of its second difference)
  if (best_d < 0) {
    long long best_jump = 0;
    for (int d = 0; d < 3; ++d) {
      const int len = box.size(d);
      if (len < 4) continue;
      const std::vector<long long>& sig = C.sig[d];
      std::vector<long long>& lap = C.lap;
      lap.assign(len, 0);
      for (int i = 1; i + 1 < len; ++i) lap[i] = sig[i - 1] - 2 * sig[i] + sig[i + 1];
      const double mid = 0.5 * (len - 1);
      for (int i = 1; i + 2 < len; ++i) {
        if ((lap[i] < 0 && lap[i + 1] > 0) || (lap[i] > 0 && lap[i + 1] < 0)) {
          const long long jump = std::llabs(lap[i + 1] - lap[i]);
          if (jump > best_jump || (jump == best_jump && best_d >= 0 && std::abs(i - mid) < best_dist)) {
            best_jump = jump;
            best_dist = std::abs(i - mid);
            best_d = d;
            best_cut = box.lo[d] + i + 1;  // first slice of the upper part
          }
        }
      }
    }
  }
  // 3) bisect the longest side
  if (best_d < 0) {
    best_d = 0;
    for (int d = 1; d < 3; ++d)
      if (box.size(d) > box.size(best_d)) best_d = d;
    best_cut = box.lo[best_d] + box.size(best_d) / 2;
  }
  const int d = best_d, cut = best_cut;
  // stable partition: the lower part in place, the upper part through C.tmp
  long long nlo = 0;
  C.tmp.clear();
  for (long long i = 0; i < count; ++i) {
    if (p[i].c[d] < cut) p[nlo++] = p[i];
    else C.tmp.push_back(p[i]);
  }
  std::copy(C.tmp.begin(), C.tmp.end(), p + nlo);
  br(C, first, nlo);
  br(C, first + nlo, count - nlo);
}

}  // namespace

// Marks the blocks met by the cubes [c - r, c + r] (periodic) around the cells c of a
// list; with `halve`, c is the coarse parent (x / 2) of each listed finer-level cell.
// Neighbouring entries (lists come in row order) mostly need the same blocks: entries
// with the same y and z block ranges whose x block ranges overlap or touch are merged
// into one range before anything is marked.
template <bool POW2>
static bool mark_blocks_t(Bits& tagged, int M, int b, int r, bool halve, const int32_t* cells, long long n,
                          std::string& err) {
  const int nb = M / b;
  const int lim = halve ? 2 * M : M;
  int sh = 0;
  while ((1 << sh) < b) ++sh;
  // floor division by the block size (an arithmetic shift rounds down for negative values)
  auto fdiv = [&](int a) { return POW2 ? (a >> sh) : floordiv(a, b); };
  int plo[3] = {1, 1, 1}, phi[3] = {0, 0, 0};   // pending ranges (none while plo > phi)
  auto flush = [&]() {
    if (plo[0] > phi[0]) return;
    if (phi[0] - plo[0] >= nb) {
      plo[0] = 0;
      phi[0] = nb - 1;
    }
    for (int z = plo[2]; z <= phi[2]; ++z)
      for (int y = plo[1]; y <= phi[1]; ++y) tagged.set_x(plo[0], phi[0], wrap(y, nb), wrap(z, nb));
  };
  for (long long t = 0; t < n; ++t) {
    int c[3], lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      c[d] = cells[3 * t + d];
      if (c[d] < 0 || c[d] >= lim) {
        err = halve ? "carried tag outside the finer level" : "tag outside the level";
        return false;
      }
      if (halve) c[d] >>= 1;
      lo[d] = fdiv(c[d] - r);
      hi[d] = fdiv(c[d] + r);
      if (hi[d] - lo[d] >= nb) {
        lo[d] = 0;
        hi[d] = nb - 1;
      }
    }
    if (lo[1] == plo[1] && lo[2] == plo[2] && hi[1] == phi[1] && hi[2] == phi[2] && lo[0] <= phi[0] + 1 &&
        hi[0] >= plo[0] - 1) {
      plo[0] = std::min(plo[0], lo[0]);
      phi[0] = std::max(phi[0], hi[0]);
      continue;
    }
    flush();
    for (int d = 0; d < 3; ++d) {
      plo[d] = lo[d];
      phi[d] = hi[d];
    }
  }
  flush();
  return true;
}

// ORs into `tagged` every octant bitset grown by one block towards its octant along x
// (bit 0 of the octant index: +x, else -x), y (bit 1) and z (bit 2), periodically.  On
// rows of whole words by word shifts and row / plane copies; otherwise set bit by set
// bit (small levels).
static void dilate_into(Bits& tagged, const Bits* oct) {
  const int nb = tagged.n;
  if (nb % 64) {
    for (int o = 0; o < 8; ++o) {
      const int dx = (o & 1) ? 1 : -1, dy = (o & 2) ? 1 : -1, dz = (o & 4) ? 1 : -1;
      const std::vector<uint64_t>& w = oct[o].w;
      for (size_t wi = 0; wi < w.size(); ++wi)
        for (uint64_t word = w[wi]; word; word &= word - 1) {
          const size_t k = (wi << 6) + __builtin_ctzll(word);
          const int x = (int)(k % nb), y = (int)((k / nb) % nb), z = (int)(k / ((size_t)nb * nb));
          for (int sz = 0; sz < 2; ++sz)
            for (int sy = 0; sy < 2; ++sy)
              for (int sx = 0; sx < 2; ++sx)
                tagged.set(wrap(x + sx * dx, nb), wrap(y + sy * dy, nb), wrap(z + sz * dz, nb));
        }
    }
    return;
  }
  const int W = nb / 64;
  const size_t nw = oct[0].w.size(), row = W, plane = (size_t)nb * W;
  std::vector<uint64_t> a(nw), c(nw);
  for (int o = 0; o < 8; ++o) {
    const std::vector<uint64_t>& s = oct[o].w;
    // x: each row of W words, shifted by one block up (o & 1) or down, with wrap
    for (size_t r0 = 0; r0 < nw; r0 += row)
      for (int k = 0; k < W; ++k) {
        const uint64_t v = s[r0 + k];
        uint64_t sh1;
        if (o & 1) sh1 = (v << 1) | (s[r0 + (k + W - 1) % W] >> 63);
        else sh1 = (v >> 1) | (s[r0 + (k + 1) % W] << 63);
        a[r0 + k] = v | sh1;
      }
    // y: whole rows, from row y to row y +- 1 of the same plane
    for (size_t p0 = 0; p0 < nw; p0 += plane)
      for (int yy = 0; yy < nb; ++yy) {
        const int src = (o & 2) ? (yy + nb - 1) % nb : (yy + 1) % nb;
        for (int k = 0; k < W; ++k) c[p0 + (size_t)yy * W + k] = a[p0 + (size_t)yy * W + k] | a[p0 + (size_t)src * W + k];
      }
    // z: whole planes, then into the tagged blocks
    for (int zz = 0; zz < nb; ++zz) {
      const int src = (o & 4) ? (zz + nb - 1) % nb : (zz + 1) % nb;
      const size_t d0 = (size_t)zz * plane, s0 = (size_t)src * plane;
      for (size_t k = 0; k < plane; ++k) tagged.w[d0 + k] |= c[d0 + k] | c[s0 + k];
    }
  }
}

// The level's own tags when 2r equals the block size b (the usual n_error_buf = 2 with
// a blocking factor of 8): every axis then meets exactly two blocks, the tag's block B and
// B + 1 when its offset in the block is >= r, else B - 1 and B.  One bit per tag goes into
// the bitset of its octant (the direction of the second block along each axis), each
// octant bitset is grown by one block towards its octant along x, y and z (periodically)
// and ORed into the tagged blocks: the same set as marking each tag's 2 x 2 x 2 blocks,
// at one bit write per tag.  Used for long lists on rows of whole words.
static bool mark_octants(Bits& tagged, int M, int b, int sh, const int32_t* cells, long long n, std::string& err) {
  const int nb = M / b, r = b / 2;
  thread_local Bits oct[8];
  for (Bits& o : oct) o.init(nb);
  for (long long t = 0; t < n; ++t) {
    const int x = cells[3 * t], y = cells[3 * t + 1], z = cells[3 * t + 2];
    if (x < 0 || x >= M || y < 0 || y >= M || z < 0 || z >= M) {
      err = "tag outside the level";
      return false;
    }
    const int o = ((x & (b - 1)) >= r ? 1 : 0) | ((y & (b - 1)) >= r ? 2 : 0) | ((z & (b - 1)) >= r ? 4 : 0);
    oct[o].set(x >> sh, y >> sh, z >> sh);
  }
  dilate_into(tagged, oct);
  return true;
}

static bool mark_blocks(Bits& tagged, int M, int b, int r, bool halve, const int32_t* cells, long long n,
                        std::string& err) {
  const bool pow2 = (b & (b - 1)) == 0;
  const int nb = M / b;
  // the dense form costs a few passes over eight block bitsets: worth it for the level's
  // own tags from about one tag per 32 blocks on (4.6 M tags: 56 -> 40 ms).  Carried
  // lists stay one by one: neighbouring fine tags share parents, which the run merging
  // absorbs, while a carried tag (parent grown by 3) would set up to eight octant bits
  // (4.6 M: 62 ms one by one, 161 ms dense).  SHAMR_DENSE_MARKING=0 in the environment
  // turns the dense form off, for comparing the two.
  const char* env = std::getenv("SHAMR_DENSE_MARKING");
  const bool dense_ok = !(env && env[0] == '0');
  if (dense_ok && !halve && pow2 && 2 * r == b && nb % 64 == 0 && n >= (long long)nb * nb * nb / 32) {
    int sh = 0;
    while ((1 << sh) < b) ++sh;
    return mark_octants(tagged, M, b, sh, cells, n, err);
  }
  return pow2 ? mark_blocks_t<true>(tagged, M, b, r, halve, cells, n, err)
              : mark_blocks_t<false>(tagged, M, b, r, halve, cells, n, err);
}

static bool check_level_args(int M, const std::vector<IBox>& level_boxes, int bf, std::string& err) {
  if (bf < 2 || (bf & 1)) {
    err = "blocking factor must be even";
    return false;
  }
  if (M % (bf / 2)) {
    err = "level size not a multiple of half the blocking factor";
    return false;
  }
  for (const IBox& L : level_boxes)
    for (int d = 0; d < 3; ++d)
      if (L.lo[d] < 0 || L.hi[d] >= M || L.lo[d] > L.hi[d]) {
        err = "level box outside the level";
        return false;
      }
  return true;
}

static bool cluster_core(int M, const std::vector<IBox>& level_boxes, bool full_level, int bf, int max_box,
                         double efficiency, const Bits& tagged, std::vector<IBox>& out);

// the bitsets keep their storage between calls on a thread (fresh allocations of a few MB
// would be page-faulted in on every regrid)
static thread_local Bits g_tagged;

bool cluster_level(int M, const std::vector<IBox>& level_boxes, bool full_level, int bf, int max_box, int nbuf,
                   double efficiency, const int32_t* tags, long long ntag, std::vector<IBox>& out, std::string& err,
                   const int32_t* carried, long long ncarried, int carry_grow) {
  out.clear();
  if (!check_level_args(M, level_boxes, bf, err)) return false;
  const int b = bf / 2;
  Bits& tagged = g_tagged;
  tagged.init(M / b);
  if (!mark_blocks(tagged, M, b, nbuf, false, tags, ntag, err)) return false;
  // tags of the next finer level: their coarse parents grown by carry_grow + nbuf cells
  if (ncarried > 0 && !mark_blocks(tagged, M, b, carry_grow + nbuf, true, carried, ncarried, err)) return false;
  return cluster_core(M, level_boxes, full_level, bf, max_box, efficiency, tagged, out);
}

long long block_words(int M, int bf) {
  const long long nb = M / (bf / 2);
  return (nb * nb * nb + 63) / 64;
}

// A caller's block bitset (x fastest) as the working bitset `t` of a level of M cells.
static bool load_bits(Bits& t, int M, int bf, const uint64_t* bits, long long nwords, std::string& err) {
  if (bf < 2 || (bf & 1) || M % (bf / 2)) {
    err = "bad blocking factor or level size";
    return false;
  }
  if (nwords != block_words(M, bf)) {
    err = "block bitset of the wrong size";
    return false;
  }
  t.init(M / (bf / 2));
  std::copy(bits, bits + nwords, t.w.begin());
  // bits past the last block (in a partial last word) are not blocks
  const long long nblk = (long long)t.n * t.n * t.n;
  if (nblk % 64) t.w.back() &= (1ull << (nblk % 64)) - 1;
  return true;
}

bool cluster_bits(int M, const std::vector<IBox>& level_boxes, bool full_level, int bf, int max_box,
                  double efficiency, const uint64_t* bits, long long nwords, std::vector<IBox>& out,
                  std::string& err) {
  out.clear();
  if (!check_level_args(M, level_boxes, bf, err) || !load_bits(g_tagged, M, bf, bits, nwords, err)) return false;
  return cluster_core(M, level_boxes, full_level, bf, max_box, efficiency, g_tagged, out);
}

bool mark_list_blocks(int M, int bf, int r, bool halve, const int32_t* cells, long long n, uint64_t* bits,
                      long long nwords, std::string& err) {
  thread_local Bits t;
  if (r < 0 || !load_bits(t, M, bf, bits, nwords, err)) return false;
  if (!mark_blocks(t, M, bf / 2, r, halve, cells, n, err)) return false;
  std::copy(t.w.begin(), t.w.end(), bits);
  return true;
}

bool dilate_octants(int M, int bf, const uint64_t* oct, uint64_t* bits, long long nwords, std::string& err) {
  thread_local Bits t, o8[8];
  if (!load_bits(t, M, bf, bits, nwords, err)) return false;
  for (int o = 0; o < 8; ++o)
    if (!load_bits(o8[o], M, bf, oct + (size_t)o * nwords, nwords, err)) return false;
  dilate_into(t, o8);
  std::copy(t.w.begin(), t.w.end(), bits);
  return true;
}

static bool cluster_core(int M, const std::vector<IBox>& level_boxes, bool full_level, int bf, int max_box,
                         double efficiency, const Bits& tagged, std::vector<IBox>& out) {
  const int b = bf / 2;
  const int nb = M / b;
  thread_local Bits cov;
  if (!full_level) {
    cov.init(nb);
    for (const IBox& L : level_boxes) {
      // blocks fully inside the box
      const int x0 = (L.lo[0] + b - 1) / b, y0 = (L.lo[1] + b - 1) / b, z0 = (L.lo[2] + b - 1) / b;
      const int x1 = (L.hi[0] + 1) / b - 1, y1 = (L.hi[1] + 1) / b - 1, z1 = (L.hi[2] + 1) / b - 1;
      if (x1 < x0) continue;
      for (int z = z0; z <= z1; ++z)
        for (int y = y0; y <= y1; ++y) cov.set_x(x0, x1, y, z);
    }
  }
  Ctx C;
  C.eff = efficiency;
  C.cov = full_level ? nullptr : &cov;
  // tagged blocks in (z, y, x) order, without those whose neighbourhood leaves the level.
  // When rows are whole words, the neighbourhood test runs on 64 blocks at once: a block
  // is allowed iff the allowed-block bits of the 3 x 3 rows around its row, each also
  // shifted by one block either way, all hold.
  const bool rows_in_words = !full_level && nb % 64 == 0;
  const int W = nb / 64;
  for (size_t wi = 0; wi < tagged.w.size(); ++wi) {
    uint64_t word = tagged.w[wi];
    if (word && rows_in_words) {
      const size_t row = wi / W;
      const int wx = (int)(wi % W), y = (int)(row % nb), z = (int)(row / nb);
      uint64_t ok = ~0ull;
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy) {
          const size_t r = ((size_t)wrap(z + dz, nb) * nb + wrap(y + dy, nb)) * W;
          const uint64_t c = cov.w[r + wx], cl = cov.w[r + (wx + W - 1) % W], cr = cov.w[r + (wx + 1) % W];
          ok &= c & ((c << 1) | (cl >> 63)) & ((c >> 1) | (cr << 63));
        }
      word &= ok;
    }
    while (word) {
      const int bit = __builtin_ctzll(word);
      word &= word - 1;
      const size_t k = (wi << 6) + bit;
      Pt q;
      q.c[0] = (int)(k % nb);
      q.c[1] = (int)((k / nb) % nb);
      q.c[2] = (int)(k / ((size_t)nb * nb));
      if (!full_level && !rows_in_words) {
        IBox one;
        for (int d = 0; d < 3; ++d) one.lo[d] = one.hi[d] = q.c[d];
        if (!clean(cov, one)) continue;
      }
      C.pts.push_back(q);
    }
  }
  br(C, 0, (long long)C.pts.size());
  // refine to the next level (block = bf fine cells) and chop to max_box
  const int mb = std::max(bf, max_box / bf * bf);
  for (const IBox& B : C.out) {
    int len[3], npc[3];
    for (int d = 0; d < 3; ++d) {
      len[d] = B.size(d);                   // in units of bf
      npc[d] = (len[d] * bf + mb - 1) / mb;  // pieces along d
    }
    for (int pz = 0; pz < npc[2]; ++pz)
      for (int py = 0; py < npc[1]; ++py)
        for (int px = 0; px < npc[0]; ++px) {
          const int p[3] = {px, py, pz};
          IBox f;
          for (int d = 0; d < 3; ++d) {
            const int base = len[d] / npc[d], extra = len[d] % npc[d];
            const int start = p[d] * base + std::min(p[d], extra);
            const int cnt = base + (p[d] < extra ? 1 : 0);
            f.lo[d] = (B.lo[d] + start) * bf;
            f.hi[d] = (B.lo[d] + start + cnt) * bf - 1;
          }
          out.push_back(f);
        }
  }
  return true;
}
