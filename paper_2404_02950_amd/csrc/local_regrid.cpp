// Local regrid (section II, "Local versus global regrid"): the existing boxes of a level
// stay; the level only grows, by whole blocks of the blocking factor, where tagged cells
// of the coarser level (with their n_error_buf buffer) reach past it, and coarser levels
// grow where the added blocks need the nesting gap.  Blocks are one bit each; the added
// ones are collected by skipping empty words and merged into boxes (x runs, then y, then
// z), so the cost follows the blocks touched by tags rather than a clustering of all
// tags.
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "sh_geom.h"

namespace {

// One bit per block of a level ([z][y][x], x fastest).
struct BlockBits {
  int nb = 0;
  std::vector<uint64_t> w;
  // cleared to nb^3 blocks (the storage is kept: a few MB freshly allocated on every
  // regrid would be page-faulted in each time)
  void reset(int nb_) {
    nb = nb_;
    w.assign(((size_t)nb_ * nb_ * nb_ + 63) / 64, 0);
  }
  static int wrap(int a, int n) { return ((a % n) + n) % n; }
  void set(int x, int y, int z) {
    const size_t k = ((size_t)z * nb + y) * nb + x;
    w[k >> 6] |= 1ull << (k & 63);
  }
  // mark blocks lo..hi per axis (inclusive, wrapping periodically; a range longer than
  // the grid marks the whole axis)
  void mark(const int lo[3], const int hi[3]) {
    int n[3];
    for (int d = 0; d < 3; ++d) n[d] = std::min(hi[d] - lo[d] + 1, nb);
    for (int k = 0; k < n[2]; ++k)
      for (int j = 0; j < n[1]; ++j)
        for (int i = 0; i < n[0]; ++i) set(wrap(lo[0] + i, nb), wrap(lo[1] + j, nb), wrap(lo[2] + k, nb));
  }
};

int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// occupancy of a level's boxes; every box must consist of whole blocks inside [0, M)
bool occupy(BlockBits& g, const std::vector<IBox>& boxes, int bf, int M, std::string& err) {
  for (const IBox& b : boxes) {
    for (int d = 0; d < 3; ++d)
      if (b.lo[d] < 0 || b.hi[d] >= M || b.lo[d] % bf || (b.hi[d] + 1) % bf || b.hi[d] < b.lo[d]) {
        err = "a box is not made of whole blocking-factor blocks inside the level";
        return false;
      }
    for (int z = b.lo[2] / bf; z <= b.hi[2] / bf; ++z)
      for (int y = b.lo[1] / bf; y <= b.hi[1] / bf; ++y)
        for (int x = b.lo[0] / bf; x <= b.hi[0] / bf; ++x) g.set(x, y, z);
  }
  return true;
}

// Greedy merge of consecutive runs along one axis: items sorted by (key, lo), a run grows
// from its lowest item while the next one has the same key, starts right after it and the
// extent stays within run_max.
struct Span {
  int key[5];  // the extents that must agree (unused entries 0)
  int lo, hi;
};

std::vector<Span> merge_spans(std::vector<Span> v, int run_max) {
  auto same = [](const Span& a, const Span& b) {
    for (int i = 0; i < 5; ++i)
      if (a.key[i] != b.key[i]) return false;
    return true;
  };
  std::sort(v.begin(), v.end(), [](const Span& a, const Span& b) {
    for (int i = 0; i < 5; ++i)
      if (a.key[i] != b.key[i]) return a.key[i] < b.key[i];
    return a.lo < b.lo;
  });
  std::vector<Span> out;
  for (size_t i = 0; i < v.size();) {
    Span r = v[i];
    size_t j = i + 1;
    while (j < v.size() && same(v[j], r) && v[j].lo == r.hi + 1 && v[j].hi - r.lo + 1 <= run_max) r.hi = v[j++].hi;
    out.push_back(r);
    i = j;
  }
  return out;
}

// blocks in `need` but not in `have` as boxes: x runs, then equal x runs over consecutive
// y rows, then equal rectangles over consecutive z planes (each at most max_box cells),
// ordered by their lowest corner (z, y, x)
void emit_boxes_of(const BlockBits& need, const BlockBits& have, int bf, int max_box, std::vector<IBox>& out) {
  const int nb = need.nb, run_max = std::max(1, max_box / bf);
  std::vector<Span> runs;  // key {z, y}, x extent
  Span cur{};
  bool open = false;
  auto close = [&]() {
    if (open) runs.push_back(cur);
    open = false;
  };
  for (size_t wi = 0; wi < need.w.size(); ++wi) {
    uint64_t m = need.w[wi] & ~have.w[wi];
    if (!m) {
      close();  // a zero word breaks any run
      continue;
    }
    for (int bit = 0; bit < 64; ++bit) {
      const size_t k = wi * 64 + bit;
      if (k >= (size_t)nb * nb * nb) break;
      if (!((m >> bit) & 1)) {
        close();
        continue;
      }
      const int x = (int)(k % nb), y = (int)((k / nb) % nb), z = (int)(k / ((size_t)nb * nb));
      if (open && cur.key[0] == z && cur.key[1] == y && x == cur.hi + 1 && x - cur.lo + 1 <= run_max) {
        cur.hi = x;
      } else {
        close();
        cur = Span{{z, y, 0, 0, 0}, x, x};
        open = true;
      }
    }
  }
  close();
  // y merge: key {z, x0, x1}
  std::vector<Span> ys;
  ys.reserve(runs.size());
  for (const Span& r : runs) ys.push_back(Span{{r.key[0], r.lo, r.hi, 0, 0}, r.key[1], r.key[1]});
  ys = merge_spans(std::move(ys), run_max);
  // z merge: key {y0, y1, x0, x1}
  std::vector<Span> zs;
  zs.reserve(ys.size());
  for (const Span& r : ys) zs.push_back(Span{{r.lo, r.hi, r.key[1], r.key[2], 0}, r.key[0], r.key[0]});
  zs = merge_spans(std::move(zs), run_max);
  std::sort(zs.begin(), zs.end(), [](const Span& a, const Span& b) {
    if (a.lo != b.lo) return a.lo < b.lo;            // z0
    if (a.key[0] != b.key[0]) return a.key[0] < b.key[0];  // y0
    return a.key[2] < b.key[2];                      // x0
  });
  for (const Span& r : zs) {
    IBox b;
    b.lo[0] = r.key[2] * bf;
    b.hi[0] = (r.key[3] + 1) * bf - 1;
    b.lo[1] = r.key[0] * bf;
    b.hi[1] = (r.key[1] + 1) * bf - 1;
    b.lo[2] = r.lo * bf;
    b.hi[2] = (r.hi + 1) * bf - 1;
    out.push_back(b);
  }
}

bool check_grid(int M, int bf, std::string& err) {
  if (bf < 2 || (bf & 1) || M < bf || M % bf) {
    err = "the level size must be a multiple of an even blocking factor";
    return false;
  }
  return true;
}

}  // namespace

bool local_tag_boxes(int M_fine, const std::vector<IBox>& fine_boxes, int bf, int nbuf, int max_box,
                     const int32_t* tags, long long ntag, std::vector<IBox>& out, std::string& err) {
  out.clear();
  if (!check_grid(M_fine, bf, err)) return false;
  const int nb = M_fine / bf, Mc = M_fine / 2;
  thread_local BlockBits have, need;
  have.reset(nb);
  need.reset(nb);
  if (!occupy(have, fine_boxes, bf, M_fine, err)) return false;
  for (long long t = 0; t < ntag; ++t) {
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      const int c = tags[3 * t + d];
      if (c < 0 || c >= Mc) {
        err = "a tag lies outside the coarser level";
        return false;
      }
      // the refined buffer cube [2(c - nbuf), 2(c + nbuf) + 1] in fine cells
      lo[d] = floordiv(2 * (c - nbuf), bf);
      hi[d] = floordiv(2 * (c + nbuf) + 1, bf);
    }
    need.mark(lo, hi);
  }
  emit_boxes_of(need, have, bf, max_box, out);
  return true;
}

bool local_nest_boxes(int M_k, const std::vector<IBox>& added_fine, const std::vector<IBox>& level_boxes, int bf,
                      int max_box, std::vector<IBox>& out, std::string& err) {
  out.clear();
  if (!check_grid(M_k, bf, err)) return false;
  const int nb = M_k / bf, h = bf / 2;
  thread_local BlockBits have, need;
  have.reset(nb);
  need.reset(nb);
  if (!occupy(have, level_boxes, bf, M_k, err)) return false;
  for (const IBox& b : added_fine) {
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      if (b.lo[d] < 0 || b.hi[d] >= 2 * M_k || b.lo[d] % bf || (b.hi[d] + 1) % bf) {
        err = "an added box is not made of whole blocking-factor blocks inside the finer level";
        return false;
      }
      // coarsened box grown by the nesting gap of bf/2 level-k cells
      lo[d] = floordiv(b.lo[d] / 2 - h, bf);
      hi[d] = floordiv((b.hi[d] + 1) / 2 - 1 + h, bf);
    }
    need.mark(lo, hi);
  }
  emit_boxes_of(need, have, bf, max_box, out);
  return true;
}
