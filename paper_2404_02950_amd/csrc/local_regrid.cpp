// Local regrid (section II, "Local versus global regrid"): the existing boxes of a level
// stay; the level only grows, by whole blocks of the blocking factor, where tagged cells
// of the coarser level (with their n_error_buf buffer) reach past it, and coarser levels
// grow where the added blocks need the nesting gap.  Everything is done on one byte per
// block of the level being grown, so the cost follows the number of blocks touched by
// tags rather than a clustering of all tags.
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "sh_geom.h"

namespace {

struct BlockGrid {
  int nb = 0;
  std::vector<uint8_t> v;  // [z][y][x]
  explicit BlockGrid(int nb_) : nb(nb_), v((size_t)nb_ * nb_ * nb_, 0) {}
  static int wrap(int a, int n) { return ((a % n) + n) % n; }
  uint8_t& at(int x, int y, int z) { return v[((size_t)z * nb + y) * nb + x]; }
  // mark blocks lo..hi per axis (inclusive, wrapping periodically; a range longer than
  // the grid marks the whole axis)
  void mark(const int lo[3], const int hi[3]) {
    int n[3];
    for (int d = 0; d < 3; ++d) n[d] = std::min(hi[d] - lo[d] + 1, nb);
    for (int k = 0; k < n[2]; ++k)
      for (int j = 0; j < n[1]; ++j)
        for (int i = 0; i < n[0]; ++i) at(wrap(lo[0] + i, nb), wrap(lo[1] + j, nb), wrap(lo[2] + k, nb)) = 1;
  }
};

int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// occupancy of a level's boxes; every box must consist of whole blocks inside [0, M)
bool occupy(BlockGrid& g, const std::vector<IBox>& boxes, int bf, int M, std::string& err) {
  for (const IBox& b : boxes) {
    for (int d = 0; d < 3; ++d)
      if (b.lo[d] < 0 || b.hi[d] >= M || b.lo[d] % bf || (b.hi[d] + 1) % bf || b.hi[d] < b.lo[d]) {
        err = "a box is not made of whole blocking-factor blocks inside the level";
        return false;
      }
    for (int z = b.lo[2] / bf; z <= b.hi[2] / bf; ++z)
      for (int y = b.lo[1] / bf; y <= b.hi[1] / bf; ++y)
        for (int x = b.lo[0] / bf; x <= b.hi[0] / bf; ++x) g.at(x, y, z) = 1;
  }
  return true;
}

// blocks marked in `need` but not in `have`, as x runs of at most max_box cells
void emit_runs(BlockGrid& need, BlockGrid& have, int bf, int max_box, std::vector<IBox>& out) {
  const int nb = need.nb, run_max = std::max(1, max_box / bf);
  for (int z = 0; z < nb; ++z)
    for (int y = 0; y < nb; ++y)
      for (int x = 0; x < nb;) {
        if (!need.at(x, y, z) || have.at(x, y, z)) {
          ++x;
          continue;
        }
        const int x0 = x;
        while (x < nb && need.at(x, y, z) && !have.at(x, y, z) && x - x0 < run_max) ++x;
        IBox b;
        b.lo[0] = x0 * bf;
        b.hi[0] = x * bf - 1;
        b.lo[1] = y * bf;
        b.hi[1] = (y + 1) * bf - 1;
        b.lo[2] = z * bf;
        b.hi[2] = (z + 1) * bf - 1;
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
  BlockGrid have(nb), need(nb);
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
  emit_runs(need, have, bf, max_box, out);
  return true;
}

bool local_nest_boxes(int M_k, const std::vector<IBox>& added_fine, const std::vector<IBox>& level_boxes, int bf,
                      int max_box, std::vector<IBox>& out, std::string& err) {
  out.clear();
  if (!check_grid(M_k, bf, err)) return false;
  const int nb = M_k / bf, h = bf / 2;
  BlockGrid have(nb), need(nb);
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
  emit_runs(need, have, bf, max_box, out);
  return true;
}
