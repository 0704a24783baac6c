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
#include <stdint.h>

#include <cstdlib>
#include <string>
#include <vector>

#include "sh_geom.h"

namespace {

struct Grid {
  int n = 0;
  std::vector<uint8_t> v;
  std::vector<int> sat;  // summed-area table, (n+1)^3
  uint8_t& at(int x, int y, int z) { return v[((size_t)z * n + y) * n + x]; }
  int S(int x, int y, int z) const { return sat[((size_t)z * (n + 1) + y) * (n + 1) + x]; }
  void build_sat() {
    const int m = n + 1;
    sat.assign((size_t)m * m * m, 0);
    for (int z = 1; z <= n; ++z)
      for (int y = 1; y <= n; ++y)
        for (int x = 1; x <= n; ++x) {
          const size_t i = ((size_t)z * m + y) * m + x;
          sat[i] = v[((size_t)(z - 1) * n + (y - 1)) * n + (x - 1)] + sat[i - 1] + sat[i - m] + sat[i - (size_t)m * m] -
                   sat[i - 1 - m] - sat[i - 1 - (size_t)m * m] - sat[i - m - (size_t)m * m] +
                   sat[i - 1 - m - (size_t)m * m];
        }
  }
  long long count(const IBox& b) const {
    if (b.empty()) return 0;
    const int x0 = b.lo[0], y0 = b.lo[1], z0 = b.lo[2], x1 = b.hi[0] + 1, y1 = b.hi[1] + 1, z1 = b.hi[2] + 1;
    return (long long)S(x1, y1, z1) - S(x0, y1, z1) - S(x1, y0, z1) - S(x1, y1, z0) + S(x0, y0, z1) + S(x0, y1, z0) +
           S(x1, y0, z0) - S(x0, y0, z0);
  }
};

IBox slice(const IBox& b, int d, int i) {
  IBox s = b;
  s.lo[d] = s.hi[d] = i;
  return s;
}

IBox bounding(const Grid& g, IBox b) {
  if (g.count(b) == 0) {
    b.hi[0] = b.lo[0] - 1;
    return b;
  }
  for (int d = 0; d < 3; ++d) {
    while (g.count(slice(b, d, b.lo[d])) == 0) ++b.lo[d];
    while (g.count(slice(b, d, b.hi[d])) == 0) --b.hi[d];
  }
  return b;
}

// g: tagged blocks; forbid: blocks a box may not contain (nesting), or null
void br(const Grid& g, const Grid* forbid, IBox box, double eff, std::vector<IBox>& out) {
  box = bounding(g, box);
  if (box.empty()) return;
  const long long n = g.count(box), vol = box.volume();
  const bool clean = !forbid || forbid->count(box) == 0;
  if (((double)n >= eff * (double)vol && clean) || vol == 1) {
    out.push_back(box);
    return;
  }
  int best_d = -1, best_cut = 0;
  // 1) a hole in a signature, the one nearest the middle of its side
  double best_dist = 1e30;
  for (int d = 0; d < 3; ++d) {
    const double mid = 0.5 * (box.lo[d] + box.hi[d]);
    for (int i = box.lo[d] + 1; i < box.hi[d]; ++i)
      if (g.count(slice(box, d, i)) == 0 && std::abs(i - mid) < best_dist) {
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
      std::vector<long long> sig(len), lap(len, 0);
      for (int i = 0; i < len; ++i) sig[i] = g.count(slice(box, d, box.lo[d] + i));
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
  IBox a = box, b = box;
  a.hi[best_d] = best_cut - 1;
  b.lo[best_d] = best_cut;
  br(g, forbid, a, eff, out);
  br(g, forbid, b, eff, out);
}

int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
int wrap(int a, int n) { return ((a % n) + n) % n; }

}  // namespace

bool cluster_level(int M, const std::vector<IBox>& level_boxes, bool full_level, int bf, int max_box, int nbuf,
                   double efficiency, const int32_t* tags, long long ntag, std::vector<IBox>& out, std::string& err) {
  out.clear();
  if (bf < 2 || (bf & 1)) {
    err = "blocking factor must be even";
    return false;
  }
  const int b = bf / 2;
  if (M % b) {
    err = "level size not a multiple of half the blocking factor";
    return false;
  }
  const int nb = M / b;
  Grid g;
  g.n = nb;
  g.v.assign((size_t)nb * nb * nb, 0);
  for (long long t = 0; t < ntag; ++t) {
    int c[3], lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      c[d] = tags[3 * t + d];
      if (c[d] < 0 || c[d] >= M) {
        err = "tag outside the level";
        return false;
      }
      lo[d] = floordiv(c[d] - nbuf, b);
      hi[d] = floordiv(c[d] + nbuf, b);
      if (hi[d] - lo[d] >= nb) {
        lo[d] = 0;
        hi[d] = nb - 1;
      }
    }
    for (int z = lo[2]; z <= hi[2]; ++z)
      for (int y = lo[1]; y <= hi[1]; ++y)
        for (int x = lo[0]; x <= hi[0]; ++x) g.at(wrap(x, nb), wrap(y, nb), wrap(z, nb)) = 1;
  }
  Grid forbid;
  if (!full_level) {
    forbid.n = nb;
    forbid.v.assign((size_t)nb * nb * nb, 0);
    std::vector<uint8_t> cov((size_t)nb * nb * nb, 0);
    for (const IBox& L : level_boxes) {
      // blocks fully inside the box
      const int x0 = (L.lo[0] + b - 1) / b, y0 = (L.lo[1] + b - 1) / b, z0 = (L.lo[2] + b - 1) / b;
      const int x1 = (L.hi[0] + 1) / b - 1, y1 = (L.hi[1] + 1) / b - 1, z1 = (L.hi[2] + 1) / b - 1;
      for (int z = z0; z <= z1; ++z)
        for (int y = y0; y <= y1; ++y)
          for (int x = x0; x <= x1; ++x) cov[((size_t)z * nb + y) * nb + x] = 1;
    }
    for (int z = 0; z < nb; ++z)
      for (int y = 0; y < nb; ++y)
        for (int x = 0; x < nb; ++x) {
          bool ok = true;
          for (int dz = -1; dz <= 1 && ok; ++dz)
            for (int dy = -1; dy <= 1 && ok; ++dy)
              for (int dx = -1; dx <= 1 && ok; ++dx)
                ok = cov[((size_t)wrap(z + dz, nb) * nb + wrap(y + dy, nb)) * nb + wrap(x + dx, nb)] != 0;
          if (!ok) {
            g.at(x, y, z) = 0;
            forbid.at(x, y, z) = 1;
          }
        }
    forbid.build_sat();
  }
  g.build_sat();
  std::vector<IBox> blk;
  IBox all;
  for (int d = 0; d < 3; ++d) {
    all.lo[d] = 0;
    all.hi[d] = nb - 1;
  }
  br(g, full_level ? nullptr : &forbid, all, efficiency, blk);
  // refine to the next level (block = bf fine cells) and chop to max_box
  const int mb = std::max(bf, max_box / bf * bf);
  for (const IBox& B : blk) {
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
