// Host-side check of the closed-form walk segmentation: for seeded rays, the
// segments of every length K, walked with the same header code the kernels
// run, must concatenate to the canonical exact walk -- same keys, same hit
// flag on the last voxel, segment start positions equal to the voxels
// before them -- every key must lie inside the map bounds, and every
// segment's voxels inside the box seg_bounds gives for it.
//
// usage: seg_walk_check <seed> <rays> ; prints "ok <rays> <voxels>" or the
// first mismatch, exit status 0 only when every check holds.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "ohm_seg_math.h"

using namespace ohm;

namespace {

uint64_t g_state;
uint64_t next_u64() {  // splitmix64
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
int64_t uniform(int64_t lo, int64_t hi) {  // inclusive
  return lo + (int64_t)(next_u64() % (uint64_t)(hi - lo + 1));
}

struct Key {
  int32_t k[3];
  bool last;
};

bool same(const Key& a, const Key& b) {
  return a.k[0] == b.k[0] && a.k[1] == b.k[1] && a.k[2] == b.k[2] && a.last == b.last;
}

void canonical(const DevMap& m, const int64_t q0[3], const int64_t q1[3], std::vector<Key>& out) {
  const int S = m.F;
  int32_t k0[3], k1[3], k[3];
  for (int a = 0; a < 3; ++a) {
    k0[a] = (int32_t)(q0[a] >> S);
    k1[a] = (int32_t)(q1[a] >> S);
    k[a] = k0[a];
  }
  const int32_t hi[3] = {m.kmax[0] - 1, m.kmax[1] - 1, m.kmax[2] - 1};
  Walk w;
  walk_init(w, q0, q1, k0, k1, m.kmin, hi, S);
  out.clear();
  out.push_back({{k[0], k[1], k[2]}, w.total == 0});
  while (w.total > 0) {
    const int a = walk_step(w);
    if (w.rem[a] == 0 && ((w.clip >> a) & 1u)) break;
    k[a] += w.sg[a];
    out.push_back({{k[0], k[1], k[2]}, w.total == 0});
  }
}

int fail(const char* what, long ray, int K, const int64_t q0[3], const int64_t q1[3], long i) {
  printf("FAIL %s ray %ld K %d at %ld: q0 %lld %lld %lld q1 %lld %lld %lld\n", what, ray, K, i, (long long)q0[0],
         (long long)q0[1], (long long)q0[2], (long long)q1[0], (long long)q1[1], (long long)q1[2]);
  return 1;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s seed rays\n", argv[0]);
    return 2;
  }
  g_state = strtoull(argv[1], nullptr, 10);
  const long n_rays = strtol(argv[2], nullptr, 10);
  const int Ks[] = {1, 2, 3, 5, 16, 64, 4096};
  std::vector<Key> ref, got;
  long voxels = 0;
  for (long ray = 0; ray < n_rays; ++ray) {
    DevMap m = {};
    m.F = (ray % 3 == 0) ? 8 : 16;
    for (int a = 0; a < 3; ++a) {
      m.kmin[a] = (int32_t)uniform(-300, 0);
      m.kmax[a] = m.kmin[a] + (int32_t)uniform(1, 400);
    }
    const int64_t one = (int64_t)1 << m.F;
    int64_t q0[3], q1[3];
    const int kind = (int)uniform(0, 9);
    // longer rays now and then, so that small K reaches the last (open) level
    const int64_t span = (ray % 50 == 0) ? 3000 : 120;
    int64_t d_shared = uniform(-span * one, span * one);
    for (int a = 0; a < 3; ++a) {
      const int64_t k0 = uniform(m.kmin[a], m.kmax[a] - 1);
      const int64_t frac = kind == 1 ? 0 : (kind == 2 ? one / 2 : uniform(0, one - 1));
      q0[a] = k0 * one + frac;
      int64_t d = uniform(-span * one, span * one);
      if (kind == 3 && a == 1) d = 0;                         // axis-parallel in y
      if (kind == 4 && a != 0) d = 0;                         // along x only
      if (kind == 5) d = (a == 2 ? -d_shared : d_shared);     // exact diagonal: ties at every corner
      if (kind == 6 && a < 2) d = d_shared;                   // ties between x and y
      if (kind == 7) d = d / 64;                              // short rays
      if (kind == 8 && a == 2) d = uniform(-2, 2);            // nearly flat
      q1[a] = q0[a] + d;
    }
    if (kind == 9) { q1[0] = q0[0]; q1[1] = q0[1]; q1[2] = q0[2]; }  // zero length
    canonical(m, q0, q1, ref);
    voxels += (long)ref.size();
    for (const Key& k : ref)
      for (int a = 0; a < 3; ++a)
        if (k.k[a] < m.kmin[a] || k.k[a] >= m.kmax[a]) return fail("canonical key out of bounds", ray, 0, q0, q1, 0);
    int32_t k0[3], k1[3];
    for (int a = 0; a < 3; ++a) {
      k0[a] = (int32_t)(q0[a] >> m.F);
      k1[a] = (int32_t)(q1[a] >> m.F);
    }
    const int32_t hi[3] = {m.kmax[0] - 1, m.kmax[1] - 1, m.kmax[2] - 1};
    Walk w;
    walk_init(w, q0, q1, k0, k1, m.kmin, hi, m.F);
    if (walk_voxels(w, q0, q1, m.F) != ref.size()) return fail("walk_voxels", ray, 0, q0, q1, (long)ref.size());
    const int M = ray_major_axis(q0, q1);
    for (int K : Ks) {
      const uint32_t nseg = seg_count(w, q0, q1, K);
      if (nseg < 1 || nseg > (uint32_t)kMaxLevels) return fail("seg_count range", ray, K, q0, q1, nseg);
      got.clear();
      for (uint32_t j = 0; j < nseg; ++j) {
        SegState s;
        seg_init(s, q0, q1, m, (int)j, K);
        if (s.empty) continue;
        if (s.pos != got.size()) return fail("segment start position", ray, K, q0, q1, (long)j);
        // every voxel of the segment lies in its seg_bounds box
        int32_t blo[3], bhi[3];
        seg_bounds(s, q0, q1, M, K, j + 1 == (uint32_t)kMaxLevels, m.F, blo, bhi);
        const size_t first = got.size();
        got.push_back({{s.k[0], s.k[1], s.k[2]}, s.w.total == 0});
        while (s.w.total > 0) {
          if (seg_advance(s, M) < 0) break;
          got.push_back({{s.k[0], s.k[1], s.k[2]}, s.w.total == 0});
          if (got.size() > ref.size()) return fail("segments overrun the walk", ray, K, q0, q1, (long)j);
        }
        for (size_t i = first; i < got.size(); ++i)
          for (int a = 0; a < 3; ++a)
            if (got[i].k[a] < blo[a] || got[i].k[a] > bhi[a]) return fail("segment outside its bounds", ray, K, q0, q1, (long)j);
      }
      if (got.size() != ref.size()) return fail("voxel count", ray, K, q0, q1, (long)got.size());
      for (size_t i = 0; i < ref.size(); ++i)
        if (!same(got[i], ref[i])) return fail("key", ray, K, q0, q1, (long)i);
    }
  }
  printf("ok %ld %ld\n", n_rays, voxels);
  return 0;
}
