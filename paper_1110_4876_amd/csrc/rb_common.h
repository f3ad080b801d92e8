// rb_common.h -- device-side constants, layouts and wave helpers shared by
// the HIP kernels of librb (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define RB_DEPTH 21                        // deepest octree level (63-bit keys)
#define RB_NLEV (RB_DEPTH + 1)             // levels 0..21
#define RB_BOTTOM 24       // counter slot of the bottom large-node list
#define RB_LARGE_SLOTS 32  // large-node counters: one per level, then RB_BOTTOM
#define RB_NONE 0xFFFFFFFFu                // absent node / end of walk
#define RB_KEY_DEAD 0xFFFFFFFFFFFFFFFFull  // key of a removed / outside particle
#define RB_TILE_MIN 64                     // slots per topology tile
#define RB_TILE_MAX 512
#define RB_MAX_IMAGES 25                   // (2*2+1)^2 for two ghost rings

// device error word bits (reported by the next synchronising call)
enum : uint32_t {
  RB_ERR_NODES = 1u,    // node capacity exceeded
  RB_ERR_OUTSIDE = 2u,  // particle outside a periodic / shear axis
  RB_ERR_STACK = 4u,    // FP32 walk traversal stack full
  RB_ERR_TREE = 8u,     // inconsistent node links (guarded, never followed)
  RB_ERR_INDEX = 16u,   // a target index outside [0, n)
  RB_ERR_SORT = 32u,    // a sort look-back wait gave up (result invalid)
  RB_ERR_COLL = 64u,    // collision queue full
};

// Walk link of a node: child_or_first = first child (internal) or first
// sorted slot (leaf); skip = next node after the subtree in depth-first
// order (RB_NONE at the end); count = particles;
// lvl = level | leaf << 8 | n_child << 9.
struct __align__(16) NodeLink {
  uint32_t child_or_first;
  uint32_t skip;
  uint32_t count;
  uint32_t lvl;
};

// The node as the FP32-mixed walk reads it: one 64-byte line.  Q is kept
// as its five independent components (it is traceless: zz = -(xx + yy)).
struct __align__(64) WNode {
  double cx, cy, cz, M;     // centre of mass, mass
  uint32_t child_or_first;  // as NodeLink
  uint32_t count;
  uint32_t lvl;
  float qxx, qxy, qxz, qyy, qyz;
};

// Per-patch constants (device array, one entry per patch).  The domain is
// n_root[a] cubic root boxes of side w0 along axis a (Sect. 2.3).  Keys
// quantise it inside one cube of side W = w0 2^nvirt, 2^nvirt >= every
// n_root: the first nvirt octree levels are cells above the root boxes
// (never leaves, always opened), level nvirt holds the root boxes, and a
// node at level l is a cube of side W 2^-l.  With one root box nvirt = 0,
// W = w0 and L = (W, W, W).
struct PatchInfo {
  double W;        // side of the quantised cube (root box side times 2^nvirt)
  double x0[3];    // domain minimum corner
  double S;        // 2^(21 - nvirt) / w0 = 2^21 / W, quantisation scale
  double L[3];     // domain extents: n_root[a] times the root box side
  double qtop[3];  // largest quantised coordinate: n_root[a] 2^(21 - nvirt) - 1
  uint32_t start;  // first slot of the patch
  uint32_t n;      // slots of the patch
  uint32_t n_active;
  uint32_t nvirt;  // octree levels above the root boxes
};

// Per-step time-dependent values, indexed by the device step counter.
// For patch p: s_half[p] = shear offset at t + dt/2 (kick, wrap after the
// first drift), s_end[p] = offset at t + dt (wrap after the second drift).
struct StepConst {
  double half;      // dt / 2
  double dt;
  double c, sn;     // cos, sin of omega dt/2 (epicycle drift)
  double cz, sz;    // cos, sin of omega_z dt/2
  double omega, omega_z;
  double jump;      // shear velocity jump factor 1.5 omega (times W per patch)
};

__device__ __forceinline__ uint32_t rb_mbcnt(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t rb_lane() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// inclusive prefix sum over the 64 lanes of a wave
__device__ __forceinline__ uint32_t rb_wave_incl_scan(uint32_t v) {
  const uint32_t lane = rb_lane();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t t = __shfl_up(v, d, 64);
    if (lane >= (uint32_t)d) v += t;
  }
  return v;
}

// number of leading octal digits two live keys share (0..21)
__device__ __forceinline__ int rb_lcp(uint64_t a, uint64_t b) {
  uint64_t x = a ^ b;
  if (x == 0) return RB_DEPTH;
  return (__clzll((long long)x) - 1) / 3;  // bit 63 is 0 in every live key
}

__device__ __forceinline__ uint64_t rb_spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

// Quantise one coordinate: q = floor((x - x0) * S).  The subtraction and
// the product are each rounded on their own (neither can be contracted); a
// value rounding up to the domain's end is clamped to qtop.  Returns false
// outside [x0, x0 + L) or for NaN.
__device__ __forceinline__ bool rb_quantise(double xa, double x0, double L, double S,
                                            double qtop, uint32_t &q) {
  double u = xa - x0;
  if (!(u >= 0.0 && u < L)) return false;
  double f = floor(u * S);
  if (f >= qtop) f = qtop;
  q = (uint32_t)f;
  return true;
}

__device__ __forceinline__ uint64_t rb_key(uint32_t qx, uint32_t qy, uint32_t qz) {
  return (rb_spread3(qx) << 2) | (rb_spread3(qy) << 1) | rb_spread3(qz);
}

// Small-system sort (k_bsort.hip): buckets of the top 12 key bits, and one
// more for removed particles (all-ones key, sorted last).
#define BS_BITS 12
#define BS_NB ((1 << BS_BITS) + 1)
#define BS_SHIFT (63 - BS_BITS)

__device__ __forceinline__ uint32_t bs_bucket(uint64_t key) {
  return key == RB_KEY_DEAD ? (uint32_t)(1 << BS_BITS) : (uint32_t)(key >> BS_SHIFT);
}

// Count a freshly written key in its (patch, bucket) counter: the lanes of
// the wave holding the same (patch, bucket) add their count with one atomic
// (neighbouring slots usually share one or two buckets).  Every active lane
// of the wave calls it; P is the number of patches.
__device__ __forceinline__ void rb_bucket_add(uint32_t *__restrict__ bcnt, uint32_t p,
                                              uint32_t P, uint64_t key) {
  const uint32_t b = bs_bucket(key);
  uint64_t peers = __ballot(true);
#pragma unroll
  for (int bit = 0; bit < BS_BITS + 1; ++bit) {
    const bool on = (b >> bit) & 1u;
    const uint64_t m = __ballot(on);
    peers &= on ? m : ~m;
  }
  if (P > 1) {
    const int pbits = 32 - __clz((int)(P - 1));
    for (int bit = 0; bit < pbits; ++bit) {
      const bool on = (p >> bit) & 1u;
      const uint64_t m = __ballot(on);
      peers &= on ? m : ~m;
    }
  }
  if (rb_mbcnt(peers) == 0) atomicAdd(&bcnt[(size_t)p * BS_NB + b], (uint32_t)__popcll(peers));
}

// index of the patch holding slot s (binary search over patch starts)
__device__ __forceinline__ uint32_t rb_patch_of(const uint32_t *__restrict__ starts,
                                                uint32_t n_patch, uint32_t s) {
  uint32_t lo = 0, hi = n_patch;  // starts[n_patch] = total
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (starts[mid] <= s) lo = mid; else hi = mid;
  }
  return lo;
}

static inline unsigned rb_div_up(uint64_t a, uint64_t b) { return (unsigned)((a + b - 1) / b); }
