// k_bsort.hip -- sort of (Morton key, slot) pairs for small systems by
// buckets of the top 12 key bits (the cells of octree level 4).
//
// Sorting by (key, slot) gives the stable order of the keys (ties keep the
// order of the slots), so the pieces below need not be stable themselves:
//   counting        -- the kernel that writes the keys counts them per
//                      (patch, bucket) (rb_bucket_add; bucket 4096 holds
//                      removed particles, whose all-ones key sorts last);
//   k_bsort_scan    -- per patch: bucket cursors, and segments: runs of
//                      whole buckets that start in the same window of 64
//                      slots (at most 127 keys), a bucket above 64 keys
//                      being a segment of its own (small segments keep
//                      more CUs busy and networks short);
//   k_bsort_scatter -- every key to its bucket (one atomic per bucket and
//                      wave);
//   k_bsort_local   -- per segment: a bitonic sort of (key, slot) held in
//                      registers, by one wave up to 512 keys (partners in
//                      the same lane or swizzled across lanes), by a
//                      workgroup up to 1024 (four rows of 256; partners
//                      within a wave by shuffles, across rows in registers,
//                      across waves through LDS), or, for a larger bucket,
//                      eight-bit radix passes over the slot and the low 51
//                      key bits by one workgroup in global memory.
// Keys and slots arrive in buffer 0, go to their buckets in buffer 1 and
// come back sorted to buffer 0.
#include "rb_internal.h"

#define BS_WIN 64    // segment window (slots)
#define BS_LDS 1024  // largest segment sorted by the bitonic network

// lanes of the wave holding the same value in the low `bits` bits
__device__ __forceinline__ uint64_t bs_match(uint64_t peers, uint32_t v, bool valid, int bits) {
  for (int bit = 0; bit < bits; ++bit) {
    const bool on = (v >> bit) & 1u;
    const uint64_t m = __ballot(valid && on);
    peers &= on ? m : ~m;
  }
  return peers;
}

// One block of 1024 threads per patch (5 buckets per thread).
__global__ __launch_bounds__(1024) void k_bsort_scan(uint32_t *__restrict__ bcnt,
                                                     uint32_t *__restrict__ bcur,
                                                     const uint32_t *__restrict__ starts,
                                                     uint2 *__restrict__ seg,
                                                     uint32_t *__restrict__ ctl) {
  constexpr int PER = (BS_NB + 1023) / 1024;
  __shared__ uint32_t wsum[16];
  __shared__ int wmax[16];
  __shared__ uint32_t s_base;
  const uint32_t p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t st = starts[p];
  uint32_t *cnt = bcnt + (size_t)p * BS_NB;
  uint32_t c[PER], tot = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const uint32_t b = tid * PER + k;
    c[k] = (b < BS_NB) ? cnt[b] : 0u;
    if (b < BS_NB) cnt[b] = 0u;  // ready for the next sort
    tot += c[k];
  }
  // bucket offsets within the patch
  const uint32_t incl = rb_wave_incl_scan(tot);
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t off = incl - tot;
  for (uint32_t q = 0; q < w; ++q) off += wsum[q];
  uint32_t start[PER];
  int win[PER], mx = -1;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    start[k] = off;
    win[k] = c[k] ? (int)(off / BS_WIN) : -1;
    mx = win[k] > mx ? win[k] : mx;
    off += c[k];
    const uint32_t b = tid * PER + k;
    if (b < BS_NB) bcur[(size_t)p * BS_NB + b] = st + start[k];
  }
  // window of the last non-empty bucket before this thread's: an
  // exclusive max-scan (windows never decrease along the buckets)
  int run = mx;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int v = __shfl_up(run, d, 64);
    if (lane >= (uint32_t)d) run = v > run ? v : run;
  }
  if (lane == 63) wmax[w] = run;
  __syncthreads();
  int prev = -1;
  for (uint32_t q = 0; q < w; ++q) prev = wmax[q] > prev ? wmax[q] : prev;
  const int up = __shfl_up(run, 1, 64);
  if (lane > 0) prev = up > prev ? up : prev;
  // a segment starts at a non-empty bucket in a new window, and at a
  // bucket above the window size
  uint32_t flags = 0, nf = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    if (c[k] && (win[k] != prev || c[k] > BS_WIN)) { flags |= 1u << k; ++nf; }
    if (c[k]) prev = win[k];
  }
  const uint32_t fin = rb_wave_incl_scan(nf);
  __syncthreads();  // wsum is reused
  if (lane == 63) wsum[w] = fin;
  __syncthreads();
  uint32_t fo = fin - nf;
  for (uint32_t q = 0; q < w; ++q) fo += wsum[q];
  if (tid == 1023) s_base = atomicAdd(&ctl[0], fo + nf);
  __syncthreads();
  const uint32_t base = s_base;
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (flags & (1u << k)) seg[base + fo++] = make_uint2(st + start[k], p);
}

__global__ __launch_bounds__(256) void k_bsort_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, const uint32_t *__restrict__ starts,
    uint32_t P, uint32_t n, uint32_t *__restrict__ bcur, uint32_t *__restrict__ ctl) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s == 0) ctl[1] = 0;  // segments taken by k_bsort_local
  const bool valid = s < n;
  const uint64_t k = valid ? kin[s] : 0ull;
  const uint32_t v = valid ? vin[s] : 0u;
  const uint32_t p = (valid && P > 1) ? rb_patch_of(starts, P, s) : 0u;
  const uint32_t b = valid ? bs_bucket(k) : 0u;
  // lanes with the same (patch, bucket) share one atomic
  uint64_t peers = bs_match(__ballot(valid), b, valid, BS_BITS + 1);
  if (P > 1) peers = bs_match(peers, p, valid, 32 - __clz((int)(P - 1)));
  const uint32_t lane = rb_lane();
  const uint32_t leader = peers ? (uint32_t)(__ffsll((long long)peers) - 1) : lane;
  uint32_t pos = 0;
  if (valid && lane == leader)
    pos = atomicAdd(&bcur[(size_t)p * BS_NB + b], (uint32_t)__popcll(peers));
  pos = (uint32_t)__shfl((int)pos, (int)leader, 64) + rb_mbcnt(peers);
  if (valid) {
    kout[pos] = k;
    vout[pos] = v;
  }
}

__device__ __forceinline__ bool bs_less(uint64_t ka, uint32_t va, uint64_t kb, uint32_t vb) {
  return ka < kb || (ka == kb && va < vb);
}

// digit q (8 bits) of the composite (low 51 key bits, slot): slot bits first
__device__ __forceinline__ uint32_t bs_digit(uint64_t k, uint32_t v, int q) {
  const uint64_t klow = k & ((1ull << 51) - 1ull);
  const uint64_t lo = (klow << 18) | (uint64_t)v;  // v < 2^18 for small systems
  return q < 8 ? (uint32_t)(lo >> (8 * q)) & 255u : (uint32_t)(klow >> 46) & 255u;
}

// One large bucket by one workgroup: nine stable 8-bit radix passes over
// the composite, from buffer 1 to buffer 0 and back (ending in buffer 0).
__device__ void bs_big(uint64_t *__restrict__ k1, uint32_t *__restrict__ v1,
                       uint64_t *__restrict__ k0, uint32_t *__restrict__ v0, uint32_t a,
                       uint32_t e, uint32_t *hist, uint32_t *wcnt /* [waves][256] */) {
  const uint32_t tid = threadIdx.x, w = tid >> 6;
  const uint32_t nw = blockDim.x >> 6;
  for (int q = 0; q < 9; ++q) {
    const uint64_t *ki = (q & 1) ? k0 : k1;
    const uint32_t *vi = (q & 1) ? v0 : v1;
    uint64_t *ko = (q & 1) ? k1 : k0;
    uint32_t *vo = (q & 1) ? v1 : v0;
    for (uint32_t i = tid; i < 256; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    for (uint32_t s = a + tid; s < e; s += blockDim.x)
      atomicAdd(&hist[bs_digit(ki[s], vi[s], q)], 1u);
    __syncthreads();
    if (tid < 64) {  // exclusive scan of the 256 bins, 4 per lane
      uint32_t h4[4], t = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) { h4[j] = hist[4 * tid + j]; t += h4[j]; }
      uint32_t o = rb_wave_incl_scan(t) - t + a;
#pragma unroll
      for (int j = 0; j < 4; ++j) { hist[4 * tid + j] = o; o += h4[j]; }
    }
    __syncthreads();
    for (uint32_t c0 = a; c0 < e; c0 += blockDim.x) {
      const uint32_t s = c0 + tid;
      const bool valid = s < e;
      const uint64_t kk = valid ? ki[s] : 0ull;
      const uint32_t vv = valid ? vi[s] : 0u;
      const uint32_t d = valid ? bs_digit(kk, vv, q) : 0u;
      const uint64_t peers = bs_match(__ballot(valid), d, valid, 8);
      const uint32_t rank = rb_mbcnt(peers);
      for (uint32_t i = tid; i < nw * 256; i += blockDim.x) wcnt[i] = 0;
      __syncthreads();
      if (valid && rank == 0) wcnt[w * 256 + d] = (uint32_t)__popcll(peers);
      __syncthreads();
      if (tid < 256) {  // per digit: offsets of the waves, running total
        uint32_t o = hist[tid];
        for (uint32_t q2 = 0; q2 < nw; ++q2) {
          const uint32_t t = wcnt[q2 * 256 + tid];
          wcnt[q2 * 256 + tid] = o;
          o += t;
        }
        hist[tid] = o;
      }
      __syncthreads();
      if (valid) {
        const uint32_t pos = wcnt[w * 256 + d] + rank;
        ko[pos] = kk;
        vo[pos] = vv;
      }
      __syncthreads();
    }
  }
}

// keep the smaller or the larger of (own, partner) key per element
__device__ __forceinline__ void bs_take(uint64_t (&k)[4], uint32_t (&v)[4], const uint64_t (&pk)[4],
                                        const uint32_t (&pv)[4], int nr, uint32_t tid,
                                        uint32_t size, uint32_t stride) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (r < nr) {
      const uint32_t el = (uint32_t)r * 256 + tid;
      const bool asc = (el & size) == 0;
      const bool keep_min = ((el & stride) == 0) == asc;
      if (keep_min == (pk[r] < k[r]) && pk[r] != k[r]) { k[r] = pk[r]; v[r] = pv[r]; }
    }
  }
}

// one stage with the partner S lanes away in the same wave
template <int S>
__device__ __forceinline__ void bs_stage_wave(uint64_t (&k)[4], uint32_t (&v)[4], int nr,
                                              uint32_t tid, uint32_t size) {
  uint64_t pk[4];
  uint32_t pv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (S < 32) {
      // ds_swizzle, bit-mask mode: lane ^ S inside each half-wave
      constexpr int pat = 0x1F | (S << 10);
      const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)k[r], pat);
      const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)(k[r] >> 32), pat);
      pk[r] = ((uint64_t)hi << 32) | lo;
      pv[r] = (uint32_t)__builtin_amdgcn_ds_swizzle((int)v[r], pat);
    } else {
      pk[r] = __shfl_xor(k[r], S, 64);
      pv[r] = __shfl_xor(v[r], S, 64);
    }
  }
  bs_take(k, v, pk, pv, nr, tid, size, (uint32_t)S);
}

// Bitonic network on (key, slot) pairs of one segment of at most 64 R
// keys by one wave, lane-major: element e = lane R + r sits in register r of
// the lane, so partners closer than R are in the same lane and the others
// R-multiples of lanes apart (ds_swizzle below 32 lanes, a shuffle at 32).
// The pairs are compared as (key, slot), so equal keys come out in slot
// order and the padding (all-ones key, all-ones slot) last.
template <int S>
__device__ __forceinline__ void bs_lane_xor(uint64_t &k, uint32_t &v) {
  if (S < 32) {
    constexpr int pat = 0x1F | (S << 10);  // bit-mask mode: lane ^ S in each half
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)k, pat);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)(k >> 32), pat);
    k = ((uint64_t)hi << 32) | lo;
    v = (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, pat);
  } else {
    k = __shfl_xor(k, S, 64);
    v = (uint32_t)__shfl_xor((int)v, S, 64);
  }
}

template <int R, int S>
__device__ __forceinline__ void bs_wave_lanes(uint64_t (&k)[R], uint32_t (&v)[R], uint32_t lane,
                                              uint32_t size) {
  // partners S lanes apart: element stride S * R
#pragma unroll
  for (int r = 0; r < R; ++r) {
    uint64_t pk = k[r];
    uint32_t pv = v[r];
    bs_lane_xor<S>(pk, pv);
    const uint32_t e = lane * R + (uint32_t)r;
    const bool asc = (e & size) == 0;
    const bool lower = (e & (uint32_t)(S * R)) == 0;
    if ((lower == asc) == bs_less(pk, pv, k[r], v[r])) { k[r] = pk; v[r] = pv; }
  }
}

template <int R>
__device__ __forceinline__ void bs_wave_sort(const uint64_t *__restrict__ k1,
                                             const uint32_t *__restrict__ v1,
                                             uint64_t *__restrict__ k0, uint32_t *__restrict__ v0,
                                             uint32_t a, uint32_t m, uint32_t lane) {
  uint64_t k[R];
  uint32_t v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t e = lane * R + (uint32_t)r;
    k[r] = e < m ? k1[a + e] : ~0ull;
    v[r] = e < m ? v1[a + e] : ~0u;
  }
#pragma unroll
  for (uint32_t size = 2; size <= 64u * R; size <<= 1) {
#pragma unroll
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride >= (uint32_t)R) {
        switch (stride / R) {
          case 1: bs_wave_lanes<R, 1>(k, v, lane, size); break;
          case 2: bs_wave_lanes<R, 2>(k, v, lane, size); break;
          case 4: bs_wave_lanes<R, 4>(k, v, lane, size); break;
          case 8: bs_wave_lanes<R, 8>(k, v, lane, size); break;
          case 16: bs_wave_lanes<R, 16>(k, v, lane, size); break;
          default: bs_wave_lanes<R, 32>(k, v, lane, size); break;
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int r2 = r | (int)stride;
          if ((r & (int)stride) == 0 && r2 < R) {
            const bool asc = ((lane * R + (uint32_t)r) & size) == 0;
            if (bs_less(k[r2], v[r2], k[r], v[r]) == asc) {
              const uint64_t tk = k[r]; k[r] = k[r2]; k[r2] = tk;
              const uint32_t tv = v[r]; v[r] = v[r2]; v[r2] = tv;
            }
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t e = lane * R + (uint32_t)r;
    if (e < m) { k0[a + e] = k[r]; v0[a + e] = v[r]; }
  }
}

// slot range [a, e) of segment i
__device__ __forceinline__ void bs_segment(const uint2 *__restrict__ seg,
                                           const uint32_t *__restrict__ starts, uint32_t nseg,
                                           uint32_t i, uint32_t &a, uint32_t &e) {
  const uint2 me = seg[i];
  a = me.x;
  e = starts[me.y + 1];
  if (i + 1 < nseg) {
    const uint2 nx = seg[i + 1];
    if (nx.y == me.y) e = nx.x;
  }
}

#define BS_WAVE_MAX 512  // segments up to this size are sorted by one wave

// Persistent workgroups of four waves take segments four at a time (the
// first four by grid position, the rest from a counter): each wave sorts
// one segment of up to BS_WAVE_MAX keys on its own, then the workgroup sorts
// the larger ones of the four together: a bitonic network over four rows of
// 256 (element i in row i / 256 of thread i % 256) up to BS_LDS keys, with
// equal keys put in slot order afterwards, or radix passes beyond.
__global__ __launch_bounds__(256) void k_bsort_local(
    uint64_t *__restrict__ k1, uint32_t *__restrict__ v1, uint64_t *__restrict__ k0,
    uint32_t *__restrict__ v0, const uint2 *__restrict__ seg, uint32_t *__restrict__ ctl,
    const uint32_t *__restrict__ starts) {
  __shared__ uint64_t sk[BS_LDS];
  __shared__ uint32_t sv[BS_LDS];
  __shared__ uint32_t s_i;
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tid >> 6));
  const uint32_t nseg = ctl[0];
  bool first = true;
  for (;;) {
    if (tid == 0) s_i = first ? 4u * blockIdx.x : 4u * gridDim.x + atomicAdd(&ctl[1], 4u);
    first = false;
    __syncthreads();
    const uint32_t i0 = s_i;
    __syncthreads();
    if (i0 >= nseg) break;  // uniform over the block
    {
      const uint32_t i = i0 + w;
      if (i < nseg) {
        uint32_t a, e;
        bs_segment(seg, starts, nseg, i, a, e);
        const uint32_t m = e - a;
        if (m == 1) {
          if (lane == 0) { k0[a] = k1[a]; v0[a] = v1[a]; }
        } else if (m <= 64) {
          bs_wave_sort<1>(k1, v1, k0, v0, a, m, lane);
        } else if (m <= 128) {
          bs_wave_sort<2>(k1, v1, k0, v0, a, m, lane);
        } else if (m <= 256) {
          bs_wave_sort<4>(k1, v1, k0, v0, a, m, lane);
        } else if (m <= BS_WAVE_MAX) {
          bs_wave_sort<8>(k1, v1, k0, v0, a, m, lane);
        }
      }
    }
    for (uint32_t q = 0; q < 4; ++q) {
      const uint32_t i = i0 + q;
      if (i >= nseg) break;  // uniform
      uint32_t a, e;
      bs_segment(seg, starts, nseg, i, a, e);
      const uint32_t m = e - a;
      if (m <= BS_WAVE_MAX) continue;  // uniform: done by a wave above
      if (m > BS_LDS) {
        // the LDS arrays serve as the radix scratch of the large-bucket path
        uint32_t *scratch = reinterpret_cast<uint32_t *>(sk);
        bs_big(k1, v1, k0, v0, a, e, scratch, scratch + 256);
        __syncthreads();  // LDS reused by the next segment
        continue;
      }
      uint32_t n2 = 256;
      while (n2 < m) n2 <<= 1;
      const int nr = (int)(n2 >> 8);  // rows in use (1, 2 or 4)
      uint64_t k[4];
      uint32_t v[4];
      // removed particles' all-ones keys become all-ones minus one, so that
      // the padding (all ones) sorts after them (live keys are below 2^63)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t j = (uint32_t)r * 256 + tid;
        const bool in = r < nr && j < m;
        const uint64_t kk = in ? k1[a + j] : RB_KEY_DEAD;
        k[r] = in && kk == RB_KEY_DEAD ? RB_KEY_DEAD - 1ull : kk;
        v[r] = in ? v1[a + j] : 0xFFFFFFFFu;
      }
      // the network orders the keys; equal keys (rare) are put in slot order
      // afterwards
      for (uint32_t size = 2; size <= n2; size <<= 1) {
        for (uint32_t stride = size >> 1; stride >= 64; stride >>= 1) {
          if (stride >= 256) {  // partner in another row of the same thread
            const int rs = (int)(stride >> 8);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int rr = r ^ rs;
              if (r < nr && r < rr) {
                const bool asc = ((((uint32_t)r * 256 + tid) & size) == 0);
                if ((k[rr] < k[r]) == asc) {
                  const uint64_t tk = k[r]; k[r] = k[rr]; k[rr] = tk;
                  const uint32_t tv = v[r]; v[r] = v[rr]; v[rr] = tv;
                }
              }
            }
          } else {  // partner in another wave: through LDS
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (r < nr) { sk[r * 256 + tid] = k[r]; sv[r * 256 + tid] = v[r]; }
            __syncthreads();
            uint64_t pk[4];
            uint32_t pv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (r < nr) {
                pk[r] = sk[(r * 256 + tid) ^ stride];
                pv[r] = sv[(r * 256 + tid) ^ stride];
              }
            __syncthreads();
            bs_take(k, v, pk, pv, nr, tid, size, stride);
          }
        }
        // partners inside the wave: constant strides
        if (size >= 64) bs_stage_wave<32>(k, v, nr, tid, size);
        if (size >= 32) bs_stage_wave<16>(k, v, nr, tid, size);
        if (size >= 16) bs_stage_wave<8>(k, v, nr, tid, size);
        if (size >= 8) bs_stage_wave<4>(k, v, nr, tid, size);
        if (size >= 4) bs_stage_wave<2>(k, v, nr, tid, size);
        bs_stage_wave<1>(k, v, nr, tid, size);
      }
      // equal keys in slot order: odd-even passes over runs of equal keys
      // until nothing moves (at most the run length)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (r < nr) { sk[r * 256 + tid] = k[r]; sv[r * 256 + tid] = v[r]; }
      __syncthreads();
      bool ties = false;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t j = (uint32_t)r * 256 + tid;
        if (r < nr && j > 0 && j < m && sk[j - 1] == sk[j]) ties = true;
      }
      if (__syncthreads_or(ties)) {
        for (uint32_t it = 0; it < m; ++it) {
          bool moved = false;
          for (int ph = 0; ph < 2; ++ph) {
            for (uint32_t j = 2 * tid + (uint32_t)ph; j + 1 < m; j += 2 * blockDim.x) {
              if (sk[j] == sk[j + 1] && sv[j + 1] < sv[j]) {
                const uint32_t t = sv[j]; sv[j] = sv[j + 1]; sv[j + 1] = t;
                moved = true;
              }
            }
            __syncthreads();
          }
          if (!__syncthreads_or(moved)) break;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (r < nr) { k[r] = sk[r * 256 + tid]; v[r] = sv[r * 256 + tid]; }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t j = (uint32_t)r * 256 + tid;
        if (r < nr && j < m) {
          k0[a + j] = k[r] == RB_KEY_DEAD - 1ull ? RB_KEY_DEAD : k[r];
          v0[a + j] = v[r];
        }
      }
      __syncthreads();  // LDS reused by the next segment
    }
  }
}

hipError_t launch_bsort(rb_ctx *c) {
  const uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bsort_scan, dim3(c->P), dim3(1024), 0, c->stream, c->d_bcnt, c->d_bcur,
                     c->d_starts, c->d_bseg, c->d_bctl);
  hipLaunchKernelGGL(k_bsort_scatter, dim3(rb_div_up(n, 256)), dim3(256), 0, c->stream,
                     c->d_key[0], c->d_idx[0], c->d_key[1], c->d_idx[1], c->d_starts, c->P, n,
                     c->d_bcur, c->d_bctl);
  const unsigned grid = (unsigned)std::min<uint64_t>(1024, rb_div_up(n, 256) + c->P);
  hipLaunchKernelGGL(k_bsort_local, dim3(grid), dim3(256), 0, c->stream, c->d_key[1],
                     c->d_idx[1], c->d_key[0], c->d_idx[0], c->d_bseg, c->d_bctl, c->d_starts);
  return hipGetLastError();
}
