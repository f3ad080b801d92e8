// k_sort.hip -- stable LSD radix sort of (Morton key, slot) pairs inside every
// patch, for large systems: 8 passes of 8-bit digits over the 64-bit keys,
// one launch per pass.  (Small systems use the bucket sort of k_bsort.hip.)
//
// Digit totals of all eight passes come from one counting launch
// (k_sort_hist), per patch.  Each pass (k_sort_pass) then works tile by tile
// (256 threads, 256 * R consecutive slots of one patch) in a single launch:
//   rank   -- every wave ranks its R rows of 64 keys in order: the lanes
//             holding the same digit find each other with 8 ballots, a
//             lane's rank is the count of equal-digit lanes below it plus
//             the digit's running count of the wave (LDS), so equal keys keep
//             their order;
//   prefix -- per digit, the tile publishes its count and looks back over
//             the preceding tiles of its patch for their published sums
//             (decoupled look-back: tiles take their index from a device
//             counter, so every tile waited on is already running);
//   scatter -- slot = patch start + keys of smaller digits in the patch +
//             keys of this digit in earlier tiles + earlier waves + rank.
// Look-back words carry a tag (sort number and pass), so stale words from
// earlier passes or sorts never match and nothing needs clearing between
// passes.  A wait that does not end within a bounded number of polls sets an
// error bit and gives up, so every wave exits.
// Sentinel keys of removed particles (all ones) sort last.
#include "rb_internal.h"

#define SORT_BITS 8
#define SORT_BINS 256
#define SORT_PASSES 8
#define LB_AGG 1ull
#define LB_PREFIX 2ull
#define LB_POLLS (1u << 22)
#define LB_WIN 32  // predecessors read per look-back step

__device__ __forceinline__ uint64_t lb_pack(uint32_t tag, uint64_t flag, uint32_t count) {
  return ((uint64_t)tag << 34) | (flag << 32) | (uint64_t)count;
}

// lanes of the wave holding the same 8-bit digit
__device__ __forceinline__ uint64_t wave_match8(uint32_t d, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < SORT_BITS; ++bit) {
    const bool on = (d >> bit) & 1u;
    const uint64_t m = __ballot(valid && on);
    peers &= on ? m : ~m;
  }
  return peers;
}

// Digit totals of every pass, per patch: block b counts the sort tiles
// [b T, (b + 1) T) in LDS and adds its non-zero bins to the patch's totals.
// Each thread loads 8 keys at a time (loads in flight together); a digit
// that the whole wave shares is added with one LDS atomic.
// Block 0 also resets the first pass's tile counter.
__global__ __launch_bounds__(256) void k_sort_hist(
    const uint64_t *__restrict__ key, const uint32_t *__restrict__ tile_start,
    const uint32_t *__restrict__ tile_end, const uint32_t *__restrict__ tile_patch,
    uint32_t n_tiles, uint32_t tiles_per_block, uint32_t P, uint32_t *__restrict__ stot,
    uint32_t *__restrict__ sctl) {
  __shared__ uint32_t h[SORT_PASSES * SORT_BINS];
  const uint32_t tid = threadIdx.x;
  const uint32_t epoch = sctl[0];
  uint32_t *tot = stot + (size_t)(epoch & 1u) * P * (SORT_PASSES * SORT_BINS);
  if (blockIdx.x == 0 && tid == 0) sctl[1] = 0;
  const uint32_t t0 = blockIdx.x * tiles_per_block;
  const uint32_t t1 = min(t0 + tiles_per_block, n_tiles);
  for (uint32_t i = tid; i < SORT_PASSES * SORT_BINS; i += 256) h[i] = 0;
  __syncthreads();
  uint32_t cur = (t0 < t1) ? tile_patch[t0] : 0u;
  auto flush = [&](uint32_t p) {
    for (uint32_t i = tid; i < SORT_PASSES * SORT_BINS; i += 256) {
      const uint32_t v = h[i];
      if (v) atomicAdd(&tot[(size_t)p * (SORT_PASSES * SORT_BINS) + i], v);
      h[i] = 0;
    }
  };
  for (uint32_t t = t0; t < t1; ++t) {
    const uint32_t p = tile_patch[t];
    if (p != cur) {  // uniform: every thread reads the same tile entry
      __syncthreads();
      flush(cur);
      __syncthreads();
      cur = p;
    }
    const uint32_t sa = tile_start[t], s1 = tile_end[t];
    for (uint32_t sb = sa; sb < s1; sb += 8 * 256) {
      uint64_t k8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t s = sb + u * 256 + tid;
        k8[u] = (s < s1) ? key[s] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool valid = sb + u * 256 + tid < s1;
        const uint64_t vm = __ballot(valid);
        if (vm == 0) continue;  // uniform over the wave
        const int first = __ffsll((long long)vm) - 1;
#pragma unroll
        for (int q = 0; q < SORT_PASSES; ++q) {
          const uint32_t d = (uint32_t)(k8[u] >> (SORT_BITS * q)) & (SORT_BINS - 1);
          // a digit shared by the whole wave (the high digits of nearby
          // keys): one atomic for all lanes
          const uint32_t d0 = (uint32_t)__shfl((int)d, first, 64);
          if (__ballot(valid && d == d0) == vm) {
            if (rb_lane() == (uint32_t)first)
              atomicAdd(&h[q * SORT_BINS + d0], (uint32_t)__popcll(vm));
          } else if (valid) {
            atomicAdd(&h[q * SORT_BINS + d], 1u);
          }
        }
      }
    }
  }
  __syncthreads();
  if (t0 < t1) flush(cur);
}

template <int R>
__global__ __launch_bounds__(256) void k_sort_pass(
    int pass, const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
    const uint32_t *__restrict__ tile_start, const uint32_t *__restrict__ tile_end,
    const uint32_t *__restrict__ tile_patch, const uint32_t *__restrict__ patch_tile0,
    const uint32_t *__restrict__ starts, uint32_t P, uint32_t n_tiles,
    uint32_t *__restrict__ stot, uint64_t *__restrict__ desc, uint32_t *__restrict__ sctl,
    uint32_t *__restrict__ err) {
  __shared__ uint32_t cnt[4][SORT_BINS];  // per-wave digit counts, then offsets
  __shared__ uint32_t base[SORT_BINS];
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t s_tile;
  const uint32_t tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int shift = SORT_BITS * pass;
  if (tid == 0) {
    const uint32_t t = atomicAdd(&sctl[1 + (pass & 1)], 1u);
    // the next pass's counter is idle until this launch ends
    if (t == 0) sctl[1 + ((pass + 1) & 1)] = 0;
    s_tile = t;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) cnt[q][tid] = 0;
  __syncthreads();
  const uint32_t t = s_tile;
  if (t >= n_tiles) {  // a counter that was not reset: report, touch nothing
    if (tid == 0) atomicOr(err, RB_ERR_SORT);
    return;  // uniform over the block
  }
  const uint32_t p = tile_patch[t], s0 = tile_start[t], s1 = tile_end[t];
  const bool first = (t == patch_tile0[p]);
  const uint32_t epoch = sctl[0];
  const uint32_t tag = (epoch * SORT_PASSES + (uint32_t)pass) & 0x3FFFFFFFu;
  uint32_t *tot_cur = stot + (size_t)(epoch & 1u) * P * (SORT_PASSES * SORT_BINS);
  // the other totals buffer is counted into by the next sort: clear this
  // patch's part (once per patch, in the first pass)
  if (pass == 0 && first) {
    uint32_t *tot_next = stot + (size_t)((epoch + 1u) & 1u) * P * (SORT_PASSES * SORT_BINS) +
                         (size_t)p * (SORT_PASSES * SORT_BINS);
    for (uint32_t i = tid; i < SORT_PASSES * SORT_BINS; i += 256) tot_next[i] = 0;
  }

  // rank: wave w owns rows [w R, (w + 1) R) of the tile
  uint64_t kk[R];
  uint32_t vv[R], lr[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t s = s0 + (w * R + r) * 64 + lane;
    const bool valid = s < s1;
    kk[r] = valid ? kin[s] : 0ull;
    vv[r] = valid ? vin[s] : 0u;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t s = s0 + (w * R + r) * 64 + lane;
    const bool valid = s < s1;
    const uint32_t d = (uint32_t)(kk[r] >> shift) & (SORT_BINS - 1);
    const uint64_t peers = wave_match8(d, valid);
    const uint32_t rank = rb_mbcnt(peers);
    // one LDS read for all lanes, then the lowest lane of each digit group
    // advances the count with the value it read (data-dependent: the read
    // of every lane precedes the write)
    const uint32_t b0 = valid ? cnt[w][d] : 0u;
    lr[r] = b0 + rank;
    if (valid && rank == 0) cnt[w][d] = b0 + (uint32_t)__popcll(peers);
  }
  __syncthreads();

  // per digit (thread tid): counts of the tile and offsets of the waves
  const uint32_t c0 = cnt[0][tid], c1 = cnt[1][tid], c2 = cnt[2][tid], c3 = cnt[3][tid];
  const uint32_t tile_cnt = c0 + c1 + c2 + c3;
  cnt[0][tid] = 0;
  cnt[1][tid] = c0;
  cnt[2][tid] = c0 + c1;
  cnt[3][tid] = c0 + c1 + c2;
  uint64_t *my = desc + (size_t)t * SORT_BINS + tid;
  uint32_t excl = 0;
  if (first) {
    __hip_atomic_store(my, lb_pack(tag, LB_PREFIX, tile_cnt), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  } else {
    __hip_atomic_store(my, lb_pack(tag, LB_AGG, tile_cnt), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    // read the predecessors LB_WIN at a time (loads in flight together),
    // then take them in order up to the first published prefix
    const uint32_t t_first = patch_tile0[p];
    uint32_t j = t;  // tiles [t_first, j) are still to be read
    uint32_t polls = 0;
    bool done = false;
    while (!done) {
      const uint32_t nwin = min((uint32_t)LB_WIN, j - t_first);
      if (nwin == 0) {  // no prefix before the patch's first tile: report, stop
        atomicOr(err, RB_ERR_SORT);
        break;
      }
      uint64_t x[LB_WIN];
#pragma unroll
      for (int q = 0; q < LB_WIN; ++q)
        if ((uint32_t)q < nwin)
          x[q] = __hip_atomic_load(desc + (size_t)(j - 1 - q) * SORT_BINS + tid,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
      for (int q = 0; q < LB_WIN; ++q) {
        if (done || (uint32_t)q >= nwin) continue;
        uint64_t v = x[q];
        // wait for this predecessor to publish (bounded)
        while (!((uint32_t)(v >> 34) == tag && ((v >> 32) & 3ull) != 0)) {
          if (++polls > LB_POLLS) {
            atomicOr(err, RB_ERR_SORT);
            v = lb_pack(tag, LB_PREFIX, 0u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          v = __hip_atomic_load(desc + (size_t)(j - 1 - q) * SORT_BINS + tid, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
        }
        excl += (uint32_t)v;
        if (((v >> 32) & 3ull) == LB_PREFIX) done = true;
      }
      j -= nwin;  // the patch's first tile publishes a prefix: j never passes it
    }
    __hip_atomic_store(my, lb_pack(tag, LB_PREFIX, excl + tile_cnt), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  // keys of smaller digits in the patch: exclusive scan of the totals
  const uint32_t dt = tot_cur[(size_t)p * (SORT_PASSES * SORT_BINS) + pass * SORT_BINS + tid];
  const uint32_t incl = rb_wave_incl_scan(dt);
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t add = 0;
  for (uint32_t q = 0; q < w; ++q) add += wsum[q];
  base[tid] = starts[p] + add + incl - dt + excl;
  __syncthreads();

  // scatter
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t s = s0 + (w * R + r) * 64 + lane;
    if (s < s1) {
      const uint32_t d = (uint32_t)(kk[r] >> shift) & (SORT_BINS - 1);
      const uint32_t pos = base[d] + cnt[w][d] + lr[r];
      kout[pos] = kk[r];
      vout[pos] = vv[r];
    }
  }
}

hipError_t launch_sort(rb_ctx *c) {
  if (c->sort_small) return launch_bsort(c);
  if (c->n_stiles == 0) return hipSuccess;
  const uint32_t tpb = c->sort_hist_tiles;
  hipLaunchKernelGGL(k_sort_hist, dim3(rb_div_up(c->n_stiles, tpb)), dim3(256), 0, c->stream,
                     c->d_key[0], c->d_stile_start, c->d_stile_end, c->d_stile_patch,
                     c->n_stiles, tpb, c->P, c->d_stot, c->d_sctl);
  int src = 0;
  for (int pass = 0; pass < SORT_PASSES; ++pass) {
#define RB_SORT_ARGS                                                                       \
  pass, c->d_key[src], c->d_idx[src], c->d_key[1 - src], c->d_idx[1 - src], c->d_stile_start, \
      c->d_stile_end, c->d_stile_patch, c->d_spatch_tile0, c->d_starts, c->P, c->n_stiles,    \
      c->d_stot, c->d_sdesc, c->d_sctl, c->d_err
    const dim3 grid(c->n_stiles), block(256);
    switch (c->sort_rows) {
      case 1: hipLaunchKernelGGL(k_sort_pass<1>, grid, block, 0, c->stream, RB_SORT_ARGS); break;
      case 2: hipLaunchKernelGGL(k_sort_pass<2>, grid, block, 0, c->stream, RB_SORT_ARGS); break;
      case 4: hipLaunchKernelGGL(k_sort_pass<4>, grid, block, 0, c->stream, RB_SORT_ARGS); break;
      default: hipLaunchKernelGGL(k_sort_pass<8>, grid, block, 0, c->stream, RB_SORT_ARGS); break;
    }
#undef RB_SORT_ARGS
    src = 1 - src;
  }
  return hipGetLastError();  // an even number of passes: the result is in buffer 0
}

// ---------------------------------------------------------------------------
// exclusive scan of the topology's per-tile level counts: one 256-thread
// block per (kind, level) row of n_tiles entries; row totals to row_tot.
__global__ __launch_bounds__(256) void k_rowscan(uint32_t *__restrict__ data, uint32_t n_tiles,
                                                 uint32_t *__restrict__ row_tot,
                                                 const uint32_t *__restrict__ reuse) {
  __shared__ uint32_t wsum[4];
  if (reuse && *reuse == 0u) return;  // the step keeps the last tree
  const uint32_t r = blockIdx.x, tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const size_t base = (size_t)r * n_tiles;
  uint32_t carry = 0;
  // 1024 entries per round: four consecutive ones per thread, summed in the
  // thread, then the threads' totals scanned across the block
  for (uint32_t off = 0; off < n_tiles; off += 1024) {
    const uint32_t i0 = off + 4 * tid;
    uint32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (i0 + k < n_tiles) ? data[base + i0 + k] : 0u;
    const uint32_t s1 = v[0], s2 = s1 + v[1], s3 = s2 + v[2], s4 = s3 + v[3];
    const uint32_t incl = rb_wave_incl_scan(s4);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t add = 0;
    for (uint32_t q = 0; q < w; ++q) add += wsum[q];
    const uint32_t tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    const uint32_t ex = carry + add + incl - s4;  // before the thread's first entry
    const uint32_t out[4] = {ex, ex + s1, ex + s2, ex + s3};
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (i0 + k < n_tiles) data[base + i0 + k] = out[k];
    carry += tot;
  }
  if (tid == 0) row_tot[r] = carry;
}

hipError_t launch_rowscan_levels(rb_ctx *c, const uint32_t *reuse) {
  hipLaunchKernelGGL(k_rowscan, dim3(2 * RB_NLEV), dim3(256), 0, c->stream, c->d_cnt,
                     c->n_tiles, c->d_lev_tot, reuse);
  return hipGetLastError();
}
