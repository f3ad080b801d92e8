// k_sort.hip -- stable LSD radix sort of (Morton key, slot) pairs inside every
// patch: 6 passes of 11-bit digits over the 64-bit keys.
//
// A tile is a run of consecutive slots of one patch handled by one wave.
// Digit counts per tile live in [patch][digit][tile-in-patch] histograms,
// double-buffered: the kernel that writes the keys counts the first digit
// (rb_hist_add), and each scatter counts the next pass's digit at the key's
// destination tile.  Per pass:
//   rowscan -- exclusive scan along every (patch, digit) row, row totals;
//              zeroes the same row of the other histogram;
//   scatter -- the wave ranks its keys 64 at a time: the lanes holding the
//              same digit find each other with 11 ballots, a lane's rank is
//              the count of equal-digit lanes below it plus the digit's
//              running count in LDS, so equal keys keep their order.
// Sentinel keys of removed particles (all ones) sort last.
#include "rb_internal.h"

#define SORT_BITS 11
#define SORT_BINS (1 << SORT_BITS)
#define SORT_PASSES 6

// block-wide inclusive scan of one value per thread (256 threads)
__device__ __forceinline__ uint32_t block_incl_scan256(uint32_t v, uint32_t *wsum,
                                                       uint32_t &total) {
  const uint32_t lane = rb_lane(), w = threadIdx.x >> 6;
  uint32_t incl = rb_wave_incl_scan(v);
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t add = 0;
  for (uint32_t k = 0; k < w; ++k) add += wsum[k];
  total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  __syncthreads();
  return incl + add;
}

// exclusive scan of rows; one 256-thread block per row.
//   mode 0 (sort): r = patch * SORT_BINS + digit, base = SORT_BINS t0 + digit nt
//   mode 1 (topology): r = kind * 22 + level, base = r * n_tiles, len = n_tiles
__global__ __launch_bounds__(256) void k_rowscan(uint32_t *__restrict__ data,
                                                 const uint32_t *__restrict__ patch_tile0,
                                                 uint32_t n_tiles, int mode,
                                                 uint32_t *__restrict__ row_tot,
                                                 uint32_t *__restrict__ zero_next) {
  __shared__ uint32_t wsum[4];
  const uint32_t r = blockIdx.x;
  size_t base;
  uint32_t len;
  if (mode == 0) {
    const uint32_t p = r / SORT_BINS, d = r % SORT_BINS;
    const uint32_t t0 = patch_tile0[p], nt = patch_tile0[p + 1] - t0;
    base = (size_t)SORT_BINS * t0 + (size_t)d * nt;
    len = nt;
  } else {
    base = (size_t)r * n_tiles;
    len = n_tiles;
  }
  uint32_t carry = 0;
  for (uint32_t off = 0; off < len; off += 256) {
    const uint32_t i = off + threadIdx.x;
    const uint32_t v = (i < len) ? data[base + i] : 0u;
    uint32_t tot;
    const uint32_t incl = block_incl_scan256(v, wsum, tot);
    if (i < len) {
      data[base + i] = carry + incl - v;
      if (zero_next) zero_next[base + i] = 0u;
    }
    carry += tot;
  }
  if (threadIdx.x == 0) row_tot[r] = carry;
}

// lanes of the wave holding the same 11-bit digit
__device__ __forceinline__ uint64_t wave_match11(uint32_t d, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < SORT_BITS; ++bit) {
    const bool on = (d >> bit) & 1u;
    const uint64_t m = __ballot(valid && on);
    peers &= on ? m : ~m;
  }
  return peers;
}

__global__ __launch_bounds__(64) void k_sort_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
    const uint32_t *__restrict__ tile_start, const uint32_t *__restrict__ tile_end,
    const uint32_t *__restrict__ tile_patch, const uint32_t *__restrict__ patch_tile0,
    const uint32_t *__restrict__ starts, const uint32_t *__restrict__ hist,
    const uint32_t *__restrict__ digit_tot, int shift, uint32_t tile,
    uint32_t *__restrict__ hist_next) {
  __shared__ uint32_t base[SORT_BINS];
  const uint32_t b = blockIdx.x, lane = threadIdx.x;
  const uint32_t p = tile_patch[b], t0 = patch_tile0[p], nt = patch_tile0[p + 1] - t0;
  // base[d] = patch start + (keys of the patch with a smaller digit) +
  // (keys with digit d in earlier tiles of the patch)
  {
    constexpr uint32_t PER = SORT_BINS / 64;
    const uint32_t *tot = digit_tot + (size_t)p * SORT_BINS + lane * PER;
    uint32_t v[PER];
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < PER; ++k) { v[k] = tot[k]; sum += v[k]; }
    uint32_t run = rb_wave_incl_scan(sum) - sum + starts[p];
    const uint32_t *hb = hist + (size_t)SORT_BINS * t0 + (b - t0);
#pragma unroll
    for (uint32_t k = 0; k < PER; ++k) {
      const uint32_t d = lane * PER + k;
      base[d] = run + hb[(size_t)d * nt];
      run += v[k];
    }
  }
  __syncthreads();
  const uint32_t s0 = tile_start[b], s1 = tile_end[b];
  for (uint32_t r0 = s0; r0 < s1; r0 += 64) {
    const uint32_t s = r0 + lane;
    const bool valid = s < s1;
    const uint64_t k = valid ? kin[s] : 0ull;
    const uint32_t v = valid ? vin[s] : 0u;
    const uint32_t d = (uint32_t)(k >> shift) & (SORT_BINS - 1);
    const uint64_t peers = wave_match11(d, valid);
    const uint32_t rank = rb_mbcnt(peers);
    uint32_t pos = 0;
    if (valid) pos = base[d] + rank;
    // every lane has read its digit's base before the lowest lane of each
    // digit group advances it (LDS operations of one wave stay in order)
    __syncthreads();
    if (valid && rank == 0) base[d] += (uint32_t)__popcll(peers);
    if (valid) {
      kout[pos] = k;
      vout[pos] = v;
      if (hist_next) {
        const uint32_t dn = (uint32_t)(k >> (shift + SORT_BITS)) & (SORT_BINS - 1);
        const uint32_t tl = (pos - starts[p]) / tile;
        atomicAdd(&hist_next[(size_t)SORT_BINS * t0 + (size_t)dn * nt + tl], 1u);
      }
    }
    __syncthreads();
  }
}

hipError_t launch_sort(rb_ctx *c) {
  if (c->n_tiles == 0) return hipSuccess;
  int src = 0;
  for (int pass = 0; pass < SORT_PASSES; ++pass) {
    const int shift = SORT_BITS * pass;
    uint32_t *h = c->d_hist[pass & 1], *hn = c->d_hist[(pass + 1) & 1];
    const bool last = pass + 1 == SORT_PASSES;
    hipLaunchKernelGGL(k_rowscan, dim3(SORT_BINS * c->P), dim3(256), 0, c->stream, h,
                       c->d_patch_tile0, c->n_tiles, 0, c->d_digit_tot, hn);
    hipLaunchKernelGGL(k_sort_scatter, dim3(c->n_tiles), dim3(64), 0, c->stream,
                       c->d_key[src], c->d_idx[src], c->d_key[1 - src], c->d_idx[1 - src],
                       c->d_tile_start, c->d_tile_end, c->d_tile_patch, c->d_patch_tile0,
                       c->d_starts, h, c->d_digit_tot, shift, c->tile, last ? nullptr : hn);
    src = 1 - src;
  }
  return hipGetLastError();  // an even number of passes: the result is in buffer 0
}

hipError_t launch_rowscan_levels(rb_ctx *c) {
  hipLaunchKernelGGL(k_rowscan, dim3(2 * RB_NLEV), dim3(256), 0, c->stream, c->d_cnt,
                     c->d_patch_tile0, c->n_tiles, 1, c->d_lev_tot, (uint32_t *)nullptr);
  return hipGetLastError();
}
