// k_build.hip -- octree construction on the GPU (Sect. 4.2 of the paper):
// Morton keys, stable LSD radix sort, permutation into Morton order,
// canonical level-ordered topology and bottom-up moments.
//
// The paper builds its tree by inserting particles one at a time.  Here the
// same tree -- every cell whose parent holds more than leaf_size particles,
// leaves of at most leaf_size particles except on level 21 -- is derived from
// the sorted keys directly: a node is a run of sorted particles sharing an
// octal key prefix, and which runs are nodes follows from the longest common
// prefixes (LCPs) of neighbouring keys.  Nodes are numbered level by level,
// patch by patch, and by prefix inside a level, so children are contiguous.
#include "rb_internal.h"

// ---------------------------------------------------------------------------
// keys of the caller's particles (no drift): key = interleaved quantised
// coordinates, x bit weighing 4, y 2, z 1 in every octal digit.

__global__ __launch_bounds__(256) void k_keys(const double *__restrict__ x,
                                              const double *__restrict__ y,
                                              const double *__restrict__ z,
                                              const PatchInfo *__restrict__ patch,
                                              const uint32_t *__restrict__ starts,
                                              uint32_t P, uint32_t n, int open_xy,
                                              uint64_t *__restrict__ key,
                                              uint32_t *__restrict__ idx,
                                              uint32_t *__restrict__ err) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  uint32_t p = (P == 1) ? 0 : rb_patch_of(starts, P, s);
  const PatchInfo pi = patch[p];
  double xs = x[s], ys = y[s], zs = z[s];
  uint32_t qx, qy, qz;
  bool okx = rb_quantise(xs, pi.x0[0], pi.W, pi.S, qx);
  bool oky = rb_quantise(ys, pi.x0[1], pi.W, pi.S, qy);
  bool okz = rb_quantise(zs, pi.x0[2], pi.W, pi.S, qz);
  uint64_t k = RB_KEY_DEAD;
  if (okx && oky && okz) {
    k = rb_key(qx, qy, qz);
  } else if (!open_xy && !(isnan(xs) || isnan(ys) || isnan(zs)) && (!okx || !oky)) {
    atomicOr(err, RB_ERR_OUTSIDE);  // a periodic axis must have been wrapped
  }
  key[s] = k;
  idx[s] = s;
}

hipError_t launch_keys(rb_ctx *c, const double *x, const double *y, const double *z,
                       double) {
  uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_keys, dim3(rb_div_up(n, 256)), dim3(256), 0, c->stream, x, y, z,
                     c->d_patch, c->d_starts, c->P, n, c->p.boundary == RB_OPEN ? 1 : 0,
                     c->d_key[0], c->d_idx[0], c->d_err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (key, slot) pairs inside every patch, 8 passes of
// 8 bits.  Tiles of RB_TILE slots never straddle a patch.  Per pass:
//   hist    -- digit counts per tile, stored [patch][digit][tile-in-patch];
//   rowscan -- exclusive scan along every (patch, digit) row, row totals;
//   scatter -- in-tile stable ranks from wave ballots, writes to
//              patch start + digits below + earlier tiles + rank.

__global__ __launch_bounds__(256) void k_sort_hist(const uint64_t *__restrict__ key,
                                                   const uint32_t *__restrict__ tile_start,
                                                   const uint32_t *__restrict__ tile_end,
                                                   const uint32_t *__restrict__ tile_patch,
                                                   const uint32_t *__restrict__ patch_tile0,
                                                   int shift, uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[256];
  const uint32_t b = blockIdx.x, tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const uint32_t s0 = tile_start[b], s1 = tile_end[b];
  for (uint32_t s = s0 + tid; s < s1; s += 256)
    atomicAdd(&h[(uint32_t)(key[s] >> shift) & 255u], 1u);
  __syncthreads();
  const uint32_t p = tile_patch[b], t0 = patch_tile0[p], nt = patch_tile0[p + 1] - t0;
  hist[256u * t0 + tid * nt + (b - t0)] = h[tid];
}

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

// exclusive scan of rows of `len` entries; one 256-thread block per row.
// Row r covers data[base(r) .. base(r) + len(r)).
//   mode 0 (sort): r = patch * 256 + digit, base = 256 t0 + digit nt, len = nt
//   mode 1 (topology): r = kind * 22 + level, base = r * n_tiles, len = n_tiles
__global__ __launch_bounds__(256) void k_rowscan(uint32_t *__restrict__ data,
                                                 const uint32_t *__restrict__ patch_tile0,
                                                 uint32_t n_tiles, int mode,
                                                 uint32_t *__restrict__ row_tot) {
  __shared__ uint32_t wsum[4];
  const uint32_t r = blockIdx.x;
  uint32_t base, len;
  if (mode == 0) {
    uint32_t p = r >> 8, d = r & 255u;
    uint32_t t0 = patch_tile0[p], nt = patch_tile0[p + 1] - t0;
    base = 256u * t0 + d * nt;
    len = nt;
  } else {
    base = r * n_tiles;
    len = n_tiles;
  }
  uint32_t carry = 0;
  for (uint32_t off = 0; off < len; off += 256) {
    uint32_t i = off + threadIdx.x;
    uint32_t v = (i < len) ? data[base + i] : 0u;
    uint32_t tot;
    uint32_t incl = block_incl_scan256(v, wsum, tot);
    if (i < len) data[base + i] = carry + incl - v;
    carry += tot;
  }
  if (threadIdx.x == 0) row_tot[r] = carry;
}

// 8-bit digit peers of this lane inside the wave
__device__ __forceinline__ uint64_t wave_match8(uint32_t d, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    bool on = (d >> bit) & 1u;
    uint64_t b = __ballot(valid && on);
    peers &= on ? b : ~b;
  }
  return peers;
}

__global__ __launch_bounds__(256) void k_sort_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
    const uint32_t *__restrict__ tile_start, const uint32_t *__restrict__ tile_end,
    const uint32_t *__restrict__ tile_patch, const uint32_t *__restrict__ patch_tile0,
    const uint32_t *__restrict__ starts, const uint32_t *__restrict__ hist,
    const uint32_t *__restrict__ digit_tot, int shift) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[4][256];
  __shared__ uint32_t wsum[4];
  const uint32_t b = blockIdx.x, tid = threadIdx.x, w = tid >> 6;
  const uint32_t p = tile_patch[b], t0 = patch_tile0[p], nt = patch_tile0[p + 1] - t0;
  {
    uint32_t v = digit_tot[p * 256u + tid], tot;
    uint32_t incl = block_incl_scan256(v, wsum, tot);
    base[tid] = starts[p] + (incl - v) + hist[256u * t0 + tid * nt + (b - t0)];
    run[tid] = 0;
  }
  const uint32_t s0 = tile_start[b], s1 = tile_end[b];
  for (uint32_t r0 = s0; r0 < s1; r0 += 256) {
    const uint32_t s = r0 + tid;
    const bool valid = s < s1;
    uint64_t k = valid ? kin[s] : 0ull;
    uint32_t v = valid ? vin[s] : 0u;
    uint32_t d = (uint32_t)(k >> shift) & 255u;
    wcnt[0][tid] = 0; wcnt[1][tid] = 0; wcnt[2][tid] = 0; wcnt[3][tid] = 0;
    __syncthreads();
    uint64_t peers = wave_match8(d, valid);
    uint32_t rank = rb_mbcnt(peers);
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pre = run[d];
      for (uint32_t q = 0; q < w; ++q) pre += wcnt[q][d];
      uint32_t pos = base[d] + pre + rank;
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
    // the next round's clearing of wcnt is ordered after this read by the
    // barrier that follows the clearing
    __syncthreads();
  }
}

hipError_t launch_sort(rb_ctx *c) {
  if (c->n_tiles == 0) return hipSuccess;
  int src = 0;
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(k_sort_hist, dim3(c->n_tiles), dim3(256), 0, c->stream,
                       c->d_key[src], c->d_tile_start, c->d_tile_end, c->d_tile_patch,
                       c->d_patch_tile0, shift, c->d_hist);
    hipLaunchKernelGGL(k_rowscan, dim3(256u * c->P), dim3(256), 0, c->stream, c->d_hist,
                       c->d_patch_tile0, c->n_tiles, 0, c->d_digit_tot);
    hipLaunchKernelGGL(k_sort_scatter, dim3(c->n_tiles), dim3(256), 0, c->stream,
                       c->d_key[src], c->d_idx[src], c->d_key[1 - src], c->d_idx[1 - src],
                       c->d_tile_start, c->d_tile_end, c->d_tile_patch, c->d_patch_tile0,
                       c->d_starts, c->d_hist, c->d_digit_tot, shift);
    src = 1 - src;
  }
  return hipGetLastError();  // 8 passes: the result is back in buffer 0
}

// ---------------------------------------------------------------------------
// permutation into Morton order

// rb_gravity / rb_tree_build: gather positions and source masses from the
// caller arrays; record the caller slot; count live particles per patch.
__global__ __launch_bounds__(256) void k_permute_gravity(
    const uint64_t *__restrict__ key, const uint32_t *__restrict__ idx,
    const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ m,
    const PatchInfo *__restrict__ patch, const uint32_t *__restrict__ starts, uint32_t P,
    uint32_t n, double *__restrict__ sx, double *__restrict__ sy, double *__restrict__ sz,
    double *__restrict__ msrc, uint32_t *__restrict__ orig, uint32_t *__restrict__ nlive) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  uint32_t p = (P == 1) ? 0 : rb_patch_of(starts, P, s);
  const uint32_t st = starts[p], en = starts[p + 1];
  const uint64_t k = key[s];
  const bool live = k != RB_KEY_DEAD;
  const uint32_t j = idx[s];
  orig[s] = j;
  if (live) {
    sx[s] = x[j];
    sy[s] = y[j];
    sz[s] = z[j];
    msrc[s] = (j - st < patch[p].n_active) ? m[j] : 0.0;
  } else {
    sx[s] = sy[s] = sz[s] = 0.0;
    msrc[s] = 0.0;
  }
  // the first dead key (or the patch end) marks the live count
  if (live && (s + 1 == en || key[s + 1] == RB_KEY_DEAD)) nlive[p] = s + 1 - st;
  if (!live && s == st) nlive[p] = 0;
}

hipError_t launch_permute_gravity(rb_ctx *c, const double *x, const double *y,
                                  const double *z, const double *m, uint32_t) {
  uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  double *const *d = c->d_px[0];
  hipLaunchKernelGGL(k_permute_gravity, dim3(rb_div_up(n, 256)), dim3(256), 0, c->stream,
                     c->d_key[0], c->d_idx[0], x, y, z, m, c->d_patch, c->d_starts, c->P, n,
                     d[0], d[1], d[2], c->d_msrc, c->d_orig[0], c->d_nlive);
  return hipGetLastError();
}

// rb_step: gather the full state from buffer src into buffer dst.
__global__ __launch_bounds__(256) void k_permute_state(
    const uint64_t *__restrict__ key, const uint32_t *__restrict__ idx,
    const double *__restrict__ ax, const double *__restrict__ ay,
    const double *__restrict__ az, const double *__restrict__ avx,
    const double *__restrict__ avy, const double *__restrict__ avz,
    const double *__restrict__ am, const uint32_t *__restrict__ aorig,
    const PatchInfo *__restrict__ patch, const uint32_t *__restrict__ starts, uint32_t P,
    uint32_t n, double *__restrict__ bx, double *__restrict__ by, double *__restrict__ bz,
    double *__restrict__ bvx, double *__restrict__ bvy, double *__restrict__ bvz,
    double *__restrict__ bm, uint32_t *__restrict__ borig, double *__restrict__ msrc,
    uint32_t *__restrict__ nlive) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  uint32_t p = (P == 1) ? 0 : rb_patch_of(starts, P, s);
  const uint32_t st = starts[p], en = starts[p + 1];
  const uint64_t k = key[s];
  const bool live = k != RB_KEY_DEAD;
  const uint32_t j = idx[s];
  const uint32_t o = aorig[j];
  bx[s] = ax[j]; by[s] = ay[j]; bz[s] = az[j];
  bvx[s] = avx[j]; bvy[s] = avy[j]; bvz[s] = avz[j];
  const double mj = am[j];
  bm[s] = mj;
  borig[s] = o;
  msrc[s] = (live && (o - st) < patch[p].n_active) ? mj : 0.0;
  if (live && (s + 1 == en || key[s + 1] == RB_KEY_DEAD)) nlive[p] = s + 1 - st;
  if (!live && s == st) nlive[p] = 0;
}

hipError_t launch_permute_state(rb_ctx *c, int src, int dst) {
  uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  double *const *a = c->d_px[src];
  double *const *b = c->d_px[dst];
  hipLaunchKernelGGL(k_permute_state, dim3(rb_div_up(n, 256)), dim3(256), 0, c->stream,
                     c->d_key[0], c->d_idx[0], a[0], a[1], a[2], a[3], a[4], a[5], a[6],
                     c->d_orig[src], c->d_patch, c->d_starts, c->P, n, b[0], b[1], b[2], b[3],
                     b[4], b[5], b[6], c->d_orig[dst], c->d_msrc, c->d_nlive);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Topology.  For sorted live slot i of a patch with n live particles:
//   c_i    = LCP(key_{i-1}, key_i) in octal digits (unused for i = 0);
//   D_i    = max over windows [j, j + L] containing i of LCP(key_j, key_{j+L}),
//            L = leaf_size (a window of L + 1 particles shares D_i digits);
//   leaf_i = min(D_i + 1, 21), or 0 when n <= L (the root is the leaf).
// The run of particles at level l holding i is a node exactly for
// l <= leaf_i, and a leaf for l = leaf_i.  Runs starting at i are the
// levels (c_i, leaf_i] (all of [0, leaf_0] for i = 0); runs ending at i are
// (c_{i+1}, leaf_i] ([0, leaf_i] for the last particle).  The k-th start and
// the k-th end on a level belong to the same node.

__global__ __launch_bounds__(256) void k_topo_leaf(const uint64_t *__restrict__ key,
                                                   const uint32_t *__restrict__ starts,
                                                   const uint32_t *__restrict__ nlive,
                                                   uint32_t P, uint32_t n, int L,
                                                   uint8_t *__restrict__ lcp,
                                                   uint8_t *__restrict__ leaf) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  uint32_t p = (P == 1) ? 0 : rb_patch_of(starts, P, s);
  const uint32_t st = starts[p], nl = nlive[p];
  const uint32_t i = s - st;
  if (i >= nl) return;
  lcp[s] = (i == 0) ? (uint8_t)0xFF : (uint8_t)rb_lcp(key[s - 1], key[s]);
  int lev = 0;
  if (nl > (uint32_t)L) {
    int D = 0;
    uint32_t jlo = (i >= (uint32_t)L) ? i - L : 0u;
    uint32_t jhi = (i <= nl - 1 - L) ? i : nl - 1 - L;
    for (uint32_t j = jlo; j <= jhi; ++j) {
      int v = rb_lcp(key[st + j], key[st + j + L]);
      D = v > D ? v : D;
    }
    lev = D + 1 < RB_DEPTH ? D + 1 : RB_DEPTH;
  }
  leaf[s] = (uint8_t)lev;
}

struct TopoRange {
  int lo_s, hi_s, lo_e, hi_e;  // start and end level ranges (empty if lo > hi)
};

__device__ __forceinline__ TopoRange topo_range(uint32_t s, uint32_t i, uint32_t nl,
                                                const uint8_t *__restrict__ lcp,
                                                const uint8_t *__restrict__ leaf) {
  TopoRange r;
  int lf = leaf[s];
  r.lo_s = (i == 0) ? 0 : (int)lcp[s] + 1;
  r.hi_s = lf;
  r.lo_e = (i + 1 == nl) ? 0 : (int)lcp[s + 1] + 1;
  r.hi_e = lf;
  return r;
}

// per-tile counts of node starts and ends on every level
__global__ __launch_bounds__(256) void k_topo_count(
    const uint32_t *__restrict__ tile_start, const uint32_t *__restrict__ tile_end,
    const uint32_t *__restrict__ tile_patch, const uint32_t *__restrict__ starts,
    const uint32_t *__restrict__ nlive, const uint8_t *__restrict__ lcp,
    const uint8_t *__restrict__ leaf, uint32_t n_tiles, uint32_t *__restrict__ cnt) {
  __shared__ uint32_t cs[RB_NLEV], ce[RB_NLEV];
  const uint32_t b = blockIdx.x, tid = threadIdx.x, lane = rb_lane();
  if (tid < RB_NLEV) { cs[tid] = 0; ce[tid] = 0; }
  __syncthreads();
  const uint32_t p = tile_patch[b], st = starts[p], nl = nlive[p];
  const uint32_t s0 = tile_start[b], s1 = tile_end[b];
  for (uint32_t r0 = s0; r0 < s1; r0 += 256) {
    const uint32_t s = r0 + tid;
    const bool valid = s < s1 && (s - st) < nl;
    TopoRange tr = {1, 0, 1, 0};
    if (valid) tr = topo_range(s, s - st, nl, lcp, leaf);
    for (int l = 0; l < RB_NLEV; ++l) {
      uint64_t bs = __ballot(l >= tr.lo_s && l <= tr.hi_s);
      uint64_t be = __ballot(l >= tr.lo_e && l <= tr.hi_e);
      if (lane == 0) {
        if (bs) atomicAdd(&cs[l], (uint32_t)__popcll(bs));
        if (be) atomicAdd(&ce[l], (uint32_t)__popcll(be));
      }
    }
  }
  __syncthreads();
  if (tid < RB_NLEV) {
    cnt[tid * n_tiles + b] = cs[tid];
    cnt[(RB_NLEV + tid) * n_tiles + b] = ce[tid];
  }
}

// write the node arrays
__global__ __launch_bounds__(256) void k_topo_write(
    const uint32_t *__restrict__ tile_start, const uint32_t *__restrict__ tile_end,
    const uint32_t *__restrict__ tile_patch, const uint32_t *__restrict__ starts,
    uint32_t *__restrict__ nlive, uint32_t n_patch, const uint8_t *__restrict__ lcp,
    const uint8_t *__restrict__ leaf, uint32_t n_tiles, const uint32_t *__restrict__ cnt,
    const uint32_t *__restrict__ lev_tot, uint32_t node_cap,
    uint32_t *__restrict__ lev_off, uint32_t *__restrict__ nfirst,
    uint32_t *__restrict__ nlast, uint32_t *__restrict__ nchild,
    uint32_t *__restrict__ nlastchild, uint32_t *__restrict__ nskip,
    uint8_t *__restrict__ nlevel, uint8_t *__restrict__ nleaf, uint32_t *__restrict__ root,
    uint32_t *__restrict__ err, uint32_t *__restrict__ gctr) {
  __shared__ uint32_t lbase[RB_NLEV + 1];
  __shared__ uint32_t bs_off[RB_NLEV], be_off[RB_NLEV];
  __shared__ uint32_t run_s[RB_NLEV], run_e[RB_NLEV];
  __shared__ uint32_t ws[4][RB_NLEV], we[4][RB_NLEV];
  const uint32_t b = blockIdx.x, tid = threadIdx.x, w = tid >> 6;
  // the grouped walk's counters (groups emitted, work items taken) restart
  // with every tree, also when this tree fails its capacity check
  if (b == 0 && tid < 2) gctr[tid] = 0;
  if (tid == 0) {
    uint32_t acc = 0;
    for (int l = 0; l < RB_NLEV; ++l) { lbase[l] = acc; acc += lev_tot[l]; }
    lbase[RB_NLEV] = acc;
  }
  if (tid < RB_NLEV) {
    bs_off[tid] = cnt[tid * n_tiles + b];
    be_off[tid] = cnt[(RB_NLEV + tid) * n_tiles + b];
    run_s[tid] = 0;
    run_e[tid] = 0;
  }
  __syncthreads();
  const uint32_t total = lbase[RB_NLEV];
  if (total > node_cap) {
    // nothing is written; the tree is left empty (no levels, no live
    // particles) so that every later kernel of the step does no work
    if (b == 0) {
      if (tid <= RB_NLEV) lev_off[tid] = 0;
      for (uint32_t q = tid; q < n_patch; q += blockDim.x) nlive[q] = 0;
      if (tid == 0) atomicOr(err, RB_ERR_NODES);
    }
    return;  // uniform over the grid
  }
  if (b == 0 && tid <= RB_NLEV) lev_off[tid] = lbase[tid];
  const uint32_t p = tile_patch[b], st = starts[p], nl = nlive[p];
  const uint32_t s0 = tile_start[b], s1 = tile_end[b];
  for (uint32_t r0 = s0; r0 < s1; r0 += 256) {
    const uint32_t s = r0 + tid;
    const bool valid = s < s1 && (s - st) < nl;
    const uint32_t i = s - st;
    TopoRange tr = {1, 0, 1, 0};
    if (valid) tr = topo_range(s, i, nl, lcp, leaf);
    if (tid < RB_NLEV) {
      ws[0][tid] = ws[1][tid] = ws[2][tid] = ws[3][tid] = 0;
      we[0][tid] = we[1][tid] = we[2][tid] = we[3][tid] = 0;
    }
    __syncthreads();
    for (int l = 0; l < RB_NLEV; ++l) {
      uint64_t bs = __ballot(l >= tr.lo_s && l <= tr.hi_s);
      uint64_t be = __ballot(l >= tr.lo_e && l <= tr.hi_e);
      if (rb_lane() == 0) {
        ws[w][l] = (uint32_t)__popcll(bs);
        we[w][l] = (uint32_t)__popcll(be);
      }
    }
    __syncthreads();
    // starts: first slot, level, leaf flag, first child (the start one level
    // down at the same slot); ends: last slot, last child, skip pointer.
    // Indices outside the level's range would mean inconsistent counts: they
    // are reported and never written.
    uint32_t prev = RB_NONE, eprev = RB_NONE, skip_to = RB_NONE;
    for (int l = 0; l < RB_NLEV; ++l) {
      const bool in_s = l >= tr.lo_s && l <= tr.hi_s;
      const bool in_e = l >= tr.lo_e && l <= tr.hi_e;
      uint64_t bs = __ballot(in_s);
      uint64_t be = __ballot(in_e);
      if (in_s) {
        uint32_t rk = run_s[l] + rb_mbcnt(bs);
        for (uint32_t q = 0; q < w; ++q) rk += ws[q][l];
        const uint32_t id = lbase[l] + bs_off[l] + rk;
        if (id < lbase[l + 1]) {
          nfirst[id] = s;
          nlevel[id] = (uint8_t)l;
          const bool is_leaf = (l == tr.hi_s);
          nleaf[id] = is_leaf ? 1 : 0;
          if (is_leaf) nchild[id] = RB_NONE;
          if (prev != RB_NONE) nchild[prev] = id;
          if (l == 0) root[p] = id;
          prev = id;
        } else {
          atomicOr(err, RB_ERR_TREE);
          prev = RB_NONE;
        }
      }
      if (in_e) {
        uint32_t rk = run_e[l] + rb_mbcnt(be);
        for (uint32_t q = 0; q < w; ++q) rk += we[q][l];
        const uint32_t id = lbase[l] + be_off[l] + rk;
        if (id < lbase[l + 1]) {
          nlast[id] = s;
          if (l == tr.lo_e) skip_to = (i + 1 == nl) ? RB_NONE : id + 1;
          nskip[id] = skip_to;
          if (eprev != RB_NONE) nlastchild[eprev] = id;
          if (l == tr.hi_e) nlastchild[id] = RB_NONE;
          eprev = id;
        } else {
          atomicOr(err, RB_ERR_TREE);
          eprev = RB_NONE;
        }
      }
    }
    __syncthreads();
    if (tid < RB_NLEV) {
      run_s[tid] += ws[0][tid] + ws[1][tid] + ws[2][tid] + ws[3][tid];
      run_e[tid] += we[0][tid] + we[1][tid] + we[2][tid] + we[3][tid];
    }
    __syncthreads();
  }
}

hipError_t launch_topology(rb_ctx *c) {
  uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0 || c->n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_topo_leaf, dim3(rb_div_up(n, 256)), dim3(256), 0, c->stream,
                     c->d_key[0], c->d_starts, c->d_nlive, c->P, n, c->p.leaf_size, c->d_lcp,
                     c->d_leaf);
  hipLaunchKernelGGL(k_topo_count, dim3(c->n_tiles), dim3(256), 0, c->stream,
                     c->d_tile_start, c->d_tile_end, c->d_tile_patch, c->d_starts, c->d_nlive,
                     c->d_lcp, c->d_leaf, c->n_tiles, c->d_cnt);
  hipLaunchKernelGGL(k_rowscan, dim3(2 * RB_NLEV), dim3(256), 0, c->stream, c->d_cnt,
                     c->d_patch_tile0, c->n_tiles, 1, c->d_lev_tot);
  hipLaunchKernelGGL(k_topo_write, dim3(c->n_tiles), dim3(256), 0, c->stream,
                     c->d_tile_start, c->d_tile_end, c->d_tile_patch, c->d_starts, c->d_nlive,
                     c->P, c->d_lcp, c->d_leaf, c->n_tiles, c->d_cnt, c->d_lev_tot,
                     (uint32_t)c->node_cap, c->d_lev_off, c->d_nfirst, c->d_nlast,
                     c->d_nchild, c->d_nlastchild, c->d_nskip, c->d_nlevel, c->d_nleaf,
                     c->d_root, c->d_err, c->d_gctr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Moments, one launch per level from the deepest up (Sect. 4.2: mass and
// centre of mass updated bottom-up; quadrupole of Hernquist 1987).
//   leaf:     M = sum m, S = sum m x over its slots in Morton order;
//             com = x of the particle for a single-particle leaf, S / M
//             otherwise; Q = sum m (3 s s^T - |s|^2 I), s = x - com.
//   internal: M, S summed over the children in octant order; com = S / M;
//             Q = sum_c Q_c + M_c (3 d d^T - |d|^2 I), d = com_c - com.
// A node without source mass gets com = 0 and Q = 0.  Contraction is off so
// that M, S and com round exactly as a plain sequential sum would.

__global__ __launch_bounds__(256) void k_moments(
    int level, const uint32_t *__restrict__ lev_off, const uint32_t *__restrict__ nfirst,
    const uint32_t *__restrict__ nlast, const uint32_t *__restrict__ nchild,
    const uint32_t *__restrict__ nlastchild, const uint32_t *__restrict__ nskip,
    const uint8_t *__restrict__ nleaf, const double *__restrict__ sx,
    const double *__restrict__ sy, const double *__restrict__ sz,
    const double *__restrict__ msrc, int quad, NodeLink *__restrict__ link,
    double4 *__restrict__ mcom, double *__restrict__ Sarr, double *__restrict__ Qarr,
    uint32_t n_slots, uint32_t *__restrict__ err) {
#pragma clang fp contract(off)
  const uint32_t lo = lev_off[level], hi = lev_off[level + 1];
  const uint32_t clo = (level < RB_DEPTH) ? lev_off[level + 1] : 0u;
  const uint32_t chi = (level < RB_DEPTH) ? lev_off[level + 2] : 0u;
  for (uint32_t id = lo + blockIdx.x * blockDim.x + threadIdx.x; id < hi;
       id += gridDim.x * blockDim.x) {
    const uint32_t first = nfirst[id], last = nlast[id];
    const bool is_leaf = nleaf[id] != 0;
    // guard against inconsistent links: such a node becomes massless and is
    // never opened by a walk
    const bool bad = is_leaf ? !(first <= last && last < n_slots)
                             : !(nchild[id] >= clo && nchild[id] <= nlastchild[id] &&
                                 nlastchild[id] < chi);
    if (bad) {
      atomicOr(err, RB_ERR_TREE);
      NodeLink lk;
      lk.child_or_first = RB_NONE;
      lk.skip = nskip[id];
      lk.count = 0;
      lk.lvl = (uint32_t)level | 256u;
      link[id] = lk;
      mcom[id] = make_double4(0.0, 0.0, 0.0, 0.0);
      Sarr[3 * (size_t)id] = Sarr[3 * (size_t)id + 1] = Sarr[3 * (size_t)id + 2] = 0.0;
      for (int a = 0; a < 6; ++a) Qarr[6 * (size_t)id + a] = 0.0;
      continue;
    }
    double M = 0.0, S0 = 0.0, S1 = 0.0, S2 = 0.0, c0, c1, c2;
    double Q0 = 0.0, Q1 = 0.0, Q2 = 0.0, Q3 = 0.0, Q4 = 0.0, Q5 = 0.0;
    const uint32_t count = last - first + 1;
    uint32_t cf = 0;
    if (is_leaf) {
      for (uint32_t s = first; s <= last; ++s) {
        const double m = msrc[s];
        M = M + m;
        S0 = S0 + m * sx[s];
        S1 = S1 + m * sy[s];
        S2 = S2 + m * sz[s];
      }
      if (M == 0.0) {
        c0 = c1 = c2 = 0.0;
      } else if (count == 1) {
        c0 = sx[first]; c1 = sy[first]; c2 = sz[first];
      } else {
        c0 = S0 / M; c1 = S1 / M; c2 = S2 / M;
        if (quad) {
          for (uint32_t s = first; s <= last; ++s) {
            const double m = msrc[s];
            const double a0 = sx[s] - c0, a1 = sy[s] - c1, a2 = sz[s] - c2;
            const double ss = a0 * a0 + a1 * a1 + a2 * a2;
            Q0 += m * (3.0 * a0 * a0 - ss);
            Q1 += m * (3.0 * a0 * a1);
            Q2 += m * (3.0 * a0 * a2);
            Q3 += m * (3.0 * a1 * a1 - ss);
            Q4 += m * (3.0 * a1 * a2);
            Q5 += m * (3.0 * a2 * a2 - ss);
          }
        }
      }
      cf = first;
    } else {
      const uint32_t ca = nchild[id], cb = nlastchild[id];
      for (uint32_t ch = ca; ch <= cb; ++ch) {
        M = M + mcom[ch].w;
        S0 = S0 + Sarr[3 * ch + 0];
        S1 = S1 + Sarr[3 * ch + 1];
        S2 = S2 + Sarr[3 * ch + 2];
      }
      if (M == 0.0) {
        c0 = c1 = c2 = 0.0;
      } else {
        c0 = S0 / M; c1 = S1 / M; c2 = S2 / M;
      }
      if (quad) {
        for (uint32_t ch = ca; ch <= cb; ++ch) {
          const double4 cm = mcom[ch];
          const double d0 = cm.x - c0, d1 = cm.y - c1, d2 = cm.z - c2;
          const double dd = d0 * d0 + d1 * d1 + d2 * d2;
          const double *q = Qarr + 6 * (size_t)ch;
          Q0 += q[0] + cm.w * (3.0 * d0 * d0 - dd);
          Q1 += q[1] + cm.w * (3.0 * d0 * d1);
          Q2 += q[2] + cm.w * (3.0 * d0 * d2);
          Q3 += q[3] + cm.w * (3.0 * d1 * d1 - dd);
          Q4 += q[4] + cm.w * (3.0 * d1 * d2);
          Q5 += q[5] + cm.w * (3.0 * d2 * d2 - dd);
        }
      }
      cf = ca;
    }
    NodeLink lk;
    lk.child_or_first = cf;
    lk.skip = nskip[id];
    lk.count = count;
    const uint32_t n_child = is_leaf ? 0u : nlastchild[id] - nchild[id] + 1u;
    lk.lvl = (uint32_t)level | (is_leaf ? 256u : 0u) | (n_child << 9);
    link[id] = lk;
    mcom[id] = make_double4(c0, c1, c2, M);
    Sarr[3 * (size_t)id + 0] = S0;
    Sarr[3 * (size_t)id + 1] = S1;
    Sarr[3 * (size_t)id + 2] = S2;
    double *q = Qarr + 6 * (size_t)id;
    q[0] = Q0; q[1] = Q1; q[2] = Q2; q[3] = Q3; q[4] = Q4; q[5] = Q5;
  }
}

hipError_t launch_moments(rb_ctx *c, const double *sx, const double *sy, const double *sz) {
  uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  unsigned grid = rb_div_up(c->cap, 256);
  if (grid > 2048) grid = 2048;
  if (grid < 1) grid = 1;
  for (int l = RB_DEPTH; l >= 0; --l) {
    hipLaunchKernelGGL(k_moments, dim3(grid), dim3(256), 0, c->stream, l, c->d_lev_off,
                       c->d_nfirst, c->d_nlast, c->d_nchild, c->d_nlastchild, c->d_nskip,
                       c->d_nleaf, sx, sy, sz, c->d_msrc, c->p.quadrupole, c->d_link,
                       c->d_mcom, c->d_S, c->d_Q, (uint32_t)c->cap, c->d_err);
  }
  return hipGetLastError();
}
