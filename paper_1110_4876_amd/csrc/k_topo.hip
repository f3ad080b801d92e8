// k_topo.hip -- the octree of Sect. 4.2 of the paper, derived from the sorted
// Morton keys instead of one-at-a-time insertion.
//
// The tree is the one insertion builds: a cell exists when its parent holds
// more than leaf_size particles (the root always), and it is a leaf when it
// holds at most leaf_size particles or sits on level 21.  In the sorted keys
// a cell is a run of particles sharing an octal prefix.  For live slot i of
// a patch with n live particles and L = leaf_size:
//   c_i    = LCP(key_{i-1}, key_i) in octal digits;
//   D_i    = max over windows [j, j + L] holding i of LCP(key_j, key_{j+L})
//            (a run of L + 1 particles around i shares D_i digits);
//   leaf_i = min(D_i + 1, 21), or 0 when n <= L (the root is the leaf).
// The cell holding i on level l exists exactly for l <= leaf_i.  Cells
// starting at i are the levels (c_i, leaf_i] (all of [0, leaf_0] for i = 0);
// cells ending at i are (c_{i+1}, leaf_i] ([0, leaf_i] for the last one).
// Nodes are numbered level by level, patch by patch, by prefix inside a
// level, so the k-th start and the k-th end of a level are the same node and
// every node's children are contiguous.
//
// One wave handles one tile of consecutive slots: count starts and ends per
// level (k_topo_count), scan the counts (rowscan), then write every node's
// first slot, last slot, first and last child and skip pointer
// (k_topo_write).  k_topo_write also lists the nodes slot by slot:
// start_ids[csr[s] + (l - first start level of s)] is the node of level l
// starting at slot s, so the moments can find a subtree's nodes from its
// slots without walking down the levels.
#include "rb_internal.h"

struct TopoRange {
  int lo_s, hi_s, lo_e, hi_e;  // start and end level ranges (empty if lo > hi)
};

__device__ __forceinline__ TopoRange rb_topo_range(const uint64_t *__restrict__ key,
                                                   uint32_t st, uint32_t i, uint32_t nl, int L,
                                                   int nvirt) {
  const uint64_t *k = key + st;
  int lf = 0;
  if (nl > (uint32_t)L) {
    int D = 0;
    const uint32_t jlo = (i >= (uint32_t)L) ? i - L : 0u;
    const uint32_t jhi = (i <= nl - 1 - L) ? i : nl - 1 - L;
    for (uint32_t j = jlo; j <= jhi; ++j) {
      const int v = rb_lcp(k[j], k[j + L]);
      D = v > D ? v : D;
    }
    lf = D + 1 < RB_DEPTH ? D + 1 : RB_DEPTH;
  }
  // the cells above the root boxes are never leaves: every occupied one
  // exists down to its root box (the root of that box's own tree)
  if (lf < nvirt) lf = nvirt;
  TopoRange r;
  r.lo_s = (i == 0) ? 0 : rb_lcp(k[i - 1], k[i]) + 1;
  r.hi_s = lf;
  r.lo_e = (i + 1 == nl) ? 0 : rb_lcp(k[i], k[i + 1]) + 1;
  r.hi_e = lf;
  return r;
}

// the levels at which any lane of the wave starts or ends a node
__device__ __forceinline__ void rb_topo_levels(const TopoRange &tr, bool valid, int &lmin,
                                               int &lmax) {
  lmin = valid ? min(tr.lo_s, tr.lo_e) : RB_NLEV;
  lmax = valid ? max(tr.hi_s, tr.hi_e) : -1;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    lmin = min(lmin, __shfl_xor(lmin, d, 64));
    lmax = max(lmax, __shfl_xor(lmax, d, 64));
  }
}

__global__ __launch_bounds__(64) void k_topo_count(
    const uint64_t *__restrict__ key, const uint32_t *__restrict__ tile_start,
    const uint32_t *__restrict__ tile_end, const uint32_t *__restrict__ tile_patch,
    const uint32_t *__restrict__ starts, const uint32_t *__restrict__ nlive, int L,
    int nvirt, uint32_t n_tiles, uint32_t *__restrict__ cnt, const uint32_t *__restrict__ reuse) {
  if (reuse && *reuse == 0u) return;  // the step keeps the last tree
  const uint32_t b = blockIdx.x, lane = threadIdx.x;
  const uint32_t p = tile_patch[b], st = starts[p], nl = nlive[p];
  const uint32_t s0 = tile_start[b], s1 = tile_end[b];
  uint32_t cs = 0, ce = 0;  // lane l < 22 keeps the counts of level l
  for (uint32_t r0 = s0; r0 < s1; r0 += 64) {
    const uint32_t s = r0 + lane;
    const bool valid = s < s1 && (s - st) < nl;
    TopoRange tr = {1, 0, 1, 0};
    if (valid) tr = rb_topo_range(key, st, s - st, nl, L, nvirt);
    int lmin, lmax;
    rb_topo_levels(tr, valid, lmin, lmax);
#pragma unroll
    for (int l = 0; l < RB_NLEV; ++l) {
      if (l < lmin || l > lmax) continue;  // uniform: nothing starts or ends here
      const uint32_t ns = (uint32_t)__popcll(__ballot(l >= tr.lo_s && l <= tr.hi_s));
      const uint32_t ne = (uint32_t)__popcll(__ballot(l >= tr.lo_e && l <= tr.hi_e));
      if (lane == (uint32_t)l) { cs += ns; ce += ne; }
    }
  }
  if (lane < RB_NLEV) {
    cnt[(size_t)lane * n_tiles + b] = cs;
    cnt[(size_t)(RB_NLEV + lane) * n_tiles + b] = ce;
  }
}

__global__ __launch_bounds__(64) void k_topo_write(
    const uint64_t *__restrict__ key, const uint32_t *__restrict__ tile_start,
    const uint32_t *__restrict__ tile_end, const uint32_t *__restrict__ tile_patch,
    const uint32_t *__restrict__ starts, uint32_t *__restrict__ nlive, uint32_t n_patch, int L,
    int nvirt, uint32_t n_tiles, const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ lev_tot,
    uint32_t node_cap, uint32_t *__restrict__ lev_off, uint32_t *__restrict__ nfirst,
    uint32_t *__restrict__ nlast, uint32_t *__restrict__ nchild,
    uint32_t *__restrict__ nlastchild, uint32_t *__restrict__ nskip,
    uint8_t *__restrict__ nlevel, uint8_t *__restrict__ nleaf, uint32_t *__restrict__ root,
    uint32_t *__restrict__ err, uint32_t *__restrict__ gctr, uint32_t *__restrict__ large_cnt,
    uint32_t *__restrict__ sort_number, uint32_t *__restrict__ csr,
    uint32_t *__restrict__ start_ids, const uint32_t *__restrict__ reuse,
    unsigned long long *__restrict__ stats) {
  const uint32_t b = blockIdx.x, lane = threadIdx.x;
  // the sort that produced these keys is complete: number the next one
  if (b == 0 && lane == 0) sort_number[0] += 1u;
  if (reuse && *reuse == 0u) {
    // the step keeps the last tree: its nodes, lists and work items stand;
    // only the grouped walk's queue restarts
    if (b == 0 && lane == 0) {
      gctr[1] = 0u;
      atomicAdd(&stats[5], 1ull);
    }
    return;
  }
  // level offsets: lane l holds the first node of level l
  const uint32_t tot = (lane < RB_NLEV) ? lev_tot[lane] : 0u;
  const uint32_t lincl = rb_wave_incl_scan(tot);
  const uint32_t lbase_lane = lincl - tot;
  const uint32_t total = __shfl(lincl, 63, 64);
  // the grouped walk's counters (node groups emitted, work items taken,
  // walk items emitted per size class) restart with every tree, also when
  // this tree fails its capacity check
  if (b == 0 && lane < 8) gctr[lane] = 0;
  if (b == 0 && lane < RB_LARGE_SLOTS) large_cnt[lane] = 0;
  if (total > node_cap) {
    // nothing is written; the tree is left empty (no levels, no live
    // particles) so that every later kernel of the step does no work
    if (b == 0) {
      if (lane <= RB_NLEV) lev_off[lane] = 0;
      for (uint32_t q = lane; q < n_patch; q += 64) nlive[q] = 0;
      if (lane == 0) atomicOr(err, RB_ERR_NODES);
    }
    return;  // uniform over the grid
  }
  if (b == 0 && lane <= RB_NLEV) lev_off[lane] = (lane < RB_NLEV) ? lbase_lane : total;
  // per level (lane l): first node of this tile's starts and ends
  uint32_t off_s = 0, off_e = 0;
  if (lane < RB_NLEV) {
    off_s = lbase_lane + cnt[(size_t)lane * n_tiles + b];
    off_e = lbase_lane + cnt[(size_t)(RB_NLEV + lane) * n_tiles + b];
  }
  const uint32_t lend_lane = lincl;  // one past the last node of level `lane`
  const uint32_t p = tile_patch[b], st = starts[p], nl = nlive[p];
  const uint32_t s0 = tile_start[b], s1 = tile_end[b];
  for (uint32_t r0 = s0; r0 < s1; r0 += 64) {
    const uint32_t s = r0 + lane;
    const bool valid = s < s1 && (s - st) < nl;
    const uint32_t i = s - st;
    TopoRange tr = {1, 0, 1, 0};
    if (valid) tr = rb_topo_range(key, st, i, nl, L, nvirt);
    // starts: first slot, level, leaf flag, first child (the start one level
    // down at the same slot); ends: last slot, last child, skip pointer.
    // Indices outside the level's range would mean inconsistent counts:
    // they are reported and never written.
    uint32_t prev = RB_NONE, eprev = RB_NONE, skip_to = RB_NONE;
    // csr_s: nodes of all levels that start before slot s (the place of
    // this slot's starts in the slot-major list start_ids): the starts
    // before this row of 64 slots, summed over the levels, plus those of
    // the lanes below in the row
    uint32_t csr_s;
    {
      const uint32_t v = (lane < RB_NLEV) ? off_s - lbase_lane : 0u;
      csr_s = __shfl(rb_wave_incl_scan(v), 63, 64);
    }
    int lmin, lmax;
    rb_topo_levels(tr, valid, lmin, lmax);
    uint32_t my_id[RB_NLEV];
#pragma unroll
    for (int l = 0; l < RB_NLEV; ++l) {
      my_id[l] = RB_NONE;
      if (l < lmin || l > lmax) continue;  // uniform: nothing starts or ends here
      const bool in_s = l >= tr.lo_s && l <= tr.hi_s;
      const bool in_e = l >= tr.lo_e && l <= tr.hi_e;
      const uint64_t bs = __ballot(in_s);
      const uint64_t be = __ballot(in_e);
      const uint32_t os = __shfl(off_s, l, 64), oe = __shfl(off_e, l, 64);
      const uint32_t lend = __shfl(lend_lane, l, 64);
      csr_s += rb_mbcnt(bs);
      if (in_s) {
        const uint32_t id = os + rb_mbcnt(bs);
        if (id < lend) {
          my_id[l] = id;
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
        const uint32_t id = oe + rb_mbcnt(be);
        if (id < lend) {
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
      if (lane == (uint32_t)l) {
        off_s += (uint32_t)__popcll(bs);
        off_e += (uint32_t)__popcll(be);
      }
    }
    if (valid) {
      csr[s] = csr_s;
#pragma unroll
      for (int l = 0; l < RB_NLEV; ++l) {
        if (l >= tr.lo_s && l <= tr.hi_s) {
          const uint32_t q = csr_s + (uint32_t)(l - tr.lo_s);
          if (q < total) start_ids[q] = my_id[l];
        }
      }
    }
  }
}

hipError_t launch_topology(rb_ctx *c, const uint32_t *reuse) {
  const uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0 || c->n_tiles == 0) return hipSuccess;
  const int L = c->p.leaf_size;
  const int nv = (int)c->h_patch[0].nvirt;
  hipLaunchKernelGGL(k_topo_count, dim3(c->n_tiles), dim3(64), 0, c->stream, c->d_key[0],
                     c->d_tile_start, c->d_tile_end, c->d_tile_patch, c->d_starts, c->d_nlive, L,
                     nv, c->n_tiles, c->d_cnt, reuse);
  hipError_t e = launch_rowscan_levels(c, reuse);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_topo_write, dim3(c->n_tiles), dim3(64), 0, c->stream, c->d_key[0],
                     c->d_tile_start, c->d_tile_end, c->d_tile_patch, c->d_starts, c->d_nlive,
                     c->P, L, nv, c->n_tiles, c->d_cnt, c->d_lev_tot, (uint32_t)c->node_cap,
                     c->d_lev_off, c->d_nfirst, c->d_nlast, c->d_nchild, c->d_nlastchild,
                     c->d_nskip, c->d_nlevel, c->d_nleaf, c->d_root, c->d_err, c->d_gctr,
                     c->d_large_cnt, c->d_sctl, c->d_csr, c->d_start_ids, reuse, c->d_stats);
  return hipGetLastError();
}

// Whether a step can keep the last tree (Sect. 4.2: the tree persists and
// only particles that left their cells move in it).  The canonical tree of
// sorted keys is a function of the octal prefix level each live key shares
// with the previous one (and of the live count): code(s) = 255 at a patch's
// first slot, 254 past its live keys, LCP(key[s-1], key[s]) otherwise.  If
// every slot's code equals the last tree's, that tree's topology, node
// lists and work items are this one's; any difference raises *flag.  The
// new codes are kept for the next step.
__global__ __launch_bounds__(256) void k_topo_check(const uint64_t *__restrict__ key,
                                                    const uint32_t *__restrict__ starts,
                                                    const uint32_t *__restrict__ nlive,
                                                    uint32_t P, uint32_t n,
                                                    uint8_t *__restrict__ lcp,
                                                    uint32_t *__restrict__ flag) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  bool changed = false;
  if (s < n) {
    const uint32_t p = (P == 1) ? 0 : rb_patch_of(starts, P, s);
    const uint32_t st = starts[p], nl = nlive[p], i = s - st;
    const uint8_t code = (i >= nl) ? (uint8_t)254 : (i == 0) ? (uint8_t)255
                                                             : (uint8_t)rb_lcp(key[s - 1], key[s]);
    changed = lcp[s] != code;
    if (changed) lcp[s] = code;
  }
  if (__ballot(changed) != 0ull && rb_lane() == 0) atomicOr(flag, 1u);
}

hipError_t launch_topo_check(rb_ctx *c, uint32_t *flag) {
  const uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_topo_check, dim3(rb_div_up(n, 256)), dim3(256), 0, c->stream,
                     c->d_key[0], c->d_starts, c->d_nlive, c->P, n, c->d_lcp, flag);
  return hipGetLastError();
}
