// k_moments.hip -- bottom-up moments of the octree (Sect. 4.2 of the paper:
// total mass and centre of mass updated from the bottom up; quadrupole of
// Hernquist 1987), and the work items of the grouped walk.
//
// Every node gets, in this order of arithmetic:
//   leaf:     M = sum m, S = sum m x over its slots in Morton order;
//             com = x of the particle for a single-particle leaf, S / M
//             otherwise; Q = sum m (3 s s^T - |s|^2 I), s = x - com;
//   internal: M, S summed over the children in octant order; com = S / M;
//             Q = sum_c Q_c + M_c (3 d d^T - |d|^2 I), d = com_c - com.
// A node without source mass gets com = 0 and Q = 0.  Contraction is off so
// that M, S and com round as a plain sequential sum would.
//
// Schedule: the maximal nodes holding at most G particles (G = group_size)
// root small subtrees.  Consecutive siblings among them, packed up to G
// particles, form the work items (also those of the grouped walk); each item
// is handled by one wave level by level from its deepest level up -- a run
// of at most 64 particles has at most 64 nodes per level.  The remaining
// "large" nodes (more than G particles) follow: those without a large child
// spread over many CUs, the others level by level, deepest first.
#include "rb_internal.h"

// ---- the arithmetic of one node, shared by every kernel below so that all
// of them round identically (contraction off) ----
struct Mom {
  double M, S0, S1, S2, c0, c1, c2, Q0, Q1, Q2, Q3, Q4, Q5;
};

__device__ __forceinline__ void mom_zero(Mom &a) {
  a.M = a.S0 = a.S1 = a.S2 = a.c0 = a.c1 = a.c2 = 0.0;
  a.Q0 = a.Q1 = a.Q2 = a.Q3 = a.Q4 = a.Q5 = 0.0;
}

// leaf, first sweep: M and S over the particles in slot order
__device__ __forceinline__ void mom_leaf_ms(Mom &a, double m, double x, double y, double z) {
#pragma clang fp contract(off)
  a.M = a.M + m;
  a.S0 = a.S0 + m * x;
  a.S1 = a.S1 + m * y;
  a.S2 = a.S2 + m * z;
}

// leaf centre of mass: the particle itself for a single-particle leaf
__device__ __forceinline__ void mom_leaf_com(Mom &a, uint32_t count, double x0, double y0,
                                             double z0) {
#pragma clang fp contract(off)
  if (a.M == 0.0) {
    a.c0 = a.c1 = a.c2 = 0.0;
  } else if (count == 1) {
    a.c0 = x0; a.c1 = y0; a.c2 = z0;
  } else {
    a.c0 = a.S0 / a.M; a.c1 = a.S1 / a.M; a.c2 = a.S2 / a.M;
  }
}

// leaf, second sweep (quadrupole, multi-particle leaves with mass only)
__device__ __forceinline__ void mom_leaf_q(Mom &a, double m, double x, double y, double z) {
#pragma clang fp contract(off)
  const double a0 = x - a.c0, a1 = y - a.c1, a2 = z - a.c2;
  const double ss = a0 * a0 + a1 * a1 + a2 * a2;
  a.Q0 += m * (3.0 * a0 * a0 - ss);
  a.Q1 += m * (3.0 * a0 * a1);
  a.Q2 += m * (3.0 * a0 * a2);
  a.Q3 += m * (3.0 * a1 * a1 - ss);
  a.Q4 += m * (3.0 * a1 * a2);
  a.Q5 += m * (3.0 * a2 * a2 - ss);
}

// internal node, first sweep: M and S over the children in octant order
__device__ __forceinline__ void mom_child_ms(Mom &a, double M, double S0, double S1,
                                             double S2) {
#pragma clang fp contract(off)
  a.M = a.M + M;
  a.S0 = a.S0 + S0;
  a.S1 = a.S1 + S1;
  a.S2 = a.S2 + S2;
}

__device__ __forceinline__ void mom_internal_com(Mom &a) {
#pragma clang fp contract(off)
  if (a.M == 0.0) {
    a.c0 = a.c1 = a.c2 = 0.0;
  } else {
    a.c0 = a.S0 / a.M; a.c1 = a.S1 / a.M; a.c2 = a.S2 / a.M;
  }
}

// internal node, second sweep: parallel-axis sum of the children's Q
__device__ __forceinline__ void mom_child_q(Mom &a, double M, double x, double y, double z,
                                            const double q[6]) {
#pragma clang fp contract(off)
  const double d0 = x - a.c0, d1 = y - a.c1, d2 = z - a.c2;
  const double dd = d0 * d0 + d1 * d1 + d2 * d2;
  a.Q0 += q[0] + M * (3.0 * d0 * d0 - dd);
  a.Q1 += q[1] + M * (3.0 * d0 * d1);
  a.Q2 += q[2] + M * (3.0 * d0 * d2);
  a.Q3 += q[3] + M * (3.0 * d1 * d1 - dd);
  a.Q4 += q[4] + M * (3.0 * d1 * d2);
  a.Q5 += q[5] + M * (3.0 * d2 * d2 - dd);
}

// fp64: write the FP64 records (links, centre of mass and mass, S, Q); the
// FP32 walk's record is written whenever wn is given
__device__ __forceinline__ void mom_store(uint32_t id, const Mom &a, NodeLink lk,
                                          NodeLink *__restrict__ link,
                                          double4 *__restrict__ mcom, double *__restrict__ Sarr,
                                          double *__restrict__ Qarr, WNode *__restrict__ wn,
                                          bool fp64 = true) {
  if (fp64) {
    link[id] = lk;
    mcom[id] = make_double4(a.c0, a.c1, a.c2, a.M);
    Sarr[3 * (size_t)id + 0] = a.S0;
    Sarr[3 * (size_t)id + 1] = a.S1;
    Sarr[3 * (size_t)id + 2] = a.S2;
    double *q = Qarr + 6 * (size_t)id;
    q[0] = a.Q0; q[1] = a.Q1; q[2] = a.Q2; q[3] = a.Q3; q[4] = a.Q4; q[5] = a.Q5;
  }
  if (wn) {
    WNode r;
    r.cx = a.c0; r.cy = a.c1; r.cz = a.c2; r.M = a.M;
    r.child_or_first = lk.child_or_first;
    r.count = lk.count;
    r.lvl = lk.lvl;
    r.qxx = (float)a.Q0; r.qxy = (float)a.Q1; r.qxz = (float)a.Q2;
    r.qyy = (float)a.Q3; r.qyz = (float)a.Q4;
    wn[id] = r;
  }
}

// One node whose links are given (its children, if any, already done).
__device__ __forceinline__ void rb_node_moments_at(
    uint32_t id, int level, uint32_t first, uint32_t last, bool is_leaf, uint32_t ca,
    uint32_t cb, uint32_t skip, uint32_t clo, uint32_t chi, const double *__restrict__ sx,
    const double *__restrict__ sy, const double *__restrict__ sz,
    const double *__restrict__ msrc, int quad, NodeLink *__restrict__ link,
    double4 *__restrict__ mcom, double *__restrict__ Sarr, double *__restrict__ Qarr,
    WNode *__restrict__ wn, uint32_t n_slots,
    uint32_t *__restrict__ err) {
  // inconsistent links make the node massless and never opened
  const bool bad = is_leaf ? !(first <= last && last < n_slots)
                           : !(ca >= clo && ca <= cb && cb < chi);
  NodeLink lk;
  lk.skip = skip;
  Mom a;
  mom_zero(a);
  if (bad) {
    atomicOr(err, RB_ERR_TREE);
    lk.child_or_first = RB_NONE;
    lk.count = 0;
    lk.lvl = (uint32_t)level | 256u;
    mom_store(id, a, lk, link, mcom, Sarr, Qarr, wn);
    return;
  }
  const uint32_t count = last - first + 1;
  uint32_t cf = 0, n_child = 0;
  if (is_leaf) {
    for (uint32_t s = first; s <= last; ++s) mom_leaf_ms(a, msrc[s], sx[s], sy[s], sz[s]);
    mom_leaf_com(a, count, sx[first], sy[first], sz[first]);
    if (quad && a.M != 0.0 && count > 1)
      for (uint32_t s = first; s <= last; ++s) mom_leaf_q(a, msrc[s], sx[s], sy[s], sz[s]);
    cf = first;
  } else {
    for (uint32_t ch = ca; ch <= cb; ++ch)
      mom_child_ms(a, mcom[ch].w, Sarr[3 * (size_t)ch + 0], Sarr[3 * (size_t)ch + 1],
                   Sarr[3 * (size_t)ch + 2]);
    mom_internal_com(a);
    if (quad) {
      for (uint32_t ch = ca; ch <= cb; ++ch) {
        const double4 cm = mcom[ch];
        const double *q = Qarr + 6 * (size_t)ch;
        const double qc[6] = {q[0], q[1], q[2], q[3], q[4], q[5]};
        mom_child_q(a, cm.w, cm.x, cm.y, cm.z, qc);
      }
    }
    cf = ca;
    n_child = cb - ca + 1;
  }
  lk.child_or_first = cf;
  lk.count = count;
  lk.lvl = (uint32_t)level | (is_leaf ? 256u : 0u) | (n_child << 9);
  mom_store(id, a, lk, link, mcom, Sarr, Qarr, wn);
}

// One node from global memory.
__device__ __forceinline__ void rb_node_moments(
    uint32_t id, int level, uint32_t clo, uint32_t chi, const uint32_t *__restrict__ nfirst,
    const uint32_t *__restrict__ nlast, const uint32_t *__restrict__ nchild,
    const uint32_t *__restrict__ nlastchild, const uint32_t *__restrict__ nskip,
    const uint8_t *__restrict__ nleaf, const double *__restrict__ sx,
    const double *__restrict__ sy, const double *__restrict__ sz,
    const double *__restrict__ msrc, int quad, NodeLink *__restrict__ link,
    double4 *__restrict__ mcom, double *__restrict__ Sarr, double *__restrict__ Qarr,
    WNode *__restrict__ wn, uint32_t n_slots,
    uint32_t *__restrict__ err) {
  const bool is_leaf = nleaf[id] != 0;
  rb_node_moments_at(id, level, nfirst[id], nlast[id], is_leaf, is_leaf ? 0u : nchild[id],
                     is_leaf ? 0u : nlastchild[id], nskip[id], clo, chi, sx, sy, sz, msrc, quad,
                     link, mcom, Sarr, Qarr, wn, n_slots, err);
}

#define RB_MOMENT_ARGS                                                                 \
  nfirst, nlast, nchild, nlastchild, nskip, nleaf, sx, sy, sz, msrc, quad, link, mcom, \
      Sarr, Qarr, wn, n_slots, err
#define RB_MOMENT_PARAMS                                                               \
  const uint32_t *__restrict__ nfirst, const uint32_t *__restrict__ nlast,               \
      const uint32_t *__restrict__ nchild, const uint32_t *__restrict__ nlastchild,     \
      const uint32_t *__restrict__ nskip, const uint8_t *__restrict__ nleaf,            \
      const double *__restrict__ sx, const double *__restrict__ sy,                     \
      const double *__restrict__ sz, const double *__restrict__ msrc, int quad,         \
      NodeLink *__restrict__ link, double4 *__restrict__ mcom, double *__restrict__ Sarr, \
      double *__restrict__ Qarr, WNode *__restrict__ wn,      \
      uint32_t n_slots, uint32_t *__restrict__ err

// Work items: the children with at most G particles of nodes with more
// than G, and roots with at most G.  Consecutive such children of one node
// are packed into items of at most G particles (a run ends at a large child
// or when the next child would overflow it), so that an item fills a
// wave's lanes even when a node's octants hold few particles each; item.node
// is the run's last child.  A leaf with more than G particles (deepest
// level, or leaf_size > G) contributes pieces of G particles (item.node =
// RB_NONE).  An item is a Morton-contiguous slot range; the walk bounds it
// by its members' box.  Items of more than G/2 particles are listed from the
// front of the table (count gctr[2]), those of more than G/4 in a second
// table (gctr[3]), the others from the back of the first (gctr[4]).  Nodes
// with more than G particles are listed for the large-node passes.
// Emission order is free: every result depends only on the node itself.
// Slots in the tables and in the lists are taken with one atomic per wave.
// size class of a walk item: more than G/2 particles, more than G/4, the rest
__device__ __forceinline__ void wi_tally(uint32_t half, uint32_t quarter, uint32_t &nb,
                                         uint32_t &nm, uint32_t &ns, uint32_t sz) {
  nb += sz > half ? 1u : 0u;
  nm += (sz > quarter && sz <= half) ? 1u : 0u;
  ns += sz <= quarter ? 1u : 0u;
}

__device__ __forceinline__ void wi_put(WalkItem *__restrict__ witems,
                                       WalkItem *__restrict__ witems_mid, uint32_t wcap,
                                       uint32_t half, uint32_t quarter, uint32_t &bpos,
                                       uint32_t &mpos, uint32_t &spos, uint32_t a, uint32_t e,
                                       uint32_t p, uint32_t node) {
  const WalkItem it = {a, e, p, node};
  const uint32_t sz = e - a;
  if (sz > half) witems[bpos++] = it;
  else if (sz > quarter) witems_mid[mpos++] = it;
  else witems[wcap - 1u - spos++] = it;
}

__global__ __launch_bounds__(256) void k_groups(
    const uint32_t *__restrict__ lev_off, const uint32_t *__restrict__ nfirst,
    const uint32_t *__restrict__ nlast, const uint32_t *__restrict__ nchild,
    const uint32_t *__restrict__ nlastchild, const uint8_t *__restrict__ nleaf,
    const uint8_t *__restrict__ nlevel, const uint32_t *__restrict__ starts, uint32_t P,
    uint32_t G, WalkItem *__restrict__ witems, WalkItem *__restrict__ witems_mid, uint32_t wcap,
    uint32_t *__restrict__ gctr, uint32_t *__restrict__ large, uint32_t *__restrict__ bottom,
    uint32_t *__restrict__ large_cnt, const uint32_t *__restrict__ reuse) {
  if (reuse && *reuse == 0u) return;  // the step keeps the last tree's items
  const uint32_t n_nodes = lev_off[RB_NLEV];
  const uint32_t lane = rb_lane();
  __shared__ uint32_t s_tot[3][4], s_base[3];
  for (uint32_t base = blockIdx.x * blockDim.x; base < n_nodes; base += gridDim.x * blockDim.x) {
    const uint32_t id = base + threadIdx.x;
    const bool in = id < n_nodes;
    uint32_t f = 0, l = 0, lvl = 0;
    bool leaf = false;
    if (in) { f = nfirst[id]; l = nlast[id]; lvl = nlevel[id]; leaf = nleaf[id] != 0; }
    const uint32_t cnt = l - f + 1;
    const bool is_large = in && cnt > G;
    uint32_t ca = 0, cb = 0;
    // Walk items by size class: more than G/2 particles (front of the
    // table), more than G/4 (second table), the rest (back of the table).
    // The walk takes them in that order, so the work left at the end of a
    // walk is in small (cheap) items.
    const uint32_t half = G / 2, quarter = G / 4;
    uint32_t n_big = 0, n_mid = 0, n_small = 0;
    if (in && !is_large && lvl == 0) wi_tally(half, quarter, n_big, n_mid, n_small, cnt);
    if (is_large && leaf) {
      for (uint32_t s0 = 0; s0 < cnt; s0 += G)
        wi_tally(half, quarter, n_big, n_mid, n_small, cnt - s0 < G ? cnt - s0 : G);
    }
    bool any_large = false;
    // the (at most eight, consecutive) children's slot ranges, all requested
    // at once
    uint32_t nch = 0, chf[8], chl[8];
    if (is_large && !leaf) {
      ca = nchild[id]; cb = nlastchild[id];
      if (ca <= cb && cb - ca < 8 && cb < n_nodes) nch = cb - ca + 1;
    }
#pragma unroll
    for (uint32_t j = 0; j < 8; ++j) {
      chf[j] = j < nch ? nfirst[ca + j] : 0u;
      chl[j] = j < nch ? nlast[ca + j] : 0u;
    }
    if (is_large && !leaf) {
      uint32_t run = 0;
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j) {
        if (j >= nch) break;
        const uint32_t cc = chl[j] - chf[j] + 1;
        if (cc <= G) {
          if (run && run + cc > G) {
            wi_tally(half, quarter, n_big, n_mid, n_small, run);
            run = 0;
          }
          run += cc;
        } else {
          any_large = true;
          if (run) wi_tally(half, quarter, n_big, n_mid, n_small, run);
          run = 0;
        }
      }
      if (run) wi_tally(half, quarter, n_big, n_mid, n_small, run);
    }
    // table slots: one atomic per workgroup and table (atomics on one
    // address serialise), the waves in order after the workgroup's base
    const uint32_t bincl = rb_wave_incl_scan(n_big);
    const uint32_t mincl = rb_wave_incl_scan(n_mid);
    const uint32_t sincl = rb_wave_incl_scan(n_small);
    const uint32_t w = threadIdx.x >> 6;
    if (lane == 63) {
      s_tot[0][w] = bincl;
      s_tot[1][w] = mincl;
      s_tot[2][w] = sincl;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
      const uint32_t t = threadIdx.x;
      const uint32_t sum = s_tot[t][0] + s_tot[t][1] + s_tot[t][2] + s_tot[t][3];
      s_base[t] = sum ? atomicAdd(&gctr[2 + t], sum) : 0u;
    }
    __syncthreads();
    uint32_t bbase = s_base[0], mbase = s_base[1], sbase = s_base[2];
    for (uint32_t v = 0; v < w; ++v) {
      bbase += s_tot[0][v];
      mbase += s_tot[1][v];
      sbase += s_tot[2][v];
    }
    __syncthreads();  // (the next round rewrites s_tot and s_base)
    uint32_t bpos = bbase + bincl - n_big, mpos = mbase + mincl - n_mid;
    uint32_t spos = sbase + sincl - n_small;
    if (n_big + n_mid + n_small) {
      const uint32_t p = (P == 1) ? 0u : rb_patch_of(starts, P, f);
      if (!is_large) {
        wi_put(witems, witems_mid, wcap, half, quarter, bpos, mpos, spos, f, l + 1, p,
               id);
      } else if (leaf) {
        for (uint32_t s = f; s <= l; s += G) {
          const uint32_t e = (s + G <= l + 1) ? s + G : l + 1;
          wi_put(witems, witems_mid, wcap, half, quarter, bpos, mpos, spos, s, e, p,
                 RB_NONE);
        }
      } else {
        uint32_t run = 0, r0 = 0, r1 = 0, rl = 0;
#pragma unroll
        for (uint32_t j = 0; j < 8; ++j) {
          if (j >= nch) break;
          const uint32_t c = ca + j, cf = chf[j], cl = chl[j], cc = cl - cf + 1;
          if (cc <= G) {
            if (run && run + cc > G) {
              wi_put(witems, witems_mid, wcap, half, quarter, bpos, mpos, spos, r0, r1, p,
                     rl);
              run = 0;
            }
            if (!run) r0 = cf;
            r1 = cl + 1;
            rl = c;
            run += cc;
          } else if (run) {
            wi_put(witems, witems_mid, wcap, half, quarter, bpos, mpos, spos, r0, r1, p,
                   rl);
            run = 0;
          }
        }
        if (run)
          wi_put(witems, witems_mid, wcap, half, quarter, bpos, mpos, spos, r0, r1, p, rl);
      }
    }
    // Large nodes without a large child (and large leaves) depend on the
    // work items' subtrees and particles only: one list for all levels.  The others are
    // listed per level; the lanes of one level share one atomic.
    const bool is_bottom = is_large && (leaf || !any_large);
    const bool listed = is_large && !is_bottom;
    const uint64_t bm = __ballot(is_bottom);
    uint32_t bb = 0;
    if (lane == 0 && bm) bb = atomicAdd(&large_cnt[RB_BOTTOM], (uint32_t)__popcll(bm));
    bb = __shfl(bb, 0, 64);
    if (is_bottom) bottom[bb + rb_mbcnt(bm)] = id;
    uint64_t peers = __ballot(listed);
#pragma unroll
    for (int bit = 0; bit < 5; ++bit) {
      const bool on = (lvl >> bit) & 1u;
      const uint64_t m = __ballot(listed && on);
      peers &= on ? m : ~m;
    }
    const uint32_t leader = peers ? (uint32_t)(__ffsll((long long)peers) - 1) : lane;
    uint32_t r = 0;
    if (listed && lane == leader) r = atomicAdd(&large_cnt[lvl], (uint32_t)__popcll(peers));
    r = __shfl(r, (int)leader, 64);
    if (listed) large[lev_off[lvl] + r + rb_mbcnt(peers)] = id;
  }
}

__device__ __forceinline__ void rb_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Moments of a work item's subtrees (consecutive siblings, at most 64
// particles in all), one wave per item, without reading the tree level by
// level: every lane holds one slot, finds from the sorted keys where cells
// begin and end at each level, and takes its nodes' ids from the slot-major
// node list.  Levels are then done bottom-up with the particles and the
// previous level's node values in LDS; a node's leader lane (the lane of its
// first slot) sums its children or particles in order, exactly as
// rb_node_moments does.  With roots_only (FP32-mixed steps, where only the
// walk's node records are read), the FP64 records are written for the run's
// subtree roots alone: the large nodes above them read those.
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_moments_group(
    const WalkItem *__restrict__ items, const WalkItem *__restrict__ items_mid, uint64_t wcap,
    const uint32_t *__restrict__ gctr, const uint64_t *__restrict__ key, const uint32_t *__restrict__ starts,
    const uint32_t *__restrict__ csr, const uint32_t *__restrict__ start_ids,
    const uint32_t *__restrict__ nskip, const uint8_t *__restrict__ nlevel,
    const uint32_t *__restrict__ lev_off, const double *__restrict__ sx,
    const double *__restrict__ sy, const double *__restrict__ sz,
    const double *__restrict__ msrc, int L, int nvirt, int quad, NodeLink *__restrict__ link,
    double4 *__restrict__ mcom, double *__restrict__ Sarr, double *__restrict__ Qarr,
    WNode *__restrict__ wn, int roots_only, uint32_t *__restrict__ err) {
  // two independent waves per workgroup (fewer workgroups to dispatch),
  // each with its own LDS slice; within a wave LDS accesses stay in order,
  // so a wave-level fence orders its writes and reads
  __shared__ double vv_all[2][13][64];  // M S com Q of the last level's nodes, by leader lane
  __shared__ double pv_all[2][4][64];   // x y z m of the group's slots
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  double(*vv)[64] = vv_all[wv];
  double(*pv)[64] = pv_all[wv];
  const uint32_t n_big = gctr[2], n_mid = gctr[3], n_nodes = lev_off[RB_NLEV];
  const uint32_t n_items = n_big + n_mid + gctr[4];
  for (uint32_t gi = 2 * blockIdx.x + wv; gi < n_items; gi += 2 * gridDim.x) {
    const WalkItem it = rb_walk_item(items, items_mid, gi, n_big, n_mid, wcap);
    const uint32_t g = it.node;  // the run's last subtree root
    if (g == RB_NONE) continue;  // a run of a large leaf: no node of its own
    const uint32_t f = it.start, cnt = it.end - it.start;
    if (cnt == 0 || cnt > 64 || g >= n_nodes) {
      if (lane == 0) atomicOr(err, RB_ERR_TREE);
      continue;
    }
    const uint32_t st = starts[it.patch];
    const int l0 = nlevel[g];
    // nodes ending at the group's last slot skip to where the group does
    const uint32_t gskip = nskip[g];
    const bool in = lane < cnt;
    const uint32_t s = f + lane;
    const uint64_t k = in ? key[s] : 0ull;
    const uint64_t kf = (f > st) ? key[f - 1] : 0ull;
    const uint32_t cs = in ? csr[s] : 0u;
    pv[0][lane] = in ? sx[s] : 0.0;
    pv[1][lane] = in ? sy[s] : 0.0;
    pv[2][lane] = in ? sz[s] : 0.0;
    pv[3][lane] = in ? msrc[s] : 0.0;
    // c: octal digits shared with the previous slot (-1 at a patch start)
    const uint64_t kp = __shfl_up(k, 1, 64);
    int c;
    if (lane == 0) c = (f > st) ? rb_lcp(kf, k) : -1;
    else c = rb_lcp(kp, k);
    // deepest level of the cell holding the slot (the group node itself is
    // a leaf when it holds at most L particles)
    int leaf = l0;
    if (cnt > (uint32_t)L) {
      const uint32_t src = (lane + (uint32_t)L < 64) ? lane + (uint32_t)L : lane;
      const uint64_t kl = __shfl(k, (int)src, 64);
      const int w = (lane + (uint32_t)L < cnt) ? rb_lcp(k, kl) : -1;
      int D = w;
      for (int d = 1; d <= L; ++d) {
        const int v = __shfl_up(w, d, 64);
        if (lane >= (uint32_t)d) D = v > D ? v : D;
      }
      leaf = D + 1 < RB_DEPTH ? D + 1 : RB_DEPTH;
      if (leaf < l0) leaf = l0;
    }
    if (leaf < nvirt) leaf = nvirt;  // no leaf above the root boxes
    const int glo = c + 1;                      // first level starting at this slot
    const int lo = (lane == 0) ? l0 : c + 1;    // first such level inside the group
    // the node starting at this slot at level l: start_ids[cs + l - glo]
    // (the slot-major node list); the node after a node ending before slot
    // `end` is the shallowest one starting at `end`, at level lo of that lane
    int lmax = in ? leaf : 0;
    for (int d = 32; d >= 1; d >>= 1) {
      const int v = __shfl_xor(lmax, d, 64);
      lmax = v > lmax ? v : lmax;
    }
    rb_wave_sync();
    // this lane's node id at the level in hand, read one level ahead; its
    // node one level deeper (the first child) is the last level's id
    uint32_t id_ahead = RB_NONE, id_below = RB_NONE;
    if (in && lo <= lmax && lmax <= leaf) {
      const uint32_t q = cs + (uint32_t)(lmax - glo);
      id_ahead = (q < n_nodes) ? start_ids[q] : RB_NONE;
    }
    for (int l = lmax; l >= l0; --l) {
      const bool lead = in && lo <= l && l <= leaf;
      const uint64_t bnd = __ballot(in && lane > 0 && c < l);
      const uint64_t above = (lane < 63) ? (bnd & (~0ull << (lane + 1))) : 0ull;
      const uint32_t end = above ? (uint32_t)(__ffsll((long long)above) - 1) : cnt;
      // the skip target's list position, from lane `end` (every lane takes
      // part in the shuffle)
      const int e_src = (int)(end < 64u ? end : 63u);
      const uint32_t q_end = (uint32_t)__shfl((int)(cs + (uint32_t)(lo - glo)), e_src, 64);
      // this node's id (read one level ahead), its first child's (this
      // lane's node one level deeper) and the skip target's (read here,
      // waited for at the store, after the sums)
      uint32_t id = RB_NONE, id_child = RB_NONE, id_skip = gskip;
      if (lead) {
        id = id_ahead;
        if (l < leaf) id_child = id_below;
        if (end < cnt) id_skip = (q_end < n_nodes) ? start_ids[q_end] : RB_NONE;
      }
      id_below = id;
      id_ahead = RB_NONE;
      if (in && lo <= l - 1 && l - 1 <= leaf && l - 1 >= l0) {
        const uint32_t q = cs + (uint32_t)(l - 1 - glo);
        id_ahead = (q < n_nodes) ? start_ids[q] : RB_NONE;
      }
      const bool is_leaf = lead && l == leaf;
      const uint64_t nxt = (l < RB_DEPTH) ? __ballot(in && lo <= l + 1 && l + 1 <= leaf) : 0ull;
      const uint64_t span = ((end >= 64) ? ~0ull : ((1ull << end) - 1ull)) & (~0ull << lane);
      uint64_t kids = nxt & span;
      Mom a;
      mom_zero(a);
      if (lead) {
        if (is_leaf) {
          for (uint32_t j = lane; j < end; ++j) mom_leaf_ms(a, pv[3][j], pv[0][j], pv[1][j], pv[2][j]);
          mom_leaf_com(a, end - lane, pv[0][lane], pv[1][lane], pv[2][lane]);
          if (quad && a.M != 0.0 && end - lane > 1)
            for (uint32_t j = lane; j < end; ++j) mom_leaf_q(a, pv[3][j], pv[0][j], pv[1][j], pv[2][j]);
        } else {
          for (uint64_t m = kids; m; m &= m - 1) {
            const int j = __ffsll((long long)m) - 1;
            mom_child_ms(a, vv[0][j], vv[1][j], vv[2][j], vv[3][j]);
          }
          mom_internal_com(a);
          if (quad) {
            for (uint64_t m = kids; m; m &= m - 1) {
              const int j = __ffsll((long long)m) - 1;
              const double qc[6] = {vv[7][j], vv[8][j], vv[9][j], vv[10][j], vv[11][j], vv[12][j]};
              mom_child_q(a, vv[0][j], vv[4][j], vv[5][j], vv[6][j], qc);
            }
          }
        }
      }
      rb_wave_sync();  // every read of the deeper level is done
      if (lead) {
        vv[0][lane] = a.M; vv[1][lane] = a.S0; vv[2][lane] = a.S1; vv[3][lane] = a.S2;
        vv[4][lane] = a.c0; vv[5][lane] = a.c1; vv[6][lane] = a.c2;
        vv[7][lane] = a.Q0; vv[8][lane] = a.Q1; vv[9][lane] = a.Q2;
        vv[10][lane] = a.Q3; vv[11][lane] = a.Q4; vv[12][lane] = a.Q5;
        const uint32_t first_child = is_leaf ? s : id_child;
        // the next node after the subtree: the shallowest node starting at
        // the slot after this node's last one
        const uint32_t skip = id_skip;
        if (id < n_nodes && (is_leaf || first_child < n_nodes)) {
          NodeLink lk;
          lk.child_or_first = first_child;
          lk.skip = skip;
          lk.count = end - lane;
          lk.lvl = (uint32_t)l | (is_leaf ? 256u : 0u) | ((uint32_t)__popcll(kids) << 9);
          mom_store(id, a, lk, link, mcom, Sarr, Qarr, wn, !roots_only || l == l0);
        } else {
          atomicOr(err, RB_ERR_TREE);
        }
      }
      rb_wave_sync();
    }
  }
}

// large nodes, deepest level first: one block with a barrier per non-empty
// level.  The per-level counts and offsets are read once; when all large
// nodes fit, their links are fetched into LDS up front, so that each level
// waits only for its children's moments.
#define ML_CAP 2048

// An internal node from its (at most eight, consecutive) children, whose
// records are all requested in one round of loads.
__device__ __forceinline__ void ml_internal(uint32_t id, int l, uint32_t first, uint32_t last,
                                            uint32_t ca, uint32_t cb, uint32_t skip, int quad,
                                            NodeLink *__restrict__ link,
                                            double4 *__restrict__ mcom,
                                            double *__restrict__ Sarr,
                                            double *__restrict__ Qarr, WNode *__restrict__ wn) {
  const uint32_t nch = cb - ca + 1;
  double cm[8], cs[8][3], cx[8][3], cq[8][6];
#pragma unroll
  for (uint32_t j = 0; j < 8; ++j) {
    if (j < nch) {
      const uint32_t ch = ca + j;
      const double4 m4 = mcom[ch];
      cm[j] = m4.w;
      cx[j][0] = m4.x; cx[j][1] = m4.y; cx[j][2] = m4.z;
#pragma unroll
      for (int b = 0; b < 3; ++b) cs[j][b] = Sarr[3 * (size_t)ch + b];
      if (quad) {
#pragma unroll
        for (int b = 0; b < 6; ++b) cq[j][b] = Qarr[6 * (size_t)ch + b];
      }
    }
  }
  Mom a;
  mom_zero(a);
#pragma unroll
  for (uint32_t j = 0; j < 8; ++j)
    if (j < nch) mom_child_ms(a, cm[j], cs[j][0], cs[j][1], cs[j][2]);
  mom_internal_com(a);
  if (quad) {
#pragma unroll
    for (uint32_t j = 0; j < 8; ++j)
      if (j < nch) mom_child_q(a, cm[j], cx[j][0], cx[j][1], cx[j][2], cq[j]);
  }
  NodeLink lk;
  lk.child_or_first = ca;
  lk.skip = skip;
  lk.count = last - first + 1;
  lk.lvl = (uint32_t)l | (nch << 9);
  mom_store(id, a, lk, link, mcom, Sarr, Qarr, wn);
}


// Touch the 128-byte lines of doubles [a, b) of p with loads that skip the
// CU's L1 (agent scope), leaving them in this XCD's L2.
__device__ __forceinline__ uint64_t ml_touch(const double *p, uint32_t a, uint32_t b) {
  uint64_t s = 0;
  for (uint32_t d = a; d < b; d = (d | 15u) + 1u)
    s ^= __hip_atomic_load(reinterpret_cast<uint64_t *>(const_cast<double *>(p + d)),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return s;
}
__global__ __launch_bounds__(512) void k_moments_large(
    const uint32_t *__restrict__ large, const uint32_t *__restrict__ large_cnt,
    const uint32_t *__restrict__ lev_off, RB_MOMENT_PARAMS) {
  __shared__ uint32_t s_cnt[RB_NLEV], s_off[RB_NLEV + 2], s_pos[RB_NLEV + 1];
  __shared__ uint32_t l_id[ML_CAP], l_first[ML_CAP], l_last[ML_CAP], l_ca[ML_CAP],
      l_cb[ML_CAP], l_skip[ML_CAP];
  __shared__ uint8_t l_leaf[ML_CAP];
  const uint32_t tid = threadIdx.x;
  if (tid < RB_NLEV) s_cnt[tid] = large_cnt[tid];
  if (tid < RB_NLEV + 2) s_off[tid] = lev_off[tid];
  __syncthreads();
  if (tid == 0) {
    uint32_t a = 0;
    for (int l = 0; l < RB_NLEV; ++l) { s_pos[l] = a; a += s_cnt[l]; }
    s_pos[RB_NLEV] = a;
  }
  __syncthreads();
  const uint32_t total = s_pos[RB_NLEV];
  const bool staged = total <= ML_CAP;
  if (staged) {
    for (uint32_t i = tid; i < total; i += blockDim.x) {
      int l = 0;
      while (l + 1 < RB_NLEV && s_pos[l + 1] <= i) ++l;
      const uint32_t id = large[s_off[l] + (i - s_pos[l])];
      const bool lf = nleaf[id] != 0;
      l_id[i] = id;
      l_first[i] = nfirst[id];
      l_last[i] = nlast[id];
      l_leaf[i] = lf ? 1 : 0;
      l_ca[i] = lf ? 0u : nchild[id];
      l_cb[i] = lf ? 0u : nlastchild[id];
      l_skip[i] = nskip[id];
    }
    __syncthreads();
    // The group pass wrote the lower children from every XCD: request all
    // children's records now, in one round, so that each level below waits
    // on L2 instead of memory.  (The loads only feed a store that never
    // happens; a child written later in this kernel is read again then.)
    uint64_t sink = 0;
    for (uint32_t i = tid; i < total; i += blockDim.x) {
      const uint32_t ca = l_ca[i], cb = l_cb[i];
      if (l_leaf[i] || cb < ca || cb - ca >= 8 || cb >= s_off[RB_NLEV]) continue;
      sink ^= ml_touch(reinterpret_cast<const double *>(mcom), 4 * ca, 4 * cb + 4);
      sink ^= ml_touch(Sarr, 3 * ca, 3 * cb + 3);
      if (quad) sink ^= ml_touch(Qarr, 6 * ca, 6 * cb + 6);
    }
    if (sink == 0x5eed5eed5eed5eedull) atomicOr(err, 0u);
  }
  // one thread per node; an internal node's (at most eight) children are
  // all fetched before any sum, so a level costs one memory round trip
  for (int l = RB_DEPTH; l >= 0; --l) {
    const uint32_t cnt = s_cnt[l], base = s_off[l];
    if (cnt == 0) continue;  // uniform over the block
    const uint32_t clo = (l < RB_DEPTH) ? s_off[l + 1] : 0u;
    const uint32_t chi = (l < RB_DEPTH) ? s_off[l + 2] : 0u;
    for (uint32_t i = tid; i < cnt; i += blockDim.x) {
      uint32_t id, first, last, ca = 0, cb = 0, skip;
      bool leaf;
      if (staged) {
        const uint32_t k = s_pos[l] + i;
        id = l_id[k]; first = l_first[k]; last = l_last[k]; leaf = l_leaf[k] != 0;
        ca = l_ca[k]; cb = l_cb[k]; skip = l_skip[k];
      } else {
        id = large[base + i];
        leaf = nleaf[id] != 0;
        first = nfirst[id]; last = nlast[id]; skip = nskip[id];
        if (!leaf) { ca = nchild[id]; cb = nlastchild[id]; }
      }
      const bool ok = !leaf && ca >= clo && ca <= cb && cb < chi && cb - ca < 8;
      if (!ok) {  // leaves, and anything inconsistent (reported there)
        rb_node_moments_at(id, l, first, last, leaf, ca, cb, skip, clo, chi, sx, sy, sz, msrc,
                           quad, link, mcom, Sarr, Qarr, wn, n_slots, err);
        continue;
      }
      ml_internal(id, l, first, last, ca, cb, skip, quad, link, mcom, Sarr, Qarr, wn);
    }
    __syncthreads();
  }
}

// large nodes of one level over the whole chip (large systems)
// The bottom large nodes, one per thread, spread over many CUs (their
// children's records are read from memory by each node's own thread).
__global__ __launch_bounds__(64) void k_moments_bottom(const uint32_t *__restrict__ bottom,
                                                       const uint32_t *__restrict__ large_cnt,
                                                       const uint32_t *__restrict__ lev_off,
                                                       const uint8_t *__restrict__ nlevel,
                                                       RB_MOMENT_PARAMS) {
  const uint32_t cnt = large_cnt[RB_BOTTOM];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
    const uint32_t id = bottom[i];
    const int l = nlevel[id];
    const bool leaf = nleaf[id] != 0;
    const uint32_t first = nfirst[id], last = nlast[id], skip = nskip[id];
    const uint32_t ca = leaf ? 0u : nchild[id], cb = leaf ? 0u : nlastchild[id];
    const uint32_t clo = (l < RB_DEPTH) ? lev_off[l + 1] : 0u;
    const uint32_t chi = (l < RB_DEPTH) ? lev_off[l + 2] : 0u;
    if (!leaf && ca >= clo && ca <= cb && cb < chi && cb - ca < 8)
      ml_internal(id, l, first, last, ca, cb, skip, quad, link, mcom, Sarr, Qarr, wn);
    else  // leaves, and anything inconsistent (reported there)
      rb_node_moments_at(id, l, first, last, leaf, ca, cb, skip, clo, chi, sx, sy, sz, msrc,
                         quad, link, mcom, Sarr, Qarr, wn, n_slots, err);
  }
}

__global__ __launch_bounds__(256) void k_moments_large_level(
    int l, const uint32_t *__restrict__ large, const uint32_t *__restrict__ large_cnt,
    const uint32_t *__restrict__ lev_off, RB_MOMENT_PARAMS) {
  const uint32_t cnt = large_cnt[l], base = lev_off[l];
  const uint32_t clo = (l < RB_DEPTH) ? lev_off[l + 1] : 0u;
  const uint32_t chi = (l < RB_DEPTH) ? lev_off[l + 2] : 0u;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x)
    rb_node_moments(large[base + i], l, clo, chi, RB_MOMENT_ARGS);
}

// the work items and large-node lists of the current tree (k_groups)
hipError_t launch_groups(rb_ctx *c, const uint32_t *reuse) {
  unsigned grid = rb_div_up(c->node_cap, 256);
  if (grid > 2048) grid = 2048;
  hipLaunchKernelGGL(k_groups, dim3(grid), dim3(256), 0, c->stream, c->d_lev_off, c->d_nfirst,
                     c->d_nlast, c->d_nchild, c->d_nlastchild, c->d_nleaf, c->d_nlevel,
                     c->d_starts, c->P, (uint32_t)c->p.group_size, c->d_witems,
                     c->d_witems_mid, (uint32_t)c->cap, c->d_gctr, c->d_large, c->d_bottom,
                     c->d_large_cnt, reuse);
  return hipGetLastError();
}

hipError_t launch_moments(rb_ctx *c, const double *sx, const double *sy, const double *sz,
                          bool roots_only, const uint32_t *reuse) {
  const uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  const uint32_t G = (uint32_t)c->p.group_size;
  // the grouped walk's node records are written only when it will run
  WNode *const wnode = c->p.precision == RB_FP32_MIXED ? c->d_wnode : nullptr;
  const hipError_t ge = launch_groups(c, reuse);
  if (ge != hipSuccess) return ge;
#define RB_MARGS                                                                          \
  c->d_nfirst, c->d_nlast, c->d_nchild, c->d_nlastchild, c->d_nskip, c->d_nleaf, sx, sy, sz, \
      c->d_msrc, c->p.quadrupole, c->d_link, c->d_mcom, c->d_S, c->d_Q, wnode,              \
      (uint32_t)c->cap, c->d_err
  unsigned sgrid = rb_div_up(n, 32);  // two waves per workgroup
  if (sgrid > 131072) sgrid = 131072;
  hipLaunchKernelGGL(k_moments_group, dim3(sgrid), dim3(128), 0, c->stream, c->d_witems,
                     c->d_witems_mid, c->cap, c->d_gctr, c->d_key[0], c->d_starts, c->d_csr, c->d_start_ids, c->d_nskip,
                     c->d_nlevel, c->d_lev_off, sx, sy, sz, c->d_msrc, c->p.leaf_size,
                     (int)c->h_patch[0].nvirt, c->p.quadrupole, c->d_link, c->d_mcom, c->d_S, c->d_Q, wnode,
                     (wnode && roots_only) ? 1 : 0, c->d_err);
  // bottom large nodes are disjoint subtrees of more than G particles each
  unsigned bgrid = rb_div_up(n / (G + 1) + 1, 64);
  if (bgrid > 2048) bgrid = 2048;
  hipLaunchKernelGGL(k_moments_bottom, dim3(bgrid), dim3(64), 0, c->stream, c->d_bottom,
                     c->d_large_cnt, c->d_lev_off, c->d_nlevel, RB_MARGS);
  const int lv = c->p.moments_level_log2 > 0 ? c->p.moments_level_log2 : 22;
  if ((uint64_t)n <= (1ull << lv)) {
    hipLaunchKernelGGL(k_moments_large, dim3(1), dim3(512), 0, c->stream, c->d_large,
                       c->d_large_cnt, c->d_lev_off, RB_MARGS);
  } else {
    for (int l = RB_DEPTH; l >= 0; --l)
      hipLaunchKernelGGL(k_moments_large_level, dim3(512), dim3(256), 0, c->stream, l,
                         c->d_large, c->d_large_cnt, c->d_lev_off, RB_MARGS);
  }
#undef RB_MARGS
  return hipGetLastError();
}
