// k_moments.hip -- bottom-up moments of the octree (Sect. 4.2 of the paper:
// total mass and centre of mass updated from the bottom up; quadrupole of
// Hernquist 1987), and the particle groups of the grouped walk.
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
// Schedule: the maximal nodes holding at most G particles (G = group_size;
// they are also the walk groups) root small subtrees, each handled by one
// wave level by level from its deepest level up -- a subtree of at most 64
// particles has at most 64 nodes per level.  The remaining "large" nodes
// (more than G particles) are listed per level and computed afterwards,
// deepest level first.  Three launches replace one launch per level.
#include "rb_internal.h"

__device__ __forceinline__ void rb_node_moments(
    uint32_t id, int level, uint32_t clo, uint32_t chi, const uint32_t *__restrict__ nfirst,
    const uint32_t *__restrict__ nlast, const uint32_t *__restrict__ nchild,
    const uint32_t *__restrict__ nlastchild, const uint32_t *__restrict__ nskip,
    const uint8_t *__restrict__ nleaf, const double *__restrict__ sx,
    const double *__restrict__ sy, const double *__restrict__ sz,
    const double *__restrict__ msrc, int quad, NodeLink *__restrict__ link,
    double4 *__restrict__ mcom, double *__restrict__ Sarr, double *__restrict__ Qarr,
    float4 *__restrict__ qf0, float2 *__restrict__ qf1, uint32_t n_slots,
    uint32_t *__restrict__ err) {
#pragma clang fp contract(off)
  const uint32_t first = nfirst[id], last = nlast[id];
  const bool is_leaf = nleaf[id] != 0;
  // inconsistent links make the node massless and never opened
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
    qf0[id] = make_float4(0.f, 0.f, 0.f, 0.f);
    qf1[id] = make_float2(0.f, 0.f);
    return;
  }
  double M = 0.0, S0 = 0.0, S1 = 0.0, S2 = 0.0, c0, c1, c2;
  double Q0 = 0.0, Q1 = 0.0, Q2 = 0.0, Q3 = 0.0, Q4 = 0.0, Q5 = 0.0;
  const uint32_t count = last - first + 1;
  uint32_t cf = 0, n_child = 0;
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
      S0 = S0 + Sarr[3 * (size_t)ch + 0];
      S1 = S1 + Sarr[3 * (size_t)ch + 1];
      S2 = S2 + Sarr[3 * (size_t)ch + 2];
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
    n_child = cb - ca + 1;
  }
  NodeLink lk;
  lk.child_or_first = cf;
  lk.skip = nskip[id];
  lk.count = count;
  lk.lvl = (uint32_t)level | (is_leaf ? 256u : 0u) | (n_child << 9);
  link[id] = lk;
  mcom[id] = make_double4(c0, c1, c2, M);
  Sarr[3 * (size_t)id + 0] = S0;
  Sarr[3 * (size_t)id + 1] = S1;
  Sarr[3 * (size_t)id + 2] = S2;
  double *q = Qarr + 6 * (size_t)id;
  q[0] = Q0; q[1] = Q1; q[2] = Q2; q[3] = Q3; q[4] = Q4; q[5] = Q5;
  qf0[id] = make_float4((float)Q0, (float)Q1, (float)Q2, (float)Q3);
  qf1[id] = make_float2((float)Q4, (float)Q5);
}

#define RB_MOMENT_ARGS                                                                 \
  nfirst, nlast, nchild, nlastchild, nskip, nleaf, sx, sy, sz, msrc, quad, link, mcom, \
      Sarr, Qarr, qf0, qf1, n_slots, err
#define RB_MOMENT_PARAMS                                                               \
  const uint32_t *__restrict__ nfirst, const uint32_t *__restrict__ nlast,               \
      const uint32_t *__restrict__ nchild, const uint32_t *__restrict__ nlastchild,     \
      const uint32_t *__restrict__ nskip, const uint8_t *__restrict__ nleaf,            \
      const double *__restrict__ sx, const double *__restrict__ sy,                     \
      const double *__restrict__ sz, const double *__restrict__ msrc, int quad,         \
      NodeLink *__restrict__ link, double4 *__restrict__ mcom, double *__restrict__ Sarr, \
      double *__restrict__ Qarr, float4 *__restrict__ qf0, float2 *__restrict__ qf1,      \
      uint32_t n_slots, uint32_t *__restrict__ err

// Groups: the children with at most G particles of nodes with more than G,
// and roots with at most G; a leaf with more than G particles (deepest
// level, or leaf_size > G) contributes runs of G particles.  group.pad is
// the group's node (RB_NONE for such runs).  Nodes with more than G
// particles are listed per level for the large-node pass.  Emission order is
// free: every result depends only on the node itself.
__global__ __launch_bounds__(256) void k_groups(
    const uint32_t *__restrict__ lev_off, const uint32_t *__restrict__ nfirst,
    const uint32_t *__restrict__ nlast, const uint32_t *__restrict__ nchild,
    const uint32_t *__restrict__ nlastchild, const uint8_t *__restrict__ nleaf,
    const uint8_t *__restrict__ nlevel, const uint32_t *__restrict__ starts, uint32_t P,
    uint32_t G, WalkItem *__restrict__ groups, uint32_t *__restrict__ gctr,
    uint32_t *__restrict__ large, uint32_t *__restrict__ large_cnt) {
  const uint32_t n_nodes = lev_off[RB_NLEV];
  for (uint32_t id = blockIdx.x * blockDim.x + threadIdx.x; id < n_nodes;
       id += gridDim.x * blockDim.x) {
    const uint32_t f = nfirst[id], l = nlast[id];
    const uint32_t cnt = l - f + 1;
    const uint32_t lvl = nlevel[id];
    if (cnt <= G) {
      if (lvl == 0) {
        const uint32_t g = atomicAdd(&gctr[0], 1u);
        groups[g] = {f, l + 1, (P == 1) ? 0u : rb_patch_of(starts, P, f), id};
      }
      continue;
    }
    const uint32_t pos = atomicAdd(&large_cnt[lvl], 1u);
    large[lev_off[lvl] + pos] = id;
    const uint32_t p = (P == 1) ? 0u : rb_patch_of(starts, P, f);
    if (nleaf[id]) {
      for (uint32_t s = f; s <= l; s += G) {
        const uint32_t g = atomicAdd(&gctr[0], 1u);
        groups[g] = {s, (s + G <= l + 1) ? s + G : l + 1, p, RB_NONE};
      }
      continue;
    }
    const uint32_t ca = nchild[id], cb = nlastchild[id];
    for (uint32_t c = ca; c <= cb; ++c) {
      const uint32_t cf = nfirst[c], cl = nlast[c];
      if (cl - cf + 1 <= G) {
        const uint32_t g = atomicAdd(&gctr[0], 1u);
        groups[g] = {cf, cl + 1, p, c};
      }
    }
  }
}

// one wave per small subtree: level ranges top-down, moments bottom-up
__global__ __launch_bounds__(64) void k_moments_small(
    const WalkItem *__restrict__ groups, const uint32_t *__restrict__ gctr,
    const uint32_t *__restrict__ lev_off, const uint8_t *__restrict__ nlevel,
    RB_MOMENT_PARAMS) {
  __shared__ uint32_t rlo[RB_NLEV], rhi[RB_NLEV];
  const uint32_t lane = threadIdx.x;
  const uint32_t n_groups = gctr[0];
  for (uint32_t gi = blockIdx.x; gi < n_groups; gi += gridDim.x) {
    const uint32_t node = groups[gi].pad;
    if (node == RB_NONE) continue;
    const int top = nlevel[node];
    uint32_t lo = node, hi = node;
    int deepest = top;
    bool ok = true;
    for (int l = top; l <= RB_DEPTH; ++l) {
      if (lane == 0) { rlo[l] = lo; rhi[l] = hi; }
      deepest = l;
      if (hi - lo >= 64) { ok = false; break; }  // more nodes than particles: bad links
      const uint32_t id = lo + lane;
      const bool in = id <= hi;
      const bool internal = in && nleaf[id] == 0;
      const uint64_t bm = __ballot(internal);
      if (bm == 0) break;
      const int fi = __ffsll((long long)bm) - 1;
      const int li = 63 - __clzll((long long)bm);
      const uint32_t a = internal ? nchild[id] : 0u;
      const uint32_t z = internal ? nlastchild[id] : 0u;
      lo = __shfl(a, fi, 64);
      hi = __shfl(z, li, 64);
      if (l == RB_DEPTH || hi < lo) { ok = false; break; }
    }
    if (!ok) {
      if (lane == 0) atomicOr(err, RB_ERR_TREE);
      continue;
    }
    __syncthreads();
    for (int l = deepest; l >= top; --l) {
      const uint32_t a = rlo[l], z = rhi[l];
      const uint32_t clo = (l < RB_DEPTH) ? lev_off[l + 1] : 0u;
      const uint32_t chi = (l < RB_DEPTH) ? lev_off[l + 2] : 0u;
      if (a + lane <= z) rb_node_moments(a + lane, l, clo, chi, RB_MOMENT_ARGS);
      // this level's results must be visible to the next level's reads
      __syncthreads();
    }
  }
}

// large nodes, deepest level first: one block with a barrier per level
__global__ __launch_bounds__(1024) void k_moments_large(
    const uint32_t *__restrict__ large, const uint32_t *__restrict__ large_cnt,
    const uint32_t *__restrict__ lev_off, RB_MOMENT_PARAMS) {
  for (int l = RB_DEPTH; l >= 0; --l) {
    const uint32_t cnt = large_cnt[l], base = lev_off[l];
    const uint32_t clo = (l < RB_DEPTH) ? lev_off[l + 1] : 0u;
    const uint32_t chi = (l < RB_DEPTH) ? lev_off[l + 2] : 0u;
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x)
      rb_node_moments(large[base + i], l, clo, chi, RB_MOMENT_ARGS);
    __syncthreads();
  }
}

// large nodes of one level over the whole chip (large systems)
__global__ __launch_bounds__(256) void k_moments_large_level(
    int l, const uint32_t *__restrict__ large, const uint32_t *__restrict__ large_cnt,
    const uint32_t *__restrict__ lev_off, RB_MOMENT_PARAMS) {
  const uint32_t cnt = large_cnt[l], base = lev_off[l];
  const uint32_t clo = (l < RB_DEPTH) ? lev_off[l + 1] : 0u;
  const uint32_t chi = (l < RB_DEPTH) ? lev_off[l + 2] : 0u;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x)
    rb_node_moments(large[base + i], l, clo, chi, RB_MOMENT_ARGS);
}

hipError_t launch_moments(rb_ctx *c, const double *sx, const double *sy, const double *sz) {
  const uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  const uint32_t G = (uint32_t)c->p.group_size;
  unsigned grid = rb_div_up(c->node_cap, 256);
  if (grid > 2048) grid = 2048;
  hipLaunchKernelGGL(k_groups, dim3(grid), dim3(256), 0, c->stream, c->d_lev_off, c->d_nfirst,
                     c->d_nlast, c->d_nchild, c->d_nlastchild, c->d_nleaf, c->d_nlevel,
                     c->d_starts, c->P, G, c->d_groups, c->d_gctr, c->d_large, c->d_large_cnt);
#define RB_MARGS                                                                          \
  c->d_nfirst, c->d_nlast, c->d_nchild, c->d_nlastchild, c->d_nskip, c->d_nleaf, sx, sy, sz, \
      c->d_msrc, c->p.quadrupole, c->d_link, c->d_mcom, c->d_S, c->d_Q, c->d_qf0, c->d_qf1,  \
      (uint32_t)c->cap, c->d_err
  unsigned sgrid = rb_div_up(n, 16);
  if (sgrid > 8192) sgrid = 8192;
  hipLaunchKernelGGL(k_moments_small, dim3(sgrid), dim3(64), 0, c->stream, c->d_groups,
                     c->d_gctr, c->d_lev_off, c->d_nlevel, RB_MARGS);
  if (n <= (1u << 22)) {
    hipLaunchKernelGGL(k_moments_large, dim3(1), dim3(1024), 0, c->stream, c->d_large,
                       c->d_large_cnt, c->d_lev_off, RB_MARGS);
  } else {
    for (int l = RB_DEPTH; l >= 0; --l)
      hipLaunchKernelGGL(k_moments_large_level, dim3(512), dim3(256), 0, c->stream, l,
                         c->d_large, c->d_large_cnt, c->d_lev_off, RB_MARGS);
  }
#undef RB_MARGS
  return hipGetLastError();
}
