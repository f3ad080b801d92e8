// k_collide.hip -- collisions at the end of a step (Sect. 5 of the paper):
// overlapping pairs found by the octree search of Eq. (3) over the ghost
// boxes, a collision queue in a random order, and hard-sphere resolution
// with a normal coefficient of restitution, one collision after the other in
// queue order.
//
// Detection: the criterion of Eq. (3) opens a cell for particle i while the
// distance from x_i to the image-shifted cell centre is below R_i + R_max +
// (sqrt 3 / 2) w; every particle of the cell that could overlap i passes it,
// so the search finds every overlap.  One wave searches for the (up to 64)
// Morton-consecutive particles of a work item at once: a cell is opened when
// it is within R_g + R_max + (sqrt 3 / 2) w of the item's bounding box (R_g
// the item's largest radius), which holds whenever it holds for any member.
// Opened leaves go to an LDS list that every lane then tests against its own
// particle: j overlaps i when |x_j + o_k - x_i| < R_i + R_j; the pair is
// queued once, from its lower caller index i, as the code i 2^35 + j 2^7 + k.
//
// Order and resolution: the queue's order is ascending h = splitmix64(seed +
// code) (a bijection, so the order is total).  Resolving collisions one after
// the other in that order is reproduced in rounds: a collision is resolved
// in the first round in which it has the smallest h among the unresolved
// collisions of both its particles (collisions without a common particle
// commute).  Resolution applies v_n' = -eps v_n, v_t' = v_t with momentum
// conservation when the pair approaches (d . u < 0, u = v_j + w_k - v_i with
// w_k the image's shear velocity).
//
// Compiled without FP contraction so that the pair tests and the velocity
// updates round exactly as a plain evaluation of the same expressions.
#include "rb_internal.h"

#define RB_COLL_LOCAL 8  // pairs a thread keeps before it writes them out

__device__ __forceinline__ uint64_t rb_splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// image k of the ghost boxes: ix outer and iy inner in [-ng, ng] (a single
// image for open boundaries); position offset and y velocity offset
__device__ __forceinline__ void rb_coll_image(int k, int ngx, int ngy, int boundary, double W,
                                              double sh, double omega, double &ox, double &oy,
                                              double &wy) {
  if (boundary == RB_OPEN) { ox = oy = wy = 0.0; return; }
  const int ny = 2 * ngy + 1;
  const int ix = k / ny - ngx, iy = k % ny - ngy;
  const double fx = (double)ix, fy = (double)iy;
  const double s = (boundary == RB_SHEAR) ? sh : 0.0;
  ox = fx * W;
  oy = fy * W - fx * s;
  wy = (boundary == RB_SHEAR) ? -1.5 * omega * W * fx : 0.0;
}

// largest radius of the live particles (as ordered bits of a non-negative
// double)
__global__ __launch_bounds__(256) void k_coll_rmax(const double *__restrict__ R,
                                                   const uint32_t *__restrict__ orig,
                                                   const uint32_t *__restrict__ starts,
                                                   const uint32_t *__restrict__ nlive,
                                                   uint32_t P, uint32_t n,
                                                   unsigned long long *__restrict__ rmax) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  double r = 0.0;
  if (s < n) {
    const uint32_t p = (P == 1) ? 0u : rb_patch_of(starts, P, s);
    if (s - starts[p] < nlive[p]) {
      const double v = R[orig[s]];
      r = v > 0.0 ? v : 0.0;
    }
  }
  for (int d = 32; d >= 1; d >>= 1) r = fmax(r, __shfl_xor(r, d, 64));
  if (rb_lane() == 0 && r > 0.0) atomicMax(rmax, (unsigned long long)__double_as_longlong(r));
}

// order a wave's LDS writes before its later reads (a wave runs in lockstep)
__device__ __forceinline__ void coll_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

#define CG_SCAP 1024  // traversal stack entries per wave (node << 5 | image)
#define CG_RESERVE (7 * RB_DEPTH + 8)
#define CG_LL 128     // opened-leaf list capacity per wave (tested at >= 64)

__device__ __forceinline__ double rb_wave_min_d(double v) {
  for (int d = 32; d >= 1; d >>= 1) v = fmin(v, __shfl_xor(v, d, 64));
  return v;
}
__device__ __forceinline__ double rb_wave_max_d(double v) {
  for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
  return v;
}

// queue a pair from the lane's local list, writing the list out when full
__device__ __forceinline__ void rb_coll_keep(uint64_t code, uint64_t (&mine)[RB_COLL_LOCAL],
                                             uint32_t &nm, uint64_t *__restrict__ queue,
                                             uint32_t qcap, uint32_t *__restrict__ qcnt,
                                             uint32_t *__restrict__ err) {
  if (nm == RB_COLL_LOCAL) {
    const uint32_t at = atomicAdd(qcnt, (uint32_t)nm);
    for (uint32_t q = 0; q < nm; ++q)
      if (at + q < qcap) queue[at + q] = mine[q];
    if (at + nm > qcap) atomicOr(err, RB_ERR_COLL);
    nm = 0;
  }
  mine[nm++] = code;
}

// One wave per work item (consecutive sibling subtrees of at most
// group_size particles), four waves per workgroup, items strided over the
// grid.
__global__ __launch_bounds__(256) void k_coll_detect(
    const WalkItem *__restrict__ items, const WalkItem *__restrict__ items_mid,
    const uint32_t *__restrict__ gctr, uint64_t cap, const double *__restrict__ sx,
    const double *__restrict__ sy, const double *__restrict__ sz,
    const uint32_t *__restrict__ orig, const double *__restrict__ R,
    const PatchInfo *__restrict__ patch, const uint32_t *__restrict__ starts,
    const uint32_t *__restrict__ nlive, const uint32_t *__restrict__ root,
    const uint32_t *__restrict__ nfirst, const uint32_t *__restrict__ nlast,
    const uint32_t *__restrict__ nchild, const uint32_t *__restrict__ nlastchild,
    const uint8_t *__restrict__ nlevel, const uint8_t *__restrict__ nleaf, int ngx, int ngy,
    int boundary, double omega, double t, const unsigned long long *__restrict__ rmax_bits,
    uint64_t *__restrict__ queue, uint32_t qcap, uint32_t *__restrict__ qcnt,
    uint32_t *__restrict__ err) {
  __shared__ uint32_t stk_all[4][CG_SCAP];
  __shared__ uint32_t leaf_all[4][CG_LL];
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  uint32_t *stk = stk_all[wv];
  uint32_t *lf = leaf_all[wv];
  const uint32_t n_big = gctr[2], n_mid = gctr[3], n_items = n_big + n_mid + gctr[4];
  for (uint32_t item = 4u * blockIdx.x + wv; item < n_items; item += 4u * gridDim.x) {
    const WalkItem it = rb_walk_item(items, items_mid, item, n_big, n_mid, cap);
    const uint32_t p = it.patch, st = starts[p];
    const uint32_t s = it.start + lane;
    const bool act = s < it.end && it.end - it.start <= 64u && s - st < nlive[p];
    if (!__ballot(act)) continue;
    const PatchInfo pi = patch[p];
    const double W = pi.W;
    const double sh = (boundary == RB_SHEAR) ? remainder(1.5 * omega * W * t, W) : 0.0;
    const double xi = act ? sx[s] : 0.0, yi = act ? sy[s] : 0.0, zi = act ? sz[s] : 0.0;
    const uint32_t oi = act ? orig[s] : 0u;
    const double Ri = act ? R[oi] : 0.0;
    const double lx = rb_wave_min_d(act ? xi : INFINITY);
    const double hx = rb_wave_max_d(act ? xi : -INFINITY);
    const double ly = rb_wave_min_d(act ? yi : INFINITY);
    const double hy = rb_wave_max_d(act ? yi : -INFINITY);
    const double lz = rb_wave_min_d(act ? zi : INFINITY);
    const double hz = rb_wave_max_d(act ? zi : -INFINITY);
    const double Rg = rb_wave_max_d(act ? Ri : 0.0);
    const double reach = Rg + __longlong_as_double((long long)rmax_bits[0]);
    const double hd = 0.8660254037844386;  // half the diagonal of a unit cube
    const int n_img = (boundary == RB_OPEN) ? 1 : (2 * ngx + 1) * (2 * ngy + 1);
    uint64_t mine[RB_COLL_LOCAL];
    uint32_t nm = 0;
    int sp = 0;
    for (int k = lane; k < n_img; k += 64) stk[k] = (root[p] << 5) | (uint32_t)k;
    sp = n_img;
    int nl = 0;
    coll_wave_sync();
    for (;;) {
      int T = sp < 64 ? sp : 64;
      if (sp + 7 * T > CG_SCAP - CG_RESERVE) {
        T = (CG_SCAP - CG_RESERVE - sp) / 7;
        if (T < 1) T = (sp > 0) ? 1 : 0;
      }
      // test the opened leaves against the lanes' particles
      if (nl >= 64 || (T == 0 && nl > 0)) {
        for (int q = 0; q < nl; ++q) {
          const uint32_t en = lf[q];
          const uint32_t node = en >> 5;
          const int k = (int)(en & 31u);
          double ox, oy, wy;
          rb_coll_image(k, ngx, ngy, boundary, W, sh, omega, ox, oy, wy);
          const bool self_img = ox == 0.0 && oy == 0.0;
          const uint32_t jl = nlast[node];
          for (uint32_t j = nfirst[node]; j <= jl; ++j) {
            const uint32_t oj = orig[j];
            if (!act || (j == s && self_img) || oi >= oj) continue;
            const double d0 = (sx[j] + ox) - xi;
            const double d1 = (sy[j] + oy) - yi;
            const double d2 = (sz[j] + 0.0) - zi;
            const double sum = Ri + R[oj];
            if (d0 * d0 + d1 * d1 + d2 * d2 < sum * sum)
              rb_coll_keep(((uint64_t)oi << 35) | ((uint64_t)oj << 7) | (uint64_t)k, mine, nm,
                           queue, qcap, qcnt, err);
          }
        }
        nl = 0;
      }
      if (T == 0) break;  // uniform
      const int base = sp - T;
      const bool has = (int)lane < T;
      const uint32_t e = has ? stk[base + (int)lane] : 0u;
      coll_wave_sync();
      sp = base;
      bool open = false, leaf = false;
      uint32_t c0 = 0, nc = 0;
      if (has) {
        const uint32_t node = e >> 5;
        const int k = (int)(e & 31u);
        double ox, oy, wy;
        rb_coll_image(k, ngx, ngy, boundary, W, sh, omega, ox, oy, wy);
        const int l = nlevel[node];
        const double w = ldexp(W, -l);
        const uint32_t f = nfirst[node];
        uint32_t qx = 0, qy = 0, qz = 0;
        (void)rb_quantise(sx[f], pi.x0[0], W, pi.S, qx);
        (void)rb_quantise(sy[f], pi.x0[1], W, pi.S, qy);
        (void)rb_quantise(sz[f], pi.x0[2], W, pi.S, qz);
        const int sft = RB_DEPTH - l;
        const double cx = pi.x0[0] + ((double)(qx >> sft) + 0.5) * w + ox;
        const double cy = pi.x0[1] + ((double)(qy >> sft) + 0.5) * w + oy;
        const double cz = pi.x0[2] + ((double)(qz >> sft) + 0.5) * w;
        const double dx = fmax(fmax(lx - cx, cx - hx), 0.0);
        const double dy = fmax(fmax(ly - cy, cy - hy), 0.0);
        const double dz = fmax(fmax(lz - cz, cz - hz), 0.0);
        const double lim = (reach + hd * w) * (1.0 + 1e-9);
        open = dx * dx + dy * dy + dz * dz < lim * lim;
        leaf = nleaf[node] != 0;
        if (open && !leaf) {
          c0 = nchild[node];
          const uint32_t c1 = nlastchild[node];
          nc = (c1 >= c0 && c1 - c0 < 8) ? c1 - c0 + 1 : 0;
          if (c1 < c0 || c1 - c0 >= 8) atomicOr(err, RB_ERR_TREE);
        }
      }
      // opened internal nodes push their children, opened leaves join the list
      const uint32_t incl = rb_wave_incl_scan(nc);
      const uint32_t tot = (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl(incl, 63, 64));
      if (sp + (int)tot > CG_SCAP) {  // cannot happen with the reserve above
        if (lane == 0) atomicOr(err, RB_ERR_STACK);
        break;
      }
      for (uint32_t q = 0; q < nc; ++q)
        stk[sp + (int)(incl - nc + q)] = ((c0 + q) << 5) | (e & 31u);
      sp += (int)tot;
      const uint64_t lm = __ballot(open && leaf);
      if (open && leaf) lf[nl + (int)rb_mbcnt(lm)] = e;
      nl += __popcll(lm);
      coll_wave_sync();
    }
    // the rest: one atomic per wave
    const uint32_t incl = rb_wave_incl_scan(nm);
    const uint32_t tot = __shfl(incl, 63, 64);
    uint32_t qbase = 0;
    if (lane == 63 && tot) qbase = atomicAdd(qcnt, tot);
    qbase = __shfl(qbase, 63, 64);
    const uint32_t at = qbase + incl - nm;
    for (uint32_t q = 0; q < nm; ++q)
      if (at + q < qcap) queue[at + q] = mine[q];
    if (nm && at + nm > qcap) atomicOr(err, RB_ERR_COLL);
  }
}

// round, step 1: every particle learns the smallest h among its unresolved
// collisions
__global__ __launch_bounds__(256) void k_coll_min(const uint64_t *__restrict__ list,
                                                  const uint32_t *__restrict__ cnt,
                                                  uint64_t seed,
                                                  unsigned long long *__restrict__ best) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= cnt[0]) return;
  const uint64_t c = list[q];
  const unsigned long long h = rb_splitmix64(seed + c);
  atomicMin(&best[c >> 35], h);
  atomicMin(&best[(c >> 7) & ((1ull << 28) - 1ull)], h);
}

// round, step 2: collisions first in line for both particles are resolved;
// the others go to the next round's list
__global__ __launch_bounds__(256) void k_coll_resolve(
    const uint64_t *__restrict__ list, const uint32_t *__restrict__ cnt,
    uint64_t *__restrict__ next, uint32_t *__restrict__ next_cnt, uint64_t seed,
    const unsigned long long *__restrict__ best, double *__restrict__ x,
    double *__restrict__ y, double *__restrict__ z, double *__restrict__ vx,
    double *__restrict__ vy, double *__restrict__ vz, const double *__restrict__ m,
    const PatchInfo *__restrict__ patch, const uint32_t *__restrict__ starts, uint32_t P,
    int ngx, int ngy, int boundary, double omega, double t, double eps,
    unsigned long long *__restrict__ n_res) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = q < cnt[0];
  uint64_t c = 0;
  bool ready = false;
  if (in) {
    c = list[q];
    const unsigned long long h = rb_splitmix64(seed + c);
    ready = best[c >> 35] == h && best[(c >> 7) & ((1ull << 28) - 1ull)] == h;
  }
  bool resolved = false;
  if (ready) {
    const uint32_t i = (uint32_t)(c >> 35), j = (uint32_t)((c >> 7) & ((1ull << 28) - 1ull));
    const int k = (int)(c & 127ull);
    const uint32_t p = (P == 1) ? 0u : rb_patch_of(starts, P, i);
    const double W = patch[p].W;
    const double sh = (boundary == RB_SHEAR) ? remainder(1.5 * omega * W * t, W) : 0.0;
    double ox, oy, wy;
    rb_coll_image(k, ngx, ngy, boundary, W, sh, omega, ox, oy, wy);
    const double d0 = (x[j] + ox) - x[i];
    const double d1 = (y[j] + oy) - y[i];
    const double d2 = (z[j] + 0.0) - z[i];
    const double u0 = vx[j] - vx[i];
    const double u1 = (vy[j] + wy) - vy[i];
    const double u2 = vz[j] - vz[i];
    const double M = m[i] + m[j];
    if (d0 * u0 + d1 * u1 + d2 * u2 < 0.0 && M > 0.0) {
      const double dist = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      const double n0 = d0 / dist, n1 = d1 / dist, n2 = d2 / dist;
      const double vn = n0 * u0 + n1 * u1 + n2 * u2;
      const double f = (1.0 + eps) * vn;
      const double fi = (m[j] / M) * f, fj = (m[i] / M) * f;
      vx[i] = vx[i] + fi * n0; vy[i] = vy[i] + fi * n1; vz[i] = vz[i] + fi * n2;
      vx[j] = vx[j] - fj * n0; vy[j] = vy[j] - fj * n1; vz[j] = vz[j] - fj * n2;
      resolved = true;
    }
  }
  const uint64_t rm = __ballot(resolved);
  if (rb_lane() == 0 && rm) atomicAdd(n_res, (unsigned long long)__popcll(rm));
  // survivors to the next list, one atomic per wave
  const bool keep = in && !ready;
  const uint64_t km = __ballot(keep);
  uint32_t base = 0;
  if (rb_lane() == 0 && km) base = atomicAdd(next_cnt, (uint32_t)__popcll(km));
  base = __shfl(base, 0, 64);
  if (keep) next[base + rb_mbcnt(km)] = c;
}

// round, step 3: the particles of this round's collisions forget their
// minimum (ready for the next round)
__global__ __launch_bounds__(256) void k_coll_reset(const uint64_t *__restrict__ list,
                                                    const uint32_t *__restrict__ cnt,
                                                    unsigned long long *__restrict__ best) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= cnt[0]) return;
  const uint64_t c = list[q];
  best[c >> 35] = ~0ull;
  best[(c >> 7) & ((1ull << 28) - 1ull)] = ~0ull;
}

hipError_t launch_coll_detect(rb_ctx *c, const double *radius, double t) {
  const uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  const unsigned grid = rb_div_up(n, 256);
  hipLaunchKernelGGL(k_coll_rmax, dim3(grid), dim3(256), 0, c->stream, radius, c->d_orig[0],
                     c->d_starts, c->d_nlive, c->P, n, c->d_cmax);
  hipError_t e = launch_groups(c);
  if (e != hipSuccess) return e;
  unsigned ggrid = rb_div_up(n, 64);
  if (ggrid > 2048) ggrid = 2048;
  hipLaunchKernelGGL(k_coll_detect, dim3(ggrid), dim3(256), 0, c->stream, c->d_witems,
                     c->d_witems_mid, c->d_gctr, c->cap, c->d_px[0][0], c->d_px[0][1],
                     c->d_px[0][2],
                     c->d_orig[0], radius, c->d_patch, c->d_starts, c->d_nlive, c->d_root,
                     c->d_nfirst, c->d_nlast, c->d_nchild, c->d_nlastchild, c->d_nlevel,
                     c->d_nleaf, c->p.n_ghost[0], c->p.n_ghost[1], c->p.boundary, c->p.omega,
                     t, c->d_cmax, c->d_cq[0], (uint32_t)c->cq_cap, c->d_ccnt, c->d_err);
  return hipGetLastError();
}

// One round over list `a` (count d_ccnt[a]) into list 1 - a.
hipError_t launch_coll_round(rb_ctx *c, int a, const rb_particles *pp, double t, double eps,
                             uint64_t seed, uint32_t count) {
  if (count == 0) return hipSuccess;
  const unsigned grid = rb_div_up(count, 256);
  uint32_t *cnt = c->d_ccnt + a, *next_cnt = c->d_ccnt + (1 - a);
  hipLaunchKernelGGL(k_coll_min, dim3(grid), dim3(256), 0, c->stream, c->d_cq[a], cnt, seed,
                     c->d_cbest);
  hipLaunchKernelGGL(k_coll_resolve, dim3(grid), dim3(256), 0, c->stream, c->d_cq[a], cnt,
                     c->d_cq[1 - a], next_cnt, seed, c->d_cbest, pp->x, pp->y, pp->z, pp->vx,
                     pp->vy, pp->vz, pp->m, c->d_patch, c->d_starts, c->P, c->p.n_ghost[0],
                     c->p.n_ghost[1], c->p.boundary, c->p.omega, t, eps, c->d_cres);
  hipLaunchKernelGGL(k_coll_reset, dim3(grid), dim3(256), 0, c->stream, c->d_cq[a], cnt,
                     c->d_cbest);
  return hipGetLastError();
}
