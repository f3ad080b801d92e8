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


__device__ __forceinline__ uint64_t rb_splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// largest radius of the live particles (as ordered bits of a non-negative
// double): slots strided over the grid, one atomic per workgroup
__global__ __launch_bounds__(256) void k_coll_rmax(const double *__restrict__ R,
                                                   const uint32_t *__restrict__ orig,
                                                   const uint32_t *__restrict__ starts,
                                                   const uint32_t *__restrict__ nlive,
                                                   uint32_t P, uint32_t n,
                                                   unsigned long long *__restrict__ rmax) {
  __shared__ double part[4];
  double r = 0.0;
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
    const uint32_t p = (P == 1) ? 0u : rb_patch_of(starts, P, s);
    if (s - starts[p] < nlive[p]) {
      const double v = R[orig[s]];
      r = v > r ? v : r;  // (a NaN radius is never larger)
    }
  }
  for (int d = 32; d >= 1; d >>= 1) r = fmax(r, __shfl_xor(r, d, 64));
  if (rb_lane() == 0) part[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    r = fmax(fmax(part[0], part[1]), fmax(part[2], part[3]));
    if (r > 0.0) atomicMax(rmax, (unsigned long long)__double_as_longlong(r));
  }
}

// order a wave's LDS writes before its later reads (a wave runs in lockstep)
__device__ __forceinline__ void coll_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

#define CG_SCAP 768   // traversal stack entries per wave (node << 5 | image)
#define CG_RESERVE (7 * RB_DEPTH + 8)
#define CG_LL 128     // opened-leaf list capacity per wave (tested at >= 64)
#ifndef CG_SUB
#define CG_SUB 16     // particles one wave searches for (64 / CG_SUB lanes each)
#endif

__device__ __forceinline__ double rb_wave_min_d(double v) {
  for (int d = 32; d >= 1; d >>= 1) v = fmin(v, __shfl_xor(v, d, 64));
  return v;
}
__device__ __forceinline__ double rb_wave_max_d(double v) {
  for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
  return v;
}

// The cell as the search reads it (one 32-byte record): the centre of the
// cell in its own root box, a = first child (internal) or first slot (leaf),
// b = leaf << 31 | level << 26 | (children - 1, or last slot - first slot).
struct __align__(32) CollNode {
  double cx, cy, cz;
  uint32_t a, b;
};

// the cells' records, from the topology of the sorted particles
__global__ __launch_bounds__(256) void k_coll_geom(
    const double *__restrict__ sx, const double *__restrict__ sy, const double *__restrict__ sz,
    const PatchInfo *__restrict__ patch, const uint32_t *__restrict__ starts, uint32_t P,
    const uint32_t *__restrict__ lev_off, uint64_t node_cap,
    const uint32_t *__restrict__ nfirst, const uint32_t *__restrict__ nlast,
    const uint32_t *__restrict__ nchild, const uint32_t *__restrict__ nlastchild,
    const uint8_t *__restrict__ nlevel, const uint8_t *__restrict__ nleaf,
    CollNode *__restrict__ out, uint32_t *__restrict__ err, uint32_t *__restrict__ clear) {
  const uint32_t node = blockIdx.x * blockDim.x + threadIdx.x;
  // (collisions inside a step: the counters of this step start at zero)
  if (clear && node < 10) clear[node] = 0u;
  const uint64_t total = lev_off[RB_NLEV];
  if (node >= total || node >= node_cap) return;
  const uint32_t f = nfirst[node];
  const uint32_t p = (P == 1) ? 0u : rb_patch_of(starts, P, f);
  const PatchInfo pi = patch[p];
  const int l = nlevel[node];
  const double w = ldexp(pi.W, -l);
  uint32_t qx = 0, qy = 0, qz = 0;
  (void)rb_quantise(sx[f], pi.x0[0], pi.L[0], pi.S, pi.qtop[0], qx);
  (void)rb_quantise(sy[f], pi.x0[1], pi.L[1], pi.S, pi.qtop[1], qy);
  (void)rb_quantise(sz[f], pi.x0[2], pi.L[2], pi.S, pi.qtop[2], qz);
  const int sft = RB_DEPTH - l;
  CollNode r;
  r.cx = pi.x0[0] + ((double)(qx >> sft) + 0.5) * w;
  r.cy = pi.x0[1] + ((double)(qy >> sft) + 0.5) * w;
  r.cz = pi.x0[2] + ((double)(qz >> sft) + 0.5) * w;
  if (nleaf[node]) {
    const uint32_t span = nlast[node] - f;
    if (nlast[node] < f || span >= (1u << 26)) atomicOr(err, RB_ERR_TREE);
    r.a = f;
    r.b = 0x80000000u | ((uint32_t)l << 26) | (span & ((1u << 26) - 1u));
  } else {
    const uint32_t c0 = nchild[node], c1 = nlastchild[node];
    const bool ok = c1 >= c0 && c1 - c0 < 8;
    if (!ok) atomicOr(err, RB_ERR_TREE);
    r.a = c0;
    // a broken range is treated as a childless cell (flagged above)
    r.b = ((uint32_t)l << 26) | (ok ? c1 - c0 : 0u) | (ok ? 0u : 0x8u);
  }
  out[node] = r;
}

// One wave searches for CG_SUB particles of a work item (consecutive sibling
// subtrees of at most group_size particles; an item is split into parts of
// CG_SUB slots, one part per wave), 64 / CG_SUB lanes per particle.  Four
// waves per workgroup, parts strided over the grid.
//
// STEP: the search at the end of a step, on the tree built mid-step.  The
// particles have moved by at most D (the largest displacement) since, and
// some have been wrapped into the box: the search runs on their unwrapped
// positions x^u = x + o(w) (w the image the wrap moved them out of) with
// every cell's reach widened by D, and a pair found through image k' of the
// unwrapped positions is the pair through image k' + w_j - w_i of the
// wrapped ones, where the contact test is evaluated.
template <bool STEP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_coll_detect(
    const WalkItem *__restrict__ items, const WalkItem *__restrict__ items_mid,
    const uint32_t *__restrict__ gctr, uint64_t cap, const double *__restrict__ sx,
    const double *__restrict__ sy, const double *__restrict__ sz,
    const uint32_t *__restrict__ orig, const double *__restrict__ R,
    const PatchInfo *__restrict__ patch, const uint32_t *__restrict__ starts,
    const uint32_t *__restrict__ nlive, const uint32_t *__restrict__ root,
    const CollNode *__restrict__ cells, int ngx, int ngy, int boundary, double omega, double t,
    const unsigned long long *__restrict__ rmax_bits, uint64_t *__restrict__ queue,
    uint32_t qcap, uint32_t *__restrict__ qcnt, uint32_t *__restrict__ err,
    const uint16_t *__restrict__ wrap, const unsigned long long *__restrict__ disp_bits,
    const double *__restrict__ sched, const uint32_t *__restrict__ ctr, int slot,
    uint32_t P) {
  constexpr uint32_t NS = 64 / CG_SUB;  // parts per item (items hold <= 64 slots)
  __shared__ uint32_t stk_all[4][CG_SCAP];
  __shared__ uint32_t lfa_all[4][CG_LL], lfb_all[4][CG_LL], lsc_all[4][64];
  // staged candidates: position, radius, caller index, image (ix + 8) |
  // (iy + 8) << 4 of the unwrapped search plus the candidate's own wrap
  __shared__ double cx_all[4][64], cy_all[4][64], cz_all[4][64], cr_all[4][64];
  __shared__ uint32_t co_all[4][64];
  __shared__ uint8_t ck_all[4][64];
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  uint32_t *stk = stk_all[wv];
  uint32_t *lfa = lfa_all[wv], *lfb = lfb_all[wv], *lsc = lsc_all[wv];
  double *cx_ = cx_all[wv], *cy_ = cy_all[wv], *cz_ = cz_all[wv], *cr_ = cr_all[wv];
  uint32_t *co_ = co_all[wv];
  uint8_t *ck_ = ck_all[wv];
  const uint32_t pidx = lane % CG_SUB, sub = lane / CG_SUB;
  const uint32_t n_big = gctr[2], n_mid = gctr[3], n_items = n_big + n_mid + gctr[4];
  const double rmax = __longlong_as_double((long long)rmax_bits[0]);
  const double slack = STEP ? __longlong_as_double((long long)disp_bits[0]) : 0.0;
  const double hd = 0.8660254037844386;  // half the diagonal of a unit cube
  const int n_img = (boundary == RB_OPEN) ? 1 : (2 * ngx + 1) * (2 * ngy + 1);
  const int ny = 2 * ngy + 1;
  const double *s_end = STEP ? sched + (size_t)ctr[slot] * 2 * P + P : nullptr;
  for (uint32_t u = 4u * blockIdx.x + wv; u < n_items * NS; u += 4u * gridDim.x) {
    const WalkItem it = rb_walk_item(items, items_mid, u / NS, n_big, n_mid, cap);
    const uint32_t s0 = it.start + (u % NS) * CG_SUB;
    if (s0 >= it.end || it.end - it.start > 64u) continue;  // uniform
    const uint32_t p = it.patch, st = starts[p];
    const uint32_t s = s0 + pidx;
    bool act = s < it.end && s - st < nlive[p];
    if (STEP && act) act = !isnan(sx[s]);  // (left an open box this step)
    if (!__ballot(act)) continue;
    const PatchInfo pi = patch[p];
    const double W = pi.W;
    const double sh = (boundary != RB_SHEAR) ? 0.0
                      : STEP ? s_end[p] : remainder(1.5 * omega * W * t, W);
    const double xi = act ? sx[s] : 0.0, yi = act ? sy[s] : 0.0, zi = act ? sz[s] : 0.0;
    const uint32_t oi = act ? orig[s] : 0u;
    const double Ri = act ? R[oi] : 0.0;
    int wxi = 0, wyi = 0;  // the lane's own wrap
    double qx = xi, qy = yi;
    if (STEP && act) {
      const uint32_t wb = wrap[s];
      wxi = (int)(wb & 15u) - 2;
      wyi = (int)(wb >> 4) - 2;
      double ox, oy, wy;
      rb_coll_image_xy(wxi, wyi, boundary, W, sh, omega, ox, oy, wy);
      qx = xi + ox;
      qy = yi + oy;
    }
    const double lx = rb_wave_min_d(act ? qx : INFINITY);
    const double hx = rb_wave_max_d(act ? qx : -INFINITY);
    const double ly = rb_wave_min_d(act ? qy : INFINITY);
    const double hy = rb_wave_max_d(act ? qy : -INFINITY);
    const double lz = rb_wave_min_d(act ? zi : INFINITY);
    const double hz = rb_wave_max_d(act ? zi : -INFINITY);
    const double reach = rb_wave_max_d(act ? Ri : 0.0) + rmax + slack;
    uint64_t mine[RB_COLL_LOCAL];
    uint32_t nm = 0;
    for (int k = lane; k < n_img; k += 64) stk[k] = (root[p] << 5) | (uint32_t)k;
    int sp = n_img;
    int nl = 0;
    coll_wave_sync();
    for (;;) {
      int T = sp < 64 ? sp : 64;
      if (sp + 7 * T > CG_SCAP - CG_RESERVE) {
        T = (CG_SCAP - CG_RESERVE - sp) / 7;
        if (T < 1) T = (sp > 0) ? 1 : 0;
      }
      // test the opened leaves' particles against the lanes' particles: up
      // to 64 leaves at a time, their particles staged in LDS 64 at a time
      // (image-shifted, one load per lane), candidate q then tested by the
      // lanes with sub = q mod (64 / CG_SUB)
      if (nl >= 64 || (T == 0 && nl > 0)) {
        for (int lb = 0; lb < nl; lb += 64) {
          const int L = min(64, nl - lb);
          const uint32_t cntq = (int)lane < L ? (lfb[lb + (int)lane] >> 5) + 1u : 0u;
          const uint32_t incl = rb_wave_incl_scan(cntq);
          const uint32_t M =
              (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl(incl, 63, 64));
          lsc[lane] = incl;
          coll_wave_sync();
          for (uint32_t e0 = 0; e0 < M; e0 += 64) {
            const uint32_t e = e0 + lane;
            if (e < M) {
              int lo = 0, hi = L - 1;  // first leaf whose inclusive count exceeds e
              while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (lsc[mid] > e) hi = mid; else lo = mid + 1;
              }
              const uint32_t eb = lfb[lb + lo];
              const uint32_t j = lfa[lb + lo] + (e - (lsc[lo] - ((eb >> 5) + 1u)));
              const int k = (int)(eb & 31u);
              const uint32_t oj = orig[j];
              if (STEP) {
                // raw position and the image relative to the box both wraps
                // are counted from (the lane's own wrap is taken off later)
                const uint32_t wb = wrap[j];
                const int kx = ((boundary == RB_OPEN) ? 0 : k / ny - ngx) + (int)(wb & 15u) - 2;
                const int ky = ((boundary == RB_OPEN) ? 0 : k % ny - ngy) + (int)(wb >> 4) - 2;
                cx_[lane] = sx[j];
                cy_[lane] = sy[j];
                ck_[lane] = (uint8_t)((kx + 8) | ((ky + 8) << 4));
              } else {
                // the image-shifted position (the lanes' particles are in the box)
                double ox, oy, wy;
                rb_coll_image(k, ngx, ngy, boundary, W, sh, omega, ox, oy, wy);
                cx_[lane] = sx[j] + ox;
                cy_[lane] = sy[j] + oy;
                ck_[lane] = (uint8_t)k;
              }
              cz_[lane] = sz[j];
              cr_[lane] = R[oj];
              co_[lane] = oj;
            }
            coll_wave_sync();
            const int C = (int)min(64u, M - e0);
            if (act) {
              for (int q = (int)sub; q < C; q += (int)NS) {
                const uint32_t oj = co_[q];
                if (oi >= oj) continue;  // each pair once, from its lower caller index
                const uint32_t kb = ck_[q];
                double d0, d1;
                uint32_t kc;
                if (STEP) {
                  // the image of j relative to i in the (wrapped) box
                  const int ix = (int)(kb & 15u) - 8 - wxi, iy = (int)(kb >> 4) - 8 - wyi;
                  if (ix < -ngx || ix > ngx || iy < -ngy || iy > ngy) continue;
                  double ox, oy, wy;
                  rb_coll_image_xy(ix, iy, boundary, W, sh, omega, ox, oy, wy);
                  d0 = (cx_[q] + ox) - xi;
                  d1 = (cy_[q] + oy) - yi;
                  kc = (boundary == RB_OPEN) ? 0u : (uint32_t)((ix + ngx) * ny + (iy + ngy));
                } else {
                  d0 = cx_[q] - xi;
                  d1 = cy_[q] - yi;
                  kc = (boundary == RB_OPEN) ? 0u : kb;
                }
                const double d2 = cz_[q] - zi;
                const double sum = Ri + cr_[q];
                if (d0 * d0 + d1 * d1 + d2 * d2 < sum * sum)
                  rb_coll_keep(((uint64_t)oi << 35) | ((uint64_t)oj << 7) | (uint64_t)kc,
                               mine, nm, queue, qcap, qcnt, err);
              }
            }
            coll_wave_sync();
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
      uint32_t c0 = 0, nc = 0, span = 0;
      if (has) {
        const CollNode cn = cells[e >> 5];
        const int k = (int)(e & 31u);
        double ox, oy, wy;
        rb_coll_image(k, ngx, ngy, boundary, W, sh, omega, ox, oy, wy);
        const int l = (int)((cn.b >> 26) & 31u);
        const double w = ldexp(W, -l);
        const double cx = cn.cx + ox, cy = cn.cy + oy, cz = cn.cz;
        const double dx = fmax(fmax(lx - cx, cx - hx), 0.0);
        const double dy = fmax(fmax(ly - cy, cy - hy), 0.0);
        const double dz = fmax(fmax(lz - cz, cz - hz), 0.0);
        const double lim = (reach + hd * w) * (1.0 + 1e-9);
        open = dx * dx + dy * dy + dz * dz < lim * lim;
        leaf = (cn.b >> 31) != 0;
        c0 = cn.a;
        span = cn.b & ((1u << 26) - 1u);
        // (a flagged broken child range has bit 3 set and opens nothing)
        if (open && !leaf && span < 8u) nc = span + 1u;
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
      if (open && leaf) {
        const int at = nl + (int)rb_mbcnt(lm);
        lfa[at] = c0;
        lfb[at] = (span << 5) | (e & 31u);
      }
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

// The rounds run on a fixed grid that strides over the list, whose length
// each kernel reads on the device (at most the queue's capacity), so the host
// launches them without knowing it.
#define CR_GRID 256

// round, step 1: every particle learns the smallest h among its unresolved
// collisions; the next list's count is cleared (that list was the previous
// round's input), and the first round saves the number of detected pairs
__global__ __launch_bounds__(256) void k_coll_min(const uint64_t *__restrict__ list,
                                                  const uint32_t *__restrict__ cnt,
                                                  uint32_t *__restrict__ next_cnt,
                                                  uint32_t *__restrict__ save, uint32_t qcap,
                                                  uint64_t seed,
                                                  unsigned long long *__restrict__ best) {
  const uint32_t n = min(cnt[0], qcap);
  const uint32_t q0 = blockIdx.x * blockDim.x + threadIdx.x;
  if (q0 == 0) {
    next_cnt[0] = 0;
    if (save) save[0] = cnt[0];
  }
  for (uint32_t q = q0; q < n; q += gridDim.x * blockDim.x) {
    const uint64_t c = list[q];
    const unsigned long long h = rb_splitmix64(seed + c);
    atomicMin(&best[c >> 35], h);
    atomicMin(&best[(c >> 7) & ((1ull << 28) - 1ull)], h);
  }
}

// Resolve the collision of code c if its particles approach (d . u < 0);
// returns whether it did.  Each particle takes part in at most one
// collision resolved in a round, so the updates of a round do not race.
// The arrays are in caller order, or (inv given: collisions inside a step)
// in the step's sorted order, inv mapping caller indices to slots; the
// shear offset is taken from the step's schedule row when s_end is given.
__device__ __forceinline__ bool rb_coll_apply(
    uint64_t c, double *__restrict__ x, double *__restrict__ y, double *__restrict__ z,
    double *__restrict__ vx, double *__restrict__ vy, double *__restrict__ vz,
    const double *__restrict__ m, const PatchInfo *__restrict__ patch,
    const uint32_t *__restrict__ starts, uint32_t P, int ngx, int ngy, int boundary,
    double omega, double t, double eps, const uint32_t *__restrict__ inv = nullptr,
    const double *__restrict__ s_end = nullptr) {
  const uint32_t ci = (uint32_t)(c >> 35), cj = (uint32_t)((c >> 7) & ((1ull << 28) - 1ull));
  const int k = (int)(c & 127ull);
  // (patches hold the same ranges in caller and sorted order)
  const uint32_t p = (P == 1) ? 0u : rb_patch_of(starts, P, ci);
  const uint32_t i = inv ? inv[ci] : ci, j = inv ? inv[cj] : cj;
  const double W = patch[p].W;
  const double sh = (boundary != RB_SHEAR) ? 0.0
                    : s_end ? s_end[p] : remainder(1.5 * omega * W * t, W);
  double ox, oy, wy;
  rb_coll_image(k, ngx, ngy, boundary, W, sh, omega, ox, oy, wy);
  const double d0 = (x[j] + ox) - x[i];
  const double d1 = (y[j] + oy) - y[i];
  const double d2 = (z[j] + 0.0) - z[i];
  const double u0 = vx[j] - vx[i];
  const double u1 = (vy[j] + wy) - vy[i];
  const double u2 = vz[j] - vz[i];
  const double M = m[i] + m[j];
  if (!(d0 * u0 + d1 * u1 + d2 * u2 < 0.0 && M > 0.0)) return false;
  const double dist = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  const double n0 = d0 / dist, n1 = d1 / dist, n2 = d2 / dist;
  const double vn = n0 * u0 + n1 * u1 + n2 * u2;
  const double f = (1.0 + eps) * vn;
  const double fi = (m[j] / M) * f, fj = (m[i] / M) * f;
  vx[i] = vx[i] + fi * n0; vy[i] = vy[i] + fi * n1; vz[i] = vz[i] + fi * n2;
  vx[j] = vx[j] - fj * n0; vy[j] = vy[j] - fj * n1; vz[j] = vz[j] - fj * n2;
  return true;
}

// round, step 2: collisions first in line for both particles are resolved;
// the others go to the next round's list
__global__ __launch_bounds__(256) void k_coll_resolve(
    const uint64_t *__restrict__ list, const uint32_t *__restrict__ cnt, uint32_t qcap,
    uint64_t *__restrict__ next, uint32_t *__restrict__ next_cnt, uint64_t seed,
    const unsigned long long *__restrict__ best, double *__restrict__ x,
    double *__restrict__ y, double *__restrict__ z, double *__restrict__ vx,
    double *__restrict__ vy, double *__restrict__ vz, const double *__restrict__ m,
    const PatchInfo *__restrict__ patch, const uint32_t *__restrict__ starts, uint32_t P,
    int ngx, int ngy, int boundary, double omega, double t, double eps,
    unsigned long long *__restrict__ n_res) {
  const uint32_t n = min(cnt[0], qcap);
  // wave-uniform trip count: a wave covers 64 consecutive entries per pass
  const uint32_t wbase = blockIdx.x * blockDim.x + (threadIdx.x & ~63u);
  for (uint32_t q0 = wbase; q0 < n; q0 += gridDim.x * blockDim.x) {
    const uint32_t q = q0 + rb_lane();
    const bool in = q < n;
    uint64_t c = 0;
    bool ready = false;
    if (in) {
      c = list[q];
      const unsigned long long h = rb_splitmix64(seed + c);
      ready = best[c >> 35] == h && best[(c >> 7) & ((1ull << 28) - 1ull)] == h;
    }
    const bool resolved = ready && rb_coll_apply(c, x, y, z, vx, vy, vz, m, patch, starts, P,
                                                 ngx, ngy, boundary, omega, t, eps);
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
}

// round, step 3: the particles of this round's collisions forget their
// minimum (ready for the next round)
__global__ __launch_bounds__(256) void k_coll_reset(const uint64_t *__restrict__ list,
                                                    const uint32_t *__restrict__ cnt,
                                                    uint32_t qcap,
                                                    unsigned long long *__restrict__ best) {
  const uint32_t n = min(cnt[0], qcap);
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += gridDim.x * blockDim.x) {
    const uint64_t c = list[q];
    best[c >> 35] = ~0ull;
    best[(c >> 7) & ((1ull << 28) - 1ull)] = ~0ull;
  }
}

// All remaining rounds in one workgroup, for short lists (at most CR_SMALL
// entries; a longer list is left as it is, for the multi-workgroup rounds).
// The lists ping-pong between l[a] and l[1 - a]; on completion both counts
// are zero.  Being the last kernel before the host reads the counts, it
// copies the error word next to them (cnt[3]).  best[] is read and cleared with device-scope atomics (its
// minima are formed by atomics, which the L1 cache does not see); the
// velocities are plain loads and stores ordered by the workgroup barriers.
#define CR_SMALL 4096
//
// Inside a step (inv given) every queue is resolved here, however long; the
// seed is the step's (seedp[0] + the step index), the shear offset the
// step's end-time offset, and the pairs and resolutions are added to the
// running totals in cum.
__global__ __launch_bounds__(1024) void k_coll_rounds1(
    uint64_t *__restrict__ l0, uint64_t *__restrict__ l1, uint32_t *__restrict__ cnt, int a,
    uint32_t *__restrict__ save, uint32_t qcap, uint64_t seed,
    unsigned long long *__restrict__ best, double *__restrict__ x, double *__restrict__ y,
    double *__restrict__ z, double *__restrict__ vx, double *__restrict__ vy,
    double *__restrict__ vz, const double *__restrict__ m,
    const PatchInfo *__restrict__ patch, const uint32_t *__restrict__ starts, uint32_t P,
    int ngx, int ngy, int boundary, double omega, double t, double eps,
    unsigned long long *__restrict__ n_res, const uint32_t *__restrict__ err,
    const uint32_t *__restrict__ inv, const uint64_t *__restrict__ seedp,
    const double *__restrict__ sched, const uint32_t *__restrict__ ctr, int slot,
    unsigned long long *__restrict__ cum) {
  __shared__ uint32_t s_n, s_next;
  __shared__ unsigned long long s_res;
  const uint32_t tid = threadIdx.x;
  const uint32_t n0 = min(cnt[a], qcap);
  if (tid == 0 && save) save[0] = cnt[a];
  const double *s_end = inv ? sched + (size_t)ctr[slot] * 2 * P + P : nullptr;
  if (inv) seed = seedp[0] + ctr[slot];
  if (!inv && n0 > CR_SMALL) {  // uniform
    if (tid == 0) cnt[3] = err[0];
    return;
  }
  if (tid == 0) {
    s_n = n0;
    s_res = 0;
  }
  uint64_t *cur = a ? l1 : l0, *nxt = a ? l0 : l1;
  __syncthreads();
  for (;;) {
    const uint32_t n = s_n;
    if (n == 0) break;  // uniform
    if (tid == 0) s_next = 0;
    for (uint32_t q = tid; q < n; q += blockDim.x) {
      const uint64_t c = cur[q];
      const unsigned long long h = rb_splitmix64(seed + c);
      atomicMin(&best[c >> 35], h);
      atomicMin(&best[(c >> 7) & ((1ull << 28) - 1ull)], h);
    }
    __syncthreads();
    for (uint32_t q0 = tid & ~63u; q0 < n; q0 += blockDim.x) {
      const uint32_t q = q0 + rb_lane();
      const bool in = q < n;
      uint64_t c = 0;
      bool ready = false;
      if (in) {
        c = cur[q];
        const unsigned long long h = rb_splitmix64(seed + c);
        ready = __hip_atomic_load(&best[c >> 35], __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT) == h &&
                __hip_atomic_load(&best[(c >> 7) & ((1ull << 28) - 1ull)], __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT) == h;
      }
      const bool resolved = ready && rb_coll_apply(c, x, y, z, vx, vy, vz, m, patch, starts,
                                                   P, ngx, ngy, boundary, omega, t, eps, inv,
                                                   s_end);
      const uint64_t rm = __ballot(resolved);
      if (rb_lane() == 0 && rm) atomicAdd(&s_res, (unsigned long long)__popcll(rm));
      const bool keep = in && !ready;
      const uint64_t km = __ballot(keep);
      uint32_t base = 0;
      if (rb_lane() == 0 && km) base = atomicAdd(&s_next, (uint32_t)__popcll(km));
      base = __shfl(base, 0, 64);
      if (keep) nxt[base + rb_mbcnt(km)] = c;
    }
    __syncthreads();
    for (uint32_t q = tid; q < n; q += blockDim.x) {
      const uint64_t c = cur[q];
      __hip_atomic_store(&best[c >> 35], ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&best[(c >> 7) & ((1ull << 28) - 1ull)], ~0ull, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    uint64_t *tmp = cur;
    cur = nxt;
    nxt = tmp;
    __syncthreads();
    if (tid == 0) s_n = s_next;
    __syncthreads();
  }
  if (tid == 0) {
    cnt[0] = 0;
    cnt[1] = 0;
    cnt[3] = err[0];
    if (s_res) atomicAdd(n_res, s_res);
    if (cum) {
      cum[0] += (unsigned long long)n0;
      cum[1] += s_res;
    }
  }
}

// R_max, the cells' records and the work items of the search
hipError_t launch_coll_prep(rb_ctx *c, const double *radius) {
  const uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  const unsigned grid = std::min(rb_div_up(n, 1024), 128u);
  hipLaunchKernelGGL(k_coll_rmax, dim3(grid), dim3(256), 0, c->stream, radius, c->d_orig[0],
                     c->d_starts, c->d_nlive, c->P, n, c->d_cmax);
  CollNode *cells = reinterpret_cast<CollNode *>(c->d_cgeo);
  hipLaunchKernelGGL(k_coll_geom, dim3(rb_div_up(c->node_cap, 256)), dim3(256), 0, c->stream,
                     c->d_px[0][0], c->d_px[0][1], c->d_px[0][2], c->d_patch, c->d_starts, c->P,
                     c->d_lev_off, c->node_cap, c->d_nfirst, c->d_nlast, c->d_nchild,
                     c->d_nlastchild, c->d_nlevel, c->d_nleaf, cells, c->d_err, nullptr);
  return launch_groups(c);
}

hipError_t launch_coll_detect(rb_ctx *c, const double *radius, double t) {
  const uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  CollNode *cells = reinterpret_cast<CollNode *>(c->d_cgeo);
  // about one wave per non-empty item part (parts average over CG_SUB / 2
  // particles); the loop strides over any others
  unsigned ggrid = rb_div_up(n, 4 * CG_SUB / 2);
  if (ggrid > 4096) ggrid = 4096;
  hipLaunchKernelGGL(k_coll_detect<false>, dim3(ggrid), dim3(256), 0, c->stream, c->d_witems,
                     c->d_witems_mid, c->d_gctr, c->cap, c->d_px[0][0], c->d_px[0][1],
                     c->d_px[0][2], c->d_orig[0], radius, c->d_patch, c->d_starts, c->d_nlive,
                     c->d_root, cells, c->p.n_ghost[0], c->p.n_ghost[1], c->p.boundary,
                     c->p.omega, t, c->d_cmax, c->d_cq[0], (uint32_t)c->cq_cap, c->d_ccnt,
                     c->d_err, nullptr, nullptr, nullptr, nullptr, 0, c->P);
  return hipGetLastError();
}

// One round over list `a` (count d_ccnt[a]) into list 1 - a.
hipError_t launch_coll_rounds1(rb_ctx *c, int a, const rb_particles *pp, double t, double eps,
                               uint64_t seed, uint32_t *save) {
  hipLaunchKernelGGL(k_coll_rounds1, dim3(1), dim3(1024), 0, c->stream, c->d_cq[0],
                     c->d_cq[1], c->d_ccnt, a, save, (uint32_t)c->cq_cap, seed, c->d_cbest,
                     pp->x, pp->y, pp->z, pp->vx, pp->vy, pp->vz, pp->m, c->d_patch,
                     c->d_starts, c->P, c->p.n_ghost[0], c->p.n_ghost[1], c->p.boundary,
                     c->p.omega, t, eps, c->d_cres, c->d_err, nullptr, nullptr, nullptr,
                     nullptr, 0, nullptr);
  return hipGetLastError();
}

hipError_t launch_coll_round(rb_ctx *c, int a, const rb_particles *pp, double t, double eps,
                             uint64_t seed, uint32_t *save) {
  uint32_t *cnt = c->d_ccnt + a, *next_cnt = c->d_ccnt + (1 - a);
  const uint32_t qcap = (uint32_t)c->cq_cap;
  hipLaunchKernelGGL(k_coll_min, dim3(CR_GRID), dim3(256), 0, c->stream, c->d_cq[a], cnt,
                     next_cnt, save, qcap, seed, c->d_cbest);
  hipLaunchKernelGGL(k_coll_resolve, dim3(CR_GRID), dim3(256), 0, c->stream, c->d_cq[a], cnt,
                     qcap, c->d_cq[1 - a], next_cnt, seed, c->d_cbest, pp->x, pp->y, pp->z,
                     pp->vx, pp->vy, pp->vz, pp->m, c->d_patch, c->d_starts, c->P,
                     c->p.n_ghost[0], c->p.n_ghost[1], c->p.boundary, c->p.omega, t, eps,
                     c->d_cres);
  hipLaunchKernelGGL(k_coll_reset, dim3(CR_GRID), dim3(256), 0, c->stream, c->d_cq[a], cnt,
                     qcap, c->d_cbest);
  return hipGetLastError();
}

// ---- collisions inside a step (the tree of the step, in its sorted order)

// before the kick: the cells' records from the build's (mid-step)
// positions in buffer buf and the step's counters cleared (R_max and the
// caller-to-slot map come from the first post kernel, k_post<1>)
hipError_t launch_coll_step_prep(rb_ctx *c, int buf) {
  const uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  CollNode *cells = reinterpret_cast<CollNode *>(c->d_cgeo);
  hipLaunchKernelGGL(k_coll_geom, dim3(rb_div_up(c->node_cap, 256)), dim3(256), 0, c->stream,
                     c->d_px[buf][0], c->d_px[buf][1], c->d_px[buf][2], c->d_patch,
                     c->d_starts, c->P, c->d_lev_off, c->node_cap, c->d_nfirst, c->d_nlast,
                     c->d_nchild, c->d_nlastchild, c->d_nlevel, c->d_nleaf, cells, c->d_err,
                     c->d_ccnt);
  return hipGetLastError();
}

// after the second drift (the end-of-step state in buffer buf): the search
hipError_t launch_coll_step_search(rb_ctx *c, int buf, int slot) {
  const uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  CollNode *cells = reinterpret_cast<CollNode *>(c->d_cgeo);
  unsigned ggrid = rb_div_up(n, 4 * CG_SUB / 2);
  if (ggrid > 4096) ggrid = 4096;
  hipLaunchKernelGGL(k_coll_detect<true>, dim3(ggrid), dim3(256), 0, c->stream, c->d_witems,
                     c->d_witems_mid, c->d_gctr, c->cap, c->d_px[buf][0], c->d_px[buf][1],
                     c->d_px[buf][2], c->d_orig[buf], c->coll_R, c->d_patch, c->d_starts,
                     c->d_nlive, c->d_root, cells, c->p.n_ghost[0], c->p.n_ghost[1],
                     c->p.boundary, c->p.omega, 0.0, c->d_cmax, c->d_cq[0],
                     (uint32_t)c->cq_cap, c->d_ccnt, c->d_err, c->d_cwrap,
                     reinterpret_cast<const unsigned long long *>(c->d_ccnt + 8), c->d_sched,
                     c->d_ctr, slot, c->P);
  return hipGetLastError();
}

// then every round of the queue, on the sorted state
hipError_t launch_coll_step_rounds(rb_ctx *c, int buf, int slot) {
  double *const *b = c->d_px[buf];
  hipLaunchKernelGGL(k_coll_rounds1, dim3(1), dim3(1024), 0, c->stream, c->d_cq[0],
                     c->d_cq[1], c->d_ccnt, 0, c->d_ccnt + 2, (uint32_t)c->cq_cap, 0ull,
                     c->d_cbest, b[0], b[1], b[2], b[3], b[4], b[5], b[6], c->d_patch,
                     c->d_starts, c->P, c->p.n_ghost[0], c->p.n_ghost[1], c->p.boundary,
                     c->p.omega, 0.0, c->coll_eps, c->d_cres, c->d_err, c->d_cinv,
                     reinterpret_cast<const uint64_t *>(c->d_ctr + 4), c->d_sched, c->d_ctr,
                     slot, reinterpret_cast<unsigned long long *>(c->d_ccnt + 10));
  return hipGetLastError();
}
