// k_collide.hip -- collisions at the end of a step (Sect. 5 of the paper):
// overlapping pairs found by the octree search of Eq. (3) over the ghost
// boxes, a collision queue in a random order, and hard-sphere resolution
// with a normal coefficient of restitution, one collision after the other in
// queue order.
//
// Detection: one thread per live particle i (Morton order) and ghost image
// o_k walks the tree with the child / skip links of the topology; it descends
// into a cell while the distance from x_i to the image-shifted cell centre is
// below R_i + R_max + (sqrt 3 / 2) w (every particle of the cell that could
// overlap i passes this test, so the search finds every overlap).  In a leaf,
// j overlaps i when |x_j + o_k - x_i| < R_i + R_j; the pair is queued once,
// from its lower caller index i, as the code i 2^35 + j 2^7 + k.
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

__global__ __launch_bounds__(256) void k_coll_detect(
    const double *__restrict__ sx, const double *__restrict__ sy, const double *__restrict__ sz,
    const uint32_t *__restrict__ orig, const double *__restrict__ R,
    const PatchInfo *__restrict__ patch, const uint32_t *__restrict__ starts,
    const uint32_t *__restrict__ nlive, const uint32_t *__restrict__ root,
    const uint32_t *__restrict__ nfirst, const uint32_t *__restrict__ nlast,
    const uint32_t *__restrict__ nchild, const uint32_t *__restrict__ nskip,
    const uint8_t *__restrict__ nlevel, const uint8_t *__restrict__ nleaf, uint32_t P,
    uint32_t n, int ngx, int ngy, int boundary, double omega, double t,
    const unsigned long long *__restrict__ rmax_bits, uint64_t *__restrict__ queue,
    uint32_t qcap, uint32_t *__restrict__ qcnt, uint32_t *__restrict__ err) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t mine[RB_COLL_LOCAL];
  uint32_t nm = 0;
  bool live = false;
  if (s < n) {
    const uint32_t p = (P == 1) ? 0u : rb_patch_of(starts, P, s);
    live = s - starts[p] < nlive[p];
    if (live) {
      const PatchInfo pi = patch[p];
      const double W = pi.W;
      const double sh = (boundary == RB_SHEAR) ? remainder(1.5 * omega * W * t, W) : 0.0;
      const double xi = sx[s], yi = sy[s], zi = sz[s];
      const uint32_t oi = orig[s];
      const double Ri = R[oi];
      const double reach = Ri + __longlong_as_double((long long)rmax_bits[0]);
      const double hd = 0.8660254037844386;  // half the diagonal of a unit cube
      const int n_img = (boundary == RB_OPEN) ? 1 : (2 * ngx + 1) * (2 * ngy + 1);
      for (int k = 0; k < n_img; ++k) {
        double ox, oy, wy;
        rb_coll_image(k, ngx, ngy, boundary, W, sh, omega, ox, oy, wy);
        const bool self_img = ox == 0.0 && oy == 0.0;
        uint32_t node = root[p];
        while (node != RB_NONE) {
          const int l = nlevel[node];
          const double w = ldexp(W, -l);
          // centre of the cell: the level-l cell of its first particle
          const uint32_t f = nfirst[node];
          uint32_t qx = 0, qy = 0, qz = 0;
          (void)rb_quantise(sx[f], pi.x0[0], W, pi.S, qx);
          (void)rb_quantise(sy[f], pi.x0[1], W, pi.S, qy);
          (void)rb_quantise(sz[f], pi.x0[2], W, pi.S, qz);
          const int sft = RB_DEPTH - l;
          const double cx = pi.x0[0] + ((double)(qx >> sft) + 0.5) * w + ox;
          const double cy = pi.x0[1] + ((double)(qy >> sft) + 0.5) * w + oy;
          const double cz = pi.x0[2] + ((double)(qz >> sft) + 0.5) * w;
          const double ex = cx - xi, ey = cy - yi, ez = cz - zi;
          const double lim = (reach + hd * w) * (1.0 + 1e-9);
          if (!(ex * ex + ey * ey + ez * ez < lim * lim)) {
            node = nskip[node];
            continue;
          }
          if (!nleaf[node]) {
            node = nchild[node];
            continue;
          }
          const uint32_t jl = nlast[node];
          for (uint32_t j = f; j <= jl; ++j) {
            if (j == s && self_img) continue;
            const uint32_t oj = orig[j];
            if (oi >= oj) continue;  // queued from the lower caller index
            const double d0 = (sx[j] + ox) - xi;
            const double d1 = (sy[j] + oy) - yi;
            const double d2 = (sz[j] + 0.0) - zi;
            const double sum = Ri + R[oj];
            if (d0 * d0 + d1 * d1 + d2 * d2 < sum * sum) {
              const uint64_t code = ((uint64_t)oi << 35) | ((uint64_t)oj << 7) | (uint64_t)k;
              if (nm == RB_COLL_LOCAL) {  // write out the full local list
                const uint32_t at = atomicAdd(qcnt, (uint32_t)nm);
                for (uint32_t q = 0; q < nm; ++q)
                  if (at + q < qcap) queue[at + q] = mine[q];
                if (at + nm > qcap) atomicOr(err, RB_ERR_COLL);
                nm = 0;
              }
              mine[nm++] = code;
            }
          }
          node = nskip[node];
        }
      }
    }
  }
  // the rest: one atomic per wave
  const uint32_t incl = rb_wave_incl_scan(nm);
  const uint32_t tot = __shfl(incl, 63, 64);
  uint32_t base = 0;
  if (rb_lane() == 63 && tot) base = atomicAdd(qcnt, tot);
  base = __shfl(base, 63, 64);
  const uint32_t at = base + incl - nm;
  for (uint32_t q = 0; q < nm; ++q)
    if (at + q < qcap) queue[at + q] = mine[q];
  if (nm && at + nm > qcap) atomicOr(err, RB_ERR_COLL);
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
  hipLaunchKernelGGL(k_coll_detect, dim3(grid), dim3(256), 0, c->stream, c->d_px[0][0],
                     c->d_px[0][1], c->d_px[0][2], c->d_orig[0], radius, c->d_patch,
                     c->d_starts, c->d_nlive, c->d_root, c->d_nfirst, c->d_nlast, c->d_nchild,
                     c->d_nskip, c->d_nlevel, c->d_nleaf, c->P, n, c->p.n_ghost[0],
                     c->p.n_ghost[1], c->p.boundary, c->p.omega, t, c->d_cmax, c->d_cq[0],
                     (uint32_t)c->cq_cap, c->d_ccnt, c->d_err);
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
