// k_step.hip -- the drift-kick-drift step of Sect. 3 around the tree walk:
// drifts (leap-frog, Sect. 3.1; exact epicycle, Sect. 3.3), the boundaries of
// Sect. 2.3, the kick, the keys of the next step, and the gathers between
// the caller's order and Morton order.
//
// Drift and boundary arithmetic is written operation for operation as the
// plain FP64 formulas, with contraction off, so a step reproduces a
// sequential FP64 implementation of the same formulas exactly.
#include "rb_internal.h"

struct PState {
  double x, y, z, vx, vy, vz;
};

// drift over tau = dt/2
__device__ __forceinline__ void rb_apply_drift(PState &q, int mode, const StepConst &sc) {
#pragma clang fp contract(off)
  if (mode == RB_DRIFT_LEAPFROG) {
    q.x = q.x + q.vx * sc.half;
    q.y = q.y + q.vy * sc.half;
    q.z = q.z + q.vz * sc.half;
    return;
  }
  const double W = sc.omega, Wz = sc.omega_z, tau = sc.half;
  const double C = q.vy + 2.0 * W * q.x;
  const double xg = 2.0 * C / W;
  const double dx = q.x - xg;
  const double u = q.vx / W;
  const double xn = xg + dx * sc.c + u * sc.sn;
  const double vxn = -W * dx * sc.sn + q.vx * sc.c;
  const double yn = q.y - 3.0 * C * tau - 2.0 * dx * sc.sn - 2.0 * u * (1.0 - sc.c);
  const double vyn = C - 2.0 * W * xn;
  const double zn = q.z * sc.cz + q.vz / Wz * sc.sz;
  const double vzn = -Wz * q.z * sc.sz + q.vz * sc.cz;
  q.x = xn; q.vx = vxn; q.y = yn; q.vy = vyn; q.z = zn; q.vz = vzn;
}

// Boundaries at the domain's faces (extents Lx, Ly, Lz): shear-periodic x
// (shift y by s and vy by 1.5 omega Lx), plain periodic x, periodic y; an
// open axis turns a leaving particle into a tombstone (NaN position, zero
// velocity).
__device__ __forceinline__ void rb_apply_boundary(PState &q, int boundary, const PatchInfo &pi,
                                            double omega, double s) {
#pragma clang fp contract(off)
  if (isnan(q.x) || isnan(q.y) || isnan(q.z) || isinf(q.x) || isinf(q.y) || isinf(q.z))
    return;
  const double Lx = pi.L[0], Ly = pi.L[1], Lz = pi.L[2];
  const double lo0 = pi.x0[0], lo1 = pi.x0[1], lo2 = pi.x0[2];
  const double hi0 = lo0 + Lx, hi1 = lo1 + Ly, hi2 = lo2 + Lz;
  const double jump = 1.5 * omega * Lx;
  if (boundary == RB_SHEAR) {
    if (q.x >= hi0) { q.x = q.x - Lx; q.y = q.y + s; q.vy = q.vy + jump; }
    else if (q.x < lo0) { q.x = q.x + Lx; q.y = q.y - s; q.vy = q.vy - jump; }
  } else if (boundary == RB_PERIODIC) {
    if (q.x >= hi0) q.x = q.x - Lx;
    else if (q.x < lo0) q.x = q.x + Lx;
  }
  if (boundary != RB_OPEN) {
    if (q.y >= hi1) q.y = q.y - Ly;
    else if (q.y < lo1) q.y = q.y + Ly;
  }
  bool out = !(q.z >= lo2 && q.z < hi2);
  if (boundary == RB_OPEN) out = out || !(q.x >= lo0 && q.x < hi0) || !(q.y >= lo1 && q.y < hi1);
  if (out) {
    q.x = q.y = q.z = __builtin_nan("");
    q.vx = q.vy = q.vz = 0.0;
  }
}

__device__ __forceinline__ uint64_t rb_state_key(const PState &q, const PatchInfo &pi,
                                                 int boundary, uint32_t *err) {
  uint32_t qx, qy, qz;
  const bool okx = rb_quantise(q.x, pi.x0[0], pi.L[0], pi.S, pi.qtop[0], qx);
  const bool oky = rb_quantise(q.y, pi.x0[1], pi.L[1], pi.S, pi.qtop[1], qy);
  const bool okz = rb_quantise(q.z, pi.x0[2], pi.L[2], pi.S, pi.qtop[2], qz);
  if (okx && oky && okz) return rb_key(qx, qy, qz);
  if (boundary != RB_OPEN && !isnan(q.x) && (!okx || !oky)) atomicOr(err, RB_ERR_OUTSIDE);
  return RB_KEY_DEAD;
}

// caller arrays -> buffer 0 (caller order), first drift, boundary, keys
__global__ __launch_bounds__(256) void k_prologue(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    const double *__restrict__ vx, const double *__restrict__ vy,
    const double *__restrict__ vz, const double *__restrict__ m,
    const PatchInfo *__restrict__ patch, const uint32_t *__restrict__ starts, uint32_t P,
    uint32_t n, int boundary, int drift, const StepConst *__restrict__ scp,
    const double *__restrict__ sched, const uint32_t *__restrict__ ctr,
    double *__restrict__ bx, double *__restrict__ by, double *__restrict__ bz,
    double *__restrict__ bvx, double *__restrict__ bvy, double *__restrict__ bvz,
    double *__restrict__ bm, uint32_t *__restrict__ orig, uint64_t *__restrict__ key,
    uint32_t *__restrict__ idx, uint32_t *__restrict__ err, uint32_t *__restrict__ bcnt,
    uint32_t *__restrict__ bctl) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint32_t p = (P == 1) ? 0 : rb_patch_of(starts, P, s);
  const PatchInfo pi = patch[p];
  const StepConst sc = *scp;
  PState q{x[s], y[s], z[s], vx[s], vy[s], vz[s]};
  const bool alive = !(isnan(q.x) || isnan(q.y) || isnan(q.z));
  if (alive) {
    rb_apply_drift(q, drift, sc);
    rb_apply_boundary(q, boundary, pi, sc.omega, sched[(size_t)ctr[0] * 2 * P + p]);
  }
  bx[s] = q.x; by[s] = q.y; bz[s] = q.z;
  bvx[s] = q.vx; bvy[s] = q.vy; bvz[s] = q.vz;
  bm[s] = m[s];
  orig[s] = s;
  const uint64_t k = rb_state_key(q, pi, boundary, err);
  key[s] = k;
  idx[s] = s;
  if (bcnt) {
    if (s == 0) bctl[0] = 0;  // segments of the bucket sort, counted anew
    rb_bucket_add(bcnt, p, P, k);
  }
}

hipError_t launch_prologue(rb_ctx *c, const rb_particles *cp) {
  const uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  double *const *b = c->d_px[0];
  hipLaunchKernelGGL(k_prologue, dim3(rb_div_up(n, 256)), dim3(256), 0, c->stream, cp->x,
                     cp->y, cp->z, cp->vx, cp->vy, cp->vz, cp->m, c->d_patch, c->d_starts,
                     c->P, n, c->p.boundary, c->p.drift, c->d_sc, c->d_sched, c->d_ctr, b[0],
                     b[1], b[2], b[3], b[4], b[5], b[6], c->d_orig[0], c->d_key[0],
                     c->d_idx[0], c->d_err,
                     c->sort_small ? c->d_bcnt : nullptr, c->d_bctl);
  return hipGetLastError();
}

// Kick with the walk's accelerations (images and parts summed in order), second drift
// and boundary; then, unless this is the last step, the next step's first
// drift, boundary and keys.  Works in place on the sorted buffer.  With
// collisions at the end of the step the work is split around them: mode 1
// stops after the second drift and records, per slot, the periodic wrap it
// applied (the image (wx, wy) the unwrapped position lies in) and the
// largest displacement since the tree was built; mode 2 then does the next
// step's first drift and keys.  Mode 0 does both at once.
template <int mode>
__global__ __launch_bounds__(256) void k_post(
    double *__restrict__ bx, double *__restrict__ by, double *__restrict__ bz,
    double *__restrict__ bvx, double *__restrict__ bvy, double *__restrict__ bvz,
    const double *__restrict__ acc, uint64_t cap, int n_acc,
    const PatchInfo *__restrict__ patch, const uint32_t *__restrict__ starts,
    const uint32_t *__restrict__ nlive, uint32_t P, uint32_t n, int boundary, int drift,
    const StepConst *__restrict__ scp, const double *__restrict__ sched,
    uint32_t *__restrict__ ctr, int slot, uint64_t *__restrict__ key,
    uint32_t *__restrict__ idx, uint32_t *__restrict__ err, uint32_t *__restrict__ bcnt,
    uint32_t *__restrict__ bctl, uint16_t *__restrict__ wrap,
    unsigned long long *__restrict__ disp, const uint32_t *__restrict__ orig,
    const double *__restrict__ radius, uint32_t *__restrict__ inv,
    unsigned long long *__restrict__ rmax) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t k = ctr[slot], nsteps = ctr[2];
  // the next step reads its index from the other slot; its keep-the-tree
  // flag (ctr[6 + slot]) starts clear, raised by its check on any change
  if (s == 0 && mode != 2) ctr[1 - slot] = k + 1;
  if (s == 0 && mode != 1) ctr[6 + (1 - slot)] = 0u;
  double moved = 0.0, rad = 0.0;
  if (s < n) {
  const uint32_t p = (P == 1) ? 0 : rb_patch_of(starts, P, s);
  const PatchInfo pi = patch[p];
  const StepConst sc = *scp;
  const bool has_next = k + 1 < nsteps && mode != 1;
  PState q{bx[s], by[s], bz[s], bvx[s], bvy[s], bvz[s]};
  const bool live = (s - pi.start) < nlive[p];
  if (mode == 1) {  // for the search and the rounds: caller index -> slot, R_max
    const uint32_t o = orig[s];
    inv[o] = s;
    if (live) {
      const double v = radius[o];
      rad = v > 0.0 ? v : 0.0;  // (a NaN radius is never larger)
    }
  }
  if (live) {
    if (mode != 2) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0;
      for (int im = 0; im < n_acc; ++im) {
        const double *a = acc + (size_t)im * 3 * cap;
        a0 += a[s]; a1 += a[cap + s]; a2 += a[2 * cap + s];
      }
      {
#pragma clang fp contract(off)
        q.vx = q.vx + a0 * sc.dt;
        q.vy = q.vy + a1 * sc.dt;
        q.vz = q.vz + a2 * sc.dt;
      }
      const double mx = q.x, my = q.y, mz = q.z;  // where the tree put the particle
      rb_apply_drift(q, drift, sc);
      const double ux = q.x, uy = q.y, uz = q.z;  // before any wrap
      const double s_end = sched[(size_t)k * 2 * P + P + p];
      rb_apply_boundary(q, boundary, pi, sc.omega, s_end);
      if (mode == 1) {
        uint16_t wv = (2u << 4) | 2u;  // (wx + 2) | (wy + 2) << 4; 0, 0 when nothing moved
        if (!(isnan(q.x) || isnan(q.y) || isnan(q.z))) {
          const double dx = ux - mx, dy = uy - my, dz = uz - mz;
          moved = sqrt(dx * dx + dy * dy + dz * dz);
          if (boundary != RB_OPEN) {
            const double fx = rint((ux - q.x) / pi.L[0]);
            const double sx = (boundary == RB_SHEAR) ? fx * s_end : 0.0;
            const double fy = rint(((uy - q.y) + sx) / pi.L[1]);
            wv = (uint16_t)(((int)fx + 2) | (((int)fy + 2) << 4));
          }
        }
        wrap[s] = wv;
      }
    }
    if (has_next) {
      const bool alive = !(isnan(q.x) || isnan(q.y) || isnan(q.z));
      if (alive) {
        rb_apply_drift(q, drift, sc);
        rb_apply_boundary(q, boundary, pi, sc.omega, sched[(size_t)(k + 1) * 2 * P + p]);
      }
    }
    bx[s] = q.x; by[s] = q.y; bz[s] = q.z;
    bvx[s] = q.vx; bvy[s] = q.vy; bvz[s] = q.vz;
  } else if (mode == 1) {
    wrap[s] = (2u << 4) | 2u;
  }
  if (has_next) {
    const uint64_t k2 = live ? rb_state_key(q, pi, boundary, err) : RB_KEY_DEAD;
    key[s] = k2;
    idx[s] = s;
    if (bcnt) {
      if (s == 0) bctl[0] = 0;
      rb_bucket_add(bcnt, p, P, k2);
    }
  }
  }
  if (mode == 1) {
    // the largest displacement and radius (ordered bits of non-negative
    // doubles), one atomic each per workgroup: both words share a cache line
    __shared__ double part[2][4];
    for (int d = 32; d >= 1; d >>= 1) {
      moved = fmax(moved, __shfl_xor(moved, d, 64));
      rad = fmax(rad, __shfl_xor(rad, d, 64));
    }
    if (rb_lane() == 0) {
      part[0][threadIdx.x >> 6] = moved;
      part[1][threadIdx.x >> 6] = rad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      moved = fmax(fmax(part[0][0], part[0][1]), fmax(part[0][2], part[0][3]));
      rad = fmax(fmax(part[1][0], part[1][1]), fmax(part[1][2], part[1][3]));
      if (moved > 0.0) atomicMax(disp, (unsigned long long)__double_as_longlong(moved));
      if (rad > 0.0) atomicMax(rmax, (unsigned long long)__double_as_longlong(rad));
    }
  }
}

hipError_t launch_post(rb_ctx *c, int buf, int slot, int mode) {
  const uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  double *const *b = c->d_px[buf];
  const int n_acc = rb_n_acc(c);
#define RB_POST_ARGS                                                                      \
  b[0], b[1], b[2], b[3], b[4], b[5], c->d_acc, c->cap, n_acc, c->d_patch, c->d_starts,    \
      c->d_nlive, c->P, n, c->p.boundary, c->p.drift, c->d_sc, c->d_sched, c->d_ctr, slot, \
      c->d_key[0], c->d_idx[0], c->d_err, c->sort_small ? c->d_bcnt : nullptr, c->d_bctl,  \
      c->d_cwrap,                                                                          \
      c->d_ccnt ? reinterpret_cast<unsigned long long *>(c->d_ccnt + 8) : nullptr,         \
      c->d_orig[buf], c->coll_R, c->d_cinv, c->d_cmax
  const dim3 g(rb_div_up(n, 256)), bl(256);
  if (mode == 1) hipLaunchKernelGGL(k_post<1>, g, bl, 0, c->stream, RB_POST_ARGS);
  else if (mode == 2) hipLaunchKernelGGL(k_post<2>, g, bl, 0, c->stream, RB_POST_ARGS);
  else hipLaunchKernelGGL(k_post<0>, g, bl, 0, c->stream, RB_POST_ARGS);
#undef RB_POST_ARGS
  return hipGetLastError();
}

// sorted buffer -> caller arrays
__global__ __launch_bounds__(256) void k_epilogue(
    const double *__restrict__ bx, const double *__restrict__ by,
    const double *__restrict__ bz, const double *__restrict__ bvx,
    const double *__restrict__ bvy, const double *__restrict__ bvz,
    const uint32_t *__restrict__ orig, uint32_t n, double *__restrict__ x,
    double *__restrict__ y, double *__restrict__ z, double *__restrict__ vx,
    double *__restrict__ vy, double *__restrict__ vz) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint32_t o = orig[s];
  x[o] = bx[s]; y[o] = by[s]; z[o] = bz[s];
  vx[o] = bvx[s]; vy[o] = bvy[s]; vz[o] = bvz[s];
}

hipError_t launch_epilogue(rb_ctx *c, rb_particles *cp, int buf) {
  const uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  double *const *b = c->d_px[buf];
  hipLaunchKernelGGL(k_epilogue, dim3(rb_div_up(n, 256)), dim3(256), 0, c->stream, b[0],
                     b[1], b[2], b[3], b[4], b[5], c->d_orig[buf], n, cp->x, cp->y, cp->z,
                     cp->vx, cp->vy, cp->vz);
  return hipGetLastError();
}

// accelerations (images and parts summed in order) -> caller order; slots outside the
// tree (removed particles) get zero
__global__ __launch_bounds__(256) void k_scatter_acc(
    const double *__restrict__ acc, uint64_t cap, int n_acc, const uint32_t *__restrict__ orig,
    const PatchInfo *__restrict__ patch, const uint32_t *__restrict__ starts,
    const uint32_t *__restrict__ nlive, uint32_t P, uint32_t n, double *__restrict__ ax,
    double *__restrict__ ay, double *__restrict__ az) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint32_t p = (P == 1) ? 0 : rb_patch_of(starts, P, s);
  const bool live = (s - patch[p].start) < nlive[p];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (live) {
    for (int im = 0; im < n_acc; ++im) {
      const double *a = acc + (size_t)im * 3 * cap;
      a0 += a[s]; a1 += a[cap + s]; a2 += a[2 * cap + s];
    }
  }
  const uint32_t o = orig[s];
  ax[o] = a0; ay[o] = a1; az[o] = a2;
}

hipError_t launch_scatter_acc(rb_ctx *c, double *ax, double *ay, double *az) {
  const uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  const int n_acc = rb_n_acc(c);
  hipLaunchKernelGGL(k_scatter_acc, dim3(rb_div_up(n, 256)), dim3(256), 0, c->stream,
                     c->d_acc, c->cap, n_acc, c->d_orig[0], c->d_patch, c->d_starts,
                     c->d_nlive, c->P, n, ax, ay, az);
  return hipGetLastError();
}
