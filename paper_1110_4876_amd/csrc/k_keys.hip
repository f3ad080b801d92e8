// k_keys.hip -- Morton keys of the caller's particles and the gathers into
// Morton order after the sort (octree construction, Sect. 4.2 of the paper).
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
                                              uint32_t *__restrict__ err,
                                              uint32_t *__restrict__ bcnt,
                                              uint32_t *__restrict__ bctl) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  uint32_t p = (P == 1) ? 0 : rb_patch_of(starts, P, s);
  const PatchInfo pi = patch[p];
  double xs = x[s], ys = y[s], zs = z[s];
  uint32_t qx, qy, qz;
  bool okx = rb_quantise(xs, pi.x0[0], pi.L[0], pi.S, pi.qtop[0], qx);
  bool oky = rb_quantise(ys, pi.x0[1], pi.L[1], pi.S, pi.qtop[1], qy);
  bool okz = rb_quantise(zs, pi.x0[2], pi.L[2], pi.S, pi.qtop[2], qz);
  uint64_t k = RB_KEY_DEAD;
  if (okx && oky && okz) {
    k = rb_key(qx, qy, qz);
  } else if (!open_xy && !(isnan(xs) || isnan(ys) || isnan(zs)) && (!okx || !oky)) {
    atomicOr(err, RB_ERR_OUTSIDE);  // a periodic axis must have been wrapped
  }
  key[s] = k;
  idx[s] = s;
  if (bcnt) {
    if (s == 0) bctl[0] = 0;  // segments of the bucket sort, counted anew
    rb_bucket_add(bcnt, p, P, k);
  }
}

hipError_t launch_keys(rb_ctx *c, const double *x, const double *y, const double *z,
                       double) {
  uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_keys, dim3(rb_div_up(n, 256)), dim3(256), 0, c->stream, x, y, z,
                     c->d_patch, c->d_starts, c->P, n, c->p.boundary == RB_OPEN ? 1 : 0,
                     c->d_key[0], c->d_idx[0], c->d_err, c->sort_small ? c->d_bcnt : nullptr,
                     c->d_bctl);
  return hipGetLastError();
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

