// k_direct.hip -- Eq. (1) by direct summation (Sect. 4.1 of the paper) for a
// list of target particles, over all sources and ghost images, FP64.
//
// Grid: (target groups of 64) x (source chunks).  A wave stages 64 sources
// at a time in LDS; every lane reads the same entry (broadcast) and adds its
// term.  Per-chunk partial sums are reduced in chunk order afterwards, so
// the result does not depend on scheduling.
//
// Two entry points share these kernels: rb_direct keeps the partial sums in
// its context's accumulator buffer; rb_direct_noalloc, for callers that
// cannot allocate, keeps them in the fixed array below.
#include <mutex>

#include "rb_internal.h"

// Partial sums of rb_direct_noalloc: one array per GPU, held until the
// process ends.  Every call on a GPU uses the same array, so calls that
// overlap on one GPU race.  Host code reaches it only through the address
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[RB_DIRECT_SCRATCH_DOUBLES];

__device__ __forceinline__ double rb_rsqrt64_d(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * (1.5 - h * y * y);
  y = y * (1.5 - h * y * y);
  return y;
}

__global__ __launch_bounds__(64) void k_direct(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    const double *__restrict__ m, uint32_t n, uint32_t n_active,
    const int64_t *__restrict__ targets, uint32_t nt, uint32_t chunk, int n_img, int ngx,
    int ngy, int boundary, double Lx, double Ly, double s, double G, double b2,
    double *__restrict__ part, uint32_t *__restrict__ err) {
  __shared__ double4 src[64];
  const uint32_t t = blockIdx.x * 64 + threadIdx.x;
  const uint32_t c = blockIdx.y;
  const bool valid = t < nt;
  const int64_t ti = valid ? targets[t] : 0;
  const bool in_range = ti >= 0 && ti < (int64_t)n;
  if (valid && !in_range && c == 0 && err) atomicOr(err, RB_ERR_INDEX);
  const uint32_t i = in_range ? (uint32_t)ti : 0u;
  double px = 0.0, py = 0.0, pz = 0.0;
  bool alive = false;
  if (valid && in_range) {
    px = x[i]; py = y[i]; pz = z[i];
    alive = !(isnan(px) || isnan(py) || isnan(pz));
  }
  const uint32_t nsrc = n_active < n ? n_active : n;
  const uint32_t j0 = c * chunk, j1 = (j0 + chunk < nsrc) ? j0 + chunk : nsrc;
  double ax = 0.0, ay = 0.0, az = 0.0;
  for (uint32_t base = j0; base < j1; base += 64) {
    const uint32_t j = base + threadIdx.x;
    double4 e = make_double4(0.0, 0.0, 0.0, 0.0);
    if (j < j1) {
      e = make_double4(x[j], y[j], z[j], m[j]);
      if (isnan(e.x) || isnan(e.y) || isnan(e.z)) e = make_double4(0.0, 0.0, 0.0, 0.0);
    }
    __syncthreads();
    src[threadIdx.x] = e;
    __syncthreads();
    const uint32_t cnt = (j1 - base < 64) ? j1 - base : 64;
    if (alive) {
      for (int im = 0; im < n_img; ++im) {
        double ox = 0.0, oy = 0.0;
        bool self = true;
        if (boundary != RB_OPEN) {
          const int ny = 2 * ngy + 1;
          const int ix = im / ny - ngx, iy = im % ny - ngy;
          const double fx = (double)ix, fy = (double)iy;
          const double sh = (boundary == RB_SHEAR) ? s : 0.0;
          ox = fx * Lx;
          oy = fy * Ly - fx * sh;
          self = (ix == 0 && iy == 0);
        }
        const double y0 = px - ox, y1 = py - oy, y2 = pz;
        for (uint32_t k = 0; k < cnt; ++k) {
          const double4 q = src[k];
          if (q.w == 0.0 || (self && base + k == i)) continue;
          const double d0 = q.x - y0, d1 = q.y - y1, d2 = q.z - y2;
          const double r2 = d0 * d0 + d1 * d1 + d2 * d2 + b2;
          const double ri = rb_rsqrt64_d(r2);
          const double f = G * q.w * (ri * ri * ri);
          ax += f * d0; ay += f * d1; az += f * d2;
        }
      }
    }
  }
  if (valid) {
    double *o = part + (size_t)c * 3 * nt;
    o[t] = ax; o[nt + t] = ay; o[2 * nt + t] = az;
  }
}

__global__ __launch_bounds__(256) void k_direct_reduce(const double *__restrict__ part,
                                                       uint32_t nt, uint32_t n_chunks,
                                                       double *__restrict__ ax,
                                                       double *__restrict__ ay,
                                                       double *__restrict__ az) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (uint32_t c = 0; c < n_chunks; ++c) {
    const double *o = part + (size_t)c * 3 * nt;
    a0 += o[t]; a1 += o[nt + t]; a2 += o[2 * nt + t];
  }
  ax[t] = a0; ay[t] = a1; az[t] = a2;
}

// Chunking of the sources: enough (target group, chunk) blocks to fill the
// chip, chunks of at least 1024 sources (a multiple of 64), at most
// max_part partial doubles (3 per target and chunk).
static void direct_chunks(uint32_t nsrc, uint32_t nt, uint64_t max_part, uint32_t &n_chunks,
                          uint32_t &chunk) {
  const uint32_t groups = rb_div_up(nt, 64);
  n_chunks = (8192 + groups - 1) / groups;
  const uint32_t max_by_src = rb_div_up(nsrc > 0 ? nsrc : 1, 1024);
  if (n_chunks > max_by_src) n_chunks = max_by_src;
  if ((uint64_t)n_chunks * 3 * nt > max_part) n_chunks = (uint32_t)(max_part / (3ull * nt));
  if (n_chunks < 1) n_chunks = 1;
  chunk = ((rb_div_up(nsrc > 0 ? nsrc : 1, n_chunks) + 63) / 64) * 64;
  n_chunks = rb_div_up(nsrc > 0 ? nsrc : 1, chunk);
}

static void direct_kernels(const rb_particles *cp, uint32_t n, uint32_t n_active,
                           const int64_t *targets, uint32_t nt, int n_img, int ngx, int ngy,
                           int boundary, double Lx, double Ly, double s, double G, double b2,
                           double *part, uint64_t max_part, uint32_t *err, double *ax,
                           double *ay, double *az, hipStream_t stream) {
  const uint32_t nsrc = n_active < n ? n_active : n;
  uint32_t n_chunks, chunk;
  direct_chunks(nsrc, nt, max_part, n_chunks, chunk);
  hipLaunchKernelGGL(k_direct, dim3(rb_div_up(nt, 64), n_chunks), dim3(64), 0, stream, cp->x,
                     cp->y, cp->z, cp->m, n, n_active, targets, nt, chunk, n_img, ngx, ngy,
                     boundary, Lx, Ly, s, G, b2, part, err);
  hipLaunchKernelGGL(k_direct_reduce, dim3(rb_div_up(nt, 256)), dim3(256), 0, stream, part, nt,
                     n_chunks, ax, ay, az);
}

hipError_t launch_direct(rb_ctx *c, const rb_particles *cp, uint32_t n, uint32_t n_active,
                         double s, const int64_t *targets, uint32_t nt, double *ax,
                         double *ay, double *az) {
  if (nt == 0) return hipSuccess;
  // the partial sums live in the accumulator buffer (all of it, whatever
  // the walk's schedule uses, so the chunking depends on the input alone)
  const uint64_t acc_doubles = (uint64_t)c->acc_sets * 3 * c->cap;
  direct_kernels(cp, n, n_active, targets, nt, c->n_img, c->p.n_ghost[0], c->p.n_ghost[1],
                 c->p.boundary, c->h_patch[0].L[0], c->h_patch[0].L[1], s, c->p.G,
                 c->p.softening * c->p.softening, c->d_acc, acc_doubles, c->d_err, ax, ay, az,
                 c->stream);
  return hipGetLastError();
}

// The device address of the current GPU's scratch array, looked up once per
// device (with that device current) and kept.
static hipError_t direct_scratch(double **out) {
  static std::mutex mu;
  static double *addr[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = (double *)p;
  }
  *out = addr[dev];
  return hipSuccess;
}

hipError_t launch_direct_noalloc(const rb_params *p, const rb_particles *cp, uint32_t n,
                                 uint32_t n_active, double s, const int64_t *targets,
                                 uint32_t nt, int n_img, double Lx, double Ly, double *ax,
                                 double *ay, double *az, hipStream_t stream) {
  if (nt == 0) return hipSuccess;
  double *part = nullptr;
  const hipError_t e = direct_scratch(&part);
  if (e != hipSuccess) return e;
  direct_kernels(cp, n, n_active, targets, nt, n_img, p->n_ghost[0], p->n_ghost[1],
                 p->boundary, Lx, Ly, s, p->G, p->softening * p->softening, part,
                 RB_DIRECT_SCRATCH_DOUBLES, nullptr, ax, ay, az, stream);
  return hipGetLastError();
}
