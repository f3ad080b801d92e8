// k_walk64.hip -- per-particle FP64 tree walk (Sect. 4.2 of the paper).
//
// One wave handles 64 Morton-consecutive particles; every lane walks the tree
// for its own particle with its own opening decisions, so the result is the
// plain per-particle Barnes-Hut sum.  The walk is stackless: nodes are
// visited in depth-first octant order by following `child` when a node is
// opened and `skip` (the next node after its subtree) otherwise.  Opening
// test, image shifts and the centre-of-mass arithmetic round exactly as in a
// plain sequential FP64 walk, so the decisions are reproducible bit for bit.
#include "rb_internal.h"

// 1 / sqrt(x): hardware estimate (relative error ~2^-23) refined by two
// Newton steps y <- y (3 - x y^2) / 2 to FP64 accuracy.
__device__ __forceinline__ double rb_rsqrt64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * (1.5 - h * y * y);
  y = y * (1.5 - h * y * y);
  return y;
}

// image ordinal -> offset (ix W, iy W - ix s, 0), ix outer, iy inner
__device__ __forceinline__ void rb_image(int im, int ngx, int ngy, int boundary, double W,
                                         double s, double &ox, double &oy, bool &self) {
  if (boundary == RB_OPEN) {
    ox = 0.0; oy = 0.0; self = true;
    return;
  }
  const int ny = 2 * ngy + 1;
  const int ix = im / ny - ngx, iy = im % ny - ngy;
  const double fx = (double)ix, fy = (double)iy;
  const double sh = (boundary == RB_SHEAR) ? s : 0.0;
  ox = fx * W;
  oy = fy * W - fx * sh;
  self = (ix == 0 && iy == 0);
}

template <bool QUAD, bool STATS>
__global__ __launch_bounds__(64) void k_walk64(
    const WalkItem *__restrict__ items, int img_split, int n_img, int ngx, int ngy,
    int boundary, const PatchInfo *__restrict__ patch, const uint32_t *__restrict__ nlive,
    const uint32_t *__restrict__ root, const NodeLink *__restrict__ link,
    const double4 *__restrict__ mcom, const double *__restrict__ Qarr,
    const double *__restrict__ sx, const double *__restrict__ sy,
    const double *__restrict__ sz, const double *__restrict__ msrc,
    const double *__restrict__ sched, const uint32_t *__restrict__ ctr, uint32_t P,
    double G, double b2, double theta2, double *__restrict__ acc, uint64_t cap,
    unsigned long long *__restrict__ stats, const uint32_t *__restrict__ lev_off,
    uint32_t *__restrict__ err, int slot) {
  // a depth-first walk visits every node at most once per image: more
  // visits, or an index past the node count, mean inconsistent links
  const uint32_t n_nodes = lev_off[RB_NLEV];
  const uint32_t item = img_split ? blockIdx.x / n_img : blockIdx.x;
  const int im0 = img_split ? (int)(blockIdx.x % n_img) : 0;
  const int im1 = img_split ? im0 + 1 : n_img;
  const WalkItem it = items[item];
  const uint32_t p = it.patch;
  const double W = patch[p].W;
  const uint32_t st = patch[p].start, nl = nlive[p];
  const uint32_t s = it.start + threadIdx.x;
  const bool valid = s < it.end && (s - st) < nl;
  const double shear = sched[(size_t)ctr[slot] * 2 * P + p];
  double px = 0.0, py = 0.0, pz = 0.0;
  if (valid) { px = sx[s]; py = sy[s]; pz = sz[s]; }
  const uint32_t r0 = valid ? root[p] : RB_NONE;
  uint32_t n_open = 0, n_cell = 0, n_pp = 0;
  double tx = 0.0, ty = 0.0, tz = 0.0;
  for (int im = im0; im < im1; ++im) {
    double ox, oy;
    bool self;
    rb_image(im, ngx, ngy, boundary, W, shear, ox, oy, self);
    const double y0 = px - ox, y1 = py - oy, y2 = pz;
    double ax = 0.0, ay = 0.0, az = 0.0;
    uint32_t cur = r0, visits = 0;
    while (cur != RB_NONE) {
      if (cur >= n_nodes || ++visits > n_nodes) {
        atomicOr(err, RB_ERR_TREE);
        break;
      }
      const NodeLink lk = link[cur];
      const double4 mc = mcom[cur];
      uint32_t next = lk.skip;
      if (mc.w != 0.0) {
        const bool leaf = (lk.lvl & 256u) != 0;
        if (leaf && lk.count == 1) {
          if (!(self && lk.child_or_first == s)) {
            const double d0 = mc.x - y0, d1 = mc.y - y1, d2 = mc.z - y2;
            const double r2 = d0 * d0 + d1 * d1 + d2 * d2 + b2;
            const double ri = rb_rsqrt64(r2);
            const double f = G * mc.w * (ri * ri * ri);
            ax += f * d0; ay += f * d1; az += f * d2;
            if (STATS) ++n_pp;
          }
        } else {
          const double d0 = mc.x - y0, d1 = mc.y - y1, d2 = mc.z - y2;
          const double R2 = __builtin_fma(d2, d2, __builtin_fma(d1, d1, d0 * d0));
          const double w = ldexp(W, -(int)(lk.lvl & 255u));
          if (STATS) ++n_open;
          if (w * w < theta2 * R2) {
            const double ri = rb_rsqrt64(R2 + b2);
            const double ri2 = ri * ri;
            const double ri3 = ri * ri2;
            const double f = G * mc.w * ri3;
            ax += f * d0; ay += f * d1; az += f * d2;
            if (QUAD) {
              const double *q = Qarr + 6 * (size_t)cur;
              const double q00 = q[0], q01 = q[1], q02 = q[2], q11 = q[3], q12 = q[4],
                           q22 = q[5];
              const double e0 = q00 * d0 + q01 * d1 + q02 * d2;
              const double e1 = q01 * d0 + q11 * d1 + q12 * d2;
              const double e2 = q02 * d0 + q12 * d1 + q22 * d2;
              const double dqd = d0 * e0 + d1 * e1 + d2 * e2;
              const double ri5 = ri3 * ri2;
              const double g5 = G * ri5;
              const double g7 = 2.5 * G * dqd * (ri5 * ri2);
              ax += g7 * d0 - g5 * e0;
              ay += g7 * d1 - g5 * e1;
              az += g7 * d2 - g5 * e2;
            }
            if (STATS) ++n_cell;
          } else if (leaf) {
            const uint32_t j0 = lk.child_or_first, j1 = j0 + lk.count;
            for (uint32_t j = j0; j < j1; ++j) {
              const double mj = msrc[j];
              if (mj == 0.0 || (self && j == s)) continue;
              const double e0 = sx[j] - y0, e1 = sy[j] - y1, e2 = sz[j] - y2;
              const double r2 = e0 * e0 + e1 * e1 + e2 * e2 + b2;
              const double ri = rb_rsqrt64(r2);
              const double f = G * mj * (ri * ri * ri);
              ax += f * e0; ay += f * e1; az += f * e2;
              if (STATS) ++n_pp;
            }
          } else {
            next = lk.child_or_first;
          }
        }
      }
      cur = next;
    }
    if (img_split) {
      if (s < it.end) {
        double *a = acc + (size_t)im * 3 * cap;
        a[s] = ax; a[cap + s] = ay; a[2 * cap + s] = az;
      }
    } else {
      tx += ax; ty += ay; tz += az;
    }
  }
  if (!img_split && s < it.end) {
    acc[s] = tx; acc[cap + s] = ty; acc[2 * cap + s] = tz;
  }
  if (STATS) {
    unsigned long long o = n_open, c = n_cell, q = n_pp;
    for (int d = 32; d >= 1; d >>= 1) {
      o += __shfl_xor(o, d, 64);
      c += __shfl_xor(c, d, 64);
      q += __shfl_xor(q, d, 64);
    }
    if (threadIdx.x == 0) {
      atomicAdd(&stats[0], o);
      atomicAdd(&stats[1], c);
      atomicAdd(&stats[2], q);
    }
  }
}

hipError_t launch_walk64(rb_ctx *c, const double *sx, const double *sy, const double *sz,
                         int slot) {
  const uint32_t n_items = (uint32_t)c->h_items64.size();
  if (n_items == 0) return hipSuccess;
  const int split = c->img_split;
  const unsigned grid = split ? n_items * (unsigned)c->n_img : n_items;
  const double b2 = c->p.softening * c->p.softening;
  const double th2 = c->p.theta * c->p.theta;
  const bool quad = c->p.quadrupole != 0, stats = (c->p.profile & 2) != 0;
#define RB_WALK64_ARGS                                                                   \
  c->d_items64, split, c->n_img, c->p.n_ghost[0], c->p.n_ghost[1], c->p.boundary,        \
      c->d_patch, c->d_nlive, c->d_root, c->d_link, c->d_mcom, c->d_Q, sx, sy, sz,       \
      c->d_msrc, c->d_sched, c->d_ctr, c->P, c->p.G, b2, th2, c->d_acc, c->cap, c->d_stats, \
      c->d_lev_off, c->d_err, slot
  if (quad && stats)
    hipLaunchKernelGGL((k_walk64<true, true>), dim3(grid), dim3(64), 0, c->stream, RB_WALK64_ARGS);
  else if (quad)
    hipLaunchKernelGGL((k_walk64<true, false>), dim3(grid), dim3(64), 0, c->stream, RB_WALK64_ARGS);
  else if (stats)
    hipLaunchKernelGGL((k_walk64<false, true>), dim3(grid), dim3(64), 0, c->stream, RB_WALK64_ARGS);
  else
    hipLaunchKernelGGL((k_walk64<false, false>), dim3(grid), dim3(64), 0, c->stream, RB_WALK64_ARGS);
#undef RB_WALK64_ARGS
  return hipGetLastError();
}
