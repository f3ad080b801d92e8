// k_sweep.hip -- collision detection by a plane sweep along x (Sect. 5 of
// the paper), for one system.
//
// Every particle's trajectory over the past time-step dt is taken as the
// straight line through its present position with its present velocity,
// x(sigma) = x + v sigma for sigma in [-dt, 0].  Particle i and image k of
// particle j collide when those lines (the image moving with v_j + w_k, w_k
// its shear velocity) come closer than R_i + R_j; the collisions then join
// the same random-order queue and hard-sphere resolution as the tree search.
//
// The sweep: each trajectory's extent along x, widened by the radius, is an
// interval [lo, hi].  Sorting the intervals by lo and stepping through them
// in that order is the plane moving along x: the particles whose intervals
// contain the plane's position are the active list of the paper, and a
// particle entering it is checked against those already there.  Here every
// interval in sorted order checks the ones after it that start before it
// ends (on the GPU, one thread per interval: the active list is implicit),
// so each pair of overlapping intervals is visited once.  With periodic or
// shear boundaries, the copies of the box shifted by ix W (ix = +-1 .. +-ng)
// are visited too: interval i looks up, in the same sorted list, the
// intervals that overlap its own once shifted by ix W (they start after
// lo_i - ix W - L, L the longest interval, and before hi_i - ix W) and keeps
// the pairs with i the lower caller index, so each pair and image is found
// once.  Ghost images along y are tested for every candidate pair.
//
// Sort keys are lo quantised on a 63-bit grid (monotone, clamped), so the
// context's Morton-key sort orders them; a scan ends at the first interval
// whose key exceeds the quantised end of its range, which visits every
// interval that starts in the range.  The intervals carry a relative
// widening of 1e-9 so that rounding never separates a pair that the exact
// test below finds in contact.
//
// Compiled without FP contraction: the contact test rounds exactly as the
// plain evaluation of the same expressions.
#include "rb_internal.h"

struct SweepGrid {
  double base, scale;  // key = clamp(floor((lo - base) * scale), 0, RB_SW_KMAX)
};
#define RB_SW_KMAX 0x7FFFFFFFFFFFF000ull

__device__ __forceinline__ uint64_t rb_sw_key(double v, SweepGrid g) {
  const double f = floor((v - g.base) * g.scale);
  if (!(f > 0.0)) return 0ull;  // (below the grid)
  if (f >= (double)RB_SW_KMAX) return RB_SW_KMAX;
  return (uint64_t)f;
}

// the trajectory's extent along x, widened by the radius and the margin
__device__ __forceinline__ void rb_sw_extent(double x, double vx, double R, double dt, double W,
                                             double &lo, double &hi) {
  // position at the start of the step (a velocity that is not a number
  // leaves only the present position, where the contact test can still hold)
  const double mv = vx * dt;
  const bool moves = !isnan(mv);
  const double xs = moves ? x - mv : x;
  const double r = fabs(R);
  const double pad = 1e-9 * (W + r + (moves ? fabs(mv) : 0.0));
  lo = fmin(x, xs) - r - pad;
  hi = fmax(x, xs) + r + pad;
}

// The azimuthal sweep (global simulations, open box): the trajectory's
// extent in phi = atan2(y, x) around the z axis, widened by the angle the
// radius subtends at the segment's closest approach to the axis (a sphere
// of radius R whose centre is at least rho from the axis lies within
// asin(R / rho) of its centre's angle); a segment that passes within R of
// the axis covers every angle.  lo is brought into [-pi, pi); hi = lo + len.
#define RB_PI 3.141592653589793
__device__ __forceinline__ void rb_sw_phi_extent(double x, double y, double vx, double vy,
                                                 double R, double dt, double &lo,
                                                 double &hi) {
  double mx = vx * dt, my = vy * dt;
  if (isnan(mx) || isnan(my)) mx = my = 0.0;  // only the present position counts
  const double x0 = x - mx, y0 = y - my;    // start of the step
  const double p1 = atan2(y, x), p0 = atan2(y0, x0);
  double dp = p1 - p0;
  if (dp > RB_PI) dp -= 2.0 * RB_PI;
  if (dp < -RB_PI) dp += 2.0 * RB_PI;
  // closest approach of the segment to the axis
  const double dd = mx * mx + my * my;
  double u = dd > 0.0 ? -(x0 * mx + y0 * my) / dd : 0.0;
  u = fmin(fmax(u, 0.0), 1.0);
  const double qx = x0 + u * mx, qy = y0 + u * my;
  const double rho = sqrt(qx * qx + qy * qy);
  const double r = fabs(R);
  double a = -RB_PI, len = 2.0 * RB_PI;
  if (rho > r * (1.0 + 1e-6) + 1e-300) {
    const double half = asin(r / rho) * (1.0 + 1e-9) + 1e-12;
    const double l = fabs(dp) + 2.0 * half + 1e-9 * (1.0 + fabs(dp));
    if (l < 2.0 * RB_PI) {
      len = l;
      a = fmin(p0, p0 + dp) - half - 0.5e-9 * (1.0 + fabs(dp));
      if (a < -RB_PI) a += 2.0 * RB_PI;
      if (a >= RB_PI) a -= 2.0 * RB_PI;
    }
  }
  lo = a;
  hi = a + len;
}

// keys of the caller's particles (live: inside the box, radius a number)
__global__ __launch_bounds__(256) void k_sw_keys(
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    const double *__restrict__ vx, const double *__restrict__ vy,
    const double *__restrict__ R, const PatchInfo *__restrict__ patch, uint32_t n,
    int open_xy, int phi, double dt, SweepGrid g, uint64_t *__restrict__ key,
    uint32_t *__restrict__ idx, uint32_t *__restrict__ err, uint32_t *__restrict__ bcnt,
    uint32_t *__restrict__ bctl, unsigned long long *__restrict__ lmax) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  double len = 0.0;
  if (s < n) {
    const PatchInfo pi = patch[0];
    const double xs = x[s], ys = y[s], zs = z[s];
    uint32_t q;
    const bool okx = rb_quantise(xs, pi.x0[0], pi.L[0], pi.S, pi.qtop[0], q);
    const bool oky = rb_quantise(ys, pi.x0[1], pi.L[1], pi.S, pi.qtop[1], q);
    const bool okz = rb_quantise(zs, pi.x0[2], pi.L[2], pi.S, pi.qtop[2], q);
    uint64_t k = RB_KEY_DEAD;
    if (okx && oky && okz) {
      const double r = R[s];
      if (!isnan(r)) {
        double lo, hi;
        if (phi)
          rb_sw_phi_extent(xs, ys, vx[s], vy[s], r, dt, lo, hi);
        else
          rb_sw_extent(xs, vx[s], r, dt, pi.W, lo, hi);
        k = (isnan(lo) || isnan(hi)) ? RB_KEY_DEAD : rb_sw_key(lo, g);
        if (k != RB_KEY_DEAD) len = hi - lo;
      }
    } else if (!open_xy && !(isnan(xs) || isnan(ys) || isnan(zs)) && (!okx || !oky)) {
      atomicOr(err, RB_ERR_OUTSIDE);  // a periodic axis must have been wrapped
    }
    key[s] = k;
    idx[s] = s;
    if (bcnt) {
      if (s == 0) bctl[0] = 0;  // segments of the bucket sort, counted anew
      rb_bucket_add(bcnt, 0, 1, k);
    }
  }
  // the longest interval (ordered bits of a non-negative double), one
  // atomic per workgroup: same-address atomics serialise
  __shared__ double part[4];
  for (int d = 32; d >= 1; d >>= 1) len = fmax(len, __shfl_xor(len, d, 64));
  if (rb_lane() == 0) part[threadIdx.x >> 6] = len;
  __syncthreads();
  if (threadIdx.x == 0) {
    len = fmax(fmax(part[0], part[1]), fmax(part[2], part[3]));
    if (len > 0.0) atomicMax(lmax, (unsigned long long)__double_as_longlong(len));
  }
}

// the particles in sorted order, each interval's end, the live count
__global__ __launch_bounds__(256) void k_sw_gather(
    const uint64_t *__restrict__ key, const uint32_t *__restrict__ idx,
    const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
    const double *__restrict__ vx, const double *__restrict__ vy,
    const double *__restrict__ vz, const double *__restrict__ R,
    const PatchInfo *__restrict__ patch, uint32_t n, int phi, double dt,
    double *__restrict__ sx,
    double *__restrict__ sy, double *__restrict__ sz, double *__restrict__ svx,
    double *__restrict__ svy, double *__restrict__ svz, double *__restrict__ sR,
    double *__restrict__ shi, uint32_t *__restrict__ orig, uint32_t *__restrict__ nlive) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint64_t k = key[s];
  const bool live = k != RB_KEY_DEAD;
  const uint32_t j = idx[s];
  orig[s] = j;
  if (live) {
    const double xj = x[j], yj = y[j], vxj = vx[j], vyj = vy[j], r = R[j];
    double lo, hi;
    if (phi)
      rb_sw_phi_extent(xj, yj, vxj, vyj, r, dt, lo, hi);
    else
      rb_sw_extent(xj, vxj, r, dt, patch[0].W, lo, hi);
    sx[s] = xj; sy[s] = yj; sz[s] = z[j];
    svx[s] = vxj; svy[s] = vyj; svz[s] = vz[j];
    sR[s] = r;
    shi[s] = hi;
  }
  if (live && (s + 1 == n || key[s + 1] == RB_KEY_DEAD)) nlive[0] = s + 1;
  if (!live && s == 0) nlive[0] = 0;
}

// The contact test along the two straight trajectories (d = x_j + o_k -
// x_i, u = v_j + w_k - v_i): in contact now, or, when now separating, at
// the closest approach within the step (the segment's far end if that
// approach lies further back).
__device__ __forceinline__ bool rb_sw_meets(double d0, double d1, double d2, double u0,
                                            double u1, double u2, double sum, double dt) {
  if (d0 * d0 + d1 * d1 + d2 * d2 < sum * sum) return true;
  const double du = d0 * u0 + d1 * u1 + d2 * u2;
  const double uu = u0 * u0 + u1 * u1 + u2 * u2;
  if (!(du > 0.0 && uu > 0.0)) return false;
  double sg = -du / uu;
  if (sg < -dt) sg = -dt;
  const double e0 = d0 + u0 * sg, e1 = d1 + u1 * sg, e2 = d2 + u2 * sg;
  return e0 * e0 + e1 * e1 + e2 * e2 < sum * sum;
}

// first sorted position whose key is at least v (n if none)
__device__ __forceinline__ uint32_t rb_sw_lower(const uint64_t *__restrict__ key, uint32_t n,
                                                uint64_t v) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (key[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// A particle record as the pair test reads it.
struct SwRec {
  double x, y, z, vx, vy, vz, R;
  uint32_t p;
};

// Test interval e (record E) against interval f (record F), F's copy
// shifted by c W along x; queue the pairs in contact.  The lower caller
// index is i, and ix is j's image relative to i.  Before the exact test an
// image iy is skipped when the pair's y separation over the step stays
// beyond R_i + R_j; that check uses approximate offsets and a margin of
// 1e-9 (R_i + R_j + W + |u_y dt|), far above their rounding.
__device__ __forceinline__ void rb_sw_test(const SwRec &E, const SwRec &F, int c, int ngx,
                                           int ngy, int boundary, double W, double sh,
                                           double omega, double dt,
                                           uint64_t (&mine)[RB_COLL_LOCAL], uint32_t &nm,
                                           uint64_t *__restrict__ queue, uint32_t qcap,
                                           uint32_t *__restrict__ qcnt,
                                           uint32_t *__restrict__ err) {
  const bool e_is_i = E.p < F.p;
  const SwRec &I = e_is_i ? E : F;
  const SwRec &J = e_is_i ? F : E;
  const int ix = e_is_i ? c : -c;
  const double sum = I.R + J.R;
  const bool shear = boundary == RB_SHEAR;
  const double fx = (double)ix;
  const double dy0 = (J.y - I.y) - (shear ? fx * sh : 0.0);
  const double uy = (J.vy - I.vy) + (shear ? -1.5 * omega * W * fx : 0.0);
  const double lim = fabs(sum) + 1e-9 * (fabs(sum) + W + fabs(uy * dt));
  const int ny = (boundary == RB_OPEN) ? 0 : ngy;
  for (int iy = -ny; iy <= ny; ++iy) {
    const double a = dy0 + (double)iy * W;  // y separation now
    const double b = a - uy * dt;           // and at the start of the step
    if (fmin(a, b) > lim || fmax(a, b) < -lim) continue;
    double ox, oy, wy;
    rb_coll_image_xy(ix, iy, boundary, W, sh, omega, ox, oy, wy);
    const double d0 = (J.x + ox) - I.x;
    const double d1 = (J.y + oy) - I.y;
    const double d2 = (J.z + 0.0) - I.z;
    const double u0 = J.vx - I.vx;
    const double u1 = (J.vy + wy) - I.vy;
    const double u2 = J.vz - I.vz;
    if (rb_sw_meets(d0, d1, d2, u0, u1, u2, sum, dt)) {
      const int k = (boundary == RB_OPEN) ? 0 : (ix + ngx) * (2 * ngy + 1) + (iy + ngy);
      rb_coll_keep(((uint64_t)I.p << 35) | ((uint64_t)J.p << 7) | (uint64_t)k, mine, nm,
                   queue, qcap, qcnt, err);
    }
  }
}

#define SW_SUB 16                // lanes per interval
#define SW_EPB (64 / SW_SUB)     // intervals per workgroup (one wave)

// One wave per SW_EPB consecutive sorted live intervals, SW_SUB lanes per
// interval (lane sub takes every SW_SUB-th candidate).  Image ix = 0: the
// intervals after e that start before it ends, read from chunks of 64
// staged in LDS.  Then for every ix != 0 the intervals that overlap e once
// shifted by ix W, read directly (they exist only near the x boundaries),
// kept when e is the lower caller index.
__global__ __launch_bounds__(64) void k_sw_pairs(
    const uint64_t *__restrict__ key, const uint32_t *__restrict__ orig,
    const double *__restrict__ sx, const double *__restrict__ sy,
    const double *__restrict__ sz, const double *__restrict__ svx,
    const double *__restrict__ svy, const double *__restrict__ svz,
    const double *__restrict__ sR, const double *__restrict__ shi,
    const uint32_t *__restrict__ nlive, const PatchInfo *__restrict__ patch, int ngx, int ngy,
    int boundary, double omega, double t, double dt, SweepGrid g,
    const unsigned long long *__restrict__ lmax_bits, uint64_t *__restrict__ queue,
    uint32_t qcap, uint32_t *__restrict__ qcnt, uint32_t *__restrict__ err) {
  __shared__ uint64_t c_key[64];
  __shared__ double c_x[64], c_y[64], c_z[64], c_vx[64], c_vy[64], c_vz[64], c_R[64];
  __shared__ uint32_t c_p[64];
  const uint32_t lane = threadIdx.x;
  const uint32_t sub = lane % SW_SUB;
  const uint32_t r0 = blockIdx.x * SW_EPB;
  const uint32_t r = r0 + lane / SW_SUB;
  const uint32_t n = nlive[0];
  if (r0 >= n) return;  // uniform over the wave
  const bool act = r < n;
  const double W = patch[0].W;
  const double sh = (boundary == RB_SHEAR) ? remainder(1.5 * omega * W * t, W) : 0.0;
  const int ngs = (boundary == RB_OPEN) ? 0 : ngx;
  uint64_t mine[RB_COLL_LOCAL];
  uint32_t nm = 0;
  SwRec E;
  double ehi = 0.0;
  if (act) {
    E.x = sx[r]; E.y = sy[r]; E.z = sz[r];
    E.vx = svx[r]; E.vy = svy[r]; E.vz = svz[r];
    E.R = sR[r]; E.p = orig[r];
    ehi = shi[r];
  }
  // image ix = 0, chunks staged in LDS
  {
    const uint64_t qend = act ? rb_sw_key(ehi, g) : 0ull;
    bool going = act;
    for (uint32_t base = r0 + 1; base < n; base += 64) {
      const uint32_t f = base + lane;
      if (f < n) {
        c_key[lane] = key[f];
        c_x[lane] = sx[f]; c_y[lane] = sy[f]; c_z[lane] = sz[f];
        c_vx[lane] = svx[f]; c_vy[lane] = svy[f]; c_vz[lane] = svz[f];
        c_R[lane] = sR[f];
        c_p[lane] = orig[f];
      }
      __syncthreads();
      if (going) {
        const uint32_t hi = min(64u, n - base);
        for (uint32_t q = ((r + 1 > base) ? r + 1 - base : 0u) + sub; q < hi; q += SW_SUB) {
          if (c_key[q] > qend) {
            going = false;
            break;
          }
          SwRec F;
          F.x = c_x[q]; F.y = c_y[q]; F.z = c_z[q];
          F.vx = c_vx[q]; F.vy = c_vy[q]; F.vz = c_vz[q];
          F.R = c_R[q]; F.p = c_p[q];
          if (F.p != E.p)
            rb_sw_test(E, F, 0, ngx, ngy, boundary, W, sh, omega, dt, mine, nm, queue, qcap,
                       qcnt, err);
        }
      }
      // (every lane reaches this barrier: the loop bounds are uniform)
      if (!__syncthreads_or(going)) break;
    }
  }
  // images ix != 0 (both ends of the sorted list, near the x boundaries)
  if (act && ngs > 0) {
    // the longest interval, widened against rounding in lo - ix W - L
    const double L =
        __longlong_as_double((long long)lmax_bits[0]) * (1.0 + 1e-9) + 1e-9 * W;
    double elo, ehi2;
    rb_sw_extent(E.x, E.vx, E.R, dt, W, elo, ehi2);
    for (int c = -ngs; c <= ngs; ++c) {
      if (c == 0) continue;
      const double sft = (double)c * W;
      const uint64_t qend = rb_sw_key(ehi - sft, g);
      for (uint32_t f = rb_sw_lower(key, n, rb_sw_key((elo - sft) - L, g)) + sub;
           f < n && key[f] <= qend; f += SW_SUB) {
        const uint32_t pf = orig[f];
        if (pf <= E.p) continue;  // kept from the lower caller index only
        SwRec F;
        F.x = sx[f]; F.y = sy[f]; F.z = sz[f];
        F.vx = svx[f]; F.vy = svy[f]; F.vz = svz[f];
        F.R = sR[f]; F.p = pf;
        rb_sw_test(E, F, c, ngx, ngy, boundary, W, sh, omega, dt, mine, nm, queue, qcap,
                   qcnt, err);
      }
    }
  }
  // the rest: one atomic per wave
  const uint32_t incl = rb_wave_incl_scan(nm);
  const uint32_t tot = __shfl(incl, 63, 64);
  uint32_t qbase = 0;
  if (rb_lane() == 63 && tot) qbase = atomicAdd(qcnt, tot);
  qbase = __shfl(qbase, 63, 64);
  const uint32_t at = qbase + incl - nm;
  for (uint32_t q = 0; q < nm; ++q)
    if (at + q < qcap) queue[at + q] = mine[q];
  if (nm && at + nm > qcap) atomicOr(err, RB_ERR_COLL);
}

// The azimuthal sweep: one wave per SW_EPB consecutive sorted intervals,
// SW_SUB lanes per interval.  The angle is periodic, so interval e checks
// the intervals that overlap it directly (c = 0) or through a turn
// (c = +-1: its own interval shifted by -c 2 pi): for each c the sorted
// intervals starting after lo_e - c 2 pi - L and before hi_e - c 2 pi.  A
// pair is a single pair whatever c (there are no images), so it is kept
// from its lower caller index, and only for the first c whose range holds
// it.
__global__ __launch_bounds__(64) void k_sw_pairs_phi(
    const uint64_t *__restrict__ key, const uint32_t *__restrict__ orig,
    const double *__restrict__ sx, const double *__restrict__ sy,
    const double *__restrict__ sz, const double *__restrict__ svx,
    const double *__restrict__ svy, const double *__restrict__ svz,
    const double *__restrict__ sR, const uint32_t *__restrict__ nlive,
    const PatchInfo *__restrict__ patch, double dt, SweepGrid g,
    const unsigned long long *__restrict__ lmax_bits, uint64_t *__restrict__ queue,
    uint32_t qcap, uint32_t *__restrict__ qcnt, uint32_t *__restrict__ err) {
  const uint32_t lane = threadIdx.x;
  const uint32_t sub = lane % SW_SUB;
  const uint32_t r = blockIdx.x * SW_EPB + lane / SW_SUB;
  const uint32_t n = nlive[0];
  const bool act = r < n;
  const double W = patch[0].W;
  uint64_t mine[RB_COLL_LOCAL];
  uint32_t nm = 0;
  if (act) {
    SwRec E;
    E.x = sx[r]; E.y = sy[r]; E.z = sz[r];
    E.vx = svx[r]; E.vy = svy[r]; E.vz = svz[r];
    E.R = sR[r]; E.p = orig[r];
    double elo, ehi;
    rb_sw_phi_extent(E.x, E.y, E.vx, E.vy, E.R, dt, elo, ehi);
    const double L = __longlong_as_double((long long)lmax_bits[0]) * (1.0 + 1e-9) + 1e-9;
    uint64_t qs[3], qe[3];
    for (int c = -1; c <= 1; ++c) {
      const double sft = (double)c * 2.0 * RB_PI;
      qs[c + 1] = rb_sw_key((elo - sft) - L, g);
      qe[c + 1] = rb_sw_key(ehi - sft, g);
    }
    for (int c = -1; c <= 1; ++c) {
      for (uint32_t f = rb_sw_lower(key, n, qs[c + 1]) + sub; f < n && key[f] <= qe[c + 1];
           f += SW_SUB) {
        const uint32_t pf = orig[f];
        if (pf <= E.p) continue;  // kept from the lower caller index only
        const uint64_t kf = key[f];
        bool seen = false;
        for (int c2 = -1; c2 < c; ++c2) seen |= kf >= qs[c2 + 1] && kf <= qe[c2 + 1];
        if (seen) continue;
        SwRec F;
        F.x = sx[f]; F.y = sy[f]; F.z = sz[f];
        F.vx = svx[f]; F.vy = svy[f]; F.vz = svz[f];
        F.R = sR[f]; F.p = pf;
        rb_sw_test(E, F, 0, 0, 0, RB_OPEN, W, 0.0, 0.0, dt, mine, nm, queue, qcap, qcnt, err);
      }
    }
  }
  // the rest: one atomic per wave
  const uint32_t incl = rb_wave_incl_scan(nm);
  const uint32_t tot = __shfl(incl, 63, 64);
  uint32_t qbase = 0;
  if (rb_lane() == 63 && tot) qbase = atomicAdd(qcnt, tot);
  qbase = __shfl(qbase, 63, 64);
  const uint32_t at = qbase + incl - nm;
  for (uint32_t q = 0; q < nm; ++q)
    if (at + q < qcap) queue[at + q] = mine[q];
  if (nm && at + nm > qcap) atomicOr(err, RB_ERR_COLL);
}

static SweepGrid sweep_grid(const rb_ctx *c, int phi) {
  // lo spans about [x0 - W/2, x0 + 3W/2): 2W over the 63-bit grid (phi:
  // x0 = -pi, W = 2 pi)
  const double W = phi ? 2.0 * RB_PI : c->h_patch[0].W;
  const double x0 = phi ? -RB_PI : c->h_patch[0].x0[0];
  SweepGrid g;
  g.base = x0 - 0.5 * W;
  g.scale = 4.0e18 / (2.0 * W);
  return g;
}

hipError_t launch_sweep_keys(rb_ctx *c, const rb_particles *pp, const double *radius,
                             double dt, int phi) {
  const uint32_t n = (uint32_t)c->h_starts[1];
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sw_keys, dim3(rb_div_up(n, 256)), dim3(256), 0, c->stream, pp->x,
                     pp->y, pp->z, pp->vx, pp->vy, radius, c->d_patch, n,
                     c->p.boundary == RB_OPEN ? 1 : 0, phi, dt, sweep_grid(c, phi), c->d_key[0],
                     c->d_idx[0], c->d_err, c->sort_small ? c->d_bcnt : nullptr, c->d_bctl,
                     c->d_cmax);
  return hipGetLastError();
}

hipError_t launch_sweep_pairs(rb_ctx *c, const rb_particles *pp, const double *radius,
                              double t, double dt, int phi) {
  const uint32_t n = (uint32_t)c->h_starts[1];
  if (n == 0) return hipSuccess;
  double **s = c->d_px[0];
  hipLaunchKernelGGL(k_sw_gather, dim3(rb_div_up(n, 256)), dim3(256), 0, c->stream,
                     c->d_key[0], c->d_idx[0], pp->x, pp->y, pp->z, pp->vx, pp->vy, pp->vz,
                     radius, c->d_patch, n, phi, dt, s[0], s[1], s[2], s[3], s[4], s[5],
                     c->d_swR, c->d_swhi, c->d_orig[0], c->d_nlive);
  if (phi) {
    hipLaunchKernelGGL(k_sw_pairs_phi, dim3(rb_div_up(n, SW_EPB)), dim3(64), 0, c->stream,
                       c->d_key[0], c->d_orig[0], s[0], s[1], s[2], s[3], s[4], s[5],
                       c->d_swR, c->d_nlive, c->d_patch, dt, sweep_grid(c, 1), c->d_cmax,
                       c->d_cq[0], (uint32_t)c->cq_cap, c->d_ccnt, c->d_err);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_sw_pairs, dim3(rb_div_up(n, SW_EPB)), dim3(64), 0, c->stream,
                     c->d_key[0], c->d_orig[0], s[0], s[1], s[2], s[3], s[4], s[5], c->d_swR,
                     c->d_swhi, c->d_nlive, c->d_patch, c->p.n_ghost[0], c->p.n_ghost[1],
                     c->p.boundary, c->p.omega, t, dt, sweep_grid(c, 0), c->d_cmax, c->d_cq[0],
                     (uint32_t)c->cq_cap, c->d_ccnt, c->d_err);
  return hipGetLastError();
}
