// k_walk64.hip -- per-particle FP64 tree walk (Sect. 4.2 of the paper).
//
// The result is the plain per-particle Barnes-Hut sum: every particle makes
// its own opening decisions, w^2 < theta^2 R^2 with R measured from its own
// position to the cell's centre of mass, and visits the nodes it needs in
// depth-first octant order.  The opening test, the image shifts and the
// term arithmetic round exactly as a plain sequential FP64 walk does, so the
// decisions are reproducible bit for bit.
//
// Two schedules give the same sums.  k_walk64 (systems with many work
// units): one wave takes 64 Morton-consecutive particles (one per lane)
// and walks the tree once for all of them.  The node in hand is the same
// for the whole wave, so its record is read with scalar loads; each lane
// tests it against its own particle.  A lane takes part in a node only if
// it opened every ancestor of that node; each lane keeps the deepest level
// down to which it did so along the current path, and a node of level l is
// its when that level is at least l.  Lanes that accept a cell add its
// monopole (and quadrupole) term; the wave descends to the children when
// any lane opened it and moves on to the next node after the subtree
// otherwise.  Every lane
// thus sees exactly the nodes, in exactly the order, that its own
// stackless walk (child link when opening, skip link otherwise) would.
// k_walk64_lane (few work units, where the wave's single chain of dependent
// node loads would leave the chip waiting): every lane follows that
// stackless walk on its own, with its own loads.
#include "rb_internal.h"

// 1 / sqrt(x): hardware estimate y (relative error ~2^-23) refined by one
// third-order step.  With e = 1 - x y^2, 1/sqrt(x) = y (1 - e)^(-1/2) =
// y (1 + e/2 + 3e^2/8 + O(e^3)), so one step takes the error from 2^-23 to
// ~2^-70, below the rounding of the last operations (about one ulp; two
// Newton steps give about two).
__device__ __forceinline__ double rb_rsqrt64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = __builtin_fma(-(x * y), y, 1.0);
  return __builtin_fma(y * e, __builtin_fma(0.375, e, 0.5), y);
}

// The terms a particle adds (d = source - particle, rho^2 = |d|^2 + b^2):
//   monopole   G M d / rho^3
//   quadrupole (5/2) G (d.Q.d) d / rho^7 - G (Q d) / rho^5
// The monopole and the radial part of the quadrupole share the factor
// (G M + (5/2) G (d.Q.d) / rho^4) / rho^3, so a cell costs two fused
// multiply-adds per axis.
__device__ __forceinline__ void w64_mono(double Gm, double d0, double d1, double d2,
                                         double r2, double &ax, double &ay, double &az) {
  const double ri = rb_rsqrt64(r2);
  const double f = Gm * (ri * (ri * ri));
  ax = __builtin_fma(f, d0, ax);
  ay = __builtin_fma(f, d1, ay);
  az = __builtin_fma(f, d2, az);
}

template <bool QUAD>
__device__ __forceinline__ void w64_cell(double G, double Gm, const double *q, double d0,
                                         double d1, double d2, double rho2, double &ax,
                                         double &ay, double &az) {
  const double ri = rb_rsqrt64(rho2);
  const double u = ri * ri, g = ri * u;  // rho^-2, rho^-3
  if (QUAD) {
    const double e0 = __builtin_fma(q[0], d0, __builtin_fma(q[1], d1, q[2] * d2));
    const double e1 = __builtin_fma(q[1], d0, __builtin_fma(q[3], d1, q[4] * d2));
    const double e2 = __builtin_fma(q[2], d0, __builtin_fma(q[4], d1, q[5] * d2));
    const double dqd = __builtin_fma(d0, e0, __builtin_fma(d1, e1, d2 * e2));
    const double gs = g * __builtin_fma((2.5 * G) * dqd, u * u, Gm);
    const double gu = (G * g) * u;
    ax = __builtin_fma(-gu, e0, __builtin_fma(gs, d0, ax));
    ay = __builtin_fma(-gu, e1, __builtin_fma(gs, d1, ay));
    az = __builtin_fma(-gu, e2, __builtin_fma(gs, d2, az));
  } else {
    const double f = Gm * g;
    ax = __builtin_fma(f, d0, ax);
    ay = __builtin_fma(f, d1, ay);
    az = __builtin_fma(f, d2, az);
  }
}

// |d|^2 + b^2
__device__ __forceinline__ double w64_r2(double d0, double d1, double d2, double b2) {
  return __builtin_fma(d0, d0, __builtin_fma(d1, d1, __builtin_fma(d2, d2, b2)));
}

// image ordinal -> offset (ix Lx, iy Ly - ix s, 0), ix outer, iy inner; Lx, Ly
// the domain's extents
__device__ __forceinline__ void rb_image(int im, int ngx, int ngy, int boundary, double Lx,
                                         double Ly, double s, double &ox, double &oy,
                                         bool &self) {
  if (boundary == RB_OPEN) {
    ox = 0.0; oy = 0.0; self = true;
    return;
  }
  const int ny = 2 * ngy + 1;
  const int ix = im / ny - ngx, iy = im % ny - ngy;
  const double fx = (double)ix, fy = (double)iy;
  const double sh = (boundary == RB_SHEAR) ? s : 0.0;
  ox = fx * Lx;
  oy = fy * Ly - fx * sh;
  self = (ix == 0 && iy == 0);
}

// Node records read through the constant address space: the node index is
// uniform over the wave, so these become scalar loads.
typedef __attribute__((address_space(4))) const uint32_t *w64_u32_p;
typedef __attribute__((address_space(4))) const double *w64_dbl_p;

// a node's walk record, in scalar registers
struct W64Rec {
  uint32_t child, skip, count, lvl;
  double cx, cy, cz, m;
};

// A node's record.  With OFF32 the byte offsets of the node's records
// (16 v, 32 v and 48 v for its quadrupole) fit 32 bits, and the scalar
// loads take them as a register offset to the arrays' base, sparing the
// 64-bit address arithmetic of every visit.
template <bool OFF32>
__device__ __forceinline__ const void *w64_at(const void *base, uint32_t v, uint32_t bytes) {
  typedef __attribute__((address_space(4))) const char *cbyte;
  if (OFF32) return (const void *)((cbyte)base + v * bytes);
  return (const void *)((cbyte)base + (size_t)v * bytes);
}

template <bool OFF32>
__device__ __forceinline__ void w64_fetch(w64_u32_p link, w64_dbl_p mcom, uint32_t v,
                                          W64Rec &r) {
  const w64_u32_p lp = (w64_u32_p)w64_at<OFF32>((const void *)link, v, 16u);
  r.child = lp[0]; r.skip = lp[1]; r.count = lp[2]; r.lvl = lp[3];
  const w64_dbl_p mp = (w64_dbl_p)w64_at<OFF32>((const void *)mcom, v, 32u);
  r.cx = mp[0]; r.cy = mp[1]; r.cz = mp[2]; r.m = mp[3];
}

__device__ __forceinline__ uint32_t w64_uniform(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// One wave per workgroup: a wave's slot on the CU is refilled as soon as it
// ends (with four waves per workgroup the slot waits for the slowest of the
// four; measured 2.6-5% slower).  Eight waves per SIMD: the register budget
// that allows them (78 scalar registers, against 106 unbounded) moves only
// set-up values out to vector lanes, none of the node loop's, and the extra
// waves cover more of the node loads' latency (measured 10% faster on the
// 256-patch ensemble).
template <bool QUAD, bool STATS, int PD, bool OFF32>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_walk64(
    const WalkItem *__restrict__ items, uint32_t n_items, int img_split, int n_img, int parts,
    int ngx, int ngy, int boundary, const PatchInfo *__restrict__ patch,
    const uint32_t *__restrict__ nlive, const uint32_t *__restrict__ root,
    const NodeLink *__restrict__ link_g, const double4 *__restrict__ mcom_g,
    const double *__restrict__ Q_g, const double *__restrict__ sx_g,
    const double *__restrict__ sy_g, const double *__restrict__ sz_g,
    const double *__restrict__ msrc_g, const double *__restrict__ sched,
    const uint32_t *__restrict__ ctr, uint32_t P, double G, double b2, double theta2,
    double *__restrict__ acc, uint64_t cap, unsigned long long *__restrict__ stats,
    const uint32_t *__restrict__ lev_off, uint32_t *__restrict__ err, int slot,
    uint32_t *__restrict__ ord) {
  const w64_u32_p link = (w64_u32_p)link_g;
  const w64_dbl_p mcom = (w64_dbl_p)mcom_g;
  const w64_dbl_p Qarr = (w64_dbl_p)Q_g;
  const w64_dbl_p msrc = (w64_dbl_p)msrc_g;
  const w64_dbl_p sxc = (w64_dbl_p)sx_g, syc = (w64_dbl_p)sy_g, szc = (w64_dbl_p)sz_g;
  const uint32_t lane = threadIdx.x & 63u;
  // a unit: a part, an item and its image (when split).  With parts, each
  // part walks one subtree one or two levels below the root (PD levels:
  // 8^PD parts), so a system of few items still gives many units, each with
  // a short chain of node loads; every particle still sees each node once,
  // and the parts' sums are added in order afterwards.  Units are
  // part-major: neighbouring waves (and an XCD's range) walk the same
  // subtree for neighbouring particles and share its node records in the
  // caches.
  const uint32_t np = PD ? (uint32_t)parts : 1u;
  const uint32_t per_part = n_items * (img_split ? (uint32_t)n_img : 1u);
  const uint32_t n_units = per_part * np;
  // One unit per wave.  Workgroups are dealt to the eight XCDs in turn;
  // block b takes its unit from the (b mod 8)-th eighth of the units, so
  // each XCD's L2 holds the nodes of one contiguous eighth of them.  An
  // ordered launch (ctl) first runs the units listed as costly (the first
  // RB_WALK64_HEAVY_MAX blocks, spread over all XCDs), then the rest in
  // that order; a listed unit's own block there has nothing left to do.
  // (only the 64-part instance is ever launched ordered)
  constexpr bool ORD = PD == 2;
  W64Ctl *const ctl = ORD ? (W64Ctl *)ord : nullptr;
  uint32_t unit = 0;
  bool run;
  if (ORD && ctl && blockIdx.x < RB_WALK64_HEAVY_MAX) {  // a listed unit
    // XCD x = b mod 8 runs the list of its own share
    const uint32_t x = blockIdx.x & 7u, j = blockIdx.x >> 3;
    run = j < min(ctl->cnt[ctl->cur & 1u][x], RB_WALK64_HEAVY_MAX / 8u);
    if (run) unit = w64_uniform(ord[RB_W64_HEAVY_OFF + x * (RB_WALK64_HEAVY_MAX / 8u) + j]);
    run = run && unit < n_units;
  } else {  // the units in order (XCD x = b mod 8 either way)
    const uint32_t off = (ORD && ctl) ? RB_WALK64_HEAVY_MAX : 0u;
    const uint32_t b = blockIdx.x - off, nb = gridDim.x - off;
    const uint32_t q = nb >> 3, r = nb & 7u, x = b & 7u;
    unit = x * q + (x < r ? x : r) + (b >> 3);
    run = unit < n_units;  // whole waves
    if (ORD && ctl && run) run = w64_uniform(ord[RB_W64_TAG_OFF + unit]) != ctl->cur;
  }
  if (!run) return;
  // a depth-first walk visits every node at most once per image: more
  // visits, or an index past the node count, mean inconsistent links
  const uint32_t n_nodes = lev_off[RB_NLEV];
  const int part = (int)(unit / per_part);
  const uint32_t sub = unit % per_part;
  const uint32_t item = img_split ? sub / (uint32_t)n_img : sub;
  const int im0 = img_split ? (int)(sub % (uint32_t)n_img) : 0;
  const int im1 = img_split ? im0 + 1 : n_img;
  const WalkItem it = items[item];
  const uint32_t p = it.patch;
  const double W = patch[p].W;
  // (W 2^-l)^2 = fl(W W) 2^-2l exactly: scaling by a power of two is exact
  const double W2 = W * W;
  const int nvirt = (int)patch[p].nvirt;
  const uint32_t st = patch[p].start, nl = nlive[p];
  const uint32_t s = it.start + lane;
  const bool valid = s < it.end && (s - st) < nl;
  const double shear = sched[(size_t)ctr[slot] * 2 * P + p];
  double px = 0.0, py = 0.0, pz = 0.0;
  if (valid) { px = sx_g[s]; py = sy_g[s]; pz = sz_g[s]; }
  const uint64_t live = __ballot(valid);
  const uint32_t r0 = live ? w64_uniform(root[p]) : RB_NONE;
  uint32_t n_open = 0, n_cell = 0, n_pp = 0, n_visits = 0;
  double tx = 0.0, ty = 0.0, tz = 0.0;
  for (int im = im0; im < im1; ++im) {
    double ox, oy;
    bool self;
    rb_image(im, ngx, ngy, boundary, patch[p].L[0], patch[p].L[1], shear, ox, oy, self);
    const double y0 = px - ox, y1 = py - oy, y2 = pz;
    double ax = 0.0, ay = 0.0, az = 0.0;
    uint32_t cur = r0, visits = 0;
    // With parts, the octal digits of part k name a path below the root:
    // k = c (PD = 1) walks the subtree of the root's child c, k = 8 c + g
    // (PD = 2) that of grandchild g of child c.  Before that the part tests
    // the nodes on the path for its lanes (only the lanes that opened them
    // go on); a node's own terms belong to the first part below it (part 0
    // for the root, 8 c for child c), as does a leaf on the path (walked
    // below).  A part stops where its subtree ends: at the next sibling
    // (children are numbered consecutively, and in depth-first order a
    // subtree ends where the next sibling starts), or after the parent's
    // subtree for the last child.
    uint32_t stop = RB_NONE;
    uint64_t act0 = live;  // lanes active at the start node, and its level
    int l0 = 0;
    if (PD > 0 && cur != RB_NONE) {
      const uint32_t digit[2] = {PD == 2 ? (uint32_t)part >> 3 : (uint32_t)part,
                                 (uint32_t)part & 7u};
      uint32_t v = cur, after = RB_NONE;
      uint64_t act = live;
      cur = RB_NONE;
#pragma unroll
      for (int depth = 0; depth < PD; ++depth) {
        if (v >= n_nodes) {
          if (lane == 0) atomicOr(err, RB_ERR_TREE);
          break;
        }
        W64Rec rc;
        w64_fetch<OFF32>(link, mcom, v, rc);
        const int l = (int)(rc.lvl & 255u);
        const uint32_t n_child = rc.lvl >> 9;
        const bool owner = depth == 0 ? part == 0 : digit[1] == 0u;
        if (rc.m == 0.0 || l > RB_DEPTH) break;
        if ((rc.lvl & 256u) != 0u) {  // a leaf: its owner walks it
          if (owner) { cur = v; stop = after; act0 = act; l0 = l; }
          break;
        }
        const bool me = ((act >> lane) & 1ull) != 0;
        const double d0 = rc.cx - y0, d1 = rc.cy - y1, d2 = rc.cz - y2;
        const double R2 = __builtin_fma(d2, d2, __builtin_fma(d1, d1, d0 * d0));
        const bool root_or_below = l >= nvirt;
        const bool take = me && root_or_below && (ldexp(W2, -2 * l) < theta2 * R2);
        const uint64_t opened = act & ~__ballot(take);
        if (owner) {
          if (STATS && me && root_or_below) ++n_open;
          if (take) {
            const w64_dbl_p qn = (w64_dbl_p)w64_at<OFF32>((const void *)Qarr, v, 48u);
            const double q[6] = {qn[0], qn[1], qn[2], qn[3], qn[4], qn[5]};
            w64_cell<QUAD>(G, G * rc.m, q, d0, d1, d2, R2 + b2, ax, ay, az);
            if (STATS) ++n_cell;
          }
        }
        const uint32_t dg = digit[depth];
        if (opened == 0ull || dg >= n_child || l >= RB_DEPTH) break;
        const uint32_t w = rc.child + dg;
        after = (dg + 1u < n_child) ? w + 1u : rc.skip;
        act = opened;
        v = w;
        if (depth == PD - 1) { cur = w; stop = after; act0 = opened; l0 = l + 1; }
      }
    }
    // A lane works on a node of level l when it opened every ancestor of
    // the node.  Along the path from the root to the node in hand those are
    // the levels 0..a of a prefix, and alev holds a (below the start node's
    // level when the lane takes no part): a node of level l is the lane's
    // when alev >= l.  When the wave descends from a node of level l, the
    // lanes working on it set alev to l + 1 if they opened it and to l if
    // they did not; nothing else changes alev.  A lane that opened the
    // parent of a node keeps alev >= its level through the earlier
    // siblings' subtrees (every change there sets alev to a deeper level),
    // and one that did not never works below the parent, so alev >= l
    // is exactly the rule.
    int alev = ((act0 >> lane) & 1ull) ? l0 : -1;
    // the node in hand: NodeLink {child_or_first, skip, count, lvl} and
    // double4 {com, M}, read with scalar loads; the other waves on the SIMD
    // cover their latency.  A walk ends at its stop node (RB_NONE for the
    // whole tree); an index past the node count before that, or more
    // visits than nodes, mean inconsistent links.
    while (cur != stop && max(cur, visits) < n_nodes) {
      ++visits;
      W64Rec rc;
      w64_fetch<OFF32>(link, mcom, cur, rc);
      const uint32_t lv = rc.lvl;
      const int l = (int)(lv & 255u);
      const bool leaf = (lv & 256u) != 0;
      const double d0 = rc.cx - y0, d1 = rc.cy - y1, d2 = rc.cz - y2;
      uint32_t next = rc.skip;
      if (rc.m != 0.0) {
        const bool me = alev >= l;
        const bool single = leaf && rc.count == 1;
        // a single-particle leaf is taken by every lane but its own
        // particle's; a cell below the root boxes by the lanes it passes
        bool take;
        double rho2;
        uint64_t opened = 0ull;
        if (single) {
          take = me && !(self && rc.child == s);
          rho2 = w64_r2(d0, d1, d2, b2);
        } else {
          const double R2 = __builtin_fma(d2, d2, __builtin_fma(d1, d1, d0 * d0));
          // cells above the root boxes are always opened
          const bool root_or_below = l >= nvirt;
          take = me && root_or_below && (ldexp(W2, -2 * l) < theta2 * R2);
          opened = __ballot(me && !take);
          rho2 = R2 + b2;
          if (STATS && me && root_or_below) ++n_open;
        }
        if (take) {
          // one body for both: a single-particle leaf's quadrupole is
          // exactly zero (the build adds none for one particle), and with
          // Q d = 0 and d.Q.d = 0 the cell's terms reduce exactly to the
          // point mass's G M d / rho^3
          const double ri = rb_rsqrt64(rho2);
          const double u = ri * ri, g = ri * u;
          double e0 = 0.0, e1 = 0.0, e2 = 0.0, dqd = 0.0;
          if (QUAD) {
            const w64_dbl_p qn = (w64_dbl_p)w64_at<OFF32>((const void *)Qarr, cur, 48u);
            const double q0 = qn[0], q1 = qn[1], q2 = qn[2], q3 = qn[3], q4 = qn[4], q5 = qn[5];
            e0 = __builtin_fma(q0, d0, __builtin_fma(q1, d1, q2 * d2));
            e1 = __builtin_fma(q1, d0, __builtin_fma(q3, d1, q4 * d2));
            e2 = __builtin_fma(q2, d0, __builtin_fma(q4, d1, q5 * d2));
            dqd = __builtin_fma(d0, e0, __builtin_fma(d1, e1, d2 * e2));
          }
          const double gs = g * __builtin_fma((2.5 * G) * dqd, u * u, G * rc.m);
          const double gu = (G * g) * u;
          ax = __builtin_fma(-gu, e0, __builtin_fma(gs, d0, ax));
          ay = __builtin_fma(-gu, e1, __builtin_fma(gs, d1, ay));
          az = __builtin_fma(-gu, e2, __builtin_fma(gs, d2, az));
          if (STATS) { if (single) ++n_pp; else ++n_cell; }
        }
        if (opened != 0ull) {
          if (leaf) {
            // a bucket leaf that failed the test: its members one by one
            const bool mine = ((opened >> lane) & 1ull) != 0;
            const uint32_t j0 = rc.child, j1 = j0 + rc.count;
            for (uint32_t j = j0; j < j1; ++j) {
              const double mj = msrc[j];
              if (mj == 0.0) continue;
              if (mine && !(self && j == s)) {
                const double f0 = sxc[j] - y0, f1 = syc[j] - y1, f2 = szc[j] - y2;
                w64_mono(G * mj, f0, f1, f2, w64_r2(f0, f1, f2, b2), ax, ay, az);
                if (STATS) ++n_pp;
              }
            }
          } else {
            if (me) alev = take ? l : l + 1;
            next = rc.child;
          }
        }
      }
      cur = w64_uniform(next);
    }
    if (cur != stop && lane == 0) atomicOr(err, RB_ERR_TREE);
    n_visits += visits;
    if (img_split) {
      if (s < it.end) {
        double *a = acc + ((size_t)im * np + part) * 3 * cap;
        a[s] = ax; a[cap + s] = ay; a[2 * cap + s] = az;
      }
    } else {
      tx += ax; ty += ay; tz += az;
    }
  }
  if (!img_split && s < it.end) {
    double *a = acc + (size_t)part * 3 * cap;
    a[s] = tx; a[cap + s] = ty; a[2 * cap + s] = tz;
  }
  if (ORD && ctl && lane == 0) ord[RB_W64_COST_OFF + unit] = n_visits;
  if (STATS) {
    unsigned long long o = n_open, c = n_cell, q2 = n_pp;
    for (int d = 32; d >= 1; d >>= 1) {
      o += __shfl_xor(o, d, 64);
      c += __shfl_xor(c, d, 64);
      q2 += __shfl_xor(q2, d, 64);
    }
    if (lane == 0) {
      atomicAdd(&stats[0], o);
      atomicAdd(&stats[1], c);
      atomicAdd(&stats[2], q2);
    }
  }
}

template <bool QUAD, bool STATS>
__global__ __launch_bounds__(64) void k_walk64_lane(
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
    rb_image(im, ngx, ngy, boundary, patch[p].L[0], patch[p].L[1], shear, ox, oy, self);
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
            w64_mono(G * mc.w, d0, d1, d2, w64_r2(d0, d1, d2, b2), ax, ay, az);
            if (STATS) ++n_pp;
          }
        } else {
          const double d0 = mc.x - y0, d1 = mc.y - y1, d2 = mc.z - y2;
          const double R2 = __builtin_fma(d2, d2, __builtin_fma(d1, d1, d0 * d0));
          const int lv = (int)(lk.lvl & 255u);
          const double w = ldexp(W, -lv);
          // cells above the root boxes are always opened
          const bool root_or_below = lv >= (int)patch[p].nvirt;
          if (STATS && root_or_below) ++n_open;
          if (root_or_below && w * w < theta2 * R2) {
            w64_cell<QUAD>(G, G * mc.w, Qarr + 6 * (size_t)cur, d0, d1, d2, R2 + b2, ax, ay,
                           az);
            if (STATS) ++n_cell;
          } else if (leaf) {
            const uint32_t j0 = lk.child_or_first, j1 = j0 + lk.count;
            for (uint32_t j = j0; j < j1; ++j) {
              const double mj = msrc[j];
              if (mj == 0.0 || (self && j == s)) continue;
              const double e0 = sx[j] - y0, e1 = sy[j] - y1, e2 = sz[j] - y2;
              w64_mono(G * mj, e0, e1, e2, w64_r2(e0, e1, e2, b2), ax, ay, az);
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

// Dispatch order of the 64-part walk's units.  Near-field units take
// several times longer than the median one, and in part-major order some
// start late and leave the chip with a tail of a few waves.  The walk
// records each unit's node visits; before the next launch the units that
// cost at least the threshold (about the top 1/32, from the costs one
// launch earlier) are listed to run first, the rest keeping their
// part-major order.  The order decides only which wave starts first: every
// unit writes its own accumulator set, so the sums do not depend on it.
// Launched for at least RB_WALK64_ORDER_MIN units (so a share holds at
// least 512).
__global__ __launch_bounds__(1024) void k_w64_list(uint32_t *__restrict__ ord,
                                                   uint32_t n_units) {
  __shared__ uint32_t lh[33];
  __shared__ uint32_t lcnt[8], lbase[8];
  __shared__ uint32_t last;
  W64Ctl *const ctl = (W64Ctl *)ord;
  const uint32_t t = threadIdx.x, lane = t & 63u, u = blockIdx.x * 1024u + t;
  const bool in = u < n_units;
  const uint32_t v = in ? ord[RB_W64_COST_OFF + u] : 0u;
  const uint32_t e = ctl->epoch;
  const bool heavy = in && v >= ctl->thr;
  if (t < 33u) lh[t] = 0u;
  if (t < 8u) lcnt[t] = 0u;
  __syncthreads();
  // the XCD share of the walk's grid the unit belongs to (share x starts at
  // unit x q + min(x, r)); a wave's 64 units span at most two shares.  Each
  // wave takes its listed units' places in the block's count of each share
  // (one LDS atomic per wave and share), and the block then reserves its
  // places in the share's list with one atomic per share.
  const uint32_t q = n_units >> 3, r = n_units & 7u;
  const uint32_t x = u < r * (q + 1u) ? u / (q + 1u) : q ? r + (u - r * (q + 1u)) / q : 7u;
  uint32_t k = 0;
  uint64_t todo = __ballot(heavy);
  while (todo) {
    const uint32_t xl = (uint32_t)__shfl((int)x, __ffsll((long long)todo) - 1, 64);
    const uint64_t mine = __ballot(heavy && x == xl);
    uint32_t base = 0;
    if (lane == (uint32_t)(__ffsll((long long)mine) - 1))
      base = atomicAdd(&lcnt[xl], (uint32_t)__popcll(mine));
    base = (uint32_t)__shfl((int)base, __ffsll((long long)mine) - 1, 64);
    if (heavy && x == xl) k = base + (uint32_t)__popcll(mine & ((1ull << lane) - 1ull));
    todo &= ~mine;
  }
  __syncthreads();
  if (t < 8u && lcnt[t] != 0u) lbase[t] = atomicAdd(&ctl->cnt[e & 1u][t], lcnt[t]);
  __syncthreads();
  if (heavy) {
    k += lbase[x];
    if (k < RB_WALK64_HEAVY_MAX / 8u) {
      ord[RB_W64_HEAVY_OFF + x * (RB_WALK64_HEAVY_MAX / 8u) + k] = u;
      ord[RB_W64_TAG_OFF + u] = e;
    }
  }
  // the costs by bit length, block by block into the launch's histogram
  // (one LDS atomic per wave and bit length present)
  const uint32_t bl = v ? 32u - (uint32_t)__clz(v) : 0u;
  uint64_t hm = __ballot(in);
  while (hm) {
    const uint32_t bb = (uint32_t)__shfl((int)bl, __ffsll((long long)hm) - 1, 64);
    const uint64_t m = __ballot(in && bl == bb);
    if (lane == (uint32_t)(__ffsll((long long)m) - 1)) atomicAdd(&lh[bb], (uint32_t)__popcll(m));
    hm &= ~m;
  }
  __syncthreads();
  if (t < 33u && lh[t] != 0u) atomicAdd(&ctl->hist[t], lh[t]);
  __threadfence();
  __syncthreads();
  if (t == 0) last = atomicAdd(&ctl->done, 1u) == gridDim.x - 1u ? 1u : 0u;
  __syncthreads();
  if (last == 0u || t >= 64u) return;
  // the last block: the next threshold is the largest power of two such
  // that at least n_units / 32 units cost that much or more (none while no
  // unit reached it)
  __threadfence();
  const uint32_t h = t < 33u ? atomicExch(&ctl->hist[t], 0u) : 0u;
  uint32_t acc = 0, thr = 0xFFFFFFFFu;
  for (int bl = 32; bl >= 1; --bl) {
    acc += (uint32_t)__builtin_amdgcn_readlane((int)h, bl);
    if (acc > 0 && acc >= n_units / 32u) {
      thr = 1u << (bl - 1);
      break;
    }
  }
  if (t == 0) {
    ctl->thr = thr;
    ctl->cur = e;
    ctl->epoch = e + 1u;
    for (int j = 0; j < 8; ++j) ctl->cnt[(e + 1u) & 1u][j] = 0u;
    ctl->done = 0u;
  }
}

hipError_t launch_walk64(rb_ctx *c, const double *sx, const double *sy, const double *sz,
                         int slot) {
  const uint32_t n_items = (uint32_t)c->h_items64.size();
  if (n_items == 0) return hipSuccess;
  const int split = c->img_split;
  const uint32_t units = split ? n_items * (uint32_t)c->n_img : n_items;
  const double b2 = c->p.softening * c->p.softening;
  const double th2 = c->p.theta * c->p.theta;
  const bool quad = c->p.quadrupole != 0, stats = (c->p.profile & 2) != 0;
  if (c->walk64_mode != 1) {
    const int parts = c->walk_parts;
    unsigned grid = units * (uint32_t)parts;  // one unit per wave and workgroup
    // the 64-part walk runs its costliest units first (by the last launch;
    // measured: the top 1/32 first beats 1/16 and 1/64, and below
    // RB_WALK64_ORDER_MIN units the listing costs more than it saves)
    const bool ordered = parts == RB_WALK64_PARTS2 && grid >= RB_WALK64_ORDER_MIN &&
                         grid <= RB_WALK64_ORDER_CAP;
    uint32_t *ord = ordered ? c->d_w64_ord : nullptr;
    if (ordered) {
      hipLaunchKernelGGL(k_w64_list, dim3(rb_div_up(grid, 1024)), dim3(1024), 0, c->stream, ord,
                         grid);
      grid += RB_WALK64_HEAVY_MAX;
    }
#define RB_WALK64_ARGS                                                                     \
  c->d_items64, n_items, split, c->n_img, parts, c->p.n_ghost[0], c->p.n_ghost[1],          \
      c->p.boundary,                                                                       \
      c->d_patch, c->d_nlive, c->d_root, c->d_link, c->d_mcom, c->d_Q, sx, sy, sz,         \
      c->d_msrc, c->d_sched, c->d_ctr, c->P, c->p.G, b2, th2, c->d_acc, c->cap,           \
      c->d_stats, c->d_lev_off, c->d_err, slot, ord
    const dim3 g(grid), bl(64);
    // 32-bit byte offsets of the node records (48 bytes for a quadrupole)
    const bool off32 = c->node_cap * 48ull < (1ull << 32);
#define RB_W64_LAUNCH(PD)                                                                          \
  do {                                                                                             \
    if (quad && stats) hipLaunchKernelGGL((k_walk64<true, true, PD, false>), g, bl, 0, c->stream, RB_WALK64_ARGS); \
    else if (quad && off32) hipLaunchKernelGGL((k_walk64<true, false, PD, true>), g, bl, 0, c->stream, RB_WALK64_ARGS); \
    else if (quad) hipLaunchKernelGGL((k_walk64<true, false, PD, false>), g, bl, 0, c->stream, RB_WALK64_ARGS); \
    else if (stats) hipLaunchKernelGGL((k_walk64<false, true, PD, false>), g, bl, 0, c->stream, RB_WALK64_ARGS); \
    else if (off32) hipLaunchKernelGGL((k_walk64<false, false, PD, true>), g, bl, 0, c->stream, RB_WALK64_ARGS); \
    else hipLaunchKernelGGL((k_walk64<false, false, PD, false>), g, bl, 0, c->stream, RB_WALK64_ARGS); \
  } while (0)
    if (parts == 64) RB_W64_LAUNCH(2);
    else if (parts == 8) RB_W64_LAUNCH(1);
    else RB_W64_LAUNCH(0);
#undef RB_W64_LAUNCH
#undef RB_WALK64_ARGS
    return hipGetLastError();
  }
  const unsigned grid = units;
#define RB_WALK64_LANE_ARGS                                                              \
  c->d_items64, split, c->n_img, c->p.n_ghost[0], c->p.n_ghost[1], c->p.boundary,        \
      c->d_patch, c->d_nlive, c->d_root, c->d_link, c->d_mcom, c->d_Q, sx, sy, sz,       \
      c->d_msrc, c->d_sched, c->d_ctr, c->P, c->p.G, b2, th2, c->d_acc, c->cap, c->d_stats, \
      c->d_lev_off, c->d_err, slot
  if (quad && stats)
    hipLaunchKernelGGL((k_walk64_lane<true, true>), dim3(grid), dim3(64), 0, c->stream, RB_WALK64_LANE_ARGS);
  else if (quad)
    hipLaunchKernelGGL((k_walk64_lane<true, false>), dim3(grid), dim3(64), 0, c->stream, RB_WALK64_LANE_ARGS);
  else if (stats)
    hipLaunchKernelGGL((k_walk64_lane<false, true>), dim3(grid), dim3(64), 0, c->stream, RB_WALK64_LANE_ARGS);
  else
    hipLaunchKernelGGL((k_walk64_lane<false, false>), dim3(grid), dim3(64), 0, c->stream, RB_WALK64_LANE_ARGS);
#undef RB_WALK64_LANE_ARGS
  return hipGetLastError();
}
