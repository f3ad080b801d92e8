// k_walk32.hip -- grouped FP32-mixed tree walk (a variant of the walk of
// Sect. 4.2 of the paper).
//
// Work items are Morton-contiguous runs of particles: consecutive children
// of one node, each holding at most G particles (G = group_size), packed up
// to G particles in all (emitted during the build), so each item is
// spatially compact and the items partition the particles.  One wave serves
// one work item (an item with all its images, or one (item, image) pair),
// pulled from a device queue by a persistent grid of workgroups of four
// independent waves; floor(64 / n) lanes share each of the item's n
// particles.  The image offsets of the item are tabulated in LDS once.  The
// wave walks the tree once for the whole group (the item's particles): a
// node is accepted for every member at once when w^2 < theta^2 R_min^2,
// R_min being the distance from the node's image-shifted centre of mass to
// the group's bounding box -- no member is closer, so every member would
// accept the node on its own.  Accepted cells
// and the particles of single-particle or opened leaves go to LDS
// interaction lists (ballot / mbcnt compaction), evaluated by all lanes
// reading the same entry (LDS broadcast).
//
// Precision: traversal, opening test, image offsets and group-relative
// positions are FP64.  List entries hold FP32 positions relative to the
// group centre in units of the root-box side W, G M / W^2 and G Q / W^4, so
// FP32 sees O(1) magnitudes.  Each list flush sums its terms in FP32 and
// adds the block sum to an FP64 accumulator.
#include "rb_internal.h"

#define W32_SCAP 1024  // traversal stack entries per wave (node << 5 | image)
#define W32_CL 96      // cell list capacity (flushed at >= 32 entries)
#define W32_CFLUSH 32
#define W32_PL 128     // particle list capacity (flushed at >= 64 entries)
#define W32_RESERVE (7 * RB_DEPTH + 8)
#ifndef W32_CELL_PAIRS
#define W32_CELL_PAIRS 1  // cells two at a time: more registers, better issue
#endif

__device__ __forceinline__ int w32_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
// a value equal in every lane, moved to scalar registers
__device__ __forceinline__ double w32_uniform_d(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// image ordinal -> offset (ix Lx, iy Ly - ix s, 0); Lx, Ly the domain's extents
__device__ __forceinline__ void w32_image(int im, int ngx, int ngy, int boundary, double Lx,
                                          double Ly, double s, double &ox, double &oy) {
  if (boundary == RB_OPEN) { ox = 0.0; oy = 0.0; return; }
  const int ny = 2 * ngy + 1;
  const int ix = im / ny - ngx, iy = im % ny - ngy;
  const double fx = (double)ix, fy = (double)iy;
  const double sh = (boundary == RB_SHEAR) ? s : 0.0;
  ox = fx * Lx;
  oy = fy * Ly - fx * sh;
}

// order a wave's LDS writes before its later reads (a wave runs in lockstep)
__device__ __forceinline__ void w32_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// an interaction-list cell: position and G M, then G Q as (xx, xy, xz, yy)
// and (yz, zz); one record per cell so that a lane reads it from one address
struct W32Cell {
  float4 pos, q0, q1;
};

struct F3 {
  float x, y, z;
};

__device__ __forceinline__ void w32_cell(const float4 a, const float4 q0, const float2 q1,
                                         float px, float py, float pz, float b2, bool quad,
                                         F3 &f) {
  const float dx = a.x - px, dy = a.y - py, dz = a.z - pz;
  const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, b2)));
  // an accepted cell's centre of mass lies outside the group's box by more
  // than its width / theta (at least 2^-21 W / theta), so r2 > 0
  const float ri = __builtin_amdgcn_rsqf(r2);
  const float u = ri * ri;
  const float g = ri * u;
  if (quad) {
    // Q d and (d.Q.d) / rho^4, ordered to keep intermediates in range
    const float qx = fmaf(q0.x, dx, fmaf(q0.y, dy, q0.z * dz));
    const float qy = fmaf(q0.y, dx, fmaf(q0.w, dy, q1.x * dz));
    const float qz = fmaf(q0.z, dx, fmaf(q1.x, dy, q1.y * dz));
    const float dqd = fmaf(dx, qx, fmaf(dy, qy, dz * qz));
    const float s = fmaf((2.5f * u) * u, dqd, a.w);
    const float gs = g * s, gu = g * u;
    f.x = fmaf(-gu, qx, fmaf(gs, dx, f.x));
    f.y = fmaf(-gu, qy, fmaf(gs, dy, f.y));
    f.z = fmaf(-gu, qz, fmaf(gs, dz, f.z));
  } else {
    const float h = g * a.w;
    f.x = fmaf(h, dx, f.x); f.y = fmaf(h, dy, f.y); f.z = fmaf(h, dz, f.z);
  }
}

// b2 carries a floor of 1e-20 (in units of W^2), so that the member's own
// entry (d = 0) and exact duplicates add d * (finite) = 0 without a branch;
// for any separation FP32 can resolve the floor changes nothing
#define W32_R2_FLOOR 1e-20f

__device__ __forceinline__ void w32_part(const float4 a, float px, float py, float pz,
                                         float b2, F3 &f) {
  const float dx = a.x - px, dy = a.y - py, dz = a.z - pz;
  const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, b2)));
  const float ri = __builtin_amdgcn_rsqf(r2);
  const float h = (ri * ri) * (ri * a.w);
  f.x = fmaf(h, dx, f.x); f.y = fmaf(h, dy, f.y); f.z = fmaf(h, dz, f.z);
}

__device__ __forceinline__ void w32_eval_cells(const W32Cell *__restrict__ cel, int cnt, int sub,
                                               int lpp, float px, float py, float pz, float b2,
                                               bool quad, double &ax, double &ay, double &az) {
  F3 f = {0.f, 0.f, 0.f};
  int e = sub;
#if W32_CELL_PAIRS
  for (; e + lpp < cnt; e += 2 * lpp) {
    const float4 a0 = cel[e].pos, a1 = cel[e + lpp].pos;
    float4 q00 = {}, q01 = {}, q10 = {}, q11 = {};
    if (quad) {
      q00 = cel[e].q0; q01 = cel[e + lpp].q0;
      q10 = cel[e].q1; q11 = cel[e + lpp].q1;
    }
    w32_cell(a0, q00, make_float2(q10.x, q10.y), px, py, pz, b2, quad, f);
    w32_cell(a1, q01, make_float2(q11.x, q11.y), px, py, pz, b2, quad, f);
  }
#endif
  for (; e < cnt; e += lpp) {
    float4 q0 = {}, q1 = {};
    if (quad) { q0 = cel[e].q0; q1 = cel[e].q1; }
    w32_cell(cel[e].pos, q0, make_float2(q1.x, q1.y), px, py, pz, b2, quad, f);
  }
  ax += (double)f.x; ay += (double)f.y; az += (double)f.z;
}

__device__ __forceinline__ void w32_eval_parts(const float4 *__restrict__ ppos, int cnt, int sub,
                                               int lpp, float px, float py, float pz, float b2,
                                               double &ax, double &ay, double &az) {
  F3 f = {0.f, 0.f, 0.f};
  int e = sub;
  for (; e + 3 * lpp < cnt; e += 4 * lpp) {
    const float4 a0 = ppos[e], a1 = ppos[e + lpp], a2 = ppos[e + 2 * lpp], a3 = ppos[e + 3 * lpp];
    w32_part(a0, px, py, pz, b2, f);
    w32_part(a1, px, py, pz, b2, f);
    w32_part(a2, px, py, pz, b2, f);
    w32_part(a3, px, py, pz, b2, f);
  }
  for (; e < cnt; e += lpp) w32_part(ppos[e], px, py, pz, b2, f);
  ax += (double)f.x; ay += (double)f.y; az += (double)f.z;
}

template <bool QUAD, bool STATS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_walk32(
    const WalkItem *__restrict__ groups, const WalkItem *__restrict__ groups_mid,
    uint32_t *__restrict__ gctr, int img_split, int n_img,
    int ngx, int ngy, int boundary, const PatchInfo *__restrict__ patch,
    const uint32_t *__restrict__ root, const WNode *__restrict__ wn,
    const double *__restrict__ sx, const double *__restrict__ sy,
    const double *__restrict__ sz, const double *__restrict__ msrc,
    const double *__restrict__ sched, const uint32_t *__restrict__ ctr, uint32_t P,
    double Gc, double soft, double theta2, double *__restrict__ acc, uint64_t cap,
    unsigned long long *__restrict__ stats, uint32_t *__restrict__ err, int slot) {
  // four independent waves per workgroup (fewer workgroups to dispatch),
  // each with its own stack, lists and image table
  __shared__ uint32_t stk_all[4][W32_SCAP];
  __shared__ W32Cell cel_all[4][W32_CL];
  __shared__ float4 ppos_all[4][W32_PL];
  __shared__ double2 img_all[4][RB_MAX_IMAGES];

  static_assert(sizeof(cel_all[0]) >= 3 * 64 * sizeof(double), "reduction space");
  // the wave index is uniform: keep it (and the LDS bases) in scalar registers
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t *stk = stk_all[wv];
  W32Cell *cel = cel_all[wv];
  float4 *ppos = ppos_all[wv];
  double2 *img = img_all[wv];
  const uint32_t n_big = gctr[2], n_mid = gctr[3];  // walk items by size
  const uint32_t n_groups = n_big + n_mid + gctr[4];
  const uint32_t per = img_split ? (uint32_t)n_img : 1u;
  const uint32_t n_items = n_groups * per;
  const double theta2d = theta2;
  const uint32_t step = ctr[slot];
  unsigned long long n_cell = 0, n_pp = 0;
  // the first item of every wave is fixed by its position in the grid; the
  // others come from the queue (one atomic each instead of one per wave at
  // start-up, when they would all hit the one counter at once)
  bool first = true;
  for (;;) {
    uint32_t item = 4u * blockIdx.x + (uint32_t)wv;
    if (!first) {
      if (lane == 0) item = 4u * gridDim.x + atomicAdd(&gctr[1], 1u);
      item = (uint32_t)w32_uniform((int)__shfl(item, 0, 64));
    }
    first = false;
    if (item >= n_items) break;
    // split items: all central images first (the heaviest), then the rest
    const uint32_t gi = img_split ? item % n_groups : item;
    const int im0 =
        img_split ? (int)((item / n_groups + (uint32_t)(n_img / 2)) % (uint32_t)n_img) : 0;
    const int nim = img_split ? 1 : n_img;
    const WalkItem grp = rb_walk_item(groups, groups_mid, gi, n_big, n_mid, cap);
    const uint32_t p = grp.patch;
    const double W = patch[p].W;
    const int nvirt = (int)patch[p].nvirt;
    const int cnt = (int)(grp.end - grp.start);
    if (cnt < 1 || cnt > 64 || grp.end > cap) {  // never emitted
      if (lane == 0) atomicOr(err, RB_ERR_TREE);
      continue;
    }
    // lpp = floor(64 / cnt) lanes per member, lane = member + cnt * sub;
    // the lanes past lpp * cnt repeat members and are left out of the sums
    const int lpp = 64 / cnt;
    const int pidx = lane % cnt, sub = lane / cnt;
    const bool valid = sub < lpp;
    const uint32_t s = grp.start + (uint32_t)pidx;

    double x = sx[s], y = sy[s], z = sz[s];
    double lx = valid ? x : INFINITY, ly = valid ? y : INFINITY, lz = valid ? z : INFINITY;
    double hx = valid ? x : -INFINITY, hy = valid ? y : -INFINITY, hz = valid ? z : -INFINITY;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      lx = fmin(lx, __shfl_xor(lx, d, 64)); ly = fmin(ly, __shfl_xor(ly, d, 64));
      lz = fmin(lz, __shfl_xor(lz, d, 64)); hx = fmax(hx, __shfl_xor(hx, d, 64));
      hy = fmax(hy, __shfl_xor(hy, d, 64)); hz = fmax(hz, __shfl_xor(hz, d, 64));
    }
    // the box is the same in every lane
    lx = w32_uniform_d(lx); ly = w32_uniform_d(ly); lz = w32_uniform_d(lz);
    hx = w32_uniform_d(hx); hy = w32_uniform_d(hy); hz = w32_uniform_d(hz);
    const double gx = 0.5 * (lx + hx), gy = 0.5 * (ly + hy), gz = 0.5 * (lz + hz);
    const double invW = 1.0 / W;
    const double gm_scale = Gc * invW * invW;
    const double gq_scale = gm_scale * invW * invW;
    const float b2 = (float)((soft * invW) * (soft * invW)) + W32_R2_FLOOR;
    const float px = (float)((x - gx) * invW), py = (float)((y - gy) * invW),
                pz = (float)((z - gz) * invW);
    const double shear = sched[(size_t)step * 2 * P + p];
    const uint32_t r0 = root[p];
    double ax = 0.0, ay = 0.0, az = 0.0;
    if (lane < n_img) {
      double ox, oy;
      w32_image(lane, ngx, ngy, boundary, patch[p].L[0], patch[p].L[1], shear, ox, oy);
      img[lane] = make_double2(ox, oy);
    }

    int sp = nim;
    if (lane < nim) stk[lane] = (r0 << 5) | (uint32_t)(im0 + lane);
    int cl = 0, pl = 0;
    bool overflow = false;
    const float gqs = (float)gq_scale;
    // Pop up to 64 entries; each may push 8 children.  Near the limit the
    // wave pops one entry per round (depth first): that path needs at most 7
    // entries per level below, which W32_RESERVE keeps free.  The node
    // records of the next batch are requested before the current lists are
    // evaluated, so their memory latency overlaps the arithmetic.
    auto pop = [&](int &k, uint32_t &e, NodeLink &lk, double4 &mc, float4 &q0, float2 &q1) {
      k = sp < 64 ? sp : 64;
      if (sp + 7 * k > W32_SCAP - W32_RESERVE) {
        k = (W32_SCAP - W32_RESERVE - sp) / 7;
        if (k < 1) k = (sp > 0) ? 1 : 0;
      }
      const int base = sp - k;
      const bool has = lane < k;
      e = has ? stk[base + lane] : 0u;
      sp = base;
      lk = {0u, 0u, 0u, 0u};
      mc = make_double4(0.0, 0.0, 0.0, 0.0);
      q0 = make_float4(0.f, 0.f, 0.f, 0.f);
      q1 = make_float2(0.f, 0.f);
      if (has) {
        const uint32_t nd = e >> 5;
        const WNode r = wn[nd];  // one 64-byte line
        lk.child_or_first = r.child_or_first;
        lk.count = r.count;
        lk.lvl = r.lvl;
        mc = make_double4(r.cx, r.cy, r.cz, r.M);
        if (QUAD) {
          q0 = make_float4(r.qxx, r.qxy, r.qxz, r.qyy);
          q1 = make_float2(r.qyz, -(r.qxx + r.qyy));
        }
      }
    };
    int k;
    uint32_t e;
    NodeLink lk;
    double4 mc;
    float4 q0;
    float2 q1;
    pop(k, e, lk, mc, q0, q1);
    while (k > 0) {
      if (sp + 8 * k > W32_SCAP) { overflow = true; break; }
      const bool has = lane < k;
      const int im = (int)(e & 31u);
      const bool alive = has && mc.w != 0.0;
      const double2 io = img[im];
      const double ox = io.x, oy = io.y;
      const double cx = mc.x + ox, cy = mc.y + oy, cz = mc.z;
      const bool leaf = (lk.lvl & 256u) != 0;
      const bool single = alive && leaf && lk.count == 1;
      const double dx = fmax(fmax(lx - cx, cx - hx), 0.0);
      const double dy = fmax(fmax(ly - cy, cy - hy), 0.0);
      const double dz = fmax(fmax(lz - cz, cz - hz), 0.0);
      const double R2 = dx * dx + dy * dy + dz * dz;
      const int lv = (int)(lk.lvl & 255u);
      const double w = ldexp(W, -lv);
      // cells above the root boxes are always opened
      const bool accept = alive && !single && lv >= nvirt && (w * w < theta2d * R2);
      const bool open_leaf = alive && !single && !accept && leaf;
      const bool open_node = alive && !single && !accept && !leaf;

      // children onto the stack
      const uint32_t nc = open_node ? ((lk.lvl >> 9) & 15u) : 0u;
      const uint32_t incl = rb_wave_incl_scan(nc);
      const int tot = w32_uniform((int)__shfl(incl, 63, 64));
      for (uint32_t q = 0; q < nc; ++q)
        stk[sp + (int)(incl - nc + q)] = ((lk.child_or_first + q) << 5) | (uint32_t)im;
      sp += tot;

      // accepted cells
      {
        const uint64_t m = __ballot(accept);
        if (accept) {
          const int pos = cl + (int)rb_mbcnt(m);
          cel[pos].pos = make_float4((float)((cx - gx) * invW), (float)((cy - gy) * invW),
                                     (float)((cz - gz) * invW), (float)(mc.w * gm_scale));
          if (QUAD) {
            cel[pos].q0 = make_float4(q0.x * gqs, q0.y * gqs, q0.z * gqs, q0.w * gqs);
            cel[pos].q1 = make_float4(q1.x * gqs, q1.y * gqs, 0.f, 0.f);
          }
        }
        cl += __popcll(m);
      }
      // single-particle leaves
      {
        const uint64_t m = __ballot(single);
        if (single) {
          const int pos = pl + (int)rb_mbcnt(m);
          ppos[pos] = make_float4((float)((cx - gx) * invW), (float)((cy - gy) * invW),
                                  (float)((cz - gz) * invW), (float)(mc.w * gm_scale));
        }
        pl += __popcll(m);
      }
      // opened bucket leaves: the wave expands them one after another
      uint64_t bm = __ballot(open_leaf);
      while (bm) {
        const int src = __ffsll((long long)bm) - 1;
        bm &= bm - 1;
        const uint32_t first = __shfl(lk.child_or_first, src, 64);
        const uint32_t count = __shfl(lk.count, src, 64);
        const double bx = __shfl(ox, src, 64), by = __shfl(oy, src, 64);
        for (uint32_t c0 = 0; c0 < count; c0 += 64) {
          if (pl + 64 > W32_PL) {
            w32_eval_parts(ppos, pl, sub, lpp, px, py, pz, b2, ax, ay, az);
            if (STATS) n_pp += (unsigned long long)pl * (unsigned long long)cnt;
            pl = 0;
          }
          const uint32_t j = first + c0 + (uint32_t)lane;
          const bool inb = c0 + (uint32_t)lane < count;
          const double mj = inb ? msrc[j] : 0.0;
          const bool use = inb && mj != 0.0;
          const uint64_t m = __ballot(use);
          if (use) {
            const int pos = pl + (int)rb_mbcnt(m);
            ppos[pos] = make_float4((float)((sx[j] + bx - gx) * invW),
                                    (float)((sy[j] + by - gy) * invW),
                                    (float)((sz[j] - gz) * invW), (float)(mj * gm_scale));
          }
          pl += __popcll(m);
        }
      }
      // next batch in flight while the lists are evaluated
      pop(k, e, lk, mc, q0, q1);
      if (cl >= W32_CFLUSH) {
        w32_eval_cells(cel, cl, sub, lpp, px, py, pz, b2, QUAD, ax, ay, az);
        if (STATS) n_cell += (unsigned long long)cl * (unsigned long long)cnt;
        cl = 0;
      }
      if (pl >= 64) {
        w32_eval_parts(ppos, pl, sub, lpp, px, py, pz, b2, ax, ay, az);
        if (STATS) n_pp += (unsigned long long)pl * (unsigned long long)cnt;
        pl = 0;
      }
    }
    if (overflow && lane == 0) atomicOr(err, RB_ERR_STACK);
    if (cl > 0) {
      w32_eval_cells(cel, cl, sub, lpp, px, py, pz, b2, QUAD, ax, ay, az);
      if (STATS) n_cell += (unsigned long long)cl * (unsigned long long)cnt;
    }
    if (pl > 0) {
      w32_eval_parts(ppos, pl, sub, lpp, px, py, pz, b2, ax, ay, az);
      if (STATS) n_pp += (unsigned long long)pl * (unsigned long long)cnt;
    }
    // lanes m, m + cnt, ... hold partial sums of member m: added in that
    // order through the wave's cell list, which is no longer needed
    double(*red)[64] = reinterpret_cast<double(*)[64]>(cel);
    w32_wave_sync();
    red[0][lane] = ax; red[1][lane] = ay; red[2][lane] = az;
    w32_wave_sync();
    if (lane < cnt) {
      double tx = red[0][lane], ty = red[1][lane], tz = red[2][lane];
      for (int k = 1; k < lpp; ++k) {
        tx += red[0][lane + k * cnt]; ty += red[1][lane + k * cnt]; tz += red[2][lane + k * cnt];
      }
      double *a = acc + (size_t)(img_split ? im0 : 0) * 3 * cap;
      a[s] = tx; a[cap + s] = ty; a[2 * cap + s] = tz;
    }
    w32_wave_sync();  // the list is rewritten by the next item
  }
  if (STATS && lane == 0) {
    atomicAdd(&stats[3], n_cell);
    atomicAdd(&stats[4], n_pp);
  }
}

// ---------------------------------------------------------------------------
// The same walk with NW waves per group (one workgroup per work item).  The
// traversal stack is shared: every round each wave takes up to 64 entries
// of the batch, tests them, and the children are written back at offsets
// fixed by the wave order, so the traversal (and every sum) is the same on
// every run.  Each wave keeps its own interaction lists and evaluates them
// for all of the group's particles; the waves' partial forces are added in
// wave order at the end.  Two barriers per round; a group's chain of
// dependent rounds is up to NW times shorter.
// list capacities of the multi-wave walk: a list is evaluated at the start
// of a round once it holds W32M_CFLUSH cells (W32M_PFLUSH particles), while
// that round's node records are in flight; a round adds at most 64 entries
// per wave.  Evaluating every round's entries in the next round keeps the
// lists (and LDS) small and spreads the arithmetic evenly over the rounds.
#ifndef W32M_CL
#define W32M_CL 64
#define W32M_CFLUSH 1
#define W32M_PL 64
#define W32M_PFLUSH 1
#endif
#ifndef W32M_WAVES_PER_EU
#define W32M_WAVES_PER_EU 4
#endif
static_assert(W32M_CL >= W32M_CFLUSH - 1 + 64 && W32M_PL >= W32M_PFLUSH - 1 + 64,
              "a round's appends must fit after a partial list");

template <bool QUAD, bool STATS, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(W32M_WAVES_PER_EU, 8))) void k_walk32m(
    const WalkItem *__restrict__ groups, const WalkItem *__restrict__ groups_mid,
    uint32_t *__restrict__ gctr, int img_split, int n_img,
    int ngx, int ngy, int boundary, const PatchInfo *__restrict__ patch,
    const uint32_t *__restrict__ root, const WNode *__restrict__ wn, const double *__restrict__ sx,
    const double *__restrict__ sy, const double *__restrict__ sz,
    const double *__restrict__ msrc, const double *__restrict__ sched,
    const uint32_t *__restrict__ ctr, uint32_t P, double Gc, double soft, double theta2,
    double *__restrict__ acc, uint64_t cap, unsigned long long *__restrict__ stats,
    uint32_t *__restrict__ err, int slot) {
  constexpr int W32M_SCAP = 512 * NW + 512;  // batches of 64 NW, 8 children each, plus depth
  __shared__ uint32_t stk[W32M_SCAP];
  __shared__ W32Cell cel_all[NW][W32M_CL];
  __shared__ float4 ppos_all[NW][W32M_PL];
  __shared__ uint32_t s_push[NW];
  __shared__ uint32_t s_item;
  __shared__ double2 img[RB_MAX_IMAGES];
  // the waves' partial forces, once the lists are no longer needed
  static_assert(sizeof(cel_all) >= NW * 3 * 64 * sizeof(double), "reduction space");
  double(*s_red)[3][64] = reinterpret_cast<double(*)[3][64]>(&cel_all[0][0]);

  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  W32Cell *cel = cel_all[w];
  float4 *ppos = ppos_all[w];
  const uint32_t n_big = gctr[2], n_mid = gctr[3];  // walk items by size
  const uint32_t n_groups = n_big + n_mid + gctr[4];
  const uint32_t per = img_split ? (uint32_t)n_img : 1u;
  const uint32_t n_items = n_groups * per;
  const double theta2d = theta2;
  const uint32_t step = ctr[slot];
  unsigned long long n_cell = 0, n_pp = 0;
  // The first item of every workgroup is fixed by its position in the
  // grid, the others come from the queue.  Workgroups are dispatched to the
  // eight XCDs in turn (workgroup b on XCD b mod 8, each XCD with its own
  // L2).  When every item has a workgroup of its own, XCD x takes the x-th
  // eighth of each size class: its items are neighbours in the tables
  // (which follow the tree's slot order within a level), so its L2 holds
  // their part of the tree, and every XCD gets the same mix of sizes.
  uint32_t item0 = blockIdx.x;
  if (!img_split && (gridDim.x & 7u) == 0 && n_items + 24u <= gridDim.x) {
    const uint32_t x = blockIdx.x & 7u, j = blockIdx.x >> 3;
    const uint32_t n_small = n_groups - n_big - n_mid;
    const uint32_t b0 = n_big * x / 8u, nb = n_big * (x + 1u) / 8u - b0;
    const uint32_t m0 = n_mid * x / 8u, nm = n_mid * (x + 1u) / 8u - m0;
    const uint32_t q0 = n_small * x / 8u, nq = n_small * (x + 1u) / 8u - q0;
    if (j < nb) item0 = b0 + j;
    else if (j < nb + nm) item0 = n_big + m0 + (j - nb);
    else if (j < nb + nm + nq) item0 = n_big + n_mid + q0 + (j - nb - nm);
    else item0 = n_items;  // no item for this workgroup
  }
  bool first = true;
  for (;;) {
    if (threadIdx.x == 0) s_item = first ? item0 : gridDim.x + atomicAdd(&gctr[1], 1u);
    first = false;
    __syncthreads();
    const uint32_t item = (uint32_t)w32_uniform((int)s_item);
    __syncthreads();  // every thread has read the item before it changes
    if (item >= n_items) break;  // uniform over the block
    const uint32_t gi = img_split ? item % n_groups : item;
    const int im0 =
        img_split ? (int)((item / n_groups + (uint32_t)(n_img / 2)) % (uint32_t)n_img) : 0;
    const int nim = img_split ? 1 : n_img;
    const WalkItem grp = rb_walk_item(groups, groups_mid, gi, n_big, n_mid, cap);
    const uint32_t p = grp.patch;
    const double W = patch[p].W;
    const int nvirt = (int)patch[p].nvirt;
    const int cnt = (int)(grp.end - grp.start);
    if (cnt < 1 || cnt > 64 || grp.end > cap) {  // never emitted
      if (lane == 0) atomicOr(err, RB_ERR_TREE);
      continue;
    }
    // lpp = floor(64 / cnt) lanes per member, lane = member + cnt * sub;
    // the lanes past lpp * cnt repeat members and are left out of the sums
    const int lpp = 64 / cnt;
    const int pidx = lane % cnt, sub = lane / cnt;
    const bool valid = sub < lpp;
    const uint32_t s = grp.start + (uint32_t)pidx;
    double x = sx[s], y = sy[s], z = sz[s];
    double lx = valid ? x : INFINITY, ly = valid ? y : INFINITY, lz = valid ? z : INFINITY;
    double hx = valid ? x : -INFINITY, hy = valid ? y : -INFINITY, hz = valid ? z : -INFINITY;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      lx = fmin(lx, __shfl_xor(lx, d, 64)); ly = fmin(ly, __shfl_xor(ly, d, 64));
      lz = fmin(lz, __shfl_xor(lz, d, 64)); hx = fmax(hx, __shfl_xor(hx, d, 64));
      hy = fmax(hy, __shfl_xor(hy, d, 64)); hz = fmax(hz, __shfl_xor(hz, d, 64));
    }
    // the box is the same in every lane
    lx = w32_uniform_d(lx); ly = w32_uniform_d(ly); lz = w32_uniform_d(lz);
    hx = w32_uniform_d(hx); hy = w32_uniform_d(hy); hz = w32_uniform_d(hz);
    const double gx = 0.5 * (lx + hx), gy = 0.5 * (ly + hy), gz = 0.5 * (lz + hz);
    const double invW = 1.0 / W;
    const double gm_scale = Gc * invW * invW;
    const double gq_scale = gm_scale * invW * invW;
    const float b2 = (float)((soft * invW) * (soft * invW)) + W32_R2_FLOOR;
    const float px = (float)((x - gx) * invW), py = (float)((y - gy) * invW),
                pz = (float)((z - gz) * invW);
    const double shear = sched[(size_t)step * 2 * P + p];
    const uint32_t r0 = root[p];
    double ax = 0.0, ay = 0.0, az = 0.0;
    if (w == 0 && lane < nim) stk[lane] = (r0 << 5) | (uint32_t)(im0 + lane);
    if (w == 0 && lane < n_img) {
      double ox, oy;
      w32_image(lane, ngx, ngy, boundary, patch[p].L[0], patch[p].L[1], shear, ox, oy);
      img[lane] = make_double2(ox, oy);
    }
    int sp = nim;  // every wave keeps the same copy
    int cl = 0, pl = 0;
    bool overflow = false;
    const float gqs = (float)gq_scale;
    __syncthreads();
    for (;;) {
      // this round's batch: the top T entries, 64 per wave
      int T = sp < 64 * NW ? sp : 64 * NW;
      if (sp + 7 * T > W32M_SCAP - W32_RESERVE) {
        T = (W32M_SCAP - W32_RESERVE - sp) / 7;
        if (T < 1) T = (sp > 0) ? 1 : 0;
      }
      if (T == 0) break;  // uniform: sp is the same in every wave
      const int base = sp - T;
      const int k = T - 64 * w < 0 ? 0 : (T - 64 * w > 64 ? 64 : T - 64 * w);
      const bool has = lane < k;
      const uint32_t e = has ? stk[base + 64 * w + lane] : 0u;
      NodeLink lk = {0u, 0u, 0u, 0u};
      double4 mc = make_double4(0.0, 0.0, 0.0, 0.0);
      float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f);
      float2 q1 = make_float2(0.f, 0.f);
      if (has) {
        const uint32_t nd = e >> 5;
        const WNode r = wn[nd];  // one 64-byte line
        lk.child_or_first = r.child_or_first;
        lk.count = r.count;
        lk.lvl = r.lvl;
        mc = make_double4(r.cx, r.cy, r.cz, r.M);
        if (QUAD) {
          q0 = make_float4(r.qxx, r.qxy, r.qxz, r.qyy);
          q1 = make_float2(r.qyz, -(r.qxx + r.qyy));
        }
      }
      // full lists are evaluated while the node records are in flight
      if (cl >= W32M_CFLUSH) {
        w32_eval_cells(cel, cl, sub, lpp, px, py, pz, b2, QUAD, ax, ay, az);
        if (STATS) n_cell += (unsigned long long)cl * (unsigned long long)cnt;
        cl = 0;
      }
      if (pl >= W32M_PFLUSH) {
        w32_eval_parts(ppos, pl, sub, lpp, px, py, pz, b2, ax, ay, az);
        if (STATS) n_pp += (unsigned long long)pl * (unsigned long long)cnt;
        pl = 0;
      }
      const int im = (int)(e & 31u);
      const bool alive = has && mc.w != 0.0;
      const double2 io = img[im];
      const double ox = io.x, oy = io.y;
      const double cx = mc.x + ox, cy = mc.y + oy, cz = mc.z;
      const bool leaf = (lk.lvl & 256u) != 0;
      const bool single = alive && leaf && lk.count == 1;
      const double dx = fmax(fmax(lx - cx, cx - hx), 0.0);
      const double dy = fmax(fmax(ly - cy, cy - hy), 0.0);
      const double dz = fmax(fmax(lz - cz, cz - hz), 0.0);
      const double R2 = dx * dx + dy * dy + dz * dz;
      const int lv = (int)(lk.lvl & 255u);
      const double wd = ldexp(W, -lv);
      // cells above the root boxes are always opened
      const bool accept = alive && !single && lv >= nvirt && (wd * wd < theta2d * R2);
      const bool open_leaf = alive && !single && !accept && leaf;
      const bool open_node = alive && !single && !accept && !leaf;
      const uint32_t nc = open_node ? ((lk.lvl >> 9) & 15u) : 0u;
      const uint32_t incl = rb_wave_incl_scan(nc);
      const uint32_t tot = (uint32_t)w32_uniform((int)__shfl(incl, 63, 64));
      if (lane == 0) s_push[w] = tot;
      __syncthreads();  // batch read everywhere, push counts known
      uint32_t off = (uint32_t)base, all = 0;
#pragma unroll
      for (int q = 0; q < NW; ++q) {
        const uint32_t t_q = s_push[q];
        if (q < w) off += t_q;
        all += t_q;
      }
      if ((uint32_t)base + all > W32M_SCAP) {
        overflow = true;  // cannot happen with the reserve above; stop cleanly
      } else {
        for (uint32_t q = 0; q < nc; ++q)
          stk[off + incl - nc + q] = ((lk.child_or_first + q) << 5) | (uint32_t)im;
      }
      sp = overflow ? 0 : base + (int)all;
      // accepted cells
      {
        const uint64_t m = __ballot(accept);
        if (accept) {
          const int pos = cl + (int)rb_mbcnt(m);
          cel[pos].pos = make_float4((float)((cx - gx) * invW), (float)((cy - gy) * invW),
                                     (float)((cz - gz) * invW), (float)(mc.w * gm_scale));
          if (QUAD) {
            cel[pos].q0 = make_float4(q0.x * gqs, q0.y * gqs, q0.z * gqs, q0.w * gqs);
            cel[pos].q1 = make_float4(q1.x * gqs, q1.y * gqs, 0.f, 0.f);
          }
        }
        cl += __popcll(m);
      }
      // single-particle leaves
      {
        const uint64_t m = __ballot(single);
        if (single) {
          const int pos = pl + (int)rb_mbcnt(m);
          ppos[pos] = make_float4((float)((cx - gx) * invW), (float)((cy - gy) * invW),
                                  (float)((cz - gz) * invW), (float)(mc.w * gm_scale));
        }
        pl += __popcll(m);
      }
      // opened bucket leaves: the wave expands them one after another
      uint64_t bm = __ballot(open_leaf);
      while (bm) {
        const int src = __ffsll((long long)bm) - 1;
        bm &= bm - 1;
        const uint32_t first = __shfl(lk.child_or_first, src, 64);
        const uint32_t count = __shfl(lk.count, src, 64);
        const double bx = __shfl(ox, src, 64), by = __shfl(oy, src, 64);
        for (uint32_t c0 = 0; c0 < count; c0 += 64) {
          if (pl + 64 > W32M_PL) {
            w32_eval_parts(ppos, pl, sub, lpp, px, py, pz, b2, ax, ay, az);
            if (STATS) n_pp += (unsigned long long)pl * (unsigned long long)cnt;
            pl = 0;
          }
          const uint32_t j = first + c0 + (uint32_t)lane;
          const bool inb = c0 + (uint32_t)lane < count;
          const double mj = inb ? msrc[j] : 0.0;
          const bool use = inb && mj != 0.0;
          const uint64_t m = __ballot(use);
          if (use) {
            const int pos = pl + (int)rb_mbcnt(m);
            ppos[pos] = make_float4((float)((sx[j] + bx - gx) * invW),
                                    (float)((sy[j] + by - gy) * invW),
                                    (float)((sz[j] - gz) * invW), (float)(mj * gm_scale));
          }
          pl += __popcll(m);
        }
      }
      __syncthreads();  // children written before the next round reads them
    }
    if (overflow && threadIdx.x == 0) atomicOr(err, RB_ERR_STACK);
    if (cl > 0) {
      w32_eval_cells(cel, cl, sub, lpp, px, py, pz, b2, QUAD, ax, ay, az);
      if (STATS) n_cell += (unsigned long long)cl * (unsigned long long)cnt;
    }
    if (pl > 0) {
      w32_eval_parts(ppos, pl, sub, lpp, px, py, pz, b2, ax, ay, az);
      if (STATS) n_pp += (unsigned long long)pl * (unsigned long long)cnt;
    }
    // the partial forces of member m sit in lanes m, m + cnt, ... of every
    // wave: added in wave order, then lane order (every wave has finished
    // its list evaluation before the lists' memory is reused)
    __syncthreads();
    s_red[w][0][lane] = ax; s_red[w][1][lane] = ay; s_red[w][2][lane] = az;
    __syncthreads();
    if (w == 0 && lane < cnt) {
      double tx = 0.0, ty = 0.0, tz = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) {
        for (int k = 0; k < lpp; ++k) {
          tx += s_red[q][0][lane + k * cnt]; ty += s_red[q][1][lane + k * cnt];
          tz += s_red[q][2][lane + k * cnt];
        }
      }
      double *a = acc + (size_t)(img_split ? im0 : 0) * 3 * cap;
      a[s] = tx; a[cap + s] = ty; a[2 * cap + s] = tz;
    }
    __syncthreads();  // s_red and the stack are reused by the next item
  }
  if (STATS && lane == 0) {
    atomicAdd(&stats[3], n_cell);
    atomicAdd(&stats[4], n_pp);
  }
}

hipError_t launch_walk32(rb_ctx *c, const double *sx, const double *sy, const double *sz,
                         int slot) {
  const uint32_t n = (uint32_t)c->h_starts[c->P];
  if (n == 0) return hipSuccess;
  if (c->node_cap >= (1ull << 27)) return hipErrorInvalidValue;  // stack entry packing
  // persistent grid: enough waves to fill every CU several times over, and
  // never more than there can be work items
  const uint64_t max_items = (uint64_t)n * (c->img_split ? (uint64_t)c->n_img : 1ull);
  uint64_t grid = 256ull * 24ull;
  if (grid > max_items) grid = max_items;
  const double th2 = c->p.theta * c->p.theta;
  const bool quad = c->p.quadrupole != 0, stats = (c->p.profile & 2) != 0;
#define RB_W32_ARGS                                                                      \
  c->d_witems, c->d_witems_mid, c->d_gctr, c->img_split, c->n_img, c->p.n_ghost[0],      \
      c->p.n_ghost[1],                                                                    \
      c->p.boundary, c->d_patch, c->d_root, c->d_wnode, sx,                               \
      sy, sz,                                                                             \
      c->d_msrc, c->d_sched, c->d_ctr, c->P, c->p.G, c->p.softening, th2, c->d_acc,       \
      c->cap, c->d_stats, c->d_err, slot
  const int nw = c->p.walk_waves;
  if (nw == 2 || nw == 4) {
    // persistent grid of workgroups
    uint64_t gridm = 256ull * (nw == 2 ? 12ull : 6ull);
    if (gridm > max_items) gridm = max_items;
    const dim3 gm((unsigned)gridm), bm(64 * nw);
#define RB_W32M(Q, S)                                                                   \
  if (nw == 2) hipLaunchKernelGGL((k_walk32m<Q, S, 2>), gm, bm, 0, c->stream, RB_W32_ARGS); \
  else hipLaunchKernelGGL((k_walk32m<Q, S, 4>), gm, bm, 0, c->stream, RB_W32_ARGS);
    if (quad && stats) { RB_W32M(true, true) }
    else if (quad) { RB_W32M(true, false) }
    else if (stats) { RB_W32M(false, true) }
    else { RB_W32M(false, false) }
#undef RB_W32M
    return hipGetLastError();
  }
  const dim3 g4((unsigned)((grid + 3) / 4)), b4(256);  // four waves per workgroup
  if (quad && stats)
    hipLaunchKernelGGL((k_walk32<true, true>), g4, b4, 0, c->stream, RB_W32_ARGS);
  else if (quad)
    hipLaunchKernelGGL((k_walk32<true, false>), g4, b4, 0, c->stream, RB_W32_ARGS);
  else if (stats)
    hipLaunchKernelGGL((k_walk32<false, true>), g4, b4, 0, c->stream, RB_W32_ARGS);
  else
    hipLaunchKernelGGL((k_walk32<false, false>), g4, b4, 0, c->stream, RB_W32_ARGS);
#undef RB_W32_ARGS
  return hipGetLastError();
}
