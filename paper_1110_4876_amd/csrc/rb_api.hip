// rb_api.hip -- host side of librb: the C ABI of include/rb.h, context and
// workspace management, the per-call kernel sequences and error reporting.
//
// Host-side time arithmetic (step times, shear offsets) is written as the
// plain FP64 expressions and compiled without contraction, so that the
// ghost offsets of every step are reproducible from (t, dt, k) alone.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "rb_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define RB_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return fail(RB_EHIP, "%s: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                      \
  } while (0)

template <class T>
int dalloc(rb_ctx *c, T **ptr, size_t count) {
  *ptr = nullptr;
  size_t bytes = count * sizeof(T);
  if (bytes == 0) bytes = 256;
  void *v = nullptr;
  if (hipMalloc(&v, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(RB_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
  }
  c->allocs.push_back(v);
  *ptr = (T *)v;
  return RB_OK;
}

#define RB_TRY(expr)          \
  do {                        \
    int r_ = (expr);          \
    if (r_ != RB_OK) return r_; \
  } while (0)

// layout uploads are rare: copy and wait, so host vectors may change freely
int upload_sync(rb_ctx *c, void *dst, const void *src, size_t bytes) {
  if (bytes == 0) return RB_OK;
  RB_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
  RB_HIP(hipStreamSynchronize(c->stream));
  return RB_OK;
}

// root boxes along axis a (Sect. 2.3): n_root[a], 0 meaning 1
int n_root_of(const rb_params &p, int a) { return p.n_root[a] > 1 ? p.n_root[a] : 1; }

// octree levels above the root boxes: the smallest D with 2^D >= every n_root
uint32_t virtual_levels(const rb_params &p) {
  int m = std::max(n_root_of(p, 0), std::max(n_root_of(p, 1), n_root_of(p, 2)));
  uint32_t D = 0;
  while ((1 << D) < m) ++D;
  return D;
}

bool is_forest(const rb_params &p) { return virtual_levels(p) > 0 || n_root_of(p, 0) > 1 ||
                                            n_root_of(p, 1) > 1 || n_root_of(p, 2) > 1; }

int n_images(const rb_params &p) {
  if (p.boundary == RB_OPEN) return 1;
  return (2 * p.n_ghost[0] + 1) * (2 * p.n_ghost[1] + 1);
}

int validate(const rb_params *p) {
  if (!p) return fail(RB_EINVAL, "null parameters");
  if (!(p->G >= 0.0) || !isfinite(p->G)) return fail(RB_EINVAL, "G must be finite and >= 0");
  if (!(p->softening >= 0.0) || !isfinite(p->softening))
    return fail(RB_EINVAL, "softening must be finite and >= 0");
  if (!(p->theta >= 0.0) || !isfinite(p->theta))
    return fail(RB_EINVAL, "theta must be finite and >= 0");
  if (p->leaf_size < 1 || p->leaf_size > 32) return fail(RB_EINVAL, "leaf_size must be 1..32");
  if (p->group_size != 16 && p->group_size != 32 && p->group_size != 64)
    return fail(RB_EINVAL, "group_size must be 16, 32 or 64");
  if (p->boundary < RB_OPEN || p->boundary > RB_SHEAR) return fail(RB_EINVAL, "bad boundary");
  if (p->drift < RB_DRIFT_LEAPFROG || p->drift > RB_DRIFT_EPICYCLE)
    return fail(RB_EINVAL, "bad drift");
  if (p->precision < RB_FP64 || p->precision > RB_FP32_MIXED)
    return fail(RB_EINVAL, "bad precision");
  if (p->boundary != RB_OPEN) {
    if (p->n_ghost[0] < 0 || p->n_ghost[1] < 0) return fail(RB_EINVAL, "n_ghost must be >= 0");
    if (p->n_ghost[0] > 2 || p->n_ghost[1] > 2)
      return fail(RB_EUNSUPPORTED, "at most two ghost rings per axis");
  }
  if (p->drift == RB_DRIFT_EPICYCLE &&
      (!(p->omega > 0.0) || !(p->omega_z > 0.0) || !isfinite(p->omega) || !isfinite(p->omega_z)))
    return fail(RB_EINVAL, "epicycle drift needs omega > 0 and omega_z > 0");
  if (p->boundary == RB_SHEAR && !(p->omega >= 0.0)) return fail(RB_EINVAL, "bad omega");
  if (p->node_factor != 0.0 && !(p->node_factor >= 1.5))
    return fail(RB_EINVAL, "node_factor must be 0 or >= 1.5");
  if (p->walk_waves != 0 && p->walk_waves != 1 && p->walk_waves != 2 && p->walk_waves != 4)
    return fail(RB_EINVAL, "walk_waves must be 0, 1, 2 or 4");
  if (p->moments_level_log2 != 0 && (p->moments_level_log2 < 6 || p->moments_level_log2 > 31))
    return fail(RB_EINVAL, "moments_level_log2 must be 0 or 6..31");
  if (p->walk64_schedule < 0 || p->walk64_schedule > 3)
    return fail(RB_EINVAL, "walk64_schedule must be 0, 1, 2 or 3");
  if (p->reuse_topology != 0 && p->reuse_topology != 1)
    return fail(RB_EINVAL, "reuse_topology must be 0 or 1");
  for (int a = 0; a < 3; ++a)
    if (p->n_root[a] < 0 || p->n_root[a] > 256) return fail(RB_EINVAL, "n_root must be 0..256");
  return RB_OK;
}

int validate_box(const rb_params *p, double W, const double *x0) {
  if (!(W > 0.0) || !isfinite(W)) return fail(RB_EINVAL, "box_size must be finite and > 0");
  for (int a = 0; a < 3; ++a)
    if (!isfinite(x0[a])) return fail(RB_EINVAL, "box_min must be finite");
  if (p->boundary == RB_SHEAR && x0[0] != -0.5 * ((double)n_root_of(*p, 0) * W))
    return fail(RB_EINVAL, "shear boundaries need box_min[0] = -n_root[0] box_size / 2");
  return RB_OK;
}

// shear offset of the ghost boxes: the domain copy at +Lx slides by
// -(3/2) omega Lx t, folded into [-Ly/2, Ly/2]
double shear_offset(const rb_params &p, double Lx, double Ly, double t) {
  if (p.boundary != RB_SHEAR) return 0.0;
  return remainder(1.5 * p.omega * Lx * t, Ly);
}

// One walk work item per (group, image) pair, or per group with all its
// images, and the FP64 walk's schedule.  The FP64 walk is split by the
// subtrees below the root (schedule 3) whenever the accumulators allow it,
// taking all images per item: measured faster than one wave per 64
// particles (schedule 2) from 10^3 to 10^7 particles (2.6x at 50,000, 11%
// at 10^6, 1-2% above 4·10^6).  Otherwise schedule 2, or per-lane walks
// (schedule 1, with a split by image) when the 64-particle items would
// leave the chip idle.  The grouped FP32 walk already draws from a device
// queue and splits only on request.
void set_split(rb_ctx *c) {
  const uint32_t n_items = (uint32_t)c->h_items64.size();
  const bool fp64 = c->p.precision == RB_FP64;
  int mode = c->p.walk64_schedule;
  if (mode == 0) {
    const uint32_t units = n_items * (uint32_t)c->n_img;
    if (c->acc_sets >= RB_WALK64_PARTS) mode = 3;
    else mode = units >= RB_WALK64_SHARED_MIN ? 2 : 1;
  }
  const int sp = c->p.split_images;
  if (c->n_img <= 1 || sp == 0) c->img_split = 0;
  else if (sp == 1) c->img_split = 1;
  else c->img_split = (fp64 && mode != 3 && n_items < 16384) ? 1 : 0;
  // parts need an accumulator set each (d_acc is sized at creation)
  const int per = c->img_split ? c->n_img : 1;
  int parts = (n_items < RB_WALK64_PARTS2_MAX_ITEMS) ? RB_WALK64_PARTS2 : RB_WALK64_PARTS;
  if (per * parts > c->acc_sets) parts = RB_WALK64_PARTS;
  if (mode == 3 && per * parts > c->acc_sets) mode = 2;
  c->walk64_mode = mode;
  c->walk_parts = (fp64 && mode == 3) ? parts : 1;
}

// tiles of RB_TILE slots inside each patch; walk items of `g` slots
int build_layout(rb_ctx *c) {
  const uint32_t P = c->P;
  c->lcp_stale = true;
  c->h_tile_start.clear(); c->h_tile_end.clear(); c->h_tile_patch.clear();
  c->h_patch_tile0.assign(P + 1, 0);
  c->max_tiles_per_patch = 0;
  // topology: about 1024 tiles over the whole system (one wave each),
  // 64..512 slots (512-slot tiles beat 1024 on 8.9M slots: more waves,
  // 0.43 -> 0.41 ms for the three topology kernels)
  {
    const uint64_t n = c->h_starts[P];
    uint32_t t = RB_TILE_MIN;
    while (t < RB_TILE_MAX && (uint64_t)t * 1024 < n) t <<= 1;
    c->tile = t;
  }
  for (uint32_t p = 0; p < P; ++p) {
    c->h_patch_tile0[p] = (uint32_t)c->h_tile_start.size();
    const uint32_t s0 = c->h_starts[p], s1 = c->h_starts[p + 1];
    uint32_t nt = 0;
    for (uint32_t s = s0; s < s1; s += c->tile) {
      c->h_tile_start.push_back(s);
      c->h_tile_end.push_back(std::min<uint32_t>(s + c->tile, s1));
      c->h_tile_patch.push_back(p);
      ++nt;
    }
    c->max_tiles_per_patch = std::max(c->max_tiles_per_patch, nt);
  }
  c->h_patch_tile0[P] = (uint32_t)c->h_tile_start.size();
  c->n_tiles = (uint32_t)c->h_tile_start.size();
  // systems (or batches) whose patches all hold at most 2^18 slots use the
  // bucket sort; larger ones the look-back radix sort, tiles of 256 x R
  // slots per 256-thread block, R growing with the system so that large
  // sorts use fewer, fuller tiles
  {
    const uint64_t n = c->h_starts[P];
    uint64_t largest = 0;
    for (uint32_t p = 0; p < P; ++p)
      largest = std::max<uint64_t>(largest, c->h_starts[p + 1] - c->h_starts[p]);
    c->sort_small = largest <= c->small_sort_max;
    c->sort_rows = n < (1u << 18) ? 1 : n < (1u << 19) ? 2 : n < (1u << 20) ? 4 : 8;
    const uint32_t st = c->sort_small ? 256u : 256u * (uint32_t)c->sort_rows;
    c->stile = st;
    c->h_stile_start.clear(); c->h_stile_end.clear(); c->h_stile_patch.clear();
    c->h_spatch_tile0.assign(P + 1, 0);
    for (uint32_t p = 0; p < P; ++p) {
      c->h_spatch_tile0[p] = (uint32_t)c->h_stile_start.size();
      const uint32_t s0 = c->h_starts[p], s1 = c->h_starts[p + 1];
      for (uint32_t s = s0; s < s1; s += st) {
        c->h_stile_start.push_back(s);
        c->h_stile_end.push_back(std::min<uint32_t>(s + st, s1));
        c->h_stile_patch.push_back(p);
      }
    }
    c->h_spatch_tile0[P] = (uint32_t)c->h_stile_start.size();
    c->n_stiles = (uint32_t)c->h_stile_start.size();
    // histogram blocks: about 256 of them, at least 2048 keys each
    {
      const uint64_t per = std::max<uint64_t>(2048, (n + 255) / 256);
      c->sort_hist_tiles = (uint32_t)std::max<uint64_t>(1, per / st);
    }
    const size_t ns = c->n_stiles;
    RB_TRY(upload_sync(c, c->d_stile_start, c->h_stile_start.data(), ns * 4));
    RB_TRY(upload_sync(c, c->d_stile_end, c->h_stile_end.data(), ns * 4));
    RB_TRY(upload_sync(c, c->d_stile_patch, c->h_stile_patch.data(), ns * 4));
    RB_TRY(upload_sync(c, c->d_spatch_tile0, c->h_spatch_tile0.data(), (P + 1) * 4));
  }
  const size_t nt = c->n_tiles;
  RB_TRY(upload_sync(c, c->d_tile_start, c->h_tile_start.data(), nt * 4));
  RB_TRY(upload_sync(c, c->d_tile_end, c->h_tile_end.data(), nt * 4));
  RB_TRY(upload_sync(c, c->d_tile_patch, c->h_tile_patch.data(), nt * 4));
  RB_TRY(upload_sync(c, c->d_patch_tile0, c->h_patch_tile0.data(), (P + 1) * 4));
  RB_TRY(upload_sync(c, c->d_starts, c->h_starts.data(), (P + 1) * 4));
  RB_TRY(upload_sync(c, c->d_patch, c->h_patch.data(), P * sizeof(PatchInfo)));

  // walk items, patches in descending cost order (n log n)
  std::vector<uint32_t> order(P);
  for (uint32_t p = 0; p < P; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
    return c->h_patch[a].n > c->h_patch[b].n;
  });
  auto make_items = [&](uint32_t g, std::vector<WalkItem> &out) {
    out.clear();
    for (uint32_t p : order) {
      const uint32_t s0 = c->h_starts[p], s1 = c->h_starts[p + 1];
      for (uint32_t s = s0; s < s1; s += g) out.push_back({s, std::min<uint32_t>(s + g, s1), p, 0});
    }
  };
  make_items(64, c->h_items64);
  if (c->h_items64.size() > c->cap / 16 + 2 * P + 8)
    return fail(RB_ECAPACITY, "walk item table overflow");
  RB_TRY(upload_sync(c, c->d_items64, c->h_items64.data(), c->h_items64.size() * sizeof(WalkItem)));
  set_split(c);
  c->graph_key = -1;
  return RB_OK;
}

int init_ctx(rb_ctx *c, const rb_params *p, uint32_t P, const int64_t *off, const double *W,
             const double *x0, void *stream) {
  c->p = *p;
  if (c->p.omega_z == 0.0) c->p.omega_z = c->p.omega;
  c->stream = (hipStream_t)stream;
  RB_HIP(hipGetDevice(&c->device));
  c->P = P;
  c->n_img = n_images(c->p);
  c->h_starts.assign(P + 1, 0);
  c->h_patch.resize(P);
  for (uint32_t k = 0; k < P; ++k) {
    PatchInfo &pi = c->h_patch[k];
    // W[k] is the root box side; keys quantise the cube of side W[k] 2^D
    const uint32_t D = virtual_levels(c->p);
    pi.nvirt = D;
    pi.W = ldexp(W[k], (int)D);
    for (int a = 0; a < 3; ++a) pi.x0[a] = x0[3 * k + a];
    pi.S = (double)(1u << (RB_DEPTH - D)) / W[k];
    for (int a = 0; a < 3; ++a) {
      pi.L[a] = (double)n_root_of(c->p, a) * W[k];
      pi.qtop[a] = (double)n_root_of(c->p, a) * ldexp(1.0, RB_DEPTH - (int)D) - 1.0;
    }
    pi.start = (uint32_t)off[k];
    pi.n = (uint32_t)(off[k + 1] - off[k]);
    pi.n_active = pi.n;
    c->h_starts[k] = (uint32_t)off[k];
  }
  c->h_starts[P] = (uint32_t)off[P];
  const uint64_t cap = c->cap;
  const double nf = c->p.node_factor > 0.0 ? c->p.node_factor : 3.0;
  c->node_cap = (uint64_t)(nf * (double)cap) + 64 * (uint64_t)P + 64;
  if (c->node_cap > 0xFFFFFFF0ull) return fail(RB_ECAPACITY, "node capacity beyond 32-bit indices");
  const uint64_t max_tiles = cap / RB_TILE_MIN + P + 1;
  const uint64_t max_items = cap / 16 + 2 * (uint64_t)P + 8;
  RB_TRY(dalloc(c, &c->d_patch, P));
  RB_TRY(dalloc(c, &c->d_starts, P + 1));
  RB_TRY(dalloc(c, &c->d_nlive, P));
  RB_TRY(dalloc(c, &c->d_root, P));
  RB_TRY(dalloc(c, &c->d_tile_start, max_tiles));
  RB_TRY(dalloc(c, &c->d_tile_end, max_tiles));
  RB_TRY(dalloc(c, &c->d_tile_patch, max_tiles));
  RB_TRY(dalloc(c, &c->d_patch_tile0, P + 1));
  for (int b = 0; b < 2; ++b) {
    RB_TRY(dalloc(c, &c->d_key[b], cap));
    RB_TRY(dalloc(c, &c->d_idx[b], cap));
    for (int f = 0; f < 7; ++f) RB_TRY(dalloc(c, &c->d_px[b][f], cap));
    RB_TRY(dalloc(c, &c->d_orig[b], cap));
  }
  // sort tiles: at least 256 slots each, at most one partial tile per patch
  const uint64_t max_stiles = cap / 256 + P + 1;
  RB_TRY(dalloc(c, &c->d_stile_start, max_stiles));
  RB_TRY(dalloc(c, &c->d_stile_end, max_stiles));
  RB_TRY(dalloc(c, &c->d_stile_patch, max_stiles));
  RB_TRY(dalloc(c, &c->d_spatch_tile0, P + 1));
  RB_TRY(dalloc(c, &c->d_stot, 2 * 2048 * (uint64_t)P));
  RB_TRY(dalloc(c, &c->d_sdesc, 256 * max_stiles));
  RB_TRY(dalloc(c, &c->d_sctl, 4));
  // totals start at zero (each sort clears the buffer the next one counts
  // into); look-back words start with no valid flag
  RB_HIP(hipMemsetAsync(c->d_stot, 0, 4 * 2 * 2048 * (size_t)P, c->stream));
  RB_HIP(hipMemsetAsync(c->d_sdesc, 0, 8 * 256 * max_stiles, c->stream));
  RB_HIP(hipMemsetAsync(c->d_sctl, 0, 16, c->stream));
  // bucket sort: patches of up to 2^18 slots (segments: at most one per
  // slot, plus one per patch)
  c->small_sort_max = std::min<uint64_t>(cap, 1u << 18);
  RB_TRY(dalloc(c, &c->d_bcnt, (uint64_t)BS_NB * P));
  RB_TRY(dalloc(c, &c->d_bcur, (uint64_t)BS_NB * P));
  RB_TRY(dalloc(c, &c->d_bseg, cap + P + 1));
  RB_TRY(dalloc(c, &c->d_bctl, 4));
  RB_HIP(hipMemsetAsync(c->d_bcnt, 0, 4 * (size_t)BS_NB * P, c->stream));
  RB_HIP(hipMemsetAsync(c->d_bctl, 0, 16, c->stream));
  RB_TRY(dalloc(c, &c->d_msrc, cap));
  RB_TRY(dalloc(c, &c->d_lcp, cap));
  RB_TRY(dalloc(c, &c->d_cnt, 2 * RB_NLEV * max_tiles));
  RB_TRY(dalloc(c, &c->d_lev_tot, 2 * RB_NLEV));
  RB_TRY(dalloc(c, &c->d_lev_off, RB_NLEV + 2));
  const uint64_t nc = c->node_cap;
  RB_TRY(dalloc(c, &c->d_nfirst, nc));
  RB_TRY(dalloc(c, &c->d_nlast, nc));
  RB_TRY(dalloc(c, &c->d_nchild, nc));
  RB_TRY(dalloc(c, &c->d_nlastchild, nc));
  RB_TRY(dalloc(c, &c->d_nskip, nc));
  RB_TRY(dalloc(c, &c->d_nlevel, nc));
  RB_TRY(dalloc(c, &c->d_nleaf, nc));
  RB_TRY(dalloc(c, &c->d_csr, cap));
  RB_TRY(dalloc(c, &c->d_start_ids, nc));
  RB_TRY(dalloc(c, &c->d_link, nc));
  RB_TRY(dalloc(c, &c->d_mcom, nc));
  RB_TRY(dalloc(c, &c->d_S, 3 * nc));
  RB_TRY(dalloc(c, &c->d_Q, 6 * nc));
  RB_TRY(dalloc(c, &c->d_wnode, nc));
  RB_TRY(dalloc(c, &c->d_items64, max_items));
  RB_TRY(dalloc(c, &c->d_witems, cap));
  RB_TRY(dalloc(c, &c->d_witems_mid, cap));
  RB_TRY(dalloc(c, &c->d_gctr, 8));
  RB_TRY(dalloc(c, &c->d_large, nc));
  RB_TRY(dalloc(c, &c->d_bottom, nc));
  RB_TRY(dalloc(c, &c->d_large_cnt, RB_LARGE_SLOTS));
  RB_HIP(hipMemsetAsync(c->d_large_cnt, 0, 4 * RB_LARGE_SLOTS, c->stream));
  RB_HIP(hipMemsetAsync(c->d_gctr, 0, 32, c->stream));
  // walk results: a set of 3 * cap doubles per image (split walks) and per
  // part of the FP64 walk's schedule 3; the first of these that costs at
  // most 2 GiB more than the images' own: 64 parts of split walks, 64 parts
  // of whole walks, 8 parts of split walks, 8 parts of whole walks
  {
    const uint64_t set_bytes = 3ull * cap * sizeof(double), budget = 2ull << 30;
    const uint64_t ni = (uint64_t)c->n_img;
    const uint64_t cand[4] = {ni * RB_WALK64_PARTS2, std::max<uint64_t>(ni, RB_WALK64_PARTS2),
                              ni * RB_WALK64_PARTS, std::max<uint64_t>(ni, RB_WALK64_PARTS)};
    c->acc_sets = (int)ni;
    for (uint64_t k : cand)
      if ((k - ni) * set_bytes <= budget) { c->acc_sets = (int)k; break; }
  }
  RB_TRY(dalloc(c, &c->d_acc, (uint64_t)c->acc_sets * 3 * cap));
  RB_TRY(dalloc(c, &c->d_w64_ord, RB_W64_ORD_WORDS));
  RB_HIP(hipMemsetAsync(c->d_w64_ord, 0, 4 * (size_t)RB_W64_ORD_WORDS, c->stream));
  {
    static_assert(sizeof(W64Ctl) <= 4 * RB_W64_COST_OFF, "control block");
    W64Ctl ctl{};
    ctl.epoch = 1;          // tags start at 0: no unit is listed
    ctl.thr = 0xFFFFFFFFu;  // nothing listed until a launch has measured costs
    RB_HIP(hipMemcpyAsync(c->d_w64_ord, &ctl, sizeof(ctl), hipMemcpyHostToDevice, c->stream));
    RB_HIP(hipStreamSynchronize(c->stream));
  }
  // per-call dynamic region: step counter (16 B), StepConst, schedule
  c->sched_cap = 1024;
  c->dyn_bytes = 256 + (size_t)(c->sched_cap + 1) * 2 * P * sizeof(double);
  RB_TRY(dalloc(c, &c->d_dyn, c->dyn_bytes));
  c->d_ctr = (uint32_t *)c->d_dyn;
  c->d_sc = (StepConst *)(c->d_dyn + 64);
  c->d_sched = (double *)(c->d_dyn + 256);
  RB_HIP(hipHostMalloc((void **)&c->h_dyn, c->dyn_bytes, hipHostMallocDefault));
  RB_HIP(hipEventCreateWithFlags(&c->dyn_ev, hipEventDisableTiming));
  RB_HIP(hipEventRecord(c->dyn_ev, c->stream));
  RB_TRY(dalloc(c, &c->d_err, 1));
  RB_TRY(dalloc(c, &c->d_stats, 8));
  RB_HIP(hipMemsetAsync(c->d_err, 0, 4, c->stream));
  RB_HIP(hipMemsetAsync(c->d_stats, 0, 64, c->stream));
  RB_HIP(hipMemsetAsync(c->d_dyn, 0, c->dyn_bytes, c->stream));
  RB_HIP(hipMemsetAsync(c->d_nlive, 0, 4 * (size_t)P, c->stream));
  RB_HIP(hipMemsetAsync(c->d_lev_off, 0, 4 * (RB_NLEV + 2), c->stream));
  for (int k = 0; k < 16; ++k) RB_HIP(hipEventCreate(&c->ev[k]));
  RB_TRY(build_layout(c));
  RB_HIP(hipStreamSynchronize(c->stream));
  return RB_OK;
}

void free_ctx(rb_ctx *c) {
  if (!c) return;
  if (c->h_dyn) (void)hipHostFree(c->h_dyn);
  if (c->h_cpin) (void)hipHostFree(c->h_cpin);
  if (c->dyn_ev) (void)hipEventDestroy(c->dyn_ev);
  for (int k = 0; k < 2; ++k) {
    if (c->graph_exec[k]) (void)hipGraphExecDestroy(c->graph_exec[k]);
    if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
  }
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (int k = 0; k < 16; ++k)
    if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
  for (void *v : c->allocs) (void)hipFree(v);
  delete c;
}

int check_particles(const rb_particles *p, bool velocities) {
  if (!p || !p->x || !p->y || !p->z || !p->m) return fail(RB_EINVAL, "null particle array");
  if (velocities && (!p->vx || !p->vy || !p->vz)) return fail(RB_EINVAL, "null velocity array");
  return RB_OK;
}

// single-system contexts accept any n <= capacity; re-layout when n or
// n_active change
int set_single_n(rb_ctx *c, int64_t n, int64_t n_active) {
  if (n < 0 || (uint64_t)n > c->cap) return fail(RB_EINVAL, "n = %lld outside [0, capacity]", (long long)n);
  if (n_active < 0) return fail(RB_EINVAL, "n_active must be >= 0");
  uint32_t na = (uint32_t)std::min<int64_t>(n_active, n);
  if (c->batch) {
    if ((uint64_t)n != c->h_starts[c->P]) return fail(RB_EINVAL, "batch context: n must equal the total");
    return RB_OK;
  }
  if (c->h_starts[1] != (uint32_t)n) {
    c->h_starts[1] = (uint32_t)n;
    c->h_patch[0].n = (uint32_t)n;
    c->h_patch[0].n_active = na;
    RB_TRY(build_layout(c));
  } else if (c->h_patch[0].n_active != na) {
    c->h_patch[0].n_active = na;
    RB_TRY(upload_sync(c, c->d_patch, c->h_patch.data(), sizeof(PatchInfo)));
  }
  return RB_OK;
}

// schedule for `nsteps` steps from t (or a single force evaluation at t when
// nsteps == 0): s_half = offset at t_k + dt/2, s_end = offset at t_{k+1}
int upload_schedule(rb_ctx *c, double t, double dt, int32_t nsteps) {
#pragma clang fp contract(off)
  const uint32_t P = c->P;
  const uint32_t rows = nsteps > 0 ? (uint32_t)nsteps : 1u;
  // the staging buffer is reused: wait for the previous upload to land
  RB_HIP(hipEventSynchronize(c->dyn_ev));
  uint32_t *ctr = (uint32_t *)c->h_dyn;
  ctr[0] = 0u; ctr[1] = 0u; ctr[2] = rows; ctr[3] = 0u;
  // words 6, 7: the steps' keep-the-tree flags (raised: rebuild); the first
  // step of a call rebuilds when the tree buffers were last written elsewhere
  ctr[6] = c->lcp_stale ? 1u : 0u;
  ctr[7] = 0u;
  // words 4-5: the collision seed of the schedule's first step
  memcpy(c->h_dyn + 16, &c->chunk_seed, 8);
  StepConst *sc = (StepConst *)(c->h_dyn + 64);
  double *sched = (double *)(c->h_dyn + 256);
  const double half = 0.5 * dt;
  for (uint32_t k = 0; k < rows; ++k) {
    for (uint32_t p = 0; p < P; ++p) {
      const double Lx = c->h_patch[p].L[0], Ly = c->h_patch[p].L[1];
      if (nsteps > 0) {
        const double tk = t + (double)k * dt;
        const double th = tk + half;
        const double te = t + (double)(k + 1) * dt;
        sched[(size_t)k * 2 * P + p] = shear_offset(c->p, Lx, Ly, th);
        sched[(size_t)k * 2 * P + P + p] = shear_offset(c->p, Lx, Ly, te);
      } else {
        sched[p] = shear_offset(c->p, Lx, Ly, t);
        sched[P + p] = sched[p];
      }
    }
  }
  sc->half = half;
  sc->dt = dt;
  sc->omega = c->p.omega;
  sc->omega_z = c->p.omega_z;
  sc->c = cos(c->p.omega * half);
  sc->sn = sin(c->p.omega * half);
  sc->cz = cos(c->p.omega_z * half);
  sc->sz = sin(c->p.omega_z * half);
  sc->jump = 1.5 * c->p.omega;
  const size_t bytes = 256 + (size_t)rows * 2 * P * sizeof(double);
  RB_HIP(hipMemcpyAsync(c->d_dyn, c->h_dyn, bytes, hipMemcpyHostToDevice, c->stream));
  RB_HIP(hipEventRecord(c->dyn_ev, c->stream));
  return RB_OK;
}

// ---- phase timing (profile = 1): event pairs per phase, resolved at sync ----
struct EvPool {
  std::vector<hipEvent_t> free_ev;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  hipEvent_t open_ev[16] = {};  // begin event of each phase (phases nest: total > others)
};

}  // namespace

// event pool per context, kept outside the struct to keep rb_internal.h lean
#include <map>
namespace {
std::map<rb_ctx *, EvPool> g_pools;

hipEvent_t get_event(rb_ctx *c) {
  EvPool &pl = g_pools[c];
  if (!pl.free_ev.empty()) {
    hipEvent_t e = pl.free_ev.back();
    pl.free_ev.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int mark(rb_ctx *c, int phase, bool begin) {
  // bit 0: every phase; bit 2: the walk and the collision search only
  // (lightest timing of a run)
  if (!(c->p.profile & 1) && !((c->p.profile & 4) && (phase == 5 || phase == 10)))
    return RB_OK;
  EvPool &pl = g_pools[c];
  hipEvent_t e = get_event(c);
  if (!e) return fail(RB_EHIP, "hipEventCreate failed");
  const hipError_t r = hipEventRecord(e, c->stream);
  if (r != hipSuccess) {
    pl.free_ev.push_back(e);
    return fail(RB_EHIP, "hipEventRecord: %s", hipGetErrorString(r));
  }
  hipEvent_t &open = pl.open_ev[phase & 15];
  if (begin) {
    if (open) pl.free_ev.push_back(open);  // an unmatched begin: reuse its event
    open = e;
  } else if (open) {
    pl.pending.push_back({phase, {open, e}});
    open = nullptr;
  } else {
    pl.free_ev.push_back(e);  // an end without a begin times nothing
  }
  return RB_OK;
}

void resolve_timers(rb_ctx *c) {
  EvPool &pl = g_pools[c];
  for (auto &q : pl.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, q.second.first, q.second.second) == hipSuccess &&
        q.first >= 0 && q.first < 16) {
      c->phase_ms[q.first] += ms;
      c->phase_calls[q.first] += 1;
    }
    pl.free_ev.push_back(q.second.first);
    pl.free_ev.push_back(q.second.second);
  }
  pl.pending.clear();
}

void drop_pool(rb_ctx *c) {
  auto it = g_pools.find(c);
  if (it == g_pools.end()) return;
  for (auto &q : it->second.pending) {
    (void)hipEventDestroy(q.second.first);
    (void)hipEventDestroy(q.second.second);
  }
  for (hipEvent_t e : it->second.free_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : it->second.open_ev)
    if (e) (void)hipEventDestroy(e);
  g_pools.erase(it);
}

enum { PH_KEYS = 0, PH_SORT, PH_PERMUTE, PH_TOPO, PH_MOMENTS, PH_WALK, PH_POST, PH_DIRECT,
       PH_COLLIDE, PH_TOTAL, PH_CSEARCH, PH_COUNT };
const char *g_phase_names[] = {"keys", "sort", "permute", "topology", "moments", "walk",
                               "kick_drift", "direct", "collide", "total", "coll_search"};

#define RB_LAUNCH(expr)                                                              \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(RB_EHIP, "%s: %s", #expr, hipGetErrorString(e_));                  \
  } while (0)

#define RB_PHASE(ph, expr)         \
  do {                             \
    RB_TRY(mark(c, ph, true));     \
    RB_LAUNCH(expr);               \
    RB_TRY(mark(c, ph, false));    \
  } while (0)

int build_tree(rb_ctx *c, const rb_particles *p) {
  RB_PHASE(PH_KEYS, launch_keys(c, p->x, p->y, p->z, 0.0));
  RB_PHASE(PH_SORT, launch_sort(c));
  RB_PHASE(PH_PERMUTE, launch_permute_gravity(c, p->x, p->y, p->z, p->m, 0));
  RB_PHASE(PH_TOPO, launch_topology(c));
  RB_PHASE(PH_MOMENTS, launch_moments(c, c->d_px[0][0], c->d_px[0][1], c->d_px[0][2]));
  c->fp64_partial = false;
  c->lcp_stale = true;
  return RB_OK;
}

// walk on the sorted state in buffer `buf`; `slot` selects the step-counter
// entry holding this step's index
int walk(rb_ctx *c, int buf, int slot) {
  double *const *b = c->d_px[buf];
  if (c->p.precision == RB_FP64) {
    RB_PHASE(PH_WALK, launch_walk64(c, b[0], b[1], b[2], slot));
  } else {
    RB_PHASE(PH_WALK, launch_walk32(c, b[0], b[1], b[2], slot));
  }
  return RB_OK;
}

int report_device_errors(rb_ctx *c) {
  uint32_t err = 0;
  RB_HIP(hipStreamSynchronize(c->stream));
  RB_HIP(hipMemcpy(&err, c->d_err, 4, hipMemcpyDeviceToHost));
  if (err) {
    RB_HIP(hipMemset(c->d_err, 0, 4));
    if (err & RB_ERR_NODES)
      return fail(RB_ECAPACITY, "node capacity (%llu) exceeded; raise node_factor",
                  (unsigned long long)c->node_cap);
    if (err & RB_ERR_STACK) return fail(RB_ECAPACITY, "FP32 walk traversal stack overflow");
    if (err & RB_ERR_TREE) return fail(RB_ECAPACITY, "inconsistent tree links (internal error)");
    if (err & RB_ERR_SORT) return fail(RB_EHIP, "radix sort look-back timed out (internal error)");
    if (err & RB_ERR_COLL) return fail(RB_ECAPACITY, "collision queue capacity exceeded");
    if (err & RB_ERR_INDEX) return fail(RB_EINVAL, "a target index lies outside [0, n)");
    if (err & RB_ERR_OUTSIDE)
      return fail(RB_EOUTSIDE, "a particle lies outside a periodic / shear box axis");
  }
  resolve_timers(c);
  return RB_OK;
}

// the kernels of one step with the state in buffer src
int step_kernels(rb_ctx *c, int src) {
  const int dst = 1 - src;
  RB_PHASE(PH_SORT, launch_sort(c));
  RB_PHASE(PH_PERMUTE, launch_permute_state(c, src, dst));
  // with reuse_topology the step keeps the last tree when no particle left
  // its cell: the check leaves the step's flag clear, and the topology and
  // work-item kernels return at once (Sect. 4.2's tree kept across steps)
  const uint32_t *reuse = nullptr;
  if (c->p.reuse_topology) {
    uint32_t *flag = c->d_ctr + 6 + src;
    RB_PHASE(PH_TOPO, launch_topo_check(c, flag));
    reuse = flag;
  }
  RB_PHASE(PH_TOPO, launch_topology(c, reuse));
  RB_PHASE(PH_MOMENTS, launch_moments(c, c->d_px[dst][0], c->d_px[dst][1], c->d_px[dst][2],
                                      c->p.precision == RB_FP32_MIXED, reuse));
  c->fp64_partial = c->p.precision == RB_FP32_MIXED;
  if (c->coll_on) RB_PHASE(PH_COLLIDE, launch_coll_step_prep(c, dst));
  RB_TRY(walk(c, dst, src));
  if (c->coll_on) {
    // collisions at the end of the step, between the second drift and the
    // next step's first drift
    RB_PHASE(PH_POST, launch_post(c, dst, src, 1));
    RB_PHASE(PH_CSEARCH, launch_coll_step_search(c, dst, src));
    RB_PHASE(PH_COLLIDE, launch_coll_step_rounds(c, dst, src));
    RB_PHASE(PH_POST, launch_post(c, dst, src, 2));
  } else {
    RB_PHASE(PH_POST, launch_post(c, dst, src));
  }
  return RB_OK;
}

void drop_graphs(rb_ctx *c) {
  for (int k = 0; k < 2; ++k) {
    if (c->graph_exec[k]) (void)hipGraphExecDestroy(c->graph_exec[k]);
    if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
    c->graph_exec[k] = nullptr;
    c->graph[k] = nullptr;
  }
}

// Capture the two step graphs.  Every argument of the step kernels is fixed
// for a context and buffer parity; the step index, times and shear offsets
// are read from device memory, so one graph serves every step.  Timers are
// not captured.
// Capture happens on a private non-blocking stream (the caller's stream may
// be the null stream, which cannot be captured); the graphs are then
// launched on the context's stream.
int capture_graphs(rb_ctx *c) {
  drop_graphs(c);
  if (!c->cap_stream) RB_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  const int32_t prof = c->p.profile;
  hipStream_t saved = c->stream;
  c->p.profile &= ~5;
  c->stream = c->cap_stream;
  int r = RB_OK;
  for (int src = 0; src < 2 && r == RB_OK; ++src) {
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { r = fail(RB_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e)); break; }
    r = step_kernels(c, src);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->stream, &g);  // always ends the capture
    if (r == RB_OK && e != hipSuccess) r = fail(RB_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    if (r != RB_OK) { if (g) (void)hipGraphDestroy(g); break; }
    c->graph[src] = g;
    e = hipGraphInstantiate(&c->graph_exec[src], g, nullptr, nullptr, 0);
    if (e != hipSuccess) r = fail(RB_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  c->stream = saved;
  c->p.profile = prof;
  if (r != RB_OK) { drop_graphs(c); return r; }
  c->graph_key = 1;
  return RB_OK;
}

int run_step(rb_ctx *c, rb_particles *p, double t, double dt, int32_t nsteps) {
  if (nsteps <= 0) return nsteps == 0 ? RB_OK : fail(RB_EINVAL, "nsteps must be >= 0");
  if (!isfinite(t) || !isfinite(dt)) return fail(RB_EINVAL, "t and dt must be finite");
  const bool graphs = c->p.use_graph != 0;
  if (graphs && c->graph_key < 0) RB_TRY(capture_graphs(c));
  int32_t done = 0;
  while (done < nsteps) {
    const int32_t chunk = std::min<int32_t>(nsteps - done, (int32_t)c->sched_cap);
    const double t0 = t + (double)done * dt;
    c->chunk_seed = c->coll_seed + c->coll_steps;
    RB_TRY(upload_schedule(c, t0, dt, chunk));
    // the steps keep the prefix-level record current only when they use it
    c->lcp_stale = c->p.reuse_topology == 0;
    if (c->coll_on) c->coll_steps += (uint64_t)chunk;
    RB_TRY(mark(c, PH_TOTAL, true));
    RB_PHASE(PH_KEYS, launch_prologue(c, p));
    int src = 0;
    for (int32_t k = 0; k < chunk; ++k) {
      if (graphs) RB_HIP(hipGraphLaunch(c->graph_exec[src], c->stream));
      else RB_TRY(step_kernels(c, src));
      src = 1 - src;
    }
    RB_LAUNCH(launch_epilogue(c, p, src));
    RB_TRY(mark(c, PH_TOTAL, false));
    done += chunk;
  }
  return RB_OK;
}

}  // namespace

// ===========================================================================
// C ABI

extern "C" {

void rb_params_default(rb_params *p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->G = 1.0;
  p->softening = 0.0;
  p->theta = 0.5;
  p->quadrupole = 0;
  p->leaf_size = 1;
  p->group_size = 64;
  p->boundary = RB_OPEN;
  p->drift = RB_DRIFT_LEAPFROG;
  p->precision = RB_FP64;
  p->box_size = 128.0;
  p->box_min[0] = p->box_min[1] = p->box_min[2] = -64.0;
  p->split_images = -1;
}

int rb_create(rb_ctx **out, const rb_params *p, int64_t capacity, void *stream) {
  if (!out) return fail(RB_EINVAL, "null context pointer");
  *out = nullptr;
  RB_TRY(validate(p));
  RB_TRY(validate_box(p, p->box_size, p->box_min));
  if (capacity < 1 || capacity > 0x7FFFFFFFll) return fail(RB_EINVAL, "capacity must be 1..2^31-1");
  rb_ctx *c = new rb_ctx();
  c->cap = (uint64_t)capacity;
  int64_t off[2] = {0, 0};
  int r = init_ctx(c, p, 1, off, &p->box_size, p->box_min, stream);
  if (r != RB_OK) { drop_pool(c); free_ctx(c); return r; }
  *out = c;
  return RB_OK;
}

int rb_batch_create(rb_ctx **out, const rb_params *p, int32_t n_patch, const int64_t *offsets,
                    const double *box_size, const double *box_min, void *stream) {
  if (!out) return fail(RB_EINVAL, "null context pointer");
  *out = nullptr;
  RB_TRY(validate(p));
  if (is_forest(*p)) return fail(RB_EUNSUPPORTED, "batch patches are single root boxes");
  if (n_patch < 1 || !offsets || !box_size || !box_min)
    return fail(RB_EINVAL, "need n_patch >= 1 and non-null offsets / boxes");
  if (offsets[0] != 0) return fail(RB_EINVAL, "offsets[0] must be 0");
  for (int32_t k = 0; k < n_patch; ++k) {
    if (offsets[k + 1] < offsets[k]) return fail(RB_EINVAL, "offsets must be non-decreasing");
    RB_TRY(validate_box(p, box_size[k], box_min + 3 * k));
  }
  if (offsets[n_patch] < 1 || offsets[n_patch] > 0x7FFFFFFFll)
    return fail(RB_EINVAL, "total particle count must be 1..2^31-1");
  rb_ctx *c = new rb_ctx();
  c->batch = true;
  c->cap = (uint64_t)offsets[n_patch];
  int r = init_ctx(c, p, (uint32_t)n_patch, offsets, box_size, box_min, stream);
  if (r != RB_OK) { drop_pool(c); free_ctx(c); return r; }
  *out = c;
  return RB_OK;
}

int rb_destroy(rb_ctx *c) {
  if (!c) return RB_OK;
  (void)hipStreamSynchronize(c->stream);
  drop_pool(c);
  free_ctx(c);
  return RB_OK;
}

int rb_set_params(rb_ctx *c, const rb_params *p) {
  if (!c) return fail(RB_EINVAL, "null context");
  RB_TRY(validate(p));
  if (p->boundary != c->p.boundary || p->n_ghost[0] != c->p.n_ghost[0] ||
      p->n_ghost[1] != c->p.n_ghost[1] || p->drift != c->p.drift)
    return fail(RB_EINVAL, "boundary, ghost rings and drift are fixed at creation");
  const int old_group = c->p.group_size, old_split = c->p.split_images;
  const double nf = c->p.node_factor;
  rb_params q = *p;
  q.box_size = c->p.box_size;
  for (int a = 0; a < 3; ++a) q.box_min[a] = c->p.box_min[a];
  for (int a = 0; a < 3; ++a) q.n_root[a] = c->p.n_root[a];
  q.node_factor = nf;
  if (q.omega_z == 0.0) q.omega_z = q.omega;
  c->p = q;
  (void)old_group;
  (void)old_split;
  set_split(c);
  c->graph_key = -1;
  c->lcp_stale = true;
  return RB_OK;
}

int rb_tree_build(rb_ctx *c, const rb_particles *p, int64_t n, int64_t n_active) {
  if (!c) return fail(RB_EINVAL, "null context");
  RB_TRY(check_particles(p, false));
  RB_TRY(set_single_n(c, n, n_active));
  RB_TRY(upload_schedule(c, 0.0, 0.0, 0));
  return build_tree(c, p);
}

int rb_tree_info(rb_ctx *c, int64_t *n_nodes, int64_t *n_live) {
  if (!c) return fail(RB_EINVAL, "null context");
  RB_TRY(report_device_errors(c));
  uint32_t off[RB_NLEV + 1];
  RB_HIP(hipMemcpy(off, c->d_lev_off, sizeof(off), hipMemcpyDeviceToHost));
  std::vector<uint32_t> nl(c->P);
  RB_HIP(hipMemcpy(nl.data(), c->d_nlive, 4 * (size_t)c->P, hipMemcpyDeviceToHost));
  if (n_nodes) *n_nodes = off[RB_NLEV];
  if (n_live) {
    int64_t s = 0;
    for (uint32_t v : nl) s += v;
    *n_live = s;
  }
  return RB_OK;
}

int rb_tree_export(rb_ctx *c, int32_t patch, rb_tree_host *o) {
  if (!c || !o) return fail(RB_EINVAL, "null argument");
  if (patch < 0 || (uint32_t)patch >= c->P) return fail(RB_EINVAL, "patch out of range");
  if (c->fp64_partial)
    return fail(RB_EUNSUPPORTED,
                "the last tree has no complete FP64 moments (an FP32-mixed step or a "
                "collision search built it): call rb_tree_build first");
  RB_TRY(report_device_errors(c));
  uint32_t off[RB_NLEV + 1];
  RB_HIP(hipMemcpy(off, c->d_lev_off, sizeof(off), hipMemcpyDeviceToHost));
  const uint32_t nn = off[RB_NLEV];
  std::vector<uint32_t> nf(nn), nl(nn), nch(nn), nlc(nn), nsk(nn);
  std::vector<uint8_t> lev(nn), lf(nn);
  std::vector<double4> mc(nn);
  std::vector<double> Q(6 * (size_t)nn);
  RB_HIP(hipMemcpy(nf.data(), c->d_nfirst, 4 * (size_t)nn, hipMemcpyDeviceToHost));
  RB_HIP(hipMemcpy(nl.data(), c->d_nlast, 4 * (size_t)nn, hipMemcpyDeviceToHost));
  RB_HIP(hipMemcpy(nch.data(), c->d_nchild, 4 * (size_t)nn, hipMemcpyDeviceToHost));
  RB_HIP(hipMemcpy(nlc.data(), c->d_nlastchild, 4 * (size_t)nn, hipMemcpyDeviceToHost));
  RB_HIP(hipMemcpy(nsk.data(), c->d_nskip, 4 * (size_t)nn, hipMemcpyDeviceToHost));
  RB_HIP(hipMemcpy(lev.data(), c->d_nlevel, (size_t)nn, hipMemcpyDeviceToHost));
  RB_HIP(hipMemcpy(lf.data(), c->d_nleaf, (size_t)nn, hipMemcpyDeviceToHost));
  RB_HIP(hipMemcpy(mc.data(), c->d_mcom, sizeof(double4) * (size_t)nn, hipMemcpyDeviceToHost));
  RB_HIP(hipMemcpy(Q.data(), c->d_Q, 48 * (size_t)nn, hipMemcpyDeviceToHost));
  const uint32_t st = c->h_starts[patch], en = c->h_starts[patch + 1];
  uint32_t nlive = 0;
  RB_HIP(hipMemcpy(&nlive, c->d_nlive + patch, 4, hipMemcpyDeviceToHost));
  std::vector<uint64_t> keys(nlive);
  std::vector<uint32_t> orig(nlive);
  if (nlive) {
    RB_HIP(hipMemcpy(keys.data(), c->d_key[0] + st, 8 * (size_t)nlive, hipMemcpyDeviceToHost));
    RB_HIP(hipMemcpy(orig.data(), c->d_orig[0] + st, 4 * (size_t)nlive, hipMemcpyDeviceToHost));
  }
  // nodes of this patch in global (level, patch, prefix) order -> local ids
  std::vector<int64_t> local(nn, -1);
  int64_t k = 0;
  for (uint32_t id = 0; id < nn; ++id)
    if (nf[id] >= st && nf[id] < en) local[id] = k++;
  for (uint32_t id = 0; id < nn; ++id) {
    const int64_t q = local[id];
    if (q < 0) continue;
    const int L = lev[id];
    if (o->level) o->level[q] = (int8_t)L;
    if (o->prefix) o->prefix[q] = keys[nf[id] - st] >> (3 * (RB_DEPTH - L));
    if (o->first) o->first[q] = nf[id] - st;
    if (o->count) o->count[q] = (int64_t)nl[id] - nf[id] + 1;
    if (o->is_leaf) o->is_leaf[q] = (int8_t)lf[id];
    if (o->n_child) o->n_child[q] = lf[id] ? 0 : (int32_t)(nlc[id] - nch[id] + 1);
    if (o->first_child) o->first_child[q] = lf[id] ? -1 : local[nch[id]];
    if (o->skip) o->skip[q] = (nsk[id] == RB_NONE) ? -1 : local[nsk[id]];
    if (o->M) o->M[q] = mc[id].w;
    if (o->com) { o->com[3 * q] = mc[id].x; o->com[3 * q + 1] = mc[id].y; o->com[3 * q + 2] = mc[id].z; }
    if (o->Q) for (int a = 0; a < 6; ++a) o->Q[6 * q + a] = Q[6 * (size_t)id + a];
  }
  for (uint32_t r = 0; r < nlive; ++r) {
    if (o->keys) o->keys[r] = keys[r];
    if (o->perm) o->perm[r] = (int64_t)orig[r] - st;
  }
  return RB_OK;
}

int rb_gravity(rb_ctx *c, const rb_particles *p, int64_t n, int64_t n_active, double t,
               double *ax, double *ay, double *az) {
  if (!c) return fail(RB_EINVAL, "null context");
  if (!ax || !ay || !az) return fail(RB_EINVAL, "null acceleration array");
  if (!isfinite(t)) return fail(RB_EINVAL, "t must be finite");
  RB_TRY(check_particles(p, false));
  RB_TRY(set_single_n(c, n, n_active));
  RB_TRY(upload_schedule(c, t, 0.0, 0));
  RB_TRY(mark(c, PH_TOTAL, true));
  RB_TRY(build_tree(c, p));
  RB_TRY(walk(c, 0, 0));
  RB_PHASE(PH_POST, launch_scatter_acc(c, ax, ay, az));
  RB_TRY(mark(c, PH_TOTAL, false));
  return RB_OK;
}

int rb_batch_gravity(rb_ctx *c, const rb_particles *p, double t, double *ax, double *ay,
                     double *az) {
  if (!c) return fail(RB_EINVAL, "null context");
  if (!c->batch) return fail(RB_EINVAL, "not a batch context");
  return rb_gravity(c, p, (int64_t)c->h_starts[c->P], (int64_t)c->h_starts[c->P], t, ax, ay, az);
}

int rb_direct(rb_ctx *c, const rb_particles *p, int64_t n, int64_t n_active, double t,
              const int64_t *targets, int64_t n_targets, double *ax, double *ay, double *az) {
  if (!c) return fail(RB_EINVAL, "null context");
  if (c->batch) return fail(RB_EUNSUPPORTED, "rb_direct needs a single-system context");
  RB_TRY(check_particles(p, false));
  if (!targets || !ax || !ay || !az) return fail(RB_EINVAL, "null target or output array");
  if (n < 0 || (uint64_t)n > c->cap) return fail(RB_EINVAL, "n outside [0, capacity]");
  if (n_targets < 0 || n_targets > n) return fail(RB_EINVAL, "n_targets outside [0, n]");
  if (n_active < 0) return fail(RB_EINVAL, "n_active must be >= 0");
  if (!isfinite(t)) return fail(RB_EINVAL, "t must be finite");
  const double s = shear_offset(c->p, c->h_patch[0].L[0], c->h_patch[0].L[1], t);
  RB_PHASE(PH_DIRECT, launch_direct(c, p, (uint32_t)n, (uint32_t)std::min(n_active, n), s,
                                    targets, (uint32_t)n_targets, ax, ay, az));
  return RB_OK;
}

int rb_direct_noalloc(const rb_params *p, const rb_particles *parts, int64_t n,
                      int64_t n_active, double t, const int64_t *targets, int64_t n_targets,
                      double *ax, double *ay, double *az, void *hip_stream) {
  RB_TRY(validate(p));
  RB_TRY(validate_box(p, p->box_size, p->box_min));
  RB_TRY(check_particles(parts, false));
  if (!targets || !ax || !ay || !az) return fail(RB_EINVAL, "null target or output array");
  if (n < 0 || n > 0x7FFFFFFFll) return fail(RB_EINVAL, "n outside [0, 2^31 - 1]");
  if (n_targets < 0 || n_targets > n) return fail(RB_EINVAL, "n_targets outside [0, n]");
  if (n_targets > (int64_t)RB_DIRECT_SCRATCH_DOUBLES / 3)
    return fail(RB_EINVAL, "n_targets = %lld is above the %u targets the fixed scratch array "
                "holds", (long long)n_targets, RB_DIRECT_SCRATCH_DOUBLES / 3);
  if (n_active < 0) return fail(RB_EINVAL, "n_active must be >= 0");
  if (!isfinite(t)) return fail(RB_EINVAL, "t must be finite");
  const double Lx = (double)n_root_of(*p, 0) * p->box_size;
  const double Ly = (double)n_root_of(*p, 1) * p->box_size;
  const double s = shear_offset(*p, Lx, Ly, t);
  const hipError_t e = launch_direct_noalloc(p, parts, (uint32_t)n,
                                             (uint32_t)std::min(n_active, n), s, targets,
                                             (uint32_t)n_targets, n_images(*p), Lx, Ly, ax, ay,
                                             az, (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(RB_EHIP, "rb_direct_noalloc: %s", hipGetErrorString(e));
  return RB_OK;
}

int rb_step(rb_ctx *c, rb_particles *p, int64_t n, int64_t n_active, double t, double dt,
            int32_t nsteps) {
  if (!c) return fail(RB_EINVAL, "null context");
  RB_TRY(check_particles(p, true));
  RB_TRY(set_single_n(c, n, n_active));
  return run_step(c, p, t, dt, nsteps);
}

int rb_batch_step(rb_ctx *c, rb_particles *p, double t, double dt, int32_t nsteps) {
  if (!c) return fail(RB_EINVAL, "null context");
  if (!c->batch) return fail(RB_EINVAL, "not a batch context");
  RB_TRY(check_particles(p, true));
  return run_step(c, p, t, dt, nsteps);
}

// collision buffers, allocated by the first collision call of a context
static int coll_alloc(rb_ctx *c) {
  if (c->cap >= (1ull << 28)) return fail(RB_EUNSUPPORTED, "pair codes need n < 2^28");
  if (c->d_cq[0]) return RB_OK;
  c->cq_cap = 8 * c->cap + 1024;
  RB_TRY(dalloc(c, &c->d_cq[0], c->cq_cap));
  RB_TRY(dalloc(c, &c->d_cq[1], c->cq_cap));
  RB_TRY(dalloc(c, &c->d_ccnt, 16));
  c->d_cmax = reinterpret_cast<unsigned long long *>(c->d_ccnt + 4);
  c->d_cres = reinterpret_cast<unsigned long long *>(c->d_ccnt + 6);
  RB_HIP(hipHostMalloc((void **)&c->h_cpin, 64, hipHostMallocDefault));
  RB_HIP(hipMemsetAsync(c->d_ccnt, 0, 64, c->stream));
  RB_TRY(dalloc(c, &c->d_cbest, c->cap));
  RB_HIP(hipMemsetAsync(c->d_cbest, 0xFF, 8 * c->cap, c->stream));
  return RB_OK;
}

static int coll_check_args(rb_ctx *c, rb_particles *p, const double *radius, double t,
                           double epsilon, uint64_t *codes, int64_t codes_cap) {
  if (!c) return fail(RB_EINVAL, "null context");
  RB_TRY(check_particles(p, true));
  if (!radius) return fail(RB_EINVAL, "null radius array");
  if (!isfinite(t)) return fail(RB_EINVAL, "t must be finite");
  if (!(epsilon >= 0.0 && epsilon <= 1.0)) return fail(RB_EINVAL, "epsilon outside [0, 1]");
  if (codes_cap < 0 || (codes_cap > 0 && !codes)) return fail(RB_EINVAL, "bad code buffer");
  if (is_forest(c->p)) return fail(RB_EUNSUPPORTED, "collisions need a single root box");
  c->lcp_stale = true;  // the search builds its own tree in the same buffers
  return RB_OK;
}

// The queue the search left in list 0: optional copy of the codes, then the
// resolution rounds, each resolving at least the collision first in the
// whole queue.  A short queue is resolved entirely by one workgroup; a long
// one first goes through batches of multi-workgroup rounds (whose kernels
// read the list's length on the device) until it is short.  The first launch
// saves the number of detected pairs in the third count.
static int coll_resolve(rb_ctx *c, rb_particles *p, double t, double epsilon, uint64_t seed,
                        uint64_t *codes, int64_t codes_cap, int64_t *n_pairs,
                        int64_t *n_resolved) {
  if (codes_cap > 0) {  // the detected pairs, before the rounds reuse their list
    uint32_t cnt = 0;
    RB_HIP(hipMemcpyAsync(&cnt, c->d_ccnt, 4, hipMemcpyDeviceToHost, c->stream));
    RB_HIP(hipStreamSynchronize(c->stream));
    RB_TRY(report_device_errors(c));
    if (cnt > 0)
      RB_HIP(hipMemcpy(codes, c->d_cq[0], 8 * (size_t)std::min<int64_t>(cnt, codes_cap),
                       hipMemcpyDeviceToHost));
  }
  int a = 0;
  uint64_t rounds = 0;
  const uint32_t *h_cnt = c->h_cpin;
  RB_PHASE(PH_COLLIDE, launch_coll_rounds1(c, a, p, t, epsilon, seed, c->d_ccnt + 2));
  for (;;) {
    RB_HIP(hipMemcpyAsync(c->h_cpin, c->d_ccnt, 32, hipMemcpyDeviceToHost, c->stream));
    RB_HIP(hipStreamSynchronize(c->stream));
    if (h_cnt[3]) return report_device_errors(c);  // (a full queue ends the call here)
    if (h_cnt[a] == 0) break;
    if (rounds > h_cnt[2])
      return fail(RB_EHIP, "collision rounds did not finish (internal error)");
    for (int r = 0; r < 4; ++r, ++rounds) {
      RB_PHASE(PH_COLLIDE, launch_coll_round(c, a, p, t, epsilon, seed, nullptr));
      a = 1 - a;
    }
    RB_PHASE(PH_COLLIDE, launch_coll_rounds1(c, a, p, t, epsilon, seed, nullptr));
  }
  RB_TRY(mark(c, PH_TOTAL, false));
  if (n_pairs) *n_pairs = (int64_t)h_cnt[2];
  if (n_resolved) {
    unsigned long long res;
    memcpy(&res, h_cnt + 6, 8);
    *n_resolved = (int64_t)res;
  }
  // (with phase timing on, wait for the last event before reading the timers)
  return (c->p.profile & 1) ? report_device_errors(c) : RB_OK;
}

int rb_collide(rb_ctx *c, rb_particles *p, const double *radius, int64_t n, double t,
               double epsilon, uint64_t seed, int64_t *n_pairs, int64_t *n_resolved,
               uint64_t *codes, int64_t codes_cap) {
  RB_TRY(coll_check_args(c, p, radius, t, epsilon, codes, codes_cap));
  if (c->batch) {
    if (n != (int64_t)c->h_starts[c->P]) return fail(RB_EINVAL, "n must be the batch total");
  } else {
    RB_TRY(set_single_n(c, n, n));
  }
  if (c->node_cap >= (1ull << 27))
    return fail(RB_EUNSUPPORTED, "the collision search needs fewer than 2^27 nodes");
  RB_TRY(coll_alloc(c));
  if (!c->d_cgeo) RB_TRY(dalloc(c, &c->d_cgeo, 4 * c->node_cap));
  RB_HIP(hipMemsetAsync(c->d_ccnt, 0, 40, c->stream));
  RB_TRY(mark(c, PH_TOTAL, true));
  RB_PHASE(PH_KEYS, launch_keys(c, p->x, p->y, p->z, 0.0));
  RB_PHASE(PH_SORT, launch_sort(c));
  RB_PHASE(PH_PERMUTE, launch_permute_gravity(c, p->x, p->y, p->z, p->m, 0));
  RB_PHASE(PH_TOPO, launch_topology(c));
  c->fp64_partial = true;  // a topology without moments
  RB_PHASE(PH_COLLIDE, launch_coll_prep(c, radius));
  RB_PHASE(PH_CSEARCH, launch_coll_detect(c, radius, t));
  return coll_resolve(c, p, t, epsilon, seed, codes, codes_cap, n_pairs, n_resolved);
}

int rb_set_collisions(rb_ctx *c, const double *radius, double epsilon, uint64_t seed,
                      int32_t enable) {
  if (!c) return fail(RB_EINVAL, "null context");
  if (enable) {
    if (!radius) return fail(RB_EINVAL, "null radius array");
    if (!(epsilon >= 0.0 && epsilon <= 1.0)) return fail(RB_EINVAL, "epsilon outside [0, 1]");
    if (c->node_cap >= (1ull << 27))
      return fail(RB_EUNSUPPORTED, "the collision search needs fewer than 2^27 nodes");
    if (is_forest(c->p)) return fail(RB_EUNSUPPORTED, "collisions need a single root box");
    RB_TRY(coll_alloc(c));
    if (!c->d_cgeo) RB_TRY(dalloc(c, &c->d_cgeo, 4 * c->node_cap));
    if (!c->d_cwrap) RB_TRY(dalloc(c, &c->d_cwrap, c->cap));
    if (!c->d_cinv) RB_TRY(dalloc(c, &c->d_cinv, c->cap));
    // the running totals start at zero
    RB_HIP(hipMemsetAsync(c->d_ccnt + 10, 0, 16, c->stream));
  }
  c->coll_on = enable != 0;
  c->coll_R = enable ? radius : nullptr;
  c->coll_eps = epsilon;
  c->coll_seed = seed;
  c->coll_steps = 0;
  c->graph_key = -1;  // the step's kernels change: capture again
  return RB_OK;
}

int rb_collision_counts(rb_ctx *c, int64_t *n_pairs, int64_t *n_resolved) {
  if (!c) return fail(RB_EINVAL, "null context");
  RB_TRY(report_device_errors(c));
  unsigned long long v[2] = {0ull, 0ull};
  if (c->d_ccnt) {
    RB_HIP(hipMemcpy(v, c->d_ccnt + 10, 16, hipMemcpyDeviceToHost));
    RB_HIP(hipMemsetAsync(c->d_ccnt + 10, 0, 16, c->stream));
    RB_HIP(hipStreamSynchronize(c->stream));
  }
  if (n_pairs) *n_pairs = (int64_t)v[0];
  if (n_resolved) *n_resolved = (int64_t)v[1];
  return RB_OK;
}

int rb_sweep(rb_ctx *c, rb_particles *p, const double *radius, int64_t n, double t, double dt,
             int32_t axis, double epsilon, uint64_t seed, int64_t *n_pairs,
             int64_t *n_resolved, uint64_t *codes, int64_t codes_cap) {
  RB_TRY(coll_check_args(c, p, radius, t, epsilon, codes, codes_cap));
  if (!(dt >= 0.0 && isfinite(dt))) return fail(RB_EINVAL, "dt must be finite and >= 0");
  if (axis != RB_SWEEP_X && axis != RB_SWEEP_PHI) return fail(RB_EINVAL, "axis must be 0 or 1");
  if (c->batch) return fail(RB_EUNSUPPORTED, "the plane sweep runs on a single system");
  if (axis == RB_SWEEP_PHI && c->p.boundary != RB_OPEN)
    return fail(RB_EUNSUPPORTED, "the azimuthal sweep needs an open box");
  const int phi = axis == RB_SWEEP_PHI ? 1 : 0;
  RB_TRY(set_single_n(c, n, n));
  RB_TRY(coll_alloc(c));
  if (!c->d_swR) {
    RB_TRY(dalloc(c, &c->d_swR, c->cap));
    RB_TRY(dalloc(c, &c->d_swhi, c->cap));
  }
  RB_HIP(hipMemsetAsync(c->d_ccnt, 0, 40, c->stream));
  RB_TRY(mark(c, PH_TOTAL, true));
  c->fp64_partial = true;  // the sort buffers now hold the sweep's order
  RB_PHASE(PH_KEYS, launch_sweep_keys(c, p, radius, dt, phi));
  RB_PHASE(PH_SORT, launch_sort(c));
  RB_PHASE(PH_CSEARCH, launch_sweep_pairs(c, p, radius, t, dt, phi));
  return coll_resolve(c, p, t, epsilon, seed, codes, codes_cap, n_pairs, n_resolved);
}

int rb_sync(rb_ctx *c) {
  if (!c) return fail(RB_EINVAL, "null context");
  return report_device_errors(c);
}

int rb_stats(rb_ctx *c, rb_stats_t *out) {
  if (!c || !out) return fail(RB_EINVAL, "null argument");
  RB_TRY(report_device_errors(c));
  unsigned long long s[8];
  RB_HIP(hipMemcpy(s, c->d_stats, sizeof(s), hipMemcpyDeviceToHost));
  memset(out, 0, sizeof(*out));
  out->open_tests = (int64_t)s[0];
  out->cells = (int64_t)s[1];
  out->pp = (int64_t)s[2];
  out->list_cells = (int64_t)s[3];
  out->list_pp = (int64_t)s[4];
  out->reused_steps = (int64_t)s[5];
  for (int k = 0; k < 16; ++k) {
    out->ms[k] = c->phase_ms[k];
    out->calls[k] = c->phase_calls[k];
    c->phase_ms[k] = 0.0;
    c->phase_calls[k] = 0;
  }
  RB_HIP(hipMemset(c->d_stats, 0, sizeof(s)));
  return RB_OK;
}

const char *rb_phase_name(int32_t phase) {
  if (phase < 0 || phase >= PH_COUNT) return "";
  return g_phase_names[phase];
}

static const char kMagic[8] = {'R', 'B', 'S', 'T', 'A', 'T', 'E', '1'};

int rb_state_save(rb_ctx *c, const rb_particles *p, int64_t n, double t, const char *path) {
  if (!c || !path) return fail(RB_EINVAL, "null argument");
  RB_TRY(check_particles(p, true));
  if (n < 0) return fail(RB_EINVAL, "n must be >= 0");
  RB_TRY(report_device_errors(c));
  std::vector<double> buf((size_t)n);
  FILE *f = fopen(path, "wb");
  if (!f) return fail(RB_EIO, "cannot open %s for writing", path);
  bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(&n, 8, 1, f) == 1 && fwrite(&t, 8, 1, f) == 1 &&
            fwrite(&c->p, sizeof(rb_params), 1, f) == 1;
  double *arr[7] = {p->x, p->y, p->z, p->vx, p->vy, p->vz, p->m};
  for (int k = 0; ok && k < 7; ++k) {
    if (n && hipMemcpy(buf.data(), arr[k], 8 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess) {
      fclose(f);
      return fail(RB_EHIP, "device to host copy failed");
    }
    ok = fwrite(buf.data(), 8, (size_t)n, f) == (size_t)n;
  }
  ok = (fclose(f) == 0) && ok;
  return ok ? RB_OK : fail(RB_EIO, "short write to %s", path);
}

int rb_state_load(rb_ctx *c, rb_particles *p, int64_t n, double *t, const char *path) {
  if (!c || !path || !t) return fail(RB_EINVAL, "null argument");
  RB_TRY(check_particles(p, true));
  FILE *f = fopen(path, "rb");
  if (!f) return fail(RB_EIO, "cannot open %s", path);
  char magic[8];
  int64_t nf = -1;
  double tf = 0.0;
  rb_params pf;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMagic, 8) == 0 &&
            fread(&nf, 8, 1, f) == 1 && fread(&tf, 8, 1, f) == 1 &&
            fread(&pf, sizeof(rb_params), 1, f) == 1;
  if (!ok) { fclose(f); return fail(RB_EIO, "%s is not an rb state file", path); }
  if (nf != n) { fclose(f); return fail(RB_EINVAL, "file holds %lld particles, expected %lld", (long long)nf, (long long)n); }
  std::vector<double> buf((size_t)n);
  double *arr[7] = {p->x, p->y, p->z, p->vx, p->vy, p->vz, p->m};
  for (int k = 0; k < 7; ++k) {
    if (fread(buf.data(), 8, (size_t)n, f) != (size_t)n) { fclose(f); return fail(RB_EIO, "short read from %s", path); }
    if (n && hipMemcpy(arr[k], buf.data(), 8 * (size_t)n, hipMemcpyHostToDevice) != hipSuccess) {
      fclose(f);
      return fail(RB_EHIP, "host to device copy failed");
    }
  }
  fclose(f);
  *t = tf;
  return RB_OK;
}

const char *rb_error_string(int code) {
  switch (code) {
    case RB_OK: return "ok";
    case RB_EINVAL: return "invalid argument";
    case RB_ENOMEM: return "out of memory";
    case RB_EHIP: return "HIP runtime error";
    case RB_ECAPACITY: return "capacity exceeded";
    case RB_EOUTSIDE: return "particle outside a periodic box";
    case RB_EUNSUPPORTED: return "unsupported";
    case RB_EIO: return "file error";
    default: return "unknown error";
  }
}

const char *rb_last_error(void) { return g_err.c_str(); }

}  // extern "C"
