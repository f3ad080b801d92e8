// rb_internal.h -- host-side context of librb and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rb.h"
#include "rb_common.h"

// Work item: a run of consecutive sorted slots of one patch.  For the
// grouped walk and the moments pass, node is the last of the consecutive
// sibling subtrees the run is made of (RB_NONE for a piece of a leaf with
// more than G particles); the FP64 walk's items leave it unused.
struct WalkItem {
  uint32_t start, end;  // slot range [start, end)
  uint32_t patch;
  uint32_t node;
};

// Item gi in the grouped walk's order: those of more than G/2 particles
// (front of the first table), of more than G/4 (second table), the rest
// (back of the first table, whose capacity is cap).
__device__ __forceinline__ WalkItem rb_walk_item(const WalkItem *__restrict__ items,
                                                 const WalkItem *__restrict__ items_mid,
                                                 uint32_t gi, uint32_t n_big, uint32_t n_mid,
                                                 uint64_t cap) {
  if (gi < n_big) return items[gi];
  if (gi < n_big + n_mid) return items_mid[gi - n_big];
  return items[(uint32_t)cap - 1u - (gi - n_big - n_mid)];
}

// Control block of the 64-part FP64 walk's dispatch order.  Before each
// walk the listing kernel lists the units whose last cost reached the
// threshold, under the launch number `epoch`, and histograms the costs (by
// bit length); its last block turns the histogram into the next threshold,
// publishes the number as `cur` for the walk and starts the next one.
struct W64Ctl {
  uint32_t done;       // blocks of the running listing that have finished
  uint32_t epoch;      // the number the next listing tags with
  uint32_t cur;        // the number of the listing the next walk runs by
  uint32_t thr;        // cost from which a unit is listed
  uint32_t cnt[2][8];  // units listed per XCD share, under an odd / even number
  uint32_t hist[33];   // costs of the listing's units by bit length
};

struct rb_ctx {
  rb_params p;
  int device = 0;
  hipStream_t stream = nullptr;
  bool batch = false;
  uint32_t P = 1;            // patches
  uint64_t cap = 0;          // slots
  uint64_t node_cap = 0;
  int n_img = 1;             // ghost images
  int img_split = 0;         // items per image (1) or all images per item (0)
  // FP64 walk: 1 (per-lane walks), 2 (wave-shared) or 3 (wave-shared, one
  // unit per child subtree of the root); walk_parts = 8 with 3, else 1
  int walk64_mode = 1;
  int walk_parts = 1;
  int acc_sets = 1;          // sets of 3 * cap doubles that d_acc holds

  // host mirrors
  std::vector<uint32_t> h_starts;  // P + 1
  std::vector<PatchInfo> h_patch;
  std::vector<uint32_t> h_tile_start, h_tile_end, h_tile_patch, h_patch_tile0;

  // patches and tiles (device)
  PatchInfo *d_patch = nullptr;
  uint32_t *d_starts = nullptr;   // P + 1
  uint32_t *d_nlive = nullptr;    // P
  uint32_t *d_root = nullptr;     // P
  uint32_t n_tiles = 0, max_tiles_per_patch = 0;
  uint32_t *d_tile_start = nullptr, *d_tile_end = nullptr, *d_tile_patch = nullptr;
  uint32_t *d_patch_tile0 = nullptr;  // P + 1

  // sort: its own tiles of 256 * sort_rows slots (never crossing a patch)
  uint64_t *d_key[2] = {nullptr, nullptr};
  uint32_t *d_idx[2] = {nullptr, nullptr};
  std::vector<uint32_t> h_stile_start, h_stile_end, h_stile_patch, h_spatch_tile0;
  uint32_t *d_stile_start = nullptr, *d_stile_end = nullptr, *d_stile_patch = nullptr;
  uint32_t *d_spatch_tile0 = nullptr;  // P + 1
  uint32_t n_stiles = 0;
  int sort_rows = 1;                   // rows of 64 keys per wave (1, 2, 4, 8)
  uint32_t stile = 256;                // slots per sort tile
  uint32_t sort_hist_tiles = 1;        // sort tiles counted per histogram block
  uint32_t *d_stot = nullptr;          // 2 x P x 8 passes x 256 digit totals
  uint64_t *d_sdesc = nullptr;         // look-back words, 256 per sort tile
  uint32_t *d_sctl = nullptr;          // [sort number, tile counter A, B, pad]
  // small systems: bucket sort (k_bsort.hip)
  bool sort_small = false;
  uint64_t small_sort_max = 0;  // largest patch the bucket sort takes
  uint32_t *d_bcnt = nullptr;   // P x 4097 bucket counts (zero between sorts)
  uint32_t *d_bcur = nullptr;   // P x 4097 scatter cursors
  uint2 *d_bseg = nullptr;      // segments (first slot, patch)
  uint32_t *d_bctl = nullptr;   // [segments, segments taken]

  // particles in sorted order (ping-pong for rb_step)
  double *d_px[2][7] = {};          // x y z vx vy vz m
  uint32_t *d_orig[2] = {nullptr, nullptr};
  double *d_msrc = nullptr;         // source mass of sorted slots
  int cur = 0;                      // buffer holding the sorted state

  // topology; d_lcp: per sorted slot, the octal prefix level it shares with
  // the previous live key of the last tree (255 first slot, 254 dead), for
  // the check that lets rb_step keep a tree (reuse_topology); lcp_stale:
  // the tree buffers were last written by another path, so the first step
  // of the next rb_step call rebuilds
  uint8_t *d_lcp = nullptr;
  bool lcp_stale = true;
  uint32_t *d_cnt = nullptr;        // 2 * 22 * n_tiles (starts, ends)
  uint32_t *d_lev_tot = nullptr;    // 2 * 22
  uint32_t *d_lev_off = nullptr;    // 23 (+1: node total)
  uint32_t *d_nfirst = nullptr, *d_nlast = nullptr, *d_nchild = nullptr,
           *d_nlastchild = nullptr, *d_nskip = nullptr;
  uint8_t *d_nlevel = nullptr, *d_nleaf = nullptr;
  uint32_t *d_csr = nullptr;        // per slot: nodes starting at earlier slots
  uint32_t *d_start_ids = nullptr;  // node ids in (start slot, level) order

  // moments
  NodeLink *d_link = nullptr;
  double4 *d_mcom = nullptr;  // com.x com.y com.z M
  double *d_S = nullptr;      // 3 per node
  double *d_Q = nullptr;      // 6 per node
  WNode *d_wnode = nullptr;   // the grouped walk's node records (FP32-mixed only)
  bool fp64_partial = false;  // the last tree (an FP32-mixed step) lacks FP64 records

  // walk
  std::vector<WalkItem> h_items64;  // FP64 walk: 64 Morton-consecutive slots
  WalkItem *d_items64 = nullptr;
  WalkItem *d_witems = nullptr;     // FP32 walk: packed work items (big ones, small ones)
  WalkItem *d_witems_mid = nullptr; // FP32 walk: packed work items of middle size
  uint32_t *d_gctr = nullptr;       // [groups emitted, items taken, big, middle, small items]
  uint32_t *d_large = nullptr;      // nodes with more than G particles, by level
  uint32_t *d_bottom = nullptr;     // those without such a child (not in d_large)
  uint32_t *d_large_cnt = nullptr;  // per-level counts, then the bottom count
  // collisions (allocated by the first rb_collide): two code lists (the
  // detected pairs, then the survivors of each resolution round), their
  // counts, each particle's smallest pending queue key, R_max, resolved
  // collisions, the cells' centres and links
  uint64_t *d_cq[2] = {nullptr, nullptr};
  uint64_t cq_cap = 0;
  // one 64-byte block [list counts 0, 1 | detected pairs | copy of the
  // error word | R_max bits (2 words) | resolved (2 words) | largest
  // displacement bits (2 words) | collisions of rb_step since they were
  // last read: pairs (2 words), resolved (2 words) | -], its first 40 bytes
  // cleared once per call or step and read back in one copy
  uint32_t *d_ccnt = nullptr;
  unsigned long long *d_cbest = nullptr;
  unsigned long long *d_cmax = nullptr;  // = d_ccnt + 4
  unsigned long long *d_cres = nullptr;  // = d_ccnt + 6
  uint32_t *h_cpin = nullptr;            // pinned host copy of the block (16 words)
  // collisions inside rb_step (rb_set_collisions): radius (caller order,
  // the caller's device array), restitution, seed of the next step, the
  // per-slot wrap of the second drift and the caller-to-slot map
  bool coll_on = false;
  const double *coll_R = nullptr;
  double coll_eps = 0.0;
  uint64_t coll_seed = 0;
  uint16_t *d_cwrap = nullptr;
  uint32_t *d_cinv = nullptr;
  uint64_t coll_steps = 0;  // steps run with collisions since they were set
  uint64_t chunk_seed = 0;  // seed of the first step of the uploaded schedule
  double *d_cgeo = nullptr;         // 4 per node: the search's cell records
  double *d_swR = nullptr, *d_swhi = nullptr;  // plane sweep: sorted radii, interval ends
  double *d_acc = nullptr;          // acc_sets * 3 * cap
  // the 64-part FP64 walk's dispatch order, one buffer: the control block,
  // then per unit (RB_WALK64_ORDER_CAP each) the node visits of the last
  // launch and the launch number that lists it to run first, then the list
  // (RB_WALK64_HEAVY_MAX)
  uint32_t *d_w64_ord = nullptr;

  // per-call dynamic region [ctr | StepConst | schedule], uploaded from a
  // pinned staging copy; schedule per step: s_half[P], s_end[P]
  char *d_dyn = nullptr, *h_dyn = nullptr;
  size_t dyn_bytes = 0;
  hipEvent_t dyn_ev = nullptr;
  StepConst *d_sc = nullptr;
  double *d_sched = nullptr;
  uint32_t sched_cap = 0;
  // [step index read by even steps, by odd steps, steps in this call]
  uint32_t *d_ctr = nullptr;
  uint32_t tile = 0;          // slots per sort / topology tile

  uint32_t *d_err = nullptr;
  unsigned long long *d_stats = nullptr;  // 8 counters

  // profiling
  hipEvent_t ev[16] = {};
  int ev_used = 0;
  double phase_ms[16] = {};
  int64_t phase_calls[16] = {};

  // graph of one step
  // captured graphs of one step, for the two buffer parities (state in
  // buffer 0 -> 1, and 1 -> 0); graph_key < 0 marks them stale
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  int graph_key = -1;
  hipStream_t cap_stream = nullptr;  // private stream used only for capture

  std::vector<void *> allocs;
};

// ---- collisions: shared by the tree search and the plane sweep ----
#define RB_COLL_LOCAL 8  // pairs a thread keeps before it writes them out

// image k of the ghost boxes: ix outer and iy inner in [-ng, ng] (a single
// image for open boundaries); position offset and y velocity offset
__device__ __forceinline__ void rb_coll_image_xy(int ix, int iy, int boundary, double W,
                                                 double sh, double omega, double &ox,
                                                 double &oy, double &wy) {
  if (boundary == RB_OPEN) { ox = oy = wy = 0.0; return; }
  const double fx = (double)ix, fy = (double)iy;
  const double s = (boundary == RB_SHEAR) ? sh : 0.0;
  ox = fx * W;
  oy = fy * W - fx * s;
  wy = (boundary == RB_SHEAR) ? -1.5 * omega * W * fx : 0.0;
}
__device__ __forceinline__ void rb_coll_image(int k, int ngx, int ngy, int boundary, double W,
                                              double sh, double omega, double &ox, double &oy,
                                              double &wy) {
  const int ny = 2 * ngy + 1;
  rb_coll_image_xy(k / ny - ngx, k % ny - ngy, boundary, W, sh, omega, ox, oy, wy);
}

// queue a pair from the lane's local list, writing the list out when full
__device__ __forceinline__ void rb_coll_keep(uint64_t code, uint64_t (&mine)[RB_COLL_LOCAL],
                                             uint32_t &nm, uint64_t *__restrict__ queue,
                                             uint32_t qcap, uint32_t *__restrict__ qcnt,
                                             uint32_t *__restrict__ err) {
  if (nm == RB_COLL_LOCAL) {
    const uint32_t at = atomicAdd(qcnt, (uint32_t)nm);
    for (uint32_t q = 0; q < nm; ++q)
      if (at + q < qcap) queue[at + q] = mine[q];
    if (at + nm > qcap) atomicOr(err, RB_ERR_COLL);
    nm = 0;
  }
  mine[nm++] = code;
}

// ---- launchers (each returns hipSuccess or the launch error) ----
hipError_t launch_keys(rb_ctx *c, const double *x, const double *y, const double *z,
                       double s_unused);
hipError_t launch_sort(rb_ctx *c);
hipError_t launch_groups(rb_ctx *c, const uint32_t *reuse = nullptr);
hipError_t launch_sweep_keys(rb_ctx *c, const rb_particles *pp, const double *radius,
                             double dt, int phi);
hipError_t launch_sweep_pairs(rb_ctx *c, const rb_particles *pp, const double *radius,
                              double t, double dt, int phi);
hipError_t launch_coll_prep(rb_ctx *c, const double *radius);
hipError_t launch_coll_step_prep(rb_ctx *c, int buf);
hipError_t launch_coll_step_search(rb_ctx *c, int buf, int slot);
hipError_t launch_coll_step_rounds(rb_ctx *c, int buf, int slot);
hipError_t launch_coll_detect(rb_ctx *c, const double *radius, double t);
hipError_t launch_coll_rounds1(rb_ctx *c, int a, const rb_particles *pp, double t, double eps,
                               uint64_t seed, uint32_t *save);
hipError_t launch_coll_round(rb_ctx *c, int a, const rb_particles *pp, double t, double eps,
                             uint64_t seed, uint32_t *save);
hipError_t launch_bsort(rb_ctx *c);
hipError_t launch_permute_state(rb_ctx *c, int src, int dst);
hipError_t launch_permute_gravity(rb_ctx *c, const double *x, const double *y,
                                  const double *z, const double *m, uint32_t n_active_single);
// reuse: the step's keep-the-tree flag (0: the last tree stands, the
// topology kernels exit at once), or nullptr to always build
hipError_t launch_topology(rb_ctx *c, const uint32_t *reuse = nullptr);
hipError_t launch_topo_check(rb_ctx *c, uint32_t *flag);
// roots_only: an FP32-mixed step, whose walk reads only the FP32 node
// records; the FP64 records below the walk items' subtree roots are skipped
hipError_t launch_moments(rb_ctx *c, const double *sx, const double *sy, const double *sz,
                          bool roots_only = false, const uint32_t *reuse = nullptr);
hipError_t launch_rowscan_levels(rb_ctx *c, const uint32_t *reuse = nullptr);
// walk results summed per particle: one set per image (when split) and per
// part of the FP64 walk, in that order
// parts of the FP64 walk's schedule 3: the subtrees one level below the
// root, or two levels below for systems of under RB_WALK64_PARTS2_MAX_ITEMS
// items (measured: 156 items 34% faster with 64 parts, 3,125 items 15%
// slower)
#define RB_WALK64_PARTS 8
#define RB_WALK64_PARTS2 64
#define RB_WALK64_PARTS2_MAX_ITEMS 1024u
// units of the 64-part walk that get a cost-ordered dispatch (at most
// RB_WALK64_PARTS2_MAX_ITEMS items of 64 parts)
#define RB_WALK64_ORDER_CAP 65536u
#define RB_WALK64_ORDER_MIN 4096u
#define RB_WALK64_HEAVY_MAX 4096u  // 8 lists (one per XCD share) of 512
// offsets (in 32-bit words) in the order buffer
#define RB_W64_COST_OFF 64u
#define RB_W64_TAG_OFF (RB_W64_COST_OFF + RB_WALK64_ORDER_CAP)
#define RB_W64_HEAVY_OFF (RB_W64_TAG_OFF + RB_WALK64_ORDER_CAP)
#define RB_W64_ORD_WORDS (RB_W64_HEAVY_OFF + RB_WALK64_HEAVY_MAX)
inline int rb_n_acc(const rb_ctx *c) { return (c->img_split ? c->n_img : 1) * c->walk_parts; }
// work units from which the wave-shared FP64 walk beats per-lane walks
#define RB_WALK64_SHARED_MIN 12288u
hipError_t launch_walk64(rb_ctx *c, const double *sx, const double *sy, const double *sz,
                         int slot);
hipError_t launch_walk32(rb_ctx *c, const double *sx, const double *sy, const double *sz,
                         int slot);
hipError_t launch_scatter_acc(rb_ctx *c, double *ax, double *ay, double *az);
hipError_t launch_prologue(rb_ctx *c, const rb_particles *cp);
// mode 0: kick, second drift, next first drift and keys; 1: up to the
// second drift (records wraps and the largest displacement for the
// collisions at the end of the step); 2: the next first drift and keys
hipError_t launch_post(rb_ctx *c, int buf, int slot, int mode = 0);
hipError_t launch_epilogue(rb_ctx *c, rb_particles *cp, int buf);
hipError_t launch_direct(rb_ctx *c, const rb_particles *cp, uint32_t n, uint32_t n_active,
                         double s, const int64_t *targets, uint32_t nt,
                         double *ax, double *ay, double *az);
// the same without a context: partial sums in a fixed per-GPU array of
// RB_DIRECT_SCRATCH_DOUBLES doubles (3 per target and source chunk)
#define RB_DIRECT_SCRATCH_DOUBLES (1u << 20)
hipError_t launch_direct_noalloc(const rb_params *p, const rb_particles *cp, uint32_t n,
                                 uint32_t n_active, double s, const int64_t *targets,
                                 uint32_t nt, int n_img, double Lx, double Ly, double *ax,
                                 double *ay, double *az, hipStream_t stream);
