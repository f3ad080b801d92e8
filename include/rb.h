/*
 * rb.h -- C ABI of librb: Barnes-Hut tree self-gravity on one AMD Instinct
 * MI355X (gfx950), the hot path of the method of Rein & Liu (2012), REBOUND.
 *
 * Conventions for every entry point
 *  - Particle arrays are DEVICE pointers to FP64 structure-of-arrays data in
 *    the caller's order; the caller owns them (typically torch tensors).
 *  - Output arrays (accelerations) are device pointers the caller owns.
 *  - A context owns all GPU workspace: keys, permutations, nodes, moments,
 *    interaction lists, schedules.  It is bound to one device and one HIP
 *    stream given at creation; every call is asynchronous on that stream
 *    unless its comment says it synchronises.
 *  - Return value: RB_OK (0) or a negative RB_E* code.  rb_last_error()
 *    returns a thread-local text with details of the last failure.  Faults
 *    detected inside kernels (capacity overflow, a particle outside a
 *    periodic box) raise a device error word that is reported by the next
 *    synchronising call (rb_sync, rb_tree_info, rb_tree_export,
 *    rb_state_save, rb_stats), like HIP's own deferred errors.
 *  - Removed particles: a particle that leaves the root box through an open
 *    face is removed from the simulation (Sect. 2.3).  It becomes a
 *    tombstone: NaN position, zero velocity.  Tombstones (any particle with
 *    a NaN coordinate) are excluded from the tree, feel no force and exert
 *    none; n is never compacted.
 */
#ifndef RB_H
#define RB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RB_OK 0
#define RB_EINVAL (-1)        /* bad parameter, null pointer, size out of range */
#define RB_ENOMEM (-2)        /* device or host allocation failed */
#define RB_EHIP (-3)          /* HIP runtime error */
#define RB_ECAPACITY (-4)     /* node, list or particle capacity exceeded */
#define RB_EOUTSIDE (-5)      /* particle outside a periodic / shear box axis */
#define RB_EUNSUPPORTED (-6)  /* valid request this library does not implement */
#define RB_EIO (-7)           /* state file could not be read or written */

typedef enum { RB_OPEN = 0, RB_PERIODIC = 1, RB_SHEAR = 2 } rb_boundary;
typedef enum { RB_FP64 = 0, RB_FP32_MIXED = 1 } rb_precision;
typedef enum { RB_DRIFT_LEAPFROG = 0, RB_DRIFT_EPICYCLE = 1 } rb_drift;

/*
 * Physical and numerical parameters (Sect. 2.3, 3, 4 of the paper).
 *  G, softening     Eq. (1): G and the Plummer softening b (b >= 0).
 *  theta            critical opening angle of Sect. 4.2: a cell of width w
 *                   at distance R from its centre of mass is used as a whole
 *                   when w^2 < theta^2 R^2.  theta = 0 gives direct
 *                   summation through the tree.
 *  quadrupole       0: mass and centre of mass only; 1: add the cell
 *                   quadrupole (Hernquist 1987), as the paper's QUADRUPOLE
 *                   switch.
 *  leaf_size        most particles a leaf above the deepest level holds
 *                   (paper: 1).  1..32.
 *  group_size       FP32-mixed walk only: particles that share one
 *                   interaction list (16, 32 or 64).
 *  boundary         RB_OPEN: particles leaving the root box are removed.
 *                   RB_PERIODIC: x and y wrap, z is open.
 *                   RB_SHEAR: shear-periodic in x, periodic in y, z open;
 *                   requires box_min[0] = -Lx / 2.
 *  drift            RB_DRIFT_LEAPFROG: x += v tau (Sect. 3.1).
 *                   RB_DRIFT_EPICYCLE: exact solution of Hill's equations
 *                   without the perturbing force (Sect. 3.3).
 *  precision        RB_FP64: per-particle FP64 walk, identical opening
 *                   decisions to a plain FP64 Barnes-Hut walk.
 *                   RB_FP32_MIXED: grouped walk, FP32 interaction
 *                   arithmetic on node-relative coordinates, FP64
 *                   positions, velocities, drift, ghost offsets and sums.
 *  box_size, box_min  side W of every cubic root box, and the domain's
 *                   minimum corner (Sect. 2.3).
 *  n_root           root boxes per axis (Sect. 2.3: an integer number of
 *                   cubic boxes along each axis, e.g. elongated boxes; 0 or
 *                   1 = one box, at most 256).  The domain is
 *                   [box_min, box_min + n_root W) per axis, extents
 *                   L = n_root W, and every root box has a tree of its own
 *                   (cells of side W 2^-k below it).  Keys quantise the
 *                   domain once, 2^(21-D) steps per root box per axis, where
 *                   2^D >= every n_root, so a root box's tree is at most
 *                   21 - D levels deep.  The exported tree lists, above the
 *                   root boxes (levels < D), the cells of side W 2^(D-l)
 *                   that hold them; those are never leaves and every walk
 *                   opens them.  Single systems only (batches, collisions
 *                   and the plane sweep refuse forests: RB_EUNSUPPORTED).
 *  n_ghost          ghost-box rings in x and y (periodic / shear only,
 *                   0..2); images are (ix Lx, iy Ly - ix s, 0), ix and iy in
 *                   [-n_ghost, n_ghost], s the shear offset
 *                   remainder(1.5 omega Lx t, Ly).
 *  omega, omega_z   orbital and vertical epicyclic frequency.
 *  node_factor      node capacity per particle (>= 1.5; 0 selects 3).
 *  split_images     1: one walk work item per (group, image) pair, 0: one
 *                   per group, -1: choose by size.
 *  profile          bit 0: record per-phase times with HIP events on the
 *                   context's stream; bit 1: count walk interactions
 *                   (atomics in the walk); bit 2: time the walk kernel
 *                   and the collision search kernel only.  All are read
 *                   by rb_stats.
 *  use_graph        1: rb_step / rb_batch_step replay a captured HIP graph
 *                   of one step.
 *  walk_waves       FP32-mixed walk only: waves that share one group's
 *                   traversal (1, 2 or 4; 0 selects 1).  More waves shorten
 *                   each group's chain of dependent steps when there are few
 *                   groups for the chip.
 *  moments_level_log2  the moments of the nodes above the walk's work items
 *                   (bottom-up, Sect. 4.2) run in one workgroup for systems
 *                   of up to 2^k slots and level by level over the whole chip
 *                   above; k = 0 selects 22.  6..31.  Both orders add the
 *                   same children in the same order, so the moments are
 *                   identical; only the speed differs.
 *  reuse_topology   1: rb_step keeps the tree from one step to the next when
 *                   it can (the tree reconstruction of Sect. 4.2).  The
 *                   particles stay in Morton order between steps; after each
 *                   step's sort a check compares, slot by slot, the octal
 *                   prefix levels consecutive keys share with the last
 *                   tree's.  The canonical tree is a function of those
 *                   levels, so when none changed (no particle left its cell)
 *                   the topology, node lists and work items are reused and
 *                   only the moments are recomputed bottom-up; otherwise the
 *                   tree is rebuilt.  Same results either way; rb_stats
 *                   counts the reused steps.  0: rebuild every step.
 *  walk64_schedule  FP64 walk: 0 chooses (3 when the accumulators allow it,
 *                   else 2 or 1 by size), 1 every lane walks for its
 *                   own particle, 2 a wave walks once for its 64 particles
 *                   (each lane keeping its own decisions), 3 as 2 with one
 *                   wave per subtree two levels below the root (64x the
 *                   work units for systems of few particles; the subtrees'
 *                   sums are added in octant order afterwards, so only
 *                   their rounding differs; a context whose accumulators
 *                   for this would exceed 2 GiB runs 2).  All visit, per
 *                   particle, the same nodes; only the speed differs.
 */
typedef struct {
  double G;
  double softening;
  double theta;
  int32_t quadrupole;
  int32_t leaf_size;
  int32_t group_size;
  int32_t boundary;
  int32_t drift;
  int32_t precision;
  double box_size;
  double box_min[3];
  int32_t n_ghost[2];
  double omega;
  double omega_z;
  double node_factor;
  int32_t split_images;
  int32_t profile;
  int32_t use_graph;
  int32_t walk_waves;
  int32_t moments_level_log2;
  int32_t walk64_schedule;
  int32_t n_root[3];
  int32_t reuse_topology;
  int32_t reserved[2];
} rb_params;

/* Device SoA of the particles, caller order, all FP64. */
typedef struct {
  double *x, *y, *z;
  double *vx, *vy, *vz;
  double *m;
} rb_particles;

/* Host buffers for rb_tree_export; each array holds n_nodes (node arrays)
 * or n_live (keys, perm) entries, sizes from rb_tree_info.  Any pointer may
 * be NULL to skip that field. */
typedef struct {
  uint64_t *keys;      /* sorted Morton keys of the live particles */
  int64_t *perm;       /* Morton rank -> caller index */
  int8_t *level;       /* node level, root = 0 */
  uint64_t *prefix;    /* key >> 3 (21 - level) */
  int64_t *first;      /* Morton rank of the node's first particle */
  int64_t *count;      /* particles in the node */
  int8_t *is_leaf;
  int32_t *n_child;
  int64_t *first_child;/* node index of the first child, -1 for leaves */
  int64_t *skip;       /* next node after the subtree in depth-first order, -1 at the end */
  double *M;           /* source mass */
  double *com;         /* 3 per node: centre of mass */
  double *Q;           /* 6 per node: xx xy xz yy yz zz traceless quadrupole */
} rb_tree_host;

/* Opaque context: owns the GPU workspace of one system or one batch. */
typedef struct rb_ctx rb_ctx;

/* Per-call interaction counts of the last walk (profile = 1). */
typedef struct {
  int64_t open_tests;   /* opening-criterion evaluations */
  int64_t cells;        /* accepted multi-particle cells */
  int64_t pp;           /* particle-particle terms */
  int64_t list_cells;   /* FP32-mixed: cell entries evaluated (all lanes) */
  int64_t list_pp;      /* FP32-mixed: particle entries evaluated */
  double ms[16];        /* phase times in ms (see rb_phase_name) */
  int64_t calls[16];    /* timed intervals per phase (e.g. walk launches) */
  int64_t reused_steps; /* steps that kept the last tree (reuse_topology) */
} rb_stats_t;

/* Defaults: theta 0.5, leaf 1, group 64, open box [-64, 64)^3, monopole. */
void rb_params_default(rb_params *p);

/*
 * Create a context for one system of up to `capacity` particles on the
 * current HIP device, issuing work on `hip_stream` (a hipStream_t; NULL =
 * the null stream).  Allocates all workspace (about 0.6 kB per particle).
 * Errors: RB_EINVAL for invalid parameters (see rb_params), RB_ENOMEM,
 * RB_EUNSUPPORTED (n_ghost > 2).
 */
int rb_create(rb_ctx **ctx, const rb_params *p, int64_t capacity, void *hip_stream);

/*
 * Create a context for a batch of independent systems (shearing-sheet
 * patches; Sect. 2.3 builds one tree per root box).  Patch k owns the
 * caller slots [offsets[k], offsets[k+1]) of every particle array; its root
 * box is box_size[k], box_min[3k..3k+2]; all other parameters are shared.
 * offsets, box_size and box_min are HOST arrays copied at creation.
 */
int rb_batch_create(rb_ctx **ctx, const rb_params *p, int32_t n_patch,
                    const int64_t *offsets, const double *box_size,
                    const double *box_min, void *hip_stream);

int rb_destroy(rb_ctx *ctx);

/* Replace theta, quadrupole, precision, leaf_size, group_size, split_images,
 * softening, G and profile of an existing context (box and boundary fixed). */
int rb_set_params(rb_ctx *ctx, const rb_params *p);

/*
 * Build the octree of Sect. 4.2 for the n caller particles: Morton keys of
 * the quantised positions q = floor((x - box_min) 2^21 / box_size), stable
 * radix sort, canonical level-ordered topology, bottom-up mass, centre of
 * mass and quadrupole.  Particles with index >= n_active are massless test
 * particles (Sect. 4).  For a batch context n_active is ignored and all
 * particles are massive.  Errors: RB_EINVAL (null, n > capacity or, for a
 * batch, n != total), deferred RB_ECAPACITY / RB_EOUTSIDE.
 */
int rb_tree_build(rb_ctx *ctx, const rb_particles *p, int64_t n, int64_t n_active);

/* Synchronise; report the node and live-particle counts of the last tree
 * (for a batch: totals). */
int rb_tree_info(rb_ctx *ctx, int64_t *n_nodes, int64_t *n_live);

/* Synchronise and copy the last tree to host buffers (single system or
 * patch `patch` of a batch; node indices are patch-local).  The last tree
 * must come from rb_tree_build, rb_gravity or an FP64 step: an FP32-mixed
 * step keeps FP64 moments only where its build needs them, and rb_collide /
 * rb_sweep reuse the tree's buffers; then RB_EUNSUPPORTED. */
int rb_tree_export(rb_ctx *ctx, int32_t patch, rb_tree_host *out);

/*
 * Accelerations of Eq. (1) approximated by the tree walk of Sect. 4.2, with
 * the ghost images of Sect. 2.3 at time t (shear offset
 * remainder(1.5 omega W t, W)).  Builds the tree first.  ax, ay, az are
 * device arrays of n entries in caller order.  FP64 precision reproduces
 * the opening decisions of a plain per-particle walk; FP32-mixed uses the
 * grouped walk.  n_active as in rb_tree_build.
 */
int rb_gravity(rb_ctx *ctx, const rb_particles *p, int64_t n, int64_t n_active,
               double t, double *ax, double *ay, double *az);

/*
 * Eq. (1) by direct summation (Sect. 4.1) for n_targets caller indices
 * `targets` (device int64), over all n sources and ghost images at time t.
 * FP64.  Outputs a*[k] for target k (device arrays of n_targets).
 */
int rb_direct(rb_ctx *ctx, const rb_particles *p, int64_t n, int64_t n_active,
              double t, const int64_t *targets, int64_t n_targets, double *ax,
              double *ay, double *az);

/*
 * rb_direct without a context, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same sum, with the same kernels, for a single
 * system described by p (box, boundary, ghost rings, omega, G, softening;
 * theta and the tree fields are ignored), issued on hip_stream (a
 * hipStream_t; NULL = the null stream).  It calls no hipMalloc, hipFree or
 * allocating library routine: the per-chunk partial sums live in a fixed
 * array of 8 MiB per GPU (2^20 doubles, 3 per target and source chunk),
 * which the library holds on every GPU it runs on until the process ends.
 * Every call on one GPU shares that array, so calls that overlap on one GPU
 * (other streams, other threads) race; calls issued one after another on
 * one stream do not.  Asynchronous; nothing is synchronised and no device
 * error word exists: a target index outside [0, n) gets zero acceleration.
 * Errors (host-side, nothing launched): RB_EINVAL for invalid parameters,
 * null arrays, n outside [0, 2^31 - 1], n_targets outside [0, n] or above
 * 349,525 (what the fixed array holds for one source chunk), RB_EHIP.
 */
int rb_direct_noalloc(const rb_params *p, const rb_particles *parts, int64_t n,
                      int64_t n_active, double t, const int64_t *targets, int64_t n_targets,
                      double *ax, double *ay, double *az, void *hip_stream);

/*
 * nsteps drift-kick-drift steps of Sect. 3 from time t with step dt: drift
 * dt/2 (leap-frog or epicycle), boundaries, tree gravity at t + dt/2, kick
 * v += a dt, drift dt/2, boundaries.  Updates x, y, z, vx, vy, vz in place,
 * keeping the caller's order; m is read only.
 */
int rb_step(rb_ctx *ctx, rb_particles *p, int64_t n, int64_t n_active, double t,
            double dt, int32_t nsteps);

/* Batch forms: every patch steps / gets forces independently, one launch
 * per kernel for all patches (work items ordered by patch cost). */
int rb_batch_step(rb_ctx *ctx, rb_particles *p, double t, double dt, int32_t nsteps);
int rb_batch_gravity(rb_ctx *ctx, const rb_particles *p, double t, double *ax,
                     double *ay, double *az);

/*
 * Collisions at the end of a step (Sect. 5 of the paper), at time t with the
 * positions and velocities of p (caller order, device): builds the octree
 * and finds every pair of live particles i < j (caller indices) that
 * overlap through ghost image k of j, |x_j + o_k - x_i| < R_i + R_j, by the
 * tree search of Eq. (3) (descend while the distance to the cell centre is
 * below R_i + R_max + (sqrt 3 / 2) w).  The pairs form a queue in the order
 * of ascending splitmix64(seed + code), code = i 2^35 + j 2^7 + k (images
 * numbered as for gravity, ix outer, iy inner); a queued pair that is
 * approaching at its turn (d . u < 0, relative velocity u including the
 * image's shear velocity -3/2 omega W ix) is resolved as free-slip hard
 * spheres: the normal relative velocity becomes -epsilon times itself, the
 * tangential one is kept, momentum is conserved.  vx, vy, vz change in
 * place; x, y, z do not.
 *  radius     device FP64, n entries, caller order.
 *  epsilon    coefficient of restitution in [0, 1].
 *  seed       any 64-bit value; the caller varies it from step to step.
 *  n_pairs, n_resolved  host outputs (may be NULL): pairs found, pairs
 *             resolved.
 *  codes, codes_cap     optional host buffer for the found codes (in no
 *             particular order; NULL / 0 to skip).
 * For a batch context n is the total and pairs stay inside their patches.
 * Synchronises.  Errors: RB_EINVAL (null pointer, epsilon, n), RB_EUNSUPPORTED
 * (capacity >= 2^28, or node capacity >= 2^27), RB_ECAPACITY (more than 8
 * pairs per particle), and the deferred errors of the tree build.  Phase
 * times: "coll_search" is the search kernel, "collide" the rest (R_max, cell
 * records, work items, resolution rounds).
 */
int rb_collide(rb_ctx *ctx, rb_particles *p, const double *radius, int64_t n, double t,
               double epsilon, uint64_t seed, int64_t *n_pairs, int64_t *n_resolved,
               uint64_t *codes, int64_t codes_cap);

/*
 * Collisions inside rb_step / rb_batch_step (Sect. 5): with enable != 0,
 * every step ends with the collision search of rb_collide on the step's own
 * tree (the one built for its kick, searched with every cell's reach
 * widened by the largest displacement since the build, across the periodic
 * wraps of the second drift) and the resolution of its queue, before the
 * next step's first drift.  The pairs, their queue order and the velocity
 * changes are those rb_collide finds and makes on the end-of-step state.
 * The k-th step run since this call uses the seed seed + k.
 *  radius     device FP64, caller order; kept by reference: the caller keeps
 *             it alive and unchanged while collisions are on.
 *  epsilon    coefficient of restitution in [0, 1].
 * enable = 0 turns them off.  Captured step graphs are captured again.
 * Errors: RB_EINVAL, RB_EUNSUPPORTED (2^27 nodes or more), RB_EHIP.
 */
int rb_set_collisions(rb_ctx *ctx, const double *radius, double epsilon, uint64_t seed,
                      int32_t enable);

/* Synchronise; the pairs found and the collisions resolved by the steps
 * since the last call (or since rb_set_collisions), then reset them. */
int rb_collision_counts(rb_ctx *ctx, int64_t *n_pairs, int64_t *n_resolved);

/* rb_sweep's axis: along x, or along the azimuth around the z axis */
enum { RB_SWEEP_X = 0, RB_SWEEP_PHI = 1 };

/*
 * Collisions found by the plane sweep (Sect. 5 of the paper), along x or
 * along the azimuthal angle phi = atan2(y, x) measured around the z axis
 * through the origin, for a single system (not a batch context), at time t
 * after a time-step dt >= 0.
 * Each particle's trajectory over the step is the straight line through its
 * present position with its present velocity, x + v sigma for sigma in
 * [-dt, 0].  Live particles i < j (caller indices) and ghost image k of j
 * (numbered as for gravity; the image moves with the shear velocity
 * -3/2 omega W ix) collide when those lines come closer than R_i + R_j: in
 * contact now, or, for a pair now separating, at their closest approach
 * within the step.  The intervals that the trajectories (widened by the
 * radii) cover along the axis are sorted, and each is checked against the
 * ones it overlaps, also across the periodic x boundary, or across phi =
 * +-pi.  The found set does not depend on the axis.  The collisions form
 * the same queue (ascending splitmix64(seed + code)) and are resolved as
 * by rb_collide: only pairs approaching now are resolved, so a pair that
 * met during the step and is now separating is found but left as it is.
 *  radius, epsilon, seed, n_pairs, n_resolved, codes, codes_cap: as for
 *             rb_collide.
 *  dt         the time-step the trajectories span; 0 finds exactly the
 *             pairs that rb_collide finds.
 *  axis       RB_SWEEP_X (any boundary) or RB_SWEEP_PHI (open box only:
 *             narrow rings in global simulations).
 * Synchronises.  Errors: RB_EINVAL (null pointer, epsilon, dt, n, axis),
 * RB_EUNSUPPORTED (batch context, phi without an open box, capacity >=
 * 2^28), RB_ECAPACITY (more
 * than 8 pairs per particle), RB_EOUTSIDE (a particle outside a periodic or
 * shear axis).  The context's tree is not kept (the sort reuses its
 * buffers).  Phase times: "coll_search" is the sweep, "collide" the
 * resolution rounds.
 */
int rb_sweep(rb_ctx *ctx, rb_particles *p, const double *radius, int64_t n, double t,
             double dt, int32_t axis, double epsilon, uint64_t seed, int64_t *n_pairs,
             int64_t *n_resolved, uint64_t *codes, int64_t codes_cap);

/*
 * Measured ceilings of the current GPU, for the rooflines (diagnostics, not
 * part of any step): kind 0 = FP32 vector FMA rate as this library compiles
 * FP32 (unpacked), 1 = FP64 vector FMA rate (flop/s, an FMA counting 2),
 * 2 = HBM rate of a 2 GiB streaming copy (bytes read + written per s).
 * Best of four timed launches on the null stream; allocates and frees its
 * own buffers (4 GiB for kind 2).  Synchronises.  Errors: RB_EINVAL (kind,
 * null value), RB_EHIP.
 */
int rb_peak_probe(int32_t kind, double *value);

/* Synchronise the context's stream and return any deferred device error. */
int rb_sync(rb_ctx *ctx);

/* Synchronise and return counts and phase times of the last call
 * (profile = 1; zeros otherwise). */
int rb_stats(rb_ctx *ctx, rb_stats_t *out);
const char *rb_phase_name(int32_t phase);

/*
 * Checkpoint: write n particles (device SoA) plus t and the parameters to a
 * binary file / read them back.  rb_state_load fills caller device arrays
 * and *t; it fails with RB_EIO on a missing, short or foreign file and with
 * RB_EINVAL if n differs.  Both synchronise.
 */
int rb_state_save(rb_ctx *ctx, const rb_particles *p, int64_t n, double t,
                  const char *path);
int rb_state_load(rb_ctx *ctx, rb_particles *p, int64_t n, double *t,
                  const char *path);

const char *rb_error_string(int code);
const char *rb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
