/*
 * rb_oracle.h -- plain CPU FP64 oracle for Barnes-Hut tree self-gravity.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library includes, links or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load the shared object built from rb_oracle.c.  It shares
 * no code, header, table or constant with the GPU path.
 *
 * What it computes (paper sections cited per function in rb_oracle.c):
 *   - Eq. (1): the Plummer-softened pairwise acceleration over N_active massive
 *     particles, summed over the ghost-box images (Sect. 2.3, Sect. 4, 4.1);
 *   - the Barnes-Hut octree of Sect. 4.2, built by one-at-a-time insertion,
 *     with bottom-up mass / centre of mass and Hernquist quadrupole moments,
 *     one tree per cubic root box of the domain (Sect. 2.3), and its
 *     reconstruction after the particles moved (Sect. 4.2);
 *   - the per-particle tree walk with opening angle theta = w/R;
 *   - the drift-kick-drift step of Sect. 3 with the leap-frog drift (3.1) or
 *     the exact epicycle drift used by the symplectic epicycle integrator (3.3);
 *   - the collisions of Sect. 5: overlapping pairs at the end of a step, a
 *     randomly ordered queue, hard-sphere resolution with restitution.
 */
#ifndef RB_ORACLE_H
#define RB_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OPEN = 0, ORC_PERIODIC = 1, ORC_SHEAR = 2 };
enum { ORC_LEAPFROG = 0, ORC_EPICYCLE = 1 };

typedef struct {
  double G;          /* gravitational constant */
  double b;          /* Plummer softening length */
  double theta;      /* critical opening angle */
  int32_t quadrupole;/* 0: monopole only, 1: add the quadrupole term */
  int32_t n_leaf;    /* max particles per leaf above the deepest level (paper: 1) */
  double W;          /* side of each cubic root box */
  double x0[3];      /* minimum corner of the domain (of root box 0) */
  int32_t boundary;  /* ORC_OPEN / ORC_PERIODIC / ORC_SHEAR */
  int32_t ng[2];     /* ghost rings in x and y (periodic / shear only) */
  int32_t drift;     /* ORC_LEAPFROG / ORC_EPICYCLE */
  double omega;      /* orbital frequency (shear offset, epicycle drift) */
  double omega_z;    /* vertical epicycle frequency */
  int32_t n_root[3]; /* root boxes per axis (Sect. 2.3); 0 or 1 = one box */
} orc_params;

typedef struct orc_tree orc_tree;

/* keys (UINT64_MAX for a particle outside the domain or with a NaN coordinate) */
void orc_keys(const orc_params *p, int64_t n, const double *x, const double *y,
              const double *z, uint64_t *keys);

orc_tree *orc_tree_build(const orc_params *p, int64_t n, int64_t n_active,
                         const double *x, const double *y, const double *z,
                         const double *m);
/* Tree reconstruction of Sect. 4.2 after the particles moved to x, y, z
 * (same particles, same masses): every particle that left the cell of its
 * leaf (or the domain) is taken out and inserted again; cells left empty
 * are destroyed and cells left with at most n_leaf particles become leaves
 * again; then the moments are updated bottom-up.  Returns the number of
 * particles re-inserted.                                                  */
int64_t orc_tree_update(orc_tree *t, const double *x, const double *y, const double *z);
void orc_tree_free(orc_tree *t);
int64_t orc_tree_n_nodes(const orc_tree *t);
int64_t orc_tree_n_live(const orc_tree *t);
/* 1 when the DFS leaf order equals the stable sort of the keys */
int orc_tree_selfcheck(const orc_tree *t);
/* canonical export: nodes level by level, by prefix inside a level */
void orc_tree_export(const orc_tree *t, int8_t *level, uint64_t *prefix,
                     int64_t *first, int64_t *count, int8_t *is_leaf,
                     int32_t *n_child, int64_t *first_child, double *M,
                     double *com /* 3 per node */, double *Q /* 6 per node */,
                     int64_t *perm /* n_live */, uint64_t *sorted_keys);

/* tree walk for the listed targets (all particles when targets == NULL);
 * stats[0] opening tests, [1] accepted multi-particle cells,
 * [2] particle-particle terms (single leaves and opened bucket members). */
void orc_bh(const orc_params *p, const orc_tree *t, int64_t n, const double *x,
            const double *y, const double *z, double s, const int64_t *targets,
            int64_t nt, double *ax, double *ay, double *az, int64_t *stats);

void orc_direct(const orc_params *p, int64_t n, int64_t n_active, const double *x,
                const double *y, const double *z, const double *m, double s,
                const int64_t *targets, int64_t nt, double *ax, double *ay,
                double *az);

double orc_shear_offset(const orc_params *p, double t);
void orc_drift(const orc_params *p, int64_t n, double *x, double *y, double *z,
               double *vx, double *vy, double *vz, double tau);
void orc_boundary(const orc_params *p, int64_t n, double *x, double *y, double *z,
                  double *vx, double *vy, double *vz, double s);
/* nsteps DKD steps from t0; use_tree 1 = Barnes-Hut kick, 0 = direct kick */
void orc_step(const orc_params *p, int64_t n, int64_t n_active, double *x,
              double *y, double *z, double *vx, double *vy, double *vz,
              const double *m, double t0, double dt, int32_t nsteps,
              int32_t use_tree);
double orc_energy(const orc_params *p, int64_t n, int64_t n_active,
                  const double *x, const double *y, const double *z,
                  const double *vx, const double *vy, const double *vz,
                  const double *m);
int orc_num_threads(void);

/* Collisions at the end of a step (Sect. 5): detects every overlapping pair
 * (i < j, ghost image k of j), orders the queue by splitmix64(seed + code)
 * with code = i 2^35 + j 2^7 + k, resolves the approaching ones in that
 * order (hard spheres, restitution eps), updating v in place.  Writes the
 * first `cap` codes in queue order; returns the number of pairs and sets
 * *n_resolved.  s is the shear offset of the ghost boxes.                  */
uint64_t orc_splitmix64(uint64_t x);
int64_t orc_collide(const orc_params *p, int64_t n, const double *x, const double *y,
                    const double *z, double *vx, double *vy, double *vz, const double *m,
                    const double *R, double s, double eps, uint64_t seed, uint64_t *codes,
                    int64_t cap, int64_t *n_resolved);
/* The same with the pairs the plane sweep finds (Sect. 5): i and image k of
 * j whose straight trajectories over the past time-step dt (through the
 * present positions, with the present velocities, the image's shear
 * velocity included) come closer than R_i + R_j.                          */
int64_t orc_sweep(const orc_params *p, int64_t n, const double *x, const double *y,
                  const double *z, double *vx, double *vy, double *vz, const double *m,
                  const double *R, double s, double dt, double eps, uint64_t seed,
                  uint64_t *codes, int64_t cap, int64_t *n_resolved);

#ifdef __cplusplus
}
#endif
#endif
