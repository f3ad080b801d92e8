/*
 * rb_oracle.c -- plain, slow, CPU FP64 oracle for Barnes-Hut tree gravity.
 *
 * TEST INFRASTRUCTURE ONLY: the GPU library never includes, links or calls
 * this file.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no code with the GPU path.
 *
 * Built with -ffp-contract=off: every product and sum below is rounded on its
 * own unless fma() is written out.  The opening test uses an explicit fma()
 * chain for R^2 so that its rounding is fixed by the source text.
 *
 * Readings of points the paper leaves open (see the module docs):
 *  - Eq. (1) is read as the softened Newtonian sum with the vector
 *    r_ji = x_j - x_i in the numerator (the printed unit vector over
 *    (r^2+b^2)^{3/2} is not dimensionally consistent).
 *  - Only the pair (j = i, image 0) is excluded; a particle's own ghost images
 *    are summed.
 *  - Octants come from integer quantised coordinates, not from comparing x
 *    with floating-point cell centres.
 *  - A leaf holds at most n_leaf particles unless it sits on the deepest level
 *    (21), where leaves collect every particle with the same key.
 *  - Mass and centre of mass are kept as M = sum m and S = sum m x, summed in
 *    octant order at internal nodes and in Morton order inside leaves; the
 *    centre of mass is S / M.  A single-particle leaf uses x_j itself.
 *  - A node is accepted when w^2 < theta^2 R^2 (strict), R measured from the
 *    image-shifted target to the node's centre of mass.
 */
#include "rb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_DEPTH 21
#define ORC_NONE (-1)

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Domain (Sect. 2.3): n_root[a] cubic root boxes of side W along axis a,
 * from the corner x0.  A single box when every n_root is 0 or 1.           */

static int orc_nr(const orc_params *p, int a) {
  return p->n_root[a] > 1 ? p->n_root[a] : 1;
}

/* domain extent along axis a */
static double orc_L(const orc_params *p, int a) { return (double)orc_nr(p, a) * p->W; }

/* root boxes per axis in powers of two: 2^D >= every n_root */
static int orc_D(const orc_params *p) {
  int m = orc_nr(p, 0);
  if (orc_nr(p, 1) > m) m = orc_nr(p, 1);
  if (orc_nr(p, 2) > m) m = orc_nr(p, 2);
  int D = 0;
  while ((1 << D) < m) ++D;
  return D;
}

/* ------------------------------------------------------------------------ */
/* Keys.  Sect. 4.2: every cell splits into eight cubic sub-cells of half the
 * width.  The domain is quantised once, 2^(21-D) steps per root box per
 * axis: q = floor((x - x0) * 2^(21-D) / W).  The root box of a particle is
 * the integer part q >> (21-D) and its cell inside that box the low bits;
 * both are read from the bits of q, never by comparing x with a floating-
 * point boundary.  The key interleaves the 21 bits of q per axis (x bit
 * weighing 4, y 2, z 1, most significant level first): its first D digits
 * name the root box, the rest the cells of the root box's own tree at
 * levels D+1..21 (level D is the root box itself).  With one root box
 * (D = 0) this is q = floor((x - x0) 2^21 / W).                             */

static int orc_quantise(const orc_params *p, double S, double xa, int a,
                        uint32_t *q) {
  double u = xa - p->x0[a];
  if (!(u >= 0.0 && u < orc_L(p, a))) return 0; /* outside, or NaN */
  double f = floor(u * S);
  double top = (double)orc_nr(p, a) * ldexp(1.0, ORC_DEPTH - orc_D(p)) - 1.0;
  if (f >= top) f = top; /* u*S may round up to the domain's end */
  *q = (uint32_t)f;
  return 1;
}

static uint64_t orc_key_of(const orc_params *p, double S, double x, double y,
                           double z) {
  uint32_t q[3];
  if (!orc_quantise(p, S, x, 0, &q[0]) || !orc_quantise(p, S, y, 1, &q[1]) ||
      !orc_quantise(p, S, z, 2, &q[2]))
    return UINT64_MAX;
  uint64_t key = 0;
  for (int l = 1; l <= ORC_DEPTH; ++l) {
    int bit = ORC_DEPTH - l;
    uint64_t o = (uint64_t)((q[0] >> bit) & 1u) * 4u +
                 (uint64_t)((q[1] >> bit) & 1u) * 2u +
                 (uint64_t)((q[2] >> bit) & 1u);
    key = key * 8u + o;
  }
  return key;
}

static double orc_S(const orc_params *p) {
  return (double)(1u << (ORC_DEPTH - orc_D(p))) / p->W;
}

void orc_keys(const orc_params *p, int64_t n, const double *x, const double *y,
              const double *z, uint64_t *keys) {
  double S = orc_S(p);
  for (int64_t i = 0; i < n; ++i) keys[i] = orc_key_of(p, S, x[i], y[i], z[i]);
}

static int orc_digit(uint64_t key, int level) {
  return (int)((key >> (3 * (ORC_DEPTH - level))) & 7u);
}

/* ------------------------------------------------------------------------ */
/* One octree per root box (Sect. 2.3), each built by inserting particles
 * one at a time (Sect. 4.2).  Node levels are counted from the domain: the
 * tree of a root box has its root at level D, and a node at level l is a
 * cube of side W 2^(D-l).                                                   */

typedef struct {
  uint64_t prefix;
  int32_t child[8];
  int64_t head, tail, nmem; /* leaf member list in insertion order */
  int8_t level, leaf;
  double M, S[3], com[3], Q[6];
  int64_t first, count; /* Morton-rank range of the subtree */
  int32_t n_child;
} onode;

struct orc_tree {
  orc_params p;
  int D;             /* levels above the root boxes */
  int64_t n, n_active, n_live;
  onode *nodes;
  int64_t n_nodes, cap;
  int64_t *roots;    /* node of every occupied root box, by root prefix */
  int64_t n_roots;
  int64_t *next;     /* member list links */
  int64_t *leaf_of;  /* leaf node holding each particle, -1 if none */
  uint64_t *keys;
  int64_t *perm;     /* Morton rank -> particle index */
  double *x, *y, *z, *msrc; /* own copies; msrc = 0 for test particles */
  double w2[ORC_DEPTH + 1];
  int ok;
};

static int64_t orc_new_node(orc_tree *t, int level, uint64_t prefix) {
  if (t->n_nodes == t->cap) {
    t->cap = t->cap ? 2 * t->cap : 1024;
    t->nodes = (onode *)realloc(t->nodes, (size_t)t->cap * sizeof(onode));
  }
  onode *nd = &t->nodes[t->n_nodes];
  memset(nd, 0, sizeof(*nd));
  nd->prefix = prefix;
  for (int c = 0; c < 8; ++c) nd->child[c] = ORC_NONE;
  nd->head = nd->tail = ORC_NONE;
  nd->level = (int8_t)level;
  nd->leaf = 1;
  return t->n_nodes++;
}

static void orc_append(orc_tree *t, int64_t node, int64_t j) {
  onode *nd = &t->nodes[node];
  t->next[j] = ORC_NONE;
  if (nd->tail == ORC_NONE) nd->head = j; else t->next[nd->tail] = j;
  nd->tail = j;
  nd->nmem++;
  t->leaf_of[j] = node;
}

static void orc_add(orc_tree *t, int64_t node, int64_t j);

static void orc_add_child(orc_tree *t, int64_t node, int64_t j) {
  int level = t->nodes[node].level + 1;
  int o = orc_digit(t->keys[j], level);
  if (t->nodes[node].child[o] == ORC_NONE) {
    uint64_t pre = t->nodes[node].prefix * 8u + (uint64_t)o;
    int64_t c = orc_new_node(t, level, pre); /* may move t->nodes */
    t->nodes[node].child[o] = (int32_t)c;
  }
  orc_add(t, t->nodes[node].child[o], j);
}

static void orc_add(orc_tree *t, int64_t node, int64_t j) {
  onode *nd = &t->nodes[node];
  if (!nd->leaf) { orc_add_child(t, node, j); return; }
  if (nd->nmem < t->p.n_leaf || nd->level == ORC_DEPTH) {
    orc_append(t, node, j);
    return;
  }
  /* the leaf is full: it becomes an internal node and its particles move
   * one level down, followed by the new one */
  int64_t k = nd->head;
  nd->leaf = 0;
  nd->head = nd->tail = ORC_NONE;
  nd->nmem = 0;
  while (k != ORC_NONE) {
    int64_t nxt = t->next[k];
    orc_add_child(t, node, k);
    k = nxt;
  }
  orc_add_child(t, node, j);
}

/* the tree of particle j's root box (created with its first particle) */
static int64_t orc_root_of(orc_tree *t, int64_t j) {
  uint64_t pre = t->keys[j] >> (3 * (ORC_DEPTH - t->D));
  int64_t lo = 0, hi = t->n_roots;
  while (lo < hi) { /* first root with prefix >= pre */
    int64_t mid = (lo + hi) / 2;
    if (t->nodes[t->roots[mid]].prefix < pre) lo = mid + 1; else hi = mid;
  }
  if (lo < t->n_roots && t->nodes[t->roots[lo]].prefix == pre) return t->roots[lo];
  int64_t r = orc_new_node(t, t->D, pre);
  memmove(t->roots + lo + 1, t->roots + lo, (size_t)(t->n_roots - lo) * sizeof(int64_t));
  t->roots[lo] = r;
  t->n_roots++;
  return r;
}

static void orc_insert(orc_tree *t, int64_t j) { orc_add(t, orc_root_of(t, j), j); }

/* Morton ranks by depth-first traversal in octant order, root boxes in the
 * order of their prefixes.  Leaf members are ranked by (key, index), i.e.
 * the stable sort of the keys.                                              */
static int64_t orc_rank(orc_tree *t, int64_t node, int64_t r) {
  onode *nd = &t->nodes[node];
  nd->first = r;
  if (nd->leaf) {
    int64_t c = 0;
    for (int64_t k = nd->head; k != ORC_NONE; k = t->next[k]) t->perm[r + c++] = k;
    /* insertion sort by (key, index) */
    for (int64_t a = 1; a < c; ++a) {
      int64_t v = t->perm[r + a], b = a - 1;
      while (b >= 0 && (t->keys[t->perm[r + b]] > t->keys[v] ||
                        (t->keys[t->perm[r + b]] == t->keys[v] && t->perm[r + b] > v))) {
        t->perm[r + b + 1] = t->perm[r + b];
        --b;
      }
      t->perm[r + b + 1] = v;
    }
    nd->count = c;
    nd->n_child = 0;
    return r + c;
  }
  int64_t r0 = r;
  int nc = 0;
  for (int o = 0; o < 8; ++o) {
    int32_t c = t->nodes[node].child[o];
    if (c != ORC_NONE) { r = orc_rank(t, c, r); ++nc; }
  }
  t->nodes[node].count = r - r0;
  t->nodes[node].n_child = nc;
  return r;
}

/* Bottom-up moments (Sect. 4.2: total mass and centre of mass updated from
 * the bottom up; quadrupole tensor after Hernquist 1987).  Traceless
 * Q_jk = sum m (3 s_j s_k - |s|^2 delta_jk), s relative to the centre of mass;
 * internal nodes combine children with the parallel-axis shift.            */
static double orc_msrc(const orc_tree *t, int64_t j) { return t->msrc[j]; }

static void orc_moments(orc_tree *t, int64_t node) {
  onode *nd = &t->nodes[node];
  double M = 0.0, S[3] = {0.0, 0.0, 0.0}, Q[6] = {0, 0, 0, 0, 0, 0}, com[3];
  if (nd->leaf) {
    for (int64_t r = nd->first; r < nd->first + nd->count; ++r) {
      int64_t j = t->perm[r];
      double mj = orc_msrc(t, j);
      M = M + mj;
      S[0] = S[0] + mj * t->x[j];
      S[1] = S[1] + mj * t->y[j];
      S[2] = S[2] + mj * t->z[j];
    }
    if (M == 0.0) {
      com[0] = com[1] = com[2] = 0.0;
    } else if (nd->count == 1) {
      int64_t j = t->perm[nd->first];
      com[0] = t->x[j]; com[1] = t->y[j]; com[2] = t->z[j];
    } else {
      com[0] = S[0] / M; com[1] = S[1] / M; com[2] = S[2] / M;
      for (int64_t r = nd->first; r < nd->first + nd->count; ++r) {
        int64_t j = t->perm[r];
        double mj = orc_msrc(t, j);
        double s0 = t->x[j] - com[0], s1 = t->y[j] - com[1], s2 = t->z[j] - com[2];
        double ss = s0 * s0 + s1 * s1 + s2 * s2;
        Q[0] += mj * (3.0 * s0 * s0 - ss);
        Q[1] += mj * (3.0 * s0 * s1);
        Q[2] += mj * (3.0 * s0 * s2);
        Q[3] += mj * (3.0 * s1 * s1 - ss);
        Q[4] += mj * (3.0 * s1 * s2);
        Q[5] += mj * (3.0 * s2 * s2 - ss);
      }
    }
  } else {
    for (int o = 0; o < 8; ++o) {
      int32_t c = t->nodes[node].child[o];
      if (c == ORC_NONE) continue;
      orc_moments(t, c);
    }
    nd = &t->nodes[node];
    for (int o = 0; o < 8; ++o) {
      int32_t c = nd->child[o];
      if (c == ORC_NONE) continue;
      const onode *ch = &t->nodes[c];
      M = M + ch->M;
      S[0] = S[0] + ch->S[0];
      S[1] = S[1] + ch->S[1];
      S[2] = S[2] + ch->S[2];
    }
    if (M == 0.0) {
      com[0] = com[1] = com[2] = 0.0;
    } else {
      com[0] = S[0] / M; com[1] = S[1] / M; com[2] = S[2] / M;
    }
    for (int o = 0; o < 8; ++o) {
      int32_t c = nd->child[o];
      if (c == ORC_NONE) continue;
      const onode *ch = &t->nodes[c];
      double d0 = ch->com[0] - com[0], d1 = ch->com[1] - com[1], d2 = ch->com[2] - com[2];
      double dd = d0 * d0 + d1 * d1 + d2 * d2;
      Q[0] += ch->Q[0] + ch->M * (3.0 * d0 * d0 - dd);
      Q[1] += ch->Q[1] + ch->M * (3.0 * d0 * d1);
      Q[2] += ch->Q[2] + ch->M * (3.0 * d0 * d2);
      Q[3] += ch->Q[3] + ch->M * (3.0 * d1 * d1 - dd);
      Q[4] += ch->Q[4] + ch->M * (3.0 * d1 * d2);
      Q[5] += ch->Q[5] + ch->M * (3.0 * d2 * d2 - dd);
    }
  }
  nd->M = M;
  for (int a = 0; a < 3; ++a) { nd->S[a] = S[a]; nd->com[a] = com[a]; }
  for (int a = 0; a < 6; ++a) nd->Q[a] = Q[a];
}

/* Morton ranks and moments of every root box's tree */
static void orc_finish(orc_tree *t) {
  int64_t r = 0;
  for (int64_t k = 0; k < t->n_roots; ++k) r = orc_rank(t, t->roots[k], r);
  for (int64_t k = 0; k < t->n_roots; ++k) orc_moments(t, t->roots[k]);
}

static void orc_set_positions(orc_tree *t, const double *x, const double *y,
                              const double *z) {
  for (int64_t j = 0; j < t->n; ++j) { t->x[j] = x[j]; t->y[j] = y[j]; t->z[j] = z[j]; }
  orc_keys(&t->p, t->n, x, y, z, t->keys);
  t->n_live = 0;
  for (int64_t j = 0; j < t->n; ++j) t->n_live += (t->keys[j] != UINT64_MAX);
}

orc_tree *orc_tree_build(const orc_params *p, int64_t n, int64_t n_active,
                         const double *x, const double *y, const double *z,
                         const double *m) {
  orc_tree *t = (orc_tree *)calloc(1, sizeof(orc_tree));
  t->p = *p;
  t->D = orc_D(p);
  t->n = n;
  t->n_active = n_active;
  size_t n1 = (size_t)(n > 0 ? n : 1);
  t->x = (double *)malloc(n1 * sizeof(double)); t->y = (double *)malloc(n1 * sizeof(double));
  t->z = (double *)malloc(n1 * sizeof(double)); t->msrc = (double *)malloc(n1 * sizeof(double));
  for (int64_t j = 0; j < n; ++j) t->msrc[j] = (j < n_active) ? m[j] : 0.0;
  t->keys = (uint64_t *)malloc(n1 * sizeof(uint64_t));
  t->next = (int64_t *)malloc(n1 * sizeof(int64_t));
  t->leaf_of = (int64_t *)malloc(n1 * sizeof(int64_t));
  t->perm = (int64_t *)malloc(n1 * sizeof(int64_t));
  size_t nr = (size_t)orc_nr(p, 0) * (size_t)orc_nr(p, 1) * (size_t)orc_nr(p, 2);
  t->roots = (int64_t *)malloc(nr * sizeof(int64_t));
  for (int64_t j = 0; j < n; ++j) t->leaf_of[j] = ORC_NONE;
  orc_set_positions(t, x, y, z);
  for (int l = 0; l <= ORC_DEPTH; ++l) {
    double w = ldexp(p->W, t->D - l);
    t->w2[l] = w * w;
  }
  for (int64_t j = 0; j < n; ++j)
    if (t->keys[j] != UINT64_MAX) orc_insert(t, j);
  orc_finish(t);
  t->ok = 1;
  return t;
}

/* ------------------------------------------------------------------------ */
/* Reconstruction (Sect. 4.2).  A particle still inside the cell of its leaf
 * stays.  Any other one is taken out of its leaf; a leaf left empty is
 * destroyed, and so is every cell above it that holds nothing else; a cell
 * left with at most n_leaf particles becomes a leaf holding them (the tree
 * an insertion of the same particles would give, so that reconstruction
 * and a fresh build agree).  The particles taken out are then inserted
 * again from their root box, and the moments are recomputed bottom-up.     */

static void orc_unlink(orc_tree *t, int64_t leaf, int64_t j) {
  onode *nd = &t->nodes[leaf];
  int64_t prev = ORC_NONE;
  for (int64_t k = nd->head; k != ORC_NONE; prev = k, k = t->next[k]) {
    if (k != j) continue;
    if (prev == ORC_NONE) nd->head = t->next[k]; else t->next[prev] = t->next[k];
    if (nd->tail == k) nd->tail = prev;
    nd->nmem--;
    break;
  }
  t->leaf_of[j] = ORC_NONE;
}

/* particles in a subtree (leaf member counts summed) */
static int64_t orc_held(const orc_tree *t, int64_t node) {
  const onode *nd = &t->nodes[node];
  if (nd->leaf) return nd->nmem;
  int64_t c = 0;
  for (int o = 0; o < 8; ++o)
    if (nd->child[o] != ORC_NONE) c += orc_held(t, nd->child[o]);
  return c;
}

/* move every particle below `node` into `dst`'s member list */
static void orc_gather(orc_tree *t, int64_t node, int64_t dst) {
  onode *nd = &t->nodes[node];
  if (nd->leaf) {
    int64_t k = nd->head;
    while (k != ORC_NONE) {
      int64_t nxt = t->next[k];
      if (node != dst) orc_append(t, dst, k);
      k = nxt;
    }
    return;
  }
  for (int o = 0; o < 8; ++o)
    if (t->nodes[node].child[o] != ORC_NONE) orc_gather(t, t->nodes[node].child[o], dst);
}

/* after removals: returns 0 when the subtree is left empty (to be destroyed) */
static int orc_prune(orc_tree *t, int64_t node) {
  onode *nd = &t->nodes[node];
  if (nd->leaf) return nd->nmem > 0;
  int64_t held = orc_held(t, node);
  if (held == 0) return 0;
  if (held <= t->p.n_leaf) {
    /* collapse: the cell becomes a leaf with the particles below it */
    int32_t ch[8];
    for (int o = 0; o < 8; ++o) ch[o] = nd->child[o];
    nd->leaf = 1;
    nd->head = nd->tail = ORC_NONE;
    nd->nmem = 0;
    for (int o = 0; o < 8; ++o) t->nodes[node].child[o] = ORC_NONE;
    for (int o = 0; o < 8; ++o)
      if (ch[o] != ORC_NONE) orc_gather(t, ch[o], node);
    return 1;
  }
  for (int o = 0; o < 8; ++o) {
    int32_t c = t->nodes[node].child[o];
    if (c != ORC_NONE && !orc_prune(t, c)) t->nodes[node].child[o] = ORC_NONE;
  }
  return 1;
}

/* drop nodes no longer reachable from a root box; indices are renumbered */
static void orc_compact(orc_tree *t) {
  int64_t *map = (int64_t *)malloc((size_t)(t->n_nodes > 0 ? t->n_nodes : 1) * sizeof(int64_t));
  for (int64_t v = 0; v < t->n_nodes; ++v) map[v] = ORC_NONE;
  int64_t *stack = (int64_t *)malloc((size_t)(t->n_nodes > 0 ? t->n_nodes : 1) * sizeof(int64_t));
  int64_t live = 0;
  for (int64_t k = 0; k < t->n_roots; ++k) {
    int64_t sp = 0;
    stack[sp++] = t->roots[k];
    while (sp > 0) {
      int64_t v = stack[--sp];
      map[v] = live++;
      for (int o = 0; o < 8; ++o)
        if (t->nodes[v].child[o] != ORC_NONE) stack[sp++] = t->nodes[v].child[o];
    }
  }
  onode *nn = (onode *)malloc((size_t)(live > 0 ? live : 1) * sizeof(onode));
  for (int64_t v = 0; v < t->n_nodes; ++v) {
    if (map[v] == ORC_NONE) continue;
    onode c = t->nodes[v];
    for (int o = 0; o < 8; ++o)
      if (c.child[o] != ORC_NONE) c.child[o] = (int32_t)map[c.child[o]];
    nn[map[v]] = c;
  }
  for (int64_t k = 0; k < t->n_roots; ++k) t->roots[k] = map[t->roots[k]];
  for (int64_t j = 0; j < t->n; ++j)
    if (t->leaf_of[j] != ORC_NONE) t->leaf_of[j] = map[t->leaf_of[j]];
  free(t->nodes);
  t->nodes = nn;
  t->n_nodes = live;
  t->cap = live > 0 ? live : 1;
  free(map);
  free(stack);
}

int64_t orc_tree_update(orc_tree *t, const double *x, const double *y, const double *z) {
  orc_set_positions(t, x, y, z);
  int64_t *moved = (int64_t *)malloc((size_t)(t->n > 0 ? t->n : 1) * sizeof(int64_t));
  int64_t n_moved = 0;
  for (int64_t j = 0; j < t->n; ++j) {
    int64_t lf = t->leaf_of[j];
    if (lf == ORC_NONE) continue; /* was outside: removed particles stay removed */
    const onode *nd = &t->nodes[lf];
    int stays = t->keys[j] != UINT64_MAX &&
                (t->keys[j] >> (3 * (ORC_DEPTH - nd->level))) == nd->prefix;
    if (stays) continue;
    orc_unlink(t, lf, j);
    if (t->keys[j] != UINT64_MAX) moved[n_moved++] = j;
  }
  /* destroy emptied cells, collapse cells left with few particles */
  int64_t kept = 0;
  for (int64_t k = 0; k < t->n_roots; ++k)
    if (orc_prune(t, t->roots[k])) t->roots[kept++] = t->roots[k];
  t->n_roots = kept;
  orc_compact(t);
  for (int64_t k = 0; k < n_moved; ++k) orc_insert(t, moved[k]);
  orc_finish(t);
  free(moved);
  return n_moved;
}

void orc_tree_free(orc_tree *t) {
  if (!t) return;
  free(t->nodes); free(t->next); free(t->leaf_of); free(t->keys); free(t->perm);
  free(t->roots);
  free(t->x); free(t->y); free(t->z); free(t->msrc);
  free(t);
}

int64_t orc_tree_n_nodes(const orc_tree *t) { return t->n_nodes; }
int64_t orc_tree_n_live(const orc_tree *t) { return t->n_live; }

int orc_tree_selfcheck(const orc_tree *t) {
  /* the DFS order must be sorted by (key, index) */
  for (int64_t r = 1; r < t->n_live; ++r) {
    uint64_t ka = t->keys[t->perm[r - 1]], kb = t->keys[t->perm[r]];
    if (ka > kb || (ka == kb && t->perm[r - 1] >= t->perm[r])) return 0;
  }
  return 1;
}

static const orc_tree *g_sort_tree; /* for the export's qsort */

static int orc_node_cmp(const void *a, const void *b) {
  const onode *na = &g_sort_tree->nodes[*(const int64_t *)a];
  const onode *nb = &g_sort_tree->nodes[*(const int64_t *)b];
  if (na->level != nb->level) return na->level < nb->level ? -1 : 1;
  if (na->prefix != nb->prefix) return na->prefix < nb->prefix ? -1 : 1;
  return 0;
}

/* canonical export: every root box's nodes together, level by level and by
 * prefix inside a level (so siblings are consecutive) */
void orc_tree_export(const orc_tree *t, int8_t *level, uint64_t *prefix,
                     int64_t *first, int64_t *count, int8_t *is_leaf,
                     int32_t *n_child, int64_t *first_child, double *M,
                     double *com, double *Q, int64_t *perm,
                     uint64_t *sorted_keys) {
  int64_t nn = t->n_nodes;
  if (nn == 0) return;
  int64_t *order = (int64_t *)malloc((size_t)nn * sizeof(int64_t));
  int64_t *pos = (int64_t *)malloc((size_t)nn * sizeof(int64_t));
  for (int64_t k = 0; k < nn; ++k) order[k] = k;
  g_sort_tree = t;
  qsort(order, (size_t)nn, sizeof(int64_t), orc_node_cmp);
  for (int64_t k = 0; k < nn; ++k) pos[order[k]] = k;
  for (int64_t k = 0; k < nn; ++k) {
    const onode *nd = &t->nodes[order[k]];
    level[k] = nd->level;
    prefix[k] = nd->prefix;
    first[k] = nd->first;
    count[k] = nd->count;
    is_leaf[k] = nd->leaf;
    n_child[k] = nd->n_child;
    first_child[k] = -1;
    for (int o = 0; o < 8; ++o)
      if (nd->child[o] != ORC_NONE) { first_child[k] = pos[nd->child[o]]; break; }
    M[k] = nd->M;
    for (int a = 0; a < 3; ++a) com[3 * k + a] = nd->com[a];
    for (int a = 0; a < 6; ++a) Q[6 * k + a] = nd->Q[a];
  }
  for (int64_t r = 0; r < t->n_live; ++r) {
    perm[r] = t->perm[r];
    sorted_keys[r] = t->keys[t->perm[r]];
  }
  free(order);
  free(pos);
}

/* ------------------------------------------------------------------------ */
/* Ghost images (Sect. 2.3: periodic and shear-periodic ghost boxes).  The
 * image of a source is x + o with o = (ix Lx, iy Ly - ix s, 0), ix outer and
 * iy inner, both in [-ng, ng]; Lx, Ly are the domain's extents (n_root W)
 * and s is the shear offset (0 for periodic boundaries).  Open boundaries
 * use the single image o = 0.                                               */

#define ORC_MAX_IMAGES 121

static int orc_images(const orc_params *p, double s, double (*o)[3], int *zero) {
  if (p->boundary == ORC_OPEN) {
    o[0][0] = o[0][1] = o[0][2] = 0.0;
    *zero = 0;
    return 1;
  }
  double sh = (p->boundary == ORC_SHEAR) ? s : 0.0;
  int k = 0;
  for (int ix = -p->ng[0]; ix <= p->ng[0]; ++ix)
    for (int iy = -p->ng[1]; iy <= p->ng[1]; ++iy) {
      double fx = (double)ix, fy = (double)iy;
      o[k][0] = fx * orc_L(p, 0);
      o[k][1] = fy * orc_L(p, 1) - fx * sh;
      o[k][2] = 0.0;
      if (ix == 0 && iy == 0) *zero = k;
      ++k;
    }
  return k;
}

/* Eq. (1) for one source: G m d / (|d|^2 + b^2)^{3/2}, d = x_j - x_i */
static void orc_pm(double G, double b2, double m, double d0, double d1,
                   double d2, double *a) {
  double r2 = d0 * d0 + d1 * d1 + d2 * d2 + b2;
  double rinv = 1.0 / sqrt(r2);
  double f = G * m * (rinv * rinv * rinv);
  a[0] += f * d0;
  a[1] += f * d1;
  a[2] += f * d2;
}

typedef struct {
  const orc_tree *t;
  double G, b2, theta2;
  int quad;
  int64_t i;        /* target particle */
  int self_img;     /* 1 while the unshifted image is walked */
  double y0, y1, y2;/* target position minus the image offset */
  double a[3];
  int64_t st[3];
} owalk;

/* Sect. 4.2: descend from the root; a cell whose opening angle w/R is below
 * theta_crit acts through its mass and centre of mass (plus its quadrupole,
 * Hernquist 1987), otherwise its sub-cells are visited in octant order.
 * Single-particle leaves are always summed directly; a bucket leaf that
 * fails the test is summed member by member.                               */
static void orc_visit(owalk *w, int64_t node) {
  const orc_tree *t = w->t;
  const onode *nd = &t->nodes[node];
  if (nd->M == 0.0) return;
  if (nd->leaf && nd->count == 1) {
    int64_t j = t->perm[nd->first];
    if (j == w->i && w->self_img) return;
    orc_pm(w->G, w->b2, nd->M, nd->com[0] - w->y0, nd->com[1] - w->y1,
           nd->com[2] - w->y2, w->a);
    w->st[2]++;
    return;
  }
  double d0 = nd->com[0] - w->y0, d1 = nd->com[1] - w->y1, d2 = nd->com[2] - w->y2;
  double R2 = fma(d2, d2, fma(d1, d1, d0 * d0));
  w->st[0]++;
  if (t->w2[nd->level] < w->theta2 * R2) {
    w->st[1]++;
    /* monopole: G M d / rho^3; quadrupole: -G Q d / rho^5
     * + (5/2) G (d.Q.d) d / rho^7, with rho^2 = R^2 + b^2 */
    double r2 = R2 + w->b2;
    double rinv = 1.0 / sqrt(r2);
    double rinv2 = rinv * rinv;
    double rinv3 = rinv * rinv2;
    double f = w->G * nd->M * rinv3;
    w->a[0] += f * d0;
    w->a[1] += f * d1;
    w->a[2] += f * d2;
    if (w->quad) {
      const double *Q = nd->Q;
      double q0 = Q[0] * d0 + Q[1] * d1 + Q[2] * d2;
      double q1 = Q[1] * d0 + Q[3] * d1 + Q[4] * d2;
      double q2 = Q[2] * d0 + Q[4] * d1 + Q[5] * d2;
      double dqd = d0 * q0 + d1 * q1 + d2 * q2;
      double rinv5 = rinv3 * rinv2;
      double rinv7 = rinv5 * rinv2;
      double g5 = w->G * rinv5;
      double g7 = 2.5 * w->G * dqd * rinv7;
      w->a[0] += -g5 * q0 + g7 * d0;
      w->a[1] += -g5 * q1 + g7 * d1;
      w->a[2] += -g5 * q2 + g7 * d2;
    }
    return;
  }
  if (nd->leaf) {
    for (int64_t r = nd->first; r < nd->first + nd->count; ++r) {
      int64_t j = t->perm[r];
      if (j == w->i && w->self_img) continue;
      double mj = t->msrc[j];
      if (mj == 0.0) continue;
      orc_pm(w->G, w->b2, mj, t->x[j] - w->y0, t->y[j] - w->y1, t->z[j] - w->y2, w->a);
      w->st[2]++;
    }
    return;
  }
  for (int o = 0; o < 8; ++o) {
    int32_t c = nd->child[o];
    if (c != ORC_NONE) orc_visit(w, c);
  }
}

void orc_bh(const orc_params *p, const orc_tree *t, int64_t n, const double *x,
            const double *y, const double *z, double s, const int64_t *targets,
            int64_t nt, double *ax, double *ay, double *az, int64_t *stats) {
  double o[ORC_MAX_IMAGES][3];
  int zero = 0;
  int ni = orc_images(p, s, o, &zero);
  int64_t count = targets ? nt : n;
  int64_t s0 = 0, s1 = 0, s2 = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : s0, s1, s2)
  for (int64_t k = 0; k < count; ++k) {
    int64_t i = targets ? targets[k] : k;
    owalk w;
    memset(&w, 0, sizeof(w));
    w.t = t;
    w.G = p->G;
    w.b2 = p->b * p->b;
    w.theta2 = p->theta * p->theta;
    w.quad = p->quadrupole;
    w.i = i;
    int live = isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]);
    if (live && t->n_nodes > 0) {
      for (int im = 0; im < ni; ++im) {
        w.self_img = (im == zero);
        w.y0 = x[i] - o[im][0];
        w.y1 = y[i] - o[im][1];
        w.y2 = z[i] - o[im][2];
        /* every root box's tree, in the order of the boxes' prefixes */
        for (int64_t r = 0; r < t->n_roots; ++r) orc_visit(&w, t->roots[r]);
      }
    }
    ax[k] = w.a[0];
    ay[k] = w.a[1];
    az[k] = w.a[2];
    s0 += w.st[0]; s1 += w.st[1]; s2 += w.st[2];
  }
  if (stats) { stats[0] = s0; stats[1] = s1; stats[2] = s2; }
}

/* Sect. 4.1: direct summation of Eq. (1) over the N_active massive
 * particles, for every image of every source. */
void orc_direct(const orc_params *p, int64_t n, int64_t n_active, const double *x,
                const double *y, const double *z, const double *m, double s,
                const int64_t *targets, int64_t nt, double *ax, double *ay,
                double *az) {
  double o[ORC_MAX_IMAGES][3];
  int zero = 0;
  int ni = orc_images(p, s, o, &zero);
  double b2 = p->b * p->b;
  int64_t count = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < count; ++k) {
    int64_t i = targets ? targets[k] : k;
    double a[3] = {0.0, 0.0, 0.0};
    int live = isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]);
    if (live) {
      for (int im = 0; im < ni; ++im) {
        double y0 = x[i] - o[im][0], y1 = y[i] - o[im][1], y2 = z[i] - o[im][2];
        for (int64_t j = 0; j < n_active && j < n; ++j) {
          if (j == i && im == zero) continue;
          if (!(isfinite(x[j]) && isfinite(y[j]) && isfinite(z[j]))) continue;
          orc_pm(p->G, b2, m[j], x[j] - y0, y[j] - y1, z[j] - y2, a);
        }
      }
    }
    ax[k] = a[0];
    ay[k] = a[1];
    az[k] = a[2];
  }
}

/* ------------------------------------------------------------------------ */
/* Shear offset of the ghost boxes: the domain copy at +Lx in x slides with
 * the mean shear flow vy = -(3/2) Omega x, so its y offset at time t is
 * -(3/2) Omega Lx t, folded into [-Ly/2, Ly/2].                             */
double orc_shear_offset(const orc_params *p, double t) {
  if (p->boundary != ORC_SHEAR) return 0.0;
  return remainder(1.5 * p->omega * orc_L(p, 0) * t, orc_L(p, 1));
}

/* Drift sub-step over tau.  Leap-frog (Sect. 3.1): x += v tau.  Epicycle
 * (Sect. 3.3): the exact solution of Hill's equations without the
 * perturbing force, x'' = 2 Omega y' + 3 Omega^2 x, y'' = -2 Omega x',
 * z'' = -Omega_z^2 z, which conserves C = vy + 2 Omega x and moves x about
 * the guiding centre xg = 2 C / Omega.                                      */
void orc_drift(const orc_params *p, int64_t n, double *x, double *y, double *z,
               double *vx, double *vy, double *vz, double tau) {
  if (p->drift == ORC_LEAPFROG) {
    for (int64_t i = 0; i < n; ++i) {
      if (!(isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]))) continue; /* removed */
      x[i] = x[i] + vx[i] * tau;
      y[i] = y[i] + vy[i] * tau;
      z[i] = z[i] + vz[i] * tau;
    }
    return;
  }
  double W = p->omega, Wz = p->omega_z;
  double c = cos(W * tau), sn = sin(W * tau);
  double cz = cos(Wz * tau), sz = sin(Wz * tau);
  for (int64_t i = 0; i < n; ++i) {
    if (!(isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]))) continue; /* removed */
    double C = vy[i] + 2.0 * W * x[i];
    double xg = 2.0 * C / W;
    double dx = x[i] - xg;
    double u = vx[i] / W;
    double xn = xg + dx * c + u * sn;
    double vxn = -W * dx * sn + vx[i] * c;
    double yn = y[i] - 3.0 * C * tau - 2.0 * dx * sn - 2.0 * u * (1.0 - c);
    double vyn = C - 2.0 * W * xn;
    double zn = z[i] * cz + vz[i] / Wz * sz;
    double vzn = -Wz * z[i] * sz + vz[i] * cz;
    x[i] = xn; vx[i] = vxn; y[i] = yn; vy[i] = vyn; z[i] = zn; vz[i] = vzn;
  }
}

/* Sect. 2.3 boundaries, at the faces of the domain (extents Lx, Ly, Lz).
 * Shear-periodic in x: a particle leaving through one x face re-enters
 * through the other, shifted in y by the shear offset and in vy by the
 * shear velocity jump (3/2) Omega Lx.  Periodic: plain wrap.
 * y wraps in both.  Open axes remove the particle (it becomes a tombstone:
 * NaN position, zero velocity) once it leaves the root box.                */
void orc_boundary(const orc_params *p, int64_t n, double *x, double *y, double *z,
                  double *vx, double *vy, double *vz, double s) {
  double Lx = orc_L(p, 0), Ly = orc_L(p, 1), Lz = orc_L(p, 2);
  double lo0 = p->x0[0], lo1 = p->x0[1], lo2 = p->x0[2];
  double hi0 = lo0 + Lx, hi1 = lo1 + Ly, hi2 = lo2 + Lz;
  double jump = 1.5 * p->omega * Lx;
  for (int64_t i = 0; i < n; ++i) {
    if (!(isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]))) continue;
    if (p->boundary == ORC_SHEAR) {
      if (x[i] >= hi0) { x[i] = x[i] - Lx; y[i] = y[i] + s; vy[i] = vy[i] + jump; }
      else if (x[i] < lo0) { x[i] = x[i] + Lx; y[i] = y[i] - s; vy[i] = vy[i] - jump; }
    } else if (p->boundary == ORC_PERIODIC) {
      if (x[i] >= hi0) x[i] = x[i] - Lx;
      else if (x[i] < lo0) x[i] = x[i] + Lx;
    }
    if (p->boundary != ORC_OPEN) {
      if (y[i] >= hi1) y[i] = y[i] - Ly;
      else if (y[i] < lo1) y[i] = y[i] + Ly;
    }
    int out = !(z[i] >= lo2 && z[i] < hi2);
    if (p->boundary == ORC_OPEN)
      out = out || !(x[i] >= lo0 && x[i] < hi0) || !(y[i] >= lo1 && y[i] < hi1);
    if (out) {
      x[i] = y[i] = z[i] = NAN;
      vx[i] = vy[i] = vz[i] = 0.0;
    }
  }
}

/* Sect. 3: drift dt/2, kick dt, drift dt/2, one global time-step.  The kick
 * uses the forces at the positions after the first drift, at time
 * t + dt/2; the ghost offset is evaluated at that time.                    */
void orc_step(const orc_params *p, int64_t n, int64_t n_active, double *x,
              double *y, double *z, double *vx, double *vy, double *vz,
              const double *m, double t0, double dt, int32_t nsteps,
              int32_t use_tree) {
  double *ax = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double *ay = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double *az = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double half = 0.5 * dt;
  for (int32_t k = 0; k < nsteps; ++k) {
    double tk = t0 + (double)k * dt;
    double th = tk + half;
    double te = t0 + (double)(k + 1) * dt;
    orc_drift(p, n, x, y, z, vx, vy, vz, half);
    orc_boundary(p, n, x, y, z, vx, vy, vz, orc_shear_offset(p, th));
    double s = orc_shear_offset(p, th);
    if (use_tree) {
      orc_tree *t = orc_tree_build(p, n, n_active, x, y, z, m);
      orc_bh(p, t, n, x, y, z, s, NULL, 0, ax, ay, az, NULL);
      orc_tree_free(t);
    } else {
      orc_direct(p, n, n_active, x, y, z, m, s, NULL, 0, ax, ay, az);
    }
    for (int64_t i = 0; i < n; ++i) {
      if (!(isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]))) continue;
      vx[i] = vx[i] + ax[i] * dt;
      vy[i] = vy[i] + ay[i] * dt;
      vz[i] = vz[i] + az[i] * dt;
    }
    orc_drift(p, n, x, y, z, vx, vy, vz, half);
    orc_boundary(p, n, x, y, z, vx, vy, vz, orc_shear_offset(p, te));
  }
  free(ax); free(ay); free(az);
}

/* kinetic plus softened pairwise potential energy (open boundaries) */
double orc_energy(const orc_params *p, int64_t n, int64_t n_active,
                  const double *x, const double *y, const double *z,
                  const double *vx, const double *vy, const double *vz,
                  const double *m) {
  double ek = 0.0, ep = 0.0, b2 = p->b * p->b;
  for (int64_t i = 0; i < n; ++i) {
    if (!(isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]))) continue;
    ek += 0.5 * m[i] * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
  }
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : ep)
  for (int64_t i = 0; i < n_active; ++i) {
    if (!(isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]))) continue;
    for (int64_t j = i + 1; j < n_active; ++j) {
      if (!(isfinite(x[j]) && isfinite(y[j]) && isfinite(z[j]))) continue;
      double d0 = x[j] - x[i], d1 = y[j] - y[i], d2 = z[j] - z[i];
      ep -= p->G * m[i] * m[j] / sqrt(d0 * d0 + d1 * d1 + d2 * d2 + b2);
    }
  }
  return ek + ep;
}

/* ------------------------------------------------------------------------ */
/* Collisions (Sect. 5): detection of overlapping pairs at the end of a step,
 * a random order for the collision queue, and hard-sphere resolution with a
 * normal coefficient of restitution (v_n' = -eps v_n, v_t' = v_t), in that
 * order, one collision after the other.
 *
 * Detection is the plain definition the tree search of Eq. (3) reaches:
 * every pair (i < j) of live particles and every ghost image k of j with
 * |x_j + o_k - x_i| < R_i + R_j.  A pair is coded c = i 2^35 + j 2^7 + k.
 * The queue's random order is ascending h(c) = splitmix64(seed + c), the
 * generator's finalising mix (Steele, Lea & Flood 2014), which is a bijection
 * of 64-bit integers, so the order is total.  A queued collision is resolved
 * only while the particles approach each other (d . u < 0, d = x_j + o_k -
 * x_i, u = v_j + w_k - v_i, w_k the image's shear velocity (0, -3/2 Omega W
 * ix, 0)); momentum is conserved and the normal relative velocity becomes
 * -eps times itself.                                                      */

uint64_t orc_splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

typedef struct {
  uint64_t h, code;
} orc_coll;

static int orc_coll_cmp(const void *a, const void *b) {
  const orc_coll *x = (const orc_coll *)a, *y = (const orc_coll *)b;
  return (x->h > y->h) - (x->h < y->h);
}

/* Does particle i meet image k of particle j?  sweep = 0: they overlap now,
 * |d| < R_i + R_j.  sweep = 1: their straight trajectories over the past
 * time-step come that close: with d(sigma) = d + u sigma for sigma in
 * [-dt, 0] (the line through the present positions with the present
 * velocities), min |d(sigma)| < R_i + R_j.  The minimum over the segment is
 * at sigma = 0 unless the pair is now separating (d . u > 0); then it is at
 * -d.u / u.u, or at -dt if that lies further back. */
static int orc_meets(int sweep, double d0, double d1, double d2, double u0, double u1,
                     double u2, double sum, double dt) {
  if (d0 * d0 + d1 * d1 + d2 * d2 < sum * sum) return 1;
  if (!sweep) return 0;
  const double du = d0 * u0 + d1 * u1 + d2 * u2;
  const double uu = u0 * u0 + u1 * u1 + u2 * u2;
  if (!(du > 0.0 && uu > 0.0)) return 0;
  double sg = -du / uu;
  if (sg < -dt) sg = -dt;
  const double e0 = d0 + u0 * sg, e1 = d1 + u1 * sg, e2 = d2 + u2 * sg;
  return e0 * e0 + e1 * e1 + e2 * e2 < sum * sum;
}

/* detection (brute force over all pairs and images; counted, then written,
 * both passes parallel over i), the queue in random order, resolution */
static int64_t orc_coll_run(const orc_params *p, int64_t n, const double *x, const double *y,
                            const double *z, double *vx, double *vy, double *vz,
                            const double *m, const double *R, double s, int sweep, double dt,
                            double eps, uint64_t seed, uint64_t *codes, int64_t cap,
                            int64_t *n_resolved) {
  double o[ORC_MAX_IMAGES][3];
  int zero = 0;
  const int ni = orc_images(p, s, o, &zero);
  double w[ORC_MAX_IMAGES];  /* y velocity of each image relative to the box */
  {
    int k = 0;
    for (int ix = -p->ng[0]; ix <= p->ng[0]; ++ix)
      for (int iy = -p->ng[1]; iy <= p->ng[1]; ++iy) {
        w[k++] = (p->boundary == ORC_SHEAR) ? -1.5 * p->omega * orc_L(p, 0) * (double)ix : 0.0;
      }
    if (p->boundary == ORC_OPEN) w[0] = 0.0;
  }
  uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
  orc_keys(p, n, x, y, z, keys);
  int64_t *per = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  orc_coll *q = NULL;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      for (int64_t i = 0; i < n; ++i) per[i + 1] += per[i];
      q = (orc_coll *)malloc(sizeof(orc_coll) * (size_t)(per[n] > 0 ? per[n] : 1));
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      if (keys[i] == UINT64_MAX) continue;
      int64_t c = 0, at = pass ? per[i] : 0;
      for (int64_t j = i + 1; j < n; ++j) {
        if (keys[j] == UINT64_MAX) continue;
        const double sum = R[i] + R[j];
        for (int k = 0; k < ni; ++k) {
          const double d0 = (x[j] + o[k][0]) - x[i];
          const double d1 = (y[j] + o[k][1]) - y[i];
          const double d2 = (z[j] + o[k][2]) - z[i];
          const double u0 = vx[j] - vx[i];
          const double u1 = (vy[j] + w[k]) - vy[i];
          const double u2 = vz[j] - vz[i];
          if (!orc_meets(sweep, d0, d1, d2, u0, u1, u2, sum, dt)) continue;
          if (pass == 0) {
            ++c;
          } else {
            const uint64_t cd = ((uint64_t)i << 35) | ((uint64_t)j << 7) | (uint64_t)k;
            q[at].code = cd;
            q[at].h = orc_splitmix64(seed + cd);
            ++at;
          }
        }
      }
      if (pass == 0) per[i + 1] = c;
    }
  }
  const int64_t count = per[n];
  free(per);
  qsort(q, (size_t)count, sizeof(orc_coll), orc_coll_cmp);
  /* resolution in queue order */
  int64_t res = 0, stored = 0;
  for (int64_t c = 0; c < count; ++c) {
    const int64_t i = (int64_t)(q[c].code >> 35);
    const int64_t j = (int64_t)((q[c].code >> 7) & ((1ull << 28) - 1ull));
    const int k = (int)(q[c].code & 127ull);
    if (stored < cap) codes[stored++] = q[c].code;
    const double d0 = (x[j] + o[k][0]) - x[i];
    const double d1 = (y[j] + o[k][1]) - y[i];
    const double d2 = (z[j] + o[k][2]) - z[i];
    const double u0 = vx[j] - vx[i];
    const double u1 = (vy[j] + w[k]) - vy[i];
    const double u2 = vz[j] - vz[i];
    if (!(d0 * u0 + d1 * u1 + d2 * u2 < 0.0)) continue;  /* not approaching */
    const double M = m[i] + m[j];
    if (!(M > 0.0)) continue;
    const double dist = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    const double n0 = d0 / dist, n1 = d1 / dist, n2 = d2 / dist;
    const double vn = n0 * u0 + n1 * u1 + n2 * u2;
    const double f = (1.0 + eps) * vn;
    const double fi = (m[j] / M) * f, fj = (m[i] / M) * f;
    vx[i] = vx[i] + fi * n0; vy[i] = vy[i] + fi * n1; vz[i] = vz[i] + fi * n2;
    vx[j] = vx[j] - fj * n0; vy[j] = vy[j] - fj * n1; vz[j] = vz[j] - fj * n2;
    ++res;
  }
  if (n_resolved) *n_resolved = res;
  free(q);
  free(keys);
  return count;
}

int64_t orc_collide(const orc_params *p, int64_t n, const double *x, const double *y,
                    const double *z, double *vx, double *vy, double *vz, const double *m,
                    const double *R, double s, double eps, uint64_t seed, uint64_t *codes,
                    int64_t cap, int64_t *n_resolved) {
  return orc_coll_run(p, n, x, y, z, vx, vy, vz, m, R, s, 0, 0.0, eps, seed, codes, cap,
                      n_resolved);
}

/* The plane-sweep modules (Sect. 5) find the pairs whose straight
 * trajectories over the time-step come within R_i + R_j: the sweep along x
 * only narrows the candidates, so its result is this set. */
int64_t orc_sweep(const orc_params *p, int64_t n, const double *x, const double *y,
                  const double *z, double *vx, double *vy, double *vz, const double *m,
                  const double *R, double s, double dt, double eps, uint64_t seed,
                  uint64_t *codes, int64_t cap, int64_t *n_resolved) {
  return orc_coll_run(p, n, x, y, z, vx, vy, vz, m, R, s, 1, dt, eps, seed, codes, cap,
                      n_resolved);
}
