/* Exercises every oracle entry point on small seeded inputs; built with the
 * address and undefined-behaviour sanitizers by test_oracle_sanitize.py so
 * that an out-of-bounds access or undefined operation in the oracle fails
 * the CPU test suite.  Returns 0 when every call completed. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/rb_oracle.h"

static uint64_t g_state = 12345u;
static double uni(void) { /* xorshift64*, uniform in [0, 1) */
  g_state ^= g_state >> 12; g_state ^= g_state << 25; g_state ^= g_state >> 27;
  return (double)((g_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static void fill(int n, double lo, double hi, double *a) {
  for (int i = 0; i < n; ++i) a[i] = lo + (hi - lo) * uni();
}

int main(void) {
  enum { N = 700 };
  static double x[N], y[N], z[N], vx[N], vy[N], vz[N], m[N], R[N], ax[N], ay[N], az[N];
  static uint64_t keys[N], codes[16 * N];
  int64_t stats[3];
  for (int cfg = 0; cfg < 6; ++cfg) {
    orc_params p = {0};
    p.G = 1.0; p.b = (cfg & 1) ? 0.01 : 0.0; p.theta = 0.3 + 0.1 * cfg;
    p.quadrupole = cfg & 1; p.n_leaf = (cfg % 3 == 0) ? 1 : 4; p.W = 1.0;
    p.n_root[0] = 1 + cfg % 3; p.n_root[1] = 1 + (cfg / 2) % 2; p.n_root[2] = 1;
    p.boundary = cfg % 3; p.ng[0] = p.ng[1] = (p.boundary ? 1 : 0);
    p.drift = (p.boundary == 2) ? 1 : 0; p.omega = 0.5; p.omega_z = 0.5;
    double Lx = p.n_root[0] * p.W, Ly = p.n_root[1] * p.W;
    p.x0[0] = -0.5 * Lx; p.x0[1] = -0.5 * Ly; p.x0[2] = -0.5;
    fill(N, -0.5 * Lx, 0.5 * Lx, x); fill(N, -0.5 * Ly, 0.5 * Ly, y); fill(N, -0.4, 0.4, z);
    fill(N, -0.1, 0.1, vx); fill(N, -0.1, 0.1, vy); fill(N, -0.1, 0.1, vz);
    fill(N, 0.5, 1.5, m); fill(N, 0.001, 0.02, R);
    for (int i = 0; i < 40; ++i) { x[i] = x[0] + 1e-14 * i; y[i] = y[0]; z[i] = z[0]; }
    x[50] = NAN;               /* a removed particle */
    orc_keys(&p, N, x, y, z, keys);
    orc_tree *t = orc_tree_build(&p, N, N - 100, x, y, z, m);
    if (!orc_tree_selfcheck(t)) return 1;
    int64_t nn = orc_tree_n_nodes(t), nl = orc_tree_n_live(t);
    int8_t *lev = malloc(nn), *leaf = malloc(nn);
    uint64_t *pre = malloc(nn * 8), *sk = malloc(nl * 8);
    int64_t *first = malloc(nn * 8), *count = malloc(nn * 8), *fc = malloc(nn * 8),
            *perm = malloc(nl * 8);
    int32_t *nc = malloc(nn * 4);
    double *M = malloc(nn * 8), *com = malloc(nn * 24), *Q = malloc(nn * 48);
    orc_tree_export(t, lev, pre, first, count, leaf, nc, fc, M, com, Q, perm, sk);
    double s = orc_shear_offset(&p, 3.0);
    orc_bh(&p, t, N, x, y, z, s, NULL, 0, ax, ay, az, stats);
    for (int i = 0; i < N; ++i) { x[i] += 0.02 * (uni() - 0.5); y[i] += 0.02 * (uni() - 0.5); }
    orc_boundary(&p, N, x, y, z, vx, vy, vz, s);
    orc_tree_update(t, x, y, z);
    if (!orc_tree_selfcheck(t)) return 2;
    orc_bh(&p, t, N, x, y, z, s, NULL, 0, ax, ay, az, stats);
    int64_t tg[5] = {0, 3, 99, 400, N - 1};
    orc_direct(&p, N, N - 100, x, y, z, m, s, tg, 5, ax, ay, az);
    orc_step(&p, N, N - 100, x, y, z, vx, vy, vz, m, 0.0, 0.01, 2, 1);
    orc_step(&p, N, N - 100, x, y, z, vx, vy, vz, m, 0.02, 0.01, 1, 0);
    (void)orc_energy(&p, N, N - 100, x, y, z, vx, vy, vz, m);
    int64_t nres = 0;
    orc_collide(&p, N, x, y, z, vx, vy, vz, m, R, s, 0.5, 7, codes, 16 * N, &nres);
    orc_sweep(&p, N, x, y, z, vx, vy, vz, m, R, s, 0.01, 0.5, 8, codes, 16 * N, &nres);
    orc_tree_free(t);
    free(lev); free(leaf); free(pre); free(sk); free(first); free(count); free(fc);
    free(perm); free(nc); free(M); free(com); free(Q);
  }
  (void)orc_splitmix64(42u);
  printf("oracle sanitize run ok\n");
  return 0;
}
