/*
 * Exercises every entry point of the 2-D and 3-D oracles on small problems
 * that reach every boundary branch (inlet, outlet, periodic, no-slip, slip,
 * slip-jump walls, obstacles, body forces, stretched widths) in every
 * scheme.  Built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py; any invalid access, leak or undefined operation
 * ends the run with a report.  Prints one line per case.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "ora.h"
#include "ora3.h"

static double widths(int k, int n) { return 0.1 + 0.05 * sin(1.3 * k + n); }

static int run2d(int periodic, int wall, int obstacles, int scheme) {
  const int nx = 23, ny = 11;
  double dx[23], dy[11], uin[11], tin[11], tw0[23], tw1[23];
  for (int i = 0; i < nx; i++) {
    dx[i] = widths(i, nx);
    tw0[i] = 1.1;
    tw1[i] = 0.9;
  }
  for (int j = 0; j < ny; j++) {
    dy[j] = widths(j, ny);
    uin[j] = 1.0;
    tin[j] = 1.0;
  }
  int oi0[2] = {6, 14}, oj0[2] = {3, 5}, oi1[2] = {8, 15}, oj1[2] = {5, 7};
  ora_setup s = {0};
  s.nx = nx;
  s.ny = ny;
  s.dx = dx;
  s.dy = dy;
  s.periodic = periodic;
  s.n_obst = obstacles ? 2 : 0;
  s.oi0 = oi0;
  s.oj0 = oj0;
  s.oi1 = oi1;
  s.oj1 = oj1;
  s.Ma = 0.8;
  s.Re = 20.0;
  s.Pr = 0.7;
  s.gamma = 1.4;
  s.u_in = uin;
  s.T_in = tin;
  s.p_in = 1.0;
  s.wall_type[0] = wall;
  s.wall_type[1] = 0;
  s.wall_u[1] = 0.3;
  s.wall_T[0] = tw0;
  s.wall_T[1] = tw1;
  s.obstacle_T = 1.2;
  s.gx = 0.1;
  s.gy = -0.2;
  s.obstacle_type = wall == 2 ? 2 : 0;
  s.kn = 0.01;
  ora_ctx *c = ora_create(&s);
  if (!c) return 1;
  double *u = calloc((size_t)(nx + 1) * ny, sizeof(double));
  double *v = calloc((size_t)nx * (ny + 1), sizeof(double));
  double *p = calloc((size_t)nx * ny, sizeof(double));
  double *T = calloc((size_t)nx * ny, sizeof(double));
  ora_get_fields(c, u, v, p, T);
  for (int k = 0; k < nx * (ny + 1); k++) v[k] = 0.01 * sin(0.7 * k);
  ora_set_fields(c, u, v, p, T);
  ora_step(c, 0.002, 4, scheme);
  ora_step_l3(c, 0.002, 3, 2, scheme);
  const int n = ora_step_tol(c, 0.002, 6, 1e-12, scheme);
  double res[6], m[3];
  ora_residuals(c, res);
  ora_mass(c, m);
  ora_eq_residuals(c, 0.002, scheme, T, u, v, p);
  ora_destroy(c);
  free(u);
  free(v);
  free(p);
  free(T);
  printf("2-D periodic=%d wall=%d obstacles=%d scheme=%d passes=%d res=%.3e mass=%.6f\n",
         periodic, wall, obstacles, scheme, n, res[0], m[0]);
  return !(isfinite(res[0]) && isfinite(m[0]));
}

static int run3d(int channel, int scheme) {
  const int n[3] = {9, 7, 6};
  double d[3][9];
  ora3_setup s = {0};
  for (int e = 0; e < 3; e++) {
    for (int k = 0; k < n[e]; k++) d[e][k] = widths(k, n[e] + e);
    s.n[e] = n[e];
    s.d[e] = d[e];
    s.bc[e] = ORA3_PERIODIC;
    s.wall_T[e][0] = 1.1;
    s.wall_T[e][1] = 0.95;
    s.g[e] = 0.1 * (e + 1);
  }
  if (channel) {
    s.bc[0] = ORA3_INLET_OUTLET;
    s.bc[1] = s.bc[2] = ORA3_WALLS;
    s.wall_type[1][1] = ORA3_SLIP;
    s.wall_vel[2][1][0] = 0.2;
    s.wall_vel[2][1][1] = -0.1;
  }
  s.Ma = 0.8;
  s.Re = 20.0;
  s.Pr = 0.7;
  s.gamma = 1.4;
  s.u_in = 1.0;
  s.T_in = 1.0;
  s.p_in = 1.0;
  ora3_ctx *c = ora3_create(&s);
  if (!c) return 1;
  size_t len[5];
  double *q[5];
  for (int f = 0; f < 5; f++) {
    len[f] = (size_t)(n[0] + (f == 0)) * (n[1] + (f == 1)) * (n[2] + (f == 2));
    q[f] = calloc(len[f], sizeof(double));
  }
  ora3_get_fields(c, q);
  for (size_t k = 0; k < len[1]; k++) q[1][k] = 0.02 * cos(0.3 * (double)k);
  ora3_set_fields(c, (const double *const *)q);
  ora3_step(c, 0.002, 4, scheme);
  double res[7];
  ora3_residuals(c, res);
  const double m = ora3_mass(c);
  ora3_eq_residuals(c, 0.002, scheme, q);
  ora3_destroy(c);
  for (int f = 0; f < 5; f++) free(q[f]);
  printf("3-D channel=%d scheme=%d res=%.3e mass=%.6f\n", channel, scheme, res[0], m);
  return !(isfinite(res[0]) && isfinite(m));
}

int main(void) {
  int bad = 0;
  for (int scheme = 0; scheme < 4; scheme++) {
    bad |= run2d(0, 0, 1, scheme);
    bad |= run2d(1, 1, 0, scheme);
    bad |= run2d(0, 2, 1, scheme);
    bad |= run3d(0, scheme);
    bad |= run3d(1, scheme);
  }
  /* invalid problems are refused */
  ora_setup z = {0};
  ora3_setup z3 = {0};
  bad |= ora_create(&z) != NULL;
  bad |= ora_create(NULL) != NULL;
  bad |= ora3_create(&z3) != NULL;
  bad |= ora3_create(NULL) != NULL;
  printf(bad ? "FAILED\n" : "OK\n");
  return bad;
}
