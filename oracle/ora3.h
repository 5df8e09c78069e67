/*
 * ora3.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU oracle of the SIMPLE-TS time step in three
 * dimensions: the paper's 2-D method (Shterev, arXiv 1802.04243; loops 1 and
 * 2 of Sec. 3.1, the discrete equations of Sec. 3.2, the pass order of
 * Appendix A) extended to a staggered Cartesian grid in x, y, z, the
 * extension its Conclusions name as the next step.  Velocity component a
 * lives on the a-faces; p and T at the cell centres.  Tests use it; the
 * product never links, loads or calls it.
 *
 * Storage (host, dense, x fastest, then y, then z):
 *   u [nz][ny][nx+1], v [nz][ny+1][nx], w [nz+1][ny][nx], p, T [nz][ny][nx].
 * Every value is nondimensional FP64.
 */
#ifndef ORA3_H
#define ORA3_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ora3_ctx ora3_ctx;

/* Boundary kind per direction: x takes ORA3_INLET_OUTLET (supersonic inlet
   at x = 0, zero-gradient outlet at x = Lx) or ORA3_PERIODIC; y and z take
   ORA3_WALLS (a wall at each end) or ORA3_PERIODIC. */
enum { ORA3_WALLS = 0, ORA3_PERIODIC = 1, ORA3_INLET_OUTLET = 2 };
/* wall types: no-slip isothermal (eqs pl38, pl39 with zero slip and jump
   lengths), slip adiabatic */
enum { ORA3_NOSLIP = 0, ORA3_SLIP = 1 };

typedef struct {
  int n[3];                 /* cells in x, y, z; each >= 4                  */
  const double *d[3];       /* [n[e]] cell widths per direction             */
  int bc[3];                /* boundary kind per direction (above)         */
  int wall_type[3][2];      /* per wall direction, low / high wall          */
  double wall_vel[3][2][3]; /* velocity of each wall (tangential components)*/
  double wall_T[3][2];      /* temperature of each no-slip wall            */
  double Ma, Re, Pr, gamma;
  double u_in, T_in, p_in;  /* uniform inlet state (x inlet)                */
  double g[3];              /* body force per unit mass                     */
} ora3_setup;

enum { ORA3_EXPLICIT = 0, ORA3_IMPLICIT = 1, ORA3_UPWIND = 0, ORA3_TVD = 2 };

/* NULL when any direction has fewer than 4 cells. */
ora3_ctx *ora3_create(const ora3_setup *s);
/* OpenMP threads of the oracle's loops (n <= 0: one). */
void ora3_set_threads(int n);
void ora3_destroy(ora3_ctx *c);
/* Replace the state (NULL keeps a field; order u, v, w, p, T), then impose
   the boundary values (inlet faces u = u_in, wall faces normal velocity 0,
   outlet face u = its upstream neighbour, periodic copies). */
void ora3_set_fields(ora3_ctx *c, const double *const q[5]);
void ora3_get_fields(const ora3_ctx *c, double *const q[5]);
/* One time step: prologue, then n_inner Jacobi passes. */
void ora3_step(ora3_ctx *c, double dt, int n_inner, int scheme);
/* Residuals of the last pass: max|du|, max|dv|, max|dw|, max|dp|, max|dT|,
   max|R| and sum R of the discrete continuity residual. */
void ora3_residuals(const ora3_ctx *c, double out[7]);
/* Total mass sum(p/T dV). */
double ora3_mass(const ora3_ctx *c);
/* Freeze the current state as both the previous time level and the old
   iterate and evaluate every discrete equation in coefficient form,
   a0*phi - sum(a_nb*phi_nb) - b (momentum also + A*area*(p_r - p_l)); the
   pressure equation with T_new = T.  Unsolved unknowns get 0.  Arrays in the
   field layouts above, order u, v, w, p, T. */
void ora3_eq_residuals(ora3_ctx *c, double dt, int scheme, double *const r[5]);

#ifdef __cplusplus
}
#endif
#endif
