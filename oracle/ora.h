/*
 * ora.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU oracle of the SIMPLE-TS time step (Shterev,
 * arXiv 1802.04243): loops 1 and 2 of the method (Sec. 3.1, Figs. of the
 * explicit and implicit GPU algorithms), the discrete equations of Sec. 3.2
 * (pl8-pl33) and the update order of Appendix A.  It exists so that tests,
 * the smoke check and the benchmark's CPU-baseline leg can check and time the
 * HIP library against an independent implementation.  The product path never
 * links, loads or calls it; it shares no code with the HIP library.
 *
 * Storage (host, dense, x fastest):
 *   u [ny][nx+1]  horizontal velocity at x-faces (x^f_i, y^v_j)
 *   v [ny+1][nx]  vertical velocity at y-faces  (x^v_i, y^f_j)
 *   p [ny][nx], T [ny][nx]  at cell centres    (x^v_i, y^v_j)
 * Every value is nondimensional and FP64.
 */
#ifndef ORA_H
#define ORA_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ora_ctx ora_ctx;

/* Problem description.  Arrays are copied by ora_create. */
typedef struct {
  int nx, ny;                 /* cells; nx, ny >= 4                        */
  const double *dx, *dy;      /* [nx], [ny] cell widths                     */
  int periodic;               /* 0: inlet (x=0) / outlet (x=Lx); 1: periodic */
  int n_obst;                 /* solid rectangles in cell indices, closed   */
  const int *oi0, *oj0, *oi1, *oj1;
  double Ma, Re, Pr, gamma;   /* gas and flow parameters                    */
  const double *u_in, *T_in;  /* [ny] inlet-face u and T                    */
  double p_in;                /* inlet pressure                             */
  int wall_type[2];           /* [0] bottom y=0, [1] top y=Ly:
                                 0 no-slip isothermal, 1 slip adiabatic,
                                 2 velocity slip + temperature jump        */
  double wall_u[2];           /* tangential wall velocity (types 0 and 2)   */
  const double *wall_T[2];    /* [nx] wall temperature per cell column      */
  double obstacle_T;          /* surface temperature of the obstacles       */
  double gx, gy;              /* body force per unit mass                   */
  int obstacle_type;          /* 0 no-slip isothermal, 2 slip + jump        */
  double kn;                  /* Knudsen number of the slip / jump walls
                                 (pl38, pl39), in the grid's length unit   */
} ora_setup;

enum { ORA_EXPLICIT = 0, ORA_IMPLICIT = 1, ORA_UPWIND = 0, ORA_TVD = 2 };

ora_ctx *ora_create(const ora_setup *s);
void ora_destroy(ora_ctx *c);
/* Replace the state by the given fields (NULL keeps a field), then impose the
   boundary values: inlet/wall/outlet faces, solid cells (T = obstacle_T,
   p = p_in). */
void ora_set_fields(ora_ctx *c, const double *u, const double *v,
                    const double *p, const double *T);
void ora_get_fields(const ora_ctx *c, double *u, double *v, double *p,
                    double *T);
/* One time step: prologue, then n_inner Jacobi passes. */
void ora_step(ora_ctx *c, double dt, int n_inner, int scheme);
/* One time step whose passes each solve the energy and pressure equations
   n3 >= 1 times (loop 3 of the CPU algorithm; n3 = 1 is ora_step). */
void ora_step_l3(ora_ctx *c, double dt, int n_inner, int n3, int scheme);
/* One time step whose loop 2 stops after the first pass with
   max(max|du|, max|dv|, max|dT|, max|dp|/p_in) <= tol, or after max_inner
   passes; returns the passes taken. */
int ora_step_tol(ora_ctx *c, double dt, int max_inner, double tol, int scheme);
/* ora_step_tol with loop 3 (n3 >= 1 energy-pressure solves) in every pass. */
int ora_step_tol_l3(ora_ctx *c, double dt, int max_inner, int n3, double tol, int scheme);
/* Residuals of the last pass: max|du|, max|dv|, max|dp|, max|dT|,
   max|R_mass|, sum R_mass. */
void ora_residuals(const ora_ctx *c, double out[6]);
/* Total fluid mass sum(p/T dV) of the current state, and the mass fluxes
   through the inlet and outlet (rho^u u dy summed over the faces). */
void ora_mass(const ora_ctx *c, double out[3]);

/* ---- pieces exposed for pin tests ---- */
/* A, B, C^{T1}_f, C^{T2}_f, C^{T3}_f for (Ma, Re, Pr, gamma). */
/* OpenMP threads of the row loops (the results do not depend on it). */
void ora_set_threads(int n);
int ora_max_threads(void);
void ora_params(double Ma, double Re, double Pr, double gamma, double out[5]);
/* Test switch (default on): off forces every TVD correction to zero. */
void ora_set_limiter(int on);
/* van Leer limiter psi(r) of r = a/b, division-safe. */
double ora_vanleer(double a, double b);
double ora_psi_s(double f1, double f2, double f3, double f4, double d1,
                 double d2, double d3, double d4, double vel);
double ora_psi_c(double f1, double f2, double f3, double f4, double d1,
                 double d2, double d3, double vel);
/* Freeze the current state as both the previous time level and the old
   iterate and evaluate every discrete equation in coefficient form,
   a0*phi_P - sum(a_nb*phi_nb) - b (momentum also + A*len*(p_P - p_nb)).
   Unsolved unknowns get 0.  Arrays have the field sizes above. */
void ora_eq_residuals(ora_ctx *c, double dt, int scheme, double *rT,
                      double *ru, double *rv, double *rp);

#ifdef __cplusplus
}
#endif
#endif
