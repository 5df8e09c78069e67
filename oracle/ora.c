/*
 * ora.c -- TEST INFRASTRUCTURE ONLY: plain FP64 CPU oracle of the SIMPLE-TS
 * time step (Shterev, arXiv 1802.04243).  Used by tests, the smoke check and
 * the benchmark's CPU-baseline leg; never by the product.  Shares no code with
 * the HIP library.
 *
 * What it computes (paper sections / equations):
 *   loop 1 (time steps) and loop 2 (inner Jacobi passes) of SIMPLE-TS, GPU
 *   form (Sec. 3.1, figures of the explicit and implicit algorithms), with a
 *   fixed pass count or until the increments fall below a tolerance;
 *   one pass in the order of Appendix A: face densities (pl10, pl11), mass
 *   fluxes (pl8, pl9), temperature (pl30 with pl31 or pl31_1, pl32, pl33,
 *   source pl28/pl29), pseudo velocities (pl20, pl21 with pl14-pl16,
 *   pl15_11), pressure (pl23, pl24), velocities (pl18, pl19);
 *   optionally loop 3 of the CPU algorithm inside each pass (the energy and
 *   pressure equations solved n3 times with the pass's coefficients);
 *   velocity-slip / temperature-jump surfaces (pl38, pl39).
 * The u-equation is not printed in the paper (it gives v only); here it is the
 * x<->y mirror image of the printed v-equation.  Boundary rules, constants and
 * the readings of garbled passages are stated where each is implemented
 * (van Leer in the (r+|r|)/(1+|r|) form, face density = upwind + psi*jump,
 * C^{T1..3}_f = gamma*C^{T1}, gamma*C^{T2}, -(gamma-1)).
 *
 * Every formula is written as the paper prints it: conductances and
 * gradients divide by the printed widths and distances, unsteady terms by
 * 2 dt or dt, the limiter takes r = a/b; nothing is precomputed or
 * refactored for speed.
 *
 * Pinned against the mathematics, not against another implementation
 * (tests/test_oracle_pins.py, test_manufactured.py, test_slip_jump_pins.py,
 * test_loop3_pins.py): closed forms (pl37 constants, compressible Couette and
 * Poiseuille with heat conduction, the hydrostatic box, slip Couette, jump
 * conduction), the continuous operators integrated over the control volumes
 * (manufactured solutions: every interior term at its truncation order, wall,
 * obstacle, inlet and outlet volumes at first order per face length), the
 * speed of sound, the convective schemes' orders, invariants (bitwise
 * free-stream preservation, mirror symmetry, the mass identity, TVD with the
 * limiter off = upwind, solid rows = a channel wall).
 *
 * Plain loops, no blocking, no fusion; OpenMP only splits rows of a loop.
 * Build with -ffp-contract=off.
 */
#include "ora.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

struct ora_ctx {
  int nx, ny, per;
  double *dx, *dy;
  unsigned char *solid; /* [ny][nx] */
  double A, B, C1, C2, C3, gx, gy;
  double *u_in, *T_in, p_in;
  int wtype[2];
  double wu[2];
  double *wT[2];
  double obsT;
  int otype;
  /* slip and jump coefficients (pl38, pl39): zeta = kz/rho, tau = kt/rho */
  double kz, kt;
  /* state: old iterate (u..T), new iterate (un..Tn), time level n-1 (um..Tm) */
  double *u, *v, *p, *T;
  double *un, *vn, *pn, *Tn;
  double *um, *vm, *pm, *Tm;
  /* loop 3: the previous sub-iterate of T and p */
  double *Ts, *ps;
  /* per-pass work arrays */
  double *rho, *gam, *rhou, *rhov, *Fx, *Fy;
  double *uh, *du, *vh, *dv;
  double *uexp, *vexp, *Texp;
  double res[6];
  double last_fin, last_fout;
};

/* ------------------------------------------------------------------ */
/* indexing                                                           */
/* ------------------------------------------------------------------ */
#define IU(c, i, j) ((size_t)(j) * (size_t)((c)->nx + 1) + (size_t)(i))
#define IC(c, i, j) ((size_t)(j) * (size_t)(c)->nx + (size_t)(i))
#define IV(c, i, j) IC(c, i, j)

/* cell column (and u-face column) index, wrapped when x is periodic */
static int cw(const ora_ctx *c, int i) {
  if (c->per) {
    i %= c->nx;
    if (i < 0) i += c->nx;
  }
  return i;
}
static double DX(const ora_ctx *c, int i) { return c->dx[cw(c, i)]; }
static int solid(const ora_ctx *c, int i, int j) {
  return c->solid[IC(c, cw(c, i), j)];
}
/* cell (i,j) is inside the domain and fluid */
static int fluid(const ora_ctx *c, int i, int j) {
  if (j < 0 || j >= c->ny) return 0;
  if (!c->per && (i < 0 || i >= c->nx)) return 0;
  return !solid(c, i, j);
}
/* field accessors with the periodic wrap in x */
static double Uat(const ora_ctx *c, const double *u, int i, int j) {
  return u[IU(c, cw(c, i), j)];
}
static double Vat(const ora_ctx *c, const double *v, int i, int j) {
  return v[IV(c, cw(c, i), j)];
}
static double Cat(const ora_ctx *c, const double *a, int i, int j) {
  return a[IC(c, cw(c, i), j)];
}

/* u-face (i,j) is an unknown of the u-equation */
static int u_solved(const ora_ctx *c, int i, int j) {
  if (!c->per && (i <= 0 || i >= c->nx)) return 0;
  if (c->per && i == c->nx) return 0; /* copy of face 0 */
  return !solid(c, i - 1, j) && !solid(c, i, j);
}
/* v-face (i,j) is an unknown of the v-equation */
static int v_solved(const ora_ctx *c, int i, int j) {
  if (j <= 0 || j >= c->ny) return 0;
  return !solid(c, i, j - 1) && !solid(c, i, j);
}

/* TVD stencil validity: four consecutive points must exist.  Cell points
   must also be fluid; face points only need to lie in the array. */
static int cells_ok_x(const ora_ctx *c, int i0, int j) {
  for (int k = 0; k < 4; k++)
    if (!fluid(c, i0 + k, j)) return 0;
  return 1;
}
static int cells_ok_y(const ora_ctx *c, int i, int j0) {
  for (int k = 0; k < 4; k++)
    if (!fluid(c, i, j0 + k)) return 0;
  return 1;
}
static int ufaces_ok_x(const ora_ctx *c, int i0) {
  return c->per || (i0 >= 0 && i0 + 3 <= c->nx);
}
static int urows_ok(const ora_ctx *c, int j0) {
  return j0 >= 0 && j0 + 3 <= c->ny - 1;
}
static int vcols_ok(const ora_ctx *c, int i0) {
  return c->per || (i0 >= 0 && i0 + 3 <= c->nx - 1);
}
static int vrows_ok(const ora_ctx *c, int j0) {
  return j0 >= 0 && j0 + 3 <= c->ny;
}

/* ------------------------------------------------------------------ */
/* elementary functions                                               */
/* ------------------------------------------------------------------ */
static double dmax(double a, double b) { return a > b ? a : b; }

/* upwind(phi1, phi2, v) = phi1 if v > 0 else phi2   (eq. pl15_12) */
static double upwind(double f1, double f2, double vel) {
  return vel > 0 ? f1 : f2;
}

/* Test switch: with the limiter off every TVD correction is zero, which
   must give the upwind scheme bit for bit (Sec. 3.2 after pl15_2: with
   upwind approximation the corrections are null). */
static int limiter_on = 1;
void ora_set_limiter(int on) { limiter_on = on ? 1 : 0; }

/* van Leer limiter psi(r) (Sec. 3.2 after pl15_2) of r = a/b.  The printed
   denominator (1+r) is read as (1+|r|), the standard van Leer form the paper
   cites: both agree wherever the printed form is defined.  r <= 0 gives 0;
   r undefined (b == 0) is taken as 0; r overflowing to infinity gives the
   limit 2. */
double ora_vanleer(double a, double b) {
  if (!limiter_on) return 0.0;
  if (!((a > 0 && b > 0) || (a < 0 && b < 0))) return 0.0;
  double r = a / b;
  if (isinf(r)) return 2.0;
  return (r + fabs(r)) / (1.0 + fabs(r));
}

/* TVD correction at a surface between two nodes, non-uniform grid (pl15_2) */
double ora_psi_s(double f1, double f2, double f3, double f4, double d1,
                 double d2, double d3, double d4, double vel) {
  if (vel > 0)
    return d2 / (d2 + d3) *
           ora_vanleer((d2 + d3) * (f2 - f1), (d1 + d2) * (f3 - f2));
  return -d3 / (d2 + d3) *
         ora_vanleer((d2 + d3) * (f4 - f3), (d3 + d4) * (f3 - f2));
}
/* psi_s at x-face k of a cell-row stencil k-2 .. k+1 (widths of those
   cells), and at y-face k */
static double psi_x(const ora_ctx *c, double f1, double f2, double f3,
                    double f4, int k, double vel) {
  return ora_psi_s(f1, f2, f3, f4, DX(c, k - 2), DX(c, k - 1), DX(c, k),
                   DX(c, k + 1), vel);
}
static double psi_y(const ora_ctx *c, double f1, double f2, double f3,
                    double f4, int k, double vel) {
  return ora_psi_s(f1, f2, f3, f4, c->dy[k - 2], c->dy[k - 1], c->dy[k],
                   c->dy[k + 1], vel);
}

/* TVD correction at a control-volume centre (pl15_1) */
double ora_psi_c(double f1, double f2, double f3, double f4, double d1,
                 double d2, double d3, double vel) {
  if (vel > 0) return 0.5 * ora_vanleer(d2 * (f2 - f1), d1 * (f3 - f2));
  return -0.5 * ora_vanleer(d2 * (f4 - f3), d3 * (f3 - f2));
}

/* Nondimensional coefficients of eqs pl4-pl6 under convective scaling
   (U_ref = inlet speed, L_ref = channel height, T_in = p_in = rho_in = 1):
   A = 1/(gamma Ma^2), B = 1/Re, and the energy equation in internal-energy
   form (the discrete source pl29 carries p div(u), not Dp/Dt):
   C^{T1}_f = gamma/(Re Pr), C^{T2}_f = gamma(gamma-1)Ma^2/Re,
   C^{T3}_f = -(gamma-1). */
void ora_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int ora_max_threads(void) { return omp_get_max_threads(); }

void ora_params(double Ma, double Re, double Pr, double g, double out[5]) {
  out[0] = 1.0 / (g * Ma * Ma);
  out[1] = 1.0 / Re;
  out[2] = g / (Re * Pr);
  out[3] = g * (g - 1.0) * Ma * Ma / Re;
  out[4] = -(g - 1.0);
}

/* harmonic mean of Gamma between two nodes (pl33) */
static double gam_harm(double dl, double gl, double dr, double gr) {
  return (dl + dr) * gl * gr / (dl * gr + dr * gl);
}
/* harmonic mean of a node value and a boundary value over the half cell
   between them (pl33 with two equal halves) */
static double gam_harm2(double a, double b) { return 2.0 * a * b / (a + b); }

/* wall temperature of wall w at the x-position of u-face i */
static double wallT_uface(const ora_ctx *c, int w, int i) {
  int l = cw(c, i - 1), r = cw(c, i);
  double dl = c->dx[l], dr = c->dx[r];
  return (dr * c->wT[w][l] + dl * c->wT[w][r]) / (dl + dr);
}

/* Gamma at the corner (x^f_i, y^f_j), bilinear in the four surrounding
   cells (Sec. 3.2 after pl15).  Inlet corners interpolate sqrt(T_in) along
   y, outlet corners take the last column (zero gradient).  Corners on the
   channel walls only ever multiply wall velocities, which are zero: 0. */
static double gam_corner(const ora_ctx *c, const double *gam, int i, int j) {
  if (j <= 0 || j >= c->ny) return 0.0;
  double dys = c->dy[j - 1], dyn = c->dy[j];
  double ws = dyn / (dys + dyn), wn = dys / (dys + dyn);
  if (!c->per && i == 0)
    return ws * sqrt(c->T_in[j - 1]) + wn * sqrt(c->T_in[j]);
  if (!c->per && i == c->nx)
    return ws * gam[IC(c, c->nx - 1, j - 1)] + wn * gam[IC(c, c->nx - 1, j)];
  int l = cw(c, i - 1), r = cw(c, i);
  double dl = c->dx[l], dr = c->dx[r];
  double wl = dr / (dl + dr), wr = dl / (dl + dr);
  return ws * (wl * gam[IC(c, l, j - 1)] + wr * gam[IC(c, r, j - 1)]) +
         wn * (wl * gam[IC(c, l, j)] + wr * gam[IC(c, r, j)]);
}

/* ------------------------------------------------------------------ */
/* rho, Gamma, face densities and mass fluxes (pl8-pl11)              */
/* ------------------------------------------------------------------ */
static void cell_props(ora_ctx *c, const double *p, const double *T) {
  size_t n = (size_t)c->nx * c->ny;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < (long)n; k++) {
    c->rho[k] = p[k] / T[k];
    c->gam[k] = sqrt(T[k]);
  }
}

/* rho^u on every u-face and rho^v on every v-face: upwind value plus the
   TVD correction times the jump (pl10, pl11), then F^x = rho^u u dy,
   F^y = rho^v v dx (pl8, pl9). */
static void face_fluxes(ora_ctx *c, const double *u, const double *v,
                        int tvd) {
  const int nx = c->nx, ny = c->ny;
  const double *rho = c->rho;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; j++) {
    for (int i = 0; i <= nx; i++) {
      double r, uf = u[IU(c, i, j)];
      if (!c->per && i == 0) {
        r = upwind(c->p_in / c->T_in[j], rho[IC(c, 0, j)], uf);
      } else if (!c->per && i == nx) {
        r = rho[IC(c, nx - 1, j)];
      } else {
        double rl = Cat(c, rho, i - 1, j), rr = Cat(c, rho, i, j);
        r = upwind(rl, rr, uf);
        if (tvd && cells_ok_x(c, i - 2, j))
          r += psi_x(c, Cat(c, rho, i - 2, j), rl, rr, Cat(c, rho, i + 1, j), i, uf) *
               (rr - rl);
      }
      c->rhou[IU(c, i, j)] = r;
      c->Fx[IU(c, i, j)] = r * uf * c->dy[j];
    }
  }
#pragma omp parallel for schedule(static)
  for (int j = 0; j <= ny; j++) {
    for (int i = 0; i < nx; i++) {
      double r, vf = v[IV(c, i, j)];
      if (j == 0) {
        r = rho[IC(c, i, 0)];
      } else if (j == ny) {
        r = rho[IC(c, i, ny - 1)];
      } else {
        double rs = rho[IC(c, i, j - 1)], rn = rho[IC(c, i, j)];
        r = upwind(rs, rn, vf);
        if (tvd && cells_ok_y(c, i, j - 2))
          r += psi_y(c, rho[IC(c, i, j - 2)], rs, rn, rho[IC(c, i, j + 1)], j, vf) *
               (rn - rs);
      }
      c->rhov[IV(c, i, j)] = r;
      c->Fy[IV(c, i, j)] = r * vf * c->dx[i];
    }
  }
}

/* ------------------------------------------------------------------ */
/* explicit convective terms, from the n-1 fields (pl15_11, pl31_1)   */
/* Called with rho, rhou, rhov, Fx, Fy computed from the n-1 fields.  */
/* ------------------------------------------------------------------ */
static double T_explicit(const ora_ctx *c, int i, int j, int tvd) {
  const double *T = c->Tm, *u = c->um, *v = c->vm;
  double TP = T[IC(c, i, j)];
  double TW = (!c->per && i == 0) ? c->T_in[j] : Cat(c, T, i - 1, j);
  double TE = (!c->per && i == c->nx - 1) ? TP : Cat(c, T, i + 1, j);
  double TS = (j == 0) ? TP : T[IC(c, i, j - 1)];
  double TN = (j == c->ny - 1) ? TP : T[IC(c, i, j + 1)];
  double FW = c->Fx[IU(c, i, j)], FE = c->Fx[IU(c, i + 1, j)];
  double FS = c->Fy[IV(c, i, j)], FN = c->Fy[IV(c, i, j + 1)];
  double uW = u[IU(c, i, j)], uE = u[IU(c, i + 1, j)];
  double vS = v[IV(c, i, j)], vN = v[IV(c, i, j + 1)];
  double pW = 0, pE = 0, pS = 0, pN = 0;
  if (tvd) {
    if (cells_ok_x(c, i - 1, j))
      pE = psi_x(c, Cat(c, T, i - 1, j), TP, TE, Cat(c, T, i + 2, j), i + 1, uE);
    if (cells_ok_x(c, i - 2, j))
      pW = psi_x(c, Cat(c, T, i - 2, j), TW, TP, TE, i, uW);
    if (cells_ok_y(c, i, j - 1))
      pN = psi_y(c, T[IC(c, i, j - 1)], TP, TN, T[IC(c, i, j + 2)], j + 1, vN);
    if (cells_ok_y(c, i, j - 2))
      pS = psi_y(c, T[IC(c, i, j - 2)], TS, TP, TN, j, vS);
  }
  return -FE * (upwind(TP, TE, uE) + (TE - TP) * pE) +
         FW * (upwind(TW, TP, uW) + (TP - TW) * pW) -
         FN * (upwind(TP, TN, vN) + (TN - TP) * pN) +
         FS * (upwind(TS, TP, vS) + (TP - TS) * pS);
}

/* v^explicit (pl15_11) */
static double v_explicit(const ora_ctx *c, int i, int j, int tvd) {
  const double *u = c->um, *v = c->vm, *rho = c->rho;
  double vP = v[IV(c, i, j)];
  double vW = (!c->per && i == 0) ? 0.0 : Vat(c, v, i - 1, j);
  double vE = (!c->per && i == c->nx - 1) ? vP : Vat(c, v, i + 1, j);
  double vS = v[IV(c, i, j - 1)], vN = v[IV(c, i, j + 1)];
  double dxi = c->dx[i];
  /* x-direction: two half faces on each side, fluxes F^x at u-faces */
  double Fe0 = c->Fx[IU(c, i + 1, j - 1)], Fe1 = c->Fx[IU(c, i + 1, j)];
  double Fw0 = c->Fx[IU(c, i, j - 1)], Fw1 = c->Fx[IU(c, i, j)];
  double ue0 = Uat(c, u, i + 1, j - 1), ue1 = Uat(c, u, i + 1, j);
  double uw0 = Uat(c, u, i, j - 1), uw1 = Uat(c, u, i, j);
  double pe0 = 0, pe1 = 0, pw0 = 0, pw1 = 0, pn = 0, ps = 0;
  double vbN = 0.5 * (vP + vN), vbS = 0.5 * (vS + vP);
  if (tvd) {
    if (vcols_ok(c, i - 1)) {
      double f1 = Vat(c, v, i - 1, j), f4 = Vat(c, v, i + 2, j);
      pe0 = psi_x(c, f1, vP, vE, f4, i + 1, ue0);
      pe1 = psi_x(c, f1, vP, vE, f4, i + 1, ue1);
    }
    if (vcols_ok(c, i - 2)) {
      double f1 = Vat(c, v, i - 2, j), f4 = Vat(c, v, i + 1, j);
      pw0 = psi_x(c, f1, vW, vP, f4, i, uw0);
      pw1 = psi_x(c, f1, vW, vP, f4, i, uw1);
    }
    if (vrows_ok(c, j - 1))
      pn = ora_psi_c(vS, vP, vN, v[IV(c, i, j + 2)], c->dy[j - 1], c->dy[j],
                     c->dy[j + 1], vbN);
    if (vrows_ok(c, j - 2))
      ps = ora_psi_c(v[IV(c, i, j - 2)], vS, vP, vN, c->dy[j - 2],
                     c->dy[j - 1], c->dy[j], vbS);
  }
  double FbN = rho[IC(c, i, j)] * vbN * dxi;
  double FbS = rho[IC(c, i, j - 1)] * vbS * dxi;
  return -0.5 * (Fe0 * (upwind(vP, vE, ue0) + (vE - vP) * pe0) +
                 Fe1 * (upwind(vP, vE, ue1) + (vE - vP) * pe1)) +
         0.5 * (Fw0 * (upwind(vW, vP, uw0) + (vP - vW) * pw0) +
                Fw1 * (upwind(vW, vP, uw1) + (vP - vW) * pw1)) -
         FbN * (upwind(vP, vN, vbN) + (vN - vP) * pn) +
         FbS * (upwind(vS, vP, vbS) + (vP - vS) * ps);
}

/* u^explicit: x<->y mirror image of pl15_11 */
static double u_explicit(const ora_ctx *c, int i, int j, int tvd) {
  const double *u = c->um, *v = c->vm, *rho = c->rho;
  int l = cw(c, i - 1), r = cw(c, i);
  double uP = Uat(c, u, i, j);
  double uW = Uat(c, u, i - 1, j), uE = Uat(c, u, i + 1, j);
  double uS = (j == 0) ? uP : u[IU(c, cw(c, i), j - 1)];
  double uN = (j == c->ny - 1) ? uP : u[IU(c, cw(c, i), j + 1)];
  double dyj = c->dy[j];
  double Fn0 = c->Fy[IV(c, l, j + 1)], Fn1 = c->Fy[IV(c, r, j + 1)];
  double Fs0 = c->Fy[IV(c, l, j)], Fs1 = c->Fy[IV(c, r, j)];
  double vn0 = v[IV(c, l, j + 1)], vn1 = v[IV(c, r, j + 1)];
  double vs0 = v[IV(c, l, j)], vs1 = v[IV(c, r, j)];
  double pn0 = 0, pn1 = 0, ps0 = 0, ps1 = 0, pe = 0, pw = 0;
  double ubE = 0.5 * (uP + uE), ubW = 0.5 * (uW + uP);
  if (tvd) {
    if (urows_ok(c, j - 1)) {
      double f1 = u[IU(c, r, j - 1)], f4 = u[IU(c, r, j + 2)];
      pn0 = psi_y(c, f1, uP, uN, f4, j + 1, vn0);
      pn1 = psi_y(c, f1, uP, uN, f4, j + 1, vn1);
    }
    if (urows_ok(c, j - 2)) {
      double f1 = u[IU(c, r, j - 2)], f4 = u[IU(c, r, j + 1)];
      ps0 = psi_y(c, f1, uS, uP, f4, j, vs0);
      ps1 = psi_y(c, f1, uS, uP, f4, j, vs1);
    }
    if (ufaces_ok_x(c, i - 1))
      pe = ora_psi_c(uW, uP, uE, Uat(c, u, i + 2, j), DX(c, i - 1), DX(c, i),
                     DX(c, i + 1), ubE);
    if (ufaces_ok_x(c, i - 2))
      pw = ora_psi_c(Uat(c, u, i - 2, j), uW, uP, uE, DX(c, i - 2),
                     DX(c, i - 1), DX(c, i), ubW);
  }
  double FbE = rho[IC(c, r, j)] * ubE * dyj;
  double FbW = rho[IC(c, l, j)] * ubW * dyj;
  return -0.5 * (Fn0 * (upwind(uP, uN, vn0) + (uN - uP) * pn0) +
                 Fn1 * (upwind(uP, uN, vn1) + (uN - uP) * pn1)) +
         0.5 * (Fs0 * (upwind(uS, uP, vs0) + (uP - uS) * ps0) +
                Fs1 * (upwind(uS, uP, vs1) + (uP - uS) * ps1)) -
         FbE * (upwind(uP, uE, ubE) + (uE - uP) * pe) +
         FbW * (upwind(uW, uP, ubW) + (uP - uW) * pw);
}

/* ------------------------------------------------------------------ */
/* temperature equation coefficients (pl30-pl33, pl28, pl29)          */
/* ------------------------------------------------------------------ */
typedef struct {
  double a[4], nb[4]; /* W, E, S, N */
  double a0, src, texp, unst;
} tco;

/* Velocity-slip / temperature-jump walls (pl38, pl39).  With the normal
   derivative taken between the wall and the node at distance d/2, pl38
   reads u_s - u_w = zeta (u_P - u_s) / (d/2): the gas velocity at the wall
   is u_s = (u_w d/2 + zeta u_P) / (d/2 + zeta) and the wall shear
   mu (u_P - u_s) / (d/2) = mu (u_P - u_w) / (d/2 + zeta), i.e. the no-slip
   half-cell conductance with the distance d/2 + zeta.  pl39 gives the same
   for the conduction with tau.  zeta = 1.1466 Kn / rho, tau = 2.1904 Kn /
   rho, rho the density of the node next to the wall (the cell for T, the
   face node for u and v). */
static double iwall(double d, double k, double rho) {
  return 1.0 / (0.5 * d + k / rho);
}
static double slip_vel(double uw, double uP, double d, double zeta) {
  return (uw * (0.5 * d) + zeta * uP) / (0.5 * d + zeta);
}

/* face-centre velocities for the dissipation term (Sec. 3.2 after pl29):
   v at (x^f_{i+1}, y^v_j) and (x^f_i, y^v_j), u at (x^v_i, y^f_{j+1}) and
   (x^v_i, y^f_j), bilinear between the four nearest nodes; a point on a
   wall takes the wall velocity (the slip velocity at a slip / jump wall,
   with the cell-centre value as the node value), the inlet v is 0, the
   outlet has zero gradient. */
static void face_centre_vel(const ora_ctx *c, int i, int j, double *vE,
                            double *vW, double *uN, double *uS) {
  const double *u = c->u, *v = c->v;
  const double zP = c->kz / c->rho[IC(c, i, j)];
  double vc = 0.5 * (v[IV(c, i, j)] + v[IV(c, i, j + 1)]);
  if (!c->per && i == c->nx - 1) {
    *vE = vc;
  } else if (solid(c, i + 1, j)) {
    *vE = (c->otype == 2) ? slip_vel(0.0, vc, c->dx[i], zP) : 0.0;
  } else {
    int r = cw(c, i + 1);
    double dxi = c->dx[i], dr = c->dx[r];
    *vE = dr / (dxi + dr) * vc +
          dxi / (dxi + dr) * (0.5 * (v[IV(c, r, j)] + v[IV(c, r, j + 1)]));
  }
  if (!c->per && i == 0) {
    *vW = 0.0;
  } else if (solid(c, i - 1, j)) {
    *vW = (c->otype == 2) ? slip_vel(0.0, vc, c->dx[i], zP) : 0.0;
  } else {
    int l = cw(c, i - 1);
    double dxi = c->dx[i], dl = c->dx[l];
    *vW = dxi / (dl + dxi) * (0.5 * (v[IV(c, l, j)] + v[IV(c, l, j + 1)])) +
          dl / (dl + dxi) * vc;
  }
  double uc = 0.5 * (Uat(c, u, i, j) + Uat(c, u, i + 1, j));
  if (j == c->ny - 1) {
    *uN = (c->wtype[1] == 0)   ? c->wu[1]
          : (c->wtype[1] == 2) ? slip_vel(c->wu[1], uc, c->dy[j], zP)
                               : uc;
  } else if (solid(c, i, j + 1)) {
    *uN = (c->otype == 2) ? slip_vel(0.0, uc, c->dy[j], zP) : 0.0;
  } else {
    double dyj = c->dy[j], dn = c->dy[j + 1];
    *uN = dn / (dyj + dn) * uc +
          dyj / (dyj + dn) *
              (0.5 * (Uat(c, u, i, j + 1) + Uat(c, u, i + 1, j + 1)));
  }
  if (j == 0) {
    *uS = (c->wtype[0] == 0)   ? c->wu[0]
          : (c->wtype[0] == 2) ? slip_vel(c->wu[0], uc, c->dy[j], zP)
                               : uc;
  } else if (solid(c, i, j - 1)) {
    *uS = (c->otype == 2) ? slip_vel(0.0, uc, c->dy[j], zP) : 0.0;
  } else {
    double dyj = c->dy[j], ds = c->dy[j - 1];
    *uS = dyj / (ds + dyj) *
              (0.5 * (Uat(c, u, i, j - 1) + Uat(c, u, i + 1, j - 1))) +
          ds / (ds + dyj) * uc;
  }
}

static tco T_coefs(const ora_ctx *c, int i, int j, double dt, int scheme) {
  const int implicit = scheme & ORA_IMPLICIT, tvd = scheme & ORA_TVD;
  const double *T = c->T, *gam = c->gam;
  tco q;
  double dxi = c->dx[i], dyj = c->dy[j], dV = dxi * dyj;
  double gP = gam[IC(c, i, j)], TP = T[IC(c, i, j)];
  double rhoP = c->rho[IC(c, i, j)];
  /* a face on an obstacle: half-cell conductance with the harmonic mean of
     the cell's and the surface's Gamma (no-slip isothermal), or with the
     cell's Gamma over the distance d/2 + tau (temperature jump) */
  const int jump = (c->otype == 2);
  double D[4], F[4], psi[4] = {0, 0, 0, 0};
  /* west face x^f_i */
  if (!c->per && i == 0) { /* inlet: T_in on the face, half cell away */
    q.nb[0] = c->T_in[j];
    D[0] = c->C1 * gam_harm2(gP, sqrt(c->T_in[j])) * dyj / (0.5 * dxi);
  } else {
    int l = cw(c, i - 1);
    q.nb[0] = T[IC(c, l, j)];
    if (c->solid[IC(c, l, j)])
      D[0] = jump ? c->C1 * gP * dyj * iwall(dxi, c->kt, rhoP)
                  : c->C1 * gam_harm2(gP, sqrt(c->obsT)) * dyj / (0.5 * dxi);
    else
      D[0] = c->C1 * gam_harm(c->dx[l], gam[IC(c, l, j)], dxi, gP) * dyj /
             (0.5 * (dxi + c->dx[l]));
  }
  /* east face x^f_{i+1} */
  if (!c->per && i == c->nx - 1) { /* outlet: zero gradient */
    q.nb[1] = TP;
    D[1] = 0.0;
  } else {
    int r = cw(c, i + 1);
    q.nb[1] = T[IC(c, r, j)];
    if (c->solid[IC(c, r, j)])
      D[1] = jump ? c->C1 * gP * dyj * iwall(dxi, c->kt, rhoP)
                  : c->C1 * gam_harm2(gP, sqrt(c->obsT)) * dyj / (0.5 * dxi);
    else
      D[1] = c->C1 * gam_harm(dxi, gP, c->dx[r], gam[IC(c, r, j)]) * dyj /
             (0.5 * (dxi + c->dx[r]));
  }
  /* south face y^f_j */
  if (j == 0) {
    if (c->wtype[0] == 0) {
      q.nb[2] = c->wT[0][i];
      D[2] = c->C1 * gam_harm2(gP, sqrt(c->wT[0][i])) * dxi / (0.5 * dyj);
    } else if (c->wtype[0] == 2) {
      q.nb[2] = c->wT[0][i];
      D[2] = c->C1 * gP * dxi * iwall(dyj, c->kt, rhoP);
    } else {
      q.nb[2] = TP;
      D[2] = 0.0;
    }
  } else {
    q.nb[2] = T[IC(c, i, j - 1)];
    if (c->solid[IC(c, i, j - 1)])
      D[2] = jump ? c->C1 * gP * dxi * iwall(dyj, c->kt, rhoP)
                  : c->C1 * gam_harm2(gP, sqrt(c->obsT)) * dxi / (0.5 * dyj);
    else
      D[2] = c->C1 * gam_harm(c->dy[j - 1], gam[IC(c, i, j - 1)], dyj, gP) *
             dxi / (0.5 * (dyj + c->dy[j - 1]));
  }
  /* north face y^f_{j+1} */
  if (j == c->ny - 1) {
    if (c->wtype[1] == 0) {
      q.nb[3] = c->wT[1][i];
      D[3] = c->C1 * gam_harm2(gP, sqrt(c->wT[1][i])) * dxi / (0.5 * dyj);
    } else if (c->wtype[1] == 2) {
      q.nb[3] = c->wT[1][i];
      D[3] = c->C1 * gP * dxi * iwall(dyj, c->kt, rhoP);
    } else {
      q.nb[3] = TP;
      D[3] = 0.0;
    }
  } else {
    q.nb[3] = T[IC(c, i, j + 1)];
    if (c->solid[IC(c, i, j + 1)])
      D[3] = jump ? c->C1 * gP * dxi * iwall(dyj, c->kt, rhoP)
                  : c->C1 * gam_harm2(gP, sqrt(c->obsT)) * dxi / (0.5 * dyj);
    else
      D[3] = c->C1 * gam_harm(dyj, gP, c->dy[j + 1], gam[IC(c, i, j + 1)]) *
             dxi / (0.5 * (dyj + c->dy[j + 1]));
  }
  F[0] = c->Fx[IU(c, i, j)];
  F[1] = c->Fx[IU(c, i + 1, j)];
  F[2] = c->Fy[IV(c, i, j)];
  F[3] = c->Fy[IV(c, i, j + 1)];
  if (implicit) {
    if (tvd) {
      double uW = c->u[IU(c, i, j)], uE = c->u[IU(c, i + 1, j)];
      double vS = c->v[IV(c, i, j)], vN = c->v[IV(c, i, j + 1)];
      if (cells_ok_x(c, i - 2, j))
        psi[0] = psi_x(c, Cat(c, T, i - 2, j), Cat(c, T, i - 1, j), TP, Cat(c, T, i + 1, j), i, uW);
      if (cells_ok_x(c, i - 1, j))
        psi[1] = psi_x(c, Cat(c, T, i - 1, j), TP, Cat(c, T, i + 1, j), Cat(c, T, i + 2, j), i + 1, uE);
      if (cells_ok_y(c, i, j - 2))
        psi[2] = psi_y(c, T[IC(c, i, j - 2)], T[IC(c, i, j - 1)], TP, T[IC(c, i, j + 1)], j, vS);
      if (cells_ok_y(c, i, j - 1))
        psi[3] = psi_y(c, T[IC(c, i, j - 1)], TP, T[IC(c, i, j + 1)], T[IC(c, i, j + 2)], j + 1, vN);
    }
    q.a[0] = dmax(0.0, F[0]) - F[0] * psi[0] + D[0];
    q.a[1] = dmax(0.0, -F[1]) - F[1] * psi[1] + D[1];
    q.a[2] = dmax(0.0, F[2]) - F[2] * psi[2] + D[2];
    q.a[3] = dmax(0.0, -F[3]) - F[3] * psi[3] + D[3];
    /* net outflow grouped on its own: it is exactly zero in a uniform flow */
    q.a0 = dt * ((q.a[0] + q.a[1] + q.a[2] + q.a[3]) +
                 ((F[1] - F[0]) + (F[3] - F[2]))) +
           rhoP * dV;
  } else {
    for (int k = 0; k < 4; k++) q.a[k] = D[k];
    q.a0 = dt * (q.a[0] + q.a[1] + q.a[2] + q.a[3]) + rhoP * dV;
  }
  /* source S^T_c (pl29), S^T_p = 0 (pl28) */
  double vE, vW, uN, uS;
  face_centre_vel(c, i, j, &vE, &vW, &uN, &uS);
  double ux = (Uat(c, c->u, i + 1, j) - Uat(c, c->u, i, j)) / dxi;
  double vy = (c->v[IV(c, i, j + 1)] - c->v[IV(c, i, j)]) / dyj;
  double vx = (vE - vW) / dxi, uy = (uN - uS) / dyj;
  double div = ux + vy;
  q.src = c->C2 * gP *
              (2.0 * (ux * ux + vy * vy) + (vx + uy) * (vx + uy) -
               2.0 / 3.0 * div * div) *
              dV +
          c->C3 * c->p[IC(c, i, j)] * div * dV;
  q.texp = (scheme & ORA_IMPLICIT) ? 0.0 : c->Texp[IC(c, i, j)];
  q.unst = (c->pm[IC(c, i, j)] / c->Tm[IC(c, i, j)]) * c->Tm[IC(c, i, j)] * dV;
  return q;
}

/* ------------------------------------------------------------------ */
/* momentum equations: v printed (pl14-pl16, pl15, pl21), u mirrored  */
/* ------------------------------------------------------------------ */
typedef struct {
  double a[4], nb[4]; /* W, E, S, N */
  double a0, b, len;  /* len: face length of the pressure force */
} mco;

static mco v_coefs(const ora_ctx *c, int i, int j, double dt, int scheme) {
  const int implicit = scheme & ORA_IMPLICIT, tvd = scheme & ORA_TVD;
  const double *u = c->u, *v = c->v, *rho = c->rho, *gam = c->gam;
  mco q;
  double dxi = c->dx[i], dys = c->dy[j - 1], dyn = c->dy[j];
  double rs = rho[IC(c, i, j - 1)], rn = rho[IC(c, i, j)];
  double gs = gam[IC(c, i, j - 1)], gn = gam[IC(c, i, j)];
  double vP = v[IV(c, i, j)], vS = v[IV(c, i, j - 1)], vN = v[IV(c, i, j + 1)];
  double vW = (!c->per && i == 0) ? 0.0 : Vat(c, v, i - 1, j);
  double vE = (!c->per && i == c->nx - 1) ? vP : Vat(c, v, i + 1, j);
  double M = (rn * dyn + rs * dys) * dxi / 2.0;
  double len = 0.5 * (dys + dyn);
  /* Gamma at the v-node, linear in y between the two cells */
  double gnode = (dyn * gs + dys * gn) / (dys + dyn);
  /* a face on an obstacle in x: half-cell shear with the mean of the
     node's and the surface's Gamma (no slip), or with the node's Gamma over
     the distance d/2 + zeta, zeta from the node density (velocity slip) */
  const int slip = (c->otype == 2);
  const double rnode = (dyn * rs + dys * rn) / (dys + dyn);
  double DW, DE;
  if (!c->per && i == 0) {
    DW = c->B * 0.5 * (gnode + gam_corner(c, gam, 0, j)) * len / (0.5 * dxi);
  } else {
    int l = cw(c, i - 1);
    if (solid(c, l, j - 1) && solid(c, l, j))
      DW = slip ? c->B * gnode * len * iwall(dxi, c->kz, rnode)
                : c->B * 0.5 * (gnode + sqrt(c->obsT)) * len / (0.5 * dxi);
    else
      DW = c->B * gam_corner(c, gam, i, j) * (dyn + dys) / (dxi + DX(c, i - 1));
  }
  if (!c->per && i == c->nx - 1) {
    DE = 0.0;
  } else {
    int r = cw(c, i + 1);
    if (solid(c, r, j - 1) && solid(c, r, j))
      DE = slip ? c->B * gnode * len * iwall(dxi, c->kz, rnode)
                : c->B * 0.5 * (gnode + sqrt(c->obsT)) * len / (0.5 * dxi);
    else
      DE = c->B * gam_corner(c, gam, i + 1, j) * (dyn + dys) / (DX(c, i + 1) + dxi);
  }
  double DS = c->B * gs * dxi / dys, DN = c->B * gn * dxi / dyn;
  double conv = 0.0;
  if (implicit) {
    double Fw0 = c->Fx[IU(c, i, j)], Fw1 = c->Fx[IU(c, i, j - 1)];
    double Fe0 = c->Fx[IU(c, i + 1, j)], Fe1 = c->Fx[IU(c, i + 1, j - 1)];
    double vbS = 0.5 * (vS + vP), vbN = 0.5 * (vP + vN);
    double FbS = rs * vbS * dxi, FbN = rn * vbN * dxi;
    double pw0 = 0, pw1 = 0, pe0 = 0, pe1 = 0, ps = 0, pn = 0;
    if (tvd) {
      if (vcols_ok(c, i - 2)) {
        double f1 = Vat(c, v, i - 2, j), f4 = Vat(c, v, i + 1, j);
        pw0 = psi_x(c, f1, vW, vP, f4, i, Uat(c, u, i, j));
        pw1 = psi_x(c, f1, vW, vP, f4, i, Uat(c, u, i, j - 1));
      }
      if (vcols_ok(c, i - 1)) {
        double f1 = Vat(c, v, i - 1, j), f4 = Vat(c, v, i + 2, j);
        pe0 = psi_x(c, f1, vP, vE, f4, i + 1, Uat(c, u, i + 1, j));
        pe1 = psi_x(c, f1, vP, vE, f4, i + 1, Uat(c, u, i + 1, j - 1));
      }
      if (vrows_ok(c, j - 2))
        ps = ora_psi_c(v[IV(c, i, j - 2)], vS, vP, vN, c->dy[j - 2], dys, dyn,
                       vbS);
      if (vrows_ok(c, j - 1))
        pn = ora_psi_c(vS, vP, vN, v[IV(c, i, j + 2)], dys, dyn, c->dy[j + 1],
                       vbN);
    }
    q.a[0] = 0.5 * (dmax(0.0, Fw0) - Fw0 * pw0 + dmax(0.0, Fw1) - Fw1 * pw1) +
             DW;
    q.a[1] =
        0.5 * (dmax(0.0, -Fe0) - Fe0 * pe0 + dmax(0.0, -Fe1) - Fe1 * pe1) + DE;
    q.a[2] = dmax(0.0, FbS) - FbS * ps + 4.0 / 3.0 * DS;
    q.a[3] = dmax(0.0, -FbN) - FbN * pn + 4.0 / 3.0 * DN;
    conv = 0.5 * (Fe0 - Fw0 + Fe1 - Fw1) + FbN - FbS;
  } else {
    q.a[0] = DW;
    q.a[1] = DE;
    q.a[2] = 4.0 / 3.0 * DS;
    q.a[3] = 4.0 / 3.0 * DN;
  }
  q.a0 = q.a[0] + q.a[1] + q.a[2] + q.a[3] + conv + M / dt;
  double Mm = (c->pm[IC(c, i, j)] / c->Tm[IC(c, i, j)] * dyn +
               c->pm[IC(c, i, j - 1)] / c->Tm[IC(c, i, j - 1)] * dys) *
              dxi / 2.0;
  double X = gam_corner(c, gam, i + 1, j) *
                 (Uat(c, u, i + 1, j) - Uat(c, u, i + 1, j - 1)) -
             gam_corner(c, gam, i, j) * (Uat(c, u, i, j) - Uat(c, u, i, j - 1)) -
             2.0 / 3.0 * gn * (Uat(c, u, i + 1, j) - Uat(c, u, i, j)) +
             2.0 / 3.0 * gs * (Uat(c, u, i + 1, j - 1) - Uat(c, u, i, j - 1));
  /* b^v (pl14) + v^explicit (pl21): the part fixed for the whole step
     first, then the cross-diffusion of the current iterate */
  q.b = (Mm / dt * c->vm[IV(c, i, j)] + c->gy * Mm +
         ((scheme & ORA_IMPLICIT) ? 0.0 : c->vexp[IV(c, i, j)])) +
        c->B * X;
  q.nb[0] = vW;
  q.nb[1] = vE;
  q.nb[2] = vS;
  q.nb[3] = vN;
  q.len = dxi;
  return q;
}

static mco u_coefs(const ora_ctx *c, int i, int j, double dt, int scheme) {
  const int implicit = scheme & ORA_IMPLICIT, tvd = scheme & ORA_TVD;
  const double *u = c->u, *v = c->v, *rho = c->rho, *gam = c->gam;
  mco q;
  int l = cw(c, i - 1), r = cw(c, i);
  double dxl = c->dx[l], dxr = c->dx[r], dyj = c->dy[j];
  double rl = rho[IC(c, l, j)], rr = rho[IC(c, r, j)];
  double gl = gam[IC(c, l, j)], gr = gam[IC(c, r, j)];
  double uP = Uat(c, u, i, j), uW = Uat(c, u, i - 1, j),
         uE = Uat(c, u, i + 1, j);
  double uS, uN, DS, DN;
  double M = (rr * dxr + rl * dxl) * dyj / 2.0;
  double len = 0.5 * (dxl + dxr);
  /* Gamma at the u-node, linear in x between the two cells */
  double gnode = (dxr * gl + dxl * gr) / (dxl + dxr);
  /* node density for the slip length of pl38; obstacle faces in y as in
     v_coefs */
  const int slip = (c->otype == 2);
  const double rnode = (dxr * rl + dxl * rr) / (dxl + dxr);
  if (j == 0) {
    if (c->wtype[0] == 0) {
      uS = c->wu[0];
      DS = c->B * 0.5 * (gnode + sqrt(wallT_uface(c, 0, i))) * len / (0.5 * dyj);
    } else if (c->wtype[0] == 2) {
      uS = c->wu[0];
      DS = c->B * gnode * len * iwall(dyj, c->kz, rnode);
    } else {
      uS = uP;
      DS = 0.0;
    }
  } else {
    uS = u[IU(c, r, j - 1)];
    if (solid(c, l, j - 1) && solid(c, r, j - 1))
      DS = slip ? c->B * gnode * len * iwall(dyj, c->kz, rnode)
                : c->B * 0.5 * (gnode + sqrt(c->obsT)) * len / (0.5 * dyj);
    else
      DS = c->B * gam_corner(c, gam, i, j) * (dxr + dxl) / (dyj + c->dy[j - 1]);
  }
  if (j == c->ny - 1) {
    if (c->wtype[1] == 0) {
      uN = c->wu[1];
      DN = c->B * 0.5 * (gnode + sqrt(wallT_uface(c, 1, i))) * len / (0.5 * dyj);
    } else if (c->wtype[1] == 2) {
      uN = c->wu[1];
      DN = c->B * gnode * len * iwall(dyj, c->kz, rnode);
    } else {
      uN = uP;
      DN = 0.0;
    }
  } else {
    uN = u[IU(c, r, j + 1)];
    if (solid(c, l, j + 1) && solid(c, r, j + 1))
      DN = slip ? c->B * gnode * len * iwall(dyj, c->kz, rnode)
                : c->B * 0.5 * (gnode + sqrt(c->obsT)) * len / (0.5 * dyj);
    else
      DN = c->B * gam_corner(c, gam, i, j + 1) * (dxr + dxl) / (c->dy[j + 1] + dyj);
  }
  double DW = c->B * gl * dyj / dxl, DE = c->B * gr * dyj / dxr;
  double conv = 0.0;
  if (implicit) {
    double Fs0 = c->Fy[IV(c, r, j)], Fs1 = c->Fy[IV(c, l, j)];
    double Fn0 = c->Fy[IV(c, r, j + 1)], Fn1 = c->Fy[IV(c, l, j + 1)];
    double ubW = 0.5 * (uW + uP), ubE = 0.5 * (uP + uE);
    double FbW = rl * ubW * dyj, FbE = rr * ubE * dyj;
    double ps0 = 0, ps1 = 0, pn0 = 0, pn1 = 0, pw = 0, pe = 0;
    if (tvd) {
      if (urows_ok(c, j - 2)) {
        double f1 = u[IU(c, r, j - 2)], f4 = u[IU(c, r, j + 1)];
        ps0 = psi_y(c, f1, uS, uP, f4, j, v[IV(c, r, j)]);
        ps1 = psi_y(c, f1, uS, uP, f4, j, v[IV(c, l, j)]);
      }
      if (urows_ok(c, j - 1)) {
        double f1 = u[IU(c, r, j - 1)], f4 = u[IU(c, r, j + 2)];
        pn0 = psi_y(c, f1, uP, uN, f4, j + 1, v[IV(c, r, j + 1)]);
        pn1 = psi_y(c, f1, uP, uN, f4, j + 1, v[IV(c, l, j + 1)]);
      }
      if (ufaces_ok_x(c, i - 2))
        pw = ora_psi_c(Uat(c, u, i - 2, j), uW, uP, uE, DX(c, i - 2), dxl, dxr,
                       ubW);
      if (ufaces_ok_x(c, i - 1))
        pe = ora_psi_c(uW, uP, uE, Uat(c, u, i + 2, j), dxl, dxr,
                       DX(c, i + 1), ubE);
    }
    /* order mirrors the printed v-coefficients: the cross-direction
       half-face pairs are the "south/north" pair of v */
    q.a[2] = 0.5 * (dmax(0.0, Fs0) - Fs0 * ps0 + dmax(0.0, Fs1) - Fs1 * ps1) +
             DS;
    q.a[3] =
        0.5 * (dmax(0.0, -Fn0) - Fn0 * pn0 + dmax(0.0, -Fn1) - Fn1 * pn1) + DN;
    q.a[0] = dmax(0.0, FbW) - FbW * pw + 4.0 / 3.0 * DW;
    q.a[1] = dmax(0.0, -FbE) - FbE * pe + 4.0 / 3.0 * DE;
    conv = 0.5 * (Fn0 - Fs0 + Fn1 - Fs1) + FbE - FbW;
  } else {
    q.a[2] = DS;
    q.a[3] = DN;
    q.a[0] = 4.0 / 3.0 * DW;
    q.a[1] = 4.0 / 3.0 * DE;
  }
  q.a0 = q.a[2] + q.a[3] + q.a[0] + q.a[1] + conv + M / dt;
  double Mm = (c->pm[IC(c, r, j)] / c->Tm[IC(c, r, j)] * dxr +
               c->pm[IC(c, l, j)] / c->Tm[IC(c, l, j)] * dxl) *
              dyj / 2.0;
  double X = gam_corner(c, gam, i, j + 1) *
                 (v[IV(c, r, j + 1)] - v[IV(c, l, j + 1)]) -
             gam_corner(c, gam, i, j) * (v[IV(c, r, j)] - v[IV(c, l, j)]) -
             2.0 / 3.0 * gr * (v[IV(c, r, j + 1)] - v[IV(c, r, j)]) +
             2.0 / 3.0 * gl * (v[IV(c, l, j + 1)] - v[IV(c, l, j)]);
  q.b = (Mm / dt * Uat(c, c->um, i, j) + c->gx * Mm +
         ((scheme & ORA_IMPLICIT) ? 0.0 : c->uexp[IU(c, r, j)])) +
        c->B * X;
  q.nb[0] = uW;
  q.nb[1] = uE;
  q.nb[2] = uS;
  q.nb[3] = uN;
  q.len = dyj;
  return q;
}

/* numerator of the Jacobi update: a_S phi_S + a_N phi_N + a_W phi_W +
   a_E phi_E (u) or a_W phi_W + a_E phi_E + a_S phi_S + a_N phi_N (v, T),
   in the same order as the sums in a0 */
static double nbsum_u(const mco *q) {
  return q->a[2] * q->nb[2] + q->a[3] * q->nb[3] + q->a[0] * q->nb[0] +
         q->a[1] * q->nb[1];
}
static double nbsum_v(const mco *q) {
  return q->a[0] * q->nb[0] + q->a[1] * q->nb[1] + q->a[2] * q->nb[2] +
         q->a[3] * q->nb[3];
}

/* ------------------------------------------------------------------ */
/* boundary values                                                    */
/* ------------------------------------------------------------------ */
static void impose_bc(ora_ctx *c, double *u, double *v, double *p,
                      double *T) {
  const int nx = c->nx, ny = c->ny;
  for (int j = 0; j < ny; j++) {
    for (int i = 0; i < nx; i++)
      if (c->solid[IC(c, i, j)]) {
        T[IC(c, i, j)] = c->obsT;
        p[IC(c, i, j)] = c->p_in;
      }
    for (int i = 0; i <= nx; i++) {
      if (!c->per && i == 0)
        u[IU(c, i, j)] = c->u_in[j];
      else if (!c->per && i == nx)
        continue;
      else if (c->per && i == nx)
        continue;
      else if (!u_solved(c, i, j))
        u[IU(c, i, j)] = 0.0;
    }
    u[IU(c, nx, j)] = c->per ? u[IU(c, 0, j)] : u[IU(c, nx - 1, j)];
  }
  for (int j = 0; j <= ny; j++)
    for (int i = 0; i < nx; i++)
      if (!v_solved(c, i, j)) v[IV(c, i, j)] = 0.0;
}

/* ------------------------------------------------------------------ */
/* context                                                            */
/* ------------------------------------------------------------------ */
static double *dalloc(size_t n) { return (double *)calloc(n, sizeof(double)); }

ora_ctx *ora_create(const ora_setup *s) {
  if (!s || s->nx < 4 || s->ny < 4) return NULL;
  ora_ctx *c = (ora_ctx *)calloc(1, sizeof(ora_ctx));
  int nx = s->nx, ny = s->ny;
  c->nx = nx;
  c->ny = ny;
  c->per = s->periodic ? 1 : 0;
  c->dx = dalloc(nx);
  c->dy = dalloc(ny);
  memcpy(c->dx, s->dx, sizeof(double) * nx);
  memcpy(c->dy, s->dy, sizeof(double) * ny);
  c->solid = (unsigned char *)calloc((size_t)nx * ny, 1);
  for (int k = 0; k < s->n_obst; k++)
    for (int j = s->oj0[k]; j <= s->oj1[k]; j++)
      for (int i = s->oi0[k]; i <= s->oi1[k]; i++)
        if (i >= 0 && i < nx && j >= 0 && j < ny) c->solid[IC(c, i, j)] = 1;
  double prm[5];
  ora_params(s->Ma, s->Re, s->Pr, s->gamma, prm);
  c->A = prm[0];
  c->B = prm[1];
  c->C1 = prm[2];
  c->C2 = prm[3];
  c->C3 = prm[4];
  c->gx = s->gx;
  c->gy = s->gy;
  c->u_in = dalloc(ny);
  c->T_in = dalloc(ny);
  for (int j = 0; j < ny; j++) {
    c->u_in[j] = s->u_in ? s->u_in[j] : 1.0;
    c->T_in[j] = s->T_in ? s->T_in[j] : 1.0;
  }
  c->p_in = s->p_in;
  for (int w = 0; w < 2; w++) {
    c->wtype[w] = s->wall_type[w];
    c->wu[w] = s->wall_u[w];
    c->wT[w] = dalloc(nx);
    for (int i = 0; i < nx; i++)
      c->wT[w][i] = s->wall_T[w] ? s->wall_T[w][i] : 1.0;
  }
  c->obsT = s->obstacle_T;
  c->otype = s->obstacle_type;
  c->kz = 1.1466 * s->kn;
  c->kt = 2.1904 * s->kn;
  size_t nu = (size_t)(nx + 1) * ny, nv = (size_t)nx * (ny + 1),
         nc = (size_t)nx * ny;
  c->u = dalloc(nu);
  c->un = dalloc(nu);
  c->um = dalloc(nu);
  c->v = dalloc(nv);
  c->vn = dalloc(nv);
  c->vm = dalloc(nv);
  c->p = dalloc(nc);
  c->pn = dalloc(nc);
  c->pm = dalloc(nc);
  c->Ts = dalloc(nc);
  c->ps = dalloc(nc);
  c->T = dalloc(nc);
  c->Tn = dalloc(nc);
  c->Tm = dalloc(nc);
  c->rho = dalloc(nc);
  c->gam = dalloc(nc);
  c->rhou = dalloc(nu);
  c->Fx = dalloc(nu);
  c->rhov = dalloc(nv);
  c->Fy = dalloc(nv);
  c->uh = dalloc(nu);
  c->du = dalloc(nu);
  c->vh = dalloc(nv);
  c->dv = dalloc(nv);
  c->uexp = dalloc(nu);
  c->vexp = dalloc(nv);
  c->Texp = dalloc(nc);
  /* initial state: the inlet state of each row, v = 0 */
  for (int j = 0; j < ny; j++) {
    for (int i = 0; i <= nx; i++) c->u[IU(c, i, j)] = c->u_in[j];
    for (int i = 0; i < nx; i++) {
      c->p[IC(c, i, j)] = c->p_in;
      c->T[IC(c, i, j)] = c->T_in[j];
    }
  }
  impose_bc(c, c->u, c->v, c->p, c->T);
  return c;
}

void ora_destroy(ora_ctx *c) {
  if (!c) return;
  double *bufs[] = {c->dx,  c->dy,   c->u_in, c->T_in, c->wT[0], c->wT[1],
                    c->u,   c->un,   c->um,   c->v,    c->vn,    c->vm,
                    c->p,   c->pn,   c->pm,   c->T,    c->Tn,    c->Tm,
                    c->rho, c->gam,  c->rhou, c->Fx,   c->rhov,  c->Fy,
                    c->uh,  c->du,   c->vh,   c->dv,   c->uexp,  c->vexp,
                    c->Texp, c->Ts,  c->ps};
  for (size_t k = 0; k < sizeof(bufs) / sizeof(bufs[0]); k++) free(bufs[k]);
  free(c->solid);
  free(c);
}

void ora_set_fields(ora_ctx *c, const double *u, const double *v,
                    const double *p, const double *T) {
  size_t nu = (size_t)(c->nx + 1) * c->ny, nv = (size_t)c->nx * (c->ny + 1),
         nc = (size_t)c->nx * c->ny;
  if (u) memcpy(c->u, u, nu * sizeof(double));
  if (v) memcpy(c->v, v, nv * sizeof(double));
  if (p) memcpy(c->p, p, nc * sizeof(double));
  if (T) memcpy(c->T, T, nc * sizeof(double));
  impose_bc(c, c->u, c->v, c->p, c->T);
}

void ora_get_fields(const ora_ctx *c, double *u, double *v, double *p,
                    double *T) {
  size_t nu = (size_t)(c->nx + 1) * c->ny, nv = (size_t)c->nx * (c->ny + 1),
         nc = (size_t)c->nx * c->ny;
  if (u) memcpy(u, c->u, nu * sizeof(double));
  if (v) memcpy(v, c->v, nv * sizeof(double));
  if (p) memcpy(p, c->p, nc * sizeof(double));
  if (T) memcpy(T, c->T, nc * sizeof(double));
}

void ora_residuals(const ora_ctx *c, double out[6]) {
  memcpy(out, c->res, sizeof(c->res));
}

void ora_mass(const ora_ctx *c, double out[3]) {
  double M = 0.0;
  for (int j = 0; j < c->ny; j++)
    for (int i = 0; i < c->nx; i++)
      if (!c->solid[IC(c, i, j)])
        M += c->p[IC(c, i, j)] / c->T[IC(c, i, j)] * c->dx[i] * c->dy[j];
  out[0] = M;
  out[1] = c->last_fin;
  out[2] = c->last_fout;
}

/* ------------------------------------------------------------------ */
/* step prologue (set the initial condition of the step; explicit terms)*/
/* ------------------------------------------------------------------ */
static void prologue(ora_ctx *c, int scheme) {
  size_t nu = (size_t)(c->nx + 1) * c->ny, nv = (size_t)c->nx * (c->ny + 1),
         nc = (size_t)c->nx * c->ny;
  memcpy(c->um, c->u, nu * sizeof(double));
  memcpy(c->vm, c->v, nv * sizeof(double));
  memcpy(c->pm, c->p, nc * sizeof(double));
  memcpy(c->Tm, c->T, nc * sizeof(double));
  memset(c->uexp, 0, nu * sizeof(double));
  memset(c->vexp, 0, nv * sizeof(double));
  memset(c->Texp, 0, nc * sizeof(double));
  if (scheme & ORA_IMPLICIT) return;
  const int tvd = scheme & ORA_TVD;
  /* F^x, F^y and the face densities from the n-1 fields (Sec. 3.2 after
     pl15_12) */
  cell_props(c, c->pm, c->Tm);
  face_fluxes(c, c->um, c->vm, tvd);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < c->ny; j++) {
    for (int i = 0; i < c->nx; i++)
      if (!c->solid[IC(c, i, j)]) c->Texp[IC(c, i, j)] = T_explicit(c, i, j, tvd);
    for (int i = 0; i <= c->nx; i++)
      if (u_solved(c, i, j)) c->uexp[IU(c, i, j)] = u_explicit(c, i, j, tvd);
  }
#pragma omp parallel for schedule(static)
  for (int j = 0; j <= c->ny; j++)
    for (int i = 0; i < c->nx; i++)
      if (v_solved(c, i, j)) c->vexp[IV(c, i, j)] = v_explicit(c, i, j, tvd);
}

/* ------------------------------------------------------------------ */
/* one pass of loop 2 (Appendix A order)                              */
/* ------------------------------------------------------------------ */
/* Energy equation (pl30) of one pass, Jacobi: T and p (neighbour values,
   the cell's own T where a boundary takes it, the pressure work) from the
   arrays c->T, c->p; rho, Gamma and the face fluxes from the pass's
   iterate (cell_props, face_fluxes).  Writes Tout. */
static void T_solve(ora_ctx *c, double dt, int scheme, double *Tout) {
  const int nx = c->nx, ny = c->ny;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      size_t k = IC(c, i, j);
      if (c->solid[k]) {
        Tout[k] = c->T[k];
        continue;
      }
      tco q = T_coefs(c, i, j, dt, scheme);
      Tout[k] = (dt * (q.a[0] * q.nb[0] + q.a[1] * q.nb[1] +
                       q.a[2] * q.nb[2] + q.a[3] * q.nb[3] + q.src) +
                 (q.unst + dt * q.texp)) /
                q.a0;
    }
}

/* Pressure equation (pl23, pl24) of one pass: the cell's T from Tcell,
   neighbour (and the cell's own) p from pold; face densities, u-hat, v-hat,
   d of the pass.  Writes pout. */
static void p_solve(ora_ctx *c, double dt, const double *pold, const double *Tcell,
                    double *pout) {
  const int nx = c->nx, ny = c->ny;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      size_t k = IC(c, i, j);
      if (c->solid[k]) {
        pout[k] = pold[k];
        continue;
      }
      double dxi = c->dx[i], dyj = c->dy[j], dV = dxi * dyj;
      size_t kw = IU(c, i, j), ke = IU(c, i + 1, j), ks = IV(c, i, j),
             kn = IV(c, i, j + 1);
      double aW = c->rhou[kw] * c->du[kw] * dyj;
      double aE = c->rhou[ke] * c->du[ke] * dyj;
      double aS = c->rhov[ks] * c->dv[ks] * dxi;
      double aN = c->rhov[kn] * c->dv[kn] * dxi;
      double bW = c->rhou[kw] * c->uh[kw] * dyj;
      double bE = c->rhou[ke] * c->uh[ke] * dyj;
      double bS = c->rhov[ks] * c->vh[ks] * dxi;
      double bN = c->rhov[kn] * c->vh[kn] * dxi;
      double pP = pold[k];
      double pW = (!c->per && i == 0) ? pP : Cat(c, pold, i - 1, j);
      double pE = (!c->per && i == nx - 1) ? pP : Cat(c, pold, i + 1, j);
      double pS = (j == 0) ? pP : pold[IC(c, i, j - 1)];
      double pN = (j == ny - 1) ? pP : pold[IC(c, i, j + 1)];
      double a0 = dV / Tcell[k] + (aW + aE + aS + aN) * dt;
      double bp = c->pm[k] / c->Tm[k] * dV - (bE - bW + bN - bS) * dt;
      pout[k] = ((aW * pW + aE * pE + aS * pS + aN * pN) * dt + bp) / a0;
    }

}

static void pass(ora_ctx *c, double dt, int scheme, int n3) {
  const int nx = c->nx, ny = c->ny, tvd = scheme & ORA_TVD;
  /* 1. rho = p/T, Gamma = sqrt(T) (pl5, pl37), face densities and fluxes */
  cell_props(c, c->p, c->T);
  face_fluxes(c, c->u, c->v, tvd);


  /* 3. pseudo velocities and d (pl18-pl21).  Faces that are not unknowns
     keep their fixed value as u-hat and get d = 0. */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; j++)
    for (int i = 0; i <= nx; i++) {
      size_t k = IU(c, i, j);
      if (u_solved(c, i, j)) {
        mco q = u_coefs(c, i, j, dt, scheme);
        c->uh[k] = (nbsum_u(&q) + q.b) / q.a0;
        c->du[k] = c->A * q.len / q.a0;
      } else {
        c->uh[k] = c->u[k];
        c->du[k] = 0.0;
      }
    }
  if (c->per)
    for (int j = 0; j < ny; j++) {
      c->uh[IU(c, nx, j)] = c->uh[IU(c, 0, j)];
      c->du[IU(c, nx, j)] = c->du[IU(c, 0, j)];
    }
#pragma omp parallel for schedule(static)
  for (int j = 0; j <= ny; j++)
    for (int i = 0; i < nx; i++) {
      size_t k = IV(c, i, j);
      if (v_solved(c, i, j)) {
        mco q = v_coefs(c, i, j, dt, scheme);
        c->vh[k] = (nbsum_v(&q) + q.b) / q.a0;
        c->dv[k] = c->A * q.len / q.a0;
      } else {
        c->vh[k] = c->v[k];
        c->dv[k] = 0.0;
      }
    }

  /* 2.-4. temperature (pl30) and pressure (pl23, pl24), Jacobi in their
     neighbours.  Loop 3 of the CPU algorithm (Sec. 3, its figure): with
     the face densities, fluxes, rho, Gamma, u-hat, v-hat and d of this
     pass fixed, the energy and pressure equations are solved n3 times,
     each time with T and p from the previous solve (n3 = 1: the pass of
     the GPU algorithm, T and p at the old iterate). */
  T_solve(c, dt, scheme, c->Tn);
  p_solve(c, dt, c->p, c->Tn, c->pn);
  if (n3 > 1) {
    double *Told = c->T, *pold = c->p;
    for (int s = 2; s <= n3; s++) {
      /* the previous sub-iterate takes the place of the old T and p */
      memcpy(c->Ts, c->Tn, sizeof(double) * (size_t)nx * ny);
      memcpy(c->ps, c->pn, sizeof(double) * (size_t)nx * ny);
      c->T = c->Ts;
      c->p = c->ps;
      T_solve(c, dt, scheme, c->Tn);
      p_solve(c, dt, c->ps, c->Tn, c->pn);
    }
    c->T = Told;
    c->p = pold;
  }

  /* 5. velocities (pl18, pl19) with this pass's pressure on both sides */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; j++) {
    for (int i = 0; i <= nx; i++) {
      size_t k = IU(c, i, j);
      if (u_solved(c, i, j))
        c->un[k] = c->uh[k] - c->du[k] * (Cat(c, c->pn, i, j) -
                                           Cat(c, c->pn, i - 1, j));
      else
        c->un[k] = c->u[k];
    }
    c->un[IU(c, nx, j)] = c->per ? c->un[IU(c, 0, j)] : c->un[IU(c, nx - 1, j)];
  }
#pragma omp parallel for schedule(static)
  for (int j = 0; j <= ny; j++)
    for (int i = 0; i < nx; i++) {
      size_t k = IV(c, i, j);
      if (v_solved(c, i, j))
        c->vn[k] = c->vh[k] - c->dv[k] * (c->pn[IC(c, i, j)] -
                                           c->pn[IC(c, i, j - 1)]);
      else
        c->vn[k] = c->v[k];
    }

  /* 6. residuals: max increments of the unknowns and the continuity
     residual R = ((p/T)_new - (p/T)^{n-1}) dV/dt + net outflow of
     rho^u u_new dy and rho^v v_new dx */
  double ru = 0, rv = 0, rp = 0, rT = 0, rm = 0, sm = 0, fin = 0, fout = 0;
  for (int j = 0; j < ny; j++) {
    double dyj = c->dy[j];
    for (int i = 0; i <= nx; i++)
      if (u_solved(c, i, j)) {
        size_t k = IU(c, i, j);
        ru = dmax(ru, fabs(c->un[k] - c->u[k]));
      }
    for (int i = 0; i < nx; i++) {
      size_t k = IC(c, i, j);
      if (c->solid[k]) continue;
      double dxi = c->dx[i], dV = dxi * dyj;
      rp = dmax(rp, fabs(c->pn[k] - c->p[k]));
      rT = dmax(rT, fabs(c->Tn[k] - c->T[k]));
      size_t kw = IU(c, i, j), ke = IU(c, i + 1, j), ks = IV(c, i, j),
             kn = IV(c, i, j + 1);
      double GW = c->rhou[kw] * c->un[kw] * dyj;
      double GE = c->rhou[ke] * c->un[ke] * dyj;
      double GS = c->rhov[ks] * c->vn[ks] * dxi;
      double GN = c->rhov[kn] * c->vn[kn] * dxi;
      double R = (c->pn[k] / c->Tn[k] * dV - c->pm[k] / c->Tm[k] * dV) / dt +
                 (GE - GW) + (GN - GS);
      rm = dmax(rm, fabs(R));
      sm += R;
      if (!c->per && i == 0) fin += GW;
      if (!c->per && i == nx - 1) fout += GE;
    }
  }
  for (int j = 0; j <= ny; j++)
    for (int i = 0; i < nx; i++)
      if (v_solved(c, i, j)) {
        size_t k = IV(c, i, j);
        rv = dmax(rv, fabs(c->vn[k] - c->v[k]));
      }
  c->res[0] = ru;
  c->res[1] = rv;
  c->res[2] = rp;
  c->res[3] = rT;
  c->res[4] = rm;
  c->res[5] = sm;
  c->last_fin = fin;
  c->last_fout = fout;

  /* 7. the new iterate becomes the old one */
  double *t;
  t = c->u; c->u = c->un; c->un = t;
  t = c->v; c->v = c->vn; c->vn = t;
  t = c->p; c->p = c->pn; c->pn = t;
  t = c->T; c->T = c->Tn; c->Tn = t;
}

void ora_step(ora_ctx *c, double dt, int n_inner, int scheme) {
  prologue(c, scheme);
  for (int k = 0; k < n_inner; k++) pass(c, dt, scheme, 1);
}

/* A step whose passes each run loop 3 with n3 >= 1 energy-pressure solves
   (n3 = 1: ora_step). */
void ora_step_l3(ora_ctx *c, double dt, int n_inner, int n3, int scheme) {
  prologue(c, scheme);
  for (int k = 0; k < n_inner; k++) pass(c, dt, scheme, n3);
}

/* Loop 2 with its convergence test (Sec. 3.1, the algorithm figures: the
   inner iterations repeat until the solution of the step has converged; the
   paper reads the maximal residuals back after every iteration, Sec. 5).
   The test: max(max|du|, max|dv|, max|dT|, max|dp| / p_in) <= tol over the
   unknowns, after each pass; at most max_inner passes.  Returns the number
   of passes taken. */
int ora_step_tol(ora_ctx *c, double dt, int max_inner, double tol, int scheme) {
  return ora_step_tol_l3(c, dt, max_inner, 1, tol, scheme);
}

/* The same with loop 3 in every pass (n3 energy-pressure solves). */
int ora_step_tol_l3(ora_ctx *c, double dt, int max_inner, int n3, double tol, int scheme) {
  prologue(c, scheme);
  int k = 0;
  while (k < max_inner) {
    pass(c, dt, scheme, n3);
    k++;
    double r = dmax(dmax(c->res[0], c->res[1]), dmax(c->res[3], c->res[2] / c->p_in));
    if (r <= tol) break;
  }
  return k;
}

void ora_eq_residuals(ora_ctx *c, double dt, int scheme, double *rT,
                      double *ru, double *rv, double *rp) {
  const int nx = c->nx, ny = c->ny;
  prologue(c, scheme);
  cell_props(c, c->p, c->T);
  face_fluxes(c, c->u, c->v, scheme & ORA_TVD);
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      size_t k = IC(c, i, j);
      rT[k] = 0.0;
      if (c->solid[k]) continue;
      tco q = T_coefs(c, i, j, dt, scheme);
      rT[k] = q.a0 * c->T[k] -
              (dt * (q.a[0] * q.nb[0] + q.a[1] * q.nb[1] + q.a[2] * q.nb[2] +
                     q.a[3] * q.nb[3] + q.src) +
               (q.unst + dt * q.texp));
    }
  for (int j = 0; j < ny; j++)
    for (int i = 0; i <= nx; i++) {
      size_t k = IU(c, i, j);
      ru[k] = 0.0;
      c->uh[k] = c->u[k];
      c->du[k] = 0.0;
      if (!u_solved(c, i, j)) continue;
      mco q = u_coefs(c, i, j, dt, scheme);
      ru[k] = q.a0 * c->u[k] - (nbsum_u(&q) + q.b) +
              c->A * q.len * (Cat(c, c->p, i, j) - Cat(c, c->p, i - 1, j));
      c->uh[k] = (nbsum_u(&q) + q.b) / q.a0;
      c->du[k] = c->A * q.len / q.a0;
    }
  if (c->per)
    for (int j = 0; j < ny; j++) {
      c->uh[IU(c, nx, j)] = c->uh[IU(c, 0, j)];
      c->du[IU(c, nx, j)] = c->du[IU(c, 0, j)];
    }
  for (int j = 0; j <= ny; j++)
    for (int i = 0; i < nx; i++) {
      size_t k = IV(c, i, j);
      rv[k] = 0.0;
      c->vh[k] = c->v[k];
      c->dv[k] = 0.0;
      if (!v_solved(c, i, j)) continue;
      mco q = v_coefs(c, i, j, dt, scheme);
      rv[k] = q.a0 * c->v[k] - (nbsum_v(&q) + q.b) +
              c->A * q.len * (c->p[IC(c, i, j)] - c->p[IC(c, i, j - 1)]);
      c->vh[k] = (nbsum_v(&q) + q.b) / q.a0;
      c->dv[k] = c->A * q.len / q.a0;
    }
  /* pressure equation with T_new = T (frozen state) */
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      size_t k = IC(c, i, j);
      rp[k] = 0.0;
      if (c->solid[k]) continue;
      double dxi = c->dx[i], dyj = c->dy[j], dV = dxi * dyj;
      size_t kw = IU(c, i, j), ke = IU(c, i + 1, j), ks = IV(c, i, j),
             kn = IV(c, i, j + 1);
      double aW = c->rhou[kw] * c->du[kw] * dyj;
      double aE = c->rhou[ke] * c->du[ke] * dyj;
      double aS = c->rhov[ks] * c->dv[ks] * dxi;
      double aN = c->rhov[kn] * c->dv[kn] * dxi;
      double bW = c->rhou[kw] * c->uh[kw] * dyj;
      double bE = c->rhou[ke] * c->uh[ke] * dyj;
      double bS = c->rhov[ks] * c->vh[ks] * dxi;
      double bN = c->rhov[kn] * c->vh[kn] * dxi;
      double pP = c->p[k];
      double pW = (!c->per && i == 0) ? pP : Cat(c, c->p, i - 1, j);
      double pE = (!c->per && i == nx - 1) ? pP : Cat(c, c->p, i + 1, j);
      double pS = (j == 0) ? pP : c->p[IC(c, i, j - 1)];
      double pN = (j == ny - 1) ? pP : c->p[IC(c, i, j + 1)];
      double a0 = dV / c->T[k] + (aW + aE + aS + aN) * dt;
      double bp = c->pm[k] / c->Tm[k] * dV - (bE - bW + bN - bS) * dt;
      rp[k] = a0 * pP - ((aW * pW + aE * pE + aS * pS + aN * pN) * dt + bp);
    }
}
