/*
 * ora3.c -- TEST INFRASTRUCTURE ONLY: plain FP64 CPU oracle of the SIMPLE-TS
 * time step in three dimensions.  Used by tests; never by the product.
 * Shares no code with the HIP library (nor with the 2-D oracle).
 *
 * The paper (Shterev, arXiv 1802.04243) states the method in 2-D (Sec. 2,
 * eqs pl4-pl7; Sec. 3.2, eqs pl8-pl33) and names 3-D flow as the next step
 * (Conclusions).  This file writes the same discretisation with a third
 * direction, reading every 2-D formula per pair of directions:
 *   - velocity component a on the a-faces, p and T at cell centres
 *     (the cell-volume figure of Sec. 3.2 with a z extent);
 *   - face densities and mass fluxes (pl8-pl11) on the faces of every
 *     direction, fluxes through face areas (products of the two other
 *     widths);
 *   - momentum of component a (pl14-pl16, pl15, pl15_11, pl18-pl21, the
 *     printed v-equation read for any a): the 4/3 factor on the
 *     conductances normal to a, tangential conductances with Gamma
 *     bilinear on the edges, the cross-diffusion of eqs pl2/pl3 written
 *     for every tangential direction b: Gamma_edge (q_b(r) - q_b(l)) over
 *     the two b-sides, minus 2/3 Gamma (q_b(b+) - q_b(b-)) of the two
 *     cells, each times the width of the third direction;
 *   - energy (pl28-pl33, pl31_1): conduction through six faces with
 *     harmonic means, dissipation Phi = 2 sum (d_e q_e)^2 +
 *     sum_{e<f} (d_f q_e + d_e q_f)^2 - 2/3 (div u)^2 with face-centre
 *     velocities bilinear in the nearest nodes, pressure work;
 *   - pressure (pl23, pl24) with six neighbours; velocities (pl18, pl19).
 * Boundary rules and readings are the 2-D oracle's: no-slip isothermal
 * walls with half-cell conductances (the mean of the node's and the wall's
 * Gamma for shear, their harmonic mean for conduction), slip-adiabatic walls,
 * a supersonic inlet in x (u = u_in, T = T_in, tangential velocities 0 on
 * the face, inflow density p_in/T_in), a zero-gradient outlet (the last
 * u-face copied), TVD stencils switched off where a point is missing, van
 * Leer psi(r) = (r+|r|)/(1+|r|) of r = a/b, face density = upwind value +
 * psi times the jump.  One pass in the order of Appendix A.
 *
 * Plain loops, no blocking, no fusion; OpenMP splits the z loop.  Build
 * with -ffp-contract=off.
 */
#include "ora3.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

struct ora3_ctx {
  int n[3];
  double *d[3];
  int bc[3];
  int wt[3][2];
  double wv[3][2][3], wT[3][2];
  double A, B, C1, C2, C3, g[3];
  double u_in, T_in, p_in;
  int dim[5][3];
  size_t len[5];
  double *q[5], *qn[5], *qm[5];  /* old iterate, new iterate, level n-1 */
  double *rho, *gam;             /* cells */
  double *rf[3], *F[3];          /* face densities, mass fluxes (face layouts) */
  double *qh[3], *dq[3];         /* pseudo velocities and d */
  double *qx[3], *Tx;            /* explicit convective terms */
  double res[7];
};

/* ------------------------------------------------------------------ */
/* indexing                                                           */
/* ------------------------------------------------------------------ */
static int per(const ora3_ctx *c, int e) { return c->bc[e] == ORA3_PERIODIC; }
/* an index along e, wrapped when e is periodic */
static int wr(const ora3_ctx *c, int e, int i) {
  if (per(c, e)) {
    i %= c->n[e];
    if (i < 0) i += c->n[e];
  }
  return i;
}
static size_t lin(const ora3_ctx *c, int f, const int x[3]) {
  int i = wr(c, 0, x[0]), j = wr(c, 1, x[1]), k = wr(c, 2, x[2]);
  return ((size_t)k * c->dim[f][1] + j) * c->dim[f][0] + i;
}
/* storage slot of an in-range index (no wrap: the last face of a periodic
   direction has a slot of its own, a copy of face 0) */
static size_t slot(const ora3_ctx *c, int f, const int x[3]) {
  return ((size_t)x[2] * c->dim[f][1] + x[1]) * c->dim[f][0] + x[0];
}
static double at(const ora3_ctx *c, const double *a, int f, const int x[3]) {
  return a[lin(c, f, x)];
}
static double W(const ora3_ctx *c, int e, int i) { return c->d[e][wr(c, e, i)]; }
/* cell index x along e exists */
static int has_cell(const ora3_ctx *c, int e, int i) {
  return per(c, e) || (i >= 0 && i < c->n[e]);
}
/* a-face index i along a exists in the array (0..n) */
static int has_face(const ora3_ctx *c, int a, int i) {
  return per(c, a) || (i >= 0 && i <= c->n[a]);
}
/* the face f of component a is an unknown (not on a wall, the inlet or the
   outlet; the last face of a periodic direction copies face 0) */
static int solved(const ora3_ctx *c, int a, const int f[3]) {
  if (per(c, a)) return f[a] < c->n[a];
  return f[a] > 0 && f[a] < c->n[a];
}
static void shift(int y[3], const int x[3], int e, int s) {
  y[0] = x[0];
  y[1] = x[1];
  y[2] = x[2];
  y[e] += s;
}
static double area(const ora3_ctx *c, int e, const int x[3]) {
  int b = (e + 1) % 3, t = (e + 2) % 3;
  return W(c, b, x[b]) * W(c, t, x[t]);
}
static double vol(const ora3_ctx *c, const int x[3]) {
  return W(c, 0, x[0]) * W(c, 1, x[1]) * W(c, 2, x[2]);
}

/* ------------------------------------------------------------------ */
/* elementary functions (Sec. 3.2)                                    */
/* ------------------------------------------------------------------ */
static double dmax(double a, double b) { return a > b ? a : b; }
static double upwind(double f1, double f2, double vel) { return vel > 0 ? f1 : f2; }
static double vanleer(double a, double b) {
  if (!((a > 0 && b > 0) || (a < 0 && b < 0))) return 0.0;
  double r = a / b;
  if (isinf(r)) return 2.0;
  return (r + fabs(r)) / (1.0 + fabs(r));
}
static double psi_s(double f1, double f2, double f3, double f4, double d1, double d2,
                    double d3, double d4, double vel) {
  if (vel > 0)
    return d2 / (d2 + d3) * vanleer((d2 + d3) * (f2 - f1), (d1 + d2) * (f3 - f2));
  return -d3 / (d2 + d3) * vanleer((d2 + d3) * (f4 - f3), (d3 + d4) * (f3 - f2));
}
static double psi_c(double f1, double f2, double f3, double f4, double d1, double d2,
                    double d3, double vel) {
  if (vel > 0) return 0.5 * vanleer(d2 * (f2 - f1), d1 * (f3 - f2));
  return -0.5 * vanleer(d2 * (f4 - f3), d3 * (f3 - f2));
}
static double hmean(double dl, double gl, double dr, double gr) {
  return (dl + dr) * gl * gr / (dl * gr + dr * gl);
}
static double hmean2(double a, double b) { return 2.0 * a * b / (a + b); }

/* ------------------------------------------------------------------ */
/* rho, Gamma, face densities and mass fluxes (pl8-pl11)              */
/* ------------------------------------------------------------------ */
static void cell_props(ora3_ctx *c, const double *p, const double *T) {
#pragma omp parallel for schedule(static)
  for (long m = 0; m < (long)c->len[3]; m++) {
    c->rho[m] = p[m] / T[m];
    c->gam[m] = sqrt(T[m]);
  }
}

static void face_fluxes(ora3_ctx *c, double *const *q, int tvd) {
  for (int a = 0; a < 3; a++) {
    const int *D = c->dim[a];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < D[2]; k++)
      for (int j = 0; j < D[1]; j++)
        for (int i = 0; i < D[0]; i++) {
          int f[3] = {i, j, k}, l[3], r[3];
          shift(l, f, a, -1);
          shift(r, f, a, 0);
          const double vel = at(c, q[a], a, f);
          double rf;
          if (!per(c, a) && f[a] == 0) {
            rf = (a == 0 && c->bc[0] == ORA3_INLET_OUTLET)
                     ? upwind(c->p_in / c->T_in, at(c, c->rho, 3, r), vel)
                     : at(c, c->rho, 3, r);
          } else if (!per(c, a) && f[a] == c->n[a]) {
            rf = at(c, c->rho, 3, l);
          } else {
            const double rl = at(c, c->rho, 3, l), rr = at(c, c->rho, 3, r);
            rf = upwind(rl, rr, vel);
            if (tvd && has_cell(c, a, f[a] - 2) && has_cell(c, a, f[a] + 1)) {
              int l2[3], r2[3];
              shift(l2, f, a, -2);
              shift(r2, f, a, 1);
              rf += psi_s(at(c, c->rho, 3, l2), rl, rr, at(c, c->rho, 3, r2),
                          W(c, a, f[a] - 2), W(c, a, f[a] - 1), W(c, a, f[a]),
                          W(c, a, f[a] + 1), vel) *
                    (rr - rl);
            }
          }
          const size_t m = slot(c, a, f);
          c->rf[a][m] = rf;
          c->F[a][m] = rf * vel * area(c, a, f);
        }
  }
}

/* ------------------------------------------------------------------ */
/* boundary lookups                                                   */
/* ------------------------------------------------------------------ */
/* the side s (0 low, 1 high) of cell x along e lies on the domain boundary:
   0 interior, 1 wall, 2 inlet, 3 outlet */
static int side_kind(const ora3_ctx *c, int e, const int x[3], int s) {
  if (per(c, e)) return 0;
  if (s == 0 && x[e] == 0) return c->bc[e] == ORA3_INLET_OUTLET ? 2 : 1;
  if (s == 1 && x[e] == c->n[e] - 1) return c->bc[e] == ORA3_INLET_OUTLET ? 3 : 1;
  return 0;
}

/* Gamma on the edge of the momentum volume of component a at face f: the
   edge runs along the third direction, at the a-face position of f and at
   the b-face between the cells f[b] - 1 + s and f[b] + s; bilinear in the
   four cells around it.  On a wall it only multiplies wall-normal
   velocities, which are zero: 0.  At the inlet it is sqrt(T_in), at the
   outlet the last cells interpolated along a. */
static double gam_edge(const ora3_ctx *c, int a, int b, const int f[3], int s) {
  const int bf = f[b] + s; /* b-face index of the edge */
  if (!per(c, b) && (bf == 0 || bf == c->n[b])) {
    if (b == 0 && c->bc[0] == ORA3_INLET_OUTLET) {
      if (bf == 0) return sqrt(c->T_in);
      int l[3], r[3];
      shift(l, f, a, -1);
      shift(r, f, a, 0);
      l[b] = r[b] = c->n[b] - 1;
      const double dl = W(c, a, l[a]), dr = W(c, a, r[a]);
      return (dr * at(c, c->gam, 3, l) + dl * at(c, c->gam, 3, r)) / (dl + dr);
    }
    return 0.0;
  }
  const double dal = W(c, a, f[a] - 1), dar = W(c, a, f[a]);
  const double dbl = W(c, b, bf - 1), dbr = W(c, b, bf);
  double g = 0.0;
  for (int ia = 0; ia < 2; ia++)
    for (int ib = 0; ib < 2; ib++) {
      int x[3] = {f[0], f[1], f[2]};
      x[a] = f[a] - 1 + ia;
      x[b] = bf - 1 + ib;
      const double wa = ia ? dal / (dal + dar) : dar / (dal + dar);
      const double wb = ib ? dbl / (dbl + dbr) : dbr / (dbl + dbr);
      g += wa * wb * at(c, c->gam, 3, x);
    }
  return g;
}

/* cell-centre value of component e in cell x */
static double qcell(const ora3_ctx *c, double *const *q, int e, const int x[3]) {
  int h[3];
  shift(h, x, e, 1);
  return 0.5 * (at(c, q[e], e, x) + at(c, q[e], e, h));
}
/* component e at the centre of the f-face on side s of cell x (bilinear in
   the nearest nodes; wall, inlet and outlet values at the boundary) */
static double qface(const ora3_ctx *c, double *const *q, int e, int f, const int x[3], int s) {
  const double qc = qcell(c, q, e, x);
  const int kind = side_kind(c, f, x, s);
  if (kind == 1) return c->wt[f][s] == ORA3_NOSLIP ? c->wv[f][s][e] : qc;
  if (kind == 2) return 0.0; /* tangential inlet velocity */
  if (kind == 3) return qc;
  int y[3];
  shift(y, x, f, s ? 1 : -1);
  const double dx = W(c, f, x[f]), dy = W(c, f, y[f]);
  return (dy * qc + dx * qcell(c, q, e, y)) / (dx + dy);
}

/* ------------------------------------------------------------------ */
/* explicit convective terms from the n-1 fields (pl15_11, pl31_1)    */
/* ------------------------------------------------------------------ */
static double T_explicit(const ora3_ctx *c, const int x[3], int tvd) {
  const double *T = c->qm[4];
  const double TP = at(c, T, 3, x);
  double sum = 0.0;
  for (int e = 0; e < 3; e++) {
    int fl[3], fh[3];
    shift(fl, x, e, 0);
    shift(fh, x, e, 1);
    const int kl = side_kind(c, e, x, 0), kh = side_kind(c, e, x, 1);
    const double Fl = at(c, c->F[e], e, fl), Fh = at(c, c->F[e], e, fh);
    const double vl = at(c, c->qm[e], e, fl), vh = at(c, c->qm[e], e, fh);
    int y[3];
    shift(y, x, e, -1);
    const double TL = kl == 2 ? c->T_in : (kl == 1 ? TP : at(c, T, 3, y));
    shift(y, x, e, 1);
    const double TH = (kh == 3 || kh == 1) ? TP : at(c, T, 3, y);
    double pl = 0.0, ph = 0.0;
    if (tvd) {
      if (has_cell(c, e, x[e] - 1) && has_cell(c, e, x[e] + 2)) {
        int y1[3], y2[3];
        shift(y1, x, e, -1);
        shift(y2, x, e, 2);
        ph = psi_s(at(c, T, 3, y1), TP, TH, at(c, T, 3, y2), W(c, e, x[e] - 1),
                   W(c, e, x[e]), W(c, e, x[e] + 1), W(c, e, x[e] + 2), vh);
      }
      if (has_cell(c, e, x[e] - 2) && has_cell(c, e, x[e] + 1)) {
        int y1[3];
        shift(y1, x, e, -2);
        pl = psi_s(at(c, T, 3, y1), TL, TP, TH, W(c, e, x[e] - 2), W(c, e, x[e] - 1),
                   W(c, e, x[e]), W(c, e, x[e] + 1), vl);
      }
    }
    sum += -Fh * (upwind(TP, TH, vh) + (TH - TP) * ph) + Fl * (upwind(TL, TP, vl) + (TP - TL) * pl);
  }
  return sum;
}

/* neighbour of component a at face f along b (s = -1, +1) for the explicit
   and implicit convective terms and the diffusion: the node value, the
   inlet's tangential 0 or the outlet's zero gradient; wall values are the
   wall's velocity (no-slip) or the node itself (slip) */
static double q_nb(const ora3_ctx *c, double *const *q, int a, int b, const int f[3], int s,
                   int *wall) {
  *wall = 0;
  if (b == a) {
    int y[3];
    shift(y, f, a, s);
    return at(c, q[a], a, y);
  }
  int x[3] = {f[0], f[1], f[2]}; /* cell row along b of the face */
  const int kind = side_kind(c, b, x, s > 0);
  if (kind == 1) {
    *wall = 1;
    return c->wt[b][s > 0] == ORA3_NOSLIP ? c->wv[b][s > 0][a] : at(c, q[a], a, f);
  }
  if (kind == 2) return 0.0;
  if (kind == 3) return at(c, q[a], a, f);
  int y[3];
  shift(y, f, b, s);
  return at(c, q[a], a, y);
}

static double q_explicit(const ora3_ctx *c, int a, const int f[3], int tvd) {
  double *const *q = c->qm;
  const double qP = at(c, q[a], a, f);
  int l[3], r[3];
  shift(l, f, a, -1);
  shift(r, f, a, 0);
  double sum = 0.0;
  for (int b = 0; b < 3; b++) {
    int wall;
    const double qL = q_nb(c, q, a, b, f, -1, &wall);
    const double qH = q_nb(c, q, a, b, f, 1, &wall);
    if (b == a) {
      /* through the cell centres of l and r */
      const double ubH = 0.5 * (qP + qH), ubL = 0.5 * (qL + qP);
      const double FbH = at(c, c->rho, 3, r) * ubH * area(c, a, f);
      const double FbL = at(c, c->rho, 3, l) * ubL * area(c, a, f);
      double pH = 0.0, pL = 0.0;
      if (tvd) {
        if (has_face(c, a, f[a] - 1) && has_face(c, a, f[a] + 2)) {
          int y[3];
          shift(y, f, a, 2);
          pH = psi_c(qL, qP, qH, at(c, q[a], a, y), W(c, a, f[a] - 1), W(c, a, f[a]),
                     W(c, a, f[a] + 1), ubH);
        }
        if (has_face(c, a, f[a] - 2) && has_face(c, a, f[a] + 1)) {
          int y[3];
          shift(y, f, a, -2);
          pL = psi_c(at(c, q[a], a, y), qL, qP, qH, W(c, a, f[a] - 2), W(c, a, f[a] - 1),
                     W(c, a, f[a]), ubL);
        }
      }
      sum += -FbH * (upwind(qP, qH, ubH) + (qH - qP) * pH) + FbL * (upwind(qL, qP, ubL) + (qP - qL) * pL);
    } else {
      /* through the b-faces of the two cells l and r, half each */
      for (int side = 0; side < 2; side++) {
        const int *cx = side ? r : l;
        int bl[3], bh[3];
        shift(bl, cx, b, 0);
        shift(bh, cx, b, 1);
        const double Fl = at(c, c->F[b], b, bl), Fh = at(c, c->F[b], b, bh);
        const double vl = at(c, q[b], b, bl), vh = at(c, q[b], b, bh);
        double pl = 0.0, ph = 0.0;
        if (tvd) {
          if (has_cell(c, b, f[b] - 1) && has_cell(c, b, f[b] + 2)) {
            int y1[3], y2[3];
            shift(y1, f, b, -1);
            shift(y2, f, b, 2);
            ph = psi_s(at(c, q[a], a, y1), qP, qH, at(c, q[a], a, y2), W(c, b, f[b] - 1),
                       W(c, b, f[b]), W(c, b, f[b] + 1), W(c, b, f[b] + 2), vh);
          }
          if (has_cell(c, b, f[b] - 2) && has_cell(c, b, f[b] + 1)) {
            int y1[3], y2[3];
            shift(y1, f, b, -2);
            shift(y2, f, b, 1);
            pl = psi_s(at(c, q[a], a, y1), qL, qP, at(c, q[a], a, y2), W(c, b, f[b] - 2),
                       W(c, b, f[b] - 1), W(c, b, f[b]), W(c, b, f[b] + 1), vl);
          }
        }
        sum += 0.5 * (-Fh * (upwind(qP, qH, vh) + (qH - qP) * ph) +
                      Fl * (upwind(qL, qP, vl) + (qP - qL) * pl));
      }
    }
  }
  return sum;
}

/* ------------------------------------------------------------------ */
/* energy equation (pl30-pl33, pl28, pl29)                            */
/* ------------------------------------------------------------------ */
typedef struct {
  double a[6], nb[6], a0, src, unst, texp;
} tco3;

static tco3 T_coefs(const ora3_ctx *c, const int x[3], double dt, int scheme) {
  const int implicit = scheme & ORA3_IMPLICIT, tvd = scheme & ORA3_TVD;
  double *const *q = c->q;
  const double *T = c->q[4];
  tco3 o;
  const double TP = at(c, T, 3, x), gP = at(c, c->gam, 3, x), rP = at(c, c->rho, 3, x);
  const double dV = vol(c, x);
  double sumF = 0.0;
  for (int e = 0; e < 3; e++) {
    const double ar = area(c, e, x), de = W(c, e, x[e]);
    for (int s = 0; s < 2; s++) {
      const int kind = side_kind(c, e, x, s);
      double D, nb;
      if (kind == 1) {
        if (c->wt[e][s] == ORA3_NOSLIP) {
          nb = c->wT[e][s];
          D = c->C1 * hmean2(gP, sqrt(c->wT[e][s])) * ar / (0.5 * de);
        } else {
          nb = TP;
          D = 0.0;
        }
      } else if (kind == 2) {
        nb = c->T_in;
        D = c->C1 * hmean2(gP, sqrt(c->T_in)) * ar / (0.5 * de);
      } else if (kind == 3) {
        nb = TP;
        D = 0.0;
      } else {
        int y[3];
        shift(y, x, e, s ? 1 : -1);
        const double dn = W(c, e, y[e]);
        nb = at(c, T, 3, y);
        D = c->C1 * (s ? hmean(de, gP, dn, at(c, c->gam, 3, y)) : hmean(dn, at(c, c->gam, 3, y), de, gP)) *
            ar / (0.5 * (de + dn));
      }
      int fx[3];
      shift(fx, x, e, s);
      const double Fv = at(c, c->F[e], e, fx);
      double a = D;
      if (implicit) {
        double psi = 0.0;
        if (tvd) {
          const double vel = at(c, q[e], e, fx);
          if (s == 0 && has_cell(c, e, x[e] - 2) && has_cell(c, e, x[e] + 1)) {
            int y0[3], y1[3], y2[3];
            shift(y0, x, e, -2);
            shift(y1, x, e, -1);
            shift(y2, x, e, 1);
            psi = psi_s(at(c, T, 3, y0), at(c, T, 3, y1), TP, at(c, T, 3, y2), W(c, e, x[e] - 2),
                        W(c, e, x[e] - 1), de, W(c, e, x[e] + 1), vel);
          }
          if (s == 1 && has_cell(c, e, x[e] - 1) && has_cell(c, e, x[e] + 2)) {
            int y0[3], y1[3], y2[3];
            shift(y0, x, e, -1);
            shift(y1, x, e, 1);
            shift(y2, x, e, 2);
            psi = psi_s(at(c, T, 3, y0), TP, at(c, T, 3, y1), at(c, T, 3, y2), W(c, e, x[e] - 1), de,
                        W(c, e, x[e] + 1), W(c, e, x[e] + 2), vel);
          }
        }
        a = (s ? dmax(0.0, -Fv) : dmax(0.0, Fv)) - Fv * psi + D;
        sumF += s ? Fv : -Fv;
      }
      o.a[2 * e + s] = a;
      o.nb[2 * e + s] = nb;
    }
  }
  double suma = 0.0;
  for (int m = 0; m < 6; m++) suma += o.a[m];
  o.a0 = implicit ? dt * (suma + sumF) + rP * dV : dt * suma + rP * dV;
  /* source (pl29): dissipation and pressure work */
  double dd[3], div = 0.0;
  for (int e = 0; e < 3; e++) {
    int h[3];
    shift(h, x, e, 1);
    dd[e] = (at(c, q[e], e, h) - at(c, q[e], e, x)) / W(c, e, x[e]);
    div += dd[e];
  }
  double phi = 2.0 * (dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
  for (int e = 0; e < 3; e++)
    for (int f = e + 1; f < 3; f++) {
      const double def = (qface(c, q, e, f, x, 1) - qface(c, q, e, f, x, 0)) / W(c, f, x[f]);
      const double dfe = (qface(c, q, f, e, x, 1) - qface(c, q, f, e, x, 0)) / W(c, e, x[e]);
      phi += (def + dfe) * (def + dfe);
    }
  phi -= 2.0 / 3.0 * div * div;
  o.src = c->C2 * gP * phi * dV + c->C3 * at(c, c->q[3], 3, x) * div * dV;
  o.texp = implicit ? 0.0 : c->Tx[lin(c, 3, x)];
  o.unst = (at(c, c->qm[3], 3, x) / at(c, c->qm[4], 3, x)) * at(c, c->qm[4], 3, x) * dV;
  return o;
}

static double T_update(const tco3 *o, double dt) {
  double s = 0.0;
  for (int m = 0; m < 6; m++) s += o->a[m] * o->nb[m];
  return (dt * (s + o->src) + (o->unst + dt * o->texp)) / o->a0;
}

/* ------------------------------------------------------------------ */
/* momentum of component a (pl14-pl16, pl15, pl21 for any a)          */
/* ------------------------------------------------------------------ */
typedef struct {
  double a[6], nb[6], a0, b, area;
} mco3;

static mco3 q_coefs(const ora3_ctx *c, int a, const int f[3], double dt, int scheme) {
  const int implicit = scheme & ORA3_IMPLICIT, tvd = scheme & ORA3_TVD;
  double *const *q = c->q;
  mco3 o;
  int l[3], r[3];
  shift(l, f, a, -1);
  shift(r, f, a, 0);
  const double dal = W(c, a, l[a]), dar = W(c, a, r[a]);
  const double rl = at(c, c->rho, 3, l), rr = at(c, c->rho, 3, r);
  const double gl = at(c, c->gam, 3, l), gr = at(c, c->gam, 3, r);
  const double Ap = area(c, a, f), len = 0.5 * (dal + dar);
  const double qP = at(c, q[a], a, f);
  const double M = (rr * dar + rl * dal) * Ap / 2.0;
  const double gnode = (dar * gl + dal * gr) / (dal + dar);
  double conv = 0.0, X = 0.0;
  for (int b = 0; b < 3; b++) {
    int wl, wh;
    const double qL = q_nb(c, q, a, b, f, -1, &wl), qH = q_nb(c, q, a, b, f, 1, &wh);
    double DL = 0.0, DH = 0.0, cl = 0.0, ch = 0.0;
    if (b == a) {
      DL = c->B * gl * Ap / dal;
      DH = c->B * gr * Ap / dar;
      if (implicit) {
        const double ubL = 0.5 * (qL + qP), ubH = 0.5 * (qP + qH);
        const double FbL = rl * ubL * Ap, FbH = rr * ubH * Ap;
        double pL = 0.0, pH = 0.0;
        if (tvd) {
          if (has_face(c, a, f[a] - 2) && has_face(c, a, f[a] + 1)) {
            int y[3];
            shift(y, f, a, -2);
            pL = psi_c(at(c, q[a], a, y), qL, qP, qH, W(c, a, f[a] - 2), dal, dar, ubL);
          }
          if (has_face(c, a, f[a] - 1) && has_face(c, a, f[a] + 2)) {
            int y[3];
            shift(y, f, a, 2);
            pH = psi_c(qL, qP, qH, at(c, q[a], a, y), dal, dar, W(c, a, f[a] + 1), ubH);
          }
        }
        cl = dmax(0.0, FbL) - FbL * pL;
        ch = dmax(0.0, -FbH) - FbH * pH;
        conv += FbH - FbL;
      }
      o.a[2 * b] = cl + 4.0 / 3.0 * DL;
      o.a[2 * b + 1] = ch + 4.0 / 3.0 * DH;
    } else {
      const int t = 3 - a - b; /* the third direction */
      const double dt3 = W(c, t, f[t]);
      const double db = W(c, b, f[b]);
      /* conductances through the two b-sides */
      for (int s = 0; s < 2; s++) {
        const int kind = side_kind(c, b, f, s);
        double D;
        if (kind == 1) {
          D = c->wt[b][s] == ORA3_NOSLIP
                  ? c->B * 0.5 * (gnode + sqrt(c->wT[b][s])) * len * dt3 / (0.5 * db)
                  : 0.0;
        } else if (kind == 2) {
          D = c->B * 0.5 * (gnode + gam_edge(c, a, b, f, 0)) * len * dt3 / (0.5 * db);
        } else if (kind == 3) {
          D = 0.0;
        } else {
          const double dn = W(c, b, f[b] + (s ? 1 : -1));
          D = c->B * gam_edge(c, a, b, f, s) * (dal + dar) * 0.5 * dt3 / (0.5 * (db + dn));
        }
        if (s) DH = D;
        else DL = D;
      }
      if (implicit) {
        for (int side = 0; side < 2; side++) {
          const int *cx = side ? r : l;
          int bl[3], bh[3];
          shift(bl, cx, b, 0);
          shift(bh, cx, b, 1);
          const double Fl = at(c, c->F[b], b, bl), Fh = at(c, c->F[b], b, bh);
          const double vl = at(c, q[b], b, bl), vh = at(c, q[b], b, bh);
          double pl = 0.0, ph = 0.0;
          if (tvd) {
            if (has_cell(c, b, f[b] - 2) && has_cell(c, b, f[b] + 1)) {
              int y1[3], y2[3];
              shift(y1, f, b, -2);
              shift(y2, f, b, 1);
              pl = psi_s(at(c, q[a], a, y1), qL, qP, at(c, q[a], a, y2), W(c, b, f[b] - 2),
                         W(c, b, f[b] - 1), db, W(c, b, f[b] + 1), vl);
            }
            if (has_cell(c, b, f[b] - 1) && has_cell(c, b, f[b] + 2)) {
              int y1[3], y2[3];
              shift(y1, f, b, -1);
              shift(y2, f, b, 2);
              ph = psi_s(at(c, q[a], a, y1), qP, qH, at(c, q[a], a, y2), W(c, b, f[b] - 1), db,
                         W(c, b, f[b] + 1), W(c, b, f[b] + 2), vh);
            }
          }
          cl += 0.5 * (dmax(0.0, Fl) - Fl * pl);
          ch += 0.5 * (dmax(0.0, -Fh) - Fh * ph);
          conv += 0.5 * (Fh - Fl);
        }
      }
      o.a[2 * b] = cl + DL;
      o.a[2 * b + 1] = ch + DH;
      /* cross-diffusion of eqs pl2/pl3 for the tangential direction b:
         d_b(Gamma d_a q_b) - 2/3 d_a(Gamma d_b q_b) over the volume */
      int rh[3], lh[3];
      shift(rh, r, b, 1);
      shift(lh, l, b, 1);
      const double qb_rl = at(c, q[b], b, r), qb_rh = at(c, q[b], b, rh);
      const double qb_ll = at(c, q[b], b, l), qb_lh = at(c, q[b], b, lh);
      X += (gam_edge(c, a, b, f, 1) * (qb_rh - qb_lh) - gam_edge(c, a, b, f, 0) * (qb_rl - qb_ll)) * dt3 -
           2.0 / 3.0 * (gr * (qb_rh - qb_rl) - gl * (qb_lh - qb_ll)) * dt3;
    }
    o.nb[2 * b] = qL;
    o.nb[2 * b + 1] = qH;
  }
  double suma = 0.0;
  for (int m = 0; m < 6; m++) suma += o.a[m];
  o.a0 = suma + conv + M / dt;
  const double Mm = (at(c, c->qm[3], 3, r) / at(c, c->qm[4], 3, r) * dar +
                     at(c, c->qm[3], 3, l) / at(c, c->qm[4], 3, l) * dal) *
                    Ap / 2.0;
  o.b = (Mm / dt * at(c, c->qm[a], a, f) + c->g[a] * Mm +
         ((scheme & ORA3_IMPLICIT) ? 0.0 : c->qx[a][lin(c, a, f)])) +
        c->B * X;
  o.area = Ap;
  return o;
}

static double nbsum(const mco3 *o) {
  double s = 0.0;
  for (int m = 0; m < 6; m++) s += o->a[m] * o->nb[m];
  return s;
}

/* ------------------------------------------------------------------ */
/* boundary values                                                    */
/* ------------------------------------------------------------------ */
/* the last a-face of a periodic direction a repeats face 0 */
static void periodic_copy(const ora3_ctx *c, int a, double *q) {
  if (!per(c, a)) return;
  const int *D = c->dim[a];
  for (int k = 0; k < D[2]; k++)
    for (int j = 0; j < D[1]; j++)
      for (int i = 0; i < D[0]; i++) {
        int f[3] = {i, j, k};
        if (f[a] != c->n[a]) continue;
        f[a] = 0;
        q[((size_t)k * D[1] + j) * D[0] + i] = q[((size_t)f[2] * D[1] + f[1]) * D[0] + f[0]];
      }
}

static void impose_bc(ora3_ctx *c, double *const *q) {
  for (int a = 0; a < 3; a++) {
    const int *D = c->dim[a];
    for (int k = 0; k < D[2]; k++)
      for (int j = 0; j < D[1]; j++)
        for (int i = 0; i < D[0]; i++) {
          int f[3] = {i, j, k};
          const size_t m = ((size_t)k * D[1] + j) * D[0] + i;
          if (per(c, a)) {
            if (f[a] == c->n[a]) {
              int y[3] = {i, j, k};
              y[a] = 0;
              q[a][m] = q[a][((size_t)y[2] * D[1] + y[1]) * D[0] + y[0]];
            }
          } else if (a == 0 && c->bc[0] == ORA3_INLET_OUTLET) {
            if (i == 0) q[a][m] = c->u_in;
            if (i == c->n[0]) q[a][m] = q[a][m - 1];
          } else if (f[a] == 0 || f[a] == c->n[a]) {
            q[a][m] = 0.0;
          }
        }
  }
}

/* ------------------------------------------------------------------ */
/* context                                                            */
/* ------------------------------------------------------------------ */
static double *dalloc(size_t n) { return (double *)calloc(n, sizeof(double)); }

ora3_ctx *ora3_create(const ora3_setup *s) {
  if (!s) return NULL;
  for (int e = 0; e < 3; e++)
    if (s->n[e] < 4) return NULL;
  ora3_ctx *c = (ora3_ctx *)calloc(1, sizeof(ora3_ctx));
  for (int e = 0; e < 3; e++) {
    c->n[e] = s->n[e];
    c->bc[e] = s->bc[e];
    c->d[e] = dalloc(s->n[e]);
    memcpy(c->d[e], s->d[e], sizeof(double) * s->n[e]);
    for (int w = 0; w < 2; w++) {
      c->wt[e][w] = s->wall_type[e][w];
      c->wT[e][w] = s->wall_T[e][w];
      for (int v = 0; v < 3; v++) c->wv[e][w][v] = s->wall_vel[e][w][v];
    }
    c->g[e] = s->g[e];
  }
  const double g = s->gamma;
  c->A = 1.0 / (g * s->Ma * s->Ma);
  c->B = 1.0 / s->Re;
  c->C1 = g / (s->Re * s->Pr);
  c->C2 = g * (g - 1.0) * s->Ma * s->Ma / s->Re;
  c->C3 = -(g - 1.0);
  c->u_in = s->u_in;
  c->T_in = s->T_in;
  c->p_in = s->p_in;
  for (int f = 0; f < 5; f++) {
    for (int e = 0; e < 3; e++) c->dim[f][e] = c->n[e] + (f == e);
    c->len[f] = (size_t)c->dim[f][0] * c->dim[f][1] * c->dim[f][2];
    c->q[f] = dalloc(c->len[f]);
    c->qn[f] = dalloc(c->len[f]);
    c->qm[f] = dalloc(c->len[f]);
  }
  c->rho = dalloc(c->len[3]);
  c->gam = dalloc(c->len[3]);
  c->Tx = dalloc(c->len[3]);
  for (int a = 0; a < 3; a++) {
    c->rf[a] = dalloc(c->len[a]);
    c->F[a] = dalloc(c->len[a]);
    c->qh[a] = dalloc(c->len[a]);
    c->dq[a] = dalloc(c->len[a]);
    c->qx[a] = dalloc(c->len[a]);
  }
  /* initial state: the inlet state (x inlet) or rest at p_in, T_in */
  for (size_t m = 0; m < c->len[0]; m++)
    c->q[0][m] = c->bc[0] == ORA3_INLET_OUTLET ? c->u_in : 0.0;
  for (size_t m = 0; m < c->len[3]; m++) {
    c->q[3][m] = c->p_in;
    c->q[4][m] = c->T_in;
  }
  impose_bc(c, c->q);
  return c;
}

void ora3_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

void ora3_destroy(ora3_ctx *c) {
  if (!c) return;
  for (int e = 0; e < 3; e++) free(c->d[e]);
  for (int f = 0; f < 5; f++) {
    free(c->q[f]);
    free(c->qn[f]);
    free(c->qm[f]);
  }
  for (int a = 0; a < 3; a++) {
    free(c->rf[a]);
    free(c->F[a]);
    free(c->qh[a]);
    free(c->dq[a]);
    free(c->qx[a]);
  }
  free(c->rho);
  free(c->gam);
  free(c->Tx);
  free(c);
}

void ora3_set_fields(ora3_ctx *c, const double *const q[5]) {
  for (int f = 0; f < 5; f++)
    if (q[f]) memcpy(c->q[f], q[f], c->len[f] * sizeof(double));
  impose_bc(c, c->q);
}

void ora3_get_fields(const ora3_ctx *c, double *const q[5]) {
  for (int f = 0; f < 5; f++)
    if (q[f]) memcpy(q[f], c->q[f], c->len[f] * sizeof(double));
}

void ora3_residuals(const ora3_ctx *c, double out[7]) { memcpy(out, c->res, sizeof(c->res)); }

double ora3_mass(const ora3_ctx *c) {
  double M = 0.0;
  for (int k = 0; k < c->n[2]; k++)
    for (int j = 0; j < c->n[1]; j++)
      for (int i = 0; i < c->n[0]; i++) {
        int x[3] = {i, j, k};
        M += at(c, c->q[3], 3, x) / at(c, c->q[4], 3, x) * vol(c, x);
      }
  return M;
}

/* ------------------------------------------------------------------ */
/* step prologue and one pass of loop 2 (Appendix A order)            */
/* ------------------------------------------------------------------ */
static void prologue(ora3_ctx *c, int scheme) {
  for (int f = 0; f < 5; f++) memcpy(c->qm[f], c->q[f], c->len[f] * sizeof(double));
  for (int a = 0; a < 3; a++) memset(c->qx[a], 0, c->len[a] * sizeof(double));
  memset(c->Tx, 0, c->len[3] * sizeof(double));
  if (scheme & ORA3_IMPLICIT) return;
  const int tvd = scheme & ORA3_TVD;
  cell_props(c, c->qm[3], c->qm[4]);
  face_fluxes(c, c->qm, tvd);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < c->n[2]; k++)
    for (int j = 0; j < c->n[1]; j++)
      for (int i = 0; i < c->n[0]; i++) {
        int x[3] = {i, j, k};
        c->Tx[lin(c, 3, x)] = T_explicit(c, x, tvd);
      }
  for (int a = 0; a < 3; a++) {
    const int *D = c->dim[a];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < D[2]; k++)
      for (int j = 0; j < D[1]; j++)
        for (int i = 0; i < D[0]; i++) {
          int f[3] = {i, j, k};
          if (solved(c, a, f)) c->qx[a][lin(c, a, f)] = q_explicit(c, a, f, tvd);
        }
  }
}

static void pass(ora3_ctx *c, double dt, int scheme) {
  const int tvd = scheme & ORA3_TVD;
  cell_props(c, c->q[3], c->q[4]);
  face_fluxes(c, c->q, tvd);
  /* temperature (pl30), Jacobi */
#pragma omp parallel for schedule(static)
  for (int k = 0; k < c->n[2]; k++)
    for (int j = 0; j < c->n[1]; j++)
      for (int i = 0; i < c->n[0]; i++) {
        int x[3] = {i, j, k};
        tco3 o = T_coefs(c, x, dt, scheme);
        c->qn[4][lin(c, 3, x)] = T_update(&o, dt);
      }
  /* pseudo velocities and d (pl18-pl21); fixed faces keep their value */
  for (int a = 0; a < 3; a++) {
    const int *D = c->dim[a];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < D[2]; k++)
      for (int j = 0; j < D[1]; j++)
        for (int i = 0; i < D[0]; i++) {
          int f[3] = {i, j, k};
          const size_t m = slot(c, a, f);
          if (solved(c, a, f)) {
            mco3 o = q_coefs(c, a, f, dt, scheme);
            c->qh[a][m] = (nbsum(&o) + o.b) / o.a0;
            c->dq[a][m] = c->A * o.area / o.a0;
          } else {
            c->qh[a][m] = c->q[a][m];
            c->dq[a][m] = 0.0;
          }
        }
    periodic_copy(c, a, c->qh[a]);
    periodic_copy(c, a, c->dq[a]);
  }
  /* pressure (pl23, pl24): T of this pass, neighbours' p old */
#pragma omp parallel for schedule(static)
  for (int k = 0; k < c->n[2]; k++)
    for (int j = 0; j < c->n[1]; j++)
      for (int i = 0; i < c->n[0]; i++) {
        int x[3] = {i, j, k};
        const size_t m = lin(c, 3, x);
        const double pP = c->q[3][m], dV = vol(c, x);
        double sa = 0.0, sap = 0.0, sb = 0.0;
        for (int e = 0; e < 3; e++) {
          int fl[3], fh[3];
          shift(fl, x, e, 0);
          shift(fh, x, e, 1);
          const double ar = area(c, e, x);
          const size_t ml = lin(c, e, fl), mh = lin(c, e, fh);
          const double aL = c->rf[e][ml] * c->dq[e][ml] * ar, aH = c->rf[e][mh] * c->dq[e][mh] * ar;
          const double bL = c->rf[e][ml] * c->qh[e][ml] * ar, bH = c->rf[e][mh] * c->qh[e][mh] * ar;
          int y[3];
          shift(y, x, e, -1);
          const double pL = side_kind(c, e, x, 0) ? pP : at(c, c->q[3], 3, y);
          shift(y, x, e, 1);
          const double pH = side_kind(c, e, x, 1) ? pP : at(c, c->q[3], 3, y);
          sa += aL + aH;
          sap += aL * pL + aH * pH;
          sb += bH - bL;
        }
        const double a0 = dV / c->qn[4][m] + sa * dt;
        const double bp = c->qm[3][m] / c->qm[4][m] * dV - sb * dt;
        c->qn[3][m] = (sap * dt + bp) / a0;
      }
  /* velocities (pl18, pl19) with the new p on both sides */
  for (int a = 0; a < 3; a++) {
    const int *D = c->dim[a];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < D[2]; k++)
      for (int j = 0; j < D[1]; j++)
        for (int i = 0; i < D[0]; i++) {
          int f[3] = {i, j, k}, l[3];
          shift(l, f, a, -1);
          const size_t m = slot(c, a, f);
          c->qn[a][m] = solved(c, a, f)
                            ? c->qh[a][m] - c->dq[a][m] * (at(c, c->qn[3], 3, f) - at(c, c->qn[3], 3, l))
                            : c->q[a][m];
        }
  }
  impose_bc(c, c->qn);
  /* residuals: increments of the unknowns, continuity residual */
  double r[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int a = 0; a < 3; a++) {
    const int *D = c->dim[a];
    for (int k = 0; k < D[2]; k++)
      for (int j = 0; j < D[1]; j++)
        for (int i = 0; i < D[0]; i++) {
          int f[3] = {i, j, k};
          const size_t m = lin(c, a, f);
          if (solved(c, a, f)) r[a] = dmax(r[a], fabs(c->qn[a][m] - c->q[a][m]));
        }
  }
  for (int k = 0; k < c->n[2]; k++)
    for (int j = 0; j < c->n[1]; j++)
      for (int i = 0; i < c->n[0]; i++) {
        int x[3] = {i, j, k};
        const size_t m = lin(c, 3, x);
        r[3] = dmax(r[3], fabs(c->qn[3][m] - c->q[3][m]));
        r[4] = dmax(r[4], fabs(c->qn[4][m] - c->q[4][m]));
        const double dV = vol(c, x);
        double R = (c->qn[3][m] / c->qn[4][m] * dV - c->qm[3][m] / c->qm[4][m] * dV) / dt;
        for (int e = 0; e < 3; e++) {
          int fl[3], fh[3];
          shift(fl, x, e, 0);
          shift(fh, x, e, 1);
          const double ar = area(c, e, x);
          R += c->rf[e][lin(c, e, fh)] * at(c, c->qn[e], e, fh) * ar -
               c->rf[e][lin(c, e, fl)] * at(c, c->qn[e], e, fl) * ar;
        }
        r[5] = dmax(r[5], fabs(R));
        r[6] += R;
      }
  memcpy(c->res, r, sizeof(r));
  for (int f = 0; f < 5; f++) {
    double *t = c->q[f];
    c->q[f] = c->qn[f];
    c->qn[f] = t;
  }
}

void ora3_step(ora3_ctx *c, double dt, int n_inner, int scheme) {
  prologue(c, scheme);
  for (int k = 0; k < n_inner; k++) pass(c, dt, scheme);
}

void ora3_eq_residuals(ora3_ctx *c, double dt, int scheme, double *const rr[5]) {
  prologue(c, scheme);
  cell_props(c, c->q[3], c->q[4]);
  face_fluxes(c, c->q, scheme & ORA3_TVD);
  for (int k = 0; k < c->n[2]; k++)
    for (int j = 0; j < c->n[1]; j++)
      for (int i = 0; i < c->n[0]; i++) {
        int x[3] = {i, j, k};
        const size_t m = lin(c, 3, x);
        tco3 o = T_coefs(c, x, dt, scheme);
        double s = 0.0;
        for (int e = 0; e < 6; e++) s += o.a[e] * o.nb[e];
        rr[4][m] = o.a0 * c->q[4][m] - (dt * (s + o.src) + (o.unst + dt * o.texp));
      }
  for (int a = 0; a < 3; a++) {
    const int *D = c->dim[a];
    for (int k = 0; k < D[2]; k++)
      for (int j = 0; j < D[1]; j++)
        for (int i = 0; i < D[0]; i++) {
          int f[3] = {i, j, k}, l[3];
          shift(l, f, a, -1);
          const size_t m = slot(c, a, f);
          rr[a][m] = 0.0;
          c->qh[a][m] = c->q[a][m];
          c->dq[a][m] = 0.0;
          if (!solved(c, a, f)) continue;
          mco3 o = q_coefs(c, a, f, dt, scheme);
          rr[a][m] = o.a0 * c->q[a][m] - (nbsum(&o) + o.b) +
                     c->A * o.area * (at(c, c->q[3], 3, f) - at(c, c->q[3], 3, l));
          c->qh[a][m] = (nbsum(&o) + o.b) / o.a0;
          c->dq[a][m] = c->A * o.area / o.a0;
        }
    periodic_copy(c, a, c->qh[a]);
    periodic_copy(c, a, c->dq[a]);
  }
  for (int k = 0; k < c->n[2]; k++)
    for (int j = 0; j < c->n[1]; j++)
      for (int i = 0; i < c->n[0]; i++) {
        int x[3] = {i, j, k};
        const size_t m = lin(c, 3, x);
        const double pP = c->q[3][m], dV = vol(c, x);
        double sa = 0.0, sap = 0.0, sb = 0.0;
        for (int e = 0; e < 3; e++) {
          int fl[3], fh[3];
          shift(fl, x, e, 0);
          shift(fh, x, e, 1);
          const double ar = area(c, e, x);
          const size_t ml = lin(c, e, fl), mh = lin(c, e, fh);
          const double aL = c->rf[e][ml] * c->dq[e][ml] * ar, aH = c->rf[e][mh] * c->dq[e][mh] * ar;
          const double bL = c->rf[e][ml] * c->qh[e][ml] * ar, bH = c->rf[e][mh] * c->qh[e][mh] * ar;
          int y[3];
          shift(y, x, e, -1);
          const double pL = side_kind(c, e, x, 0) ? pP : at(c, c->q[3], 3, y);
          shift(y, x, e, 1);
          const double pH = side_kind(c, e, x, 1) ? pP : at(c, c->q[3], 3, y);
          sa += aL + aH;
          sap += aL * pL + aH * pH;
          sb += bH - bL;
        }
        const double a0 = dV / c->q[4][m] + sa * dt;
        const double bp = c->qm[3][m] / c->qm[4][m] * dV - sb * dt;
        rr[3][m] = a0 * pP - (sap * dt + bp);
      }
}
