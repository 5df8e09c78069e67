// Three-dimensional SIMPLE-TS step: kernels and the C ABI of include/sts3.h.
//
// One thread per unknown.  A pass is a chain of streaming stencil kernels,
// each reading its neighbours through the L1/L2 caches (no LDS tiles):
//   Gamma on the cell edges along each direction      (k3_edge<c>)
//   energy equation (pl30-pl33, pl28, pl29), and the pseudo velocities and
//   d of each component (pl14-pl16, pl18-pl21 read for any component a),
//   all from the old iterate                          (k3_eqs)
//   pressure equation (pl23, pl24), six neighbours, and rho = p/T,
//   Gamma = sqrt(T) of the new iterate               (k3_pressure)
//   velocity update (pl18, pl19) and the new iterate's face densities
//   (pl10-pl11 read per direction)                   (k3_velocity<a>)
// The step prologue computes rho, Gamma and the face densities of the state
// (k3_cell, k3_rf<a>) and stores the per-step constants (the level n-1 parts
// of b^u, b^v, b^w, b^T, b^p and, for the explicit schemes, the explicit
// convective terms pl15_11 / pl31_1).  The last pass of a step reduces the
// increments and the continuity residual in fixed-order block partials.
//
// Every field array holds (nz+1+2G) x (ny+1+2G) rows of a pitch of at least
// nx+1+2G doubles (x fastest): one index serves cells and the faces of every
// direction, and G = 2 ghost layers around the domain let every neighbour of
// a stencil be loaded at a constant offset.  In a periodic direction each
// kernel that writes an array also writes the periodic images of the entries
// within G of either end (face n is the image of face 0); elsewhere the
// ghost entries hold finite values that no equation uses.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/sts3.h"
#include "sts_internal.h"

namespace sts3 {
namespace {

constexpr int BX = 64, BY = 4, NTB = BX * BY;  // 256 threads per block
constexpr int NR = 8;                           // residual partials per block
constexpr int G = 2;                            // ghost layers

struct P3 {
  int n[3];
  int per[3];
  int io;  // inlet / outlet in x
  int wt[3][2];
  double wv[3][2][3];
  double wT[3][2], sqwT[3][2];
  double A, B, C1, C2, C3, g[3];
  double u_in, T_in, p_in, rho_in, sqT_in;
  double dt, idt;
  long sy, sz, off;  // strides; index of (0, 0, 0)
  // per direction, index 0 = the first cell or face (G ghost entries before):
  // widths d, their inverses id; at face i (between cells i-1 and i) the
  // weights of cells i-1 and i in the linear interpolation to the face,
  // wlo = d_i / (d_{i-1} + d_i) and whi = d_{i-1} / (d_{i-1} + d_i), and the
  // inverse centre distance ic = 2 / (d_{i-1} + d_i); interleaved, five
  // values per index (one pointer per direction keeps the kernels' uniform
  // values within the scalar register file)
  const double *geo[3];
};
constexpr int NGEO = 5;  // d, 1/d, wlo, whi, ic

struct Fld {
  double *q[5];  // u, v, w, p, T
};

struct Work {
  double *rho, *gam;
  double *rf[3];            // face densities
  double *qh[3], *dq[3];    // pseudo velocities and d
  double *cq[3], *cT, *cp;  // per-step constants
  double *ge[3];            // Gamma on the cell edges along each direction
};

// ---------------------------------------------------------------------------
// indexing
// ---------------------------------------------------------------------------
__device__ __forceinline__ long lin(const P3 &P, int i, int j, int k) {
  return P.off + (long)k * P.sz + (long)j * P.sy + i;
}
__device__ __forceinline__ long stride(const P3 &P, int e) {
  return e == 0 ? 1 : (e == 1 ? P.sy : P.sz);
}
// value of an array at x (+ s along e); x may lie up to G outside the domain
__device__ __forceinline__ double cv(const P3 &P, const double *a, const int x[3], int e = 0,
                                     int s = 0) {
  return a[lin(P, x[0], x[1], x[2]) + s * stride(P, e)];
}
__device__ __forceinline__ double fv(const P3 &P, const double *a, int f, const int x[3],
                                     int e = 0, int s = 0) {
  (void)f;
  return cv(P, a, x, e, s);
}
__device__ __forceinline__ double W(const P3 &P, int e, int i) { return P.geo[e][NGEO * i]; }
__device__ __forceinline__ double IW(const P3 &P, int e, int i) { return P.geo[e][NGEO * i + 1]; }
__device__ __forceinline__ double WLO(const P3 &P, int e, int i) { return P.geo[e][NGEO * i + 2]; }
__device__ __forceinline__ double WHI(const P3 &P, int e, int i) { return P.geo[e][NGEO * i + 3]; }
__device__ __forceinline__ double IC(const P3 &P, int e, int i) { return P.geo[e][NGEO * i + 4]; }
// store v at x and, in periodic directions, at the images of x within the
// ghost layers (FM: bit e set where the array's index along e is a face
// index, 0 for a cell array)
template <int FM>
__device__ void put(const P3 &P, double *a, const int x[3], double v) {
  const long m = lin(P, x[0], x[1], x[2]);
  a[m] = v;
  int o[3][3], no[3];
#pragma unroll
  for (int e = 0; e < 3; e++) {
    no[e] = 1;
    o[e][0] = 0;
    if (P.per[e]) {
      if (x[e] <= (((FM >> e) & 1) ? G : G - 1)) o[e][no[e]++] = P.n[e];
      if (x[e] >= P.n[e] - G) o[e][no[e]++] = -P.n[e];
    }
  }
  if (no[0] + no[1] + no[2] == 3) return;
  for (int a0 = 0; a0 < no[0]; a0++)
    for (int a1 = 0; a1 < no[1]; a1++)
      for (int a2 = 0; a2 < no[2]; a2++)
        if (a0 | a1 | a2) a[m + o[0][a0] + (long)o[1][a1] * P.sy + (long)o[2][a2] * P.sz] = v;
}
__device__ __forceinline__ bool has_cell(const P3 &P, int e, int i) {
  return P.per[e] || (i >= 0 && i < P.n[e]);
}
__device__ __forceinline__ bool has_face(const P3 &P, int e, int i) {
  return P.per[e] || (i >= 0 && i <= P.n[e]);
}
// side s (0 low, 1 high) of cell index xe along e: 0 interior, 1 wall,
// 2 inlet, 3 outlet
__device__ __forceinline__ int side(const P3 &P, int e, int xe, int s) {
  if (P.per[e]) return 0;
  if (s == 0 && xe == 0) return (e == 0 && P.io) ? 2 : 1;
  if (s == 1 && xe == P.n[e] - 1) return (e == 0 && P.io) ? 3 : 1;
  return 0;
}
__device__ __forceinline__ bool solved(const P3 &P, int a, int fa) {
  return P.per[a] ? fa < P.n[a] : (fa > 0 && fa < P.n[a]);
}
// area of the e-faces of cell x
__device__ __forceinline__ double area(const P3 &P, int e, const int x[3]) {
  const int b = e == 0 ? 1 : 0, t = e == 2 ? 1 : 2;
  return W(P, b, x[b]) * W(P, t, x[t]);
}

// ---------------------------------------------------------------------------
// elementary functions (Sec. 3.2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double upw(double f1, double f2, double vel) {
  return vel > 0.0 ? f1 : f2;
}
// a / b as a reciprocal refined by Newton steps and a residual correction
// (within one ulp of the IEEE quotient), and 1 / b
__device__ __forceinline__ double ddiv(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = __builtin_fma(__builtin_fma(-b, r, 1.0), r, r);
  const double q = a * r;
  return __builtin_fma(__builtin_fma(-b, q, a), r, q);
}
__device__ __forceinline__ double drcp(double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = __builtin_fma(__builtin_fma(-b, r, 1.0), r, r);
  return __builtin_fma(__builtin_fma(-b, r, 1.0), r, r);
}
// van Leer psi(r) = (r + |r|) / (1 + |r|) of r = a/b, written as 2a / (a + b)
// where a and b have one sign (0 otherwise)
__device__ __forceinline__ double vanleer(double a, double b) {
  const bool same = (a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0);
  const double q = ddiv(2.0 * a, a + b);
  return same ? q : 0.0;
}
// psi_s of the face i along e between nodes 2 and 3 (cells i-1 and i), with
// the stencil widths d1..d4 and the face's weights d2/(d2+d3), d3/(d2+d3)
__device__ __forceinline__ double psi_s(const P3 &P, int e, int i, double f1, double f2, double f3,
                                        double f4, double vel) {
  const double d1 = W(P, e, i - 2), d2 = W(P, e, i - 1), d3 = W(P, e, i), d4 = W(P, e, i + 1);
  if (vel > 0.0) return WHI(P, e, i) * vanleer((d2 + d3) * (f2 - f1), (d1 + d2) * (f3 - f2));
  return -WLO(P, e, i) * vanleer((d2 + d3) * (f4 - f3), (d3 + d4) * (f3 - f2));
}
__device__ __forceinline__ double psi_c(double f1, double f2, double f3, double f4, double d1,
                                        double d2, double d3, double vel) {
  if (vel > 0.0) return 0.5 * vanleer(d2 * (f2 - f1), d1 * (f3 - f2));
  return -0.5 * vanleer(d2 * (f4 - f3), d3 * (f3 - f2));
}
__device__ __forceinline__ double hmean(double dl, double gl, double dr, double gr) {
  return ddiv((dl + dr) * gl * gr, dl * gr + dr * gl);
}
__device__ __forceinline__ double hmean2(double a, double b) { return ddiv(2.0 * a * b, a + b); }

// thread -> point of an index space of extent (X, Y, Z): one block per
// BX x BY tile of an x-y plane, blockIdx.z the plane.  (Dealing each XCD a
// contiguous slab of planes, as the 2-D pass deals tile bands, was measured
// and made no kernel faster: these kernels are bound by their per-thread
// load chains, not by L2 misses.)
// A wave covers one row of its tile (BX = 64 lanes), so y and z are uniform
// across it: taken from the first lane, they live in scalar registers, and
// the widths, weights and boundary tests along y and z become scalar loads
// and scalar branches.
static_assert(BX == 64, "one tile row per wave");
__device__ __forceinline__ bool point(int X, int Y, int Z, int x[3]) {
  x[0] = blockIdx.x * BX + threadIdx.x;
  x[1] = __builtin_amdgcn_readfirstlane((int)(blockIdx.y * BY + threadIdx.y));
  x[2] = blockIdx.z;
  return x[0] < X && x[1] < Y && x[2] < Z;
}

// ---------------------------------------------------------------------------
// cell properties and face densities
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NTB) void k3_cell(P3 P, Fld S, Work Wk) {
  int x[3];
  if (!point(P.n[0], P.n[1], P.n[2], x)) return;
  const long m = lin(P, x[0], x[1], x[2]);
  const double p = S.q[3][m], T = S.q[4][m];
  put<0>(P, Wk.rho, x, ddiv(p, T));
  put<0>(P, Wk.gam, x, sqrt(T));
}

// face density of the A-face f with velocity vel there, from rho in Wk
template <int A, bool TV>
__device__ __forceinline__ double rf_at(const P3 &P, const Work &Wk, const int f[3], double vel) {
  const int fa = f[A];
  double r;
  if (!P.per[A] && fa == 0) {
    const double rr = cv(P, Wk.rho, f);
    r = (A == 0 && P.io) ? upw(P.rho_in, rr, vel) : rr;
  } else if (!P.per[A] && fa == P.n[A]) {
    r = cv(P, Wk.rho, f, A, -1);
  } else {
    const double rl = cv(P, Wk.rho, f, A, -1), rr = cv(P, Wk.rho, f);
    r = upw(rl, rr, vel);
    if (TV && has_cell(P, A, fa - 2) && has_cell(P, A, fa + 1))
      r += psi_s(P, A, fa, cv(P, Wk.rho, f, A, -2), rl, rr, cv(P, Wk.rho, f, A, 1), vel) *
           (rr - rl);
  }
  return r;
}

template <int A, bool TV>
__global__ __launch_bounds__(NTB) void k3_rf(P3 P, Fld S, Work Wk) {
  int f[3];
  if (!point(P.n[0] + (A == 0), P.n[1] + (A == 1), P.n[2] + (A == 2), f)) return;
  if (P.per[A] && f[A] == P.n[A]) return;  // the image of face 0
  put<1 << A>(P, Wk.rf[A], f, rf_at<A, TV>(P, Wk, f, S.q[A][lin(P, f[0], f[1], f[2])]));
}

// mass flux through the e-face of cell x on side s (0 low, 1 high)
__device__ __forceinline__ double flux(const P3 &P, const Fld &S, const Work &Wk, int e,
                                       const int x[3], int s) {
  int y[3] = {x[0], x[1], x[2]};
  y[e] += s;
  return fv(P, Wk.rf[e], e, y) * fv(P, S.q[e], e, y) * area(P, e, x);
}

// ---------------------------------------------------------------------------
// energy equation
// ---------------------------------------------------------------------------
// T of the neighbour of cell x across side s of direction e, as the
// convective terms take it (inlet T_in, wall and outlet the cell's own)
__device__ __forceinline__ double T_nb(const P3 &P, const double *T, int e, const int x[3],
                                       int s, double TP) {
  const int k = side(P, e, x[e], s);
  if (k == 2) return P.T_in;
  if (k) return TP;
  return cv(P, T, x, e, s ? 1 : -1);
}

// explicit convective term of T (pl31_1) at level n-1 (S, rho, rf of n-1)
template <bool TV>
__device__ double T_explicit(const P3 &P, const Fld &S, const Work &Wk, const int x[3]) {
  const double *T = S.q[4];
  const double TP = cv(P, T, x);
  double sum = 0.0;
#pragma unroll
  for (int e = 0; e < 3; e++) {
    const double TL = T_nb(P, T, e, x, 0, TP), TH = T_nb(P, T, e, x, 1, TP);
    int yh[3] = {x[0], x[1], x[2]};
    yh[e] += 1;
    const double vl = fv(P, S.q[e], e, x), vh = fv(P, S.q[e], e, yh);
    const double Fl = flux(P, S, Wk, e, x, 0), Fh = flux(P, S, Wk, e, x, 1);
    double pl = 0.0, ph = 0.0;
    if (TV) {
      const int xe = x[e];
      if (has_cell(P, e, xe - 1) && has_cell(P, e, xe + 2))
        ph = psi_s(P, e, xe + 1, cv(P, T, x, e, -1), TP, TH, cv(P, T, x, e, 2), vh);
      if (has_cell(P, e, xe - 2) && has_cell(P, e, xe + 1))
        pl = psi_s(P, e, xe, cv(P, T, x, e, -2), TL, TP, TH, vl);
    }
    sum += -Fh * (upw(TP, TH, vh) + (TH - TP) * ph) + Fl * (upw(TL, TP, vl) + (TP - TL) * pl);
  }
  return sum;
}

// cell-centre value of component e in cell x (+ s along f)
__device__ __forceinline__ double qcell(const P3 &P, const Fld &S, int e, const int x[3], int f,
                                        int s) {
  int y[3] = {x[0], x[1], x[2]};
  y[f] += s;
  int z[3] = {y[0], y[1], y[2]};
  z[e] += 1;
  return 0.5 * (fv(P, S.q[e], e, y) + fv(P, S.q[e], e, z));
}
// component e at the centre of the f-face on side s of cell x: bilinear in
// the nearest nodes; the wall's velocity (no slip) or the cell's (slip) on a
// wall, 0 (tangential) at the inlet, the cell's at the outlet
__device__ double qface(const P3 &P, const Fld &S, int e, int f, const int x[3], int s) {
  const double qc = qcell(P, S, e, x, f, 0);
  const int k = side(P, f, x[f], s);
  if (k == 1) return P.wt[f][s] == STS3_NOSLIP ? P.wv[f][s][e] : qc;
  if (k == 2) return 0.0;
  if (k == 3) return qc;
  const double qn = qcell(P, S, e, x, f, s ? 1 : -1);
  return s ? WLO(P, f, x[f] + 1) * qc + WHI(P, f, x[f] + 1) * qn
           : WHI(P, f, x[f]) * qc + WLO(P, f, x[f]) * qn;
}

// new T of cell x (pl28-pl33)
template <bool IM, bool TV>
__device__ __forceinline__ void energy_at(const P3 &P, const Fld &S, const Work &Wk,
                                          double *Tout, const int x[3]) {
  const double *T = S.q[4];
  const double TP = cv(P, T, x), gP = cv(P, Wk.gam, x), rP = cv(P, Wk.rho, x);
  const double dV = W(P, 0, x[0]) * W(P, 1, x[1]) * W(P, 2, x[2]);
  double sa = 0.0, sn = 0.0, sF = 0.0;
#pragma unroll
  for (int e = 0; e < 3; e++) {
    const double ar = area(P, e, x), de = W(P, e, x[e]);
#pragma unroll
    for (int s = 0; s < 2; s++) {
      const int k = side(P, e, x[e], s);
      double D, nb;
      if (k == 1) {
        if (P.wt[e][s] == STS3_NOSLIP) {
          nb = P.wT[e][s];
          D = P.C1 * hmean2(gP, P.sqwT[e][s]) * ar * 2.0 * IW(P, e, x[e]);
        } else {
          nb = TP;
          D = 0.0;
        }
      } else if (k == 2) {
        nb = P.T_in;
        D = P.C1 * hmean2(gP, P.sqT_in) * ar * 2.0 * IW(P, e, x[e]);
      } else if (k == 3) {
        nb = TP;
        D = 0.0;
      } else {
        const int sg = s ? 1 : -1;
        const double dn = W(P, e, x[e] + sg), gn = cv(P, Wk.gam, x, e, sg);
        nb = cv(P, T, x, e, sg);
        D = P.C1 * (s ? hmean(de, gP, dn, gn) : hmean(dn, gn, de, gP)) * ar * IC(P, e, x[e] + s);
      }
      double a = D;
      if (IM) {
        const double Fv = flux(P, S, Wk, e, x, s);
        double psi = 0.0;
        if (TV) {
          int yf[3] = {x[0], x[1], x[2]};
          yf[e] += s;
          const double vel = fv(P, S.q[e], e, yf);
          const int xe = x[e];
          if (s == 0 && has_cell(P, e, xe - 2) && has_cell(P, e, xe + 1))
            psi = psi_s(P, e, xe, cv(P, T, x, e, -2), cv(P, T, x, e, -1), TP, cv(P, T, x, e, 1), vel);
          if (s == 1 && has_cell(P, e, xe - 1) && has_cell(P, e, xe + 2))
            psi = psi_s(P, e, xe + 1, cv(P, T, x, e, -1), TP, cv(P, T, x, e, 1), cv(P, T, x, e, 2),
                        vel);
        }
        a = (s ? fmax(0.0, -Fv) : fmax(0.0, Fv)) - Fv * psi + D;
        sF += s ? Fv : -Fv;
      }
      sa += a;
      sn += a * nb;
    }
  }
  const double a0 = P.dt * (sa + sF) + rP * dV;
  // dissipation (strain rates from the face values) and pressure work
  double dd[3], div = 0.0;
#pragma unroll
  for (int e = 0; e < 3; e++) {
    dd[e] = (fv(P, S.q[e], e, x, e, 1) - fv(P, S.q[e], e, x)) * IW(P, e, x[e]);
    div += dd[e];
  }
  double phi = 2.0 * (dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
#pragma unroll
  for (int e = 0; e < 3; e++)
#pragma unroll
    for (int f = e + 1; f < 3; f++) {
      const double sef = (qface(P, S, e, f, x, 1) - qface(P, S, e, f, x, 0)) * IW(P, f, x[f]) +
                         (qface(P, S, f, e, x, 1) - qface(P, S, f, e, x, 0)) * IW(P, e, x[e]);
      phi += sef * sef;
    }
  phi -= 2.0 / 3.0 * div * div;
  const double src = P.C2 * gP * phi * dV + P.C3 * cv(P, S.q[3], x) * div * dV;
  const long m = lin(P, x[0], x[1], x[2]);
  put<0>(P, Tout, x, ddiv(P.dt * (sn + src) + Wk.cT[m], a0));
}

// ---------------------------------------------------------------------------
// momentum of component A
// ---------------------------------------------------------------------------
// Gamma on the edge of the A-momentum volume at face f towards side s of
// direction b (the edge runs along the third direction): bilinear in the
// four cells around it; 0 on a wall (it multiplies wall-normal velocities
// only), sqrt(T_in) at the inlet, the last cells along A at the outlet
template <int A>
__device__ __forceinline__ double gam_edge(const P3 &P, const Work &Wk, int b, const int f[3],
                                           int s) {
  return cv(P, Wk.ge[3 - A - b], f, b, s);
}

// Gamma on the edges along direction C (k3_edge): at the a-face and b-face
// positions of the edge ({a, b} the two other directions) and cell index
// along C; bilinear in the four cells around it.  An edge on one boundary:
// 0 on a wall (it multiplies wall-normal velocities only), sqrt(T_in) at the
// inlet, at the outlet the last cells interpolated along the other
// direction; an edge on two boundaries is never used (0).
template <int C>
__global__ __launch_bounds__(NTB) void k3_edge(P3 P, Work Wk) {
  constexpr int a = C == 0 ? 1 : 0, b = C == 2 ? 1 : 2;
  int x[3];
  if (!point(P.n[0] + (C != 0), P.n[1] + (C != 1), P.n[2] + (C != 2), x)) return;
  if ((P.per[a] && x[a] == P.n[a]) || (P.per[b] && x[b] == P.n[b])) return;  // images
  const bool ba = !P.per[a] && (x[a] == 0 || x[a] == P.n[a]);
  const bool bb = !P.per[b] && (x[b] == 0 || x[b] == P.n[b]);
  double g = 0.0;
  if (ba != bb) {
    const int d = ba ? a : b, o = ba ? b : a;
    if (d == 0 && P.io) {
      if (x[d] == 0) {
        g = P.sqT_in;
      } else {
        int l[3] = {x[0], x[1], x[2]}, r[3] = {x[0], x[1], x[2]};
        l[d] = r[d] = P.n[d] - 1;
        l[o] -= 1;
        g = WLO(P, o, x[o]) * cv(P, Wk.gam, l) + WHI(P, o, x[o]) * cv(P, Wk.gam, r);
      }
    }
  } else if (!ba) {
#pragma unroll
    for (int ia = 0; ia < 2; ia++)
#pragma unroll
      for (int ib = 0; ib < 2; ib++) {
        int y[3] = {x[0], x[1], x[2]};
        y[a] = x[a] - 1 + ia;
        y[b] = x[b] - 1 + ib;
        const double wa = ia ? WHI(P, a, x[a]) : WLO(P, a, x[a]);
        const double wb = ib ? WHI(P, b, x[b]) : WLO(P, b, x[b]);
        g += wa * wb * cv(P, Wk.gam, y);
      }
  }
  put<(1 << a) | (1 << b)>(P, Wk.ge[C], x, g);
}

// neighbour of component A at face f across side s (-1, +1) of direction b
template <int A>
__device__ __forceinline__ double q_nb(const P3 &P, const double *q, int b, const int f[3],
                                       int s, double qP) {
  if (b == A) return fv(P, q, A, f, A, s);
  const int k = side(P, b, f[b], s > 0);
  if (k == 1) return P.wt[b][s > 0] == STS3_NOSLIP ? P.wv[b][s > 0][A] : qP;
  if (k == 2) return 0.0;
  if (k == 3) return qP;
  return fv(P, q, A, f, b, s);
}

// explicit convective term of component A (pl15_11) at level n-1
template <int A, bool TV>
__device__ double q_explicit(const P3 &P, const Fld &S, const Work &Wk, const int f[3]) {
  const double *q = S.q[A];
  const double qP = fv(P, q, A, f);
  int l[3] = {f[0], f[1], f[2]};
  l[A] -= 1;
  double sum = 0.0;
#pragma unroll
  for (int b = 0; b < 3; b++) {
    const double qL = q_nb<A>(P, q, b, f, -1, qP), qH = q_nb<A>(P, q, b, f, 1, qP);
    if (b == A) {
      const double Ap = area(P, A, f);
      const double ubH = 0.5 * (qP + qH), ubL = 0.5 * (qL + qP);
      const double FbH = cv(P, Wk.rho, f) * ubH * Ap, FbL = cv(P, Wk.rho, l) * ubL * Ap;
      double pH = 0.0, pL = 0.0;
      if (TV) {
        const int fa = f[A];
        if (has_face(P, A, fa - 1) && has_face(P, A, fa + 2))
          pH = psi_c(qL, qP, qH, fv(P, q, A, f, A, 2), W(P, A, fa - 1), W(P, A, fa),
                     W(P, A, fa + 1), ubH);
        if (has_face(P, A, fa - 2) && has_face(P, A, fa + 1))
          pL = psi_c(fv(P, q, A, f, A, -2), qL, qP, qH, W(P, A, fa - 2), W(P, A, fa - 1),
                     W(P, A, fa), ubL);
      }
      sum += -FbH * (upw(qP, qH, ubH) + (qH - qP) * pH) + FbL * (upw(qL, qP, ubL) + (qP - qL) * pL);
    } else {
      const int fb = f[b];
      double pl = 0.0, ph = 0.0;
      const bool okh = TV && has_cell(P, b, fb - 1) && has_cell(P, b, fb + 2);
      const bool okl = TV && has_cell(P, b, fb - 2) && has_cell(P, b, fb + 1);
      const double q1h = okh ? fv(P, q, A, f, b, -1) : 0.0, q4h = okh ? fv(P, q, A, f, b, 2) : 0.0;
      const double q1l = okl ? fv(P, q, A, f, b, -2) : 0.0, q4l = okl ? fv(P, q, A, f, b, 1) : 0.0;
#pragma unroll
      for (int sd = 0; sd < 2; sd++) {
        const int *cx = sd ? f : l;
        int bh[3] = {cx[0], cx[1], cx[2]};
        bh[b] += 1;
        const double vl = fv(P, S.q[b], b, cx), vh = fv(P, S.q[b], b, bh);
        const double Fl = flux(P, S, Wk, b, cx, 0), Fh = flux(P, S, Wk, b, cx, 1);
        if (okh)
          ph = psi_s(P, b, fb + 1, q1h, qP, qH, q4h, vh);
        if (okl)
          pl = psi_s(P, b, fb, q1l, qL, qP, q4l, vl);
        sum += 0.5 * (-Fh * (upw(qP, qH, vh) + (qH - qP) * ph) +
                      Fl * (upw(qL, qP, vl) + (qP - qL) * pl));
      }
    }
  }
  return sum;
}

// pseudo velocity and d of component A at its face f (pl14-pl16, pl18-pl21)
template <int A, bool IM, bool TV>
__device__ __forceinline__ void mom_at(const P3 &P, const Fld &S, const Work &Wk, const int f[3]) {
  if (P.per[A] && f[A] == P.n[A]) return;  // the image of face 0
  const long m = lin(P, f[0], f[1], f[2]);
  const double *q = S.q[A];
  const double qP = q[m];
  if (!solved(P, A, f[A])) {
    put<1 << A>(P, Wk.qh[A], f, qP);
    put<1 << A>(P, Wk.dq[A], f, 0.0);
    return;
  }
  int l[3] = {f[0], f[1], f[2]};
  l[A] -= 1;
  const double dal = W(P, A, f[A] - 1), dar = W(P, A, f[A]);
  const double rl = cv(P, Wk.rho, l), rr = cv(P, Wk.rho, f);
  const double gl = cv(P, Wk.gam, l), gr = cv(P, Wk.gam, f);
  const double Ap = area(P, A, f), len = 0.5 * (dal + dar);
  const double M = (rr * dar + rl * dal) * Ap / 2.0;
  const double gnode = WLO(P, A, f[A]) * gl + WHI(P, A, f[A]) * gr;
  double sa = 0.0, sn = 0.0, conv = 0.0, X = 0.0;
#pragma unroll
  for (int b = 0; b < 3; b++) {
    const double qL = q_nb<A>(P, q, b, f, -1, qP), qH = q_nb<A>(P, q, b, f, 1, qP);
    double aL, aH;
    if (b == A) {
      const double DL = P.B * gl * Ap * IW(P, A, f[A] - 1), DH = P.B * gr * Ap * IW(P, A, f[A]);
      double cl = 0.0, ch = 0.0;
      if (IM) {
        const double ubL = 0.5 * (qL + qP), ubH = 0.5 * (qP + qH);
        const double FbL = rl * ubL * Ap, FbH = rr * ubH * Ap;
        double pL = 0.0, pH = 0.0;
        if (TV) {
          const int fa = f[A];
          if (has_face(P, A, fa - 2) && has_face(P, A, fa + 1))
            pL = psi_c(fv(P, q, A, f, A, -2), qL, qP, qH, W(P, A, fa - 2), dal, dar, ubL);
          if (has_face(P, A, fa - 1) && has_face(P, A, fa + 2))
            pH = psi_c(qL, qP, qH, fv(P, q, A, f, A, 2), dal, dar, W(P, A, fa + 1), ubH);
        }
        cl = fmax(0.0, FbL) - FbL * pL;
        ch = fmax(0.0, -FbH) - FbH * pH;
        conv += FbH - FbL;
      }
      aL = cl + 4.0 / 3.0 * DL;
      aH = ch + 4.0 / 3.0 * DH;
    } else {
      const int t = 3 - A - b;
      const double d3 = W(P, t, f[t]);
      double D[2];
#pragma unroll
      for (int s = 0; s < 2; s++) {
        const int k = side(P, b, f[b], s);
        if (k == 1)
          D[s] = P.wt[b][s] == STS3_NOSLIP
                     ? P.B * (gnode + P.sqwT[b][s]) * len * d3 * IW(P, b, f[b])
                     : 0.0;
        else if (k == 2)
          D[s] = P.B * (gnode + gam_edge<A>(P, Wk, b, f, 0)) * len * d3 * IW(P, b, f[b]);
        else if (k == 3)
          D[s] = 0.0;
        else
          D[s] = P.B * gam_edge<A>(P, Wk, b, f, s) * len * d3 * IC(P, b, f[b] + s);
      }
      double cl = 0.0, ch = 0.0;
      if (IM) {
        const int fb = f[b];
        const bool okl = TV && has_cell(P, b, fb - 2) && has_cell(P, b, fb + 1);
        const bool okh = TV && has_cell(P, b, fb - 1) && has_cell(P, b, fb + 2);
#pragma unroll
        for (int sd = 0; sd < 2; sd++) {
          const int *cx = sd ? f : l;
          int bh[3] = {cx[0], cx[1], cx[2]};
          bh[b] += 1;
          const double vl = fv(P, S.q[b], b, cx), vh = fv(P, S.q[b], b, bh);
          const double Fl = flux(P, S, Wk, b, cx, 0), Fh = flux(P, S, Wk, b, cx, 1);
          double pl = 0.0, ph = 0.0;
          if (okl)
            pl = psi_s(P, b, fb, fv(P, q, A, f, b, -2), qL, qP, fv(P, q, A, f, b, 1), vl);
          if (okh)
            ph = psi_s(P, b, fb + 1, fv(P, q, A, f, b, -1), qP, qH, fv(P, q, A, f, b, 2), vh);
          cl += 0.5 * (fmax(0.0, Fl) - Fl * pl);
          ch += 0.5 * (fmax(0.0, -Fh) - Fh * ph);
          conv += 0.5 * (Fh - Fl);
        }
      }
      aL = cl + D[0];
      aH = ch + D[1];
      // cross-diffusion for the tangential direction b
      int rh[3] = {f[0], f[1], f[2]}, lh[3] = {l[0], l[1], l[2]};
      rh[b] += 1;
      lh[b] += 1;
      const double *qb = S.q[b];
      const double b_rl = fv(P, qb, b, f), b_rh = fv(P, qb, b, rh);
      const double b_ll = fv(P, qb, b, l), b_lh = fv(P, qb, b, lh);
      X += (gam_edge<A>(P, Wk, b, f, 1) * (b_rh - b_lh) - gam_edge<A>(P, Wk, b, f, 0) * (b_rl - b_ll)) *
               d3 -
           2.0 / 3.0 * (gr * (b_rh - b_rl) - gl * (b_lh - b_ll)) * d3;
    }
    sa += aL + aH;
    sn += aL * qL + aH * qH;
  }
  const double a0 = sa + conv + M * P.idt;
  const double b = Wk.cq[A][m] + P.B * X;
  const double ia0 = drcp(a0);
  put<1 << A>(P, Wk.qh[A], f, (sn + b) * ia0);
  put<1 << A>(P, Wk.dq[A], f, P.A * Ap * ia0);
}

// Equations that read only the old iterate, several in one launch (M: bit 0
// energy, bit 1 + a momentum of component a): the thread at index x takes
// the cell x and the low face of that cell in each direction (the threads
// one past the last cell along a direction take that direction's last faces
// only).  Their inputs overlap (velocities, face densities, rho, Gamma and
// the edge Gamma around x), so a block's neighbour loads are served by the
// caches of one launch instead of being fetched again by each.  (A grid
// banded by x per XCD halved the launch's L2 misses but not its time: the
// launch holds more uniform values than the scalar registers take, and its
// spill traffic through vector lanes grew with that layout.)
template <bool IM, bool TV, int M>
__global__ __launch_bounds__(NTB) void k3_eqs(P3 P, Fld S, Work Wk, double *Tout) {
  int x[3];
  if (!point(P.n[0] + 1, P.n[1] + 1, P.n[2] + 1, x)) return;
  const bool i0 = x[0] < P.n[0], i1 = x[1] < P.n[1], i2 = x[2] < P.n[2];
  if ((M & 1) && i0 && i1 && i2) energy_at<IM, TV>(P, S, Wk, Tout, x);
  if ((M & 2) && i1 && i2) mom_at<0, IM, TV>(P, S, Wk, x);
  if ((M & 4) && i0 && i2) mom_at<1, IM, TV>(P, S, Wk, x);
  if ((M & 8) && i0 && i1) mom_at<2, IM, TV>(P, S, Wk, x);
}

// ---------------------------------------------------------------------------
// pressure and velocities
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NTB) void k3_pressure(P3 P, Fld S, Work Wk, const double *Tn,
                                                   double *pout) {
  int x[3];
  if (!point(P.n[0], P.n[1], P.n[2], x)) return;
  const long m = lin(P, x[0], x[1], x[2]);
  const double pP = S.q[3][m];
  const double dV = W(P, 0, x[0]) * W(P, 1, x[1]) * W(P, 2, x[2]);
  double sa = 0.0, sap = 0.0, sb = 0.0;
#pragma unroll
  for (int e = 0; e < 3; e++) {
    int xh[3] = {x[0], x[1], x[2]};
    xh[e] += 1;
    const double ar = area(P, e, x);
    const double rL = fv(P, Wk.rf[e], e, x), rH = fv(P, Wk.rf[e], e, xh);
    const double aL = rL * fv(P, Wk.dq[e], e, x) * ar, aH = rH * fv(P, Wk.dq[e], e, xh) * ar;
    const double bL = rL * fv(P, Wk.qh[e], e, x) * ar, bH = rH * fv(P, Wk.qh[e], e, xh) * ar;
    const double pL = side(P, e, x[e], 0) ? pP : cv(P, S.q[3], x, e, -1);
    const double pH = side(P, e, x[e], 1) ? pP : cv(P, S.q[3], x, e, 1);
    sa += aL + aH;
    sap += aL * pL + aH * pH;
    sb += bH - bL;
  }
  const double Tm = Tn[m];
  const double a0 = ddiv(dV, Tm) + sa * P.dt;
  const double pm = ddiv(sap * P.dt + (Wk.cp[m] - sb * P.dt), a0);
  put<0>(P, pout, x, pm);
  // rho and Gamma of the new iterate, which the next pass reads (nothing
  // later in this pass reads those of the old one)
  put<0>(P, Wk.rho, x, ddiv(pm, Tm));
  put<0>(P, Wk.gam, x, sqrt(Tm));
}

template <int A>
__device__ __forceinline__ double q_update(const P3 &P, const Work &Wk, const double *pn,
                                           const int f[3]) {
  return fv(P, Wk.qh[A], A, f) - fv(P, Wk.dq[A], A, f) * (cv(P, pn, f) - cv(P, pn, f, A, -1));
}

// new velocity of component A (pl18, pl19); RF: also the face density of the
// new iterate at the face (the next pass's, from the rho the pressure kernel
// stored), which replaces the old one (read by nothing later in this pass
// but the residuals of the last pass, which launches without RF)
template <int A, bool RF, bool TV>
__global__ __launch_bounds__(NTB) void k3_velocity(P3 P, Fld S, Work Wk, const double *pn,
                                                   double *qout) {
  int f[3];
  if (!point(P.n[0] + (A == 0), P.n[1] + (A == 1), P.n[2] + (A == 2), f)) return;
  const int fa = f[A];
  if (P.per[A] && fa == P.n[A]) return;  // the image of face 0
  const long m = lin(P, f[0], f[1], f[2]);
  double qn;
  if (solved(P, A, fa)) {
    qn = q_update<A>(P, Wk, pn, f);
  } else if (A == 0 && P.io && fa == P.n[0]) {  // outlet: zero gradient
    int g[3] = {f[0], f[1], f[2]};
    g[A] = fa - 1;
    qn = q_update<A>(P, Wk, pn, g);
  } else {
    qn = S.q[A][m];  // inlet u_in, wall faces 0
  }
  put<1 << A>(P, qout, f, qn);
  if (RF) put<1 << A>(P, Wk.rf[A], f, rf_at<A, TV>(P, Wk, f, qn));
}

// ---------------------------------------------------------------------------
// per-step constants (prologue), from the state S as level n-1, with rho and
// the face densities of S in Wk
// ---------------------------------------------------------------------------
template <bool EX, bool TV>
__global__ __launch_bounds__(NTB) void k3_const_cell(P3 P, Fld S, Work Wk) {
  int x[3];
  if (!point(P.n[0], P.n[1], P.n[2], x)) return;
  const long m = lin(P, x[0], x[1], x[2]);
  const double dV = W(P, 0, x[0]) * W(P, 1, x[1]) * W(P, 2, x[2]);
  const double r = Wk.rho[m];
  Wk.cp[m] = r * dV;
  Wk.cT[m] = r * S.q[4][m] * dV + (EX ? P.dt * T_explicit<TV>(P, S, Wk, x) : 0.0);
}

template <int A, bool EX, bool TV>
__global__ __launch_bounds__(NTB) void k3_const_face(P3 P, Fld S, Work Wk) {
  int f[3];
  if (!point(P.n[0] + (A == 0), P.n[1] + (A == 1), P.n[2] + (A == 2), f)) return;
  const long m = lin(P, f[0], f[1], f[2]);
  if (!solved(P, A, f[A])) {
    Wk.cq[A][m] = 0.0;
    return;
  }
  int l[3] = {f[0], f[1], f[2]};
  l[A] -= 1;
  const double dal = W(P, A, f[A] - 1), dar = W(P, A, f[A]);
  const double Mm = (cv(P, Wk.rho, f) * dar + cv(P, Wk.rho, l) * dal) * area(P, A, f) / 2.0;
  Wk.cq[A][m] = Mm * P.idt * S.q[A][m] + P.g[A] * Mm + (EX ? q_explicit<A, TV>(P, S, Wk, f) : 0.0);
}

// ---------------------------------------------------------------------------
// residuals of the last pass: increments of the unknowns, continuity
// residual; block partials in a fixed order, then one block folds them
// ---------------------------------------------------------------------------
__device__ void block_reduce(double v[NR], double *out) {
  __shared__ double red[NTB / 64][NR];
  const int t = threadIdx.y * BX + threadIdx.x, lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int q = 0; q < NR; q++) {
    double a = v[q];
    for (int o = 32; o > 0; o >>= 1) {
      const double b = __shfl_down(a, o, 64);
      a = (q == 6 || q == 7) ? a + b : fmax(a, b);
    }
    if (lane == 0) red[wv][q] = a;
  }
  __syncthreads();
  if (t < NR) {
    double a = red[0][t];
    for (int w = 1; w < NTB / 64; w++) a = (t == 6 || t == 7) ? a + red[w][t] : fmax(a, red[w][t]);
    out[t] = a;
  }
}

// partial slot of a block (blocks of the cell kernel first, then those of
// the three face kernels)
__device__ __forceinline__ long block_slot(int base) {
  return base + ((long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
}

__global__ __launch_bounds__(NTB) void k3_resid_cell(P3 P, Fld O, Fld N, Work Wk,
                                                     double *part) {
  int x[3];
  double v[NR] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (point(P.n[0], P.n[1], P.n[2], x)) {
    const long m = lin(P, x[0], x[1], x[2]);
    const double dV = W(P, 0, x[0]) * W(P, 1, x[1]) * W(P, 2, x[2]);
    const double pn = N.q[3][m], Tn = N.q[4][m];
    v[3] = fabs(pn - O.q[3][m]);
    v[4] = fabs(Tn - O.q[4][m]);
    double R = (pn / Tn * dV - Wk.cp[m]) / P.dt;
#pragma unroll
    for (int e = 0; e < 3; e++) {
      int xh[3] = {x[0], x[1], x[2]};
      xh[e] += 1;
      const double ar = area(P, e, x);
      R += fv(P, Wk.rf[e], e, xh) * fv(P, N.q[e], e, xh) * ar -
           fv(P, Wk.rf[e], e, x) * fv(P, N.q[e], e, x) * ar;
    }
    v[5] = fabs(R);
    v[6] = R;
    v[7] = (double)(!isfinite(pn)) + (double)(!isfinite(Tn));
  }
  block_reduce(v, part + block_slot(0) * NR);
}

template <int A>
__global__ __launch_bounds__(NTB) void k3_resid_face(P3 P, Fld O, Fld N, double *part, int base) {
  int f[3];
  double v[NR] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (point(P.n[0] + (A == 0), P.n[1] + (A == 1), P.n[2] + (A == 2), f)) {
    const long m = lin(P, f[0], f[1], f[2]);
    const double qn = N.q[A][m];
    if (solved(P, A, f[A])) v[A] = fabs(qn - O.q[A][m]);
    v[7] = (double)(!isfinite(qn));
  }
  block_reduce(v, part + block_slot(base) * NR);
}

// fold rows [blockIdx.x * chunk, (blockIdx.x + 1) * chunk) of nrows into
// row blockIdx.x of out (fixed order)
__global__ __launch_bounds__(NTB) void k3_resid_fold(const double *part, int nrows, int chunk,
                                                     double *out) {
  double v[NR] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int t = threadIdx.y * BX + threadIdx.x;
  const int b0 = blockIdx.x * chunk, b1 = min(nrows, b0 + chunk);
  for (int b = b0 + t; b < b1; b += NTB)
#pragma unroll
    for (int q = 0; q < NR; q++)
      v[q] = (q == 6 || q == 7) ? v[q] + part[(long)b * NR + q] : fmax(v[q], part[(long)b * NR + q]);
  block_reduce(v, out + (long)blockIdx.x * NR);
}
constexpr int FOLD_BLOCKS = 512;

}  // namespace
}  // namespace sts3

// ===========================================================================
// host side
// ===========================================================================
using namespace sts3;

struct sts3_ctx {
  P3 P;
  int n[3];
  long pitch, sy, sz, off;
  size_t field_bytes;
  hipStream_t stream;
  bool own_stream;
  int device;
  std::vector<void *> allocs;
  Fld st[2];
  int cur;
  Work Wk;
  double *d_d[3];  // per direction: NGEO values per index (G ghosts each end)
  double *part, *dres;
  double *hres;  // pinned
  int nblk_cell, nblk_face[3], nblocks;
  bool stepped;
  std::vector<double> wid[3];
  int bc[3];
  double u_in;
};

namespace {
sts_status fail3(sts_status s, const char *msg) { return sts::report_error(s, msg); }

#define HIP3(call)                                                         \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess) {                                                \
      std::string m_ = std::string(#call) + " failed: " + hipGetErrorString(e_); \
      return fail3(STS_EDEVICE, m_.c_str());                               \
    }                                                                      \
  } while (0)

// as HIP3, for sts3_create after the context exists: releases it first
#define HIP3_CREATE(call)                                                  \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess) {                                                \
      std::string m_ = std::string(#call) + " failed: " + hipGetErrorString(e_); \
      sts3_destroy(c);                                                     \
      return fail3(STS_EDEVICE, m_.c_str());                               \
    }                                                                      \
  } while (0)

dim3 grid_of(const sts3_ctx *c, int X, int Y, int Z) {
  (void)c;
  return dim3((X + BX - 1) / BX, (Y + BY - 1) / BY, Z);
}
dim3 grid_face(const sts3_ctx *c, int a) {
  return grid_of(c, c->n[0] + (a == 0), c->n[1] + (a == 1), c->n[2] + (a == 2));
}

void launch_rf(sts3_ctx *c, const Fld &S, bool tv) {
  const dim3 b(BX, BY);
  if (tv) {
    hipLaunchKernelGGL((k3_rf<0, true>), grid_face(c, 0), b, 0, c->stream, c->P, S, c->Wk);
    hipLaunchKernelGGL((k3_rf<1, true>), grid_face(c, 1), b, 0, c->stream, c->P, S, c->Wk);
    hipLaunchKernelGGL((k3_rf<2, true>), grid_face(c, 2), b, 0, c->stream, c->P, S, c->Wk);
  } else {
    hipLaunchKernelGGL((k3_rf<0, false>), grid_face(c, 0), b, 0, c->stream, c->P, S, c->Wk);
    hipLaunchKernelGGL((k3_rf<1, false>), grid_face(c, 1), b, 0, c->stream, c->P, S, c->Wk);
    hipLaunchKernelGGL((k3_rf<2, false>), grid_face(c, 2), b, 0, c->stream, c->P, S, c->Wk);
  }
}

// Per-step constants from S, and rho, Gamma and the face densities of S,
// which the first pass reads as those of its old iterate (EX, TV: explicit
// convective terms of that scheme; tvd: TVD face densities).
template <bool EX, bool TV>
void launch_prologue3(sts3_ctx *c, const Fld &S, bool tvd) {
  const dim3 b(BX, BY), gc = grid_of(c, c->n[0], c->n[1], c->n[2]);
  hipLaunchKernelGGL(k3_cell, gc, b, 0, c->stream, c->P, S, c->Wk);
  launch_rf(c, S, tvd);
  hipLaunchKernelGGL((k3_const_cell<EX, TV>), gc, b, 0, c->stream, c->P, S, c->Wk);
  hipLaunchKernelGGL((k3_const_face<0, EX, TV>), grid_face(c, 0), b, 0, c->stream, c->P, S, c->Wk);
  hipLaunchKernelGGL((k3_const_face<1, EX, TV>), grid_face(c, 1), b, 0, c->stream, c->P, S, c->Wk);
  hipLaunchKernelGGL((k3_const_face<2, EX, TV>), grid_face(c, 2), b, 0, c->stream, c->P, S, c->Wk);
}

// One pass from O to N.  rho, Gamma and the face densities of O are in Wk on
// entry (from the prologue, or the previous pass's pressure and velocity
// kernels); a pass other than the last leaves those of N there.
template <bool IM, bool TV>
void launch_pass3d(sts3_ctx *c, const Fld &O, const Fld &N, bool last) {
  const dim3 b(BX, BY), gc = grid_of(c, c->n[0], c->n[1], c->n[2]);
  hipLaunchKernelGGL((k3_edge<0>), grid_of(c, c->n[0], c->n[1] + 1, c->n[2] + 1), b, 0, c->stream,
                     c->P, c->Wk);
  hipLaunchKernelGGL((k3_edge<1>), grid_of(c, c->n[0] + 1, c->n[1], c->n[2] + 1), b, 0, c->stream,
                     c->P, c->Wk);
  hipLaunchKernelGGL((k3_edge<2>), grid_of(c, c->n[0] + 1, c->n[1] + 1, c->n[2]), b, 0, c->stream,
                     c->P, c->Wk);
  const dim3 ge = grid_of(c, c->n[0] + 1, c->n[1] + 1, c->n[2] + 1);
  hipLaunchKernelGGL((k3_eqs<IM, TV, 15>), ge, b, 0, c->stream, c->P, O, c->Wk, N.q[4]);
  hipLaunchKernelGGL(k3_pressure, gc, b, 0, c->stream, c->P, O, c->Wk, N.q[4], N.q[3]);
  if (last) {
    hipLaunchKernelGGL((k3_velocity<0, false, TV>), grid_face(c, 0), b, 0, c->stream, c->P, O, c->Wk, N.q[3], N.q[0]);
    hipLaunchKernelGGL((k3_velocity<1, false, TV>), grid_face(c, 1), b, 0, c->stream, c->P, O, c->Wk, N.q[3], N.q[1]);
    hipLaunchKernelGGL((k3_velocity<2, false, TV>), grid_face(c, 2), b, 0, c->stream, c->P, O, c->Wk, N.q[3], N.q[2]);
  } else {
    hipLaunchKernelGGL((k3_velocity<0, true, TV>), grid_face(c, 0), b, 0, c->stream, c->P, O, c->Wk, N.q[3], N.q[0]);
    hipLaunchKernelGGL((k3_velocity<1, true, TV>), grid_face(c, 1), b, 0, c->stream, c->P, O, c->Wk, N.q[3], N.q[1]);
    hipLaunchKernelGGL((k3_velocity<2, true, TV>), grid_face(c, 2), b, 0, c->stream, c->P, O, c->Wk, N.q[3], N.q[2]);
  }
  if (last) {
    hipLaunchKernelGGL(k3_resid_cell, gc, b, 0, c->stream, c->P, O, N, c->Wk, c->part);
    int base = c->nblk_cell;
    hipLaunchKernelGGL((k3_resid_face<0>), grid_face(c, 0), b, 0, c->stream, c->P, O, N, c->part, base);
    base += c->nblk_face[0];
    hipLaunchKernelGGL((k3_resid_face<1>), grid_face(c, 1), b, 0, c->stream, c->P, O, N, c->part, base);
    base += c->nblk_face[1];
    hipLaunchKernelGGL((k3_resid_face<2>), grid_face(c, 2), b, 0, c->stream, c->P, O, N, c->part, base);
    const int chunk = (c->nblocks + FOLD_BLOCKS - 1) / FOLD_BLOCKS;
    double *rows = c->part + (long)c->nblocks * NR;
    hipLaunchKernelGGL(k3_resid_fold, dim3(FOLD_BLOCKS), b, 0, c->stream, c->part, c->nblocks,
                       chunk, rows);
    hipLaunchKernelGGL(k3_resid_fold, dim3(1), b, 0, c->stream, rows, FOLD_BLOCKS, FOLD_BLOCKS,
                       c->dres);
  }
}

int nblk(const dim3 &g) { return (int)(g.x * g.y * g.z); }

// host-side boundary values of a dense state (the oracle's rules)
void impose(const sts3_ctx *c, std::vector<double> *q) {
  const int *n = c->n;
  for (int a = 0; a < 3; a++) {
    const int D0 = n[0] + (a == 0), D1 = n[1] + (a == 1), D2 = n[2] + (a == 2);
    for (int k = 0; k < D2; k++)
      for (int j = 0; j < D1; j++)
        for (int i = 0; i < D0; i++) {
          const int f[3] = {i, j, k};
          const size_t m = ((size_t)k * D1 + j) * D0 + i;
          if (c->bc[a] == STS3_PERIODIC) {
            if (f[a] == n[a]) {
              int g[3] = {i, j, k};
              g[a] = 0;
              q[a][m] = q[a][((size_t)g[2] * D1 + g[1]) * D0 + g[0]];
            }
          } else if (a == 0 && c->bc[0] == STS3_INLET_OUTLET) {
            if (i == 0) q[a][m] = c->u_in;
            if (i == n[0]) q[a][m] = q[a][m - 1];
          } else if (f[a] == 0 || f[a] == n[a]) {
            q[a][m] = 0.0;
          }
        }
  }
}

size_t field_elems(const int n[3], long *pitch) {
  const long p = (long)((n[0] + 1 + 2 * G + 31) / 32) * 32;
  if (pitch) *pitch = p;
  return (size_t)p * (n[1] + 1 + 2 * G) * (n[2] + 1 + 2 * G);
}

// dense host array of field f (x fastest, extents n + (f == e)) <-> the
// padded device layout; the ghost entries get the periodic images, or
// `ghost` (finite, unused) in a direction that is not periodic
void to_padded(const sts3_ctx *c, int f, const std::vector<double> &dense,
               std::vector<double> &pad, double ghost) {
  const int *n = c->n;
  const int D[3] = {n[0] + (f == 0), n[1] + (f == 1), n[2] + (f == 2)};
  const long E[3] = {c->pitch, n[1] + 1 + 2 * G, n[2] + 1 + 2 * G};
  pad.assign(c->field_bytes / sizeof(double), ghost);
  auto at = [&](int i, int j, int k) -> double & {
    return pad[(size_t)(k + G) * c->sz + (size_t)(j + G) * c->sy + (size_t)(i + G)];
  };
  for (int k = 0; k < D[2]; k++)
    for (int j = 0; j < D[1]; j++)
      for (int i = 0; i < D[0]; i++) at(i, j, k) = dense[((size_t)k * D[1] + j) * D[0] + i];
  for (int e = 0; e < 3; e++) {
    if (c->bc[e] != STS3_PERIODIC) continue;
    const int ne = n[e], top = (f == e) ? ne + 1 : ne;  // first index above the domain
    const int lo[3] = {-G, -G, -G};
    const int hi[3] = {(int)E[0] - G, (int)E[1] - G, (int)E[2] - G};
    int x[3];
    for (x[2] = lo[2]; x[2] < hi[2]; x[2]++)
      for (x[1] = lo[1]; x[1] < hi[1]; x[1]++)
        for (x[0] = lo[0]; x[0] < hi[0]; x[0]++) {
          const int xe = x[e];
          if (xe >= 0 && xe < top) continue;
          if (xe >= top + G) continue;
          int y[3] = {x[0], x[1], x[2]};
          y[e] = xe < 0 ? xe + ne : xe - ne;
          at(x[0], x[1], x[2]) = at(y[0], y[1], y[2]);
        }
  }
}
void from_padded(const sts3_ctx *c, int f, const std::vector<double> &pad, double *dense) {
  const int *n = c->n;
  const int D[3] = {n[0] + (f == 0), n[1] + (f == 1), n[2] + (f == 2)};
  for (int k = 0; k < D[2]; k++)
    for (int j = 0; j < D[1]; j++)
      for (int i = 0; i < D[0]; i++)
        dense[((size_t)k * D[1] + j) * D[0] + i] =
            pad[(size_t)(k + G) * c->sz + (size_t)(j + G) * c->sy + (size_t)(i + G)];
}
constexpr int NFIELDS = 29;  // 2 states x 5, rho, gam, rf x3, qh x3, dq x3, cq x3, cT, cp, ge x3
}  // namespace

extern "C" sts_status sts3_device_bytes(const int n[3], size_t *bytes) {
  if (!n || !bytes) return fail3(STS_EINVAL, "NULL argument");
  for (int e = 0; e < 3; e++)
    if (n[e] < 4) return fail3(STS_EINVAL, "every direction needs >= 4 cells");
  const size_t fe = field_elems(n, nullptr);
  *bytes = NFIELDS * fe * sizeof(double);
  return STS_OK;
}

extern "C" void sts3_destroy(sts3_ctx *c) {
  if (!c) return;
  if (c->device >= 0) (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (void *p : c->allocs) (void)hipFree(p);
  if (c->hres) (void)hipHostFree(c->hres);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

extern "C" sts_status sts3_create(const sts3_setup *s, void *hip_stream, sts3_ctx **out) {
  if (!s || !out) return fail3(STS_EINVAL, "NULL argument");
  for (int e = 0; e < 3; e++) {
    if (s->n[e] < 4) return fail3(STS_EINVAL, "every direction needs >= 4 cells");
    if (!s->d[e]) return fail3(STS_EINVAL, "cell widths missing");
    for (int i = 0; i < s->n[e]; i++)
      if (!(s->d[e][i] > 0) || !isfinite(s->d[e][i]))
        return fail3(STS_EINVAL, "cell widths must be positive and finite");
    const int bc = s->bc[e];
    if (e == 0 && bc != STS3_PERIODIC && bc != STS3_INLET_OUTLET)
      return fail3(STS_EINVAL, "x is inlet/outlet or periodic");
    if (e > 0 && bc != STS3_PERIODIC && bc != STS3_WALLS)
      return fail3(STS_EINVAL, "y and z are walls or periodic");
    for (int w = 0; w < 2; w++) {
      if (s->wall_type[e][w] != STS3_NOSLIP && s->wall_type[e][w] != STS3_SLIP)
        return fail3(STS_EINVAL, "unknown wall type");
      if (bc == STS3_WALLS && s->wall_type[e][w] == STS3_NOSLIP && !(s->wall_T[e][w] > 0))
        return fail3(STS_EINVAL, "wall temperatures must be > 0");
    }
  }
  if (!(s->Ma > 0) || !(s->Re > 0) || !(s->Pr > 0) || !(s->gamma > 1))
    return fail3(STS_EINVAL, "Ma, Re, Pr must be > 0 and gamma > 1");
  if (!(s->T_in > 0) || !(s->p_in > 0) || !isfinite(s->u_in))
    return fail3(STS_EINVAL, "T_in, p_in must be > 0 and u_in finite");
  size_t bytes = 0;
  sts_status st = sts3_device_bytes(s->n, &bytes);
  if (st != STS_OK) return st;

  sts3_ctx *c = new sts3_ctx();
  c->device = -1;
  c->hres = nullptr;
  c->stream = nullptr;
  c->own_stream = false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    delete c;
    return fail3(STS_EDEVICE, "no HIP device");
  }
  c->device = dev;
  for (int e = 0; e < 3; e++) {
    c->n[e] = s->n[e];
    c->bc[e] = s->bc[e];
    c->wid[e].assign(s->d[e], s->d[e] + s->n[e]);
  }
  c->u_in = s->u_in;
  const size_t fe = field_elems(c->n, &c->pitch);
  c->sy = c->pitch;
  c->sz = c->pitch * (c->n[1] + 1 + 2 * G);
  c->off = (long)G * c->sz + (long)G * c->sy + G;
  c->field_bytes = fe * sizeof(double);
  auto alloc = [&](size_t b, void **p) -> bool {
    if (hipMalloc(p, b) != hipSuccess) return false;
    c->allocs.push_back(*p);
    return true;
  };
  std::vector<double *> fields(NFIELDS);
  for (int k = 0; k < NFIELDS; k++)
    if (!alloc(c->field_bytes, (void **)&fields[k])) {
      sts3_destroy(c);
      return fail3(STS_ENOMEM, "device allocation failed");
    }
  int k = 0;
  for (int b = 0; b < 2; b++)
    for (int f = 0; f < 5; f++) c->st[b].q[f] = fields[k++];
  c->Wk.rho = fields[k++];
  c->Wk.gam = fields[k++];
  for (int a = 0; a < 3; a++) c->Wk.rf[a] = fields[k++];
  for (int a = 0; a < 3; a++) c->Wk.qh[a] = fields[k++];
  for (int a = 0; a < 3; a++) c->Wk.dq[a] = fields[k++];
  for (int a = 0; a < 3; a++) c->Wk.cq[a] = fields[k++];
  c->Wk.cT = fields[k++];
  c->Wk.cp = fields[k++];
  for (int a = 0; a < 3; a++) c->Wk.ge[a] = fields[k++];
  for (int e = 0; e < 3; e++)
    if (!alloc(sizeof(double) * NGEO * (c->n[e] + 2 * G), (void **)&c->d_d[e])) {
      sts3_destroy(c);
      return fail3(STS_ENOMEM, "device allocation failed");
    }
  c->nblk_cell = nblk(grid_of(c, c->n[0], c->n[1], c->n[2]));
  c->nblocks = c->nblk_cell;
  for (int a = 0; a < 3; a++) {
    c->nblk_face[a] = nblk(grid_face(c, a));
    c->nblocks += c->nblk_face[a];
  }
  if (!alloc(sizeof(double) * NR * ((size_t)c->nblocks + FOLD_BLOCKS), (void **)&c->part) ||
      !alloc(256, (void **)&c->dres) || hipHostMalloc((void **)&c->hres, 256) != hipSuccess) {
    c->hres = nullptr;
    sts3_destroy(c);
    return fail3(STS_ENOMEM, "allocation failed");
  }
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      c->stream = nullptr;
      sts3_destroy(c);
      return fail3(STS_EDEVICE, "hipStreamCreate failed");
    }
    c->own_stream = true;
  }
  // parameters (eqs pl2-pl6 coefficients as in the 2-D library)
  P3 &P = c->P;
  memset(&P, 0, sizeof P);
  for (int e = 0; e < 3; e++) {
    P.n[e] = c->n[e];
    P.per[e] = s->bc[e] == STS3_PERIODIC;
    P.g[e] = s->g[e];
    P.geo[e] = c->d_d[e] + NGEO * G;
    for (int w = 0; w < 2; w++) {
      P.wt[e][w] = s->wall_type[e][w];
      P.wT[e][w] = s->wall_T[e][w];
      P.sqwT[e][w] = s->wall_T[e][w] > 0 ? sqrt(s->wall_T[e][w]) : 0.0;
      for (int v = 0; v < 3; v++) P.wv[e][w][v] = s->wall_vel[e][w][v];
    }
  }
  P.io = s->bc[0] == STS3_INLET_OUTLET;
  const double g = s->gamma;
  P.A = 1.0 / (g * s->Ma * s->Ma);
  P.B = 1.0 / s->Re;
  P.C1 = g / (s->Re * s->Pr);
  P.C2 = g * (g - 1.0) * s->Ma * s->Ma / s->Re;
  P.C3 = -(g - 1.0);
  P.u_in = s->u_in;
  P.T_in = s->T_in;
  P.p_in = s->p_in;
  P.rho_in = s->p_in / s->T_in;
  P.sqT_in = sqrt(s->T_in);
  P.sy = c->sy;
  P.sz = c->sz;
  P.off = c->off;
  // widths with G ghosts at each end: periodic images, or the end cell's
  for (int e = 0; e < 3; e++) {
    const int ne = c->n[e];
    auto width = [&](int i) {
      const int w = P.per[e] ? ((i % ne) + ne) % ne : std::min(std::max(i, 0), ne - 1);
      return c->wid[e][w];
    };
    std::vector<double> g;
    for (int i = -G; i < ne + G; i++) {
      const double dl = width(i - 1), d = width(i);
      g.push_back(d);
      g.push_back(1.0 / d);
      g.push_back(d / (dl + d));
      g.push_back(dl / (dl + d));
      g.push_back(2.0 / (dl + d));
    }
    HIP3_CREATE(hipMemcpy(c->d_d[e], g.data(), sizeof(double) * g.size(), hipMemcpyHostToDevice));
  }
  // clear every array (frame entries stay finite), then the initial state
  for (int k2 = 0; k2 < NFIELDS; k2++)
    HIP3_CREATE(hipMemsetAsync(fields[k2], 0, c->field_bytes, c->stream));
  c->cur = 0;
  c->stepped = false;
  std::vector<double> q[5];
  for (int f = 0; f < 5; f++) {
    const size_t len = (size_t)(c->n[0] + (f == 0)) * (c->n[1] + (f == 1)) * (c->n[2] + (f == 2));
    q[f].assign(len, f == 0 ? (P.io ? s->u_in : 0.0) : (f == 3 ? s->p_in : (f == 4 ? s->T_in : 0.0)));
  }
  const double *qp[5] = {q[0].data(), q[1].data(), q[2].data(), q[3].data(), q[4].data()};
  st = sts3_set_fields(c, qp);
  if (st != STS_OK) {
    sts3_destroy(c);
    return st;
  }
  *out = c;
  return STS_OK;
}

extern "C" sts_status sts3_set_fields(sts3_ctx *c, const double *const q[5]) {
  if (!c || !q) return fail3(STS_EINVAL, "NULL argument");
  HIP3(hipSetDevice(c->device));
  HIP3(hipStreamSynchronize(c->stream));
  std::vector<double> dense[5], pad;
  const int *n = c->n;
  for (int f = 0; f < 5; f++) {
    const size_t len = (size_t)(n[0] + (f == 0)) * (n[1] + (f == 1)) * (n[2] + (f == 2));
    dense[f].resize(len);
    if (q[f]) {
      memcpy(dense[f].data(), q[f], len * sizeof(double));
    } else {  // keep the current field
      pad.resize(c->field_bytes / sizeof(double));
      HIP3(hipMemcpy(pad.data(), c->st[c->cur].q[f], c->field_bytes, hipMemcpyDeviceToHost));
      from_padded(c, f, pad, dense[f].data());
    }
  }
  impose(c, dense);
  for (int f = 0; f < 5; f++) {
    to_padded(c, f, dense[f], pad, f >= 3 ? 1.0 : 0.0);
    // both state buffers: faces that the passes do not write keep these values
    for (int b = 0; b < 2; b++)
      HIP3(hipMemcpy(c->st[b].q[f], pad.data(), c->field_bytes, hipMemcpyHostToDevice));
  }
  c->stepped = false;
  return STS_OK;
}

extern "C" sts_status sts3_fields(sts3_ctx *c, double *const q[5]) {
  if (!c || !q) return fail3(STS_EINVAL, "NULL argument");
  HIP3(hipSetDevice(c->device));
  HIP3(hipStreamSynchronize(c->stream));
  std::vector<double> pad(c->field_bytes / sizeof(double));
  for (int f = 0; f < 5; f++) {
    if (!q[f]) continue;
    HIP3(hipMemcpy(pad.data(), c->st[c->cur].q[f], c->field_bytes, hipMemcpyDeviceToHost));
    from_padded(c, f, pad, q[f]);
  }
  return STS_OK;
}

extern "C" sts_status sts3_step(sts3_ctx *c, double dt, int n_inner, int scheme) {
  if (!c) return fail3(STS_EINVAL, "ctx is NULL");
  if (!(dt > 0) || !isfinite(dt)) return fail3(STS_EINVAL, "dt must be > 0");
  if (n_inner < 1) return fail3(STS_EINVAL, "n_inner must be >= 1");
  if (scheme & ~(STS_IMPLICIT | STS_TVD)) return fail3(STS_EINVAL, "unknown scheme bits");
  HIP3(hipSetDevice(c->device));
  c->P.dt = dt;
  c->P.idt = 1.0 / dt;
  const bool im = scheme & STS_IMPLICIT, tv = scheme & STS_TVD;
  const Fld S0 = c->st[c->cur];
  if (im) launch_prologue3<false, false>(c, S0, tv);
  else if (tv) launch_prologue3<true, true>(c, S0, true);
  else launch_prologue3<true, false>(c, S0, false);
  for (int k = 0; k < n_inner; k++) {
    const Fld O = c->st[c->cur], N = c->st[c->cur ^ 1];
    const bool last = k == n_inner - 1;
    if (im && tv) launch_pass3d<true, true>(c, O, N, last);
    else if (im) launch_pass3d<true, false>(c, O, N, last);
    else if (tv) launch_pass3d<false, true>(c, O, N, last);
    else launch_pass3d<false, false>(c, O, N, last);
    c->cur ^= 1;
  }
  HIP3(hipGetLastError());
  HIP3(hipMemcpyAsync(c->hres, c->dres, NR * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  c->stepped = true;
  return STS_OK;
}

extern "C" sts_status sts3_residuals(sts3_ctx *c, double out[7]) {
  if (!c || !out) return fail3(STS_EINVAL, "NULL argument");
  HIP3(hipSetDevice(c->device));
  HIP3(hipStreamSynchronize(c->stream));
  for (int k = 0; k < 7; k++) out[k] = c->stepped ? c->hres[k] : 0.0;
  if (c->stepped && c->hres[7] != 0.0) return fail3(STS_ENONFINITE, "the last step produced non-finite values");
  return STS_OK;
}
