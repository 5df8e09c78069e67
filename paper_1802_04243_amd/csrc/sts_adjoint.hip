// Hand-written adjoint (reverse mode) of the explicit-scheme SIMPLE-TS step
// for gfx950, and the obstacle drag used as its loss.
//
// The step (Sec. 3.1, explicit convective terms eqs pl15_11 and pl31_1) is
// a prologue (per-step constants from the level n-1 fields) followed by
// n_inner Jacobi passes, each of which computes, from the old iterate:
//   (0) rho = p/T and Gamma = sqrt(T) per cell,
//   (1) face densities rho^u, rho^v (eqs pl10, pl11, upwind or TVD),
//   (2) T (eqs pl30-pl33, pl28, pl29), u-hat, d^u, v-hat, d^v (eqs pl14-pl21),
//   (3) p (eqs pl23, pl24),
//   (4) u, v (eqs pl18, pl19).
// The reverse of a pass runs (4), (3), (2), (1), (0) backwards; each kernel
// below takes one output item (cell or face), recomputes its local
// quantities from the stored old iterate and the pass's intermediates (kept
// by the forward pass kernel, so they are bitwise those of the forward run)
// and adds the output's adjoint times the local partial derivatives to the
// adjoints of its inputs.  Contributions of several items to one input are
// summed with hardware FP64 atomics: the result is exact up to the order of
// those sums.  The functions mirror the general (boundary-aware) forward
// bodies for a channel that is not periodic.
#include "sts_internal.h"

namespace sts {
namespace {

constexpr int AB = 256;  // threads per block of the adjoint kernels

__device__ __forceinline__ long ix(const Params &P, int i, int j) {
  return P.off + (long)j * P.pitch + i;
}
__device__ __forceinline__ double at(const double *a, const Params &P, int i, int j) {
  return a[ix(P, i, j)];
}
__device__ __forceinline__ void aadd(double *a, const Params &P, int i, int j, double x) {
  unsafeAtomicAdd(a + ix(P, i, j), x);
}
__device__ __forceinline__ bool fl(const Params &P, int i, int j) {
  if (i < 0 || i >= P.nx || j < 0 || j >= P.ny) return false;
  return P.fl[ix(P, i, j)] != 0;
}
// geometry: q = 0 width, 1 inverse width, 2 face sum, 3 its inverse,
// 4/5 weight of the low/high cell at the face
__device__ __forceinline__ double gx(const Params &P, int q, int i) { return P.gx6[6 * (i + XPAD) + q]; }
__device__ __forceinline__ double gy(const Params &P, int q, int j) { return P.gy6[6 * (j + XPAD) + q]; }
__device__ __forceinline__ double rho(const Params &P, const State &o, int i, int j) {
  return at(o.p, P, i, j) / at(o.T, P, i, j);
}
__device__ __forceinline__ double gam(const Params &P, const State &o, int i, int j) {
  return sqrt(at(o.T, P, i, j));
}
// rho and Gamma of a state's cells computed once (k_cell_cache) and read by
// the stages that need them many times per item; the same values as above
struct Cache {
  const double *r, *g;
};
__device__ __forceinline__ double rho(const Params &P, const Cache &c, int i, int j) {
  return at(c.r, P, i, j);
}
__device__ __forceinline__ double gam(const Params &P, const Cache &c, int i, int j) {
  return at(c.g, P, i, j);
}
__device__ __forceinline__ bool u_solved(const Params &P, int i, int j) {
  return i >= 1 && i <= P.nx - 1 && fl(P, i - 1, j) && fl(P, i, j);
}
__device__ __forceinline__ bool v_solved(const Params &P, int i, int j) {
  return j >= 1 && j <= P.ny - 1 && fl(P, i, j - 1) && fl(P, i, j);
}
__device__ __forceinline__ double upw(double a, double b, double vel) { return vel > 0.0 ? a : b; }

// van Leer limiter (as in the forward pass) and its partial derivatives
__device__ __forceinline__ double vl(double a, double b, double &da, double &db) {
  const bool pos = (a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0);
  if (!pos) {
    da = db = 0.0;
    return 0.0;
  }
  const double s = a + b;
  da = 2.0 * b / (s * s);
  db = -2.0 * a / (s * s);
  return 2.0 * a / s;
}
// psi_s at a face between nodes 2 and 3 (factors s12, s23, s34, w2, w3);
// g[0..3] receive d psi / d f1..f4
__device__ double psi_s_d(double f1, double f2, double f3, double f4, double s12, double s23,
                          double s34, double w2, double w3, double vel, double g[4]) {
  const bool up = vel > 0.0;
  const double a = s23 * (up ? f2 - f1 : f4 - f3);
  const double sb = up ? s12 : s34;
  const double b = sb * (f3 - f2);
  const double w = up ? w2 : -w3;
  double da, db;
  const double q = vl(a, b, da, db);
  // a = s23 (f2 - f1) or s23 (f4 - f3); b = sb (f3 - f2)
  g[0] = up ? -w * da * s23 : 0.0;
  g[1] = (up ? w * da * s23 : 0.0) - w * db * sb;
  g[2] = (up ? 0.0 : -w * da * s23) + w * db * sb;
  g[3] = up ? 0.0 : w * da * s23;
  return w * q;
}
__device__ __forceinline__ double psix_d(const Params &P, double f1, double f2, double f3,
                                         double f4, int k, double vel, double g[4]) {
  return psi_s_d(f1, f2, f3, f4, gx(P, 2, k - 1), gx(P, 2, k), gx(P, 2, k + 1), gx(P, 5, k),
                 gx(P, 4, k), vel, g);
}
__device__ __forceinline__ double psiy_d(const Params &P, double f1, double f2, double f3,
                                         double f4, int k, double vel, double g[4]) {
  return psi_s_d(f1, f2, f3, f4, gy(P, 2, k - 1), gy(P, 2, k), gy(P, 2, k + 1), gy(P, 5, k),
                 gy(P, 4, k), vel, g);
}
// psi_c at a control-volume centre (widths d1, d2, d3)
__device__ double psi_c_d(double f1, double f2, double f3, double f4, double d1, double d2,
                          double d3, double vel, double g[4]) {
  const bool up = vel > 0.0;
  const double a = d2 * (up ? f2 - f1 : f4 - f3);
  const double sb = up ? d1 : d3;
  const double b = sb * (f3 - f2);
  const double w = up ? 0.5 : -0.5;
  double da, db;
  const double q = vl(a, b, da, db);
  g[0] = up ? -w * da * d2 : 0.0;
  g[1] = (up ? w * da * d2 : 0.0) - w * db * sb;
  g[2] = (up ? 0.0 : -w * da * d2) + w * db * sb;
  g[3] = up ? 0.0 : w * da * d2;
  return w * q;
}
// harmonic means and their partial derivatives in the Gamma arguments
__device__ __forceinline__ double hmean_d(double dl, double gl, double dr, double gr,
                                          double &dgl, double &dgr) {
  const double s = dl + dr, den = dl * gr + dr * gl;
  dgl = s * dl * gr * gr / (den * den);
  dgr = s * dr * gl * gl / (den * den);
  return s * gl * gr / den;
}
__device__ __forceinline__ double hmean2_d(double a, double b, double &da, double &db) {
  const double s = a + b;
  da = 2.0 * b * b / (s * s);
  db = 2.0 * a * a / (s * s);
  return 2.0 * a * b / s;
}
// velocity-slip / temperature-jump surface (eqs pl38, pl39): the conductance
// K g / (d/2 + k/r) of the half cell to the surface, with node Gamma g and
// node density r, and its partials in g and r
__device__ __forceinline__ double jwall_d(double K, double g, double d, double k, double r,
                                          double &dg, double &dr) {
  const double w = 1.0 / (0.5 * d + k / r);
  dg = K * w;
  dr = K * g * w * w * k / (r * r);
  return K * g * w;
}
// the gas velocity at such a surface, (u_w d/2 + zeta u_P) / (d/2 + zeta) with
// zeta = k / r, and its partials in u_P and r
__device__ __forceinline__ double slip_d(double uw, double uP, double d, double k, double r,
                                         double &du, double &dr) {
  const double h = 0.5 * d, z = k / r, den = h + z;
  du = z / den;
  dr = -(h * (uP - uw) / (den * den)) * z / r;
  return (uw * h + z * uP) / den;
}

// Gamma at the corner (x^f_i, y^f_j) and its adjoint
template <class Src>
__device__ double gamc(const Params &P, const Src &o, int i, int j) {
  if (j <= 0 || j >= P.ny) return 0.0;
  const double ws = gy(P, 4, j), wn = gy(P, 5, j);
  if (i == 0) return ws * P.inl[4 * (j - 1) + 2] + wn * P.inl[4 * (j) + 2];
  if (i == P.nx) return ws * gam(P, o, i - 1, j - 1) + wn * gam(P, o, i - 1, j);
  const double wl = gx(P, 4, i), wr = gx(P, 5, i);
  return ws * (wl * gam(P, o, i - 1, j - 1) + wr * gam(P, o, i, j - 1)) +
         wn * (wl * gam(P, o, i - 1, j) + wr * gam(P, o, i, j));
}
template <class S>
__device__ void gamc_adj(S &sk, int slot, const Params &P, int i, int j, double l) {
  if (l == 0.0 || j <= 0 || j >= P.ny || i == 0) return;
  const double ws = gy(P, 4, j), wn = gy(P, 5, j);
  if (i == P.nx) {
    sk.add(slot, P, i - 1, j - 1, l * ws);
    sk.add(slot, P, i - 1, j, l * wn);
    return;
  }
  const double wl = gx(P, 4, i), wr = gx(P, 5, i);
  sk.add(slot, P, i - 1, j - 1, l * ws * wl);
  sk.add(slot, P, i, j - 1, l * ws * wr);
  sk.add(slot, P, i - 1, j, l * wn * wl);
  sk.add(slot, P, i, j, l * wn * wr);
}
// d sqrt(Tw at u-face i) / d Tw of the two neighbouring columns
// w: 0 bottom wall, 1 top wall (sqrt of its temperature at u-face i in
// P.wu[2 i + w])
__device__ void sqtwu_adj(const Params &P, int w, double *gtw, int i, double l) {
  const int L = i - 1 < 0 ? 0 : i - 1, R = i > P.nx - 1 ? P.nx - 1 : i;
  const double d = l / (2.0 * P.wu[2 * i + w]);
  unsafeAtomicAdd(gtw + L, d * gx(P, 4, i));
  unsafeAtomicAdd(gtw + R, d * gx(P, 5, i));
}

// element (i, j) of the (nx+1) x (ny+1) index space of a thread
__device__ __forceinline__ bool elem(const Params &P, int &i, int &j) {
  const long t = (long)blockIdx.x * AB + threadIdx.x;
  if (t >= (long)(P.nx + 1) * (P.ny + 1)) return false;
  i = (int)(t % (P.nx + 1));
  j = (int)(t / (P.nx + 1));
  return true;
}

// Scatter with block-level pre-summation.  A block takes a TW x TH tile of
// the element space; a reverse kernel adds lambda_out * d(out)/d(in) to the
// adjoints of inputs within R elements of the output (R = 1 for the energy,
// u-hat and v-hat stages, 2 for the face densities).  Contributions to NA
// registered arrays inside the tile grown by R are summed in LDS (FP64 LDS
// atomics); then every nonzero entry goes to global memory once: entries at
// least R inside the tile receive contributions from this block only and are
// added with a plain read-modify-write (EXCL; not when blocks of several
// stages of one launch add to the same arrays), the others with a hardware
// FP64 atomic.  Targets outside the window (none for the stencils here) are added
// directly.  Like the plain scatter, the result is exact up to the order of
// the sums.
constexpr int TW = 32, TH = 8;
// tile of block b of n: blocks are dealt round-robin to the 8 XCDs (b mod
// 8); each XCD gets one contiguous band of tiles, so that the halo rows a
// tile shares with its neighbours are read through the same L2
__device__ __forceinline__ int tile_of_block(int b, int n) {
  const int k = b & 7, m = b >> 3, q = n >> 3, r = n & 7;
  return k * q + (k < r ? k : r) + m;
}
static_assert(TW * TH == AB, "one element per thread");
typedef __attribute__((address_space(3))) double lds_double;
template <int NA, int R, bool EXCL = true>
struct Tiled {
  static constexpr int WW = TW + 2 * R, WH = TH + 2 * R, WN = WW * WH;
  lds_double *w;     // LDS [NA][WH][WW]
  double *a[NA];     // the registered arrays (field layout)
  int x0, y0;        // tile origin
  __device__ void begin(const Params &P, int &i, int &j) {
    const int ntx = (P.nx + 1 + TW - 1) / TW;
    const int tile = tile_of_block(blockIdx.x, gridDim.x);
    x0 = (tile % ntx) * TW;
    y0 = (tile / ntx) * TH;
    i = x0 + (int)threadIdx.x % TW;
    j = y0 + (int)threadIdx.x / TW;
    for (int e = threadIdx.x; e < NA * WN; e += AB) w[e] = 0.0;
    __syncthreads();
  }
  __device__ __forceinline__ void add(int s, const Params &P, int i, int j, double x) {
    const int wi = i - x0 + R, wj = j - y0 + R;
    if ((unsigned)wi < (unsigned)WW && (unsigned)wj < (unsigned)WH)
      __hip_atomic_fetch_add(w + (s * WH + wj) * WW + wi, x, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
    else
      unsafeAtomicAdd(a[s] + ix(P, i, j), x);
  }
  __device__ void end(const Params &P) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NA; s++)
      for (int r = threadIdx.x; r < WN; r += AB) {
        const double v = w[s * WN + r];
        if (v == 0.0) continue;
        const int wj = r / WW, wi = r % WW;
        double *q = a[s] + ix(P, x0 - R + wi, y0 - R + wj);
        if (EXCL && wi >= 2 * R && wi < TW && wj >= 2 * R && wj < TH) *q += v;
        else unsafeAtomicAdd(q, v);
      }
  }
};
static dim3 tgrid(const Params &P) {
  return dim3((unsigned)(((P.nx + 1 + TW - 1) / TW) * ((P.ny + 1 + TH - 1) / TH)));
}

// ---------------------------------------------------------------------------
// (4) velocity update and cell outputs, and (3) the pressure equation:
// gather form, one launch (no atomics)
// ---------------------------------------------------------------------------
// Velocity update: u = u-hat - d^u (p_P - p_W) on solved faces, else a copy
// of the old value; the outlet face takes the new value of face nx-1.  Cell
// outputs: the adjoints of the new T and p seed those of T-new and p-new
// (fluid), the new p collecting its part of the four velocity updates around
// the cell, or pass to the old values (solid cells are copied).
// Pressure: p = N / a0 with N = (sum a_nb p_nb) dt + C_p - (bE - bW + bN -
// bS) dt, a0 = dV/T + (sum a_nb) dt, a_W = rho^u d^u dy and b_W = rho^u
// u-hat dy on the faces.  Per fluid cell lN = lambda/a0 and la0 = -lambda
// p/a0; the old pressure of a cell collects lN a dt of its four neighbours'
// equations, each face the a- and b-adjoints of the (at most two) cells it
// borders.
__device__ __forceinline__ double lam_u(const Params &P, const State &ln, int i, int j) {
  const long k = ix(P, i, j);
  return i == P.nx - 1 ? ln.u[k] + ln.u[k + 1] : ln.u[k];
}
// adjoint of the new p of fluid cell (i, j) (its own output and the four
// velocity updates around it)
__device__ __forceinline__ double lam_pnew(const Params &P, const State &ln, const Inter &I,
                                           int i, int j, long k) {
  double lp = ln.p[k];
  if (u_solved(P, i, j)) lp += -lam_u(P, ln, i, j) * I.du[k];
  if (u_solved(P, i + 1, j)) lp += lam_u(P, ln, i + 1, j) * I.du[k + 1];
  if (v_solved(P, i, j)) lp += -ln.v[k] * I.dv[k];
  if (v_solved(P, i, j + 1)) lp += ln.v[k + P.pitch] * I.dv[k + P.pitch];
  return lp;
}
// lN, la0 of fluid cell (i, j) from the adjoint l of its new p; tn, dV out
__device__ __forceinline__ void press_adj(const Params &P, const Inter &I, int i, int j, long k,
                                          double l, double &lN, double &la0, double &tn,
                                          double &dV) {
  const long kE = k + 1, kN = k + P.pitch;
  const double dxi = gx(P, 0, i), dyj = gy(P, 0, j), dt = P.dt;
  dV = dxi * dyj;
  const double aW = I.ru[k] * I.du[k] * dyj, aE = I.ru[kE] * I.du[kE] * dyj;
  const double aS = I.rv[k] * I.dv[k] * dxi, aN = I.rv[kN] * I.dv[kN] * dxi;
  tn = I.tn[k];
  const double pn = I.pn[k];
  const double a0 = dV / tn + (aW + aE + aS + aN) * dt;
  lN = l / a0;
  la0 = -l * pn / a0;
}

// One block per TW x TH tile of elements (u-face, v-face and cell (i, j)).
// Phase 1: lN, la0 of the tile's cells and of the ring of cells around it
// (the ring recomputed by both neighbouring blocks), kept in LDS.  Phase 2:
// every element assigns the entries of the temporaries and of the outgoing
// adjoint state that it or a later stage adds to (nothing is cleared before
// a pass), and ρ = p/T, Γ = √T of the iterate for the later stages.
constexpr int CW = TW + 2, CH = TH + 2;
__global__ __launch_bounds__(AB) void k_adj_front(const Params P, const State o,
                                                  const State ln, const State lo,
                                                  const Consts lC, const Inter I,
                                                  const AdjTmp A) {
  __shared__ double sq0[CH * CW], sq1[CH * CW];
  const int ntx = (P.nx + 1 + TW - 1) / TW;
  const int tile = tile_of_block(blockIdx.x, gridDim.x);
  const int x0 = (tile % ntx) * TW, y0 = (tile / ntx) * TH;
  for (int c = threadIdx.x; c < CW * CH; c += AB) {
    const int ci = x0 - 1 + c % CW, cj = y0 - 1 + c / CW;
    double lN = 0.0, la0 = 0.0;
    if (ci >= 0 && ci < P.nx && cj >= 0 && cj < P.ny && fl(P, ci, cj)) {
      const long k = ix(P, ci, cj);
      double tn, dV;
      press_adj(P, I, ci, cj, k, lam_pnew(P, ln, I, ci, cj, k), lN, la0, tn, dV);
    }
    sq0[c] = lN;
    sq1[c] = la0;
  }
  __syncthreads();
  const int i = x0 + (int)threadIdx.x % TW, j = y0 + (int)threadIdx.x / TW;
  if (i > P.nx || j > P.ny) return;
  const long k = ix(P, i, j);
  const int c = (j - y0 + 1) * CW + (i - x0 + 1);  // cell (i, j) in the LDS ring layout
  const double dt = P.dt;

  // cell (i, j)
  const bool cell = i < P.nx && j < P.ny, fluid = cell && fl(P, i, j);
  double lTn = 0.0;
  if (fluid) {  // lN, la0 of this cell from phase 1
    const double tn = I.tn[k], dV = gx(P, 0, i) * gy(P, 0, j);
    lTn = ln.T[k] + sq1[c] * (-dV / (tn * tn));
    lC.Cp[k] += sq0[c];
  }
  A.ltn[k] = lTn;
  double lpo = cell && !fluid ? ln.p[k] : 0.0;  // old pressure
  if (cell) {
    const double dxi = gx(P, 0, i), dyj = gy(P, 0, j);
    double s = 0.0;
    if (i >= 1) s += sq0[c - 1] * (I.ru[k] * I.du[k] * dyj) * dt;
    if (i + 1 < P.nx) s += sq0[c + 1] * (I.ru[k + 1] * I.du[k + 1] * dyj) * dt;
    if (j >= 1) s += sq0[c - CW] * (I.rv[k] * I.dv[k] * dxi) * dt;
    if (j + 1 < P.ny) s += sq0[c + CW] * (I.rv[k + P.pitch] * I.dv[k + P.pitch] * dxi) * dt;
    lpo += s;
    A.cr[k] = o.p[k] / o.T[k];
    A.cg[k] = sqrt(o.T[k]);
  }
  lo.p[k] = lpo;
  lo.T[k] = cell && !fluid ? ln.T[k] : 0.0;

  // u-face (i, j): velocity update, then the west face of cell (i, j) and
  // the east face of cell (i-1, j) in the pressure equation; an unsolved
  // face passes its u-hat adjoint to the old velocity
  if (j < P.ny) {
    const bool us = i < P.nx && u_solved(P, i, j);
    const double lu = i < P.nx ? lam_u(P, ln, i, j) : 0.0;
    double luh = us ? lu : 0.0, ldu = us ? -lu * (I.pn[k] - I.pn[k - 1]) : 0.0, lru = 0.0;
    const double dyj = gy(P, 0, j);
    double pl = 0.0, pd = 0.0, ph = 0.0;
    if (i < P.nx && fl(P, i, j)) {
      const double lN = sq0[c];
      const double laW = lN * at(o.p, P, i - 1, j) * dt + sq1[c] * dt, lbW = lN * dt;
      pl += (laW * I.du[k] + lbW * I.uh[k]) * dyj;
      pd += laW * I.ru[k] * dyj;
      ph += lbW * I.ru[k] * dyj;
    }
    if (i >= 1 && fl(P, i - 1, j)) {
      const double lN = sq0[c - 1];
      const double laE = lN * at(o.p, P, i, j) * dt + sq1[c - 1] * dt, lbE = -lN * dt;
      pl += (laE * I.du[k] + lbE * I.uh[k]) * dyj;
      pd += laE * I.ru[k] * dyj;
      ph += lbE * I.ru[k] * dyj;
    }
    lru = pl;
    ldu += pd;
    luh += ph;
    A.lru[k] = lru;
    A.ldu[k] = ldu;
    A.luh[k] = luh;
    lo.u[k] = us ? 0.0 : (i < P.nx ? lu : 0.0) + luh;
  } else {
    A.luh[k] = 0.0;
    A.ldu[k] = 0.0;
    lo.u[k] = 0.0;
  }
  // v-face (i, j): the same with the south face of cell (i, j) and the
  // north face of cell (i, j-1)
  if (i < P.nx) {
    const bool vs = v_solved(P, i, j);
    const double lv = ln.v[k];
    double lvh = vs ? lv : 0.0, ldv = vs ? -lv * (I.pn[k] - I.pn[k - P.pitch]) : 0.0;
    const double dxi = gx(P, 0, i);
    double pl = 0.0, pd = 0.0, ph = 0.0;
    if (j < P.ny && fl(P, i, j)) {
      const double lN = sq0[c];
      const double laS = lN * at(o.p, P, i, j - 1) * dt + sq1[c] * dt, lbS = lN * dt;
      pl += (laS * I.dv[k] + lbS * I.vh[k]) * dxi;
      pd += laS * I.rv[k] * dxi;
      ph += lbS * I.rv[k] * dxi;
    }
    if (j >= 1 && fl(P, i, j - 1)) {
      const double lN = sq0[c - CW];
      const double laN = lN * at(o.p, P, i, j) * dt + sq1[c - CW] * dt, lbN = -lN * dt;
      pl += (laN * I.dv[k] + lbN * I.vh[k]) * dxi;
      pd += laN * I.rv[k] * dxi;
      ph += lbN * I.rv[k] * dxi;
    }
    ldv += pd;
    lvh += ph;
    A.lrv[k] = pl;
    A.ldv[k] = ldv;
    A.lvh[k] = lvh;
    lo.v[k] = vs ? 0.0 : lv + lvh;
  } else {
    A.lvh[k] = 0.0;
    A.ldv[k] = 0.0;
    lo.v[k] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// (2) energy equation of a fluid cell (explicit scheme)
// ---------------------------------------------------------------------------
template <bool SJ, class S>
__device__ void energy_item(const Params &P, const State o, const Cache cc, const State lo, const Consts C,
                            const Consts lC, const Inter I, const AdjTmp A, double *gtw0,
                            double *gtw1, int i, int j, S &sk) {
  if (i >= P.nx || j >= P.ny || !fl(P, i, j)) return;
  const long k = ix(P, i, j);
  const double l = A.ltn[k];
  if (l == 0.0) return;
  const double dxi = gx(P, 0, i), dyj = gy(P, 0, j), dV = dxi * dyj, dt = P.dt;
  const double idx = gx(P, 1, i), idy = gy(P, 1, j);
  const double gP = gam(P, cc, i, j), TP = at(o.T, P, i, j);
  const double rP = rho(P, cc, i, j);
  const bool jo = SJ && P.otype == 2;  // slip-jump obstacle surfaces
  // conductances and neighbour values (the forward's rules), with the
  // partials of each conductance in Gamma_P, Gamma_nb, the wall sqrt(T) and
  // (slip-jump surfaces) rho_P
  double nW, nE, nS, nN, DW, DE, DS, DN;
  double dWP = 0, dWn = 0, dEP = 0, dEn = 0, dSP = 0, dSn = 0, dNP = 0, dNn = 0, dSw = 0, dNw = 0;
  double dWr = 0, dEr = 0, dSr = 0, dNr = 0;
  double x;
  if (i == 0) {
    nW = P.inl[4 * (j) + 1];
    const double K = P.C1 * dyj * (2.0 * idx);
    DW = K * hmean2_d(gP, P.inl[4 * (j) + 2], dWP, x);
    dWP *= K;
  } else {
    nW = at(o.T, P, i - 1, j);
    if (!fl(P, i - 1, j) && jo) {
      DW = jwall_d(P.C1 * dyj, gP, dxi, P.kt, rP, dWP, dWr);
    } else if (!fl(P, i - 1, j)) {
      const double K = P.C1 * dyj * (2.0 * idx);
      DW = K * hmean2_d(gP, P.sq_obsT, dWP, x);
      dWP *= K;
    } else {
      const double K = P.C1 * dyj * (2.0 * gx(P, 3, i));
      DW = K * hmean_d(gx(P, 0, i - 1), gam(P, cc, i - 1, j), dxi, gP, dWn, dWP);
      dWn *= K;
      dWP *= K;
    }
  }
  if (i == P.nx - 1) {
    nE = TP;
    DE = 0.0;
  } else {
    nE = at(o.T, P, i + 1, j);
    if (!fl(P, i + 1, j) && jo) {
      DE = jwall_d(P.C1 * dyj, gP, dxi, P.kt, rP, dEP, dEr);
    } else if (!fl(P, i + 1, j)) {
      const double K = P.C1 * dyj * (2.0 * idx);
      DE = K * hmean2_d(gP, P.sq_obsT, dEP, x);
      dEP *= K;
    } else {
      const double K = P.C1 * dyj * (2.0 * gx(P, 3, i + 1));
      DE = K * hmean_d(dxi, gP, gx(P, 0, i + 1), gam(P, cc, i + 1, j), dEP, dEn);
      dEP *= K;
      dEn *= K;
    }
  }
  if (j == 0) {
    if (P.wtype0 == 0) {
      nS = P.wl[4 * (i)];
      const double K = P.C1 * dxi * (2.0 * idy);
      DS = K * hmean2_d(gP, P.wl[4 * (i) + 2], dSP, dSw);
      dSP *= K;
      dSw *= K;
    } else if (SJ && P.wtype0 == 2) {
      nS = P.wl[4 * (i)];
      DS = jwall_d(P.C1 * dxi, gP, dyj, P.kt, rP, dSP, dSr);
    } else {
      nS = TP;
      DS = 0.0;
    }
  } else {
    nS = at(o.T, P, i, j - 1);
    if (!fl(P, i, j - 1) && jo) {
      DS = jwall_d(P.C1 * dxi, gP, dyj, P.kt, rP, dSP, dSr);
    } else if (!fl(P, i, j - 1)) {
      const double K = P.C1 * dxi * (2.0 * idy);
      DS = K * hmean2_d(gP, P.sq_obsT, dSP, x);
      dSP *= K;
    } else {
      const double K = P.C1 * dxi * (2.0 * gy(P, 3, j));
      DS = K * hmean_d(gy(P, 0, j - 1), gam(P, cc, i, j - 1), dyj, gP, dSn, dSP);
      dSn *= K;
      dSP *= K;
    }
  }
  if (j == P.ny - 1) {
    if (P.wtype1 == 0) {
      nN = P.wl[4 * (i) + 1];
      const double K = P.C1 * dxi * (2.0 * idy);
      DN = K * hmean2_d(gP, P.wl[4 * (i) + 3], dNP, dNw);
      dNP *= K;
      dNw *= K;
    } else if (SJ && P.wtype1 == 2) {
      nN = P.wl[4 * (i) + 1];
      DN = jwall_d(P.C1 * dxi, gP, dyj, P.kt, rP, dNP, dNr);
    } else {
      nN = TP;
      DN = 0.0;
    }
  } else {
    nN = at(o.T, P, i, j + 1);
    if (!fl(P, i, j + 1) && jo) {
      DN = jwall_d(P.C1 * dxi, gP, dyj, P.kt, rP, dNP, dNr);
    } else if (!fl(P, i, j + 1)) {
      const double K = P.C1 * dxi * (2.0 * idy);
      DN = K * hmean2_d(gP, P.sq_obsT, dNP, x);
      dNP *= K;
    } else {
      const double K = P.C1 * dxi * (2.0 * gy(P, 3, j + 1));
      DN = K * hmean_d(dyj, gP, gy(P, 0, j + 1), gam(P, cc, i, j + 1), dNP, dNn);
      dNP *= K;
      dNn *= K;
    }
  }
  const double a0 = dt * (DW + DE + DS + DN) + rP * dV;
  const double tn = I.tn[k];
  // T = (dt (sum D n + Sc) + C_T) / a0
  const double lnum = l / a0, la0 = -l * tn / a0;
  lC.CT[k] += lnum;
  sk.add(4, P, i, j, la0 * dV);  // rho_P (u-hat, v-hat and the face densities add to it too)
  const double lDW = lnum * dt * nW + la0 * dt, lDE = lnum * dt * nE + la0 * dt;
  const double lDS = lnum * dt * nS + la0 * dt, lDN = lnum * dt * nN + la0 * dt;
  double lgP = lDW * dWP + lDE * dEP + lDS * dSP + lDN * dNP;
  double lrw = lDW * dWr + lDE * dEr + lDS * dSr + lDN * dNr;  // more of rho_P's adjoint
  if (i > 0) {
    sk.add(0, P, i - 1, j, lnum * dt * DW);
    if (dWn != 0.0) sk.add(1, P, i - 1, j, lDW * dWn);
  }
  if (i == P.nx - 1) sk.add(0, P, i, j, lnum * dt * DE);
  else {
    sk.add(0, P, i + 1, j, lnum * dt * DE);
    if (dEn != 0.0) sk.add(1, P, i + 1, j, lDE * dEn);
  }
  if (j == 0) {
    if (P.wtype0 == 0) {
      unsafeAtomicAdd(gtw0 + i, lnum * dt * DS + lDS * dSw / (2.0 * P.wl[4 * (i) + 2]));
    } else if (SJ && P.wtype0 == 2) {
      unsafeAtomicAdd(gtw0 + i, lnum * dt * DS);
    } else {
      sk.add(0, P, i, j, lnum * dt * DS);
    }
  } else {
    sk.add(0, P, i, j - 1, lnum * dt * DS);
    if (dSn != 0.0) sk.add(1, P, i, j - 1, lDS * dSn);
  }
  if (j == P.ny - 1) {
    if (P.wtype1 == 0) {
      unsafeAtomicAdd(gtw1 + i, lnum * dt * DN + lDN * dNw / (2.0 * P.wl[4 * (i) + 3]));
    } else if (SJ && P.wtype1 == 2) {
      unsafeAtomicAdd(gtw1 + i, lnum * dt * DN);
    } else {
      sk.add(0, P, i, j, lnum * dt * DN);
    }
  } else {
    sk.add(0, P, i, j + 1, lnum * dt * DN);
    if (dNn != 0.0) sk.add(1, P, i, j + 1, lDN * dNn);
  }
  // source: dissipation and pressure work
  const double lSc = lnum * dt;
  const double U0 = at(o.u, P, i, j), U1 = at(o.u, P, i + 1, j);
  const double V0 = at(o.v, P, i, j), V1 = at(o.v, P, i, j + 1);
  const double vc = 0.5 * (V0 + V1), uc = 0.5 * (U0 + U1);
  double vE, vW, uN, uS;
  // 0 constant, 1 vc/uc, 2 interpolated, 3 slip velocity (partials s* in
  // vc/uc and r* in rho_P)
  int cvE = 0, cvW = 0, cuN = 0, cuS = 0;
  double svE = 0, svW = 0, suN = 0, suS = 0, rvE = 0, rvW = 0, ruN = 0, ruS = 0;
  if (i == P.nx - 1) { vE = vc; cvE = 1; }
  else if (!fl(P, i + 1, j) && jo) { vE = slip_d(0.0, vc, dxi, P.kz, rP, svE, rvE); cvE = 3; }
  else if (!fl(P, i + 1, j)) vE = 0.0;
  else {
    vE = gx(P, 4, i + 1) * vc + gx(P, 5, i + 1) * (0.5 * (at(o.v, P, i + 1, j) + at(o.v, P, i + 1, j + 1)));
    cvE = 2;
  }
  if (i > 0 && !fl(P, i - 1, j) && jo) { vW = slip_d(0.0, vc, dxi, P.kz, rP, svW, rvW); cvW = 3; }
  else if (i == 0 || !fl(P, i - 1, j)) vW = 0.0;
  else {
    vW = gx(P, 4, i) * (0.5 * (at(o.v, P, i - 1, j) + at(o.v, P, i - 1, j + 1))) + gx(P, 5, i) * vc;
    cvW = 2;
  }
  if (j == P.ny - 1) {
    if (P.wtype1 == 0) uN = P.wu1;
    else if (SJ && P.wtype1 == 2) { uN = slip_d(P.wu1, uc, dyj, P.kz, rP, suN, ruN); cuN = 3; }
    else { uN = uc; cuN = 1; }
  } else if (!fl(P, i, j + 1) && jo) { uN = slip_d(0.0, uc, dyj, P.kz, rP, suN, ruN); cuN = 3; }
  else if (!fl(P, i, j + 1)) uN = 0.0;
  else {
    uN = gy(P, 4, j + 1) * uc + gy(P, 5, j + 1) * (0.5 * (at(o.u, P, i, j + 1) + at(o.u, P, i + 1, j + 1)));
    cuN = 2;
  }
  if (j == 0) {
    if (P.wtype0 == 0) uS = P.wu0;
    else if (SJ && P.wtype0 == 2) { uS = slip_d(P.wu0, uc, dyj, P.kz, rP, suS, ruS); cuS = 3; }
    else { uS = uc; cuS = 1; }
  } else if (!fl(P, i, j - 1) && jo) { uS = slip_d(0.0, uc, dyj, P.kz, rP, suS, ruS); cuS = 3; }
  else if (!fl(P, i, j - 1)) uS = 0.0;
  else {
    uS = gy(P, 4, j) * (0.5 * (at(o.u, P, i, j - 1) + at(o.u, P, i + 1, j - 1))) + gy(P, 5, j) * uc;
    cuS = 2;
  }
  const double ux = (U1 - U0) * idx, vy = (V1 - V0) * idy;
  const double vx = (vE - vW) * idx, uy = (uN - uS) * idy, dv = ux + vy;
  const double S1 = 2.0 * (ux * ux + vy * vy) + (vx + uy) * (vx + uy) - 2.0 / 3.0 * dv * dv;
  const double pP = at(o.p, P, i, j);
  lgP += lSc * P.C2 * S1 * dV;
  sk.add(5, P, i, j, lSc * P.C3 * dv * dV);  // p_P
  const double lS1 = lSc * P.C2 * gP * dV;
  const double ldv = lSc * P.C3 * pP * dV - lS1 * (4.0 / 3.0) * dv;
  const double lux = lS1 * 4.0 * ux + ldv, lvy = lS1 * 4.0 * vy + ldv;
  const double lvx = lS1 * 2.0 * (vx + uy), luy = lvx;
  double lU0 = -lux * idx, lU1 = lux * idx, lV0 = -lvy * idy, lV1 = lvy * idy;
  const double lvE = lvx * idx, lvW = -lvx * idx, luN = luy * idy, luS = -luy * idy;
  double lvc = 0.0, luc = 0.0;
  if (cvE == 3) { lvc += lvE * svE; lrw += lvE * rvE; }
  if (cvW == 3) { lvc += lvW * svW; lrw += lvW * rvW; }
  if (cuN == 3) { luc += luN * suN; lrw += luN * ruN; }
  if (cuS == 3) { luc += luS * suS; lrw += luS * ruS; }
  if (cvE == 1) lvc += lvE;
  else if (cvE == 2) {
    lvc += lvE * gx(P, 4, i + 1);
    const double q = lvE * gx(P, 5, i + 1) * 0.5;
    sk.add(3, P, i + 1, j, q);
    sk.add(3, P, i + 1, j + 1, q);
  }
  if (cvW == 2) {
    const double q = lvW * gx(P, 4, i) * 0.5;
    sk.add(3, P, i - 1, j, q);
    sk.add(3, P, i - 1, j + 1, q);
    lvc += lvW * gx(P, 5, i);
  }
  if (cuN == 1) luc += luN;
  else if (cuN == 2) {
    luc += luN * gy(P, 4, j + 1);
    const double q = luN * gy(P, 5, j + 1) * 0.5;
    sk.add(2, P, i, j + 1, q);
    sk.add(2, P, i + 1, j + 1, q);
  }
  if (cuS == 1) luc += luS;
  else if (cuS == 2) {
    const double q = luS * gy(P, 4, j) * 0.5;
    sk.add(2, P, i, j - 1, q);
    sk.add(2, P, i + 1, j - 1, q);
    luc += luS * gy(P, 5, j);
  }
  lV0 += 0.5 * lvc;
  lV1 += 0.5 * lvc;
  lU0 += 0.5 * luc;
  lU1 += 0.5 * luc;
  sk.add(2, P, i, j, lU0);
  sk.add(2, P, i + 1, j, lU1);
  sk.add(3, P, i, j, lV0);
  sk.add(3, P, i, j + 1, lV1);
  sk.add(1, P, i, j, lgP);
  if (lrw != 0.0) sk.add(4, P, i, j, lrw);
}

// ---------------------------------------------------------------------------
// (2) u-hat, d^u of a solved u-face (explicit scheme)
// ---------------------------------------------------------------------------
template <bool SJ, class S>
__device__ void uhat_item(const Params &P, const State o, const Cache cc, const State lo, const Consts C,
                          const Consts lC, const Inter I, const AdjTmp A, double *gtw0,
                          double *gtw1, int i, int j, S &sk) {
  if (j >= P.ny || !u_solved(P, i, j)) return;
  const long k = ix(P, i, j);
  const double luh = A.luh[k], ldu = A.ldu[k];
  if (luh == 0.0 && ldu == 0.0) return;
  const double B = P.B;
  const double dxl = gx(P, 0, i - 1), dxr = gx(P, 0, i), dyj = gy(P, 0, j), idy = gy(P, 1, j);
  const double gl = gam(P, cc, i - 1, j), gr = gam(P, cc, i, j);
  const double uP = at(o.u, P, i, j), uW = at(o.u, P, i - 1, j), uE = at(o.u, P, i + 1, j);
  const double len = 0.5 * (dxl + dxr);
  const double gnode = gx(P, 4, i) * gl + gx(P, 5, i) * gr;
  // slip surfaces: the node density interpolated like gnode
  const double rnode = gx(P, 4, i) * rho(P, cc, i - 1, j) + gx(P, 5, i) * rho(P, cc, i, j);
  double uS, uN, DS, DN;
  // kS, kN: 0 wall (constant u), 1 uP, 2 neighbour; D kinds dS, dN: 0 none,
  // 1 wall, 2 obstacle, 3 corner, 4 slip wall or obstacle (partials jSg,
  // jNg in gnode and jSr, jNr in rnode)
  int kS, kN;
  int dS, dN;
  double jSg = 0, jSr = 0, jNg = 0, jNr = 0;
  if (j == 0) {
    if (P.wtype0 == 0) {
      uS = P.wu0; kS = 0; dS = 1;
      DS = B * 0.5 * (gnode + P.wu[2 * (i)]) * len * (2.0 * idy);
    } else if (SJ && P.wtype0 == 2) {
      uS = P.wu0; kS = 0; dS = 4;
      DS = jwall_d(B * len, gnode, dyj, P.kz, rnode, jSg, jSr);
    } else { uS = uP; kS = 1; dS = 0; DS = 0.0; }
  } else {
    uS = at(o.u, P, i, j - 1); kS = 2;
    if (!fl(P, i - 1, j - 1) && !fl(P, i, j - 1) && SJ && P.otype == 2) {
      dS = 4; DS = jwall_d(B * len, gnode, dyj, P.kz, rnode, jSg, jSr);
    } else if (!fl(P, i - 1, j - 1) && !fl(P, i, j - 1)) {
      dS = 2; DS = B * 0.5 * (gnode + P.sq_obsT) * len * (2.0 * idy);
    } else {
      dS = 3; DS = B * gamc(P, cc, i, j) * gx(P, 2, i) * gy(P, 3, j);
    }
  }
  if (j == P.ny - 1) {
    if (P.wtype1 == 0) {
      uN = P.wu1; kN = 0; dN = 1;
      DN = B * 0.5 * (gnode + P.wu[2 * (i) + 1]) * len * (2.0 * idy);
    } else if (SJ && P.wtype1 == 2) {
      uN = P.wu1; kN = 0; dN = 4;
      DN = jwall_d(B * len, gnode, dyj, P.kz, rnode, jNg, jNr);
    } else { uN = uP; kN = 1; dN = 0; DN = 0.0; }
  } else {
    uN = at(o.u, P, i, j + 1); kN = 2;
    if (!fl(P, i - 1, j + 1) && !fl(P, i, j + 1) && SJ && P.otype == 2) {
      dN = 4; DN = jwall_d(B * len, gnode, dyj, P.kz, rnode, jNg, jNr);
    } else if (!fl(P, i - 1, j + 1) && !fl(P, i, j + 1)) {
      dN = 2; DN = B * 0.5 * (gnode + P.sq_obsT) * len * (2.0 * idy);
    } else {
      dN = 3; DN = B * gamc(P, cc, i, j + 1) * gx(P, 2, i) * gy(P, 3, j + 1);
    }
  }
  const double DW = B * gl * dyj * gx(P, 1, i - 1), DE = B * gr * dyj * gx(P, 1, i);
  const double aS = DS, aN = DN, aW = 4.0 / 3.0 * DW, aE = 4.0 / 3.0 * DE;
  const double M = (rho(P, cc, i, j) * dxr + rho(P, cc, i - 1, j) * dxl) * dyj / 2.0;
  const double a0 = aS + aN + aW + aE + 0.0 + M * P.idt;
  const double gcN = gamc(P, cc, i, j + 1), gcS = gamc(P, cc, i, j);
  const double v00 = at(o.v, P, i - 1, j), v10 = at(o.v, P, i, j);
  const double v01 = at(o.v, P, i - 1, j + 1), v11 = at(o.v, P, i, j + 1);
  const double X = gcN * (v11 - v01) - gcS * (v10 - v00) - 2.0 / 3.0 * gr * (v11 - v10) +
                   2.0 / 3.0 * gl * (v01 - v00);
  const double b = C.Cu[k] + B * X;
  const double num = aS * uS + aN * uN + aW * uW + aE * uE + b;
  const double uh = num / a0, du = P.A * dyj / a0;
  const double lnum = luh / a0, la0 = -(luh * uh + ldu * du) / a0;
  lC.Cu[k] += lnum;
  // neighbour values
  sk.add(0, P, i - 1, j, lnum * aW);
  sk.add(0, P, i + 1, j, lnum * aE);
  double lself = 0.0;
  if (kS == 1) lself += lnum * aS;
  else if (kS == 2) sk.add(0, P, i, j - 1, lnum * aS);
  if (kN == 1) lself += lnum * aN;
  else if (kN == 2) sk.add(0, P, i, j + 1, lnum * aN);
  if (lself != 0.0) sk.add(0, P, i, j, lself);
  // coefficients
  const double laS = lnum * uS + la0, laN = lnum * uN + la0;
  const double laW = lnum * uW + la0, laE = lnum * uE + la0;
  double lgl = laW * 4.0 / 3.0 * B * dyj * gx(P, 1, i - 1);
  double lgr = laE * 4.0 / 3.0 * B * dyj * gx(P, 1, i);
  double lgn = 0.0, lrn = 0.0;  // adjoints of gnode, rnode
  double lgcS = 0.0, lgcN = 0.0;
  if (dS == 1) {
    const double q = laS * B * 0.5 * len * (2.0 * idy);
    lgn += q;
    sqtwu_adj(P, 0, gtw0, i, q);
  } else if (dS == 2) lgn += laS * B * 0.5 * len * (2.0 * idy);
  else if (dS == 3) lgcS += laS * B * gx(P, 2, i) * gy(P, 3, j);
  else if (dS == 4) { lgn += laS * jSg; lrn += laS * jSr; }
  if (dN == 1) {
    const double q = laN * B * 0.5 * len * (2.0 * idy);
    lgn += q;
    sqtwu_adj(P, 1, gtw1, i, q);
  } else if (dN == 2) lgn += laN * B * 0.5 * len * (2.0 * idy);
  else if (dN == 3) lgcN += laN * B * gx(P, 2, i) * gy(P, 3, j + 1);
  else if (dN == 4) { lgn += laN * jNg; lrn += laN * jNr; }
  lgl += lgn * gx(P, 4, i);
  lgr += lgn * gx(P, 5, i);
  // M = (rho_P dxr + rho_W dxl) dy / 2
  const double lM = la0 * P.idt;
  sk.add(2, P, i, j, lM * dxr * dyj / 2.0 + lrn * gx(P, 5, i));
  sk.add(2, P, i - 1, j, lM * dxl * dyj / 2.0 + lrn * gx(P, 4, i));
  // cross-diffusion X
  const double lX = lnum * B;
  lgcN += lX * (v11 - v01);
  lgcS += -lX * (v10 - v00);
  lgr += -lX * 2.0 / 3.0 * (v11 - v10);
  lgl += lX * 2.0 / 3.0 * (v01 - v00);
  sk.add(1, P, i, j + 1, lX * (gcN - 2.0 / 3.0 * gr));
  sk.add(1, P, i - 1, j + 1, lX * (-gcN + 2.0 / 3.0 * gl));
  sk.add(1, P, i, j, lX * (-gcS + 2.0 / 3.0 * gr));
  sk.add(1, P, i - 1, j, lX * (gcS - 2.0 / 3.0 * gl));
  gamc_adj(sk, 3, P, i, j, lgcS);
  gamc_adj(sk, 3, P, i, j + 1, lgcN);
  sk.add(3, P, i - 1, j, lgl);
  sk.add(3, P, i, j, lgr);
}

// ---------------------------------------------------------------------------
// (2) v-hat, d^v of a solved v-face (explicit scheme)
// ---------------------------------------------------------------------------
template <bool SJ, class S>
__device__ void vhat_item(const Params &P, const State o, const Cache cc, const State lo, const Consts C,
                          const Consts lC, const Inter I, const AdjTmp A, int i, int j, S &sk) {
  if (i >= P.nx || !v_solved(P, i, j)) return;
  const long k = ix(P, i, j);
  const double lvh = A.lvh[k], ldv = A.ldv[k];
  if (lvh == 0.0 && ldv == 0.0) return;
  const double B = P.B;
  const double dxi = gx(P, 0, i), dys = gy(P, 0, j - 1), dyn = gy(P, 0, j), idx = gx(P, 1, i);
  const double gs = gam(P, cc, i, j - 1), gn = gam(P, cc, i, j);
  const double vP = at(o.v, P, i, j), vS = at(o.v, P, i, j - 1), vN = at(o.v, P, i, j + 1);
  const bool inl = i == 0, outl = i == P.nx - 1;
  const double vW = inl ? 0.0 : at(o.v, P, i - 1, j);
  const double vE = outl ? vP : at(o.v, P, i + 1, j);
  const double len = 0.5 * (dys + dyn);
  const double gnode = gy(P, 4, j) * gs + gy(P, 5, j) * gn;
  const double gcW = gamc(P, cc, i, j), gcE = gamc(P, cc, i + 1, j);
  const double rnode = gy(P, 4, j) * rho(P, cc, i, j - 1) + gy(P, 5, j) * rho(P, cc, i, j);
  double DW, DE;
  // 1 inlet, 2 obstacle, 3 corner, 4 slip obstacle (partials j*g in gnode,
  // j*r in rnode); 0 none
  int dW, dE;
  double jWg = 0, jWr = 0, jEg = 0, jEr = 0;
  const bool so = SJ && P.otype == 2;
  if (inl) { dW = 1; DW = B * 0.5 * (gnode + gcW) * len * (2.0 * idx); }
  else if (!fl(P, i - 1, j - 1) && !fl(P, i - 1, j) && so) {
    dW = 4; DW = jwall_d(B * len, gnode, dxi, P.kz, rnode, jWg, jWr);
  } else if (!fl(P, i - 1, j - 1) && !fl(P, i - 1, j)) {
    dW = 2; DW = B * 0.5 * (gnode + P.sq_obsT) * len * (2.0 * idx);
  } else { dW = 3; DW = B * gcW * gy(P, 2, j) * gx(P, 3, i); }
  if (outl) { dE = 0; DE = 0.0; }
  else if (!fl(P, i + 1, j - 1) && !fl(P, i + 1, j) && so) {
    dE = 4; DE = jwall_d(B * len, gnode, dxi, P.kz, rnode, jEg, jEr);
  } else if (!fl(P, i + 1, j - 1) && !fl(P, i + 1, j)) {
    dE = 2; DE = B * 0.5 * (gnode + P.sq_obsT) * len * (2.0 * idx);
  } else { dE = 3; DE = B * gcE * gy(P, 2, j) * gx(P, 3, i + 1); }
  const double DS = B * gs * dxi * gy(P, 1, j - 1), DN = B * gn * dxi * gy(P, 1, j);
  const double aW = DW, aE = DE, aS = 4.0 / 3.0 * DS, aN = 4.0 / 3.0 * DN;
  const double M = (rho(P, cc, i, j) * dyn + rho(P, cc, i, j - 1) * dys) * dxi / 2.0;
  const double a0 = aW + aE + aS + aN + 0.0 + M * P.idt;
  const double u00 = at(o.u, P, i, j - 1), u10 = at(o.u, P, i + 1, j - 1);
  const double u01 = at(o.u, P, i, j), u11 = at(o.u, P, i + 1, j);
  const double X = gcE * (u11 - u10) - gcW * (u01 - u00) - 2.0 / 3.0 * gn * (u11 - u01) +
                   2.0 / 3.0 * gs * (u10 - u00);
  const double b = C.Cv[k] + B * X;
  const double num = aW * vW + aE * vE + aS * vS + aN * vN + b;
  const double vh = num / a0, dv = P.A * dxi / a0;
  const double lnum = lvh / a0, la0 = -(lvh * vh + ldv * dv) / a0;
  lC.Cv[k] += lnum;
  if (!inl) sk.add(1, P, i - 1, j, lnum * aW);
  if (outl) sk.add(1, P, i, j, lnum * aE);
  else sk.add(1, P, i + 1, j, lnum * aE);
  sk.add(1, P, i, j - 1, lnum * aS);
  sk.add(1, P, i, j + 1, lnum * aN);
  const double laW = lnum * vW + la0, laE = lnum * vE + la0;
  const double laS = lnum * vS + la0, laN = lnum * vN + la0;
  double lgs = laS * 4.0 / 3.0 * B * dxi * gy(P, 1, j - 1);
  double lgn_ = laN * 4.0 / 3.0 * B * dxi * gy(P, 1, j);
  double lgnode = 0.0, lgcW = 0.0, lgcE = 0.0, lrn = 0.0;
  if (dW == 1) {
    const double q = laW * B * 0.5 * len * (2.0 * idx);
    lgnode += q;
    lgcW += q;
  } else if (dW == 2) lgnode += laW * B * 0.5 * len * (2.0 * idx);
  else if (dW == 3) lgcW += laW * B * gy(P, 2, j) * gx(P, 3, i);
  else { lgnode += laW * jWg; lrn += laW * jWr; }
  if (dE == 2) lgnode += laE * B * 0.5 * len * (2.0 * idx);
  else if (dE == 3) lgcE += laE * B * gy(P, 2, j) * gx(P, 3, i + 1);
  else if (dE == 4) { lgnode += laE * jEg; lrn += laE * jEr; }
  lgs += lgnode * gy(P, 4, j);
  lgn_ += lgnode * gy(P, 5, j);
  const double lM = la0 * P.idt;
  sk.add(2, P, i, j, lM * dyn * dxi / 2.0 + lrn * gy(P, 5, j));
  sk.add(2, P, i, j - 1, lM * dys * dxi / 2.0 + lrn * gy(P, 4, j));
  const double lX = lnum * B;
  lgcE += lX * (u11 - u10);
  lgcW += -lX * (u01 - u00);
  lgn_ += -lX * 2.0 / 3.0 * (u11 - u01);
  lgs += lX * 2.0 / 3.0 * (u10 - u00);
  sk.add(0, P, i + 1, j, lX * (gcE - 2.0 / 3.0 * gn));
  sk.add(0, P, i + 1, j - 1, lX * (-gcE + 2.0 / 3.0 * gs));
  sk.add(0, P, i, j, lX * (-gcW + 2.0 / 3.0 * gn));
  sk.add(0, P, i, j - 1, lX * (gcW - 2.0 / 3.0 * gs));
  gamc_adj(sk, 3, P, i, j, lgcW);
  gamc_adj(sk, 3, P, i + 1, j, lgcE);
  sk.add(3, P, i, j - 1, lgs);
  sk.add(3, P, i, j, lgn_);
}

// ---------------------------------------------------------------------------
// (1) face densities (upwind value + TVD correction x jump)
// ---------------------------------------------------------------------------
template <bool TV, class S>
__device__ void rho_faces_item(const Params &P, const State &o, const Cache cc, const double *lru,
                               const double *lrv, int i, int j, S &sk) {
  if (j < P.ny) {  // u-face
    const double l = lru[ix(P, i, j)];
    if (l != 0.0) {
      const double uf = at(o.u, P, i, j);
      if (i == 0) {
        if (!(uf > 0.0)) sk.add(0, P, 0, j, l);
      } else if (i == P.nx) {
        sk.add(0, P, P.nx - 1, j, l);
      } else {
        sk.add(0, P, uf > 0.0 ? i - 1 : i, j, l);
        if (TV && fl(P, i - 2, j) && fl(P, i - 1, j) && fl(P, i, j) && fl(P, i + 1, j)) {
          const double r1 = rho(P, cc, i - 2, j), rl = rho(P, cc, i - 1, j);
          const double rr = rho(P, cc, i, j), r4 = rho(P, cc, i + 1, j);
          double g[4];
          const double ps = psix_d(P, r1, rl, rr, r4, i, uf, g);
          const double lj = l * (rr - rl);
          sk.add(0, P, i - 2, j, lj * g[0]);
          sk.add(0, P, i - 1, j, lj * g[1] - l * ps);
          sk.add(0, P, i, j, lj * g[2] + l * ps);
          sk.add(0, P, i + 1, j, lj * g[3]);
        }
      }
    }
  }
  if (i < P.nx) {  // v-face
    const double l = lrv[ix(P, i, j)];
    if (l != 0.0) {
      if (j == 0) sk.add(0, P, i, 0, l);
      else if (j == P.ny) sk.add(0, P, i, P.ny - 1, l);
      else {
        const double vf = at(o.v, P, i, j);
        sk.add(0, P, i, vf > 0.0 ? j - 1 : j, l);
        if (TV && fl(P, i, j - 2) && fl(P, i, j - 1) && fl(P, i, j) && fl(P, i, j + 1)) {
          const double r1 = rho(P, cc, i, j - 2), rs = rho(P, cc, i, j - 1);
          const double rn = rho(P, cc, i, j), r4 = rho(P, cc, i, j + 1);
          double g[4];
          const double ps = psiy_d(P, r1, rs, rn, r4, j, vf, g);
          const double lj = l * (rn - rs);
          sk.add(0, P, i, j - 2, lj * g[0]);
          sk.add(0, P, i, j - 1, lj * g[1] - l * ps);
          sk.add(0, P, i, j, lj * g[2] + l * ps);
          sk.add(0, P, i, j + 1, lj * g[3]);
        }
      }
    }
  }
}

template <bool TV>
__global__ __launch_bounds__(AB) void k_adj_rho_faces(const Params P, const State o,
                                                      const Cache cc, const double *lru,
                                                      const double *lrv, double *lr) {
  __shared__ double wl[Tiled<1, 2>::WN];
  Tiled<1, 2> sk{(lds_double *)wl, {lr}};
  int i, j;
  sk.begin(P, i, j);
  if (i <= P.nx && j <= P.ny) rho_faces_item<TV>(P, o, cc, lru, lrv, i, j, sk);
  sk.end(P);
}


// Slot adapter: an item's slot s goes to slot S<s> of a window shared by
// several items.
template <class T, int S0, int S1 = 0, int S2 = 0, int S3 = 0, int S4 = 0, int S5 = 0>
struct Slots {
  T &t;
  __device__ __forceinline__ void add(int s, const Params &P, int i, int j, double x) {
    t.add(s == 0 ? S0 : (s == 1 ? S1 : (s == 2 ? S2 : (s == 3 ? S3 : (s == 4 ? S4 : S5)))), P, i,
          j, x);
  }
};

// The energy, u-hat, v-hat and face-density stages read disjoint adjoint
// inputs and add into shared targets.  A block runs the four stages of its
// tile one after the other into one window of the six target arrays and
// flushes it once: the global atomic adds of the flush take most of these
// stages' time, and one flush for the four halves them (against four
// windows, whether the stages run as four launches or side by side in one).
// The flush also takes the rho and Gamma adjoints of each domain cell back
// to p and T (rho = p/T, Gamma = sqrt(T) of the iterate), so they reach
// global memory only as parts of the p and T adjoints (the frame's stand for
// boundary values and are dropped).  Every scatter of these stages lies
// within two elements of its item, inside the window, and reaches global
// memory only through the flush's atomic adds.
// SJ: the problem has slip-jump surfaces (their branches are compiled only
// into these instances, which keeps the others' registers as without them).
// The others fit 5 waves per SIMD (91 VGPRs; 3.5 % shorter backward on
// 4096x1024 than at 4); the slip-jump ones would spill there and keep 4.
template <bool TV, bool SJ>
__global__ __launch_bounds__(AB) __attribute__((amdgpu_waves_per_eu(SJ ? 4 : 5))) void k_adj_stage2(const Params P, const State o,
                                                   const State lo, const Consts C,
                                                   const Consts lC, const Inter I,
                                                   const AdjTmp A, double *gtw0, double *gtw1) {
  using W = Tiled<6, 2, false>;
  __shared__ double wl[6 * W::WN];
  const Cache cc{A.cr, A.cg};
  W sk{(lds_double *)wl, {lo.T, lo.u, lo.v, A.lr, A.lg, lo.p}};
  int i, j;
  sk.begin(P, i, j);
  if (i <= P.nx && j <= P.ny) {
    Slots<W, 0, 4, 1, 2, 3, 5> se{sk};  // energy: T, Gamma, u, v, rho, p
    energy_item<SJ>(P, o, cc, lo, C, lC, I, A, gtw0, gtw1, i, j, se);
    Slots<W, 1, 2, 3, 4> sq{sk};  // u-hat, v-hat: u, v, rho, Gamma
    uhat_item<SJ>(P, o, cc, lo, C, lC, I, A, gtw0, gtw1, i, j, sq);
    vhat_item<SJ>(P, o, cc, lo, C, lC, I, A, i, j, sq);
    Slots<W, 3> sr{sk};  // face densities: rho
    rho_faces_item<TV>(P, o, cc, A.lru, A.lrv, i, j, sr);
  }
  __syncthreads();
  for (int r = threadIdx.x; r < W::WN; r += AB) {
    const double du = wl[W::WN + r], dv = wl[2 * W::WN + r];
    const double lr = wl[3 * W::WN + r], lg = wl[4 * W::WN + r];
    double dT = wl[r], dp = wl[5 * W::WN + r];
    const int gi = sk.x0 - 2 + r % W::WW, gj = sk.y0 - 2 + r / W::WW;
    const long k = ix(P, gi, gj);
    if (du != 0.0) unsafeAtomicAdd(lo.u + k, du);
    if (dv != 0.0) unsafeAtomicAdd(lo.v + k, dv);
    if ((lr != 0.0 || lg != 0.0) && gi >= 0 && gi < P.nx && gj >= 0 && gj < P.ny) {
      const double p = o.p[k], T = o.T[k];
      dp += lr / T;
      dT += -lr * p / (T * T) + lg / (2.0 * sqrt(T));
    }
    if (dp != 0.0) unsafeAtomicAdd(lo.p + k, dp);
    if (dT != 0.0) unsafeAtomicAdd(lo.T + k, dT);
  }
}

// ---------------------------------------------------------------------------
// (0) rho = p / T and Gamma = sqrt(T) per cell: the rho and Gamma adjoints
// back to p and T (the reverse of the prologue; the passes do this in the
// stage-2 flush)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(AB) void k_adj_cell_props(const Params P, const State o,
                                                       const State lo, const double *lr,
                                                       const double *lg) {
  int i, j;
  if (!elem(P, i, j) || i >= P.nx || j >= P.ny) return;
  const long k = ix(P, i, j);
  if (lr[k] == 0.0 && lg[k] == 0.0) return;
  const double p = o.p[k], T = o.T[k];
  lo.p[k] += lr[k] / T;
  lo.T[k] += -lr[k] * p / (T * T) + lg[k] / (2.0 * sqrt(T));
}

// ---------------------------------------------------------------------------
// prologue: C_T = rho T dV + dt T^exp, C_p = rho dV, C_u = M u / dt + g_x M +
// u^exp, C_v likewise (explicit convective terms with the face densities of
// the level n-1 fields, ru0 / rv0)
// ---------------------------------------------------------------------------
template <bool TV, class SK>
__device__ __forceinline__ void prologue_item(const Params &P, const State &m, const Consts &lC,
                                              const double *ru0, const double *rv0, int i, int j,
                                              SK &sk) {
  const double dt = P.dt;
  // ---- cell constants
  if (i < P.nx && j < P.ny && fl(P, i, j)) {
    const long k = ix(P, i, j);
    const double lCT = lC.CT[k], lCp = lC.Cp[k];
    const double dxi = gx(P, 0, i), dyj = gy(P, 0, j), dV = dxi * dyj;
    const double TP = m.T[k], rP = rho(P, m, i, j);
    sk.add(3, P, i, j, lCT * TP * dV + lCp * dV);
    double lTP = lCT * rP * dV;
    const double lt = lCT * dt;  // adjoint of T^exp
    if (lt != 0.0) {
      const bool inl = i == 0, outl = i == P.nx - 1, bot = j == 0, top = j == P.ny - 1;
      const double TW = inl ? P.inl[4 * (j) + 1] : at(m.T, P, i - 1, j);
      const double TE = outl ? TP : at(m.T, P, i + 1, j);
      const double TS = bot ? TP : at(m.T, P, i, j - 1);
      const double TN = top ? TP : at(m.T, P, i, j + 1);
      const double uW = at(m.u, P, i, j), uE = at(m.u, P, i + 1, j);
      const double vS = at(m.v, P, i, j), vN = at(m.v, P, i, j + 1);
      const double rW = ru0[k], rE = ru0[k + 1], rS = rv0[k], rN = rv0[k + P.pitch];
      const double FW = rW * uW * dyj, FE = rE * uE * dyj, FS = rS * vS * dxi, FN = rN * vN * dxi;
      double gE[4] = {0, 0, 0, 0}, gW[4] = {0, 0, 0, 0}, gN[4] = {0, 0, 0, 0}, gS[4] = {0, 0, 0, 0};
      double pE = 0, pW = 0, pN = 0, pS = 0;
      bool tE = false, tW = false, tN = false, tS = false;
      if (TV) {
        tE = fl(P, i - 1, j) && fl(P, i + 1, j) && fl(P, i + 2, j);
        tW = fl(P, i - 2, j) && fl(P, i - 1, j) && fl(P, i + 1, j);
        tN = fl(P, i, j - 1) && fl(P, i, j + 1) && fl(P, i, j + 2);
        tS = fl(P, i, j - 2) && fl(P, i, j - 1) && fl(P, i, j + 1);
        if (tE) pE = psix_d(P, at(m.T, P, i - 1, j), TP, TE, at(m.T, P, i + 2, j), i + 1, uE, gE);
        if (tW) pW = psix_d(P, at(m.T, P, i - 2, j), TW, TP, TE, i, uW, gW);
        if (tN) pN = psiy_d(P, at(m.T, P, i, j - 1), TP, TN, at(m.T, P, i, j + 2), j + 1, vN, gN);
        if (tS) pS = psiy_d(P, at(m.T, P, i, j - 2), TS, TP, TN, j, vS, gS);
      }
      // T^exp = -FE phiE + FW phiW - FN phiN + FS phiS
      const double phE = upw(TP, TE, uE) + (TE - TP) * pE;
      const double phW = upw(TW, TP, uW) + (TP - TW) * pW;
      const double phN = upw(TP, TN, vN) + (TN - TP) * pN;
      const double phS = upw(TS, TP, vS) + (TP - TS) * pS;
      const double lFE = -lt * phE, lFW = lt * phW, lFN = -lt * phN, lFS = lt * phS;
      const double lpE = -lt * FE, lpW = lt * FW, lpN = -lt * FN, lpS = lt * FS;
      sk.add(4, P, i, j, lFW * uW * dyj);
      sk.add(4, P, i + 1, j, lFE * uE * dyj);
      sk.add(5, P, i, j, lFS * vS * dxi);
      sk.add(5, P, i, j + 1, lFN * vN * dxi);
      sk.add(0, P, i, j, lFW * rW * dyj);
      sk.add(0, P, i + 1, j, lFE * rE * dyj);
      sk.add(1, P, i, j, lFS * rS * dxi);
      sk.add(1, P, i, j + 1, lFN * rN * dxi);
      // face values: d phi / d (nodes)
      double lTW = 0, lTE = 0, lTS = 0, lTN = 0;
      // phiE = upw(TP, TE) + (TE - TP) psiE(T_{i-1}, TP, TE, T_{i+2})
      if (uE > 0.0) lTP += lpE; else lTE += lpE;
      lTE += lpE * pE;
      lTP -= lpE * pE;
      if (tE) {
        const double q = lpE * (TE - TP);
        sk.add(2, P, i - 1, j, q * gE[0]);
        lTP += q * gE[1];
        lTE += q * gE[2];
        sk.add(2, P, i + 2, j, q * gE[3]);
      }
      if (uW > 0.0) lTW += lpW; else lTP += lpW;
      lTP += lpW * pW;
      lTW -= lpW * pW;
      if (tW) {
        const double q = lpW * (TP - TW);
        sk.add(2, P, i - 2, j, q * gW[0]);
        lTW += q * gW[1];
        lTP += q * gW[2];
        lTE += q * gW[3];
      }
      if (vN > 0.0) lTP += lpN; else lTN += lpN;
      lTN += lpN * pN;
      lTP -= lpN * pN;
      if (tN) {
        const double q = lpN * (TN - TP);
        sk.add(2, P, i, j - 1, q * gN[0]);
        lTP += q * gN[1];
        lTN += q * gN[2];
        sk.add(2, P, i, j + 2, q * gN[3]);
      }
      if (vS > 0.0) lTS += lpS; else lTP += lpS;
      lTP += lpS * pS;
      lTS -= lpS * pS;
      if (tS) {
        const double q = lpS * (TP - TS);
        sk.add(2, P, i, j - 2, q * gS[0]);
        lTS += q * gS[1];
        lTP += q * gS[2];
        lTN += q * gS[3];
      }
      // neighbour values that are boundary rules
      if (!inl) sk.add(2, P, i - 1, j, lTW);
      if (outl) lTP += lTE; else sk.add(2, P, i + 1, j, lTE);
      if (bot) lTP += lTS; else sk.add(2, P, i, j - 1, lTS);
      if (top) lTP += lTN; else sk.add(2, P, i, j + 1, lTN);
    }
    sk.add(2, P, i, j, lTP);
  }
  // ---- u-face constant
  if (j < P.ny && u_solved(P, i, j)) {
    const long k = ix(P, i, j);
    const double l = lC.Cu[k];
    if (l != 0.0) {
      const double dxl = gx(P, 0, i - 1), dxr = gx(P, 0, i), dyj = gy(P, 0, j);
      const double uP = m.u[k];
      const double M = (rho(P, m, i, j) * dxr + rho(P, m, i - 1, j) * dxl) * dyj / 2.0;
      const double lM = l * (P.idt * uP + P.gx);
      sk.add(0, P, i, j, l * M * P.idt);
      sk.add(3, P, i, j, lM * dxr * dyj / 2.0);
      sk.add(3, P, i - 1, j, lM * dxl * dyj / 2.0);
      // u^exp
      const bool bot = j == 0, top = j == P.ny - 1;
      const double uW = at(m.u, P, i - 1, j), uE = at(m.u, P, i + 1, j);
      const double uS = bot ? uP : at(m.u, P, i, j - 1), uN = top ? uP : at(m.u, P, i, j + 1);
      const double vn0 = at(m.v, P, i - 1, j + 1), vn1 = at(m.v, P, i, j + 1);
      const double vs0 = at(m.v, P, i - 1, j), vs1 = at(m.v, P, i, j);
      const double rn0 = rv0[k - 1 + P.pitch], rn1 = rv0[k + P.pitch];
      const double rs0 = rv0[k - 1], rs1 = rv0[k];
      const double Fn0 = rn0 * vn0 * dxl, Fn1 = rn1 * vn1 * dxr;
      const double Fs0 = rs0 * vs0 * dxl, Fs1 = rs1 * vs1 * dxr;
      const double ubE = 0.5 * (uP + uE), ubW = 0.5 * (uW + uP);
      const double rE = rho(P, m, i, j), rW = rho(P, m, i - 1, j);
      const double FbE = rE * ubE * dyj, FbW = rW * ubW * dyj;
      double gn0[4] = {0, 0, 0, 0}, gn1[4] = {0, 0, 0, 0}, gs0[4] = {0, 0, 0, 0},
             gs1[4] = {0, 0, 0, 0}, ge[4] = {0, 0, 0, 0}, gw[4] = {0, 0, 0, 0};
      double pn0 = 0, pn1 = 0, ps0 = 0, ps1 = 0, pe = 0, pw = 0;
      bool tn = false, ts = false, te = false, tw = false;
      if (TV) {
        tn = j - 1 >= 0 && j + 2 <= P.ny - 1;
        ts = j - 2 >= 0 && j + 1 <= P.ny - 1;
        te = i - 1 >= 0 && i + 2 <= P.nx;
        tw = i - 2 >= 0 && i + 1 <= P.nx;
        if (tn) {
          const double f1 = at(m.u, P, i, j - 1), f4 = at(m.u, P, i, j + 2);
          pn0 = psiy_d(P, f1, uP, uN, f4, j + 1, vn0, gn0);
          pn1 = psiy_d(P, f1, uP, uN, f4, j + 1, vn1, gn1);
        }
        if (ts) {
          const double f1 = at(m.u, P, i, j - 2), f4 = at(m.u, P, i, j + 1);
          ps0 = psiy_d(P, f1, uS, uP, f4, j, vs0, gs0);
          ps1 = psiy_d(P, f1, uS, uP, f4, j, vs1, gs1);
        }
        if (te) pe = psi_c_d(uW, uP, uE, at(m.u, P, i + 2, j), dxl, dxr, gx(P, 0, i + 1), ubE, ge);
        if (tw) pw = psi_c_d(at(m.u, P, i - 2, j), uW, uP, uE, gx(P, 0, i - 2), dxl, dxr, ubW, gw);
      }
      const double phn0 = upw(uP, uN, vn0) + (uN - uP) * pn0, phn1 = upw(uP, uN, vn1) + (uN - uP) * pn1;
      const double phs0 = upw(uS, uP, vs0) + (uP - uS) * ps0, phs1 = upw(uS, uP, vs1) + (uP - uS) * ps1;
      const double phe = upw(uP, uE, ubE) + (uE - uP) * pe, phw = upw(uW, uP, ubW) + (uP - uW) * pw;
      // u^exp = -0.5 (Fn0 phn0 + Fn1 phn1) + 0.5 (Fs0 phs0 + Fs1 phs1) - FbE phe + FbW phw
      const double lFn0 = -0.5 * l * phn0, lFn1 = -0.5 * l * phn1;
      const double lFs0 = 0.5 * l * phs0, lFs1 = 0.5 * l * phs1;
      const double lFbE = -l * phe, lFbW = l * phw;
      const double lpn0 = -0.5 * l * Fn0, lpn1 = -0.5 * l * Fn1;
      const double lps0 = 0.5 * l * Fs0, lps1 = 0.5 * l * Fs1;
      const double lpe = -l * FbE, lpw = l * FbW;
      sk.add(5, P, i - 1, j + 1, lFn0 * vn0 * dxl);
      sk.add(5, P, i, j + 1, lFn1 * vn1 * dxr);
      sk.add(5, P, i - 1, j, lFs0 * vs0 * dxl);
      sk.add(5, P, i, j, lFs1 * vs1 * dxr);
      sk.add(1, P, i - 1, j + 1, lFn0 * rn0 * dxl);
      sk.add(1, P, i, j + 1, lFn1 * rn1 * dxr);
      sk.add(1, P, i - 1, j, lFs0 * rs0 * dxl);
      sk.add(1, P, i, j, lFs1 * rs1 * dxr);
      sk.add(3, P, i, j, lFbE * ubE * dyj);
      sk.add(3, P, i - 1, j, lFbW * ubW * dyj);
      const double lubE = lFbE * rE * dyj, lubW = lFbW * rW * dyj;
      double luP = 0.5 * (lubE + lubW), luW = 0.5 * lubW, luE = 0.5 * lubE, luS = 0, luN = 0;
      // face values
      if (vn0 > 0.0) luP += lpn0; else luN += lpn0;
      if (vn1 > 0.0) luP += lpn1; else luN += lpn1;
      luN += (lpn0 * pn0 + lpn1 * pn1);
      luP -= (lpn0 * pn0 + lpn1 * pn1);
      if (vs0 > 0.0) luS += lps0; else luP += lps0;
      if (vs1 > 0.0) luS += lps1; else luP += lps1;
      luP += (lps0 * ps0 + lps1 * ps1);
      luS -= (lps0 * ps0 + lps1 * ps1);
      if (ubE > 0.0) luP += lpe; else luE += lpe;
      luE += lpe * pe;
      luP -= lpe * pe;
      if (ubW > 0.0) luW += lpw; else luP += lpw;
      luP += lpw * pw;
      luW -= lpw * pw;
      if (tn) {
        const double q0 = lpn0 * (uN - uP), q1 = lpn1 * (uN - uP);
        sk.add(0, P, i, j - 1, q0 * gn0[0] + q1 * gn1[0]);
        luP += q0 * gn0[1] + q1 * gn1[1];
        luN += q0 * gn0[2] + q1 * gn1[2];
        sk.add(0, P, i, j + 2, q0 * gn0[3] + q1 * gn1[3]);
      }
      if (ts) {
        const double q0 = lps0 * (uP - uS), q1 = lps1 * (uP - uS);
        sk.add(0, P, i, j - 2, q0 * gs0[0] + q1 * gs1[0]);
        luS += q0 * gs0[1] + q1 * gs1[1];
        luP += q0 * gs0[2] + q1 * gs1[2];
        sk.add(0, P, i, j + 1, q0 * gs0[3] + q1 * gs1[3]);
      }
      if (te) {
        const double q = lpe * (uE - uP);
        luW += q * ge[0];
        luP += q * ge[1];
        luE += q * ge[2];
        sk.add(0, P, i + 2, j, q * ge[3]);
      }
      if (tw) {
        const double q = lpw * (uP - uW);
        sk.add(0, P, i - 2, j, q * gw[0]);
        luW += q * gw[1];
        luP += q * gw[2];
        luE += q * gw[3];
      }
      if (bot) luP += luS; else sk.add(0, P, i, j - 1, luS);
      if (top) luP += luN; else sk.add(0, P, i, j + 1, luN);
      sk.add(0, P, i - 1, j, luW);
      sk.add(0, P, i + 1, j, luE);
      sk.add(0, P, i, j, luP);
    }
  }
  // ---- v-face constant
  if (i < P.nx && v_solved(P, i, j)) {
    const long k = ix(P, i, j);
    const double l = lC.Cv[k];
    if (l != 0.0) {
      const double dxi = gx(P, 0, i), dys = gy(P, 0, j - 1), dyn = gy(P, 0, j);
      const double vP = m.v[k];
      const double M = (rho(P, m, i, j) * dyn + rho(P, m, i, j - 1) * dys) * dxi / 2.0;
      const double lM = l * (P.idt * vP + P.gy);
      sk.add(1, P, i, j, l * M * P.idt);
      sk.add(3, P, i, j, lM * dyn * dxi / 2.0);
      sk.add(3, P, i, j - 1, lM * dys * dxi / 2.0);
      const bool inl = i == 0, outl = i == P.nx - 1;
      const double vW = inl ? 0.0 : at(m.v, P, i - 1, j);
      const double vE = outl ? vP : at(m.v, P, i + 1, j);
      const double vS = at(m.v, P, i, j - 1), vN = at(m.v, P, i, j + 1);
      const double ue0 = at(m.u, P, i + 1, j - 1), ue1 = at(m.u, P, i + 1, j);
      const double uw0 = at(m.u, P, i, j - 1), uw1 = at(m.u, P, i, j);
      const double re0 = ru0[k + 1 - P.pitch], re1 = ru0[k + 1];
      const double rw0 = ru0[k - P.pitch], rw1 = ru0[k];
      const double Fe0 = re0 * ue0 * dys, Fe1 = re1 * ue1 * dyn;
      const double Fw0 = rw0 * uw0 * dys, Fw1 = rw1 * uw1 * dyn;
      const double vbN = 0.5 * (vP + vN), vbS = 0.5 * (vS + vP);
      const double rN = rho(P, m, i, j), rS = rho(P, m, i, j - 1);
      const double FbN = rN * vbN * dxi, FbS = rS * vbS * dxi;
      double ge0[4] = {0, 0, 0, 0}, ge1[4] = {0, 0, 0, 0}, gw0[4] = {0, 0, 0, 0},
             gw1[4] = {0, 0, 0, 0}, gn[4] = {0, 0, 0, 0}, gs[4] = {0, 0, 0, 0};
      double pe0 = 0, pe1 = 0, pw0 = 0, pw1 = 0, pn = 0, ps = 0;
      bool te = false, tw = false, tn = false, ts = false;
      if (TV) {
        te = i - 1 >= 0 && i + 2 <= P.nx - 1;
        tw = i - 2 >= 0 && i + 1 <= P.nx - 1;
        tn = j - 1 >= 0 && j + 2 <= P.ny;
        ts = j - 2 >= 0 && j + 1 <= P.ny;
        if (te) {
          const double f1 = at(m.v, P, i - 1, j), f4 = at(m.v, P, i + 2, j);
          pe0 = psix_d(P, f1, vP, vE, f4, i + 1, ue0, ge0);
          pe1 = psix_d(P, f1, vP, vE, f4, i + 1, ue1, ge1);
        }
        if (tw) {
          const double f1 = at(m.v, P, i - 2, j), f4 = at(m.v, P, i + 1, j);
          pw0 = psix_d(P, f1, vW, vP, f4, i, uw0, gw0);
          pw1 = psix_d(P, f1, vW, vP, f4, i, uw1, gw1);
        }
        if (tn) pn = psi_c_d(vS, vP, vN, at(m.v, P, i, j + 2), dys, dyn, gy(P, 0, j + 1), vbN, gn);
        if (ts) ps = psi_c_d(at(m.v, P, i, j - 2), vS, vP, vN, gy(P, 0, j - 2), dys, dyn, vbS, gs);
      }
      const double phe0 = upw(vP, vE, ue0) + (vE - vP) * pe0, phe1 = upw(vP, vE, ue1) + (vE - vP) * pe1;
      const double phw0 = upw(vW, vP, uw0) + (vP - vW) * pw0, phw1 = upw(vW, vP, uw1) + (vP - vW) * pw1;
      const double phn = upw(vP, vN, vbN) + (vN - vP) * pn, phs = upw(vS, vP, vbS) + (vP - vS) * ps;
      const double lFe0 = -0.5 * l * phe0, lFe1 = -0.5 * l * phe1;
      const double lFw0 = 0.5 * l * phw0, lFw1 = 0.5 * l * phw1;
      const double lFbN = -l * phn, lFbS = l * phs;
      const double lpe0 = -0.5 * l * Fe0, lpe1 = -0.5 * l * Fe1;
      const double lpw0 = 0.5 * l * Fw0, lpw1 = 0.5 * l * Fw1;
      const double lpn = -l * FbN, lps = l * FbS;
      sk.add(4, P, i + 1, j - 1, lFe0 * ue0 * dys);
      sk.add(4, P, i + 1, j, lFe1 * ue1 * dyn);
      sk.add(4, P, i, j - 1, lFw0 * uw0 * dys);
      sk.add(4, P, i, j, lFw1 * uw1 * dyn);
      sk.add(0, P, i + 1, j - 1, lFe0 * re0 * dys);
      sk.add(0, P, i + 1, j, lFe1 * re1 * dyn);
      sk.add(0, P, i, j - 1, lFw0 * rw0 * dys);
      sk.add(0, P, i, j, lFw1 * rw1 * dyn);
      sk.add(3, P, i, j, lFbN * vbN * dxi);
      sk.add(3, P, i, j - 1, lFbS * vbS * dxi);
      const double lvbN = lFbN * rN * dxi, lvbS = lFbS * rS * dxi;
      double lvP = 0.5 * (lvbN + lvbS), lvN = 0.5 * lvbN, lvS = 0.5 * lvbS, lvW = 0, lvE = 0;
      if (ue0 > 0.0) lvP += lpe0; else lvE += lpe0;
      if (ue1 > 0.0) lvP += lpe1; else lvE += lpe1;
      lvE += lpe0 * pe0 + lpe1 * pe1;
      lvP -= lpe0 * pe0 + lpe1 * pe1;
      if (uw0 > 0.0) lvW += lpw0; else lvP += lpw0;
      if (uw1 > 0.0) lvW += lpw1; else lvP += lpw1;
      lvP += lpw0 * pw0 + lpw1 * pw1;
      lvW -= lpw0 * pw0 + lpw1 * pw1;
      if (vbN > 0.0) lvP += lpn; else lvN += lpn;
      lvN += lpn * pn;
      lvP -= lpn * pn;
      if (vbS > 0.0) lvS += lps; else lvP += lps;
      lvP += lps * ps;
      lvS -= lps * ps;
      if (te) {
        const double q0 = lpe0 * (vE - vP), q1 = lpe1 * (vE - vP);
        sk.add(1, P, i - 1, j, q0 * ge0[0] + q1 * ge1[0]);
        lvP += q0 * ge0[1] + q1 * ge1[1];
        lvE += q0 * ge0[2] + q1 * ge1[2];
        sk.add(1, P, i + 2, j, q0 * ge0[3] + q1 * ge1[3]);
      }
      if (tw) {
        const double q0 = lpw0 * (vP - vW), q1 = lpw1 * (vP - vW);
        sk.add(1, P, i - 2, j, q0 * gw0[0] + q1 * gw1[0]);
        lvW += q0 * gw0[1] + q1 * gw1[1];
        lvP += q0 * gw0[2] + q1 * gw1[2];
        sk.add(1, P, i + 1, j, q0 * gw0[3] + q1 * gw1[3]);
      }
      if (tn) {
        const double q = lpn * (vN - vP);
        lvS += q * gn[0];
        lvP += q * gn[1];
        lvN += q * gn[2];
        sk.add(1, P, i, j + 2, q * gn[3]);
      }
      if (ts) {
        const double q = lps * (vP - vS);
        sk.add(1, P, i, j - 2, q * gs[0]);
        lvS += q * gs[1];
        lvP += q * gs[2];
        lvN += q * gs[3];
      }
      if (!inl) sk.add(1, P, i - 1, j, lvW);
      if (outl) lvP += lvE; else sk.add(1, P, i + 1, j, lvE);
      sk.add(1, P, i, j - 1, lvS);
      sk.add(1, P, i, j + 1, lvN);
      sk.add(1, P, i, j, lvP);
    }
  }
}

// Reverse of the prologue.  Its scatters are summed per tile in LDS first
// (slots: lambda of u, v, T of level n-1, of rho, of the u- and v-face
// densities), then added to the arrays once per touched window entry.
template <bool TV>
__global__ __launch_bounds__(AB) void k_adj_prologue(const Params P, const State m,
                                                     const Consts lC, const State lm,
                                                     const double *ru0, const double *rv0,
                                                     double *lru, double *lrv, double *lr) {
  __shared__ double wl[6 * Tiled<6, 2, false>::WN];
  Tiled<6, 2, false> sk{(lds_double *)wl, {lm.u, lm.v, lm.T, lr, lru, lrv}};
  int i, j;
  sk.begin(P, i, j);
  if (i <= P.nx && j <= P.ny) prologue_item<TV>(P, m, lC, ru0, rv0, i, j, sk);
  sk.end(P);
}

// face densities of a state (as in the forward pass), for the prologue
template <bool TV>
__global__ __launch_bounds__(AB) void k_face_densities(const Params P, const State m,
                                                       double *ru, double *rv) {
  int i, j;
  if (!elem(P, i, j)) return;
  double g[4];
  if (j < P.ny) {
    const double uf = at(m.u, P, i, j);
    double r;
    if (i == 0) r = uf > 0.0 ? P.inl[4 * (j) + 3] : rho(P, m, 0, j);
    else if (i == P.nx) r = rho(P, m, P.nx - 1, j);
    else {
      const double rl = rho(P, m, i - 1, j), rr = rho(P, m, i, j);
      r = upw(rl, rr, uf);
      if (TV && fl(P, i - 2, j) && fl(P, i - 1, j) && fl(P, i, j) && fl(P, i + 1, j))
        r += psix_d(P, rho(P, m, i - 2, j), rl, rr, rho(P, m, i + 1, j), i, uf, g) * (rr - rl);
    }
    ru[ix(P, i, j)] = r;
  }
  if (i < P.nx) {
    double r;
    if (j == 0) r = rho(P, m, i, 0);
    else if (j == P.ny) r = rho(P, m, i, P.ny - 1);
    else {
      const double vf = at(m.v, P, i, j);
      const double rs = rho(P, m, i, j - 1), rn = rho(P, m, i, j);
      r = upw(rs, rn, vf);
      if (TV && fl(P, i, j - 2) && fl(P, i, j - 1) && fl(P, i, j) && fl(P, i, j + 1))
        r += psiy_d(P, rho(P, m, i, j - 2), rs, rn, rho(P, m, i, j + 1), j, vf, g) * (rn - rs);
    }
    rv[ix(P, i, j)] = r;
  }
}

// ---------------------------------------------------------------------------
// drag on the obstacles and its adjoint seed
// ---------------------------------------------------------------------------
// D = sum over fluid cells next to a solid cell of: A p dy (solid to the
// east), -A p dy (solid to the west), and the wall shear B Gamma u_c dx /
// (dy / 2) (solid to the south or north), u_c the cell-centre x-velocity.
__device__ double drag_cell(const Params &P, const State &o, int i, int j, double g[4]) {
  // g: d D_cell / d (p, u_i, u_{i+1}, T)
  g[0] = g[1] = g[2] = g[3] = 0.0;
  if (!fl(P, i, j)) return 0.0;
  const double dxi = gx(P, 0, i), dyj = gy(P, 0, j);
  double d = 0.0;
  const double p = at(o.p, P, i, j);
  const bool sE = i + 1 < P.nx && !fl(P, i + 1, j), sW = i - 1 >= 0 && !fl(P, i - 1, j);
  const bool sS = j - 1 >= 0 && !fl(P, i, j - 1), sN = j + 1 < P.ny && !fl(P, i, j + 1);
  if (sE) { d += P.A * p * dyj; g[0] += P.A * dyj; }
  if (sW) { d -= P.A * p * dyj; g[0] -= P.A * dyj; }
  const int ns = (sS ? 1 : 0) + (sN ? 1 : 0);
  if (ns) {
    const double T = at(o.T, P, i, j), G = sqrt(T);
    const double uc = 0.5 * (at(o.u, P, i, j) + at(o.u, P, i + 1, j));
    const double K = ns * P.B * dxi / (0.5 * dyj);
    d += K * G * uc;
    g[1] += 0.5 * K * G;
    g[2] += 0.5 * K * G;
    g[3] += K * uc / (2.0 * G);
  }
  return d;
}
__global__ __launch_bounds__(AB) void k_drag(const Params P, const State o, double *out) {
  __shared__ double red[AB / 64];
  double s = 0.0, g[4];
  for (long t = (long)blockIdx.x * AB + threadIdx.x; t < (long)P.nx * P.ny; t += (long)gridDim.x * AB)
    s += drag_cell(P, o, (int)(t % P.nx), (int)(t / P.nx), g);
  for (int q = 32; q > 0; q >>= 1) s += __shfl_xor(s, q, 64);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < AB / 64; w++) r += red[w];
    out[blockIdx.x] = r;
  }
}
// sum of n partials in a fixed order (one block)
__global__ __launch_bounds__(AB) void k_sum(const double *in, int n, double *out) {
  __shared__ double red[AB / 64];
  double r = 0.0;
  for (int q = threadIdx.x; q < n; q += AB) r += in[q];
  for (int o = 32; o > 0; o >>= 1) r += __shfl_xor(r, o, 64);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < AB / 64; w++) t += red[w];
    *out = t;
  }
}
__global__ __launch_bounds__(AB) void k_drag_seed(const Params P, const State o, const State lam,
                                                  double w) {
  int i, j;
  if (!elem(P, i, j) || i >= P.nx || j >= P.ny) return;
  double g[4];
  drag_cell(P, o, i, j, g);
  if (g[0] != 0.0) aadd(lam.p, P, i, j, w * g[0]);
  if (g[1] != 0.0) aadd(lam.u, P, i, j, w * g[1]);
  if (g[2] != 0.0) aadd(lam.u, P, i + 1, j, w * g[2]);
  if (g[3] != 0.0) aadd(lam.T, P, i, j, w * g[3]);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static dim3 agrid(const Params &P) {
  return dim3((unsigned)(((long)(P.nx + 1) * (P.ny + 1) + AB - 1) / AB));
}

// rho = p/T and Gamma = sqrt(T) of a state's cells and of the first two
// frame layers around them (the values the stencils read there)
__global__ __launch_bounds__(AB) void k_cell_cache(const Params P, const State o, double *r,
                                                   double *g) {
  const long t = (long)blockIdx.x * AB + threadIdx.x;
  const int W = P.nx + 4, H = P.ny + 4;
  if (t >= (long)W * H) return;
  const int i = (int)(t % W) - 2, j = (int)(t / W) - 2;
  const long k = ix(P, i, j);
  r[k] = o.p[k] / o.T[k];
  g[k] = sqrt(o.T[k]);
}
static dim3 cgrid(const Params &P) {
  return dim3((unsigned)(((long)(P.nx + 4) * (P.ny + 4) + AB - 1) / AB));
}

void launch_cell_cache(const Params &P, State o, double *r, double *g, hipStream_t st) {
  hipLaunchKernelGGL(k_cell_cache, cgrid(P), dim3(AB), 0, st, P, o, r, g);
}

void launch_adjoint_pass(const Params &P, State o, Consts C, Inter I, State ln, State lo,
                         Consts lC, AdjTmp A, double *gtw0, double *gtw1, int scheme,
                         hipStream_t st) {
  const dim3 b(AB), gt = tgrid(P);
  hipLaunchKernelGGL(k_adj_front, gt, b, 0, st, P, o, ln, lo, lC, I, A);
  if (scheme & 2) {
    if (P.sj) hipLaunchKernelGGL((k_adj_stage2<true, true>), gt, b, 0, st, P, o, lo, C, lC, I, A, gtw0, gtw1);
    else hipLaunchKernelGGL((k_adj_stage2<true, false>), gt, b, 0, st, P, o, lo, C, lC, I, A, gtw0, gtw1);
  } else {
    if (P.sj) hipLaunchKernelGGL((k_adj_stage2<false, true>), gt, b, 0, st, P, o, lo, C, lC, I, A, gtw0, gtw1);
    else hipLaunchKernelGGL((k_adj_stage2<false, false>), gt, b, 0, st, P, o, lo, C, lC, I, A, gtw0, gtw1);
  }
}

void launch_adjoint_prologue(const Params &P, State m, Consts lC, State lm, AdjTmp A,
                             int scheme, hipStream_t st) {
  const dim3 g = agrid(P), b(AB);
  const bool tv = (scheme & 2) != 0;
  // face densities of the level n-1 fields into the (free) u-hat / v-hat
  // temporaries, then the reverse of the constants
  if (tv) hipLaunchKernelGGL((k_face_densities<true>), g, b, 0, st, P, m, A.luh, A.lvh);
  else hipLaunchKernelGGL((k_face_densities<false>), g, b, 0, st, P, m, A.luh, A.lvh);
  if (tv)
    hipLaunchKernelGGL((k_adj_prologue<true>), tgrid(P), b, 0, st, P, m, lC, lm, A.luh, A.lvh,
                       A.lru, A.lrv, A.lr);
  else
    hipLaunchKernelGGL((k_adj_prologue<false>), tgrid(P), b, 0, st, P, m, lC, lm, A.luh, A.lvh,
                       A.lru, A.lrv, A.lr);
  hipLaunchKernelGGL(k_cell_cache, cgrid(P), b, 0, st, P, m, A.cr, A.cg);
  if (tv)
    hipLaunchKernelGGL((k_adj_rho_faces<true>), tgrid(P), b, 0, st, P, m, Cache{A.cr, A.cg},
                       A.lru, A.lrv, A.lr);
  else
    hipLaunchKernelGGL((k_adj_rho_faces<false>), tgrid(P), b, 0, st, P, m, Cache{A.cr, A.cg},
                       A.lru, A.lrv, A.lr);
  hipLaunchKernelGGL(k_adj_cell_props, g, b, 0, st, P, m, lm, A.lr, A.lg);
}

int drag_blocks(const Params &P) {
  long n = ((long)P.nx * P.ny + AB - 1) / AB;
  return (int)(n > 1024 ? 1024 : n);
}
void launch_drag(const Params &P, State o, double *partial, double *out, hipStream_t st) {
  const int nb = drag_blocks(P);
  hipLaunchKernelGGL(k_drag, dim3(nb), dim3(AB), 0, st, P, o, partial);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(AB), 0, st, partial, nb, out);
}
void launch_drag_seed(const Params &P, State o, State lam, double w, hipStream_t st) {
  hipLaunchKernelGGL(k_drag_seed, agrid(P), dim3(AB), 0, st, P, o, lam, w);
}

}  // namespace sts
