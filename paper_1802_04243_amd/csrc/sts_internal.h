// Internal declarations shared by the host runtime and the kernels of
// libsts.so (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/sts.h"

namespace sts {
// set the thread's last-error message of the C ABI (sts_last_error) and
// return s
sts_status report_error(sts_status s, const char *msg);


// Tiling of the Jacobi pass: a block of BX x BY threads computes T, p,
// u-hat, v-hat on the owned TX x TY cells plus a one-cell halo, and writes
// the owned cells / faces.  The LDS window of old fields has a halo of HB.
constexpr int TX = 30, TY = 14;
constexpr int BX = TX + 2, BY = TY + 2;
constexpr int NT = BX * BY;  // 512 cell positions (threads of the prologue)
// Threads of a pass block: the NT cell threads plus NT/2 more, so that the
// cell, u-face and v-face items of a pass (3 NT) take two rounds.
constexpr int NTP = 3 * NT / 2;
constexpr int HB = 3;
constexpr int LW = TX + 2 * HB, LH = TY + 2 * HB;

// Device layout of every field array: a frame of ghost columns/rows around
// the domain so that any window load stays inside the allocation.
constexpr int XO = 32;  // column of i = 0 (256-byte aligned rows)
constexpr int YO = 4;   // row of j = 0
constexpr int XPAD = 4; // ghost entries of the padded 1-D width arrays

struct State {
  double *u, *v, *p, *T;
};
struct Consts {
  double *Cu, *Cv, *CT, *Cp;
};

struct Params {
  int nx, ny, per;
  int tiles_x, tiles_y;
  long pitch;  // doubles per row
  long off;    // element index of (0,0)
  double dt, idt, A, B, C1, C2, C3, gx, gy, obsT, sq_obsT;
  int wtype0, wtype1;  // STS_WALL_* of the bottom and top walls
  int otype;           // STS_WALL_* of the obstacle surfaces
  int sj;              // some surface is slip-jump (selects the kernel instances)
  double wu0, wu1;
  // slip / jump length times rho of the slip-jump surfaces (eqs pl38, pl39):
  // zeta = kz / rho, tau = kt / rho
  double kz, kt;
  // geometry per column i, six values interleaved at gx6[6 (i + XPAD) + q]
  // (wrapped or clamped outside the domain): [0] dx_i, [1] 1/dx_i; per
  // x-face i (between cells i-1 and i): [2] s = dx_{i-1} + dx_i, [3] 1/s,
  // [4] dx_i/s (weight of cell i-1), [5] dx_{i-1}/s (weight of cell i).
  // The same in y.  One pointer per direction keeps the kernels' scalar
  // registers free (six pointers each spilled them into vector lanes).
  const double *gx6, *gy6;
  // boundary data, interleaved like the geometry: per row j of the inlet
  // inl[4 j + q], q = u_in, T_in, sqrt(T_in), rho_in = p_in / T_in; per cell
  // column i of the walls wl[4 i + q], q = bottom T, top T, their square
  // roots; per u-face i wu[2 i + q], q = sqrt of the bottom, top wall T at
  // the face's x
  const double *inl, *wl, *wu;
  const unsigned char *fl;   // 1 = fluid cell, frame = 0; cell layout
  const unsigned char *clean; // [tiles] 1 = no boundary rule in the window
};

// residual partial per block: max|du|, max|dv|, max|dp|, max|dT|, max|R|,
// sum R, non-finite count
constexpr int NRES = 8;
// offset (in doubles) of the loop-2 control block in the residual buffer
constexpr int RES_CTL = 16;
constexpr int RES_BLOCKS = 2048;  // blocks of the continuity-residual kernel

// Outputs of the last pass of a step used by the residual reduction: the
// face mass fluxes rho^u u dy (u-face layout) and rho^v v dx (v-face layout)
// of the new velocities, and one row of NRES partials per tile.  stop: NULL,
// or the device flag of a loop 2 run to convergence (Loop2); once it is set,
// the residual-producing pass and the reduction kernels return at once.
struct Resid {
  double *gu, *gv;
  double *partials;  // [tiles + RES_BLOCKS][NRES]
  const int *stop;
};

// Device-side convergence control of loop 2: ctl[0] = stop flag, ctl[1] =
// passes run.  The reduction after pass k writes ctl[1] = k and sets the flag
// when max(max|du|, max|dv|, max|dT|, max|dp| / p_in) <= tol or some value is
// non-finite (some pass's per-tile non-finite count is not zero).  hist: the
// residual history, row k - 1 = max|du|, max|dv|, max|dp|, max|dT| of pass
// k for k <= HIST_CAP (NULL: not recorded).
constexpr int HIST_CAP = 4096;
struct Loop2 {
  int *ctl;
  double tol, p_in;
  int k;
  double *hist = nullptr;
};

// Intermediates of one pass (face densities, u-hat, d^u, v-hat, d^v, new p,
// new T) in the field layout, stored for the adjoint's reverse sweep; all
// NULL in a plain pass.
struct Inter {
  double *ru, *rv, *uh, *du, *vh, *dv, *pn, *tn;
};

// Adjoints of the pass intermediates (u-hat, d^u, v-hat, d^v, face
// densities, rho, Gamma, new T), field layout.
struct AdjTmp {
  double *luh, *ldu, *lvh, *ldv, *lru, *lrv, *lr, *lg, *ltn;
  // rho = p/T and Gamma = sqrt(T) of the iterate being reversed (its frame
  // entries hold the values of the constant ghost state)
  double *cr, *cg;
};

void launch_prologue(const Params &P, State m, Consts C, int scheme,
                     hipStream_t st);
void launch_pass(const Params &P, State o, State n, Consts C, int scheme,
                 const Resid *last, const Inter *inter, hipStream_t st);
// the step prologue fused into the step's first pass (a step of at least two
// passes): writes the step constants and the first iterate
void launch_pass_first(const Params &P, State o, State n, Consts C, int scheme, hipStream_t st);
// one energy-pressure solve of a pass with loop 3 (FP64 schemes): L3 = 1 a
// solve before the last (T, p into To, po; Ts = NULL for the first, whose T
// and p are the iterate's), 2 the last (Ts, ps: the previous solve; the
// pass's outputs in n, with the residual inputs when last != NULL)
void launch_pass3(const Params &P, State o, State n, Consts C, int scheme, const Resid *last,
                  int L3, const double *Ts, const double *ps, double *To, double *po,
                  hipStream_t st);
void launch_residual(const Params &P, State n, Consts C, Resid R, double *out,
                     hipStream_t st);
// loop 2 run to convergence: clear the control block; after pass L.k, fold
// the pass's per-tile rows and take the decision (returns at once once the
// flag is set); at the end, the residuals of the last pass run, whose state
// is `even` or `odd` as ctl[1] is
void launch_loop2_reset(int *ctl, hipStream_t st);
void launch_loop2_check(const Params &P, Resid R, double *out, const Loop2 &L, hipStream_t st);
void launch_loop2_final(const Params &P, State even, State odd, Consts C, Resid R, double *out,
                        const int *ctl, hipStream_t st);

// adjoint of the explicit step (reverse of one pass; reverse of the prologue)
void launch_adjoint_pass(const Params &P, State o, Consts C, Inter I, State ln, State lo,
                         Consts lC, AdjTmp A, double *gtw0, double *gtw1, int scheme,
                         hipStream_t st);
void launch_cell_cache(const Params &P, State o, double *r, double *g, hipStream_t st);
void launch_adjoint_prologue(const Params &P, State m, Consts lC, State lm, AdjTmp A,
                             int scheme, hipStream_t st);
// drag on the obstacles of a state (partial: drag_blocks doubles) and the
// adjoint seed lam += w dD/d(state)
int drag_blocks(const Params &P);
void launch_drag(const Params &P, State o, double *partial, double *out, hipStream_t st);
void launch_drag_seed(const Params &P, State o, State lam, double w, hipStream_t st);

}  // namespace sts
