/*
 * sts.h -- C ABI of the MI355X SIMPLE-TS library (libsts.so).
 *
 * SIMPLE-TS (Shterev, arXiv 1802.04243) advances the unsteady, viscous,
 * compressible, heat-conductive 2-D Navier-Stokes-Fourier system (Sec. 2,
 * eqs pl4-pl7) on a staggered Cartesian finite-volume grid (Sec. 3.2, the
 * cell-volume figure).  One time step (loop 1) is a step prologue followed by
 * n_inner Jacobi passes of loop 2 (Sec. 3.1, figures of the explicit and
 * implicit GPU algorithms; pass order of Appendix A).  Every computation runs
 * in hand-written HIP kernels on the GPU the context was created on.
 *
 * Conventions
 *   - Every function returns sts_status (0 = OK, < 0 = error) and never
 *     aborts.  On error sts_last_error() returns a message (thread-local).
 *   - All quantities are nondimensional FP64: lengths in channel heights,
 *     velocities in inlet speeds, T, p, rho relative to the inlet state.
 *   - Host field arrays are dense, x fastest:
 *       u [ny][nx+1]  x-velocity at x-faces (x^f_i, y^v_j)
 *       v [ny+1][nx]  y-velocity at y-faces (x^v_i, y^f_j)
 *       p [ny][nx], T [ny][nx]  at cell centres.
 *   - One context per host thread.  Calls on one context are ordered on its
 *     HIP stream; sts_step is asynchronous, sts_residuals / sts_fields wait.
 */
#ifndef STS_H
#define STS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STS_OK = 0,
  STS_EINVAL = -1,     /* invalid argument; the context is unchanged        */
  STS_ENOMEM = -2,     /* device or host allocation failed                  */
  STS_EDEVICE = -3,    /* a HIP call failed                                  */
  STS_ENONFINITE = -4, /* the last step produced a non-finite value; the
                          state is left as computed, for inspection         */
  STS_ESTATE = -5      /* call not valid in the current state               */
} sts_status;

typedef struct sts_ctx sts_ctx; /* opaque; owns all device state */

/* Grid (cell-volume figure, Sec. 3.2).  nx, ny >= 4 cells.  If dx (dy) is
   NULL the spacing is uniform lx/nx (ly/ny); otherwise dx[nx] (dy[ny]) are the
   positive cell widths.  Arrays are copied. */
typedef struct {
  int nx, ny;
  double lx, ly;
  const double *dx, *dy;
} sts_grid;

/* Solid obstacles: n closed rectangles of cells [i0, i1] x [j0, j1] (cell
   indices).  A cell is solid iff it lies in a rectangle.  With inlet/outlet
   in x, every rectangle must keep i0 >= 2 and i1 <= nx - 3.  Arrays copied. */
typedef struct {
  int n;
  const int *i0, *j0, *i1, *j1;
} sts_obstacles;

enum { STS_X_INLET_OUTLET = 0, STS_X_PERIODIC = 1 };
enum { STS_WALL_NOSLIP_ISOTHERMAL = 0, STS_WALL_SLIP_ADIABATIC = 1, STS_WALL_SLIP_JUMP = 2 };

/* Boundary conditions (test case of Sec. 4).  Wall and obstacle surfaces:
     STS_WALL_NOSLIP_ISOTHERMAL  eqs pl38/pl39 with zero slip and jump lengths;
     STS_WALL_SLIP_ADIABATIC     no shear, no heat flux;
     STS_WALL_SLIP_JUMP          velocity slip (pl38, zeta = 1.1466 kn / rho)
                                 and temperature jump (pl39, tau = 2.1904 kn
                                 / rho), rho of the node next to the surface;
                                 the normal derivative is taken over the half
                                 cell, so the wall conductance is that node's
                                 Gamma over d/2 + zeta (d/2 + tau).
     x_mode        inlet at x = 0 and outlet at x = Lx, or periodic in x.
     u_in, T_in    [ny] inlet-face u and T (NULL -> 1); inlet v = 0.
     p_in          inlet pressure (sets the inflow density p_in/T_in).
     wall_type     [0] bottom wall y = 0, [1] top wall y = Ly.
     wall_u        tangential velocity of each wall (no-slip and slip-jump;
                   moving walls of the particle frame, Sec. 4).
     wall_T        [nx] wall temperature per cell column (NULL -> 1).
     obstacle_T    surface temperature of the obstacles (at rest).
     gx, gy        body force per unit mass (rho g in eqs pl2, pl3).
     obstacle_type STS_WALL_NOSLIP_ISOTHERMAL or STS_WALL_SLIP_JUMP.
     kn            Knudsen number of the slip-jump surfaces, in the grid's
                   length unit (>= 0; unused by the other types).
   Arrays are copied. */
typedef struct {
  int x_mode;
  const double *u_in, *T_in;
  double p_in;
  int wall_type[2];
  double wall_u[2];
  const double *wall_T[2];
  double obstacle_T;
  double gx, gy;
  int obstacle_type;
  double kn;
} sts_bc;

/* scheme bits for sts_step: convective terms explicit (Forward Euler) or
   implicit (Backward Euler) in time, upwind or TVD (van Leer) in space
   (Sec. 3.1, the four variants).  STS_MIXED selects the mixed-precision
   form of any variant: the T, u and v coefficients are assembled and the
   Jacobi corrections formed in FP32, applied to the FP64 state through an
   FP64 defect of each equation; face densities, the pressure equation, the
   velocity update, the per-step constants and the residuals stay FP64.  The
   FP64 defect keeps the state and its increments in FP64 but is formed from
   the FP32-rounded coefficients, so loop 2 converges to the solution of the
   FP32-perturbed operator: results differ from the FP64 form at the level of
   FP32 rounding of the coefficients (about 1e-7 relative), which the defect
   does not remove. */
enum {
  STS_EXPLICIT = 0,
  STS_IMPLICIT = 1,
  STS_UPWIND = 0,
  STS_TVD = 2,
  STS_MIXED = 4,
  STS_SCHEME_MASK = 7
};

/* Device bytes the library needs for a grid (state, per-step constants,
   reduction buffers), for callers that bring their own workspace. */
sts_status sts_workspace_bytes(const sts_grid *grid, size_t *bytes);

/* Create a solver.  Ma, Re, Pr > 0, gamma > 1 give the coefficients of
   eqs pl2-pl6 (A = 1/(gamma Ma^2), B = 1/Re, energy equation in internal
   energy form).  hip_stream: a hipStream_t to order all work on, or NULL for
   a stream owned by the context.  workspace: device memory of at least
   sts_workspace_bytes(), owned by the caller and kept alive until
   sts_destroy, or NULL to let the library allocate.  The initial state is
   the inlet state of each row (u = u_in, v = 0, p = p_in, T = T_in) with
   the boundary values imposed.  *out is set only on success. */
sts_status sts_create(const sts_grid *grid, const sts_obstacles *obstacles,
                      double Ma, double Re, double Pr, double gamma,
                      const sts_bc *bc, void *hip_stream, void *workspace,
                      size_t workspace_bytes, sts_ctx **out);

/* Advance one time step of size dt > 0 with n_inner >= 1 Jacobi passes of
   loop 2 (scheme: STS_* bits).  Enqueues on the context's stream and returns
   without waiting.  The residuals of the last pass are reduced on the device
   and copied to pinned host memory.  With n_inner >= 2 the step prologue
   runs inside the first pass's launch (the same values). */
sts_status sts_step(sts_ctx *ctx, double dt, int n_inner, int scheme);

/* One time step of n_inner passes, each running loop 3 of the CPU
   algorithm (Sec. 3, its figure): the energy and pressure equations are
   solved n3 times per pass with the face densities, convective fluxes, rho,
   Gamma, u-hat, v-hat and d of the pass's iterate fixed, each solve taking T
   and p (the Jacobi neighbour values, the pressure work, the cell's T in the
   pressure equation) from the previous one; then the velocities.  n3 = 1 is
   sts_step (the GPU algorithm's pass).  Every scheme, STS_MIXED included
   (each solve then assembles the T, u and v coefficients in FP32 as
   sts_step does).  Allocates four field arrays on first use with n3 > 1
   (STS_ENOMEM if that fails).  STS_EINVAL for dt <= 0, n_inner < 1, n3
   outside [1, 64] or unknown scheme bits (state unchanged). */
sts_status sts_step_l3(sts_ctx *ctx, double dt, int n_inner, int n3, int scheme);

/* One time step whose loop 2 runs until convergence (Sec. 3.1: the inner
   iterations repeat until the step's solution has converged; Sec. 5: the
   maximal residuals are checked after every iteration): after each pass the
   residuals of sts_residuals are reduced on the device, and loop 2 stops at
   the first pass with
     max(max|du|, max|dv|, max|dT|, max|dp| / p_in) <= tol,
   or after max_inner passes, or at a non-finite value (sts_residuals then
   returns STS_ENONFINITE).  *n_inner receives the passes taken.  Every pass
   is the residual-producing variant.  The decision is taken on the device:
   passes queued after the converged one return without work, and the host
   waits for the stream only every second pass and once at the end (the
   call returns after the step is complete).  STS_EINVAL for dt <= 0,
   max_inner < 1, tol < 0 or not finite, unknown scheme bits, NULL n_inner
   (state unchanged). */
sts_status sts_step_tol(sts_ctx *ctx, double dt, int max_inner, double tol, int scheme,
                        int *n_inner);

/* sts_step_tol with loop 3 (n3 energy-pressure solves, as sts_step_l3) in
   every pass; n3 = 1 is sts_step_tol.  STS_EINVAL as sts_step_tol, and for
   n3 outside [1, 64]; STS_ENOMEM as sts_step_l3. */
sts_status sts_step_tol_l3(sts_ctx *ctx, double dt, int max_inner, int n3, double tol,
                           int scheme, int *n_inner);

/* Wait for the stream; out[6] = max|du|, max|dv|, max|dp|, max|dT| of the
   last pass over the unknowns, max|R| and sum R of the discrete continuity
   residual R = ((p/T)_new - (p/T)^{n-1}) dV/dt + net outflow of
   rho^u u_new dy and rho^v v_new dx.  Returns STS_ENONFINITE if the last
   step produced a non-finite value. */
sts_status sts_residuals(sts_ctx *ctx, double out[6]);

/* Per-pass residuals of the last sts_step_tol or sts_step_tol_l3 call
   (Sec. 5: the maximal residuals are read after every inner iteration of
   loop 2).  Waits for the stream, then copies min(max_rows, *rows) rows of
   {max|du|, max|dv|, max|dp|, max|dT|} of passes 1, 2, ... over the unknowns
   into out[max_rows][4] (host, caller-owned; NULL allowed when max_rows is
   0) and sets *rows to the passes recorded: the passes that call ran, at
   most 4096 (later passes are run but not recorded), and 0 after any other
   kind of step or before the first.  STS_EINVAL for NULL ctx or rows,
   max_rows < 0, or NULL out with max_rows > 0. */
sts_status sts_residual_history(sts_ctx *ctx, double *out, int max_rows, int *rows);

/* Wait for the stream and copy the current state to host arrays (layout
   above; caller-owned; NULL skips a field). */
sts_status sts_fields(sts_ctx *ctx, double *u, double *v, double *p,
                      double *T);

/* Replace the state by host arrays (NULL keeps a field), then impose the
   boundary values: inlet faces u = u_in, wall and obstacle faces 0, outlet
   face u = its upstream neighbour, solid cells T = obstacle_T, p = p_in.
   Synchronous. */
sts_status sts_set_fields(sts_ctx *ctx, const double *u, const double *v,
                          const double *p, const double *T);

/* Device pointers of the current state and the element index of (0,0) and
   row pitch (in doubles) of each array: element (i,j) of field f is
   f[origin + j*pitch + i].  Valid until the next sts_step. */
sts_status sts_field_ptrs(sts_ctx *ctx, double **u, double **v, double **p,
                          double **T, size_t *origin, size_t *pitch);

/* Per-step kernel timing with HIP events recorded on the context's stream:
   enable (1) or disable (0); enabling waits and clears the accumulation. */
sts_status sts_timing(sts_ctx *ctx, int enable);

/* Wait, then return the kernel time summed over the steps recorded since
   timing was enabled or last read: out_ms[0] step prologues, [1] the Jacobi
   passes, [2] residual reductions (with the residual copy), in milliseconds;
   out_n[0] = steps, out_n[1] = passes counted in [1].  A step with
   n_inner >= 2 runs its prologue inside its first pass: [0] then holds that
   fused launch and [1] the other n_inner - 1 passes.
   Clears the accumulation. */
sts_status sts_read_timing(sts_ctx *ctx, double out_ms[3], long long out_n[2]);

/* ---- loss, checkpoints and the adjoint of the explicit step ----
   The loss is built from the drag on the obstacles,
     D = sum over fluid cells next to a solid cell of
         A p dy (solid to the east) - A p dy (solid to the west)
         + B Gamma u_c dx / (dy/2) (solid to the south or north),
   A = 1/(gamma Ma^2), B = 1/Re, Gamma = sqrt(T), u_c = the cell-centre mean
   of the two u-faces (pressure and wall-shear force on the obstacles, in
   the units of the momentum equations, eqs pl2-pl3). */

/* Wait and return D of the current state. */
sts_status sts_drag(sts_ctx *ctx, double *out);

/* For callers that cannot allocate device or pinned memory (code under HIP
   graph capture, serving loops, harnesses that forbid hipMalloc): sts_drag
   without any allocation and without waiting.  Enqueues the drag D of the
   current state on the context's stream and writes it to d_out[0], device
   memory of the context's GPU owned by the caller (the value is there once
   the stream reaches this point).  The reduction's block partials (at most
   1024 doubles) live in a fixed array of the library that each GPU holds
   until the process ends, shared by every context on that GPU: calls that
   overlap on one GPU (other streams or threads) race on it.  The result is
   bitwise sts_drag's.  STS_EINVAL for NULL arguments, slip-jump obstacles
   (as sts_drag) or a reduction needing more partials than the array
   holds. */
sts_status sts_drag_noalloc(sts_ctx *ctx, double *d_out);

/* Device checkpoint storage: (re)allocate n >= 0 state slots owned by the
   context (n = 0 frees them; previous contents are lost).  STS_ENOMEM if
   the allocation fails.  sts_state_save copies the current state into a
   slot; sts_state_load makes a slot the current state.  Both enqueue on
   the context's stream; slot outside [0, n) -> STS_EINVAL. */
sts_status sts_state_slots(sts_ctx *ctx, int n);
sts_status sts_state_save(sts_ctx *ctx, int slot);
sts_status sts_state_load(sts_ctx *ctx, int slot);

/* Adjoint (reverse mode) of the explicit-scheme FP64 step, upwind or TVD,
   for channels with an inlet and an outlet (not periodic: STS_EINVAL).
   The adjoint state lambda is the derivative of a scalar loss L with
   respect to (u, v, p, T) of one time level; the parameters are the inlet
   profile u_in[ny] (held by the inlet faces at every level) and the wall
   temperatures wall_T[0][nx], wall_T[1][nx] (isothermal walls).

   sts_adjoint_begin: allocate the buffers for n_inner passes per step
   (library-owned, 12 n_inner + 23 field arrays: the iterates and the
   intermediates of every pass of one step, the adjoint temporaries and
   states), set lambda and the wall-temperature gradients to zero.  Every
   wall and obstacle type is supported, velocity-slip / temperature-jump
   surfaces (eqs pl38, pl39) included: their conductances and slip
   velocities are differentiated in the node's Gamma and rho.
   sts_adjoint_seed_drag: lambda += w dD/d(current state); call it with the
   current state at level n before the adjoint of step n.  The drag is that
   of no-slip obstacle surfaces (STS_EINVAL for slip-jump obstacles).
   sts_adjoint_seed: lambda += the host arrays w_u, w_v, w_p, w_T (layouts
   of sts_fields; NULL skips a field), i.e. the derivative of the loss
   term sum w . state of the current level; waits for the stream.
   STS_EINVAL for a non-finite entry (lambda unchanged).
   sts_adjoint_step: the current state must be level n-1 and lambda the
   derivative with respect to level n; recomputes the step (same dt,
   n_inner and scheme as the forward step) and replaces lambda by the
   derivative with respect to level n-1 (reverse of the n_inner passes and
   of the prologue), adding the wall-temperature contributions.  The
   current state is left unchanged.  With STS_MIXED the iterates are
   recomputed by the mixed-precision pass (the forward that produced the
   states) and the reverse is the FP64 step's transpose evaluated at them.
   STS_EINVAL for the implicit scheme bit or an n_inner other than
   sts_adjoint_begin's; STS_ESTATE before sts_adjoint_begin.
   sts_adjoint_read: wait and copy to host arrays (NULL skips): dL/du_in[ny]
   (the inlet entries of lambda_u: complete once the adjoint has reached
   the initial level), dL/dwall_T[0][nx], dL/dwall_T[1][nx], and lambda in
   the field layouts of sts_fields. */
sts_status sts_adjoint_begin(sts_ctx *ctx, int n_inner);
sts_status sts_adjoint_seed_drag(sts_ctx *ctx, double w);
sts_status sts_adjoint_seed(sts_ctx *ctx, const double *w_u, const double *w_v,
                            const double *w_p, const double *w_T);
sts_status sts_adjoint_step(sts_ctx *ctx, double dt, int n_inner, int scheme);
sts_status sts_adjoint_read(sts_ctx *ctx, double *g_uin, double *g_Tw0, double *g_Tw1,
                            double *lambda_u, double *lambda_v, double *lambda_p,
                            double *lambda_T);

/* Wait and copy to host arrays (layouts of sts_fields; NULL skips) the
   gradient with respect to the fields given to sts_set_fields at the
   current level: lambda mapped through the transpose of that call's
   boundary-value projection.  Entries the projection overwrites (inlet,
   wall and obstacle faces, solid cells) get 0; the outlet face is a copy of
   face nx-1, so its entry of lambda is added to that face's (when face
   nx-1 is an unknown) and the outlet entry itself gets 0.  At the initial
   level this is dL/d(initial fields).  STS_ESTATE before
   sts_adjoint_begin. */
sts_status sts_adjoint_read_state_grad(sts_ctx *ctx, double *g_u, double *g_v, double *g_p,
                                       double *g_T);

/* Release everything the context owns.  NULL-safe. */
void sts_destroy(sts_ctx *ctx);

/* Message of the last error on this thread ("" if none). */
const char *sts_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* STS_H */
