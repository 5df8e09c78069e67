/*
 * sts3.h -- C ABI of the three-dimensional SIMPLE-TS step in libsts.so.
 *
 * The paper (Shterev, arXiv 1802.04243) gives the method in two dimensions
 * (Sec. 2, eqs pl4-pl7; Sec. 3.2, eqs pl8-pl33; pass order of Appendix A)
 * and names 3-D flow as its next step (Conclusions).  This interface runs the
 * same step on a staggered Cartesian grid in x, y, z: velocity component a on
 * the a-faces, p and T at the cell centres; every 2-D formula is read per
 * pair of directions (face densities and fluxes through the face areas,
 * normal stresses with the 4/3 factor, tangential shear with Gamma bilinear
 * on the cell edges, the cross-diffusion of the stress for every tangential
 * direction, energy with six conduction faces, the 3-D dissipation, the
 * pressure equation with six neighbours).  Every computation runs in HIP
 * kernels on the GPU the context was created on.
 *
 * Conventions (as sts.h): sts_status return codes, messages through
 * sts_last_error(), nondimensional FP64 values.  Host field arrays are dense,
 * x fastest, then y, then z:
 *   u [nz][ny][nx+1], v [nz][ny+1][nx], w [nz+1][ny][nx], p, T [nz][ny][nx].
 * One context per host thread; calls on one context are ordered on its HIP
 * stream; sts3_step is asynchronous, sts3_residuals and sts3_fields wait.
 */
#ifndef STS3_H
#define STS3_H

#include "sts.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sts3_ctx sts3_ctx; /* opaque; owns all device state */

/* Boundary kind per direction: x takes STS3_INLET_OUTLET (supersonic inlet
   at x = 0 with u = u_in, T = T_in, tangential velocities 0 and inflow
   density p_in/T_in; zero-gradient outlet at x = Lx) or STS3_PERIODIC; y and
   z take STS3_WALLS (a wall at each end) or STS3_PERIODIC. */
enum { STS3_WALLS = 0, STS3_PERIODIC = 1, STS3_INLET_OUTLET = 2 };
/* Wall types: no-slip isothermal (eqs pl38, pl39 with zero slip and jump
   lengths; half-cell conductances with the mean of the node's and the
   wall's Gamma for shear, their harmonic mean for conduction), or slip
   adiabatic (no shear, no heat flux). */
enum { STS3_NOSLIP = 0, STS3_SLIP = 1 };

typedef struct {
  int n[3];                 /* cells in x, y, z; each >= 4                   */
  const double *d[3];       /* [n[e]] positive cell widths per direction     */
  int bc[3];                /* boundary kind per direction                   */
  int wall_type[3][2];      /* per wall direction, low / high wall           */
  double wall_vel[3][2][3]; /* velocity of each no-slip wall (tangential)    */
  double wall_T[3][2];      /* temperature of each no-slip wall (> 0)        */
  double Ma, Re, Pr, gamma; /* > 0, > 0, > 0, > 1                            */
  double u_in, T_in, p_in;  /* inlet state (T_in, p_in > 0)                  */
  double g[3];              /* body force per unit mass                      */
} sts3_setup;

/* Create a solver (arrays copied).  hip_stream: a hipStream_t to order all
   work on, or NULL for a stream owned by the context.  The library allocates
   its device memory (29 field arrays of (nz+5)(ny+5) rows of a padded x
   pitch).  Initial state: u = u_in (inlet/outlet in x) or 0, v = w = 0,
   p = p_in, T = T_in, with the boundary values imposed.  STS_EINVAL for an
   invalid setup (x WALLS, y or z INLET_OUTLET, n < 4, non-positive widths or
   parameters); STS_ENOMEM, STS_EDEVICE.  *out is set only on success. */
sts_status sts3_create(const sts3_setup *setup, void *hip_stream, sts3_ctx **out);

/* Device bytes sts3_create allocates for a grid. */
sts_status sts3_device_bytes(const int n[3], size_t *bytes);

/* One time step of size dt > 0: the prologue (per-step constants from the
   current state as level n-1) and n_inner >= 1 Jacobi passes in the order of
   Appendix A (scheme: STS_EXPLICIT / STS_IMPLICIT | STS_UPWIND / STS_TVD of
   sts.h; STS_MIXED is not supported: STS_EINVAL).  Asynchronous; the
   residuals of the last pass are reduced on the device. */
sts_status sts3_step(sts3_ctx *ctx, double dt, int n_inner, int scheme);

/* Wait; out[7] = max|du|, max|dv|, max|dw|, max|dp|, max|dT| of the last pass
   over the unknowns, max|R| and sum R of the discrete continuity residual
   R = ((p/T)_new - (p/T)^{n-1}) dV/dt + net outflow of rho^f q_new through
   the six faces.  STS_ENONFINITE if the last step produced a non-finite
   value. */
sts_status sts3_residuals(sts3_ctx *ctx, double out[7]);

/* Wait and copy the state to host arrays (layout above; order u, v, w, p, T;
   NULL skips a field). */
sts_status sts3_fields(sts3_ctx *ctx, double *const q[5]);

/* Replace the state by host arrays (NULL keeps a field), then impose the
   boundary values (inlet faces u = u_in, wall faces normal velocity 0, outlet
   face u = its upstream neighbour, last face of a periodic direction = face
   0).  Synchronous. */
sts_status sts3_set_fields(sts3_ctx *ctx, const double *const q[5]);

/* Release everything the context owns.  NULL-safe. */
void sts3_destroy(sts3_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
