/*
 * ora_tlm.cc -- TEST INFRASTRUCTURE ONLY: the tangent-linear model of the
 * oracle.  ora.c compiled on the dual numbers of tlm.h (the same source,
 * every branch taken on the value), with a plain-double ABI: values and
 * ORA_TLM_K tangent directions ([K][n] arrays) go in and out separately.
 * Used by the adjoint tests (dot-product test: <lambda, TLM delta> against
 * <adjoint gradient, delta>).
 */
#include "tlm.h"

#include "ora.c"

#undef double

namespace {
void to_dual(dual *out, const ora_f64 *val, const ora_f64 *tan, size_t n) {
  for (size_t i = 0; i < n; i++) {
    out[i].v = val[i];
    for (int k = 0; k < ORA_TLM_K; k++) out[i].d[k] = tan ? tan[(size_t)k * n + i] : 0.0;
  }
}
void from_dual(const dual *in, ora_f64 *val, ora_f64 *tan, size_t n) {
  for (size_t i = 0; i < n; i++) {
    if (val) val[i] = in[i].v;
    if (tan)
      for (int k = 0; k < ORA_TLM_K; k++) tan[(size_t)k * n + i] = in[i].d[k];
  }
}
}  // namespace

extern "C" {

/* Setup as ora_setup in plain doubles, plus optional tangents ([K][len])
   of the inlet profile u_in and of the two wall temperature rows. */
struct tlm_setup {
  int nx, ny;
  const ora_f64 *dx, *dy;
  int periodic;
  int n_obst;
  const int *oi0, *oj0, *oi1, *oj1;
  ora_f64 Ma, Re, Pr, gamma;
  const ora_f64 *u_in, *T_in;
  ora_f64 p_in;
  int wall_type[2];
  ora_f64 wall_u[2];
  const ora_f64 *wall_T[2];
  ora_f64 obstacle_T, gx, gy;
  int obstacle_type;
  ora_f64 kn;
  const ora_f64 *u_in_t, *wall_T_t[2];
};

int tlm_k(void) { return ORA_TLM_K; }

ora_ctx *tlm_create(const tlm_setup *s) {
  const int nx = s->nx, ny = s->ny;
  dual *dx = new dual[nx], *dy = new dual[ny], *uin = new dual[ny], *tin = new dual[ny];
  dual *tw0 = new dual[nx], *tw1 = new dual[nx];
  to_dual(dx, s->dx, nullptr, nx);
  to_dual(dy, s->dy, nullptr, ny);
  to_dual(uin, s->u_in, s->u_in_t, ny);
  to_dual(tin, s->T_in, nullptr, ny);
  to_dual(tw0, s->wall_T[0], s->wall_T_t[0], nx);
  to_dual(tw1, s->wall_T[1], s->wall_T_t[1], nx);
  ora_setup d;
  d.nx = nx;
  d.ny = ny;
  d.dx = dx;
  d.dy = dy;
  d.periodic = s->periodic;
  d.n_obst = s->n_obst;
  d.oi0 = s->oi0;
  d.oj0 = s->oj0;
  d.oi1 = s->oi1;
  d.oj1 = s->oj1;
  d.Ma = s->Ma;
  d.Re = s->Re;
  d.Pr = s->Pr;
  d.gamma = s->gamma;
  d.u_in = uin;
  d.T_in = tin;
  d.p_in = s->p_in;
  d.wall_type[0] = s->wall_type[0];
  d.wall_type[1] = s->wall_type[1];
  d.wall_u[0] = s->wall_u[0];
  d.wall_u[1] = s->wall_u[1];
  d.wall_T[0] = tw0;
  d.wall_T[1] = tw1;
  d.obstacle_T = s->obstacle_T;
  d.gx = s->gx;
  d.gy = s->gy;
  d.obstacle_type = s->obstacle_type;
  d.kn = s->kn;
  ora_ctx *c = ora_create(&d);
  delete[] dx;
  delete[] dy;
  delete[] uin;
  delete[] tin;
  delete[] tw0;
  delete[] tw1;
  return c;
}

void tlm_destroy(ora_ctx *c) { ora_destroy(c); }

static void sizes(const ora_ctx *c, size_t n[4]) {
  n[0] = (size_t)(c->nx + 1) * c->ny;
  n[1] = (size_t)c->nx * (c->ny + 1);
  n[2] = n[3] = (size_t)c->nx * c->ny;
}

/* Values (NULL keeps a field) and tangents ([K][n], NULL = zero). */
void tlm_set_fields(ora_ctx *c, const ora_f64 *const val[4], const ora_f64 *const tan[4]) {
  size_t n[4];
  sizes(c, n);
  dual *f[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int q = 0; q < 4; q++)
    if (val[q]) {
      f[q] = new dual[n[q]];
      to_dual(f[q], val[q], tan[q], n[q]);
    }
  ora_set_fields(c, f[0], f[1], f[2], f[3]);
  for (int q = 0; q < 4; q++) delete[] f[q];
}

void tlm_get_fields(const ora_ctx *c, ora_f64 *const val[4], ora_f64 *const tan[4]) {
  size_t n[4];
  sizes(c, n);
  const dual *f[4] = {c->u, c->v, c->p, c->T};
  for (int q = 0; q < 4; q++) from_dual(f[q], val[q], tan[q], n[q]);
}

void tlm_step(ora_ctx *c, ora_f64 dt, int n_inner, int scheme) { ora_step(c, dt, n_inner, scheme); }

void tlm_set_threads(int n) { ora_set_threads(n); }

}  // extern "C"
