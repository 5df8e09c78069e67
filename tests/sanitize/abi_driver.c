/*
 * Host-side checks of the C ABI built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py): every entry point
 * refuses invalid arguments with STS_EINVAL and a message, the workspace
 * size (a function of nx and ny) is computed for valid grids, and sts_create's failure paths (no GPU
 * in the build container, so a valid call fails at the first device call)
 * release what they built.  Prints one line per case; exit status 0 when
 * every check holds.
 */
#include <stdio.h>
#include <string.h>

#include "sts.h"

static int bad = 0;
static void expect(int cond, const char *what) {
  if (!cond) {
    printf("FAIL %s (last error: %s)\n", what, sts_last_error());
    bad = 1;
  }
}
static void einval(sts_status s, const char *what) {
  expect(s == STS_EINVAL && strlen(sts_last_error()) > 0, what);
}

int main(void) {
  double dx[8] = {0.1, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1, 0.1};
  double bad_dx[8] = {0.1, 0.1, -0.1, 0.1, 0.1, 0.1, 0.1, 0.1};
  sts_grid g = {8, 6, 1.0, 1.0, NULL, NULL};
  size_t b = 0;
  expect(sts_workspace_bytes(&g, &b) == STS_OK && b > 0, "workspace bytes of a valid grid");
  sts_grid g2 = g;
  g2.dx = dx;
  size_t b2 = 0;
  expect(sts_workspace_bytes(&g2, &b2) == STS_OK && b2 == b, "explicit widths, same bytes");
  einval(sts_workspace_bytes(NULL, &b), "workspace: NULL grid");
  einval(sts_workspace_bytes(&g, NULL), "workspace: NULL bytes");
  sts_grid g3 = g;
  g3.nx = 3;
  einval(sts_workspace_bytes(&g3, &b), "workspace: nx < 4");

  sts_bc bc;
  memset(&bc, 0, sizeof bc);
  bc.p_in = 1.0;
  bc.obstacle_T = 1.0;
  sts_ctx *ctx = NULL;
  einval(sts_create(NULL, NULL, 1, 10, 0.7, 1.4, &bc, NULL, NULL, 0, &ctx), "create: NULL grid");
  einval(sts_create(&g, NULL, 1, 10, 0.7, 1.4, &bc, NULL, NULL, 0, NULL), "create: NULL out");
  einval(sts_create(&g, NULL, 0.0, 10, 0.7, 1.4, &bc, NULL, NULL, 0, &ctx), "create: Ma = 0");
  einval(sts_create(&g, NULL, 1, -10, 0.7, 1.4, &bc, NULL, NULL, 0, &ctx), "create: Re < 0");
  einval(sts_create(&g, NULL, 1, 10, 0.7, 1.0, &bc, NULL, NULL, 0, &ctx), "create: gamma = 1");
  sts_bc bc2 = bc;
  bc2.wall_type[0] = 7;
  einval(sts_create(&g, NULL, 1, 10, 0.7, 1.4, &bc2, NULL, NULL, 0, &ctx), "create: wall type");
  bc2 = bc;
  bc2.x_mode = 5;
  einval(sts_create(&g, NULL, 1, 10, 0.7, 1.4, &bc2, NULL, NULL, 0, &ctx), "create: x mode");
  bc2 = bc;
  bc2.kn = -1.0;
  einval(sts_create(&g, NULL, 1, 10, 0.7, 1.4, &bc2, NULL, NULL, 0, &ctx), "create: kn < 0");
  g3 = g;
  g3.dx = bad_dx;
  einval(sts_create(&g3, NULL, 1, 10, 0.7, 1.4, &bc, NULL, NULL, 0, &ctx), "create: negative width");
  g3 = g;
  g3.ly = -1.0;
  einval(sts_create(&g3, NULL, 1, 10, 0.7, 1.4, &bc, NULL, NULL, 0, &ctx), "create: negative length");
  int i0[1] = {0}, j0[1] = {1}, i1[1] = {2}, j1[1] = {2};
  sts_obstacles ob = {1, i0, j0, i1, j1};
  einval(sts_create(&g, &ob, 1, 10, 0.7, 1.4, &bc, NULL, NULL, 0, &ctx),
         "create: obstacle at the inlet");
  expect(ctx == NULL, "no context after refused calls");
  /* a valid call: fails at the first device call where there is no GPU,
     and must release everything it built on the way */
  sts_status s = sts_create(&g, NULL, 1, 10, 0.7, 1.4, &bc, NULL, NULL, 0, &ctx);
  printf("create with valid arguments: %d (%s)\n", (int)s, sts_last_error());
  if (s == STS_OK) {
    sts_destroy(ctx);
    ctx = NULL;
  } else {
    expect(s == STS_EDEVICE || s == STS_ENOMEM, "valid create fails only at the device");
    expect(ctx == NULL, "no context after a failed create");
  }

  /* every entry point refuses a NULL context */
  double out[8];
  int n = 0;
  long long nn[2];
  double *pp = NULL;
  size_t o1, o2;
  einval(sts_step(NULL, 0.1, 1, 0), "step");
  einval(sts_step_l3(NULL, 0.1, 1, 2, 0), "step_l3");
  einval(sts_step_tol(NULL, 0.1, 5, 1e-6, 0, &n), "step_tol");
  einval(sts_step_tol_l3(NULL, 0.1, 5, 2, 1e-6, 0, &n), "step_tol_l3");
  einval(sts_residuals(NULL, out), "residuals");
  einval(sts_residual_history(NULL, out, 1, &n), "residual_history");
  einval(sts_fields(NULL, out, NULL, NULL, NULL), "fields");
  einval(sts_set_fields(NULL, out, NULL, NULL, NULL), "set_fields");
  einval(sts_field_ptrs(NULL, &pp, &pp, &pp, &pp, &o1, &o2), "field_ptrs");
  einval(sts_timing(NULL, 1), "timing");
  einval(sts_read_timing(NULL, out, nn), "read_timing");
  einval(sts_drag(NULL, out), "drag");
  einval(sts_drag_noalloc(NULL, out), "drag_noalloc");
  einval(sts_state_slots(NULL, 1), "state_slots");
  einval(sts_state_save(NULL, 0), "state_save");
  einval(sts_state_load(NULL, 0), "state_load");
  einval(sts_adjoint_begin(NULL, 2), "adjoint_begin");
  einval(sts_adjoint_seed_drag(NULL, 1.0), "adjoint_seed_drag");
  einval(sts_adjoint_seed(NULL, out, NULL, NULL, NULL), "adjoint_seed");
  einval(sts_adjoint_step(NULL, 0.1, 2, 0), "adjoint_step");
  einval(sts_adjoint_read(NULL, out, NULL, NULL, NULL, NULL, NULL, NULL), "adjoint_read");
  einval(sts_adjoint_read_state_grad(NULL, out, NULL, NULL, NULL), "adjoint_read_state_grad");
  sts_destroy(NULL);
  printf(bad ? "FAILED\n" : "OK\n");
  return bad;
}
