// Host runtime of libsts.so: the C ABI declared in include/sts.h.
//
// Owns the device state (two ping-pong state buffers, four per-step constant
// arrays, boundary data, reduction buffers), validates every argument, and
// drives one time step as: prologue kernel, n_inner pass kernels (buffer swap,
// no copy), residual kernel + finalize, and one asynchronous copy of the
// reduced residuals to pinned host memory -- the only device-to-host traffic
// of a step (Sec. 5 of the paper: only the max residuals of loop 2 cross).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sts.h"

#include "sts_internal.h"

using namespace sts;

namespace {
thread_local std::string g_err;

sts_status fail(sts_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}
#define HIPCHK(call)                                                     \
  do {                                                                   \
    hipError_t e_ = (call);                                              \
    if (e_ != hipSuccess)                                                \
      return fail(STS_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
  long pitch, rows, off;
  size_t field_bytes;  // one FP64 field array
  size_t mask_bytes;
};
Layout make_layout(int nx, int ny) {
  Layout L;
  L.pitch = (long)align_up((size_t)(XO + nx + 1 + XPAD), 32);
  L.rows = ny + 1 + 2 * YO;
  L.off = (long)YO * L.pitch + XO;
  L.field_bytes = align_up((size_t)L.pitch * L.rows * sizeof(double), 256);
  L.mask_bytes = align_up((size_t)L.pitch * L.rows, 256);
  return L;
}
struct Sizes {
  size_t state, consts, mask, small, partials, res, hist, total;
};
Sizes make_sizes(int nx, int ny, const Layout &L) {
  Sizes S;
  S.state = 8 * L.field_bytes;   // two buffers of u, v, p, T
  S.consts = 6 * L.field_bytes;  // C_u, C_v, C_T, C_p, face mass fluxes
  S.mask = L.mask_bytes;
  // 1-D boundary arrays (see ctx_build), tile flags
  const size_t tiles = (size_t)((nx + TX - 1) / TX) * ((ny + TY - 1) / TY);
  S.small = align_up(sizeof(double) * ((size_t)6 * (nx + 2 * XPAD) + 6 * (ny + 2 * XPAD) +
                                        4 * (size_t)ny + 4 * (size_t)nx + 2 * (size_t)(nx + 1)),
                     256) +
            align_up(tiles, 256);
  S.partials = align_up(sizeof(double) * NRES * (tiles + RES_BLOCKS), 256);
  S.res = 256;  // NRES doubles, then the loop-2 control block at RES_CTL
  S.hist = align_up(sizeof(double) * 4 * HIST_CAP, 256);  // per-pass residuals of loop 2
  S.total = S.state + S.consts + S.mask + S.small + S.partials + S.res + S.hist;
  return S;
}

}  // namespace

struct sts_ctx {
  int nx, ny, per;
  Layout L;
  Sizes S;
  Params P;
  hipStream_t stream;
  bool own_stream;
  int device;
  char *base;
  bool own_mem;
  State st[2];
  int cur;
  Consts C;
  Resid X;
  double *dres;   // NRES residuals; at RES_CTL the loop-2 control block
  double *hres;   // pinned: NRES residuals; at RES_CTL host copies of it
  double *dhist;  // [HIST_CAP][4] per-pass residuals of the last tolerance step
  int hist_rows = 0;
  hipEvent_t l2ev[2] = {nullptr, nullptr};
  bool stepped;
  int last_scheme;
  // host copies of the boundary data
  std::vector<double> dx, dy, u_in, T_in, Tw[2];
  std::vector<unsigned char> solid;  // [ny][nx]
  double p_in, obsT;
  int otype = STS_WALL_NOSLIP_ISOTHERMAL;
  bool slip_jump = false;  // some wall or obstacle surface is slip-jump
  // adjoint of the explicit step (allocated on first use, library-owned):
  // the iterates x_0 .. x_K of a step, one pass's intermediates, the
  // adjoints of the intermediates, two adjoint states, the adjoints of the
  // step constants and of the wall temperatures; device state slots for
  // checkpoints; drag reduction buffers
  char *adj_mem = nullptr;
  int adj_K = 0;
  bool adj_frames = false;  // iterate buffers hold the boundary values
  std::vector<State> it;   // it[1..K]: the iterates of a step (it[0] unused)
  std::vector<Inter> Iv;   // Iv[1..K]: the intermediates of each pass
  AdjTmp A{};
  State lam[2]{};
  int lcur = 0;
  Consts lC{};
  double *gtw = nullptr;  // [2 nx]
  size_t adj_clear_bytes = 0;
  char *slot_mem = nullptr;
  int nslots = 0;
  // loop 3: two (T, p) pairs of the energy-pressure solves of a pass
  // (allocated on first use; frames hold the ghost values p = T = 1)
  char *l3_mem = nullptr;
  double *l3T[2] = {nullptr, nullptr}, *l3p[2] = {nullptr, nullptr};
  double *aux = nullptr;   // drag partials + result
  double *haux = nullptr;  // pinned
  // timing
  bool timing;
  std::vector<hipEvent_t> ev;  // 4 per recorded step
  int ev_used;
  long long t_steps, t_passes;
  double t_ms[3];
};

extern "C" const char *sts_last_error(void) { return g_err.c_str(); }

sts_status sts::report_error(sts_status s, const char *msg) {
  g_err = msg;
  return s;
}

namespace {
// Block partials of the drag reduction of sts_drag_noalloc: a fixed array
// that every GPU running this library holds in its copy of the code object
// (8 KiB, until the process ends).  Host code never names the array after
// set-up: sts_create resolves its device address once per device, with that
// device current, and the entry point passes that address to the kernels.
constexpr int NOALLOC_PARTIALS = 1024;
static __device__ __align__(256) double scratch[NOALLOC_PARTIALS];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch[MAX_DEVICES] = {};

sts_status resolve_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return fail(STS_EDEVICE, "device %d out of range", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return STS_OK;
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(STS_EDEVICE, "hipGetSymbolAddress of the drag scratch array: %s", hipGetErrorString(e));
  g_scratch[device] = (double *)p;
  return STS_OK;
}
double *scratch_of(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[device];
}
}  // namespace

extern "C" sts_status sts_workspace_bytes(const sts_grid *grid, size_t *bytes) {
  if (!grid || !bytes) return fail(STS_EINVAL, "NULL argument");
  if (grid->nx < 4 || grid->ny < 4) return fail(STS_EINVAL, "nx, ny must be >= 4");
  Layout L = make_layout(grid->nx, grid->ny);
  *bytes = make_sizes(grid->nx, grid->ny, L).total;
  return STS_OK;
}

namespace {

sts_status validate(const sts_grid *g, const sts_obstacles *ob, double Ma,
                    double Re, double Pr, double gamma, const sts_bc *bc) {
  if (!g || !bc) return fail(STS_EINVAL, "grid and bc are required");
  if (g->nx < 4 || g->ny < 4) return fail(STS_EINVAL, "nx, ny must be >= 4");
  if ((long)g->nx * g->ny > (1L << 31)) return fail(STS_EINVAL, "grid too large");
  if (!g->dx && !(g->lx > 0 && isfinite(g->lx))) return fail(STS_EINVAL, "lx must be > 0");
  if (!g->dy && !(g->ly > 0 && isfinite(g->ly))) return fail(STS_EINVAL, "ly must be > 0");
  if (g->dx)
    for (int i = 0; i < g->nx; i++)
      if (!(g->dx[i] > 0 && isfinite(g->dx[i]))) return fail(STS_EINVAL, "dx[%d] must be > 0", i);
  if (g->dy)
    for (int j = 0; j < g->ny; j++)
      if (!(g->dy[j] > 0 && isfinite(g->dy[j]))) return fail(STS_EINVAL, "dy[%d] must be > 0", j);
  if (!(Ma > 0 && isfinite(Ma)) || !(Re > 0 && isfinite(Re)) ||
      !(Pr > 0 && isfinite(Pr)) || !(gamma > 1 && isfinite(gamma)))
    return fail(STS_EINVAL, "need Ma, Re, Pr > 0 and gamma > 1");
  if (bc->x_mode != STS_X_INLET_OUTLET && bc->x_mode != STS_X_PERIODIC)
    return fail(STS_EINVAL, "unknown x_mode %d", bc->x_mode);
  for (int w = 0; w < 2; w++)
    if (bc->wall_type[w] != STS_WALL_NOSLIP_ISOTHERMAL &&
        bc->wall_type[w] != STS_WALL_SLIP_ADIABATIC && bc->wall_type[w] != STS_WALL_SLIP_JUMP)
      return fail(STS_EINVAL, "unknown wall_type[%d] = %d", w, bc->wall_type[w]);
  if (bc->obstacle_type != STS_WALL_NOSLIP_ISOTHERMAL && bc->obstacle_type != STS_WALL_SLIP_JUMP)
    return fail(STS_EINVAL, "obstacle_type must be no-slip isothermal or slip-jump (%d)",
                bc->obstacle_type);
  if (!(bc->kn >= 0 && isfinite(bc->kn))) return fail(STS_EINVAL, "kn must be >= 0 and finite");
  if (!(bc->p_in > 0 && isfinite(bc->p_in))) return fail(STS_EINVAL, "p_in must be > 0");
  if (!(bc->obstacle_T > 0 && isfinite(bc->obstacle_T)))
    return fail(STS_EINVAL, "obstacle_T must be > 0");
  for (int j = 0; j < g->ny; j++) {
    if (bc->T_in && !(bc->T_in[j] > 0 && isfinite(bc->T_in[j])))
      return fail(STS_EINVAL, "T_in[%d] must be > 0", j);
    if (bc->u_in && !isfinite(bc->u_in[j])) return fail(STS_EINVAL, "u_in[%d] not finite", j);
  }
  for (int w = 0; w < 2; w++)
    if (bc->wall_T[w])
      for (int i = 0; i < g->nx; i++)
        if (!(bc->wall_T[w][i] > 0 && isfinite(bc->wall_T[w][i])))
          return fail(STS_EINVAL, "wall_T[%d][%d] must be > 0", w, i);
  if (!isfinite(bc->wall_u[0]) || !isfinite(bc->wall_u[1]) || !isfinite(bc->gx) ||
      !isfinite(bc->gy))
    return fail(STS_EINVAL, "wall_u, gx, gy must be finite");
  if (ob && ob->n > 0) {
    if (!ob->i0 || !ob->j0 || !ob->i1 || !ob->j1) return fail(STS_EINVAL, "obstacle arrays are NULL");
    for (int k = 0; k < ob->n; k++) {
      if (ob->i0[k] > ob->i1[k] || ob->j0[k] > ob->j1[k] || ob->i0[k] < 0 ||
          ob->j0[k] < 0 || ob->i1[k] >= g->nx || ob->j1[k] >= g->ny)
        return fail(STS_EINVAL, "obstacle %d outside the grid or empty", k);
      if (bc->x_mode == STS_X_INLET_OUTLET && (ob->i0[k] < 2 || ob->i1[k] > g->nx - 3))
        return fail(STS_EINVAL, "obstacle %d touches the inlet or outlet", k);
    }
  } else if (ob && ob->n < 0) {
    return fail(STS_EINVAL, "negative obstacle count");
  }
  return STS_OK;
}

bool u_is_unknown(const sts_ctx *c, int i, int j) {
  if (!c->per && (i <= 0 || i >= c->nx)) return false;
  if (c->per && i >= c->nx) return false;
  const int l = (i - 1 + c->nx) % c->nx;
  return !c->solid[(size_t)j * c->nx + l] && !c->solid[(size_t)j * c->nx + i];
}
bool v_is_unknown(const sts_ctx *c, int i, int j) {
  if (j <= 0 || j >= c->ny) return false;
  return !c->solid[(size_t)(j - 1) * c->nx + i] && !c->solid[(size_t)j * c->nx + i];
}

// Impose the boundary values on host state arrays (dense layout).
void project(const sts_ctx *c, double *u, double *v, double *p, double *T) {
  const int nx = c->nx, ny = c->ny;
  for (int j = 0; j < ny; j++) {
    for (int i = 0; i < nx; i++)
      if (c->solid[(size_t)j * nx + i]) {
        T[(size_t)j * nx + i] = c->obsT;
        p[(size_t)j * nx + i] = c->p_in;
      }
    double *ur = u + (size_t)j * (nx + 1);
    for (int i = 0; i < nx; i++) {
      if (!c->per && i == 0) ur[0] = c->u_in[j];
      else if (!u_is_unknown(c, i, j)) ur[i] = 0.0;
    }
    ur[nx] = c->per ? ur[0] : ur[nx - 1];
  }
  for (int j = 0; j <= ny; j++)
    for (int i = 0; i < nx; i++)
      if (!v_is_unknown(c, i, j)) v[(size_t)j * nx + i] = 0.0;
}

// Upload dense host fields into device buffer b (frame values untouched).
sts_status upload(sts_ctx *c, int b, const double *u, const double *v,
                  const double *p, const double *T) {
  const int nx = c->nx, ny = c->ny;
  const long P = c->L.pitch;
  HIPCHK(hipMemcpy2DAsync(c->st[b].u + c->L.off, P * 8, u, (nx + 1) * 8, (nx + 1) * 8, ny,
                          hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpy2DAsync(c->st[b].v + c->L.off, P * 8, v, nx * 8, nx * 8, ny + 1,
                          hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpy2DAsync(c->st[b].p + c->L.off, P * 8, p, nx * 8, nx * 8, ny,
                          hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpy2DAsync(c->st[b].T + c->L.off, P * 8, T, nx * 8, nx * 8, ny,
                          hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return STS_OK;
}

sts_status fill_frames(sts_ctx *c) {
  // every field buffer: u, v = 0 and p, T = 1 outside the domain
  const size_t n = (size_t)c->L.pitch * c->L.rows;
  std::vector<double> one(n, 1.0);
  for (int b = 0; b < 2; b++) {
    HIPCHK(hipMemsetAsync(c->st[b].u, 0, n * 8, c->stream));
    HIPCHK(hipMemsetAsync(c->st[b].v, 0, n * 8, c->stream));
    HIPCHK(hipMemcpyAsync(c->st[b].p, one.data(), n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->st[b].T, one.data(), n * 8, hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(hipMemsetAsync(c->C.Cu, 0, 6 * c->L.field_bytes, c->stream));  // C_*, fluxes
  HIPCHK(hipStreamSynchronize(c->stream));
  return STS_OK;
}

sts_status build(sts_ctx *c, const sts_bc *bc) {
  const int nx = c->nx, ny = c->ny;
  Params &P = c->P;
  char *q = c->base;
  for (int b = 0; b < 2; b++) {
    c->st[b].u = (double *)q; q += c->L.field_bytes;
    c->st[b].v = (double *)q; q += c->L.field_bytes;
    c->st[b].p = (double *)q; q += c->L.field_bytes;
    c->st[b].T = (double *)q; q += c->L.field_bytes;
  }
  c->C.Cu = (double *)q; q += c->L.field_bytes;
  c->C.Cv = (double *)q; q += c->L.field_bytes;
  c->C.CT = (double *)q; q += c->L.field_bytes;
  c->C.Cp = (double *)q; q += c->L.field_bytes;
  c->X.gu = (double *)q; q += c->L.field_bytes;
  c->X.gv = (double *)q; q += c->L.field_bytes;
  unsigned char *fl = (unsigned char *)q; q += c->S.mask;
  char *small = q; q += c->S.small;
  c->X.partials = (double *)q; q += c->S.partials;
  c->dres = (double *)q; q += c->S.res;
  c->dhist = (double *)q; q += c->S.hist;

  // host-side boundary data
  std::vector<double> hs;
  auto put = [&](const std::vector<double> &a) {
    size_t at = hs.size();
    hs.insert(hs.end(), a.begin(), a.end());
    return at;
  };
  // geometry factors (see Params): widths and inverse widths per column,
  // width sums, their inverses and interpolation weights per face
  auto geometry = [](const std::vector<double> &d, int n, bool per,
                     std::vector<double> out[6]) {
    auto idx = [&](int i) {
      return per ? ((i % n) + n) % n : (i < 0 ? 0 : (i >= n ? n - 1 : i));
    };
    for (int q = 0; q < 6; q++) out[q].resize(n + 2 * XPAD);
    for (int i = -XPAD; i < n + XPAD; i++) {
      const double w = d[idx(i)], wl = d[idx(i - 1)], sum = wl + w;
      out[0][i + XPAD] = w;
      out[1][i + XPAD] = 1.0 / w;
      out[2][i + XPAD] = sum;
      out[3][i + XPAD] = 1.0 / sum;
      out[4][i + XPAD] = w / sum;
      out[5][i + XPAD] = wl / sum;
    }
  };
  std::vector<double> gxv[6], gyv[6];
  geometry(c->dx, nx, c->per != 0, gxv);
  geometry(c->dy, ny, false, gyv);
  std::vector<double> sqTin(ny), rhoin(ny), sqTw0(nx), sqTw1(nx), sqTwu0(nx + 1), sqTwu1(nx + 1);
  for (int j = 0; j < ny; j++) {
    sqTin[j] = sqrt(c->T_in[j]);
    rhoin[j] = c->p_in / c->T_in[j];
  }
  for (int i = 0; i < nx; i++) {
    sqTw0[i] = sqrt(c->Tw[0][i]);
    sqTw1[i] = sqrt(c->Tw[1][i]);
  }
  // wall temperature at the x-position of u-face i: linear between the two
  // neighbouring cell columns
  for (int i = 0; i <= nx; i++) {
    int l = i - 1, r = i;
    if (c->per) { l = (l + nx) % nx; r = r % nx; }
    else { if (l < 0) l = 0; if (r > nx - 1) r = nx - 1; }
    const double wl = gxv[4][i + XPAD], wr = gxv[5][i + XPAD];
    sqTwu0[i] = sqrt(wl * c->Tw[0][l] + wr * c->Tw[0][r]);
    sqTwu1[i] = sqrt(wl * c->Tw[1][l] + wr * c->Tw[1][r]);
  }
  auto interleave = [](const std::vector<double> *g) {
    std::vector<double> a(6 * g[0].size());
    for (size_t i = 0; i < g[0].size(); i++)
      for (int q = 0; q < 6; q++) a[6 * i + q] = g[q][i];
    return a;
  };
  const size_t o_gx = put(interleave(gxv)), o_gy = put(interleave(gyv));
  std::vector<double> inl(4 * (size_t)ny), wl(4 * (size_t)nx), wu(2 * (size_t)(nx + 1));
  for (int j = 0; j < ny; j++) {
    inl[4 * j] = c->u_in[j];
    inl[4 * j + 1] = c->T_in[j];
    inl[4 * j + 2] = sqTin[j];
    inl[4 * j + 3] = rhoin[j];
  }
  for (int i = 0; i < nx; i++) {
    wl[4 * i] = c->Tw[0][i];
    wl[4 * i + 1] = c->Tw[1][i];
    wl[4 * i + 2] = sqTw0[i];
    wl[4 * i + 3] = sqTw1[i];
  }
  for (int i = 0; i <= nx; i++) {
    wu[2 * i] = sqTwu0[i];
    wu[2 * i + 1] = sqTwu1[i];
  }
  const size_t o_inl = put(inl), o_wl = put(wl), o_wu = put(wu);
  HIPCHK(hipMemcpyAsync(small, hs.data(), hs.size() * 8, hipMemcpyHostToDevice, c->stream));
  const double *sd = (const double *)small;
  P.gx6 = sd + o_gx;
  P.gy6 = sd + o_gy;
  P.inl = sd + o_inl;
  P.wl = sd + o_wl;
  P.wu = sd + o_wu;
  unsigned char *clean_dev = (unsigned char *)(small + align_up(hs.size() * 8, 256));

  // fluid mask with frame
  std::vector<unsigned char> hfl((size_t)c->L.pitch * c->L.rows, 0);
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++)
      hfl[(size_t)(j + YO) * c->L.pitch + XO + i] = c->solid[(size_t)j * nx + i] ? 0 : 1;
  HIPCHK(hipMemcpyAsync(fl, hfl.data(), hfl.size(), hipMemcpyHostToDevice, c->stream));
  P.fl = fl;

  // clean tiles: the whole window lies inside the domain (away from the
  // inlet, outlet and walls) and contains no solid cell
  P.tiles_x = (nx + TX - 1) / TX;
  P.tiles_y = (ny + TY - 1) / TY;
  std::vector<unsigned char> cl((size_t)P.tiles_x * P.tiles_y, 0);
  for (int ty = 0; ty < P.tiles_y; ty++)
    for (int tx = 0; tx < P.tiles_x; tx++) {
      const int x0 = tx * TX, y0 = ty * TY;
      const int xa = x0 - HB, xb = x0 + TX + HB - 1, ya = y0 - HB, yb = y0 + TY + HB - 1;
      bool ok = ya >= 0 && yb <= ny - 1 && (c->per ? (xb - xa + 1 <= nx) : (xa >= 0 && xb <= nx - 1));
      if (c->per && (x0 + TX > nx)) ok = false;  // partial periodic tile: general path
      for (int j = ya; ok && j <= yb; j++)
        for (int i = xa; ok && i <= xb; i++) {
          const int ii = c->per ? ((i % nx) + nx) % nx : i;
          if (c->solid[(size_t)j * nx + ii]) ok = false;
        }
      cl[(size_t)ty * P.tiles_x + tx] = ok ? 1 : 0;
    }
  HIPCHK(hipMemcpyAsync(clean_dev, cl.data(), cl.size(), hipMemcpyHostToDevice, c->stream));
  P.clean = clean_dev;
  P.nx = nx;
  P.ny = ny;
  P.per = c->per;
  P.pitch = c->L.pitch;
  P.off = c->L.off;
  P.wtype0 = bc->wall_type[0];
  P.wtype1 = bc->wall_type[1];
  P.wu0 = bc->wall_u[0];
  P.wu1 = bc->wall_u[1];
  P.gx = bc->gx;
  P.gy = bc->gy;
  P.obsT = c->obsT;
  P.sq_obsT = sqrt(c->obsT);
  P.otype = c->otype;
  P.sj = c->slip_jump ? 1 : 0;
  HIPCHK(hipStreamSynchronize(c->stream));
  return fill_frames(c);
}

sts_status initial_state(sts_ctx *c) {
  const int nx = c->nx, ny = c->ny;
  std::vector<double> u((size_t)(nx + 1) * ny), v((size_t)nx * (ny + 1), 0.0),
      p((size_t)nx * ny), T((size_t)nx * ny);
  for (int j = 0; j < ny; j++) {
    for (int i = 0; i <= nx; i++) u[(size_t)j * (nx + 1) + i] = c->u_in[j];
    for (int i = 0; i < nx; i++) {
      p[(size_t)j * nx + i] = c->p_in;
      T[(size_t)j * nx + i] = c->T_in[j];
    }
  }
  project(c, u.data(), v.data(), p.data(), T.data());
  sts_status s = upload(c, 0, u.data(), v.data(), p.data(), T.data());
  if (s != STS_OK) return s;
  s = upload(c, 1, u.data(), v.data(), p.data(), T.data());
  c->cur = 0;
  return s;
}

void release(sts_ctx *c) {
  if (!c) return;
  if (c->adj_mem) (void)hipFree(c->adj_mem);
  if (c->slot_mem) (void)hipFree(c->slot_mem);
  if (c->l3_mem) (void)hipFree(c->l3_mem);
  if (c->aux) (void)hipFree(c->aux);
  if (c->haux) (void)hipHostFree(c->haux);
  if (c->base && c->own_mem) (void)hipFree(c->base);
  if (c->hres) (void)hipHostFree(c->hres);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->l2ev)
    if (e) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

}  // namespace

extern "C" sts_status sts_create(const sts_grid *grid, const sts_obstacles *obstacles,
                                 double Ma, double Re, double Pr, double gamma,
                                 const sts_bc *bc, void *hip_stream, void *workspace,
                                 size_t workspace_bytes, sts_ctx **out) {
  if (!out) return fail(STS_EINVAL, "out is NULL");
  sts_status s = validate(grid, obstacles, Ma, Re, Pr, gamma, bc);
  if (s != STS_OK) return s;
  sts_ctx *c = new (std::nothrow) sts_ctx();
  if (!c) return fail(STS_ENOMEM, "host allocation failed");
  const int nx = grid->nx, ny = grid->ny;
  c->nx = nx;
  c->ny = ny;
  c->per = bc->x_mode == STS_X_PERIODIC;
  c->L = make_layout(nx, ny);
  c->S = make_sizes(nx, ny, c->L);
  c->dx.resize(nx);
  c->dy.resize(ny);
  for (int i = 0; i < nx; i++) c->dx[i] = grid->dx ? grid->dx[i] : grid->lx / nx;
  for (int j = 0; j < ny; j++) c->dy[j] = grid->dy ? grid->dy[j] : grid->ly / ny;
  c->u_in.resize(ny);
  c->T_in.resize(ny);
  for (int j = 0; j < ny; j++) {
    c->u_in[j] = bc->u_in ? bc->u_in[j] : 1.0;
    c->T_in[j] = bc->T_in ? bc->T_in[j] : 1.0;
  }
  for (int w = 0; w < 2; w++) {
    c->Tw[w].resize(nx);
    for (int i = 0; i < nx; i++) c->Tw[w][i] = bc->wall_T[w] ? bc->wall_T[w][i] : 1.0;
  }
  c->solid.assign((size_t)nx * ny, 0);
  if (obstacles)
    for (int k = 0; k < obstacles->n; k++)
      for (int j = obstacles->j0[k]; j <= obstacles->j1[k]; j++)
        for (int i = obstacles->i0[k]; i <= obstacles->i1[k]; i++)
          c->solid[(size_t)j * nx + i] = 1;
  c->p_in = bc->p_in;
  c->obsT = bc->obstacle_T;
  c->otype = bc->obstacle_type;
  c->slip_jump = bc->obstacle_type == STS_WALL_SLIP_JUMP || bc->wall_type[0] == STS_WALL_SLIP_JUMP ||
                 bc->wall_type[1] == STS_WALL_SLIP_JUMP;
  // slip and jump lengths per unit 1/rho (eqs pl38, pl39)
  c->P.kz = 1.1466 * bc->kn;
  c->P.kt = 2.1904 * bc->kn;
  // coefficients of eqs pl2-pl6 in convective scaling: A = 1/(gamma Ma^2),
  // B = 1/Re, energy equation in internal-energy form (the discrete source
  // carries p div u): C1 = gamma/(Re Pr), C2 = gamma(gamma-1)Ma^2/Re,
  // C3 = -(gamma-1)
  c->P.A = 1.0 / (gamma * Ma * Ma);
  c->P.B = 1.0 / Re;
  c->P.C1 = gamma / (Re * Pr);
  c->P.C2 = gamma * (gamma - 1.0) * Ma * Ma / Re;
  c->P.C3 = -(gamma - 1.0);
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(STS_EDEVICE, "no HIP device");
  }
  {
    sts_status s = resolve_scratch(c->device);
    if (s != STS_OK) {
      delete c;
      return s;
    }
  }
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
    c->own_stream = false;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(STS_EDEVICE, "hipStreamCreate failed");
    }
    c->own_stream = true;
  }
  if (workspace) {
    if (workspace_bytes < c->S.total || ((uintptr_t)workspace % 256) != 0) {
      release(c);
      return fail(STS_EINVAL, "workspace needs %zu bytes, 256-byte aligned", c->S.total);
    }
    c->base = (char *)workspace;
    c->own_mem = false;
  } else {
    if (hipMalloc((void **)&c->base, c->S.total) != hipSuccess) {
      c->base = nullptr;
      release(c);
      return fail(STS_ENOMEM, "hipMalloc of %zu bytes failed", c->S.total);
    }
    c->own_mem = true;
  }
  if (hipHostMalloc((void **)&c->hres, 256, hipHostMallocDefault) != hipSuccess) {
    c->hres = nullptr;
    release(c);
    return fail(STS_ENOMEM, "pinned host allocation failed");
  }
  memset(c->hres, 0, 256);
  for (hipEvent_t &e : c->l2ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      e = nullptr;
      release(c);
      return fail(STS_ENOMEM, "event creation failed");
    }
  if ((s = build(c, bc)) != STS_OK || (s = initial_state(c)) != STS_OK) {
    std::string msg = g_err;
    release(c);
    g_err = msg;
    return s;
  }
  *out = c;
  return STS_OK;
}

extern "C" void sts_destroy(sts_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  release(ctx);
}

namespace {
sts_status record(sts_ctx *c, int k) {
  if (!c->timing) return STS_OK;
  const size_t need = (size_t)c->ev_used * 4 + k + 1;
  while (c->ev.size() < need) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    c->ev.push_back(e);
  }
  HIPCHK(hipEventRecord(c->ev[(size_t)c->ev_used * 4 + k], c->stream));
  return STS_OK;
}
}  // namespace

extern "C" sts_status sts_step(sts_ctx *c, double dt, int n_inner, int scheme) {
  if (!c) return fail(STS_EINVAL, "ctx is NULL");
  if (!(dt > 0) || !isfinite(dt)) return fail(STS_EINVAL, "dt must be > 0");
  if (n_inner < 1) return fail(STS_EINVAL, "n_inner must be >= 1");
  if (scheme & ~STS_SCHEME_MASK) return fail(STS_EINVAL, "unknown scheme bits 0x%x", scheme);
  c->P.dt = dt;
  c->P.idt = 1.0 / dt;
  sts_status s;
  // the prologue runs inside the first pass (its iterate is the level n-1
  // state); the timing slot of the prologue then holds both
  const bool fused = n_inner >= 2;
  if ((s = record(c, 0)) != STS_OK) return s;
  if (fused) {
    launch_pass_first(c->P, c->st[c->cur], c->st[c->cur ^ 1], c->C, scheme, c->stream);
    c->cur ^= 1;
  } else {
    launch_prologue(c->P, c->st[c->cur], c->C, scheme, c->stream);
  }
  HIPCHK(hipGetLastError());
  if ((s = record(c, 1)) != STS_OK) return s;
  for (int k = fused ? 1 : 0; k < n_inner; k++) {
    launch_pass(c->P, c->st[c->cur], c->st[c->cur ^ 1], c->C, scheme,
                k == n_inner - 1 ? &c->X : nullptr, nullptr, c->stream);
    c->cur ^= 1;
  }
  HIPCHK(hipGetLastError());
  if ((s = record(c, 2)) != STS_OK) return s;
  launch_residual(c->P, c->st[c->cur], c->C, c->X, c->dres, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->hres, c->dres, NRES * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  if ((s = record(c, 3)) != STS_OK) return s;
  if (c->timing) {
    c->ev_used++;
    c->t_passes += fused ? n_inner - 1 : n_inner;
  }
  c->stepped = true;
  c->hist_rows = 0;
  c->last_scheme = scheme;
  return STS_OK;
}

namespace {
// the scratch (T, p) pairs of loop 3, allocated on first use
sts_status ensure_l3(sts_ctx *c) {
  if (c->l3_mem) return STS_OK;
  const size_t fb = c->L.field_bytes;
  if (hipMalloc((void **)&c->l3_mem, 4 * fb) != hipSuccess) {
    c->l3_mem = nullptr;
    return fail(STS_ENOMEM, "hipMalloc of %zu bytes failed", 4 * fb);
  }
  const size_t n = (size_t)c->L.pitch * c->L.rows;
  std::vector<double> one(n, 1.0);
  for (int q = 0; q < 2; q++) {
    c->l3T[q] = (double *)(c->l3_mem + (2 * q) * fb);
    c->l3p[q] = (double *)(c->l3_mem + (2 * q + 1) * fb);
    HIPCHK(hipMemcpyAsync(c->l3T[q], one.data(), n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->l3p[q], one.data(), n * 8, hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return STS_OK;
}

// one pass with loop 3 from iterate o into nw (n3 >= 2 launches); X: the
// residual inputs of the pass (last pass of a step, or every pass of a loop 2
// run to convergence, whose stop flag every launch honours), or NULL
void launch_l3_pass(sts_ctx *c, State o, State nw, int n3, int scheme, const Resid *X) {
  launch_pass3(c->P, o, nw, c->C, scheme, X, 1, nullptr, nullptr, c->l3T[0], c->l3p[0],
               c->stream);
  int q = 0;  // the pair holding the previous solve
  for (int sub = 2; sub < n3; sub++, q ^= 1)
    launch_pass3(c->P, o, nw, c->C, scheme, X, 1, c->l3T[q], c->l3p[q], c->l3T[q ^ 1],
                 c->l3p[q ^ 1], c->stream);
  launch_pass3(c->P, o, nw, c->C, scheme, X, 2, c->l3T[q], c->l3p[q], nullptr, nullptr, c->stream);
}
}  // namespace

// Loop 2 with its convergence test.  Every pass produces its increment
// maxima (the last-pass kernel variant); one small reduction over its tile
// rows takes the convergence decision on the device (a flag and a pass count,
// Loop2), and once the flag is set the passes and reductions still queued
// return at once.  The continuity residual is reduced once, for the last
// pass run.  The host launches
// passes in groups of L2_GROUP, copies the flag back after each group and
// waits only for the group before the one just queued, so the device never
// runs dry; at most two groups of empty launches follow the converged pass.
// The paper's GPU algorithm reads the residuals back after every pass
// (Sec. 5); the passes taken and the state reached are the same.
constexpr int L2_GROUP = 2;

namespace {
sts_status step_tol(sts_ctx *c, double dt, int max_inner, int n3, double tol, int scheme,
                    int *n_inner) {
  if (!c || !n_inner) return fail(STS_EINVAL, "NULL argument");
  if (!(dt > 0) || !isfinite(dt)) return fail(STS_EINVAL, "dt must be > 0");
  if (max_inner < 1) return fail(STS_EINVAL, "max_inner must be >= 1");
  if (!(tol >= 0) || !isfinite(tol)) return fail(STS_EINVAL, "tol must be >= 0 and finite");
  if (scheme & ~STS_SCHEME_MASK) return fail(STS_EINVAL, "unknown scheme bits 0x%x", scheme);
  if (n3 < 1 || n3 > 64) return fail(STS_EINVAL, "n3 must be in [1, 64]");
  if (n3 > 1) {
    const sts_status s = ensure_l3(c);
    if (s != STS_OK) return s;
  }
  c->P.dt = dt;
  c->P.idt = 1.0 / dt;
  launch_prologue(c->P, c->st[c->cur], c->C, scheme, c->stream);
  int *ctl = (int *)(c->dres + RES_CTL);
  int *hctl = (int *)(c->hres + RES_CTL);  // [3][2]: two group slots, the final copy
  launch_loop2_reset(ctl, c->stream);
  HIPCHK(hipGetLastError());
  Resid X = c->X;
  X.stop = ctl;
  Loop2 L{ctl, tol, c->p_in, 0, c->dhist};
  const int cur0 = c->cur;
  c->stepped = true;
  c->hist_rows = 0;
  c->last_scheme = scheme;
  int slot = 0, waiting = -1;
  for (int k = 0; k < max_inner;) {
    for (const int e = std::min(k + L2_GROUP, max_inner); k < e; k++) {
      const int a = cur0 ^ (k & 1);
      if (n3 == 1) launch_pass(c->P, c->st[a], c->st[a ^ 1], c->C, scheme, &X, nullptr, c->stream);
      else launch_l3_pass(c, c->st[a], c->st[a ^ 1], n3, scheme, &X);
      L.k = k + 1;
      launch_loop2_check(c->P, X, c->dres, L, c->stream);
    }
    HIPCHK(hipGetLastError());
    if (k == max_inner) break;
    HIPCHK(hipMemcpyAsync(hctl + 2 * slot, ctl, 2 * sizeof(int), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipEventRecord(c->l2ev[slot], c->stream));
    if (waiting >= 0) {
      HIPCHK(hipEventSynchronize(c->l2ev[waiting]));
      if (hctl[2 * waiting]) break;
    }
    waiting = slot;
    slot ^= 1;
  }
  launch_loop2_final(c->P, c->st[cur0], c->st[cur0 ^ 1], c->C, c->X, c->dres, ctl, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(hctl + 4, ctl, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(c->hres, c->dres, NRES * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const int k = hctl[5];
  if (k < 1 || k > max_inner) return fail(STS_EDEVICE, "loop 2 control block reads %d passes", k);
  c->cur = cur0 ^ (k & 1);
  c->hist_rows = std::min(k, HIST_CAP);
  *n_inner = k;
  return STS_OK;
}
}  // namespace

extern "C" sts_status sts_step_tol(sts_ctx *c, double dt, int max_inner, double tol, int scheme,
                                   int *n_inner) {
  return step_tol(c, dt, max_inner, 1, tol, scheme, n_inner);
}

extern "C" sts_status sts_step_tol_l3(sts_ctx *c, double dt, int max_inner, int n3, double tol,
                                      int scheme, int *n_inner) {
  return step_tol(c, dt, max_inner, n3, tol, scheme, n_inner);
}


// Loop 3 of the CPU algorithm inside every pass (n3 energy-pressure solves):
// the first solve from the pass's iterate, then n3 - 2 solves into the two
// scratch pairs in turn, then the last, which also updates the velocities
// and writes the new iterate.  Every solve recomputes the face densities and
// pseudo-velocities of the pass's iterate (bitwise the same each time) and
// takes T and p from the previous solve.
extern "C" sts_status sts_step_l3(sts_ctx *c, double dt, int n_inner, int n3, int scheme) {
  if (!c) return fail(STS_EINVAL, "ctx is NULL");
  if (!(dt > 0) || !isfinite(dt)) return fail(STS_EINVAL, "dt must be > 0");
  if (n_inner < 1) return fail(STS_EINVAL, "n_inner must be >= 1");
  if (n3 < 1 || n3 > 64) return fail(STS_EINVAL, "n3 must be in [1, 64]");
  if (scheme & ~STS_SCHEME_MASK) return fail(STS_EINVAL, "unknown scheme bits 0x%x", scheme);
  if (n3 == 1) return sts_step(c, dt, n_inner, scheme);
  sts_status s;
  if ((s = ensure_l3(c)) != STS_OK) return s;
  c->P.dt = dt;
  c->P.idt = 1.0 / dt;
  launch_prologue(c->P, c->st[c->cur], c->C, scheme, c->stream);
  for (int k = 0; k < n_inner; k++) {
    launch_l3_pass(c, c->st[c->cur], c->st[c->cur ^ 1], n3, scheme,
                   k == n_inner - 1 ? &c->X : nullptr);
    c->cur ^= 1;
  }
  HIPCHK(hipGetLastError());
  launch_residual(c->P, c->st[c->cur], c->C, c->X, c->dres, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->hres, c->dres, NRES * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  c->stepped = true;
  c->hist_rows = 0;
  c->last_scheme = scheme;
  return STS_OK;
}

extern "C" sts_status sts_residual_history(sts_ctx *c, double *out, int max_rows, int *rows) {
  if (!c || !rows) return fail(STS_EINVAL, "NULL argument");
  if (max_rows < 0 || (max_rows > 0 && !out)) return fail(STS_EINVAL, "bad output buffer");
  HIPCHK(hipStreamSynchronize(c->stream));
  const int n = std::min(max_rows, c->hist_rows);
  if (n > 0) HIPCHK(hipMemcpy(out, c->dhist, sizeof(double) * 4 * n, hipMemcpyDeviceToHost));
  *rows = c->hist_rows;
  return STS_OK;
}

extern "C" sts_status sts_residuals(sts_ctx *c, double out[6]) {
  if (!c || !out) return fail(STS_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int k = 0; k < 6; k++) out[k] = c->stepped ? c->hres[k] : 0.0;
  if (c->stepped && c->hres[6] != 0.0)
    return fail(STS_ENONFINITE, "the last step produced %g non-finite values", c->hres[6]);
  return STS_OK;
}

extern "C" sts_status sts_fields(sts_ctx *c, double *u, double *v, double *p, double *T) {
  if (!c) return fail(STS_EINVAL, "ctx is NULL");
  const int nx = c->nx, ny = c->ny;
  const long P = c->L.pitch;
  const State &s = c->st[c->cur];
  if (u) HIPCHK(hipMemcpy2DAsync(u, (nx + 1) * 8, s.u + c->L.off, P * 8, (nx + 1) * 8, ny,
                                 hipMemcpyDeviceToHost, c->stream));
  if (v) HIPCHK(hipMemcpy2DAsync(v, nx * 8, s.v + c->L.off, P * 8, nx * 8, ny + 1,
                                 hipMemcpyDeviceToHost, c->stream));
  if (p) HIPCHK(hipMemcpy2DAsync(p, nx * 8, s.p + c->L.off, P * 8, nx * 8, ny,
                                 hipMemcpyDeviceToHost, c->stream));
  if (T) HIPCHK(hipMemcpy2DAsync(T, nx * 8, s.T + c->L.off, P * 8, nx * 8, ny,
                                 hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return STS_OK;
}

extern "C" sts_status sts_set_fields(sts_ctx *c, const double *u, const double *v,
                                     const double *p, const double *T) {
  if (!c) return fail(STS_EINVAL, "ctx is NULL");
  const int nx = c->nx, ny = c->ny;
  std::vector<double> hu((size_t)(nx + 1) * ny), hv((size_t)nx * (ny + 1)), hp((size_t)nx * ny),
      hT((size_t)nx * ny);
  sts_status s = sts_fields(c, hu.data(), hv.data(), hp.data(), hT.data());
  if (s != STS_OK) return s;
  if (u) memcpy(hu.data(), u, hu.size() * 8);
  if (v) memcpy(hv.data(), v, hv.size() * 8);
  if (p) memcpy(hp.data(), p, hp.size() * 8);
  if (T) memcpy(hT.data(), T, hT.size() * 8);
  project(c, hu.data(), hv.data(), hp.data(), hT.data());
  if ((s = upload(c, 0, hu.data(), hv.data(), hp.data(), hT.data())) != STS_OK) return s;
  if ((s = upload(c, 1, hu.data(), hv.data(), hp.data(), hT.data())) != STS_OK) return s;
  c->cur = 0;
  c->stepped = false;
  return STS_OK;
}

extern "C" sts_status sts_field_ptrs(sts_ctx *c, double **u, double **v, double **p,
                                     double **T, size_t *origin, size_t *pitch) {
  if (!c) return fail(STS_EINVAL, "ctx is NULL");
  const State &s = c->st[c->cur];
  if (u) *u = s.u;
  if (v) *v = s.v;
  if (p) *p = s.p;
  if (T) *T = s.T;
  if (origin) *origin = (size_t)c->L.off;
  if (pitch) *pitch = (size_t)c->L.pitch;
  return STS_OK;
}

extern "C" sts_status sts_timing(sts_ctx *c, int enable) {
  if (!c) return fail(STS_EINVAL, "ctx is NULL");
  HIPCHK(hipStreamSynchronize(c->stream));
  c->timing = enable != 0;
  c->ev_used = 0;
  c->t_passes = 0;
  return STS_OK;
}

extern "C" sts_status sts_read_timing(sts_ctx *c, double out_ms[3], long long out_n[2]) {
  if (!c || !out_ms || !out_n) return fail(STS_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(c->stream));
  double t[3] = {0, 0, 0};
  for (int k = 0; k < c->ev_used; k++) {
    float a = 0, b = 0, d = 0;
    HIPCHK(hipEventElapsedTime(&a, c->ev[(size_t)k * 4 + 0], c->ev[(size_t)k * 4 + 1]));
    HIPCHK(hipEventElapsedTime(&b, c->ev[(size_t)k * 4 + 1], c->ev[(size_t)k * 4 + 2]));
    HIPCHK(hipEventElapsedTime(&d, c->ev[(size_t)k * 4 + 2], c->ev[(size_t)k * 4 + 3]));
    t[0] += a;
    t[1] += b;
    t[2] += d;
  }
  for (int k = 0; k < 3; k++) out_ms[k] = t[k];
  out_n[0] = c->ev_used;
  out_n[1] = c->t_passes;
  c->ev_used = 0;
  c->t_passes = 0;
  return STS_OK;
}

// ---------------------------------------------------------------------------
// drag, state slots, adjoint of the explicit step
// ---------------------------------------------------------------------------
namespace {
State carve(char *&q, const Layout &L) {
  State s;
  s.u = (double *)q; q += L.field_bytes;
  s.v = (double *)q; q += L.field_bytes;
  s.p = (double *)q; q += L.field_bytes;
  s.T = (double *)q; q += L.field_bytes;
  return s;
}
sts_status copy_state(sts_ctx *c, State dst, State src) {
  const size_t n = c->L.field_bytes;
  HIPCHK(hipMemcpyAsync(dst.u, src.u, n, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(dst.v, src.v, n, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(dst.p, src.p, n, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(dst.T, src.T, n, hipMemcpyDeviceToDevice, c->stream));
  return STS_OK;
}
sts_status ensure_aux(sts_ctx *c) {
  if (c->aux) return STS_OK;
  HIPCHK(hipMalloc((void **)&c->aux, sizeof(double) * (drag_blocks(c->P) + 1)));
  HIPCHK(hipHostMalloc((void **)&c->haux, sizeof(double)));
  return STS_OK;
}
State slot_state(sts_ctx *c, int k) {
  char *q = c->slot_mem + (size_t)k * 4 * c->L.field_bytes;
  return carve(q, c->L);
}
}  // namespace

extern "C" sts_status sts_drag(sts_ctx *c, double *out) {
  if (!c || !out) return fail(STS_EINVAL, "NULL argument");
  if (c->otype != STS_WALL_NOSLIP_ISOTHERMAL)
    return fail(STS_EINVAL, "the drag is defined for no-slip obstacle surfaces");
  sts_status s;
  if ((s = ensure_aux(c)) != STS_OK) return s;
  launch_drag(c->P, c->st[c->cur], c->aux, c->aux + drag_blocks(c->P), c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->haux, c->aux + drag_blocks(c->P), sizeof(double),
                        hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *out = *c->haux;
  return STS_OK;
}

extern "C" sts_status sts_drag_noalloc(sts_ctx *c, double *d_out) {
  if (!c || !d_out) return fail(STS_EINVAL, "NULL argument");
  if (c->otype != STS_WALL_NOSLIP_ISOTHERMAL)
    return fail(STS_EINVAL, "the drag is defined for no-slip obstacle surfaces");
  const int nb = drag_blocks(c->P);
  if (nb > NOALLOC_PARTIALS)
    return fail(STS_EINVAL, "the drag reduction needs %d partials; the fixed array holds %d", nb,
                NOALLOC_PARTIALS);
  double *part = scratch_of(c->device);
  if (!part) return fail(STS_ESTATE, "the drag scratch array of device %d is not resolved", c->device);
  // every block assigns its partial and the sum reads exactly nb of them:
  // nothing in the array has to start at zero
  launch_drag(c->P, c->st[c->cur], part, d_out, c->stream);
  HIPCHK(hipGetLastError());
  return STS_OK;
}

extern "C" sts_status sts_state_slots(sts_ctx *c, int n) {
  if (!c) return fail(STS_EINVAL, "ctx is NULL");
  if (n < 0 || n > 1000000) return fail(STS_EINVAL, "slot count %d out of range", n);
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->slot_mem) {
    HIPCHK(hipFree(c->slot_mem));
    c->slot_mem = nullptr;
    c->nslots = 0;
  }
  if (n == 0) return STS_OK;
  const size_t bytes = (size_t)n * 4 * c->L.field_bytes;
  if (hipMalloc((void **)&c->slot_mem, bytes) != hipSuccess) {
    c->slot_mem = nullptr;
    return fail(STS_ENOMEM, "cannot allocate %d state slots (%zu bytes)", n, bytes);
  }
  c->nslots = n;
  return STS_OK;
}

extern "C" sts_status sts_state_save(sts_ctx *c, int slot) {
  if (!c) return fail(STS_EINVAL, "ctx is NULL");
  if (slot < 0 || slot >= c->nslots) return fail(STS_EINVAL, "slot %d out of range", slot);
  return copy_state(c, slot_state(c, slot), c->st[c->cur]);
}

extern "C" sts_status sts_state_load(sts_ctx *c, int slot) {
  if (!c) return fail(STS_EINVAL, "ctx is NULL");
  if (slot < 0 || slot >= c->nslots) return fail(STS_EINVAL, "slot %d out of range", slot);
  // into the current buffer only: a pass writes every entry of its output
  // buffer except the boundary entries, which are the same in every state
  sts_status s;
  if ((s = copy_state(c, c->st[c->cur], slot_state(c, slot))) != STS_OK) return s;
  c->stepped = false;
  return STS_OK;
}

extern "C" sts_status sts_adjoint_begin(sts_ctx *c, int n_inner) {
  if (!c) return fail(STS_EINVAL, "ctx is NULL");
  if (c->per) return fail(STS_EINVAL, "the adjoint supports inlet/outlet channels only");
  if (n_inner < 1 || n_inner > 10000) return fail(STS_EINVAL, "n_inner must be in [1, 10000]");
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->adj_K != n_inner) {
    if (c->adj_mem) HIPCHK(hipFree(c->adj_mem));
    c->adj_mem = nullptr;
    c->adj_K = 0;
    // K iterates, 8 intermediates per pass, 9 adjoint intermediates and 2
    // cached arrays, 2 adjoint states, 4 constant adjoints, wall gradients
    const size_t F = c->L.field_bytes;
    const size_t bytes = (size_t)n_inner * 4 * F + (size_t)n_inner * 8 * F + 11 * F + 8 * F +
                         4 * F + align_up(sizeof(double) * 2 * c->nx, 256);
    if (hipMalloc((void **)&c->adj_mem, bytes) != hipSuccess) {
      c->adj_mem = nullptr;
      return fail(STS_ENOMEM, "cannot allocate the adjoint buffers (%zu bytes)", bytes);
    }
    char *q = c->adj_mem;
    c->it.assign(1, State{});
    c->Iv.assign(1, Inter{});
    for (int k = 1; k <= n_inner; k++) c->it.push_back(carve(q, c->L));
    for (int k = 1; k <= n_inner; k++) {
      Inter I;
      double **ip[8] = {&I.ru, &I.rv, &I.uh, &I.du, &I.vh, &I.dv, &I.pn, &I.tn};
      for (auto p : ip) { *p = (double *)q; q += F; }
      c->Iv.push_back(I);
    }
    c->adj_frames = false;
    double **ap[9] = {&c->A.luh, &c->A.ldu, &c->A.lvh, &c->A.ldv, &c->A.lru,
                      &c->A.lrv, &c->A.lr,  &c->A.lg,  &c->A.ltn};
    for (auto p : ap) { *p = (double *)q; q += F; }
    c->A.cr = (double *)q; q += F;
    c->A.cg = (double *)q; q += F;
    c->lam[0] = carve(q, c->L);
    c->lam[1] = carve(q, c->L);
    c->lC.Cu = (double *)q; q += F;
    c->lC.Cv = (double *)q; q += F;
    c->lC.CT = (double *)q; q += F;
    c->lC.Cp = (double *)q; q += F;
    c->gtw = (double *)q;
    c->adj_K = n_inner;
  }
  c->lcur = 0;
  // rho, Gamma of a state including the frame (the cells are recomputed for
  // every iterate by the reverse kernels; the frame is the same in all)
  launch_cell_cache(c->P, c->st[c->cur], c->A.cr, c->A.cg, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemsetAsync(c->lam[0].u, 0, 8 * c->L.field_bytes, c->stream));
  HIPCHK(hipMemsetAsync(c->gtw, 0, sizeof(double) * 2 * c->nx, c->stream));
  return STS_OK;
}

extern "C" sts_status sts_adjoint_seed_drag(sts_ctx *c, double w) {
  if (!c) return fail(STS_EINVAL, "ctx is NULL");
  if (!c->adj_K) return fail(STS_ESTATE, "sts_adjoint_begin has not been called");
  if (!isfinite(w)) return fail(STS_EINVAL, "weight must be finite");
  if (c->otype != STS_WALL_NOSLIP_ISOTHERMAL)
    return fail(STS_EINVAL, "the drag is defined for no-slip obstacle surfaces");
  launch_drag_seed(c->P, c->st[c->cur], c->lam[c->lcur], w, c->stream);
  HIPCHK(hipGetLastError());
  return STS_OK;
}

extern "C" sts_status sts_adjoint_seed(sts_ctx *c, const double *wu, const double *wv,
                                       const double *wp, const double *wT) {
  if (!c) return fail(STS_EINVAL, "ctx is NULL");
  if (!c->adj_K) return fail(STS_ESTATE, "sts_adjoint_begin has not been called");
  const int nx = c->nx, ny = c->ny;
  const long Pt = c->L.pitch;
  const State &l = c->lam[c->lcur];
  struct Part {
    double *dev;
    const double *w;
    int width, height;
  };
  const Part parts[4] = {{l.u, wu, nx + 1, ny}, {l.v, wv, nx, ny + 1}, {l.p, wp, nx, ny},
                         {l.T, wT, nx, ny}};
  for (const Part &q : parts)
    if (q.w)
      for (size_t m = 0; m < (size_t)q.width * q.height; m++)
        if (!isfinite(q.w[m])) return fail(STS_EINVAL, "non-finite seed value");
  std::vector<double> h;
  for (const Part &q : parts) {
    if (!q.w) continue;
    h.resize((size_t)q.width * q.height);
    HIPCHK(hipMemcpy2DAsync(h.data(), q.width * 8, q.dev + c->L.off, Pt * 8, q.width * 8, q.height,
                            hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t m = 0; m < h.size(); m++) h[m] += q.w[m];
    HIPCHK(hipMemcpy2DAsync(q.dev + c->L.off, Pt * 8, h.data(), q.width * 8, q.width * 8, q.height,
                            hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  return STS_OK;
}

extern "C" sts_status sts_adjoint_step(sts_ctx *c, double dt, int n_inner, int scheme) {
  if (!c) return fail(STS_EINVAL, "ctx is NULL");
  if (!c->adj_K) return fail(STS_ESTATE, "sts_adjoint_begin has not been called");
  if (n_inner != c->adj_K) return fail(STS_EINVAL, "n_inner %d differs from sts_adjoint_begin's %d", n_inner, c->adj_K);
  if (!(dt > 0) || !isfinite(dt)) return fail(STS_EINVAL, "dt must be > 0");
  if (scheme & ~(STS_TVD | STS_MIXED))
    return fail(STS_EINVAL, "the adjoint is of the explicit scheme (scheme 0x%x)", scheme);
  c->P.dt = dt;
  c->P.idt = 1.0 / dt;
  const int K = n_inner;
  sts_status s;
  // recompute the step from the current state x_0 (read in place), storing
  // the iterates x_1..x_K and every pass's intermediates, with the form that
  // produced the state (FP64 or mixed); the reverse below is the FP64 step's
  // transpose at these iterates.  A pass writes every cell and face of its
  // output except the constant boundary entries (top wall faces, frame), so
  // the iterate buffers take those once from a copy of the state.
  const State x0 = c->st[c->cur];
  if (!c->adj_frames) {
    for (int k = 1; k <= K; k++)
      if ((s = copy_state(c, c->it[k], x0)) != STS_OK) return s;
    c->adj_frames = true;
  }
  auto iterate = [&](int k) { return k == 0 ? x0 : c->it[k]; };
  launch_prologue(c->P, x0, c->C, scheme, c->stream);
  for (int k = 1; k <= K; k++)
    launch_pass(c->P, iterate(k - 1), c->it[k], c->C, scheme, nullptr, &c->Iv[k], c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemsetAsync(c->lC.Cu, 0, 4 * c->L.field_bytes, c->stream));
  // reverse of the passes
  for (int k = K; k >= 1; k--) {
    State ln = c->lam[c->lcur], lo = c->lam[c->lcur ^ 1];
    // (the reverse of the pass assigns its temporaries before adding to them)
    launch_adjoint_pass(c->P, iterate(k - 1), c->C, c->Iv[k], ln, lo, c->lC, c->A, c->gtw,
                        c->gtw + c->nx, scheme, c->stream);
    HIPCHK(hipGetLastError());
    c->lcur ^= 1;
  }
  // reverse of the prologue, onto the adjoint of x_0
  HIPCHK(hipMemsetAsync(c->A.luh, 0, 9 * c->L.field_bytes, c->stream));
  launch_adjoint_prologue(c->P, x0, c->lC, c->lam[c->lcur], c->A, scheme, c->stream);
  HIPCHK(hipGetLastError());
  return STS_OK;
}

extern "C" sts_status sts_adjoint_read_state_grad(sts_ctx *c, double *gu, double *gv, double *gp,
                                                  double *gT) {
  if (!c) return fail(STS_EINVAL, "ctx is NULL");
  if (!c->adj_K) return fail(STS_ESTATE, "sts_adjoint_begin has not been called");
  const int nx = c->nx, ny = c->ny;
  std::vector<double> lu((size_t)(nx + 1) * ny), lv((size_t)nx * (ny + 1)), lp((size_t)nx * ny),
      lT((size_t)nx * ny);
  sts_status s = sts_adjoint_read(c, nullptr, nullptr, nullptr, lu.data(), lv.data(), lp.data(),
                                  lT.data());
  if (s != STS_OK) return s;
  // the transpose of sts_set_fields' boundary-value projection: entries it
  // overwrites with a fixed value pass no derivative; the outlet face is a
  // copy of face nx-1, so its adjoint adds to that face's
  auto solid = [&](int i, int j) { return c->solid[(size_t)j * nx + i] != 0; };
  if (gu)
    for (int j = 0; j < ny; j++) {
      double *row = gu + (size_t)j * (nx + 1);
      const double *lrow = lu.data() + (size_t)j * (nx + 1);
      for (int i = 0; i <= nx; i++)
        row[i] = (i >= 1 && i <= nx - 1 && !solid(i - 1, j) && !solid(i, j)) ? lrow[i] : 0.0;
      if (!solid(nx - 2, j) && !solid(nx - 1, j)) row[nx - 1] += lrow[nx];
    }
  if (gv)
    for (int j = 0; j <= ny; j++)
      for (int i = 0; i < nx; i++) {
        const size_t k = (size_t)j * nx + i;
        gv[k] = (j >= 1 && j <= ny - 1 && !solid(i, j - 1) && !solid(i, j)) ? lv[k] : 0.0;
      }
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      const size_t k = (size_t)j * nx + i;
      if (gp) gp[k] = solid(i, j) ? 0.0 : lp[k];
      if (gT) gT[k] = solid(i, j) ? 0.0 : lT[k];
    }
  return STS_OK;
}

extern "C" sts_status sts_adjoint_read(sts_ctx *c, double *g_uin, double *g_Tw0, double *g_Tw1,
                                       double *lu, double *lv, double *lp, double *lT) {
  if (!c) return fail(STS_EINVAL, "ctx is NULL");
  if (!c->adj_K) return fail(STS_ESTATE, "sts_adjoint_begin has not been called");
  const int nx = c->nx, ny = c->ny;
  const long Pt = c->L.pitch;
  const State &l = c->lam[c->lcur];
  if (g_uin)  // the inlet faces hold u_in at every level
    HIPCHK(hipMemcpy2DAsync(g_uin, 8, l.u + c->L.off, Pt * 8, 8, ny, hipMemcpyDeviceToHost, c->stream));
  if (g_Tw0) HIPCHK(hipMemcpyAsync(g_Tw0, c->gtw, 8 * nx, hipMemcpyDeviceToHost, c->stream));
  if (g_Tw1) HIPCHK(hipMemcpyAsync(g_Tw1, c->gtw + nx, 8 * nx, hipMemcpyDeviceToHost, c->stream));
  if (lu) HIPCHK(hipMemcpy2DAsync(lu, (nx + 1) * 8, l.u + c->L.off, Pt * 8, (nx + 1) * 8, ny,
                                  hipMemcpyDeviceToHost, c->stream));
  if (lv) HIPCHK(hipMemcpy2DAsync(lv, nx * 8, l.v + c->L.off, Pt * 8, nx * 8, ny + 1,
                                  hipMemcpyDeviceToHost, c->stream));
  if (lp) HIPCHK(hipMemcpy2DAsync(lp, nx * 8, l.p + c->L.off, Pt * 8, nx * 8, ny,
                                  hipMemcpyDeviceToHost, c->stream));
  if (lT) HIPCHK(hipMemcpy2DAsync(lT, nx * 8, l.T + c->L.off, Pt * 8, nx * 8, ny,
                                  hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return STS_OK;
}
