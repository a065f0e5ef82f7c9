// Host side of libpond.so: configuration checks, arena layout, the initial
// state, the step loop and the observables.  Every computation on the state
// runs in the kernels of pond_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pond.h"
#include "pond_internal.h"
#include "pond_state.h"

namespace pond {

static thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(POND_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define POND_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(e_, #call);    \
  } while (0)

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int validate(const pond_config* c) {
  if (!c) return fail(POND_ERR_INVALID, "null config");
  if (c->dim != 1 && c->dim != 2) return fail(POND_ERR_INVALID, "dim must be 1 or 2");
  if (c->nx < 4 || (c->dim == 2 && c->ny < 4) || (c->dim == 1 && c->ny != 1))
    return fail(POND_ERR_INVALID, "grid needs nx >= 4 and, in 2D, ny >= 4 (ny = 1 in 1D)");
  if ((c->dim == 1 && c->lattice != POND_D1Q4) ||
      (c->dim == 2 && c->lattice != POND_D2Q16 && c->lattice != POND_D2Q9 &&
       c->lattice != POND_D2Q9_D2Q16 && c->lattice != POND_D2Q25))
    return fail(POND_ERR_INVALID,
                "lattice must be D1Q4 in 1D and D2Q16, D2Q9, D2Q9_D2Q16 or D2Q25 in 2D");
  if (c->lattice == POND_D2Q25 && c->transform != POND_TF_GRAD)
    return fail(POND_ERR_INVALID, "the D2Q25 f-lattice uses the fourth-order Grad projection");
  if ((c->lattice == POND_D2Q9 || c->lattice == POND_D2Q9_D2Q16) && c->transform != POND_TF_GRAD)
    return fail(POND_ERR_INVALID, "the D2Q9 and multiscale f-lattices use Grad's projection");
  if (c->lattice == POND_D2Q9_D2Q16 && !(c->ms_threshold >= 0.0 && std::isfinite(c->ms_threshold)))
    return fail(POND_ERR_INVALID, "the multiscale threshold must be finite and >= 0");
  if (c->precision != POND_FP64 && c->precision != POND_MIXED)
    return fail(POND_ERR_INVALID, "unknown precision");
  if (c->transform != POND_TF_LAGRANGE && c->transform != POND_TF_GRAD)
    return fail(POND_ERR_INVALID, "unknown transform");
  if (!(c->gamma > 1.0)) return fail(POND_ERR_INVALID, "gamma must exceed 1");
  if (!(c->tau > 0.0)) return fail(POND_ERR_INVALID, "tau must be positive");
  if (!(c->prandtl > 0.0 && c->prandtl <= 1.0)) return fail(POND_ERR_INVALID, "Pr must lie in (0, 1]");
  if (!(c->cfl > 0.0)) return fail(POND_ERR_INVALID, "cfl must be positive");
  if (!(c->dx >= 0.0) || !std::isfinite(c->dx)) return fail(POND_ERR_INVALID, "dx must be >= 0");
  if (c->limiter != POND_LIM_VANLEER && c->limiter != POND_LIM_MINMOD)
    return fail(POND_ERR_INVALID, "unknown limiter");
  if (c->n_corr < 0 || c->n_corr > 4) return fail(POND_ERR_INVALID, "n_corr must lie in 0..4");
  const int nside = c->dim == 2 ? 4 : 2;
  for (int k = 0; k < nside; ++k)
    if (c->bc[k] < POND_BC_PERIODIC || c->bc[k] > POND_BC_WALL)
      return fail(POND_ERR_INVALID, "unknown boundary condition");
  for (int k = 0; k < nside; ++k) {
    if (c->bc[k] != POND_BC_WALL) continue;
    if (c->dim != 2 || c->lattice != POND_D2Q16)
      return fail(POND_ERR_UNSUPPORTED, "walls need dim 2 and the D2Q16 f-lattice");
    const double* w = c->wall[k];
    if (!(w[2] > 0.0) || !std::isfinite(w[2]) || !std::isfinite(w[0]) || !std::isfinite(w[1]))
      return fail(POND_ERR_INVALID, "a wall needs a positive temperature and a finite velocity");
    if (w[k < 2 ? 0 : 1] != 0.0) return fail(POND_ERR_INVALID, "a wall cannot move along its normal");
  }
  if (!std::isfinite(c->accel[0]) || !std::isfinite(c->accel[1]))
    return fail(POND_ERR_INVALID, "the body force must be finite");
  if ((c->accel[0] != 0.0 || c->accel[1] != 0.0) && (c->dim != 2 || c->lattice != POND_D2Q16))
    return fail(POND_ERR_UNSUPPORTED, "a body force needs dim 2 and the D2Q16 f-lattice");
  for (int k = 0; k < nside; k += 2)
    if ((c->bc[k] == POND_BC_PERIODIC) != (c->bc[k + 1] == POND_BC_PERIODIC))
      return fail(POND_ERR_INVALID, "a periodic axis needs periodic conditions on both sides");
  for (int k = 0; k < nside; ++k)
    if (c->bc[k] == POND_BC_INFLOW) {
      const double* s = c->inflow[k];
      if (!(s[0] > 0.0) || !(s[3] > 0.0) || !std::isfinite(s[1]) || !std::isfinite(s[2]))
        return fail(POND_ERR_INVALID, "inflow state needs positive density and pressure");
    }
  return POND_OK;
}

Layout layout_of(const pond_config* c) {
  Layout L;
  L.D = c->dim;
  L.q25 = c->dim == 2 && c->lattice == POND_D2Q25;
  L.QF = c->dim == 2 ? (L.q25 ? 25 : 16) : 4;
  L.QG = c->dim == 2 ? 9 : 3;
  L.NP = L.QF + L.QG;
  L.fp64 = c->precision == POND_FP64;
  L.cells = size_t(c->nx) * size_t(c->ny);
  const size_t elt = L.fp64 ? 8 : 4;
  L.pop_bytes = align256(size_t(L.NP) * L.cells * elt);
  L.led_bytes = align256(4 * L.cells * sizeof(long long));
  L.red_blocks = 256;
  L.red_bytes = align256(size_t(L.red_blocks) * 8 * sizeof(long long));
  L.stage_rows = size_t(std::max(4, L.NP + 3));
  L.stage_cells = std::min(L.cells, size_t(kStagingBytes / (8 * L.stage_rows)));
  L.stage_bytes = align256(L.stage_rows * L.stage_cells * 8);
  L.tab_bytes = align256(sizeof(BatchEntry));
  L.ms = c->dim == 2 && (c->lattice == POND_D2Q9 || c->lattice == POND_D2Q9_D2Q16);
  L.lat_bytes = L.ms ? align256(L.cells) : 0;
  L.theta_bytes = L.ms ? align256(L.cells * sizeof(double)) : 0;
  bool walls = false;
  for (int k = 0; k < 2 * c->dim; ++k) walls |= c->bc[k] == POND_BC_WALL;
  // wall ghosts: [side][layer][t] entries, t along the wall (max(nx, ny))
  L.wall_len = walls ? size_t(std::max(c->nx, c->ny)) : 0;
  L.wall_bytes = walls ? align256(size_t(8) * L.wall_len * (4 * sizeof(long long) + L.NP * elt)) : 0;
  if (L.q25) {
    L.q25_nfx = size_t(c->nx + 1) * c->ny;
    L.q25_nfy = size_t(c->nx) * (c->ny + 1);
    L.q25_P = align256(size_t(L.NP) * L.cells * elt);
    L.q25_fr = align256(3 * L.cells * sizeof(double));
    for (size_t nf : {L.q25_nfx, L.q25_nfy})
      L.q25_bytes += align256(size_t(L.NP) * nf * elt) + align256(3 * nf * sizeof(double)) +
                     align256(4 * nf * sizeof(long long));
    L.q25_bytes += L.q25_P + L.q25_fr;
  }
  L.total = 2 * L.pop_bytes + 2 * L.led_bytes + 512 + L.tab_bytes + L.red_bytes + L.stage_bytes +
            2 * L.lat_bytes + L.theta_bytes + L.wall_bytes + L.q25_bytes;
  return L;
}

static int check_device() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(POND_ERR_DEVICE, std::string("libpond needs a gfx950 device, found ") + prop.gcnArchName);
  return POND_OK;
}

// Fixed-point exponent E of the ledger: the largest |conserved moment| M of
// the initial data must satisfy M 2^E <= 2^56, leaving a factor 64 of
// headroom below the 2^62 overflow guard.
static int ledger_bits(double M) {
  int e = 0;
  std::frexp(std::max(M, 1e-300), &e);  // M < 2^e
  return 56 - e;
}

static void conserved_of(double rho, double ux, double uy, double p, double cv, double out[4]) {
  out[0] = rho;
  out[1] = rho * ux;
  out[2] = rho * uy;
  out[3] = cv * p + 0.5 * rho * (ux * ux + uy * uy);
}

static int sync_flag(pond_state* s) {
  POND_HIP(hipStreamSynchronize(s->stream));
  int flag = 0;
  POND_HIP(hipMemcpy(&flag, s->flag, sizeof(int), hipMemcpyDeviceToHost));
  if (flag & 2) return fail(POND_ERR_UNSTABLE, "conserved-moment ledger overflow");
  if (flag & 1) return fail(POND_ERR_UNSTABLE, "non-physical state (rho <= 0, T <= 0 or non-finite)");
  return POND_OK;
}

// The 2D step runs the batched kernel with a one-entry table (the same
// machine code as a solve inside the serving batch, so results agree bit for
// bit): entry.args[p] advances buffer p to buffer 1 - p.
int upload_table(pond_state* s) {
  if (s->cfg.dim != 2) return POND_OK;
  BatchEntry e{};
  for (int par = 0; par < 2; ++par) {
    e.args[par] = s->args;
    e.args[par].n_in = s->n[par];
    e.args[par].n_out = s->n[1 - par];
    e.args[par].U_in = s->U[par];
    e.args[par].U_out = s->U[1 - par];
    e.args[par].lat_in = s->lat[par];
    e.args[par].lat_out = s->lat[1 - par];
    if (s->cfg.lattice == POND_D2Q9_D2Q16) {
      e.args[par].q16_in = s->q16 + par;
      e.args[par].q16_out = s->q16 + 1 - par;
    }
  }
  e.tile_begin = 0;
  e.tiles = s->args.tiles_x * s->args.tiles_y;
  POND_HIP(hipMemcpyAsync(s->tab, &e, sizeof e, hipMemcpyHostToDevice, s->stream));
  POND_HIP(hipStreamSynchronize(s->stream));
  return POND_OK;
}

int step_launches(pond_state* s, int in, hipStream_t st) {
  StepArgs a = s->args;
  a.n_in = s->n[in];
  a.n_out = s->n[1 - in];
  a.U_in = s->U[in];
  a.U_out = s->U[1 - in];
  if (s->L.q25) {
    POND_HIP(launch_q25_step(s->L.fp64, a, s->qP, s->qfr, s->qfp[0], s->qfp[1], s->qff[0],
                             s->qff[1], s->qps[0], s->qps[1], st));
  } else if (s->cfg.dim == 2) {
    if (s->cfg.lattice == POND_D2Q9_D2Q16) {
      // this step's f-lattices, from the state at its start
      POND_HIP(launch_switch(s->args, s->U[in], s->cfg.ms_threshold, s->cfg.gamma,
                             s->q16 + 1 - in, s->theta, s->lat[1 - in], st));
    }
    // wall ghosts from the state at the start of this step
    if (s->L.wall_bytes) POND_HIP(launch_wall_ghosts(s->L.fp64, a, s->wU, s->wN, st));
    unsigned mask = 1u << kind_of(s->cfg.transform, s->args.ms);
    // a multiscale step may run in the D2Q9 kernel (all cells on D2Q9)
    if (s->cfg.lattice == POND_D2Q9_D2Q16) mask |= 1u << kind_of(POND_TF_GRAD, 3);
    POND_HIP(launch_step_batch(s->L.fp64, mask, s->tab, 1, s->args.tiles_x * s->args.tiles_y,
                               in, st));
  } else {
    POND_HIP(launch_step_1d(s->L.fp64, a, st));
  }
  return POND_OK;
}

}  // namespace pond

using namespace pond;

extern "C" {

int pond_last_error(char* buf, size_t n) {
  if (buf && n) {
    std::strncpy(buf, g_last_error.c_str(), n - 1);
    buf[n - 1] = 0;
  }
  return POND_OK;
}

size_t pond_state_bytes(const pond_config* cfg) {
  if (validate(cfg) != POND_OK) return 0;
  return layout_of(cfg).total;
}

int pond_create(const pond_config* cfg, void* dev_arena, size_t arena_bytes, void* hip_stream,
                pond_state** out) {
  if (!out) return fail(POND_ERR_INVALID, "null output handle");
  *out = nullptr;
  int rc = validate(cfg);
  if (rc) return rc;
  if ((rc = check_device())) return rc;
  const Layout L = layout_of(cfg);
  if (!dev_arena || (reinterpret_cast<uintptr_t>(dev_arena) & 255))
    return fail(POND_ERR_INVALID, "arena must be a 256-byte aligned device pointer");
  if (arena_bytes < L.total)
    return fail(POND_ERR_NOMEM, "arena of " + std::to_string(arena_bytes) + " bytes, need " +
                                    std::to_string(L.total));
  pond_state* s = new pond_state();
  s->cfg = *cfg;
  s->L = L;
  s->stream = static_cast<hipStream_t>(hip_stream);
  char* p = static_cast<char*>(dev_arena);
  s->n[0] = p; p += L.pop_bytes;
  s->n[1] = p; p += L.pop_bytes;
  s->U[0] = reinterpret_cast<long long*>(p); p += L.led_bytes;
  s->U[1] = reinterpret_cast<long long*>(p); p += L.led_bytes;
  s->flag = reinterpret_cast<int*>(p);
  s->q16 = s->flag + 16;  // in the flag word's 256-byte slot
  p += 256;
  s->inflow_dev = reinterpret_cast<long long*>(p); p += 256;
  s->tab = reinterpret_cast<BatchEntry*>(p); p += L.tab_bytes;
  s->red = reinterpret_cast<long long*>(p); p += L.red_bytes;
  s->stage = reinterpret_cast<double*>(p); p += L.stage_bytes;
  if (L.ms) {
    s->lat[0] = reinterpret_cast<unsigned char*>(p); p += L.lat_bytes;
    s->lat[1] = reinterpret_cast<unsigned char*>(p); p += L.lat_bytes;
    s->theta = reinterpret_cast<double*>(p); p += L.theta_bytes;
  }
  if (L.wall_bytes) {
    s->wU = reinterpret_cast<long long*>(p); p += size_t(8) * L.wall_len * 4 * sizeof(long long);
    s->wN = p;
  }
  if (L.q25) {
    p = static_cast<char*>(dev_arena) + (L.total - L.q25_bytes);
    const size_t elt = L.fp64 ? 8 : 4;
    s->qP = p; p += L.q25_P;
    s->qfr = reinterpret_cast<double*>(p); p += L.q25_fr;
    const size_t nfs[2] = {L.q25_nfx, L.q25_nfy};
    for (int ax = 0; ax < 2; ++ax) {
      s->qfp[ax] = p; p += align256(size_t(L.NP) * nfs[ax] * elt);
      s->qff[ax] = reinterpret_cast<double*>(p); p += align256(3 * nfs[ax] * sizeof(double));
      s->qps[ax] = reinterpret_cast<long long*>(p); p += align256(4 * nfs[ax] * sizeof(long long));
    }
  }
  s->dx = cfg->dx > 0.0 ? cfg->dx : 1.0 / cfg->nx;
  s->cv = 1.0 / (cfg->gamma - 1.0);
  hipError_t e = hipMemsetAsync(s->flag, 0, sizeof(int), s->stream);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "hipMemsetAsync");
  }
  *out = s;
  return POND_OK;
}

int pond_init_fields(pond_state* s, const double* rho, const double* ux, const double* uy,
                     const double* p) {
  if (!s || !rho || !ux || !p) return fail(POND_ERR_INVALID, "null argument");
  const pond_config& c = s->cfg;
  const size_t n = s->L.cells;
  const bool twod = c.dim == 2;
  if (twod && !uy) return fail(POND_ERR_INVALID, "uy is required in 2D");
  // dt from the CFL rule at t = 0 (Sec. V): max over cells, nodes and axes
  // of |sqrt(T) c_ia + u_a| (largest node of the f-lattice in use)
  const double cmax = c.lattice == POND_D2Q9 ? kR3 : (c.lattice == POND_D2Q25 ? kB5 : kB);
  double vmax = 0.0, M = 0.0, U4[4];
  for (size_t k = 0; k < n; ++k) {
    const double vy = twod ? uy[k] : 0.0;
    if (!(rho[k] > 0.0) || !(p[k] > 0.0) || !std::isfinite(rho[k]) || !std::isfinite(p[k]) ||
        !std::isfinite(ux[k]) || !std::isfinite(vy))
      return fail(POND_ERR_INVALID, "initial density and pressure must be positive and finite");
    const double rt = std::sqrt(p[k] / rho[k]);
    vmax = std::max(vmax, std::fabs(ux[k]) + rt * cmax);
    if (twod) vmax = std::max(vmax, std::fabs(vy) + rt * cmax);
    conserved_of(rho[k], ux[k], vy, p[k], s->cv, U4);
    for (double v : U4) M = std::max(M, std::fabs(v));
  }
  const int nside = twod ? 4 : 2;
  for (int k = 0; k < nside; ++k)
    if (c.bc[k] == POND_BC_INFLOW) {
      const double* st = c.inflow[k];
      conserved_of(st[0], st[1], twod ? st[2] : 0.0, st[3], s->cv, U4);
      for (double v : U4) M = std::max(M, std::fabs(v));
    }
  s->dt = c.cfl * s->dx / vmax;
  s->scale_bits = ledger_bits(M);
  s->scale = std::ldexp(1.0, s->scale_bits);
  for (int k = 0; k < 4; ++k) {
    const double* st = c.inflow[k];
    if (c.bc[k] != POND_BC_INFLOW) {
      for (int q = 0; q < 4; ++q) s->inflow_U[k][q] = 0;
      continue;
    }
    conserved_of(st[0], st[1], twod ? st[2] : 0.0, st[3], s->cv, U4);
    for (int q = 0; q < 4; ++q) s->inflow_U[k][q] = (long long)std::nearbyint(U4[q] * s->scale);
  }
  // D2Q25: the init kernel writes the 25 planes of D2Q16; clear the rest
  if (s->L.q25) POND_HIP(hipMemsetAsync(s->n[0], 0, s->L.pop_bytes, s->stream));
  // upload the primitive fields chunk by chunk and build the equilibrium state
  const size_t chunk = s->L.stage_cells;
  std::vector<double> host(4 * chunk);
  for (size_t first = 0; first < n; first += chunk) {
    const size_t cnt = std::min(chunk, n - first);
    for (size_t k = 0; k < cnt; ++k) {
      host[k] = rho[first + k];
      host[cnt + k] = ux[first + k];
      host[2 * cnt + k] = twod ? uy[first + k] : 0.0;
      host[3 * cnt + k] = p[first + k];
    }
    POND_HIP(hipMemcpyAsync(s->stage, host.data(), 4 * cnt * sizeof(double), hipMemcpyHostToDevice,
                            s->stream));
    POND_HIP(launch_init(c.dim, s->L.fp64, s->stage, n, first, cnt, s->scale, s->cv, s->n[0],
                         s->U[0], s->stream));
    POND_HIP(hipStreamSynchronize(s->stream));
  }
  POND_HIP(hipMemsetAsync(s->flag, 0, sizeof(int), s->stream));
  if (s->L.ms) {
    // D2Q9: every cell on D2Q9; multiscale: D2Q16 until the first switch
    const int q1 = c.lattice == POND_D2Q9 ? 3 : 4;
    POND_HIP(hipMemsetAsync(s->lat[0], q1, s->L.lat_bytes, s->stream));
    POND_HIP(hipMemsetAsync(s->lat[1], q1, s->L.lat_bytes, s->stream));
    POND_HIP(hipMemsetAsync(s->theta, 0, s->L.theta_bytes, s->stream));
  }
  {
    // "some cell may be on D2Q16" for both lattice planes until a switch says
    // otherwise (1 is always safe: it only turns off the all-D2Q9 fast path)
    const int one[2] = {1, 1};
    POND_HIP(hipMemcpyAsync(s->q16, one, sizeof one, hipMemcpyHostToDevice, s->stream));
  }
  POND_HIP(hipStreamSynchronize(s->stream));
  s->cur = 0;
  s->nstep = 0;
  s->initialized = true;
  // constant part of the step arguments
  StepArgs& a = s->args;
  a = StepArgs{};
  a.nx = c.nx;
  a.ny = c.ny;
  for (int k = 0; k < 4; ++k) a.bc[k] = c.bc[k];
  a.n_corr = c.n_corr;
  a.limiter = c.limiter;
  a.transform = c.transform;
  bool ext = c.accel[0] != 0.0 || c.accel[1] != 0.0;
  for (int k = 0; k < 2 * c.dim; ++k) ext |= c.bc[k] == POND_BC_WALL;
  a.ms = s->L.ms ? (c.lattice == POND_D2Q9 ? 3 : 1) : (ext ? 2 : 0);
  if (twod) {
    a.tiles_x = (c.nx + kTX2 - 1) / kTX2;
    a.tiles_y = (c.ny + kTY2 - 1) / kTY2;
  } else {
    a.tiles_x = (c.nx + kTX1 - 1) / kTX1;
    a.tiles_y = 1;
  }
  a.scale = s->scale;
  a.inv_scale = std::ldexp(1.0, -s->scale_bits);
  a.cv = s->cv;
  a.icv = 1.0 / s->cv;
  a.geq = s->cv - 0.5 * c.dim;
  a.lam = s->dt / s->dx;
  // tau is tau1 / dt; with tau1 = tau dt all DUGKS coefficients depend on tau only
  const double t = c.tau;
  a.a_pre = (2.0 * t - 0.5) / (2.0 * t + 1.0);
  a.b_upd = (2.0 * t - 1.0) / (2.0 * t + 1.0);
  a.c_face1 = 4.0 * t / (4.0 * t + 1.0);
  a.c_face2 = 1.0 / (4.0 * t + 1.0);
  a.kappa = 0.5 * (1.0 / t - c.prandtl / t);  // (dt/2)(1/tau1 - 1/tau2) with tau2 = tau1/Pr
  POND_HIP(hipMemcpyAsync(s->inflow_dev, s->inflow_U, sizeof(s->inflow_U), hipMemcpyHostToDevice,
                          s->stream));
  POND_HIP(hipStreamSynchronize(s->stream));
  a.inflow = s->inflow_dev;
  a.cells = n;
  a.flag = s->flag;
  a.force = (c.accel[0] != 0.0 || c.accel[1] != 0.0) ? 1 : 0;
  a.hax = 0.5 * s->dt * c.accel[0];
  a.hay = 0.5 * s->dt * c.accel[1];
  if (s->L.wall_bytes) {
    a.wU = s->wU;
    a.wN = s->wN;
    a.wall_len = int(s->L.wall_len);
    a.wall_n = 8 * s->L.wall_len;
    for (int k = 0; k < 4; ++k)
      for (int q = 0; q < 3; ++q) a.wall[k][q] = c.wall[k][q];
    a.idx2 = 0.5 / s->dx;
    a.tau1 = t * s->dt;
    a.tau2 = t * s->dt / c.prandtl;
    a.kf = 1.0 + 0.5 / t;
  }
  return upload_table(s);
}

int pond_step(pond_state* s, int nsteps) {
  if (!s || nsteps < 0) return fail(POND_ERR_INVALID, "bad arguments");
  if (!s->initialized) return fail(POND_ERR_INVALID, "fields not initialised");
  for (int k = 0; k < nsteps; ++k) {
    const int rc = step_launches(s, s->cur, s->stream);
    if (rc != POND_OK) return rc;
    s->cur ^= 1;
    s->nstep++;
  }
  return POND_OK;
}

int pond_moments(pond_state* s, double* rho, double* ux, double* uy, double* T) {
  if (!s || !s->initialized) return fail(POND_ERR_INVALID, "fields not initialised");
  int rc = sync_flag(s);
  const size_t n = s->L.cells, chunk = s->L.stage_cells;
  std::vector<double> host(4 * chunk);
  double* outs[4] = {rho, ux, uy, T};
  for (size_t first = 0; first < n; first += chunk) {
    const size_t cnt = std::min(chunk, n - first);
    POND_HIP(launch_moments(s->cfg.dim, s->U[s->cur], n, first, cnt, s->args.inv_scale,
                            s->args.icv, s->stage, s->stream));
    POND_HIP(hipMemcpyAsync(host.data(), s->stage, 4 * cnt * sizeof(double), hipMemcpyDeviceToHost,
                            s->stream));
    POND_HIP(hipStreamSynchronize(s->stream));
    for (int q = 0; q < 4; ++q)
      if (outs[q]) std::memcpy(outs[q] + first, host.data() + q * cnt, cnt * sizeof(double));
  }
  return rc;
}

static int totals128(pond_state* s, __int128 tot[4]) {
  POND_HIP(launch_totals(s->U[s->cur], s->L.cells, s->L.red_blocks, s->red, s->stream));
  std::vector<long long> host(size_t(s->L.red_blocks) * 8);
  POND_HIP(hipMemcpyAsync(host.data(), s->red, host.size() * sizeof(long long),
                          hipMemcpyDeviceToHost, s->stream));
  POND_HIP(hipStreamSynchronize(s->stream));
  for (int q = 0; q < 4; ++q) tot[q] = 0;
  for (int b = 0; b < s->L.red_blocks; ++b)
    for (int q = 0; q < 4; ++q) {
      const unsigned __int128 hi = (unsigned __int128)(unsigned long long)host[(b * 4 + q) * 2];
      const unsigned __int128 lo = (unsigned long long)host[(b * 4 + q) * 2 + 1];
      tot[q] += (__int128)((hi << 64) | lo);
    }
  return POND_OK;
}

int pond_totals_fixed(pond_state* s, int64_t out[8], int* scale_bits) {
  if (!s || !s->initialized || !out) return fail(POND_ERR_INVALID, "bad arguments");
  int rc = sync_flag(s);
  __int128 tot[4];
  int r2 = totals128(s, tot);
  if (r2) return r2;
  for (int q = 0; q < 4; ++q) {
    out[2 * q] = (int64_t)(tot[q] >> 64);
    out[2 * q + 1] = (int64_t)(uint64_t)tot[q];
  }
  if (scale_bits) *scale_bits = s->scale_bits;
  return rc;
}

int pond_totals(pond_state* s, double out[4]) {
  if (!s || !s->initialized || !out) return fail(POND_ERR_INVALID, "bad arguments");
  int rc = sync_flag(s);
  __int128 tot[4];
  int r2 = totals128(s, tot);
  if (r2) return r2;
  const double vol = s->cfg.dim == 2 ? s->dx * s->dx : s->dx;
  for (int q = 0; q < 4; ++q) out[q] = std::ldexp((double)tot[q], -s->scale_bits) * vol;
  return rc;
}

// D2Q25 export on the host: the stored planes hold f~ - rho W (25 tensor
// weights of the D1Q5 rule) and g~ - (C_v - D/2) T rho W^g, as the fused
// lattices store them; the frame comes from the ledger (eqs.
// ConservationLaws, E), and the equilibria are added back in FP64.
static int export_q25(pond_state* s, double* f, double* g, double* frame) {
  int rc = sync_flag(s);
  const size_t n = s->L.cells, chunk = std::min(n, size_t(1) << 18);
  const size_t es = s->L.fp64 ? sizeof(double) : sizeof(float);
  const int QF = s->L.QF, QG = s->L.QG, NP = s->L.NP;
  const double w5[5] = {kW5B, kW5A, 8.0 / 15.0, kW5A, kW5B};
  const double w3[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
  std::vector<unsigned char> raw(size_t(NP) * chunk * es);
  std::vector<long long> led(4 * chunk);
  const unsigned char* dn = static_cast<const unsigned char*>(s->n[s->cur]);
  for (size_t first = 0; first < n; first += chunk) {
    const size_t cnt = std::min(chunk, n - first);
    for (int p = 0; p < NP; ++p)
      POND_HIP(hipMemcpyAsync(raw.data() + size_t(p) * chunk * es, dn + (size_t(p) * n + first) * es,
                              cnt * es, hipMemcpyDeviceToHost, s->stream));
    for (int q = 0; q < 4; ++q)
      POND_HIP(hipMemcpyAsync(led.data() + size_t(q) * chunk, s->U[s->cur] + size_t(q) * n + first,
                              cnt * sizeof(long long), hipMemcpyDeviceToHost, s->stream));
    POND_HIP(hipStreamSynchronize(s->stream));
    auto stored = [&](int p, size_t k) {
      const unsigned char* at = raw.data() + (size_t(p) * chunk + k) * es;
      if (s->L.fp64) {
        double v;
        std::memcpy(&v, at, sizeof v);
        return v;
      }
      float v;
      std::memcpy(&v, at, sizeof v);
      return double(v);
    };
    const double inv = s->args.inv_scale;
    for (size_t k = 0; k < cnt; ++k) {
      const size_t c = first + k;
      const double rho = double(led[k]) * inv;
      const double mx = double(led[chunk + k]) * inv, my = double(led[2 * chunk + k]) * inv;
      const double e = double(led[3 * chunk + k]) * inv;
      const double ux = mx / rho, uy = my / rho;
      const double T = (e - 0.5 * (mx * ux + my * uy)) / rho * s->args.icv;
      if (f)
        for (int i = 0; i < QF; ++i) f[size_t(i) * n + c] = rho * (w5[i % 5] * w5[i / 5]) + stored(i, k);
      if (g)
        for (int i = 0; i < QG; ++i)
          g[size_t(i) * n + c] = s->args.geq * T * rho * (w3[i % 3] * w3[i / 3]) + stored(QF + i, k);
      if (frame) {
        frame[c] = ux;
        frame[n + c] = uy;
        frame[2 * n + c] = T;
      }
    }
  }
  return rc;
}

int pond_export_state(pond_state* s, double* f, double* g, double* frame) {
  if (!s || !s->initialized) return fail(POND_ERR_INVALID, "fields not initialised");
  if (s->L.q25) return export_q25(s, f, g, frame);
  int rc = sync_flag(s);
  const size_t n = s->L.cells, chunk = s->L.stage_cells, rows = size_t(s->L.NP + 3);
  const int QF = s->L.QF, QG = s->L.QG;
  std::vector<double> host(rows * chunk);
  for (size_t first = 0; first < n; first += chunk) {
    const size_t cnt = std::min(chunk, n - first);
    POND_HIP(launch_export(s->cfg.dim, s->L.fp64, s->n[s->cur], s->U[s->cur], n, first, cnt,
                           s->args.inv_scale, s->args.icv, s->args.geq, s->stage, s->stream));
    POND_HIP(hipMemcpyAsync(host.data(), s->stage, rows * cnt * sizeof(double),
                            hipMemcpyDeviceToHost, s->stream));
    POND_HIP(hipStreamSynchronize(s->stream));
    for (int i = 0; i < QF; ++i)
      if (f) std::memcpy(f + i * n + first, host.data() + i * cnt, cnt * sizeof(double));
    for (int i = 0; i < QG; ++i)
      if (g) std::memcpy(g + i * n + first, host.data() + (QF + i) * cnt, cnt * sizeof(double));
    for (int i = 0; i < 3; ++i)
      if (frame)
        std::memcpy(frame + i * n + first, host.data() + (QF + QG + i) * cnt, cnt * sizeof(double));
  }
  return rc;
}

int pond_lattice_map(pond_state* s, int* q, double* theta) {
  if (!s || !s->initialized) return fail(POND_ERR_INVALID, "fields not initialised");
  POND_HIP(hipStreamSynchronize(s->stream));
  const size_t n = s->L.cells;
  const int q_all = s->cfg.dim == 2 ? (s->L.q25 ? 25 : 16) : 4;
  if (q) {
    if (!s->L.ms) {
      for (size_t k = 0; k < n; ++k) q[k] = q_all;
    } else {
      std::vector<unsigned char> lat(n);
      POND_HIP(hipMemcpy(lat.data(), s->lat[s->cur], n, hipMemcpyDeviceToHost));
      for (size_t k = 0; k < n; ++k) q[k] = int(lat[k]) * int(lat[k]);
    }
  }
  if (theta) {
    if (s->cfg.lattice == POND_D2Q9_D2Q16) {
      POND_HIP(hipMemcpy(theta, s->theta, n * sizeof(double), hipMemcpyDeviceToHost));
    } else {
      for (size_t k = 0; k < n; ++k) theta[k] = 0.0;
    }
  }
  return POND_OK;
}

int pond_get_time(pond_state* s, double* dt, int64_t* nsteps) {
  if (!s) return fail(POND_ERR_INVALID, "null state");
  if (dt) *dt = s->dt;
  if (nsteps) *nsteps = s->nstep;
  return POND_OK;
}

namespace {
struct CkptHeader {
  char magic[8];
  pond_config cfg;
  double dt;
  int64_t nstep;
  int scale_bits;
  int fp64;
  uint64_t pop_bytes, led_bytes;
};
}  // namespace

int pond_save(pond_state* s, const char* path) {
  if (!s || !s->initialized || !path) return fail(POND_ERR_INVALID, "bad arguments");
  POND_HIP(hipStreamSynchronize(s->stream));
  CkptHeader h{};
  std::memcpy(h.magic, "PONDCKP1", 8);
  h.cfg = s->cfg;
  h.dt = s->dt;
  h.nstep = s->nstep;
  h.scale_bits = s->scale_bits;
  h.fp64 = s->L.fp64;
  const size_t elt = s->L.fp64 ? 8 : 4;
  h.pop_bytes = size_t(s->L.NP) * s->L.cells * elt;
  h.led_bytes = 4 * s->L.cells * sizeof(long long);
  const size_t lat_n = s->L.ms ? s->L.cells : 0;  // f-lattice of each cell (D2Q9 / multiscale)
  std::vector<char> buf(h.pop_bytes + h.led_bytes + lat_n);
  POND_HIP(hipMemcpy(buf.data(), s->n[s->cur], h.pop_bytes, hipMemcpyDeviceToHost));
  POND_HIP(hipMemcpy(buf.data() + h.pop_bytes, s->U[s->cur], h.led_bytes, hipMemcpyDeviceToHost));
  if (lat_n)
    POND_HIP(hipMemcpy(buf.data() + h.pop_bytes + h.led_bytes, s->lat[s->cur], lat_n,
                       hipMemcpyDeviceToHost));
  FILE* fp = std::fopen(path, "wb");
  if (!fp) return fail(POND_ERR_INVALID, std::string("cannot open ") + path);
  const bool ok = std::fwrite(&h, sizeof h, 1, fp) == 1 && std::fwrite(buf.data(), 1, buf.size(), fp) == buf.size();
  std::fclose(fp);
  return ok ? POND_OK : fail(POND_ERR_INVALID, "short write");
}

int pond_load(pond_state* s, const char* path) {
  if (!s || !path) return fail(POND_ERR_INVALID, "bad arguments");
  FILE* fp = std::fopen(path, "rb");
  if (!fp) return fail(POND_ERR_INVALID, std::string("cannot open ") + path);
  CkptHeader h{};
  if (std::fread(&h, sizeof h, 1, fp) != 1 || std::memcmp(h.magic, "PONDCKP1", 8) != 0 ||
      std::memcmp(&h.cfg, &s->cfg, sizeof(pond_config)) != 0) {
    std::fclose(fp);
    return fail(POND_ERR_INVALID, "checkpoint does not match this configuration");
  }
  const size_t lat_n = s->L.ms ? s->L.cells : 0;
  std::vector<char> buf(h.pop_bytes + h.led_bytes + lat_n);
  const bool ok = std::fread(buf.data(), 1, buf.size(), fp) == buf.size();
  std::fclose(fp);
  if (!ok) return fail(POND_ERR_INVALID, "short read");
  // rebuild the constant step arguments from a neutral field, then overwrite
  if (!s->initialized) {
    std::vector<double> one(s->L.cells, 1.0), zero(s->L.cells, 0.0);
    int rc = pond_init_fields(s, one.data(), zero.data(), zero.data(), one.data());
    if (rc) return rc;
  }
  s->dt = h.dt;
  s->nstep = h.nstep;
  s->scale_bits = h.scale_bits;
  s->scale = std::ldexp(1.0, h.scale_bits);
  s->args.scale = s->scale;
  s->args.inv_scale = std::ldexp(1.0, -h.scale_bits);
  s->args.lam = s->dt / s->dx;
  // the arguments that scale with dt (body force, wall relaxation times)
  s->args.hax = 0.5 * s->dt * s->cfg.accel[0];
  s->args.hay = 0.5 * s->dt * s->cfg.accel[1];
  s->args.tau1 = s->cfg.tau * s->dt;
  s->args.tau2 = s->cfg.tau * s->dt / s->cfg.prandtl;
  for (int k = 0; k < 4; ++k) {
    const double* st = s->cfg.inflow[k];
    double U4[4];
    conserved_of(st[0], st[1], s->cfg.dim == 2 ? st[2] : 0.0, st[3], s->cv, U4);
    for (int q = 0; q < 4; ++q)
      s->inflow_U[k][q] = s->cfg.bc[k] == POND_BC_INFLOW ? (long long)std::nearbyint(U4[q] * s->scale) : 0;
  }
  POND_HIP(hipMemcpy(s->inflow_dev, s->inflow_U, sizeof(s->inflow_U), hipMemcpyHostToDevice));
  s->cur = 0;
  POND_HIP(hipMemcpy(s->n[0], buf.data(), h.pop_bytes, hipMemcpyHostToDevice));
  POND_HIP(hipMemcpy(s->U[0], buf.data() + h.pop_bytes, h.led_bytes, hipMemcpyHostToDevice));
  if (lat_n) {
    POND_HIP(hipMemcpy(s->lat[0], buf.data() + h.pop_bytes + h.led_bytes, lat_n, hipMemcpyHostToDevice));
    POND_HIP(hipMemcpy(s->lat[1], buf.data() + h.pop_bytes + h.led_bytes, lat_n, hipMemcpyHostToDevice));
  }
  const int zero = 0;  // a checkpoint holds a healthy state: clear the status flag
  POND_HIP(hipMemcpy(s->flag, &zero, sizeof(int), hipMemcpyHostToDevice));
  // whether the restored lattice plane has a D2Q16 cell, as the switch
  // records it each step (so a resumed run takes the same kernels)
  int any16 = lat_n ? 0 : 1;
  for (size_t k = 0; k < lat_n; ++k)
    any16 |= buf[h.pop_bytes + h.led_bytes + k] == 4;
  const int q16[2] = {any16, any16};
  POND_HIP(hipMemcpy(s->q16, q16, sizeof q16, hipMemcpyHostToDevice));
  return upload_table(s);
}

int pond_destroy(pond_state* s) {
  if (!s) return POND_OK;
  hipError_t e = hipStreamSynchronize(s->stream);
  delete s;
  return e == hipSuccess ? POND_OK : hip_fail(e, "hipStreamSynchronize");
}

int pond_lattice_constants(double out[14]) {
  if (!out) return fail(POND_ERR_INVALID, "null argument");
  const double v[14] = {-kB, -kA, kA, kB, kWB, kWA, kWA, kWB, -kR3, 0.0, kR3, 1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
  std::memcpy(out, v, sizeof v);
  return POND_OK;
}

}  // extern "C"
