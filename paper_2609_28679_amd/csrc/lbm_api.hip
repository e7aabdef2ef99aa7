// C-ABI host layer: parameter validation, device memory ownership, launch sequencing,
// diagnostics bookkeeping and error reporting. All numerical work runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {
thread_local std::string g_err;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
}  // namespace

struct lbm_ctx {
  lbm_params p{};
  int D = 2, Q = 9;
  int kind = 0;  // 0: float32 populations, 1: float64
  int fmt = 0;   // DDF storage format: 0 float32, 1 float64, 2 bfloat16, 3 float16 (reduced)
  bool ddf = false;  // double-distribution ideal-gas model
  int codec = -1;    // reduced storage: 0 = bfloat16, 1 = float16 (scaled); -1 = none
  float s_enc = 1.0f, s_dec = 1.0f;
  int planes = 9;    // stored population planes per buffer
  bool aa = false;   // one buffer, in place (isothermal model): layout alternates with t parity
  DdfParams dp{};
  double* fld = nullptr;  // D3Q27 double distribution: derivative fields
  void* nb = nullptr;     // non-equilibrium extrapolation walls: boundary rows
  Layout L{};
  Grid G{};
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;
  void* A = nullptr;  // post-collision populations of the current time
  void* B = nullptr;  // second buffer of the two-buffer layout (NULL with one buffer)
  double* partials = nullptr;  // per-workgroup diagnostics partial sums
  int partial_slots = 0;
  double* history = nullptr;   // ring of kHistoryCap rows {t, totals[5]}
  double* readout = nullptr;   // nodes * (D + 2) doubles for moment read-out
  int64_t hist_written = 0;
  int64_t t = 0;
  double omega = 0.0;
  Force F;        // uniform body force of the next collision (zero: none)
  Force F_state;  // force of the collision that produced the stored state (read-outs)
  double heat = 0.0, heat_state = 0.0;  // heat source Q (DDF): next collision / stored state
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  float* mlp_w = nullptr;                  // surrogate weights (kMlpParams floats)
  unsigned long long* mlp_cnt = nullptr;   // {fallbacks, updates}
  bool mlp_set = false;
  double mlp_tol = 0.0;
  std::string err;
};

struct lbm_mlp {
  hipStream_t stream = nullptr;
  float* w = nullptr;  // float32 master weights
  float* m = nullptr;  // Adam first moment
  float* v = nullptr;  // Adam second moment
  float* partials = nullptr;
  size_t partial_rows = 0;
  float* scratch = nullptr;  // loss
  int64_t t = 0;             // Adam steps taken
  int64_t offset = 0;        // next training sample
};

namespace {

int fail(lbm_ctx* c, int code, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    g_err = msg;
  return code;
}

int hip_fail(lbm_ctx* c, hipError_t e, const char* where) {
  return fail(c, LBM_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                  \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr); \
  } while (0)

// The double-distribution kernels take the sources of the next collision from DdfParams.
void sync_sources(lbm_ctx* c) {
  c->dp.Fx = c->F.x;
  c->dp.Fy = c->F.y;
  c->dp.Fz = c->F.z;
  c->dp.Q = c->heat;
  c->dp.src = c->F.on() || c->heat != 0.0;
}

struct Plan {
  int D, Q, kind, planes, codec;
  size_t off_fld;  // D3Q27 double distribution: derivative fields (8 planes of the storage type)
  size_t off_nb;   // non-equilibrium extrapolation walls: boundary rows (2D) or planes (3D)
  bool ddf, aa;
  Layout L;
  Grid G;
  size_t elem;
  size_t off_A, off_B, off_part, off_hist, off_read, off_mlp, total;
  int partial_slots;
};

// Product-form factors must be positive: Psi_0 = 1 - theta - u^2 > 0 and
// Psi_+- = (theta + u^2 +- u)/2 > 0 for every component.
bool admissible(double theta, double u) {
  const double z = theta + u * u;
  return z < 1.0 && z > std::fabs(u);
}

// Sources: a body force needs the paper's collision and FP32 or FP64 storage (isothermal or
// double-distribution model), a heat source in addition the double-distribution model. Both
// must be finite; the force's z component must be zero on D2Q9.
int validate_sources(const lbm_params* p, const double* force, double heat, std::string& why) {
  const bool forced = force[0] != 0.0 || force[1] != 0.0 || force[2] != 0.0;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(force[a])) { why = "force must be finite"; return LBM_EINVAL; }
  if (!std::isfinite(heat)) { why = "heat_source must be finite"; return LBM_EINVAL; }
  const bool plain = p->collision == LBM_COLLIDE_PLAIN &&
                     (p->storage == LBM_STORE_FP32 || p->storage == LBM_STORE_FP64);
  if (forced && !plain) {
    why = "a body force needs the paper's collision and FP32 or FP64 storage";
    return LBM_EINVAL;
  }
  if (heat != 0.0 && (p->model != LBM_MODEL_DDF || !plain)) {
    why = "a heat_source needs the double-distribution model with FP32 or FP64 storage";
    return LBM_EINVAL;
  }
  if (forced && p->lattice == LBM_D2Q9 && force[2] != 0.0) { why = "D2Q9 requires force[2] = 0"; return LBM_EINVAL; }
  if ((forced || heat != 0.0) && p->wall_y == 2) { why = "force and heat_source are not supported with wall_y = 2"; return LBM_EINVAL; }
  return LBM_OK;
}

int validate(const lbm_params* p, std::string& why) {
  if (!p) { why = "params is NULL"; return LBM_EINVAL; }
  if (p->lattice != LBM_D2Q9 && p->lattice != LBM_D3Q27) { why = "lattice must be D2Q9 or D3Q27"; return LBM_EINVAL; }
  if (p->model != LBM_MODEL_BGK && p->model != LBM_MODEL_DDF) { why = "unknown model"; return LBM_EINVAL; }
  if (p->storage < LBM_STORE_FP32 || p->storage > LBM_STORE_FP64) { why = "unknown storage"; return LBM_EINVAL; }
  if (p->collision != LBM_COLLIDE_PLAIN && p->collision != LBM_COLLIDE_MLP) { why = "unknown collision"; return LBM_EINVAL; }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) { why = "lattice sizes must be >= 1"; return LBM_EINVAL; }
  if (p->lattice == LBM_D2Q9 && p->nz != 1) { why = "D2Q9 requires nz = 1"; return LBM_EINVAL; }
  if ((int64_t)p->nx * p->ny * p->nz > (int64_t)1 << 34) { why = "lattice too large"; return LBM_EINVAL; }
  if (p->wall_y < 0 || p->wall_y > 2) { why = "wall_y must be 0, 1 or 2"; return LBM_EINVAL; }
  if (p->wall_y == 2) {
    if (p->model != LBM_MODEL_DDF ||
        (p->storage != LBM_STORE_FP32 && p->storage != LBM_STORE_FP64) || p->ny < 3) {
      why = "non-equilibrium extrapolation walls (wall_y = 2) need the double-distribution model, FP32 or FP64 storage and ny >= 3";
      return LBM_EINVAL;
    }
    // tangential wall velocities: along x (D2Q9), along x and z (D3Q27); for the ideal gas the
    // wall equilibrium's factors at theta_W = R T_W must be positive (for the van der Waals
    // fluid theta_W depends on the boundary density, known only during the run)
    const bool d3 = p->lattice == LBM_D3Q27;
    for (int side = 0; side < 2; ++side) {
      const double T = p->wall_T[side], ux = p->wall_u[side][0], uz = p->wall_u[side][2];
      const bool ok_state = p->eos == 1 || (admissible(p->R * T, ux) &&
                                            admissible(p->R * T, uz) && admissible(p->R * T, 0.0));
      if (!(T > 0.0) || !std::isfinite(T) || !std::isfinite(ux) || !std::isfinite(uz) ||
          p->wall_u[side][1] != 0.0 || (!d3 && uz != 0.0) || !ok_state) {
        why = "wall_T must be positive and wall_u tangential (x; x and z in D3Q27) and admissible";
        return LBM_EINVAL;
      }
    }
    if (p->wall_density != 0 && p->wall_density != 1) { why = "wall_density must be 0 or 1"; return LBM_EINVAL; }
    // van der Waals fluid with the pressure-continued wall density: the isotherms of the wall
    // temperatures must be supercritical (T_W > T_cr = 8 a / (27 b R), b > 0) so that
    // P(rho, T_W) = P_N has exactly one root with 1 - b rho > 0
    if (p->eos == 1 && p->wall_density == 0) {
      const double Tcr = p->vdw_b > 0.0 ? 8.0 * p->vdw_a / (27.0 * p->vdw_b * p->R) : INFINITY;
      if (!(p->wall_T[0] > Tcr) || !(p->wall_T[1] > Tcr)) {
        why = "NEQ walls with the van der Waals fluid and wall_density 0 need vdw_b > 0 and wall temperatures above T_cr = 8 a / (27 b R)";
        return LBM_EINVAL;
      }
    }
  }
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) { why = "tau must be a finite value > 1/2"; return LBM_EINVAL; }
  if (p->diag_every < 0) { why = "diag_every must be >= 0"; return LBM_EINVAL; }
  if (p->model == LBM_MODEL_DDF) {
    if (!(p->R > 0.0) || !(p->cv > 0.0) || !std::isfinite(p->R) || !std::isfinite(p->cv)) { why = "R and cv must be positive"; return LBM_EINVAL; }
    if (p->phi < 0 || p->phi > 2) { why = "phi must be 0 (off), 1 (central) or 2 (upwind)"; return LBM_EINVAL; }
  }
  if (p->eos != 0 && p->eos != 1) { why = "eos must be 0 (ideal gas) or 1 (van der Waals)"; return LBM_EINVAL; }
  if (p->eos == 1) {
    if (p->model != LBM_MODEL_DDF ||
        (p->storage != LBM_STORE_FP32 && p->storage != LBM_STORE_FP64)) {
      why = "the van der Waals eos needs the double-distribution model and FP32 or FP64 storage";
      return LBM_EINVAL;
    }
    if (!(p->vdw_a >= 0.0) || !(p->vdw_b >= 0.0) || !std::isfinite(p->vdw_a) || !std::isfinite(p->vdw_b)) {
      why = "vdw_a and vdw_b must be finite and >= 0";
      return LBM_EINVAL;
    }
  }
  if (!(p->prandtl > 0.0) || !std::isfinite(p->prandtl)) { why = "prandtl must be a finite value > 0"; return LBM_EINVAL; }
  if (!std::isfinite(p->eta_over_mu)) { why = "eta_over_mu must be finite"; return LBM_EINVAL; }
  if ((p->prandtl != 1.0 || p->eta_over_mu >= 0.0) &&
      (p->model != LBM_MODEL_DDF || (p->storage != LBM_STORE_FP32 && p->storage != LBM_STORE_FP64))) {
    why = "prandtl != 1 and eta_over_mu >= 0 need the double-distribution model with FP32 or FP64 storage";
    return LBM_EINVAL;
  }
  const bool reduced = p->storage == LBM_STORE_BF16 || p->storage == LBM_STORE_FP16;
  if (reduced && p->lattice != LBM_D2Q9) { why = "reduced storage is D2Q9 only"; return LBM_EINVAL; }
  if (p->storage == LBM_STORE_FP16 && (p->fp16_scale_log2 < 0 || p->fp16_scale_log2 > 24)) { why = "fp16_scale_log2 must be in [0, 24]"; return LBM_EINVAL; }
  if (p->collision == LBM_COLLIDE_MLP &&
      (p->lattice != LBM_D2Q9 || p->model != LBM_MODEL_BGK || p->storage != LBM_STORE_FP32)) {
    why = "the surrogate collision needs D2Q9, the isothermal model and float32 storage";
    return LBM_EINVAL;
  }
  if (!(p->mlp_tol >= 0.0)) { why = "mlp_tol must be >= 0"; return LBM_EINVAL; }
  if (int rc = validate_sources(p, p->force, p->heat_source, why)) return rc;
  if (p->streaming < LBM_STREAM_AUTO || p->streaming > LBM_STREAM_ONE_BUFFER) { why = "unknown streaming layout"; return LBM_EINVAL; }
  if (p->streaming == LBM_STREAM_ONE_BUFFER &&
      (p->model != LBM_MODEL_BGK || p->collision != LBM_COLLIDE_PLAIN ||
       (p->storage != LBM_STORE_FP32 && p->storage != LBM_STORE_FP64))) {
    why = "one-buffer streaming needs the isothermal model, the paper's collision and FP32 or FP64 storage";
    return LBM_EINVAL;
  }
  if (p->workspace && (reinterpret_cast<uintptr_t>(p->workspace) & 255u)) { why = "workspace must be 256-byte aligned"; return LBM_EINVAL; }
  return LBM_OK;
}

void make_plan(const lbm_params* p, Plan& P) {
  P.D = p->lattice == LBM_D2Q9 ? 2 : 3;
  P.Q = P.D == 2 ? 9 : 27;
  P.kind = p->storage == LBM_STORE_FP64 ? 1 : 0;
  P.codec = p->storage == LBM_STORE_BF16 ? 0 : (p->storage == LBM_STORE_FP16 ? 1 : -1);
  P.ddf = p->model == LBM_MODEL_DDF;
  P.planes = P.ddf ? 2 * P.Q : P.Q;
  P.elem = P.kind ? 8 : 4;
  P.L = make_layout(p->nx, p->ny, p->nz, (int)P.elem);
  if (P.ddf && P.D == 2)
    P.G = make_grid_ddf(P.L, p->phi == 2 ? 2 : 1, P.codec >= 0);
  else if (P.ddf)
    P.G = make_grid_ddf3(P.L);
  else if (p->collision == LBM_COLLIDE_MLP)
    P.G = make_grid_mlp(P.L);
  else if (P.codec >= 0)
    P.G = make_grid_red(P.L);
  else
    P.G = make_grid(P.L);
  P.partial_slots = std::max(P.G.blocks(), 1024);
  if (P.ddf && P.D == 3)  // the one-launch step and the upwind sweeps have their own grids
    P.partial_slots = (int)std::max<int64_t>(P.partial_slots, ddf3_max_records(P.L, P.G));
  // One in-place buffer where supported and either requested or small enough to profit from
  // the 256 MB last-level cache. Measured float32 D2Q9 step times (one vs two buffers): 44 vs
  // 51 us at 151 MB per buffer, 122 vs 131 us at 340 MB, equal at 399 MB, 235 vs 209 us at
  // 604 MB; the crossover is taken as 384 MiB.
  const bool aa_ok = !P.ddf && P.codec < 0 && p->collision == LBM_COLLIDE_PLAIN;
  const size_t one_buffer = (size_t)P.planes * P.L.plane * P.elem;
  P.aa = aa_ok && (p->streaming == LBM_STREAM_ONE_BUFFER ||
                   (p->streaming == LBM_STREAM_AUTO && one_buffer <= ((size_t)384 << 20)));
  size_t off = 0;
  // reduced storage: float32 moment planes + uint16 non-equilibrium planes
  // (isothermal: 3 + 6, double distribution: 4 + 6 + 8)
  const size_t pop = P.codec >= 0 ? (P.ddf ? (size_t)P.L.plane * (4 * 4 + 14 * 2)
                                           : red_state_bytes(P.L))
                                   : (size_t)P.planes * P.L.plane * P.elem;
  P.off_A = off; off = align_up(off + pop, 256);
  P.off_B = off; if (!P.aa) off = align_up(off + pop, 256);
  P.off_part = off; off = align_up(off + (size_t)P.partial_slots * kDiagValues * 8, 256);
  P.off_hist = off; off = align_up(off + (size_t)kHistoryCap * 6 * 8, 256);
  P.off_read = off; off = align_up(off + (size_t)P.L.nodes() * (P.D + 3) * 8, 256);
  // surrogate region: 16 bytes of 64-bit counters (8-byte aligned for the atomics), then the
  // weights 256 bytes further
  P.off_mlp = off; off = align_up(off + 256 + (size_t)kMlpParams * 4, 256);
  P.off_fld = off;
  if (P.ddf && P.D == 3) off = align_up(off + (size_t)8 * P.L.plane * P.elem, 256);
  P.off_nb = off;
  // D2Q9: 2 x 18 rows; D3Q27: 2 x 54 planes of nz x pitch
  if (p->wall_y == 2)
    off = align_up(off + (size_t)(P.D == 2 ? 36 : 108 * (size_t)P.L.nz) * P.L.pitch * P.elem, 256);
  P.total = off;
}

// Every region of the workspace starts on a 256-byte boundary (the caller's workspace is
// 256-byte aligned), so the 64-bit atomic counters of the surrogate at off_mlp and the float64
// arrays are naturally aligned: a misaligned 64-bit atomic faults the GPU. Checked for every
// plan before any device work.
bool plan_aligned(const Plan& P) {
  const size_t offs[] = {P.off_A, P.off_B, P.off_part, P.off_hist, P.off_read,
                         P.off_mlp, P.off_mlp + 256, P.off_fld, P.off_nb, P.total};
  for (size_t o : offs)
    if (o % 256 != 0) return false;
  return true;
}

// Layout of the stored state for the read-out kernels: -1 two buffers, else the parity of t.
int view_of(const lbm_ctx* c) { return c->aa ? (int)(c->t & 1) : -1; }


}  // namespace

extern "C" {

void lbm_default_params(lbm_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->lattice = LBM_D2Q9;
  p->model = LBM_MODEL_BGK;
  p->storage = LBM_STORE_FP32;
  p->collision = LBM_COLLIDE_PLAIN;
  p->nx = 64;
  p->ny = 64;
  p->nz = 1;
  p->wall_y = 0;
  p->tau = 0.8;
  p->R = 1.0 / 3.0;
  p->cv = 5.0 / 6.0;
  p->prandtl = 1.0;
  p->eta_over_mu = -1.0;
  p->phi = 1;
  p->fp16_scale_log2 = 16;
  p->diag_every = 0;
  p->streaming = LBM_STREAM_AUTO;
  p->mlp_tol = 0.05;
  p->stream = nullptr;
  p->workspace = nullptr;
  p->workspace_bytes = 0;
}

int lbm_workspace_size(const lbm_params* p, size_t* bytes) {
  std::string why;
  int rc = validate(p, why);
  if (rc) return fail(nullptr, rc, why);
  if (!bytes) return fail(nullptr, LBM_EINVAL, "bytes is NULL");
  Plan P;
  make_plan(p, P);
  if (!plan_aligned(P)) return fail(nullptr, LBM_EINVAL, "internal: misaligned workspace plan");
  *bytes = P.total;
  return LBM_OK;
}

int lbm_create(const lbm_params* p, const double* rho0, const double* u0, const double* T0,
               lbm_ctx** out) {
  if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  int rc = validate(p, why);
  if (rc) return fail(nullptr, rc, why);
  if (!rho0 || !u0) return fail(nullptr, LBM_EINVAL, "rho0 and u0 are required");
  Plan P;
  make_plan(p, P);
  if (!plan_aligned(P)) return fail(nullptr, LBM_EINVAL, "internal: misaligned workspace plan");
  if (P.ddf && !T0) return fail(nullptr, LBM_EINVAL, "the double-distribution model needs T0");
  const int64_t nodes = P.L.nodes();
  // host-side admissibility of the initial state
  for (int64_t n = 0; n < nodes; ++n) {
    if (!(rho0[n] > 0.0) || !std::isfinite(rho0[n]))
      return fail(nullptr, LBM_EINVAL, "initial density must be finite and positive at node " + std::to_string(n));
    double theta = 1.0 / 3.0;
    if (P.ddf) {
      if (!(T0[n] > 0.0) || !std::isfinite(T0[n]))
        return fail(nullptr, LBM_EINVAL, "initial temperature must be finite and positive at node " + std::to_string(n));
      theta = p->R * T0[n];
      if (p->eos == 1) {  // van der Waals: theta = P / rho, with 1 - b rho > 0 and P > 0
        const double omb = 1.0 - p->vdw_b * rho0[n];
        theta = p->R * T0[n] / omb - p->vdw_a * rho0[n];
        if (!(omb > 0.0) || !(theta > 0.0))
          return fail(nullptr, LBM_EINVAL, "initial state outside the van der Waals range (1 - b rho > 0, P > 0) at node " + std::to_string(n));
      }
    }
    for (int a = 0; a < P.D; ++a) {
      const double ua = u0[a * nodes + n];
      if (!std::isfinite(ua) || !admissible(theta, ua))
        return fail(nullptr, LBM_EINVAL, "initial state outside the positive product-form range at node " + std::to_string(n));
    }
  }
  lbm_ctx* c = new lbm_ctx();
  c->p = *p;
  c->D = P.D;
  c->Q = P.Q;
  c->kind = P.kind;
  c->ddf = P.ddf;
  c->codec = P.codec;
  c->fmt = P.codec >= 0 ? 2 + P.codec : P.kind;
  if (P.codec == 1) {
    c->s_enc = std::ldexp(1.0f, p->fp16_scale_log2);
    c->s_dec = std::ldexp(1.0f, -p->fp16_scale_log2);
  }
  c->planes = P.planes;
  c->aa = P.aa;
  c->dp.R = p->R;
  c->dp.cv = p->cv;
  c->dp.r_cv = p->R / p->cv;
  c->dp.inv_R = 1.0 / p->R;
  c->dp.mu = (p->tau - 0.5) * (1.0 / 3.0);  // mu = (tau - 1/2) P0 at the reference P0 = 1/3
  c->dp.phi = p->phi;
  if (p->wall_y == 2) {
    c->dp.neq = 1;
    c->dp.neq_literal = p->wall_density;
    for (int side = 0; side < 2; ++side) {
      for (int a = 0; a < 3; ++a) c->dp.uw[side][a] = p->wall_u[side][a];
      c->dp.Tw[side] = p->wall_T[side];
    }
  }
  {
    // alpha = (D+2)/D - rho c_s^2/P - eta/mu with rho c_s^2/P = gamma = 1 + R/c_v (ideal gas);
    // exactly 0 for the Navier-Stokes bulk viscosity. qc = c_p - k/mu, k/mu = c_p / Pr.
    const double D = (double)P.D, gamma = 1.0 + p->R / p->cv, cp = p->cv + p->R;
    c->dp.alpha = p->eta_over_mu >= 0.0 ? (D + 2.0) / D - gamma - p->eta_over_mu : 0.0;
    c->dp.qc = p->prandtl != 1.0 ? cp - cp / p->prandtl : 0.0;
    c->dp.full = c->dp.alpha != 0.0 || c->dp.qc != 0.0;
    if (p->eos == 1) {  // van der Waals: alpha and q^c per node, always the extended path
      c->dp.eos = 1;
      c->dp.va = p->vdw_a;
      c->dp.vb = p->vdw_b;
      c->dp.eta = p->eta_over_mu >= 0.0 ? p->eta_over_mu : 2.0 / D - p->R / p->cv;
      c->dp.kmu = cp / p->prandtl;
      c->dp.full = true;
    }
  }
  c->L = P.L;
  c->G = P.G;
  c->stream = static_cast<hipStream_t>(p->stream);
  c->omega = 1.0 / p->tau;  // omega = 2 beta = 1/tau_LB
  c->F.x = p->force[0];
  c->F.y = p->force[1];
  c->F.z = c->D == 3 ? p->force[2] : 0.0;
  c->F_state = c->F;
  c->heat = c->heat_state = p->heat_source;
  sync_sources(c);
  c->partial_slots = P.partial_slots;
  auto cleanup_fail = [&](int code) {
    std::string m = c->err;
    lbm_destroy(c);
    return fail(nullptr, code, m);
  };
  if (p->workspace) {
    if (p->workspace_bytes < P.total) {
      c->err = "workspace too small: need " + std::to_string(P.total) + " bytes";
      return cleanup_fail(LBM_ENOMEM);
    }
    c->ws = static_cast<char*>(p->workspace);
    c->own_ws = false;
  } else {
    hipError_t e = hipMalloc(&c->ws, P.total);
    if (e != hipSuccess) {
      c->ws = nullptr;
      c->err = std::string("hipMalloc of ") + std::to_string(P.total) + " bytes: " + hipGetErrorString(e);
      return cleanup_fail(LBM_ENOMEM);
    }
    c->own_ws = true;
  }
  c->ws_bytes = P.total;
  c->A = c->ws + P.off_A;
  c->B = P.aa ? nullptr : c->ws + P.off_B;
  c->partials = reinterpret_cast<double*>(c->ws + P.off_part);
  c->history = reinterpret_cast<double*>(c->ws + P.off_hist);
  c->readout = reinterpret_cast<double*>(c->ws + P.off_read);
  if (P.ddf && P.D == 3) c->fld = reinterpret_cast<double*>(c->ws + P.off_fld);
  if (p->wall_y == 2) c->nb = c->ws + P.off_nb;
  c->mlp_cnt = reinterpret_cast<unsigned long long*>(c->ws + P.off_mlp);
  c->mlp_w = reinterpret_cast<float*>(c->ws + P.off_mlp + 256);
  c->mlp_tol = p->mlp_tol;
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    c->err = "hipEventCreate failed";
    return cleanup_fail(LBM_EDEVICE);
  }
  // padding between rows and planes is never read by the kernels, but keep it defined
  hipError_t e = hipMemsetAsync(c->ws, 0, P.off_read, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->readout, rho0, nodes * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->readout + nodes, u0, (size_t)P.D * nodes * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (P.ddf) {
    // Fig. 1: f <- f^eq, g <- g^eq into B, then one collide-only pass B -> A so that A holds
    // the post-collision state of t = 0 (f* differs from f^eq when Phi is on)
    double* d_T0 = c->readout + (size_t)(1 + P.D) * nodes;
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_T0, T0, nodes * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
      e = P.D == 2 ? launch_ddf_rest_state(c->dp, c->partials, c->stream)
                   : launch_ddf3_rest_state(c->dp, c->partials, c->stream);
    double rest[54];
    if (e == hipSuccess) e = hipMemcpyAsync(rest, c->partials, sizeof(rest), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    c->dp.wsum_f = c->dp.wsum_g = 0.0;
    for (int i = 0; i < P.Q; ++i) {
      c->dp.wf[i] = rest[i];
      c->dp.wg[i] = rest[P.Q + i];
      c->dp.wsum_f += rest[i];
      c->dp.wsum_g += rest[P.Q + i];
    }
    if (P.D == 2) {
      if (e == hipSuccess) e = launch_init_ddf(c->fmt, c->readout, c->readout + nodes, d_T0, c->B, c->L, c->dp, c->stream);
      if (e == hipSuccess) e = launch_ddf(c->fmt, p->wall_y != 0, false, c->B, c->A, c->L, c->G, c->dp, c->s_enc, c->s_dec, nullptr, c->nb, nullptr, c->stream);
    } else {
      if (e == hipSuccess) e = launch_init_ddf3(c->kind, c->readout, c->readout + nodes, d_T0, c->B, c->L, c->dp, c->stream);
      if (e == hipSuccess) e = launch_ddf3(c->kind, p->wall_y != 0, false, c->B, c->A, c->L, c->G, c->dp, c->fld, c->nb, nullptr, nullptr, c->stream);
    }
  } else if (e == hipSuccess && c->codec >= 0) {
    e = launch_init_bgk_red(c->readout, c->readout + nodes, c->A, c->L, c->stream);
  } else if (e == hipSuccess) {
    e = launch_init_bgk(c->kind, c->D, c->readout, c->readout + nodes, c->A, c->L, c->aa, c->omega, c->F, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    c->err = std::string("initialisation: ") + hipGetErrorString(e);
    return cleanup_fail(LBM_EDEVICE);
  }
  *out = c;
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int64_t n) {
  if (!c) return fail(nullptr, LBM_ESTATE, "NULL context");
  if (n < 0) return fail(c, LBM_EINVAL, "n must be >= 0");
  const int de = c->p.diag_every;
  const int64_t hist_before = c->hist_written;
  for (int64_t k = 0; k < n; ++k) {
    const int64_t tn = c->t + 1;
    const bool diag = de > 0 && tn % de == 0;
    double* part = diag ? c->partials : nullptr;
    int records = c->G.blocks();  // diagnostics records the step writes
    hipError_t e;
    if (c->p.collision == LBM_COLLIDE_MLP) {
      if (!c->mlp_set) return fail(c, LBM_ESTATE, "surrogate weights not installed (lbm_set_mlp)");
      e = launch_bgk_d2q9_mlp(c->A, c->B, c->L, c->G, c->omega, c->p.wall_y != 0, c->mlp_w, c->mlp_tol, c->mlp_cnt, part, c->stream);
    } else if (c->ddf && c->D == 3)
      e = launch_ddf3(c->kind, c->p.wall_y != 0, true, c->A, c->B, c->L, c->G, c->dp, c->fld, c->nb, part, &records, c->stream);
    else if (c->ddf)
      e = launch_ddf(c->fmt, c->p.wall_y != 0, true, c->A, c->B, c->L, c->G, c->dp, c->s_enc, c->s_dec, part, c->nb, &records, c->stream);
    else if (c->codec >= 0)
      e = launch_bgk_d2q9_red(c->codec, c->A, c->B, c->L, c->G, c->omega, c->p.wall_y != 0, c->s_enc, c->s_dec, part, c->stream);
    else if (c->aa && c->D == 2)
      e = launch_bgk_d2q9_aa(c->kind, (c->t & 1) != 0, c->A, c->L, c->G, c->omega, c->F, c->p.wall_y != 0, part, c->stream);
    else if (c->aa)
      e = launch_bgk_d3q27_aa(c->kind, (c->t & 1) != 0, c->A, c->L, c->G, c->omega, c->F, c->p.wall_y != 0, part, c->stream);
    else if (c->D == 2)
      e = launch_bgk_d2q9(c->kind, c->A, c->B, c->L, c->G, c->omega, c->F, c->p.wall_y != 0, part, c->stream);
    else
      e = launch_bgk_d3q27(c->kind, c->A, c->B, c->L, c->G, c->omega, c->F, c->p.wall_y != 0, part, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "step kernel launch");
    if (diag) {
      double* slot = c->history + (c->hist_written % kHistoryCap) * 6;
      e = launch_diag_finalize(c->partials, records, (double)tn, slot, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "diagnostics launch");
      ++c->hist_written;
    }
    if (!c->aa) std::swap(c->A, c->B);
    c->t = tn;
    c->F_state = c->F;
    c->heat_state = c->heat;
  }
  if (c->hist_written > hist_before) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int64_t cnt = std::min<int64_t>(c->hist_written - hist_before, kHistoryCap);
    std::vector<double> h((size_t)kHistoryCap * 6);
    HIP_TRY(c, hipMemcpy(h.data(), c->history, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < cnt; ++k) {
      const int64_t slot = (c->hist_written - 1 - k) % kHistoryCap;
      for (int v = 1; v < 6; ++v)
        if (!std::isfinite(h[slot * 6 + v]))
          return fail(c, LBM_EUNSTABLE, "non-finite conservation total at t = " + std::to_string((int64_t)h[slot * 6]));
    }
  }
  return LBM_OK;
}

int lbm_set_force(lbm_ctx* c, const double* force) {
  if (!c) return fail(nullptr, LBM_ESTATE, "NULL context");
  if (!force) return fail(c, LBM_EINVAL, "force is NULL");
  std::string why;
  if (int rc = validate_sources(&c->p, force, c->heat, why)) return fail(c, rc, why);
  c->F.x = force[0];
  c->F.y = force[1];
  c->F.z = c->D == 3 ? force[2] : 0.0;
  sync_sources(c);
  return LBM_OK;
}

int lbm_set_heat_source(lbm_ctx* c, double heat_source) {
  if (!c) return fail(nullptr, LBM_ESTATE, "NULL context");
  const double f[3] = {c->F.x, c->F.y, c->F.z};
  std::string why;
  if (int rc = validate_sources(&c->p, f, heat_source, why)) return fail(c, rc, why);
  c->heat = heat_source;
  sync_sources(c);
  return LBM_OK;
}

int lbm_time_steps(lbm_ctx* c, int64_t n, float* ms) {
  if (!c) return fail(nullptr, LBM_ESTATE, "NULL context");
  if (!ms) return fail(c, LBM_EINVAL, "ms is NULL");
  HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
  int rc = lbm_step(c, n);
  if (rc) return rc;
  HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
  HIP_TRY(c, hipEventSynchronize(c->ev1));
  HIP_TRY(c, hipEventElapsedTime(ms, c->ev0, c->ev1));
  return LBM_OK;
}

int lbm_moments(lbm_ctx* c, double* rho, double* u, double* T, double* totals) {
  if (!c) return fail(nullptr, LBM_ESTATE, "NULL context");
  const int64_t nodes = c->L.nodes();
  double* d_rho = c->readout;
  double* d_u = c->readout + nodes;
  double* d_T = c->readout + (1 + c->D) * nodes;
  double* d_e = d_T + nodes;
  if (c->ddf) {
    // the read-out removes the sources of the collision that produced the stored state
    DdfParams rd = c->dp;
    rd.Fx = c->F_state.x;
    rd.Fy = c->F_state.y;
    rd.Fz = c->F_state.z;
    rd.Q = c->heat_state;
    if (c->D == 3)
      HIP_TRY(c, launch_moments_ddf3(c->kind, c->A, c->L, rd, d_rho, d_u, d_T, d_e, c->stream));
    else
      HIP_TRY(c, launch_moments_ddf(c->fmt, c->A, c->L, rd, d_rho, d_u, d_T, d_e, c->stream));
  } else if (c->codec >= 0)
    HIP_TRY(c, launch_moments_bgk_red(c->A, c->L, d_rho, d_u, c->stream));
  else
    HIP_TRY(c, launch_moments_bgk(c->kind, c->D, c->A, c->L, view_of(c), c->p.wall_y != 0, c->F_state, d_rho, d_u, c->stream));
  if (totals) {
    const int nparts = std::min(512, c->partial_slots - 2);
    double* out = c->partials + (size_t)nparts * kDiagValues;  // 6 doubles after the partials
    HIP_TRY(c, launch_field_totals(c->D, d_rho, d_u, c->ddf ? d_e : nullptr, nodes, !c->ddf, c->partials, nparts, out, c->stream));
    double h[6];
    HIP_TRY(c, hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < kDiagValues; ++k) totals[k] = h[1 + k];
  }
  if (rho) HIP_TRY(c, hipMemcpyAsync(rho, d_rho, nodes * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (u) HIP_TRY(c, hipMemcpyAsync(u, d_u, (size_t)c->D * nodes * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (T && c->ddf) HIP_TRY(c, hipMemcpyAsync(T, d_T, nodes * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int lbm_populations(lbm_ctx* c, double* f, double* g) {
  if (!c) return fail(nullptr, LBM_ESTATE, "NULL context");
  if (!f) return fail(c, LBM_EINVAL, "f is NULL");
  const int64_t nodes = c->L.nodes();
  for (int i = 0; i < c->planes; ++i) {
    double* dst = i < c->Q ? f + (size_t)i * nodes : (g ? g + (size_t)(i - c->Q) * nodes : nullptr);
    if (!dst) continue;
    if (c->ddf)
      HIP_TRY(c, launch_decode_ddf(c->fmt, c->Q, i, c->A, c->L, c->dp, c->s_dec, c->readout, c->stream));
    else if (c->codec >= 0)
      HIP_TRY(c, launch_decode_bgk_red(c->codec, i, c->A, c->L, c->s_dec, c->readout, c->stream));
    else
      HIP_TRY(c, launch_decode_f(c->kind, c->D, i, c->A, c->L, view_of(c), c->p.wall_y != 0, c->readout, c->stream));
    HIP_TRY(c, hipMemcpyAsync(dst, c->readout, nodes * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return LBM_OK;
}

int lbm_time(const lbm_ctx* c, int64_t* t) {
  if (!c) return fail(nullptr, LBM_ESTATE, "NULL context");
  if (!t) return LBM_EINVAL;
  *t = c->t;
  return LBM_OK;
}

int lbm_diag_history(lbm_ctx* c, double* out, int32_t max_entries, int32_t* n_entries) {
  if (!c) return fail(nullptr, LBM_ESTATE, "NULL context");
  if (!out || !n_entries || max_entries < 0) return fail(c, LBM_EINVAL, "invalid output arguments");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int64_t avail = std::min<int64_t>(c->hist_written, kHistoryCap);
  const int64_t cnt = std::min<int64_t>(avail, max_entries);
  std::vector<double> h((size_t)kHistoryCap * 6);
  HIP_TRY(c, hipMemcpy(h.data(), c->history, h.size() * sizeof(double), hipMemcpyDeviceToHost));
  const int64_t first = c->hist_written - avail;  // oldest kept entry
  for (int64_t k = 0; k < cnt; ++k) {
    const int64_t slot = (first + k) % kHistoryCap;
    std::memcpy(out + k * 6, h.data() + slot * 6, 6 * sizeof(double));
  }
  *n_entries = (int32_t)cnt;
  return LBM_OK;
}

int lbm_set_mlp(lbm_ctx* c, const float* weights, double tol) {
  if (!c) return fail(nullptr, LBM_ESTATE, "NULL context");
  if (c->p.collision != LBM_COLLIDE_MLP) return fail(c, LBM_EINVAL, "context was not created with collision = LBM_COLLIDE_MLP");
  if (!weights) return fail(c, LBM_EINVAL, "weights is NULL");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(c, LBM_EINVAL, "tol must be finite and >= 0");
  for (int k = 0; k < kMlpParams; ++k)
    if (!std::isfinite(weights[k])) return fail(c, LBM_EINVAL, "non-finite weight at index " + std::to_string(k));
  HIP_TRY(c, hipMemcpyAsync(c->mlp_w, weights, (size_t)kMlpParams * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->mlp_cnt, 0, 16, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->mlp_tol = tol;
  c->mlp_set = true;
  return LBM_OK;
}

int lbm_mlp_stats(lbm_ctx* c, int64_t* fallbacks, int64_t* updates) {
  if (!c) return fail(nullptr, LBM_ESTATE, "NULL context");
  if (c->p.collision != LBM_COLLIDE_MLP) return fail(c, LBM_EINVAL, "no surrogate collision in this context");
  unsigned long long h[2] = {0, 0};
  HIP_TRY(c, hipMemcpyAsync(h, c->mlp_cnt, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (fallbacks) *fallbacks = (int64_t)h[0];
  if (updates) *updates = (int64_t)h[1];
  return LBM_OK;
}

int lbm_harvest(lbm_ctx* c, int64_t n, const int64_t* dev_nodes, float* dev_x, float* dev_y) {
  if (!c) return fail(nullptr, LBM_ESTATE, "NULL context");
  if (c->D != 2 || c->ddf || c->kind != 0 || c->codec >= 0 || c->F.on() || c->F_state.on())
    return fail(c, LBM_EINVAL, "harvest needs a D2Q9 isothermal context with float32 storage and no force");
  if (n < 0 || (n > 0 && (!dev_nodes || !dev_x || !dev_y))) return fail(c, LBM_EINVAL, "invalid harvest buffers");
  if (n == 0) return LBM_OK;
  HIP_TRY(c, launch_harvest(c->A, c->L, c->p.wall_y != 0, view_of(c), c->omega, dev_nodes, n, dev_x, dev_y, c->stream));
  return LBM_OK;
}

namespace {
int mlp_fail(int code, const std::string& msg) { return fail(nullptr, code, msg); }

int mlp_ensure_partials(lbm_mlp* m, int B) {
  const size_t rows = (size_t)mlp_partial_count(B);
  if (rows <= m->partial_rows) return LBM_OK;
  if (m->partials) (void)hipFree(m->partials);
  m->partials = nullptr;
  m->partial_rows = 0;
  hipError_t e = hipMalloc(&m->partials, rows * (kMlpParams + 1) * sizeof(float));
  if (e != hipSuccess) return mlp_fail(LBM_ENOMEM, std::string("trainer partials: ") + hipGetErrorString(e));
  m->partial_rows = rows;
  return LBM_OK;
}
}  // namespace

int lbm_mlp_create(const float* weights, void* stream, lbm_mlp** out) {
  if (!out) return mlp_fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!weights) return mlp_fail(LBM_EINVAL, "weights is NULL");
  lbm_mlp* m = new lbm_mlp();
  m->stream = static_cast<hipStream_t>(stream);
  const size_t bytes = (size_t)kMlpParams * 4;
  hipError_t e = hipMalloc(&m->w, bytes);
  if (e == hipSuccess) e = hipMalloc(&m->m, bytes);
  if (e == hipSuccess) e = hipMalloc(&m->v, bytes);
  if (e == hipSuccess) e = hipMalloc(&m->scratch, 256);
  if (e == hipSuccess) e = hipMemcpyAsync(m->w, weights, bytes, hipMemcpyHostToDevice, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->m, 0, bytes, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->v, 0, bytes, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) {
    lbm_mlp_destroy(m);
    return mlp_fail(LBM_ENOMEM, std::string("trainer allocation: ") + hipGetErrorString(e));
  }
  *out = m;
  return LBM_OK;
}

void lbm_mlp_destroy(lbm_mlp* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->stream);
  if (m->w) (void)hipFree(m->w);
  if (m->m) (void)hipFree(m->m);
  if (m->v) (void)hipFree(m->v);
  if (m->partials) (void)hipFree(m->partials);
  if (m->scratch) (void)hipFree(m->scratch);
  delete m;
}

int lbm_mlp_get(lbm_mlp* m, float* w) {
  if (!m) return mlp_fail(LBM_ESTATE, "NULL trainer");
  if (!w) return mlp_fail(LBM_EINVAL, "w is NULL");
  hipError_t e = hipMemcpyAsync(w, m->w, (size_t)kMlpParams * 4, hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  return e == hipSuccess ? LBM_OK : mlp_fail(LBM_EDEVICE, hipGetErrorString(e));
}

int lbm_mlp_forward(lbm_mlp* m, const float* x, int64_t n, float* y) {
  if (!m) return mlp_fail(LBM_ESTATE, "NULL trainer");
  if (n < 0 || (n > 0 && (!x || !y))) return mlp_fail(LBM_EINVAL, "invalid buffers");
  if (n == 0) return LBM_OK;
  hipError_t e = launch_mlp_forward(x, n, m->w, y, m->stream);
  return e == hipSuccess ? LBM_OK : mlp_fail(LBM_EDEVICE, hipGetErrorString(e));
}

int lbm_mlp_grad(lbm_mlp* m, const float* x, const float* t, int64_t n, float* g, float* loss) {
  // n is capped at the training batch limit (checked first, before any state): the partials
  // hold one row of 5578 floats per 64 samples (22 KiB), about 360 MB at 2^20 samples
  if (n <= 0 || n > (1 << 20)) return mlp_fail(LBM_EINVAL, "n outside [1, 2^20]");
  if (!m) return mlp_fail(LBM_ESTATE, "NULL trainer");
  if (!x || !t || !g) return mlp_fail(LBM_EINVAL, "invalid buffers");
  int rc = mlp_ensure_partials(m, (int)n);
  if (rc) return rc;
  hipError_t e = launch_mlp_grad(x, t, n, 0, (int)n, m->w, m->partials, m->stream);
  if (e == hipSuccess)
    e = launch_mlp_reduce_adam(m->partials, mlp_partial_count((int)n), g, m->scratch, m->w, m->m, m->v, false, 0.0f, 1, m->stream);
  if (e == hipSuccess && loss) {
    e = hipMemcpyAsync(loss, m->scratch, sizeof(float), hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  }
  return e == hipSuccess ? LBM_OK : mlp_fail(LBM_EDEVICE, hipGetErrorString(e));
}

int lbm_mlp_train(lbm_mlp* m, const float* x, const float* t, int64_t n, int32_t batch, int64_t steps, float lr) {
  if (!m) return mlp_fail(LBM_ESTATE, "NULL trainer");
  if (n <= 0 || batch <= 0 || batch > (1 << 20) || steps < 0 || !x || !t || !(lr > 0.0f))
    return mlp_fail(LBM_EINVAL, "invalid training arguments");
  int rc = mlp_ensure_partials(m, batch);
  if (rc) return rc;
  for (int64_t k = 0; k < steps; ++k) {
    hipError_t e = launch_mlp_grad(x, t, n, m->offset, batch, m->w, m->partials, m->stream);
    m->t += 1;
    if (e == hipSuccess)
      e = launch_mlp_reduce_adam(m->partials, mlp_partial_count(batch), nullptr, nullptr, m->w, m->m, m->v, true, lr, m->t, m->stream);
    if (e != hipSuccess) return mlp_fail(LBM_EDEVICE, hipGetErrorString(e));
    m->offset = (m->offset + batch) % n;
  }
  return LBM_OK;
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  if (c->stream || c->ws) (void)hipStreamSynchronize(c->stream);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->own_ws && c->ws) (void)hipFree(c->ws);
  delete c;
}

}  // extern "C"
