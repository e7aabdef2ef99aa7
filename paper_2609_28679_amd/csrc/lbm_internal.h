// Internal declarations shared by the C-ABI host code and the HIP kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbm {

constexpr int kBlock = 256;          // threads per workgroup of the streaming kernels
constexpr int kDiagValues = 5;       // mass, j_x, j_y, j_z, energy
constexpr int kHistoryCap = 4096;    // diagnostics ring entries
constexpr int kNumXcd = 8;           // MI355X: 8 accelerator complex dies, round-robin dispatch

// Structure-of-arrays population layout: element (q, z, y, x) lives at
// q * plane + (z * ny + y) * pitch + x.
struct Layout {
  int nx, ny, nz;
  int64_t pitch;  // elements per x row (nx rounded up to 64 elements)
  int64_t plane;  // elements per population plane (padded so planes do not alias channels)
  int64_t nodes() const { return (int64_t)nx * ny * nz; }
};

// Streaming-kernel launch geometry shared by every population kernel.
struct Grid {
  int bx;        // workgroup width in threads (<= kBlock, multiple of 64)
  int nbx;       // workgroups along x
  int rows;      // (y, z) rows processed by one workgroup
  int nby;       // workgroups along the row index
  int blocks() const { return nbx * nby; }
};

// Uniform body force per unit volume (lattice units); zero when the context has none.
struct Force {
  double x = 0.0, y = 0.0, z = 0.0;
  bool on() const { return x != 0.0 || y != 0.0 || z != 0.0; }
};

// Workgroups along the second grid dimension are kept within 65536 (the launch limit of this
// dimension on the device): lattices with more rows give each workgroup more rows.
constexpr int kMaxGridY = 65536;
inline void fit_rows(Grid& G, int64_t nrows) {
  if (G.rows < 1) G.rows = 1;
  if ((nrows + G.rows - 1) / G.rows > kMaxGridY) G.rows = (int)((nrows + kMaxGridY - 1) / kMaxGridY);
  G.nby = (int)((nrows + G.rows - 1) / G.rows);
}

// Population layout for elements of `elem` bytes (row pitch and padded plane stride).
Layout make_layout(int nx, int ny, int nz, int elem);
Grid make_grid(const Layout& L);

// Ideal-gas double-distribution parameters (lattice units).
struct DdfParams {
  double R;    // gas constant
  double cv;   // heat capacity at constant volume
  double r_cv; // R / cv (theta = R T = (R / cv) e)
  double inv_R;  // 1 / R (T = theta / R)
  double mu;   // dynamic shear viscosity; tau = mu / P per node
  int phi;     // 0: no Galilean correction, 1: central derivative, 2: upwind derivative
  // uniform body force (Fx, Fy) and heat source Q of the collision (lattice units); src = any
  // of them non-zero
  double Fx = 0.0, Fy = 0.0, Fz = 0.0, Q = 0.0;
  bool src = false;
  // transport control: alpha = (D+2)/D - gamma - eta/mu in theta* (bulk viscosity eta) and
  // qc = c_p - k/mu in q^c = P qc grad T (Prandtl number); full = either non-zero
  double alpha = 0.0, qc = 0.0;
  bool full = false;
  // van der Waals fluid (eos = 1): P = rho R T / (1 - vb rho) - va rho^2, e = c_v T - va rho.
  // Its alpha is computed per node with the bulk viscosity ratio eta, and its heat flux
  // q^c = P (grad h - kmu grad T) uses kmu = k / mu = (c_v + R) / Pr; it always takes the
  // extended path (full).
  int eos = 0;
  double va = 0.0, vb = 0.0, eta = 0.0, kmu = 0.0;
  // the kernels take the extended path (shifted state with sources and/or transport terms)
  bool ext() const { return src || full; }
  // non-equilibrium extrapolation walls (rows, in D3Q27 planes, y = 0 and ny-1 on the walls):
  // wall velocity uw[side][axis] (x, y, z; y is 0, z is 0 in D2Q9) and temperature Tw[side]
  // (side 0: y = 0, 1: y = ny - 1); neq_literal selects rho_B = rho_N instead of
  // rho_N T_N / T_W
  int neq = 0, neq_literal = 0;
  double uw[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  double Tw[2] = {1.0, 1.0};
  // storage shift: f^eq and g^eq at rest at the reference state rho = 1, T = 1 (computed by
  // launch_ddf_rest_state / launch_ddf3_rest_state on the device at context creation; the
  // first 9 entries for D2Q9, 27 for D3Q27)
  double wf[27];
  double wg[27];
  // their totals sum_i wf_i and sum_i wg_i (D3Q27: the moments sum the stored deviations and
  // add these once)
  double wsum_f = 0.0, wsum_g = 0.0;
};

// ---- launchers (return the first HIP error) -----------------------------------------------
// Real = float (kind 0) or double (kind 1).
hipError_t launch_bgk_d2q9(int kind, const void* A, void* B, const Layout& L, const Grid& G,
                           double omega, const Force& F, bool walls, double* partials,
                           hipStream_t s);
hipError_t launch_bgk_d3q27(int kind, const void* A, void* B, const Layout& L, const Grid& G,
                            double omega, const Force& F, bool walls, double* partials,
                            hipStream_t s);
// Single-buffer steps (in place on A); odd = the step count so far is odd.
hipError_t launch_bgk_d2q9_aa(int kind, bool odd, void* A, const Layout& L, const Grid& G,
                              double omega, const Force& F, bool walls, double* partials,
                              hipStream_t s);
hipError_t launch_bgk_d3q27_aa(int kind, bool odd, void* A, const Layout& L, const Grid& G,
                               double omega, const Force& F, bool walls, double* partials,
                               hipStream_t s);
// swap: store population i in slot Q-1-i (single-buffer state at an even step count). With a
// force the equilibrium is collided once (the stored state is post-collision at t = 0).
hipError_t launch_init_bgk(int kind, int D, const double* rho, const double* u, void* A,
                           const Layout& L, bool swap, double omega, const Force& F,
                           hipStream_t s);
// view: -1 two-buffer state; 0 / 1 single-buffer state after an even / odd step count.
hipError_t launch_moments_bgk(int kind, int D, const void* A, const Layout& L, int view,
                              bool walls, const Force& F, double* rho, double* u, hipStream_t s);
// Post-collision population i of the stored state decoded to float64 f_i (nodes values, no
// padding).
hipError_t launch_decode_f(int kind, int D, int i, const void* A, const Layout& L, int view,
                           bool walls, double* f, hipStream_t s);
// Double-distribution kernels (D2Q9). Storage format fmt / kind: 0 float32, 1 float64 (planes
// 0..8 hold f - w, 9..17 hold g - v); 2 bfloat16, 3 float16 reduced storage (4 float32 moment
// planes, then 6 f and 8 g uint16 planes).
Grid make_grid_ddf(const Layout& L, int halo, bool reduced);
// out[0..8] = f^eq, out[9..17] = g^eq at rho = 1, u = 0, T = 1 (18 doubles, device memory).
hipError_t launch_ddf_rest_state(const DdfParams& prm, double* out, hipStream_t s);
// nb: boundary-row buffer of the non-equilibrium extrapolation walls (2 x 18 rows of `pitch`
// storage elements; used when prm.neq, NULL otherwise).
// records: set to the number of per-workgroup diagnostics records the step writes to partials
// (at most G.blocks(); may be NULL).
hipError_t launch_ddf(int fmt, bool walls, bool pull, const void* A, void* B, const Layout& L,
                      const Grid& G, const DdfParams& prm, float s_enc, float s_dec,
                      double* partials, void* nb, int* records, hipStream_t s);
hipError_t launch_init_ddf(int kind, const double* rho, const double* u, const double* T,
                           void* A, const Layout& L, const DdfParams& prm, hipStream_t s);
hipError_t launch_moments_ddf(int kind, const void* A, const Layout& L, const DdfParams& prm,
                              double* rho, double* u, double* T, double* edens, hipStream_t s);
hipError_t launch_decode_ddf(int kind, int Q, int i, const void* A, const Layout& L,
                             const DdfParams& prm, float s_dec, double* out, hipStream_t s);
// D3Q27 double distribution (float32 kind 0 / float64 kind 1 storage, 54 planes). One step is
// two launches: fluxes (and, with transport control, T and u; for the van der Waals fluid also
// the enthalpy) into `fld` (8 fields of L.plane elements in the storage type, float32 or
// float64), then the collision; pull = false collides in place of streaming. With the central
// derivative of Phi, one launch that marches along z takes both instead (after the
// boundary-plane rebuild with NEQ walls).
Grid make_grid_ddf3(const Layout& L);
hipError_t launch_ddf3_rest_state(const DdfParams& prm, double* out, hipStream_t s);
hipError_t launch_init_ddf3(int kind, const double* rho, const double* u, const double* T,
                            void* A, const Layout& L, const DdfParams& prm, hipStream_t s);
// nb: boundary planes of the non-equilibrium extrapolation walls (2 x 54 planes of nz x pitch
// storage elements; used when prm.neq, NULL otherwise).
// records: set to the number of per-workgroup diagnostics records the step writes to
// partials (may be NULL).
hipError_t launch_ddf3(int kind, bool walls, bool pull, const void* A, void* B, const Layout& L,
                       const Grid& G, const DdfParams& prm, double* fld, void* nb,
                       double* partials, int* records, hipStream_t s);
// Most diagnostics records any D3Q27 double-distribution step writes (grid G of the plan).
int64_t ddf3_max_records(const Layout& L, const Grid& G);
hipError_t launch_moments_ddf3(int kind, const void* A, const Layout& L, const DdfParams& prm,
                               double* rho, double* u, double* T, double* edens, hipStream_t s);
// Reduced storage (D2Q9 isothermal): 3 float32 moment planes then 6 uint16 planes.
// codec 0 = bfloat16, 1 = float16 with scale s_enc = 2^S, s_dec = 2^-S.
Grid make_grid_red(const Layout& L);
// bytes of one isothermal reduced-storage state buffer (planes and strip edge records)
size_t red_state_bytes(const Layout& L);
hipError_t launch_bgk_d2q9_red(int codec, const void* A, void* B, const Layout& L, const Grid& G,
                               double omega, bool walls, float s_enc, float s_dec,
                               double* partials, hipStream_t s);
hipError_t launch_init_bgk_red(const double* rho, const double* u, void* A, const Layout& L,
                               hipStream_t s);
hipError_t launch_moments_bgk_red(const void* A, const Layout& L, double* rho, double* u,
                                  hipStream_t s);
hipError_t launch_decode_bgk_red(int codec, int i, const void* A, const Layout& L, float s_dec,
                                 double* out, hipStream_t s);
// Learned collision surrogate (D2Q9 isothermal, float32 storage).
constexpr int kMlpParams = 5577;
hipError_t launch_mlp_grad(const float* X, const float* T, int64_t n, int64_t start, int B,
                           const float* w, float* partials, hipStream_t s);
int mlp_partial_count(int B);  // partial gradient rows written by launch_mlp_grad (x 5578 floats)
hipError_t launch_mlp_reduce_adam(const float* partials, int nw, float* grad, float* loss, float* w,
                                  float* m, float* v, bool adam, float lr, int64_t t, hipStream_t s);
hipError_t launch_mlp_forward(const float* X, int64_t n, const float* w, float* Y, hipStream_t s);
hipError_t launch_harvest(const void* A, const Layout& L, bool walls, int view, double omega,
                          const int64_t* nodes, int64_t n, float* X, float* Y, hipStream_t s);
Grid make_grid_mlp(const Layout& L);
hipError_t launch_bgk_d2q9_mlp(const void* A, void* B, const Layout& L, const Grid& G, double omega,
                               bool walls, const float* wblob, double tol,
                               unsigned long long* counters, double* partials, hipStream_t s);
// Deterministic final pass over per-block partials: out[0] = t, out[1..5] = totals.
hipError_t launch_diag_finalize(const double* partials, int nblocks, double t, double* out,
                                hipStream_t s);
// Totals of float64 node fields (rho [nodes], u [D][nodes], energy density e [nodes] or NULL).
hipError_t launch_field_totals(int D, const double* rho, const double* u, const double* edens,
                               int64_t nodes, bool kinetic, double* partials, int nparts,
                               double* out, hipStream_t s);

}  // namespace lbm
