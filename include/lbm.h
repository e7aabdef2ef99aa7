/*
 * lbm.h - C ABI of the MI355X (gfx950) lattice Boltzmann collide-and-stream library.
 *
 * The library advances the discrete-velocity populations of the lattice Boltzmann scheme of
 * Chatterjee, Strassle, Hosseini and Karlin, "Consistent lattice Boltzmann model with body
 * force and heat source for compressible flows of generic fluids":
 *   - lattice: nearest-neighbour velocities c_ia in {-1,0,1} (Sec. II C; D3Q27 and its
 *     two-dimensional restriction D2Q9);
 *   - equilibrium: product form f_i^eq = rho prod_a Psi_ia(u_a, theta + u_a^2) (Sec. II C);
 *     energy populations g_i^eq from the operator product acting on E = e + u^2/2 (Sec. II C);
 *   - relaxation: f_i(x + c_i, t + 1) = f_i + 2 beta (f_i^eq - f_i) + (1 - beta)(f_i^* - f_i^eq),
 *     beta = dt / (2 tau + dt) (Eq. LBM_f, LBM_g of Sec. II C, beta of Sec. II B);
 *   - streaming to the neighbours x + c_i, periodic or with half-way bounce-back walls.
 *
 * Conventions shared by every entry point
 *   - Lattice units: dt = 1, c = 1, varsigma^2 = 1/3.
 *   - Host field arrays are float64, C order, indexed [y][x] (2D) or [z][y][x] (3D); a vector
 *     field holds its components first: u[a][y][x] with a = x, y (, z).
 *   - Velocity ordering i = (c_x+1) + 3 (c_y+1) [+ 9 (c_z+1)]; the opposite of i is Q-1-i.
 *   - Every call returns LBM_OK (0) or a negative error code; no exception crosses the ABI.
 *     The text of the most recent error of a context is returned by lbm_last_error(ctx);
 *     errors raised before a context exists are returned by lbm_last_error(NULL) (per thread).
 *   - Work is enqueued on the caller's HIP stream (params.stream, NULL = the null stream).
 *     Calls that hand results to host memory synchronise that stream first.
 *   - A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------------------- */
#define LBM_OK 0
#define LBM_EINVAL (-1)    /* invalid argument or unsupported combination */
#define LBM_ENOMEM (-2)    /* device allocation failed or caller workspace too small */
#define LBM_EDEVICE (-3)   /* a HIP runtime call failed; its text is in lbm_last_error */
#define LBM_EUNSTABLE (-4) /* a conservation diagnostic became non-finite; state left as is */
#define LBM_ESTATE (-5)    /* NULL context, or call not valid in the context's state */

/* ---- parameter values ----------------------------------------------------------------- */
#define LBM_D2Q9 0
#define LBM_D3Q27 1

#define LBM_MODEL_BGK 0 /* isothermal: theta = 1/3, f* = f^eq, g not evolved */
#define LBM_MODEL_DDF 1 /* double distribution, ideal gas P = rho R T, Galilean correction */

#define LBM_STORE_FP32 0 /* populations stored as float32 */
#define LBM_STORE_BF16 1 /* float32 moments + bfloat16 non-equilibrium part f - f^eq */
#define LBM_STORE_FP16 2 /* float32 moments + float16 (f - f^eq) * 2^S */
#define LBM_STORE_FP64 3 /* populations stored and computed in float64 */

#define LBM_COLLIDE_PLAIN 0 /* the paper's collision */
#define LBM_COLLIDE_MLP 1   /* learned surrogate with per-node fallback to the paper's collision */

/* Streaming layout of the population state (isothermal model, D2Q9 or D3Q27, with FP32/FP64
   storage and the paper's collision; every other configuration uses two buffers). */
#define LBM_STREAM_AUTO 0        /* one buffer when its size is at most 384 MiB, else two */
#define LBM_STREAM_TWO_BUFFERS 1 /* pull from buffer A, write buffer B, swap */
#define LBM_STREAM_ONE_BUFFER 2  /* in place, alternating two access patterns (half the memory) */

typedef struct lbm_ctx lbm_ctx; /* opaque; owned by the library */

typedef struct {
  int32_t lattice;   /* LBM_D2Q9 or LBM_D3Q27 */
  int32_t model;     /* LBM_MODEL_BGK or LBM_MODEL_DDF (DDF on D3Q27: FP32/FP64 storage) */
  int32_t storage;   /* LBM_STORE_*; reduced storage (BF16, FP16): D2Q9 only */
  int32_t collision; /* LBM_COLLIDE_*; MLP: D2Q9 BGK with FP32 storage only */
  int32_t nx, ny, nz; /* lattice size in nodes; nz = 1 for D2Q9; each >= 1 (nx, ny >= 3) */
  int32_t wall_y;     /* 0: periodic in y; 1: half-way bounce-back walls at y = -1/2 and ny-1/2;
                         2 (DDF, D2Q9 or D3Q27, FP32/FP64, ny >= 3, no sources; ideal gas or
                         van der Waals): non-equilibrium extrapolation walls on the rows (D2Q9)
                         or planes (D3Q27) y = 0 and y = ny-1 with the velocities wall_u and
                         temperatures wall_T (App. B, thermal Couette). With the upwind Phi
                         derivative (phi = 2) the side on those rows follows the wall velocity
                         (central in y there). */
  double tau;  /* BGK: tau_LB = 1/(2 beta) > 1/2, so nu = (tau - 1/2)/3.
                  DDF: the same value at the reference pressure P0 = 1/3 defines the dynamic
                  viscosity mu = (tau - 1/2) P0; per node tau_kin = mu / P (Sec. II A). */
  double R, cv;        /* DDF ideal gas constant and heat capacity (Sec. III A); Pr = 1 and the
                          bulk viscosity eta = mu (2/D - R/c_v) (Sec. II E) so alpha = 0 */
  double force[3];     /* uniform body force per unit volume F (lattice units), applied through
                          the shifted equilibria at u* = u + F/rho (Sec. II C) with
                          rho u = sum c f + F/2 (DDF: also T* and rho E = sum g + u.F/2).
                          The paper's collision with FP32/FP64 storage only; force[2] = 0 for
                          D2Q9; all zero = no force. */
  double heat_source;  /* DDF only: uniform heat source Q per unit volume and time step, applied
                          through theta* = theta + (gamma - 1) Q/rho and T* = T + Q/(rho c_v)
                          with rho E = sum g + Q/2 (Sec. II C); FP32/FP64 storage; 0 = none. */
  double prandtl;      /* DDF: Prandtl number Pr = mu c_p / k > 0 (default 1); Pr != 1 adds the
                          heat-flux term c_i.q^c/2, q^c = P (grad h - (k/mu) grad T), to g*
                          (Sec. II C, Eq. qc_1; central differences). FP32/FP64 storage. */
  double eta_over_mu;  /* DDF: bulk viscosity ratio eta/mu >= 0, or < 0 (default -1) for the
                          Navier-Stokes value 2/D - R/c_v; sets alpha = (D+2)/D - gamma - eta/mu
                          in theta* = theta + alpha theta div u (Sec. II A). Values >= 0 need
                          FP32/FP64 storage. */
  int32_t eos;         /* DDF equation of state: 0 = ideal gas (Sec. III A), 1 = van der Waals
                          P = rho R T / (1 - b rho) - a rho^2 with e = c_v T - a rho (Sec. III C);
                          van der Waals: D2Q9 or D3Q27, FP32/FP64 storage, any wall_y.
                          Its alpha and q^c are per node (k/mu = (c_v + R) / prandtl). */
  double vdw_a, vdw_b; /* van der Waals a >= 0, b >= 0 (lattice units); 1 - b rho > 0 */
  double wall_u[2][3]; /* wall_y = 2: wall velocity [bottom (y = 0), top (y = ny-1)][x, y, z];
                          tangential: y component 0; z component 0 in D2Q9 */
  double wall_T[2];    /* wall_y = 2: wall temperatures [bottom, top], > 0 */
  int32_t wall_density; /* wall_y = 2: boundary density rho_B; 0 (default) = the density with
                          P(rho_B, T_W) = P(rho_N, T_N), the neighbour's pressure continued to the
                          wall (ideal gas: rho_N T_N / T_W; van der Waals: the root on the wall
                          isotherm, which must be supercritical: T_W > 8 a / (27 b R), b > 0),
                          1 = rho_N (the extrapolation as written in App. B; it leaks mass where
                          T_N != T_W). The wall equilibrium takes theta_W = P(rho_B, T_W)/rho_B
                          and e_W = e(rho_B, T_W). */
  int32_t phi;         /* DDF: 1 = Galilean correction Phi on (the paper), 0 = off */
  int32_t fp16_scale_log2; /* LBM_STORE_FP16: S in [0, 24]; stored value = (f - f^eq) * 2^S */
  int32_t diag_every;  /* > 0: every diag_every steps record float64 totals (mass, momentum,
                          energy) computed inside the step kernel; 0 = off */
  int32_t streaming;   /* LBM_STREAM_*; LBM_STREAM_ONE_BUFFER is rejected where unsupported.
                          The choice changes memory use and speed, not the results. */
  double mlp_tol;      /* LBM_COLLIDE_MLP fallback threshold (see lbm_set_mlp) */
  void* stream;        /* hipStream_t for all work of this context; NULL = null stream */
  void* workspace;     /* optional caller-owned device memory (>= lbm_workspace_size bytes,
                          256-byte aligned); NULL: the library allocates and frees its own */
  size_t workspace_bytes;
} lbm_params;

/* Fill p with defaults: D2Q9 BGK FP32 plain, 64 x 64 x 1, periodic, tau 0.8, R = 1/3,
   c_v = 5/6, ideal gas, no force or heat source, Pr 1, Navier-Stokes bulk viscosity, phi 1, S = 16, no diagnostics, automatic streaming layout, tol 0.05, null
   stream, no workspace. */
void lbm_default_params(lbm_params* p);

/* Device bytes the context needs for p (population buffers: one or two, reduction scratch,
   diagnostics history). Returns LBM_EINVAL for invalid parameters. */
int lbm_workspace_size(const lbm_params* p, size_t* bytes);

/* Create a context and initialise the populations to the equilibrium of the initial fields
   (Fig. 1: f <- f^eq, g <- g^eq). rho0: [nodes], u0: [D][nodes], T0: [nodes] for the DDF
   model (NULL otherwise); all float64 host arrays, copied. For the DDF model with Phi on, a
   collide-only pass is applied so the stored state is the post-collision state of t = 0.
   Rejects tau <= 1/2, invalid sizes, unsupported combinations, and initial states whose
   product-form factors are not all positive (theta + u_a^2 >= 1 or theta + u_a^2 <= |u_a|).
   *out is NULL on failure. */
int lbm_create(const lbm_params* p, const double* rho0, const double* u0, const double* T0,
               lbm_ctx** out);

/* Advance n >= 0 time steps (one fused pull stream-collide kernel launch per step), enqueued
   asynchronously on the context stream. With diag_every > 0 the call synchronises once at its
   end and returns LBM_EUNSTABLE if any totals recorded during the call are non-finite. */
int lbm_step(lbm_ctx* ctx, int64_t n);

/* Replace the uniform body force (force[3], as lbm_params.force) for the collisions of the
   following steps, e.g. a force that varies in time. The stored state keeps the force of the
   collision that produced it, which lbm_moments uses (rho u = sum c f~ - F/2 after a forced
   collision). LBM_EINVAL where lbm_params.force would be rejected; no device work. */
int lbm_set_force(lbm_ctx* ctx, const double* force);

/* The same for the heat source Q (lbm_params.heat_source; DDF only). */
int lbm_set_heat_source(lbm_ctx* ctx, double heat_source);

/* Time n steps with HIP events recorded on the context stream around the launches; *ms is
   the elapsed time in milliseconds. Synchronises. */
int lbm_time_steps(lbm_ctx* ctx, int64_t n, float* ms);

/* Moments of the pre-collision populations at the current time t (Sec. II C: rho = sum f,
   rho u = sum c f (+ F/2 with a body force), rho E = sum g (+ (u.F + Q)/2 with sources)). rho: [nodes], u: [D][nodes], T: [nodes] (DDF only, may be
   NULL), totals: {mass, rho u_x, rho u_y, rho u_z, energy} as float64 sums (energy = kinetic
   energy sum rho |u|^2 / 2 for BGK, total energy sum rho E for DDF); any output may be NULL.
   Caller-owned host buffers. Synchronises. */
int lbm_moments(lbm_ctx* ctx, double* rho, double* u, double* T, double* totals);

/* Stored post-collision populations of the current time, decoded to float64:
   f: [Q][nodes]; g: [Q][nodes] for DDF (may be NULL otherwise). Synchronises. */
int lbm_populations(lbm_ctx* ctx, double* f, double* g);

/* Current time step count (number of steps taken since creation). */
int lbm_time(const lbm_ctx* ctx, int64_t* t);

/* Diagnostics recorded since creation (oldest first, capacity 4096 entries kept as a ring):
   out receives up to max_entries rows of 6 doubles {t, mass, rho u_x, rho u_y, rho u_z,
   energy}; *n_entries is the number written. Synchronises. */
int lbm_diag_history(lbm_ctx* ctx, double* out, int32_t max_entries, int32_t* n_entries);

/* ---- learned collision surrogate (D2Q9, isothermal model) -------------------------------
   Network 12 -> 64 -> 64 -> 9 with GELU (tanh form) on the hidden layers, followed by the
   exact projection of the outputs onto zero mass and momentum. Inputs per node, with f the
   pre-collision populations and f^eq the product-form equilibrium:
     x = [1024 (f_i - f_i^eq)/rho (i = 0..8), 16 u_x, 16 u_y, omega]
   output y decodes to f~_i = f_i^eq + rho y_i / 1024. Parameter blob (float32, 5577 values):
     W1[64][12], b1[64], W2[64][64], b2[64], W3[9][64], b3[9].
   Matrix products run on bfloat16 matrix cores with float32 accumulation. */

#define LBM_MLP_NPARAM 5577

/* Install surrogate weights (host float32 blob, copied) and the fallback tolerance tol >= 0:
   a node uses the surrogate result only if |f~_mlp - f~_plain|_2 <= tol |f~_plain - f^eq|_2,
   otherwise the paper's collision. Requires collision = LBM_COLLIDE_MLP. */
int lbm_set_mlp(lbm_ctx* ctx, const float* weights, double tol);

/* Fallback statistics since lbm_set_mlp: nodes that used the plain collision, and node
   updates done with the surrogate collision. Synchronises. */
int lbm_mlp_stats(lbm_ctx* ctx, int64_t* fallbacks, int64_t* updates);

/* Training-pair harvest at the current time: for n node indices (device int64 array, values
   in [0, nodes)), write the network inputs of the populations the next step would collide
   (dev_x: [n][12] float32) and the plain-collision targets 1024 (f~_i - f_i^eq)/rho
   (dev_y: [n][9] float32). D2Q9 BGK with float32 storage and no body force only. */
int lbm_harvest(lbm_ctx* ctx, int64_t n, const int64_t* dev_nodes, float* dev_x, float* dev_y);

typedef struct lbm_mlp lbm_mlp; /* trainer: float32 master weights + Adam state on device */

/* Create a trainer from a host float32 parameter blob; stream as in lbm_params. */
int lbm_mlp_create(const float* weights, void* stream, lbm_mlp** out);
void lbm_mlp_destroy(lbm_mlp* m);
/* Copy the float32 master weights to host (5577 values). Synchronises. */
int lbm_mlp_get(lbm_mlp* m, float* weights);
/* Forward pass for n samples: dev_x [n][12] -> dev_y [n][9] (projected outputs). */
int lbm_mlp_forward(lbm_mlp* m, const float* dev_x, int64_t n, float* dev_y);
/* Mean-squared-error loss and its gradient for one batch of 1 <= n <= 2^20 samples
   (dev_x [n][12], dev_t [n][9]); dev_grad receives 5577 float32 values in the blob layout,
   *loss the loss (pass NULL to skip the loss read, which avoids a synchronisation). The
   per-64-sample partial gradients live in a trainer buffer (22 KiB per 64 samples) that is
   allocated, or grown, on the first call that needs it. */
int lbm_mlp_grad(lbm_mlp* m, const float* dev_x, const float* dev_t, int64_t n,
                 float* dev_grad, float* loss);
/* Train: for each of `steps` batches of `batch` consecutive samples (wrapping around n),
   compute the gradient and apply one Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8). */
int lbm_mlp_train(lbm_mlp* m, const float* dev_x, const float* dev_t, int64_t n,
                  int32_t batch, int64_t steps, float lr);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
   or training loops, harnesses that forbid hipMalloc): the loss and gradient of lbm_mlp_grad
   without a trainer and without any allocation. dev_weights: the float32 parameter blob
   (5577 values, device); dev_x [n][12], dev_t [n][9] as in lbm_mlp_grad, with
   1 <= n <= LBM_MLP_STATIC_MAX_SAMPLES; dev_grad receives 5577 float32 values; dev_loss one
   float32 (device) or NULL. Enqueued on `stream` (hipStream_t, NULL = null stream); no
   synchronisation. The per-64-sample partial gradients go to a fixed array of the library
   (about 5.5 MiB per GPU, held until the process ends) instead of a trainer buffer: calls that
   overlap on one GPU race on it, so serialise them (one stream, or events). Returns LBM_EINVAL
   for n outside the range or NULL buffers, LBM_EDEVICE if a launch fails; the text of neither
   is kept (no context). Results equal lbm_mlp_grad's for the same weights. */
#define LBM_MLP_STATIC_MAX_SAMPLES 16384
int lbm_mlp_grad_static(const float* dev_weights, const float* dev_x, const float* dev_t,
                        int64_t n, float* dev_grad, float* dev_loss, void* stream);

/* ---- measurement ------------------------------------------------------------------------
   Not part of the method: a device-to-device copy of `bytes` bytes (src and dst device
   pointers, 16-byte aligned, not overlapping), enqueued on `stream` with the access pattern of a
   streaming step (every byte read once and written once, 16-byte non-temporal loads and
   stores). Its bandwidth is the practical ceiling the roofline figures are compared with.
   LBM_EINVAL for NULL or misaligned pointers, LBM_EDEVICE if the launch fails. */
int lbm_device_copy(const void* src, void* dst, size_t bytes, void* stream);

/* Text of the last error of ctx, or of the calling thread's last context-free error if ctx
   is NULL. Never NULL; valid until the next call on the same context or thread. */
const char* lbm_last_error(const lbm_ctx* ctx);

/* Release the context and its device memory (not a caller workspace). NULL-safe. */
void lbm_destroy(lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
