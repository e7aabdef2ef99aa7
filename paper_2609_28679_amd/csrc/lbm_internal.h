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

Grid make_grid(const Layout& L);

// Reduced storage: float32 moment planes + 16-bit non-equilibrium planes.
struct Reduced {
  float* mom;       // [nm][nodes-with-pitch]: rho, u_x, u_y (+ T for the DDF model)
  uint16_t* neq;    // [nn][nodes-with-pitch]
};

// ---- launchers (return the first HIP error) -----------------------------------------------
// Real = float (kind 0) or double (kind 1).
hipError_t launch_bgk_d2q9(int kind, const void* A, void* B, const Layout& L, const Grid& G,
                           double omega, bool walls, double* partials, hipStream_t s);
hipError_t launch_bgk_d3q27(int kind, const void* A, void* B, const Layout& L, const Grid& G,
                            double omega, bool walls, double* partials, hipStream_t s);
hipError_t launch_init_bgk(int kind, int D, const double* rho, const double* u, void* A,
                           const Layout& L, hipStream_t s);
hipError_t launch_moments_bgk(int kind, int D, const void* A, const Layout& L, double* rho,
                              double* u, hipStream_t s);
// Population plane i of the stored state decoded to float64 f_i (nodes values, no padding).
hipError_t launch_decode_f(int kind, int D, int i, const void* A, const Layout& L, double* f,
                           hipStream_t s);
// Deterministic final pass over per-block partials: out[0] = t, out[1..5] = totals.
hipError_t launch_diag_finalize(const double* partials, int nblocks, double t, double* out,
                                hipStream_t s);
// Totals of float64 node fields (rho [nodes], u [D][nodes], energy density e [nodes] or NULL).
hipError_t launch_field_totals(int D, const double* rho, const double* u, const double* edens,
                               int64_t nodes, bool kinetic, double* partials, int nparts,
                               double* out, hipStream_t s);

}  // namespace lbm
