// Lattice Boltzmann internals shared by the solver (lbm_api.hip) and the
// immersed-boundary coupling of the rod runtime (rod_api.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace lbmx {

struct Lattice {
  int nx, ny, nz;
  int walls;             // 0 periodic in z; 1 no-slip walls in z; 2 no-slip bottom, free-slip top
  long cells;
  double tau, gx, gy, gz;
  const double* gfield;  // [3][cells] force density added to the uniform one, or null
  double lidx, lidy;     // velocity of the top wall (walls == 1)
};

}  // namespace lbmx

struct lbm_ctx {
  lbmx::Lattice L;
  double* f[2] = {nullptr, nullptr};
  int cur = 0;
  hipStream_t s = nullptr;
  double* work = nullptr;  // coupling: density, velocity [3] and force field [3] per cell
};

namespace lbmx {
// One step with the uniform force plus gfield (nullable); the moments with the
// uniform force's half shift; interpolation of u [3][cells] at X [3][n] into
// U [3][n]; spreading of -scale F [3][n] at X into g [3][cells]; zero fill.
hipError_t launch_lbm_step(lbm_ctx* c, const double* gfield, hipStream_t s);
hipError_t launch_lbm_moments(const lbm_ctx* c, double* rho, double* u, hipStream_t s);
hipError_t launch_ibm_interp(const lbm_ctx* c, const double* u, const double* X, long n, double* U,
                             hipStream_t s);
hipError_t launch_ibm_spread(const lbm_ctx* c, const double* X, const double* F, long n,
                             double scale, double* g, hipStream_t s);
hipError_t launch_fill0(double* a, long n, hipStream_t s);
}  // namespace lbmx
