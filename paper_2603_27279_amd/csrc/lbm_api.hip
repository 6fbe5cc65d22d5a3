// Lattice Boltzmann fluid solver (Methods, "Lattice Boltzmann method"): one
// fused kernel per step. Each thread owns a cell: it reads the cell's 19
// populations (coalesced, SoA by direction), forms density and velocity (the
// velocity shifted by half the body force), relaxes towards the second-order
// equilibrium (BGK), adds Guo's forcing term and pushes every post-collision
// population to the neighbouring cell along its direction: for each direction
// consecutive threads write consecutive addresses, so the writes stay as
// coalesced as the reads. At a bounce-back wall the population comes back
// reversed at its own cell (less the moving lid's momentum term), at a
// free-slip wall with its z component reversed. 304 bytes move per cell update,
// 19 doubles in and 19 out; the kernel is bound by HBM bandwidth.
#include "rod.h"
#include "lbm.h"
#include "lbm_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

namespace lbmx {

// D3Q19 in the order of lbm.h (the loops over i are unrolled, so every lookup
// is a compile-time constant).
__device__ __forceinline__ constexpr int CX(int i) {
  constexpr int v[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  return v[i];
}
__device__ __forceinline__ constexpr int CY(int i) {
  constexpr int v[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  return v[i];
}
__device__ __forceinline__ constexpr int CZ(int i) {
  constexpr int v[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  return v[i];
}
__device__ __forceinline__ constexpr int OPP(int i) {
  constexpr int v[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  return v[i];
}
// The direction with the z component reversed (specular reflection).
__device__ __forceinline__ constexpr int FLIPZ(int i) {
  constexpr int v[19] = {0, 1, 2, 3, 4, 6, 5, 7, 8, 9, 10, 13, 14, 11, 12, 17, 18, 15, 16};
  return v[i];
}

__device__ __forceinline__ double weight(int i) {
  return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}


__global__ __launch_bounds__(256) void k_lbm(Lattice L, const double* __restrict__ src,
                                             double* __restrict__ dst) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= L.cells) return;
  const int x = (int)(c % L.nx);
  const long r = c / L.nx;
  const int y = (int)(r % L.ny), z = (int)(r / L.ny);
  double f[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) f[i] = src[i * L.cells + c];
  double rho = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    rho += f[i];
    mx += CX(i) * f[i]; my += CY(i) * f[i]; mz += CZ(i) * f[i];
  }
  double gx = L.gx, gy = L.gy, gz = L.gz;  // uniform force plus the spread field
  if (L.gfield) {
    gx += L.gfield[c]; gy += L.gfield[L.cells + c]; gz += L.gfield[2 * L.cells + c];
  }
  const double ux = (mx + 0.5 * gx) / rho, uy = (my + 0.5 * gy) / rho, uz = (mz + 0.5 * gz) / rho;
  const double uu = ux * ux + uy * uy + uz * uz, ug = ux * gx + uy * gy + uz * gz;
  const double omega = 1.0 / L.tau, pre = 1.0 - 0.5 / L.tau;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const double cu = CX(i) * ux + CY(i) * uy + CZ(i) * uz;
    const double cg = CX(i) * gx + CY(i) * gy + CZ(i) * gz;
    const double w = weight(i);
    const double feq = w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    const double fs = f[i] - omega * (f[i] - feq) + pre * w * (3.0 * (cg - ug) + 9.0 * cu * cg);
    int zd = z + CZ(i);
    if (L.walls && (zd < 0 || zd >= L.nz)) {
      if (zd >= L.nz && L.walls == 2) {  // free-slip top: z reversed, at this cell
        dst[FLIPZ(i) * L.cells + c] = fs;
      } else {  // halfway bounce-back, less 6 w rho (c . lid) at a moving top wall
        const double mv = zd >= L.nz ? 6.0 * w * rho * (CX(i) * L.lidx + CY(i) * L.lidy) : 0.0;
        dst[OPP(i) * L.cells + c] = fs - mv;
      }
      continue;
    }
    zd = (zd + L.nz) % L.nz;
    const int xd = (x + CX(i) + L.nx) % L.nx, yd = (y + CY(i) + L.ny) % L.ny;
    dst[i * L.cells + ((long)zd * L.ny + yd) * L.nx + xd] = fs;
  }
}

__global__ __launch_bounds__(256) void k_lbm_moments(Lattice L, const double* __restrict__ f,
                                                     double* rho_o, double* u_o) {
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= L.cells) return;
  double rho = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const double v = f[i * L.cells + c];
    rho += v;
    mx += CX(i) * v; my += CY(i) * v; mz += CZ(i) * v;
  }
  rho_o[c] = rho;
  u_o[c] = (mx + 0.5 * L.gx) / rho;
  u_o[L.cells + c] = (my + 0.5 * L.gy) / rho;
  u_o[2 * L.cells + c] = (mz + 0.5 * L.gz) / rho;
}

// ---------------------------------------------------------------- immersed boundary
// Peskin's four-point delta along one axis.
__device__ __forceinline__ double peskin4(double r) {
  r = fabs(r);
  if (r <= 1.0) return (3.0 - 2.0 * r + sqrt(1.0 + 4.0 * r - 4.0 * r * r)) * 0.125;
  if (r <= 2.0) return (5.0 - 2.0 * r - sqrt(-7.0 + 12.0 * r - 4.0 * r * r)) * 0.125;
  return 0.0;
}

// One node of the 4 x 4 x 4 stencil of position (x, y, z) per lane: lane k of
// the particle's wave takes x offset k & 3, y offset (k >> 2) & 3, z offset
// k >> 4 from floor - 1, so the 64 lanes of a wave touch 64 distinct nodes.
// Returns the node's cell index (wrapped periodically) and its weight
// (phi_z phi_y) phi_x. With walls in z a node beyond them takes no part: its
// weight is 0 (and its index clamped into the lattice).
__device__ __forceinline__ long stencil_node(const Lattice& L, double x, double y, double z, int k,
                                             double& w) {
  const int ox = k & 3, oy = (k >> 2) & 3, oz = k >> 4;
  const int nx = (int)floor(x) - 1 + ox, ny = (int)floor(y) - 1 + oy, nz = (int)floor(z) - 1 + oz;
  w = peskin4((double)nz - z) * peskin4((double)ny - y) * peskin4((double)nx - x);
  const int ix = ((nx % L.nx) + L.nx) % L.nx, iy = ((ny % L.ny) + L.ny) % L.ny;
  int iz;
  if (L.walls) {
    if (nz < 0 || nz >= L.nz) w = 0.0;
    iz = nz < 0 ? 0 : (nz >= L.nz ? L.nz - 1 : nz);
  } else {
    iz = ((nz % L.nz) + L.nz) % L.nz;
  }
  return ((long)iz * L.ny + iy) * L.nx + ix;
}

// Fluid velocity at each particle: U(X) = sum over the 64 stencil nodes of
// u(x) delta(x - X); u [3][cells] (the velocity plane of the moments). One
// wave per particle, the node terms summed across the wave.
__global__ __launch_bounds__(256) void k_ibm_interp(Lattice L, const double* __restrict__ u,
                                                   const double* __restrict__ X, long n,
                                                   double* U) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long p = t >> 6;
  if (p >= n) return;  // whole waves: 64 divides the block size
  const int k = (int)(t & 63);
  double w;
  const long c = stencil_node(L, X[p], X[n + p], X[2 * n + p], k, w);
  double ax = u[c] * w, ay = u[L.cells + c] * w, az = u[2 * L.cells + c] * w;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    ax += __shfl_xor(ax, o);
    ay += __shfl_xor(ay, o);
    az += __shfl_xor(az, o);
  }
  if (k == 0) {
    U[p] = ax; U[n + p] = ay; U[2 * n + p] = az;
  }
}

// Spread -scale F_p of every particle onto the force field g [3][cells]: one
// wave per particle, each lane adding its node's share with a hardware FP64
// atomic (device memory from hipMalloc is coarse-grained, where these are
// exact adds; the sums agree to rounding with any order).
__global__ __launch_bounds__(256) void k_ibm_spread(Lattice L, const double* __restrict__ X,
                                                   const double* __restrict__ F, long n,
                                                   double scale, double* g) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long p = t >> 6;
  if (p >= n) return;
  const int k = (int)(t & 63);
  double w;
  const long c = stencil_node(L, X[p], X[n + p], X[2 * n + p], k, w);
  if (w == 0.0) return;  // outside the support, or beyond a wall
  const double fx = -scale * F[p], fy = -scale * F[n + p], fz = -scale * F[2 * n + p];
  unsafeAtomicAdd(&g[c], fx * w);
  unsafeAtomicAdd(&g[L.cells + c], fy * w);
  unsafeAtomicAdd(&g[2 * L.cells + c], fz * w);
}

__global__ __launch_bounds__(256) void k_fill0(double* a, long n) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) a[k] = 0.0;
}

}  // namespace lbmx

using namespace lbmx;

namespace lbmx {
static unsigned blocks_of(long n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_lbm_step(lbm_ctx* c, const double* gfield, hipStream_t s) {
  Lattice L = c->L;
  L.gfield = gfield;
  hipLaunchKernelGGL(k_lbm, dim3(blocks_of(L.cells)), dim3(256), 0, s, L,
                     (const double*)c->f[c->cur], c->f[1 - c->cur]);
  c->cur = 1 - c->cur;
  return hipGetLastError();
}
hipError_t launch_lbm_moments(const lbm_ctx* c, double* rho, double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_lbm_moments, dim3(blocks_of(c->L.cells)), dim3(256), 0, s, c->L,
                     (const double*)c->f[c->cur], rho, u);
  return hipGetLastError();
}
hipError_t launch_ibm_interp(const lbm_ctx* c, const double* u, const double* X, long n, double* U,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ibm_interp, dim3(blocks_of(64 * n)), dim3(256), 0, s, c->L, u, X, n, U);
  return hipGetLastError();
}
hipError_t launch_ibm_spread(const lbm_ctx* c, const double* X, const double* F, long n,
                             double scale, double* g, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ibm_spread, dim3(blocks_of(64 * n)), dim3(256), 0, s, c->L, X, F, n, scale, g);
  return hipGetLastError();
}
hipError_t launch_fill0(double* a, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill0, dim3(blocks_of(n)), dim3(256), 0, s, a, n);
  return hipGetLastError();
}
}  // namespace lbmx


static thread_local std::string g_lbm_err;

static int lfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_lbm_err = buf;
  return code;
}

#define LHIP(x)                                                                     \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) return lfail(ROD_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

static unsigned lblocks(long cells) { return (unsigned)((cells + 255) / 256); }

extern "C" {

const char* lbm_last_error(void) { return g_lbm_err.c_str(); }

int lbm_init(lbm_ctx** out, const lbm_desc* d, const double* f0, void* hip_stream) {
  if (!out || !d || !f0) return lfail(ROD_E_INVALID, "NULL argument");
  *out = nullptr;
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) return lfail(ROD_E_INVALID, "nx, ny, nz must be >= 1");
  const long cells = (long)d->nx * d->ny * d->nz;
  if (cells > 2147483647L) return lfail(ROD_E_INVALID, "more than 2^31 - 1 cells");
  if (!(d->tau > 0.5) || !std::isfinite(d->tau)) return lfail(ROD_E_INVALID, "tau must be > 1/2");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(d->force[k])) return lfail(ROD_E_INVALID, "force must be finite");
  if (d->walls_z < 0 || d->walls_z > 2) return lfail(ROD_E_INVALID, "walls_z must be 0, 1 or 2");
  if (!std::isfinite(d->lid_velocity[0]) || !std::isfinite(d->lid_velocity[1]))
    return lfail(ROD_E_INVALID, "lid_velocity must be finite");
  if ((d->lid_velocity[0] != 0.0 || d->lid_velocity[1] != 0.0) && d->walls_z != 1)
    return lfail(ROD_E_INVALID, "a lid velocity needs walls_z = 1 (a no-slip top wall)");
  lbm_ctx* c = new lbm_ctx();
  c->L = Lattice{d->nx, d->ny, d->nz, d->walls_z, cells, d->tau, d->force[0], d->force[1],
                 d->force[2], nullptr, d->lid_velocity[0], d->lid_velocity[1]};
  c->s = (hipStream_t)hip_stream;
  const size_t bytes = 19 * sizeof(double) * (size_t)cells;
  hipError_t e = hipMalloc(&c->f[0], bytes);
  if (e == hipSuccess) e = hipMalloc(&c->f[1], bytes);
  if (e == hipSuccess) e = hipMemcpyAsync(c->f[0], f0, bytes, hipMemcpyDeviceToDevice, c->s);
  if (e != hipSuccess) {
    if (c->f[0]) (void)hipFree(c->f[0]);
    if (c->f[1]) (void)hipFree(c->f[1]);
    delete c;
    return lfail(ROD_E_HIP, "allocation or copy failed: %s", hipGetErrorString(e));
  }
  *out = c;
  return ROD_OK;
}

int lbm_step(lbm_ctx* c, int64_t n) {
  if (!c) return lfail(ROD_E_INVALID, "context is NULL");
  if (n < 0) return lfail(ROD_E_INVALID, "n must be >= 0");
  for (int64_t k = 0; k < n; ++k) {
    hipLaunchKernelGGL(k_lbm, dim3(lblocks(c->L.cells)), dim3(256), 0, c->s, c->L,
                       (const double*)c->f[c->cur], c->f[1 - c->cur]);
    LHIP(hipGetLastError());
    c->cur = 1 - c->cur;
  }
  return ROD_OK;
}

int lbm_populations(lbm_ctx* c, double* f) {
  if (!c || !f) return lfail(ROD_E_INVALID, "NULL argument");
  LHIP(hipMemcpyAsync(f, c->f[c->cur], 19 * sizeof(double) * (size_t)c->L.cells,
                      hipMemcpyDeviceToDevice, c->s));
  return ROD_OK;
}

int lbm_moments(lbm_ctx* c, double* rho, double* u) {
  if (!c || !rho || !u) return lfail(ROD_E_INVALID, "NULL argument");
  hipLaunchKernelGGL(k_lbm_moments, dim3(lblocks(c->L.cells)), dim3(256), 0, c->s, c->L,
                     (const double*)c->f[c->cur], rho, u);
  LHIP(hipGetLastError());
  return ROD_OK;
}

int lbm_free(lbm_ctx* c) {
  if (!c) return ROD_OK;
  (void)hipStreamSynchronize(c->s);
  (void)hipDeviceSynchronize();  // a coupled cycle may have used it on another stream
  (void)hipFree(c->f[0]);
  (void)hipFree(c->f[1]);
  if (c->work) (void)hipFree(c->work);
  delete c;
  return ROD_OK;
}

}  // extern "C"
