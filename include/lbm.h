/* lbm.h: C ABI of the lattice Boltzmann fluid solver (the paper's Methods,
 * "Lattice Boltzmann method"): D3Q19 populations relaxed by BGK towards the
 * second-order equilibrium, a uniform body force through Guo's forcing term
 * (velocity shifted by half the force), and streaming one link per step along
 * periodic axes, or with halfway bounce-back walls at z = -1/2 and
 * z = nz - 1/2. Lattice units: dx = dt = 1, c_s^2 = 1/3, viscosity
 * nu = (tau - 1/2) / 3. FP64 throughout.
 *
 * Velocity set, in this order: rest; +x, -x, +y, -y, +z, -z;
 * (+x+y), (-x-y), (+x-y), (-x+y), (+x+z), (-x-z), (+x-z), (-x+z),
 * (+y+z), (-y-z), (+y-z), (-y+z); weights 1/3, 1/18 (faces), 1/36 (edges).
 *
 * Populations are device arrays [19][nz][ny][nx] (x fastest), SoA by
 * direction. One step: for every cell, density and velocity from its
 * populations, collision, then each post-collision population moves to the
 * neighbouring cell along its direction (or comes back reversed at a wall).
 * The populations the library holds are those after streaming.
 *
 * Every call returns ROD_OK (0) or a negative ROD_E_* code (rod.h) and sets
 * the message that lbm_last_error() returns. All work is enqueued on the
 * stream given to lbm_init. The immersed-boundary coupling of rods to the
 * fluid is not part of this interface.
 */
#ifndef LBM_H
#define LBM_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef struct lbm_desc {
  int32_t nx, ny, nz;  /* lattice size, each >= 1; nx * ny * nz <= 2^31 - 1 */
  double tau;          /* relaxation time > 1/2 */
  double force[3];     /* uniform body force density (finite) */
  int32_t walls_z;     /* 0: periodic in z; 1: halfway bounce-back walls below z = 0 and above nz - 1 */
} lbm_desc;

/* Allocate the two population buffers (2 x 19 x cells doubles) and copy the
 * initial populations f0 (device [19][nz][ny][nx]; the caller keeps it). */
int lbm_init(lbm_ctx** out, const lbm_desc* d, const double* f0, void* hip_stream);

/* Advance n >= 0 steps. */
int lbm_step(lbm_ctx* c, int64_t n);

/* Copy the current populations to f (device [19][nz][ny][nx]). */
int lbm_populations(lbm_ctx* c, double* f);

/* Density [nz][ny][nx] and velocity [3][nz][ny][nx] of the current populations
 * (device), the velocity shifted by half the body force as in the collision. */
int lbm_moments(lbm_ctx* c, double* rho, double* u);

/* Release the context (synchronises). NULL is accepted. */
int lbm_free(lbm_ctx* c);

/* Message of the last error on the calling thread ("" if none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
