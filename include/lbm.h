/* lbm.h: C ABI of the lattice Boltzmann fluid solver (the paper's Methods,
 * "Lattice Boltzmann method"): D3Q19 populations relaxed by BGK towards the
 * second-order equilibrium, a uniform body force through Guo's forcing term
 * (velocity shifted by half the force), and streaming one link per step along
 * periodic axes, or with walls at z = -1/2 and z = nz - 1/2: no-slip walls by
 * halfway bounce-back (the top one optionally moving tangentially), or a
 * no-slip bottom under a free-slip top (specular reflection) -- the bounds of
 * the paper's channel (Results, "Fluid-structure interaction") and of its
 * cilia carpet (Results, "Fluid pumping by magnetic cilia arrays"). Lattice
 * units: dx = dt = 1, c_s^2 = 1/3, viscosity nu = (tau - 1/2) / 3. FP64
 * throughout.
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
 * stream given to lbm_init. rod_lbm_cycles couples a rod context to a lattice
 * (the immersed-boundary method).
 */
#ifndef LBM_H
#define LBM_H
#include <stdint.h>
#include "rod.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef struct lbm_desc {
  int32_t nx, ny, nz;  /* lattice size, each >= 1; nx * ny * nz <= 2^31 - 1 */
  double tau;          /* relaxation time > 1/2 */
  double force[3];     /* uniform body force density (finite) */
  int32_t walls_z;     /* 0: periodic in z; 1: no-slip walls below z = 0 and above nz - 1
                          (halfway bounce-back; a population crossing a wall comes back
                          reversed at the cell it left); 2: a no-slip bottom and a free-slip
                          top (there a population comes back with its z component reversed) */
  double lid_velocity[2]; /* (u_x, u_y) of the top wall, walls_z = 1 only (else both 0): the
                          reflected population loses 6 w_i rho (c_i . u_lid), rho the cell's
                          density (a moving no-slip wall) */
} lbm_desc;

/* Allocate the two population buffers (2 x 19 x cells doubles) and copy the
 * initial populations f0 (device [19][nz][ny][nx]; the caller keeps it). */
int lbm_init(lbm_ctx** out, const lbm_desc* d, const double* f0, void* hip_stream);

/* Advance n >= 0 steps. */
int lbm_step(lbm_ctx* c, int64_t n);

/* Copy the current populations to f (device [19][nz][ny][nx]). */
int lbm_populations(lbm_ctx* c, double* f);

/* Density [nz][ny][nx] and velocity [3][nz][ny][nx] of the current populations
 * (device), the velocity shifted by half the uniform body force (the force
 * field spread by rod_lbm_cycles, which the last collision also saw, is not
 * included). */
int lbm_moments(lbm_ctx* c, double* rho, double* u);

/* Release the context (synchronises). NULL is accepted. */
int lbm_free(lbm_ctx* c);

/* Message of the last error on the calling thread ("" if none). */
const char* lbm_last_error(void);

/* Rods immersed in the lattice (Methods, "Immersed boundary coupling"), for
 * n_cycles >= 0 lattice steps with n_sub >= 1 rod steps each. Particle
 * positions are in lattice units (nodes at integer coordinates); the rod time
 * step must be 1 / n_sub of the lattice step (|dt n_sub - 1| <= 1e-12). The
 * lattice is periodic in x and y; in z it may have walls, and then the stencil
 * nodes beyond a wall take no part (the fluid velocity there counts as zero in
 * the interpolation, and the share of a spread force that would fall there
 * goes to the wall). One cycle:
 *   1. density and velocity u of the lattice (velocity shifted by half the
 *      uniform force);
 *   2. U_p = sum over the 4 x 4 x 4 nodes x around X_p of u(x) delta(x - X_p),
 *      delta the product over the axes of Peskin's four-point function
 *      phi(r) = (3 - 2|r| + sqrt(1 + 4|r| - 4r^2)) / 8 for |r| <= 1,
 *      (5 - 2|r| - sqrt(-7 + 12|r| - 4r^2)) / 8 for 1 < |r| <= 2, 0 beyond
 *      (indices wrap periodically, except across walls);
 *   3. n_sub rod steps; every force evaluation adds the penalty force
 *      F_p = m_p (U_p - v_p) (lattice step 1) with the half-step velocity, and
 *      after each step -F_p / n_sub is spread with the same delta at the
 *      particles' new positions into a force field;
 *   4. one lattice step with the uniform force plus that field.
 * The rod state at entry carries no penalty force. Work runs on the rod
 * context's stream: the lattice's stream is synchronised first, and later work
 * on it waits for the cycles. The coupling buffers (7 doubles per cell, 6 per
 * particle) are allocated on first use and freed with their contexts. Errors:
 * ROD_E_INVALID (arguments, time step), ROD_E_STATE (a tape is being
 * recorded), ROD_E_HIP; the message is rod_last_error()'s. Non-finite states and
 * list overflows are reported by the next rod_sync, as for rod_step. */
int rod_lbm_cycles(rod_ctx* c, lbm_ctx* l, int32_t n_sub, int64_t n_cycles);

#ifdef __cplusplus
}
#endif
#endif
