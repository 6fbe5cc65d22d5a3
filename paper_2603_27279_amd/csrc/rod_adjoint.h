// Tape and reverse pass (checkpoint-and-recompute adjoint of the time step).
#pragma once
#include "rod.h"
#include "rod_internal.h"
#include <cstdint>
#include <vector>

int rodmx_fail(int code, const char* msg);

namespace rodmx {

// Layout of one recorded state: x(3N) v(3N) q(4N) w(3N) F(3N) T(3N), then the
// dipole field of that level (3N) in the segment buffers.
constexpr int STATE_PLANES = 19;
constexpr int SEG_PLANES = 22;

// Device work arrays of the reverse pass (SoA planes of length N).
struct Adj {
  double *cx, *cv, *cq, *cw, *cF, *cT;  // cotangent of the state (STATE_PLANES x N, contiguous)
  double *Fe, *Te;      // cotangents of the level's force and torque that reach the kicks
  double *h;            // cotangent of the dipole field, T-bar x m
  double *mloc, *xloc;  // local contributions to m-bar and x-bar (torques, Zeeman)
  double *vbar, *wbar;  // cotangents of the velocities used by damping (half-step)
  double *wh;           // recomputed half-step angular velocity
  double *fieldc;       // [12][N] per-particle contributions to the field gradient
  double *bvjp;         // [11][N] per bond: r-bar (3), q1-bar (4), q2-bar (4)
  double *mbbar;        // [3N] gradient w.r.t. the body dipoles
  double *fieldbar;     // [L][M][12] gradient w.r.t. the field table
  double *scratch;      // [6N] outputs of evaluations whose values are not needed
  long long* level;     // [3] time-level counters of the recompute view
  long long* lbase;     // [1] first level of the segment being reversed
  long long* levels;    // [every + 1][3]: counters of the reverse view of level lbase + k
};

struct Tape {
  int every = 0, capacity = 0;
  bool active = false;
  int64_t start_step = 0;
  double* ckpt = nullptr;  // [capacity / every + 1][STATE_PLANES N]
  double* seg = nullptr;   // [every + 1][SEG_PLANES N]
  Adj a{};
  // graphs of one full segment: recompute and reverse (captured on first use)
  hipGraphExec_t g_recompute = nullptr, g_reverse = nullptr;
};

int tape_init(Tape& t, const Dev& d, int every, int capacity, std::vector<void*>& allocs);
int tape_start(Tape& t, const Dev& d, hipStream_t s, int64_t step);
int tape_before_step(Tape& t, const Dev& d, hipStream_t s, int64_t step);
int adjoint_run(Tape& t, const Dev& d, int precision, const DipWork* work, int nwork,
                hipStream_t s, int64_t end_step, const rod_cotangent* gy, rod_gradients* gx);
void tape_release(Tape& t);

}  // namespace rodmx
