// Tape and reverse pass (checkpoint-and-recompute adjoint of the time step).
#pragma once
#include "rod.h"
#include "rod_internal.h"
#include <cstdint>
#include <vector>

int rodmx_fail(int code, const char* msg);

namespace rodmx {

struct Tape {
  int every = 0, capacity = 0;
  bool active = false;
  int64_t start_step = 0;
  double* ckpt = nullptr;  // checkpoints of the full state
  int n_ckpt = 0;
};

int tape_init(Tape& t, const Dev& d, int every, int capacity, std::vector<void*>& allocs);
int tape_start(Tape& t, const Dev& d, hipStream_t s, int64_t step);
int tape_before_step(Tape& t, const Dev& d, hipStream_t s, int64_t step);
int adjoint_run(Tape& t, const Dev& d, int precision, const DipWork* work, int nwork,
                hipStream_t s, int64_t end_step, const rod_cotangent* gy, rod_gradients* gx);

}  // namespace rodmx
