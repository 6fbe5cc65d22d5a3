// Reverse pass of the time step (checkpoint-and-recompute).
#include "rod_adjoint.h"

namespace rodmx {

int tape_init(Tape& t, const Dev&, int every, int capacity, std::vector<void*>&) {
  t.every = every;
  t.capacity = capacity;
  return ROD_OK;
}
int tape_start(Tape& t, const Dev&, hipStream_t, int64_t step) {
  t.active = true;
  t.start_step = step;
  return ROD_OK;
}
int tape_before_step(Tape&, const Dev&, hipStream_t, int64_t) { return ROD_OK; }
int adjoint_run(Tape&, const Dev&, int, const DipWork*, int, hipStream_t, int64_t,
                const rod_cotangent*, rod_gradients*) {
  return rodmx_fail(ROD_E_NOTAPE, "reverse pass not available in this build");
}

}  // namespace rodmx
