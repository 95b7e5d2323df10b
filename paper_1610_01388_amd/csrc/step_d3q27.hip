// step_d3q27.hip -- stream-collide kernel instantiations (single domain and
// batched) for one lattice.
#include "batch_impl.hpp"

namespace lbm {
template hipError_t launch_step_lattice<2>(int, int, int, bool, int, const StepArgs&, hipStream_t);
template hipError_t launch_batch_lattice<2>(int, int, bool, const BatchArgs&, int, hipStream_t);
}
