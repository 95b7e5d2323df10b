// step_d3q19.hip -- stream-collide kernel instantiations (single domain and
// batched) for one lattice.
#include "batch_impl.hpp"

namespace lbm {
template hipError_t launch_step_lattice<1>(int, int, int, bool, int, const StepArgs&, hipStream_t);
template hipError_t launch_batch_lattice<1>(int, int, bool, const BatchArgs&, int, hipStream_t);
}
