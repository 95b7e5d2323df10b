// step_d3q27.hip -- stream-collide kernel instantiations for one lattice.
#include "step_impl.hpp"

namespace lbm {
template hipError_t launch_step_lattice<2>(int, int, int, bool, int, const StepArgs&, hipStream_t);
}
