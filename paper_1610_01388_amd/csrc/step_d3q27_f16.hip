// step_d3q27_f16.hip -- single-domain stream-collide kernels, D3Q27, FP16 storage
// (one translation unit per lattice and precision keeps the builds parallel).
#include "step_impl.hpp"

namespace lbm {
template hipError_t launch_step_prec<2, PREC_F16>(int, int, bool, int, const StepArgs&, hipStream_t);
}
