// step_d3q19_f16.hip -- single-domain stream-collide kernels, D3Q19, FP16 storage
// (one translation unit per lattice and precision keeps the builds parallel).
#include "step_impl.hpp"

namespace lbm {
template hipError_t launch_step_prec<1, PREC_F16>(int, int, bool, int, const StepArgs&, hipStream_t);
}
