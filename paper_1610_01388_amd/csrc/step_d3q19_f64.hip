// step_d3q19_f64.hip -- single-domain stream-collide kernels, D3Q19, FP64 storage
// (one translation unit per lattice and precision keeps the builds parallel).
#include "step_impl.hpp"

namespace lbm {
template hipError_t launch_step_prec<1, PREC_F64>(int, int, bool, int, const StepArgs&, hipStream_t);
}
