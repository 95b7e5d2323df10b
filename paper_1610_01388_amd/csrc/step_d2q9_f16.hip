// step_d2q9_f16.hip -- single-domain stream-collide kernels, D2Q9, FP16 storage
// (one translation unit per lattice and precision keeps the builds parallel).
#include "step_impl.hpp"

namespace lbm {
template hipError_t launch_step_prec<0, PREC_F16>(int, int, bool, int, const StepArgs&, hipStream_t);
}
