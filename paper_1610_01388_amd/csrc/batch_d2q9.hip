// batch_d2q9.hip -- batched-sweep kernels, D2Q9.
#include "batch_impl.hpp"

namespace lbm {
template hipError_t launch_batch_lattice<0>(int, int, bool, const BatchArgs&, int, hipStream_t);
}
