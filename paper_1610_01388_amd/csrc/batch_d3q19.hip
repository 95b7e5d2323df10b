// batch_d3q19.hip -- batched-sweep kernels, D3Q19.
#include "batch_impl.hpp"

namespace lbm {
template hipError_t launch_batch_lattice<1>(int, int, bool, const BatchArgs&, int, hipStream_t);
}
