// batch_d3q27.hip -- batched-sweep kernels, D3Q27.
#include "batch_impl.hpp"

namespace lbm {
template hipError_t launch_batch_lattice<2>(int, int, bool, const BatchArgs&, int, hipStream_t);
}
