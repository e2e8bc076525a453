// FP32 production instantiation: packet transport in single precision, FP64
// table totals and energy sums.
#include "transport_kernel.h"

namespace mcrt {
hipError_t launch_transport_f32(const TransportArgs<float, float> &a, int grid, hipStream_t stream)
{
    return launch_transport_impl<float, float>(a, grid, stream);
}
} // namespace mcrt
