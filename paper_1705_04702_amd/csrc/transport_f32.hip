// FP32 production instantiations: packet transport in single precision, FP64
// table totals and energy sums; one kernel per grid type.
#include "transport_kernel.h"

namespace mcrt {
hipError_t launch_transport_f32c(const TransportArgs<float, float, 0> &a, int grid, hipStream_t stream)
{
    return launch_transport_impl<float, float, 0>(a, grid, stream);
}
hipError_t launch_transport_f32o(const TransportArgs<float, float, 1> &a, int grid, hipStream_t stream)
{
    return launch_transport_impl<float, float, 1>(a, grid, stream);
}
hipError_t launch_batch_f32(const BatchArgs<float, float> &a, int grid, hipStream_t stream, int slots)
{
    if (slots == 8) return launch_batch_impl<float, float, 8>(a, grid, stream);
    return launch_batch_impl<float, float, 16>(a, grid, stream);
}
} // namespace mcrt
