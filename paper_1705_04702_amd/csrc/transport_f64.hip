// FP64 validation instantiations: the same kernels in double precision, built
// without floating-point contraction so that every operation rounds like the
// FP64 reference.
#include "transport_kernel.h"

namespace mcrt {
hipError_t launch_transport_f64c(const TransportArgs<double, double, 0> &a, int grid, hipStream_t stream)
{
    return launch_transport_impl<double, double, 0>(a, grid, stream);
}
hipError_t launch_transport_f64o(const TransportArgs<double, double, 1> &a, int grid, hipStream_t stream)
{
    return launch_transport_impl<double, double, 1>(a, grid, stream);
}
hipError_t launch_batch_f64(const BatchArgs<double, double> &a, int grid, hipStream_t stream)
{
    return launch_batch_impl<double, double, 0>(a, grid, stream);
}
} // namespace mcrt
