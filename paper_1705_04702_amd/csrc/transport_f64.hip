// FP64 validation instantiation: the same kernel in double precision, built
// without floating-point contraction so that every operation rounds like the
// FP64 reference.
#include "transport_kernel.h"

namespace mcrt {
hipError_t launch_transport_f64(const TransportArgs<double, double> &a, int grid, hipStream_t stream)
{
    return launch_transport_impl<double, double>(a, grid, stream);
}
} // namespace mcrt
