// Field solves of x-lines of 2048 and 4096 points, one block per sim.
#include "kernels.hpp"

namespace vog {

template <int N>
static void launch_field(const Batch &b, int, hipStream_t st) {
    hipLaunchKernelGGL((field_kernel<N>), dim3(b.n), dim3(Fft<double, N>::TPF), 0, st, b);
}

// x-lines of 2048 and 4096 points (shorter ones go through field_mixed_kernel).
LaunchFn field_launcher(int nx) {
    if (nx == 2048) return &launch_field<2048>;
    if (nx == 4096) return &launch_field<4096>;
    return nullptr;
}

}  // namespace vog
