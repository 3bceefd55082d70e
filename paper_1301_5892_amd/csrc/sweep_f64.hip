// FP64 sweep kernels of one line length per launch (v-sweeps, and
// x-sweeps on the transposed copy) and their launchers.
#include "kernels.hpp"

namespace vog {

template <typename T, int N, int KIND>
static void launch_sweep(const SweepBatch &b, int max_lines, hipStream_t st) {
    if constexpr (KIND == 3 && !Sweep<T, N>::COMPOSED) {
        // no composed kernel for these lines: two one-step launches
        launch_sweep<T, N, 0>(b, max_lines, st);
        launch_sweep<T, N, 0>(b, max_lines, st);
    } else {
        constexpr int PPB = 256 / Fft<T, N>::TPF;
        const int blocks = (max_lines / 2 + PPB - 1) / PPB;
        hipLaunchKernelGGL((sweep_kernel<T, N, KIND>), dim3(blocks, b.n), dim3(256), 0, st, b);
    }
}

template <typename T, int KIND, int... L>
static SweepFn pick_sweep(int logn, std::integer_sequence<int, L...>) {
    SweepFn fns[] = {&launch_sweep<T, (8 << L), KIND>...};
    return fns[logn - 3];
}

SweepFn sweep_launcher_f64(int n, int kind) {
    const int logn = ilog2(n);
    using Seq = std::make_integer_sequence<int, 10>;
    return kind == 0   ? pick_sweep<double, 0>(logn, Seq{})
           : kind == 1 ? pick_sweep<double, 1>(logn, Seq{})
           : kind == 2 ? pick_sweep<double, 2>(logn, Seq{})
                       : pick_sweep<double, 3>(logn, Seq{});
}

}  // namespace vog
