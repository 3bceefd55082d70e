// x-sweeps on the v-fastest layout (tiles of whole x-lines), one line
// length per launch, and their launchers.
#include "kernels.hpp"

namespace vog {

template <typename T, int N>
static void launch_xsweep_fused(const SweepBatch &b, int max_lines, hipStream_t st) {
    using C = Fused<T, N>;
    const int blocks = max_lines / C::B;
    hipLaunchKernelGGL((xsweep_fused_kernel<T, N>), dim3(blocks, b.n), dim3(C::TB), 0, st, b);
}

template <typename T, int... L>
static SweepFn pick_fused(int logn, std::integer_sequence<int, L...>) {
    SweepFn fns[] = {&launch_xsweep_fused<T, (64 << L)>...};
    return fns[logn - 6];
}

// Lines per tile of the x-sweep on the v-fastest layout for x-lines of nx
// points (64 .. 4096), 0 where it does not apply.
int fused_lines_per_block(bool fp64, int nx) {
    const int logn = ilog2(nx);
    if (nx < 64 || nx > VOG_MAX_N || (1 << logn) != nx) return 0;
    constexpr int tf[7] = {Fused<float, 64>::B, Fused<float, 128>::B, Fused<float, 256>::B,
                           Fused<float, 512>::B, Fused<float, 1024>::B, Fused<float, 2048>::B,
                           Fused<float, 4096>::B};
    constexpr int td[7] = {Fused<double, 64>::B, Fused<double, 128>::B, Fused<double, 256>::B,
                           Fused<double, 512>::B, Fused<double, 1024>::B, Fused<double, 2048>::B,
                           Fused<double, 4096>::B};
    return fp64 ? td[logn - 6] : tf[logn - 6];
}

SweepFn fused_xsweep_launcher(bool fp64, int nx) {
    if (fused_lines_per_block(fp64, nx) == 0) return nullptr;
    using Seq = std::make_integer_sequence<int, 7>;
    return fp64 ? pick_fused<double>(ilog2(nx), Seq{}) : pick_fused<float>(ilog2(nx), Seq{});
}

}  // namespace vog
