// Launches over sims of mixed line lengths (the serving batches): FP32
// v- and x-sweeps and the field solves of x-lines up to 1024 points.
#include "kernels.hpp"

namespace vog {

// FP32 v-sweeps of sims with lines of 64 .. 4096 points in one launch: every
// block runs the body of its sim's line length (each block carries 8192
// values whatever the length).
// KIND 0: one v half-step; KIND 2: two in a row; KIND 3: two composed in
// Fourier space (sweep_body).
constexpr int kMixedSmem3 = [] {
    int m = 0;
    const int s[] = {Sweep<float, 64>::SMEM3,   Sweep<float, 128>::SMEM3, Sweep<float, 256>::SMEM3,
                     Sweep<float, 512>::SMEM3,  Sweep<float, 1024>::SMEM3, Sweep<float, 2048>::SMEM3,
                     Sweep<float, 4096>::SMEM3};
    for (int x : s) m = x > m ? x : m;
    return m;
}();
template <int KIND>
__global__ __launch_bounds__(256, (KIND == 3 ? 2 : 3)) void sweep_v_mixed_kernel(const SweepBatch b,
                                                                               const SweepMap m) {
    // the largest of 64 .. 4096
    __shared__ float smem[KIND == 3 ? kMixedSmem3 : Sweep<float, 64>::SMEM];
    const int bid = (int)blockIdx.x;
    const int k = mixed_sim(b, m, bid);
    const int blk = bid - m.first[k];
    switch (m.lgn[k]) {
    case 6: sweep_body<float, 64, KIND, false>(b, k, blk, smem); break;
    case 7: sweep_body<float, 128, KIND, false>(b, k, blk, smem); break;
    case 8: sweep_body<float, 256, KIND, false>(b, k, blk, smem); break;
    case 9: sweep_body<float, 512, KIND, false>(b, k, blk, smem); break;
    case 10: sweep_body<float, 1024, KIND, false>(b, k, blk, smem); break;
    case 11: sweep_body<float, 2048, KIND, false>(b, k, blk, smem); break;
    case 12: sweep_body<float, 4096, KIND, false>(b, k, blk, smem); break;
    default: break;
    }
}

// FP32 x-sweeps of sims with x-lines of 64 .. 1024 points in one launch
// (256-thread blocks for all of them).  Each sim's first block is a multiple
// of 8, so the XCD-aware tile order holds.
__global__ __launch_bounds__(256, 3) void xsweep_mixed_kernel(const SweepBatch b, const SweepMap m) {
    __shared__ float smem[Fused<float, 64>::SMEM];  // the largest of 64 .. 1024
    const int bid = (int)blockIdx.x;
    const int k = mixed_sim(b, m, bid);
    const int hb = bid - m.first[k];
    switch (m.lgn[k]) {
    case 6: xsweep_body<float, 64>(b, k, hb, smem); break;
    case 7: xsweep_body<float, 128>(b, k, hb, smem); break;
    case 8: xsweep_body<float, 256>(b, k, hb, smem); break;
    case 9: xsweep_body<float, 512>(b, k, hb, smem); break;
    case 10: xsweep_body<float, 1024>(b, k, hb, smem); break;
    default: break;
    }
}

static_assert(Fused<float, 64>::TB == 256 && Fused<float, 1024>::TB == 256 &&
                  Fused<float, 64>::WAVES == 3 && Fused<float, 1024>::WAVES == 3,
              "mixed x-sweep: 256-thread blocks at 3 waves for 64 .. 1024 points");
static_assert(Fused<float, 64>::SMEM >= Fused<float, 128>::SMEM &&
                  Fused<float, 64>::SMEM >= Fused<float, 256>::SMEM &&
                  Fused<float, 64>::SMEM >= Fused<float, 512>::SMEM &&
                  Fused<float, 64>::SMEM >= Fused<float, 1024>::SMEM,
              "mixed x-sweep LDS");
static_assert(Sweep<float, 64>::SMEM >= Sweep<float, 128>::SMEM &&
                  Sweep<float, 64>::SMEM >= Sweep<float, 256>::SMEM &&
                  Sweep<float, 64>::SMEM >= Sweep<float, 512>::SMEM &&
                  Sweep<float, 64>::SMEM >= Sweep<float, 1024>::SMEM &&
                  Sweep<float, 64>::SMEM >= Sweep<float, 2048>::SMEM &&
                  Sweep<float, 64>::SMEM >= Sweep<float, 4096>::SMEM,
              "mixed v-sweep LDS");

bool sweep_mixed_ok(bool vsweep, int n) {
    const int logn = ilog2(n);
    return (1 << logn) == n && n >= 64 && n <= (vsweep ? 4096 : 1024);
}

int sweep_blocks_mixed(bool vsweep, int n, int lines) {
    if (!sweep_mixed_ok(vsweep, n)) return 0;
    if (vsweep) {
        const int ppb = 256 / (n / fft_regs(n));
        return (lines / 2 + ppb - 1) / ppb;
    }
    const int tiles = lines / (2 * (256 / (n / fft_regs(n))));
    return (tiles + 7) / 8 * 8;
}

void launch_sweep_mixed(int kind, const SweepBatch &b, const SweepMap &m, hipStream_t st) {
    const int blocks = m.first[b.n];
    if (kind == 0) hipLaunchKernelGGL(sweep_v_mixed_kernel<0>, dim3(blocks), dim3(256), 0, st, b, m);
    else if (kind == 2) hipLaunchKernelGGL(sweep_v_mixed_kernel<2>, dim3(blocks), dim3(256), 0, st, b, m);
    else if (kind == 3) hipLaunchKernelGGL(sweep_v_mixed_kernel<3>, dim3(blocks), dim3(256), 0, st, b, m);
    else hipLaunchKernelGGL(xsweep_mixed_kernel, dim3(blocks), dim3(256), 0, st, b, m);
}

// Field solves of sims with 8 .. 1024 points in x, any mix of lengths, in
// one launch: one wave per sim, whose first TPF lanes run the body of the
// sim's length (a one-wave block needs no barrier between its lanes).
__global__ __launch_bounds__(64) void field_mixed_kernel(const Batch b, const BlockMap m) {
    __shared__ double smem[Field<1024>::SMEM];
    const int k = (int)blockIdx.x;  // one block per sim
    const int t = (int)threadIdx.x;
    switch (m.lgn[k]) {
    case 3: if (t < Field<8>::TPF) field_body<8>(b, k, smem); break;
    case 4: if (t < Field<16>::TPF) field_body<16>(b, k, smem); break;
    case 5: if (t < Field<32>::TPF) field_body<32>(b, k, smem); break;
    case 6: if (t < Field<64>::TPF) field_body<64>(b, k, smem); break;
    case 7: if (t < Field<128>::TPF) field_body<128>(b, k, smem); break;
    case 8: if (t < Field<256>::TPF) field_body<256>(b, k, smem); break;
    case 9: if (t < Field<512>::TPF) field_body<512>(b, k, smem); break;
    case 10: field_body<1024>(b, k, smem); break;
    default: break;
    }
}

static_assert(Field<1024>::TPF == 64 && Field<1024>::SMEM >= Field<512>::SMEM,
              "mixed field solve: one wave, LDS of the 1024-point body");

bool field_mixed_ok(int nx) { return nx >= 8 && nx <= 1024 && (nx & (nx - 1)) == 0; }

void launch_field_mixed(const Batch &b, const BlockMap &m, hipStream_t st) {
    hipLaunchKernelGGL(field_mixed_kernel, dim3(b.n), dim3(64), 0, st, b, m);
}

}  // namespace vog
