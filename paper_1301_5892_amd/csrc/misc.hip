// Transposes, rho, moments, init, fill and the finite-flag gather, and
// the dispatch of the single-length sweep launchers.
#include "kernels.hpp"

#include <mutex>

namespace vog {

SweepFn sweep_launcher_f32(int n, int kind);
SweepFn sweep_launcher_f64(int n, int kind);

SweepFn sweep_launcher(bool fp64, int n, int kind) {
    const int logn = ilog2(n);
    if (n < VOG_MIN_N || n > VOG_MAX_N || (1 << logn) != n || kind < 0 || kind > 3) return nullptr;
    return fp64 ? sweep_launcher_f64(n, kind) : sweep_launcher_f32(n, kind);
}

// ----------------------------------------------------------------- transpose

// TO_V false: f [nx][nv] -> g [nv][nx].  TO_V true: g [nv][nx] -> f [nx][nv]
// and part[jt][i] = FP64 sum of the tile's (up to 64) velocities of column
// i, accumulated in a fixed order.  One 64 x 64 tile per block.
template <typename T, bool TO_V>
__global__ __launch_bounds__(256) void transpose_kernel(const Batch b) {
    __shared__ T tile[kTile][kTile + 1];
    const SimDev &S = *b.s[blockIdx.y];
    const int rows = TO_V ? S.nv : S.nx;
    const int cols = TO_V ? S.nx : S.nv;
    const T *in = (const T *)(TO_V ? S.g : S.f);
    T *out = (T *)(TO_V ? S.f : S.g);
    const int tilesC = (cols + kTile - 1) / kTile;
    const int tilesR = (rows + kTile - 1) / kTile;
    const int tr = blockIdx.x / tilesC, tc = blockIdx.x % tilesC;
    if (tr >= tilesR) return;
    const int r0 = tr * kTile, c0 = tc * kTile;
    const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;
    constexpr int kRows = 256 / kTile;  // tile rows handled per pass of the block
#pragma unroll
    for (int i = 0; i < kTile / kRows; ++i) {
        const int rr = ty + i * kRows;
        const int r = r0 + rr, c = c0 + tx;
        if (r < rows && c < cols) tile[rr][tx] = in[(size_t)r * cols + c];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kTile / kRows; ++i) {
        const int cc = ty + i * kRows;
        const int c = c0 + cc, r = r0 + tx;
        if (r < rows && c < cols) out[(size_t)c * rows + r] = tile[tx][cc];
    }
    if constexpr (TO_V) {
        if (threadIdx.x < kTile) {
            const int c = c0 + threadIdx.x;
            if (c < cols) {
                const int nr = rows - r0 < kTile ? rows - r0 : kTile;
                double acc = 0.0;
                for (int rr = 0; rr < nr; ++rr) acc += (double)tile[rr][threadIdx.x];
                S.part[(size_t)tr * cols + c] = acc;
            }
        }
    }
}

// rho from the partial velocity sums, one block per 16 x-columns.
__global__ __launch_bounds__(256) void rho_reduce_kernel(const SweepBatch b) {
    __shared__ double red[256];
    const SimDev &S = *b.s[blockIdx.y];
    if ((int)blockIdx.x * kRhoCols >= S.nx) return;  // whole block
    rho_columns<256 / kRhoCols, 16>(S, (int)blockIdx.x * kRhoCols, red);
}

void launch_rho_reduce(const SweepBatch &b, int max_nx, hipStream_t st) {
    hipLaunchKernelGGL(rho_reduce_kernel, dim3((max_nx + kRhoCols - 1) / kRhoCols, b.n), dim3(256), 0, st, b);
}

void launch_transpose(bool fp64, bool to_v, const Batch &b, int max_tiles, hipStream_t st) {
    dim3 grid(max_tiles, b.n), block(256);
    if (fp64) {
        if (to_v) hipLaunchKernelGGL((transpose_kernel<double, true>), grid, block, 0, st, b);
        else hipLaunchKernelGGL((transpose_kernel<double, false>), grid, block, 0, st, b);
    } else {
        if (to_v) hipLaunchKernelGGL((transpose_kernel<float, true>), grid, block, 0, st, b);
        else hipLaunchKernelGGL((transpose_kernel<float, false>), grid, block, 0, st, b);
    }
}

// ----------------------------------------------------------------- rho (v layout)

// rho_i = dv sum_j f[i][j] + feq_const, FP64 accumulation in a fixed order:
// one wave per x-column i (4 per block), 16-byte loads, xor-shuffle reduction.
template <typename T>
__global__ __launch_bounds__(256) void rho_v_kernel(const Batch b) {
    const SimDev &S = *b.s[blockIdx.y];
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= S.nx) return;  // wave-uniform; no block barrier follows
    constexpr int VEC = 16 / sizeof(T);
    const T *row = (const T *)S.f + (size_t)i * S.nv;
    double acc = 0.0;
    if (S.nv % (64 * VEC) == 0) {
        for (int j = lane * VEC; j < S.nv; j += 64 * VEC) {
            if constexpr (sizeof(T) == 4) {
                const float4 x = *reinterpret_cast<const float4 *>(row + j);
                acc += ((double)x.x + (double)x.y) + ((double)x.z + (double)x.w);
            } else {
                const double2 x = *reinterpret_cast<const double2 *>(row + j);
                acc += x.x + x.y;
            }
        }
    } else {
        for (int j = lane; j < S.nv; j += 64) acc += (double)row[j];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) S.rho[i] = S.dv * acc + S.feq_const;
}

void launch_rho_v(bool fp64, const Batch &b, int max_nx, hipStream_t st) {
    const int blocks = (max_nx + 3) / 4;
    if (fp64) hipLaunchKernelGGL((rho_v_kernel<double>), dim3(blocks, b.n), dim3(256), 0, st, b);
    else hipLaunchKernelGGL((rho_v_kernel<float>), dim3(blocks, b.n), dim3(256), 0, st, b);
}

// ----------------------------------------------------------------- moments

// mom[i] = (sum_j f_ij^2, sum_j f_ij v_j^2) of the full f (f_eq added back
// for delta f), FP64, fixed order.
template <typename T>
__global__ __launch_bounds__(256) void moments_line_kernel(const Batch b) {
    __shared__ double r1[256], r2[256];
    const SimDev &S = *b.s[blockIdx.y];
    const int i = blockIdx.x;
    if (i >= S.nx) return;
    const T *row = (const T *)S.f + (size_t)i * S.nv;
    double a1 = 0.0, a2 = 0.0;
    for (int j = threadIdx.x; j < S.nv; j += 256) {
        double f = (double)row[j];
        if (S.deltaf) f += S.feq64[j];
        const double vj = S.vmin + j * S.dv;
        a1 += f * f;
        a2 += f * vj * vj;
    }
    r1[threadIdx.x] = a1;
    r2[threadIdx.x] = a2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            r1[threadIdx.x] += r1[threadIdx.x + h];
            r2[threadIdx.x] += r2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        S.mom[2 * i] = r1[0];
        S.mom[2 * i + 1] = r2[0];
    }
}

// L2 = dx dv sum f^2; energy = dx dv sum f v^2 / 2 + dx / 2 sum E^2
// (Section 4.2), written into the step's diagnostics record.
__global__ __launch_bounds__(256) void moments_final_kernel(const Batch b) {
    __shared__ double r1[256], r2[256], r3[256];
    const SimDev &S = *b.s[blockIdx.x];
    double a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int i = threadIdx.x; i < S.nx; i += 256) {
        a1 += S.mom[2 * i];
        a2 += S.mom[2 * i + 1];
        a3 += S.E[i] * S.E[i];
    }
    r1[threadIdx.x] = a1;
    r2[threadIdx.x] = a2;
    r3[threadIdx.x] = a3;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            r1[threadIdx.x] += r1[threadIdx.x + h];
            r2[threadIdx.x] += r2[threadIdx.x + h];
            r3[threadIdx.x] += r3[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        vog_diag &d = S.ring[b.step[blockIdx.x] % kRingCap];
        d.l2 = S.dx * S.dv * r1[0];
        d.energy = 0.5 * S.dx * S.dv * r2[0] + 0.5 * S.dx * r3[0];
    }
}

void launch_moments(bool fp64, const Batch &b, int max_nx, hipStream_t st) {
    if (fp64) hipLaunchKernelGGL((moments_line_kernel<double>), dim3(max_nx, b.n), dim3(256), 0, st, b);
    else hipLaunchKernelGGL((moments_line_kernel<float>), dim3(max_nx, b.n), dim3(256), 0, st, b);
    hipLaunchKernelGGL(moments_final_kernel, dim3(b.n), dim3(256), 0, st, b);
}

// ----------------------------------------------------------------- init / fill

struct InitArgs {
    int nmodes;
    double amp[8], kx[8], ph[8];
};

// f0 = (1 + sum_m amp_m cos(kx_m x_i + ph_m)) f_eq(v_j); delta f stores the
// perturbation part only.
template <typename T>
__global__ __launch_bounds__(256) void init_kernel(const SimDev *sp, const InitArgs a) {
    const SimDev &S = *sp;
    const size_t cells = (size_t)S.nx * S.nv;
    for (size_t idx = blockIdx.x * (size_t)256 + threadIdx.x; idx < cells;
         idx += (size_t)gridDim.x * 256) {
        const int i = (int)(idx / S.nv), j = (int)(idx % S.nv);
        const double x = i * S.dx;
        double p = 0.0;
        for (int m = 0; m < a.nmodes; ++m) p += a.amp[m] * cos(a.kx[m] * x + a.ph[m]);
        const double fe = S.feq64[j];
        ((T *)S.f)[idx] = (T)(S.deltaf ? p * fe : (1.0 + p) * fe);
    }
}

void launch_init(bool fp64, const SimDev *s, int cells, int nmodes, const double *amp,
                 const double *kx, const double *ph, hipStream_t st) {
    InitArgs a{};
    a.nmodes = nmodes;
    for (int m = 0; m < nmodes; ++m) {
        a.amp[m] = amp[m];
        a.kx[m] = kx[m];
        a.ph[m] = ph[m];
    }
    int blocks = (cells + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (fp64) hipLaunchKernelGGL((init_kernel<double>), dim3(blocks), dim3(256), 0, st, s, a);
    else hipLaunchKernelGGL((init_kernel<float>), dim3(blocks), dim3(256), 0, st, s, a);
}

__global__ __launch_bounds__(64) void finite_gather_kernel(const Batch b, int *out) {
    const int k = (int)threadIdx.x;
    if (k >= b.n) return;
    const SimDev &S = *b.s[k];
    const int64_t st = b.step[k];
    int ok = 1;
    if (st > 0 && !S.field_zero) {
        const vog_diag &d = S.ring[st % kRingCap];
        if (d.step == st && !d.finite) ok = 0;
    }
    out[k] = ok;
}

void launch_finite_gather(const Batch &b, int *out, hipStream_t st) {
    hipLaunchKernelGGL(finite_gather_kernel, dim3(1), dim3(64), 0, st, b, out);
}

// Flag buffer of vog_sync_batch_noalloc: a fixed array in the library's own
// device memory (one copy per GPU, held until the process ends) in place of
// an allocation.  Host code never passes the array's name to a kernel: it
// passes the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) int scratch[kNoAllocFlags];

int *noalloc_flags(int device) {
    static std::mutex mu;
    static int *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        addr[device] = (int *)p;
    }
    return addr[device];
}

__global__ __launch_bounds__(256) void fill_kernel(uint32_t *p, size_t nwords) {
    for (size_t k = blockIdx.x * (size_t)256 + threadIdx.x; k < nwords; k += (size_t)gridDim.x * 256)
        p[k] = 0u;
}

void launch_fill(void *p, size_t bytes, hipStream_t st) {
    const size_t nwords = bytes / 4;
    if (nwords == 0) return;
    size_t blocks = (nwords + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t *)p, nwords);
}


}  // namespace vog
