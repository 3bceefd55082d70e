#pragma once
// Device code of the split step (gfx950, wave64), shared by the kernel
// translation units sweep_f32.hip, sweep_f64.hip, xsweep.hip, mixed.hip,
// field.hip and misc.hip (which instantiate the kernels and their launchers).
//
//  sweep_kernel     one constant advection (Section 1.2) for a batch of lines:
//                   forward FFT of two real lines packed as one complex line,
//                   multiply by the diagonal of the circulant in Fourier space
//                   (Lagrange or B-spline symbol), inverse FFT, integer part of
//                   the shift applied as an exact cyclic index offset on the
//                   store, delta-f source term (Section 3.1) on v-sweeps;
//                   between two steps, the two v half-steps with one field
//                   in one launch (transformed in turn, or composed in
//                   Fourier space with one inverse transform).
//  xsweep_fused_kernel
//                   the x-advection on the v-fastest layout, tiles of whole
//                   x-lines loaded straight into registers.
//  sweep_v_mixed_kernel, xsweep_mixed_kernel, field_mixed_kernel
//                   one launch over sims of different line lengths (batches of
//                   the serving loop): each block finds its sim and runs the
//                   body compiled for that sim's length.
//  transpose_kernel tiled LDS transpose between the v-fastest and x-fastest
//                   layouts for grids the tiled x-sweep does not cover; the
//                   x->v direction also emits FP64 partial sums of f over 64
//                   velocities for rho = int f dv.
//  field_kernel     FFT (or trapezoidal) Poisson solve in FP64 (Section 3.2),
//                   E and E - E_app, and the per-step diagnostics record
//                   (x-lines of 2048 and 4096 points; shorter ones go through
//                   field_mixed_kernel).
//  rho_v_kernel     rho = int f dv from the v-fastest layout; moments
//                   kernels, init and fill helpers.

#include "addr.hpp"
#include "fft.hpp"
#include "vog_internal.hpp"

#include <math.h>

namespace vog {
// ----------------------------------------------------------------- helpers

// Lagrange 2d+1 coefficient of node q for the fractional shift s in [0, 1)
// (Section 1.2): prod_{k != q} (s - k) / (q - k), nodes k = -d .. d+1.
__device__ __forceinline__ double lagrange_weight(int d, int q, double s) {
    if (q < -d || q > d + 1) return 0.0;
    double num = 1.0, den = 1.0;
    for (int k = -d; k <= d + 1; ++k) {
        if (k == q) continue;
        num *= s - (double)k;
        den *= (double)(q - k);
    }
    return num / den;
}

// B-spline coefficient of node q for the fractional shift s in [0, 1)
// (Section 1.2, degree k = 2d+1): B^k(d + 1 - q + s), B^k the uniform
// B-spline of degree k on [0, k+1).  The values B^p(s + j), j = 0..p, are
// raised one degree at a time with B^p(x) = x/p B^{p-1}(x) +
// (p+1-x)/p B^{p-1}(x-1); the loops are unrolled to the largest degree so
// that the table stays in registers.  Not inlined: it runs once per line
// pair, and as a call its registers do not add to those of the transform.
__device__ __attribute__((noinline)) double bspline_weight(int d, int q, double s) {
    if (q < -d || q > d + 1) return 0.0;
    const int k = 2 * d + 1;
    double b[kTaps];
    static_for<0, kTaps>([&](auto jc) { b[decltype(jc)::value] = 0.0; });
    b[0] = 1.0;
    static_for<1, kTaps>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        if (p <= k) {
            constexpr double ip = 1.0 / (double)p;
            static_for<0, p + 1>([&](auto jc) {
                constexpr int j = p - decltype(jc)::value;  // descending: b[j-1] still of degree p-1
                const double x = s + (double)j;
                double v = x * ip * b[j];
                if constexpr (j > 0) v = fma((double)(p + 1) * ip - x * ip, b[j - 1], v);
                b[j] = v;
            });
        }
    });
    const int jq = d + 1 - q;
    double r = 0.0;
    static_for<0, kTaps>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (j == jq) r = b[j];
    });
    return r;
}

// beta = b + s with b integer and s in [0, 1).  A non-finite or absurdly
// large beta (a diverged field) gives b = 0 and s = NaN, so the line becomes
// NaN and the failure shows in the field's finite flag.
__device__ __forceinline__ void split_shift(double beta, long long &b, double &s) {
    if (!(fabs(beta) < 1e15)) {
        b = 0;
        s = __builtin_nan("");
        return;
    }
    double fb = floor(beta);
    double r = beta - fb;
    if (r >= 1.0) {
        r = 0.0;
        fb += 1.0;
    }
    b = (long long)fb;
    s = r;
}

template <typename T>
__device__ __forceinline__ T expm1_t(T x);
template <>
__device__ __forceinline__ float expm1_t<float>(float x) { return expm1f(x); }
template <>
__device__ __forceinline__ double expm1_t<double>(double x) { return expm1(x); }

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) { return __builtin_fma(a, b, c); }

// Device pointers known to address global memory: accesses through them
// compile to global_* instructions (a 32-bit offset from a base, LDS
// counters untouched) instead of flat ones.
template <typename T>
using gmem = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ gmem<T> *as_global(T *p) { return (gmem<T> *)p; }
template <typename T>
__device__ __forceinline__ const gmem<T> *as_global(const T *p) { return (const gmem<T> *)p; }
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// acc + a b, complex, with four fused multiply-adds.
template <typename T>
__device__ __forceinline__ cx<T> cmac(cx<T> acc, cx<T> a, cx<T> b) {
    return {fma_t<T>(a.re, b.re, fma_t<T>(-a.im, b.im, acc.re)), fma_t<T>(a.re, b.im, fma_t<T>(a.im, b.re, acc.im))};
}

// Raw buffer access: a descriptor with the base address in scalar registers
// and 32-bit byte offsets per lane (voff) and per instruction (soff), so an
// access needs no 64-bit address arithmetic.  Accesses at or past `bytes`
// read 0 and drop the store.  Word 3 of the descriptor selects the 32-bit
// data format of the gfx9 family.
constexpr int kBufWord3 = 0x00020000;

// base and bytes must be the same in every lane of the wave (they are taken
// from the first active lane, so that the descriptor lives in scalar
// registers and the compiler emits no per-lane loop around the accesses).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, unsigned bytes) {
    const uint64_t a = (uint64_t)base;
    const uint64_t u = addr_join(__builtin_amdgcn_readfirstlane(addr_lo(a)),
                                 __builtin_amdgcn_readfirstlane(addr_hi(a)));
    return __builtin_amdgcn_make_buffer_rsrc((void *)u, 0, (int)__builtin_amdgcn_readfirstlane(bytes),
                                             kBufWord3);
}

// A value the same in every lane, moved to scalar registers.
__device__ __forceinline__ double uniform_d(double x) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    return __builtin_bit_cast(double, addr_join(__builtin_amdgcn_readfirstlane(addr_lo(u)),
                                                __builtin_amdgcn_readfirstlane(addr_hi(u))));
}
__device__ __forceinline__ long long uniform_ll(long long x) {
    return (long long)__builtin_bit_cast(uint64_t, uniform_d(__builtin_bit_cast(double, x)));
}

// The value of lane (lane ^ X) of the wave; X = 1, 2 by a DPP quad permute
// of each 32-bit half, larger X through ds_bpermute.  All lanes active.
template <int X>
__device__ __forceinline__ double xor_lane(double x) {
    if constexpr (X == 1 || X == 2) {
        constexpr int ctrl = X == 1 ? 0xB1 : 0x4E;  // quad_perm [1,0,3,2], [2,3,0,1]
        const uint64_t u = __builtin_bit_cast(uint64_t, x);
        return __builtin_bit_cast(double, addr_join(__builtin_amdgcn_update_dpp(0, addr_lo(u), ctrl, 0xF, 0xF, false),
                                                    __builtin_amdgcn_update_dpp(0, addr_hi(u), ctrl, 0xF, 0xF, false)));
    } else {
        return __shfl_xor(x, X, 64);
    }
}

template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <typename T>
__device__ __forceinline__ void buf_store(T x, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, voff, soff, 0);
    } else {
        using U = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, x), r, voff, soff, 0);
    }
}

}  // namespace vog

#include "pair4096.hpp"  // uses fma_t, kTaps

namespace vog {
// ----------------------------------------------------------------- sweep

// delta-f source of one line along the thread's output positions
// pos_k = (p0 + k TPF) mod N, k = 0..R-1 (Section 3.1):
//   f_eq(v - tau E) - f_eq(v) = sum_g f_g(v) expm1(A_g v + C_g),
//   A_g = tau E / sigma_g^2, C_g = -A_g c_g - (tau E)^2 / (2 sigma_g^2).
// The positions increase by TPF and wrap around the periodic velocity grid
// at most once, at k = kw.  expm1 is evaluated exactly at k = 0 and at k = kw;
// in between it follows the exact identity
//   expm1(y + d) = expm1(y) + expm1(d) (1 + expm1(y)),  d = A_g TPF dv.
template <typename T, int N, int R, int TPF>
__device__ __forceinline__ void deltaf_source(const SimDev &S, double tauE, int p0,
                                              const unsigned (&pos)[R], T (&src)[R]) {
    static_for<0, R>([&](auto kc) { src[decltype(kc)::value] = (T)0; });
    // table rows f_g(v_j), N values each; pos[k] = byte offset of pos_k in a row
    const __amdgpu_buffer_rsrc_t fg = buf_rsrc(S.feq_g, (unsigned)(S.n_feq * N * sizeof(T)));
    const T vmin = (T)S.vmin, dv = (T)S.dv;
    const int kw = (N - p0 + TPF - 1) / TPF;  // first wrapped k (R when none)
    const int pw = p0 + kw * TPF - N;         // its position
    for (int g = 0; g < S.n_feq; ++g) {
        const double is2 = S.feq_inv_s2[g];
        const double A64 = tauE * is2;
        const T A = (T)A64;
        const T C = (T)(-A64 * S.feq_c[g] - 0.5 * tauE * tauE * is2);
        const T rm1 = expm1_t<T>((T)(A64 * (double)TPF * S.dv));
        const unsigned row = (unsigned)(g * N * sizeof(T));
        const T e0 = expm1_t<T>(fma_t<T>(A, vmin + (T)p0 * dv, C));
        const T ew = expm1_t<T>(fma_t<T>(A, vmin + (T)(kw < R ? pw : 0) * dv, C));
        T e = e0;
        static_for<0, R>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            if constexpr (k > 0) {
                const T er = e + fma_t<T>(rm1, e, rm1);
                e = k == kw ? ew : er;
            }
            src[k] = fma_t<T>(buf_load<T>(fg, pos[k], row), e, src[k]);
        });
    }
}

// Emits a transformed line pair: out(k) (k a compile-time index) is the
// result at unshifted position t + TPF k, lines A (real part) and B
// (imaginary part).  Unshifted index j goes to line position (j - b) mod N;
// sinkA(pos, x) and sinkB(pos, x) receive each value x with the byte offset
// pos of its position in the line.  VSWEEP: adds the delta-f source
// (Section 3.1) with tau E of each line.  CACHE 1: also keeps line A's source
// values in srcA[k TPF + t]; CACHE 2: takes them from there instead of
// computing them (the same positions, tau and E).
template <typename T, int N, int R, int TPF, bool VSWEEP, int CACHE = 0, typename Out, typename SinkA,
          typename SinkB>
__device__ __forceinline__ void emit_pair(const SimDev &S, double tauEA, double tauEB, long long bA,
                                          long long bB, int t, Out &&out, SinkA &&sinkA, SinkB &&sinkB,
                                          T *srcA = nullptr) {
    constexpr unsigned LB = N * sizeof(T);  // bytes per line
    const int p0A = (t - (int)(bA & (N - 1))) & (N - 1);
    const int p0B = (t - (int)(bB & (N - 1))) & (N - 1);
    auto positions = [&](int p0, unsigned (&pos)[R]) {
        const unsigned p = (unsigned)p0 * sizeof(T);
        static_for<0, R>([&](auto kc) {
            constexpr unsigned k = decltype(kc)::value;
            pos[k] = (p + k * TPF * sizeof(T)) & (LB - 1);
        });
    };
    unsigned pos[R];
    if constexpr (VSWEEP) {
        if (S.deltaf) {
            T src[R];
            positions(p0A, pos);
            if constexpr (CACHE == 2) {
                static_for<0, R>([&](auto kc) { src[decltype(kc)::value] = srcA[decltype(kc)::value * TPF + t]; });
            } else {
                deltaf_source<T, N, R, TPF>(S, tauEA, p0A, pos, src);
                if constexpr (CACHE == 1)
                    static_for<0, R>([&](auto kc) { srcA[decltype(kc)::value * TPF + t] = src[decltype(kc)::value]; });
            }
            static_for<0, R>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                sinkA(pos[k], out(kc).re + src[k]);
            });
            positions(p0B, pos);
            deltaf_source<T, N, R, TPF>(S, tauEB, p0B, pos, src);
            static_for<0, R>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                sinkB(pos[k], out(kc).im + src[k]);
            });
            return;
        }
    }
    positions(p0A, pos);
    static_for<0, R>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        sinkA(pos[k], out(kc).re);
    });
    positions(p0B, pos);
    static_for<0, R>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        sinkB(pos[k], out(kc).im);
    });
}

// emit_pair into f: lines A and B through their descriptors and offsets.
template <typename T, int N, int R, int TPF, bool VSWEEP, int CACHE = 0, typename Out>
__device__ __forceinline__ void store_pair(const SimDev &S, double tauEA, double tauEB, long long bA,
                                           long long bB, int t, __amdgpu_buffer_rsrc_t rA, unsigned oA,
                                           __amdgpu_buffer_rsrc_t rB, unsigned oB, Out &&out,
                                           T *srcA = nullptr) {
    emit_pair<T, N, R, TPF, VSWEEP, CACHE>(
        S, tauEA, tauEB, bA, bB, t, out, [&](unsigned pos, T x) { buf_store<T>(x, rA, oA + pos, 0); },
        [&](unsigned pos, T x) { buf_store<T>(x, rB, oB + pos, 0); }, srcA);
}

// delta-f source of one line at the positions (t + k TPF - b) mod N that the
// unshifted indices t + k TPF of a result go to under the shift by b.
template <typename T, int N, int R, int TPF>
__device__ __forceinline__ void line_source(const SimDev &S, double tauE, long long b, int t, T (&src)[R]) {
    constexpr unsigned LB = N * sizeof(T);  // bytes per line
    const int p0 = (t - (int)(b & (N - 1))) & (N - 1);
    const unsigned p = (unsigned)p0 * sizeof(T);
    unsigned pos[R];
    static_for<0, R>([&](auto kc) {
        constexpr unsigned k = decltype(kc)::value;
        pos[k] = (p + k * TPF * sizeof(T)) & (LB - 1);
    });
    deltaf_source<T, N, R, TPF>(S, tauE, p0, pos, src);
}

// Weights of a line pair for its fractional shifts sA, sB, combined for the
// packed transform: wP = (wA + wB) / (2N), wQ = (wA - wB) / (2N) (the 1/N
// folds the scale of the inverse FFT), times `half` (0.5 for the 4096-point
// transform, which builds its symbols from (wP + i wQ) / 2).  Threads t = 0.. of the pair share the
// 2 x kTaps values; visible to the pair after the next barrier.
template <typename T, int N, int TPF>
__device__ __forceinline__ void pair_weights(int d, int interp, double sA, double sB, int t, T *wP,
                                             T *wQ, double half = 1.0) {
    for (int qi = t; qi < kTaps; qi += TPF) {
        const int q = qi - kDMax;
        const double wa = interp ? bspline_weight(d, q, sA) : lagrange_weight(d, q, sA);
        const double wb = interp ? bspline_weight(d, q, sB) : lagrange_weight(d, q, sB);
        const double sc = 0.5 * half / (double)N;
        wP[qi] = (T)((wa + wb) * sc);
        wQ[qi] = (T)((wa - wb) * sc);
    }
}

// Symbol of the kernel with weights w for the modes m = t + k TPF of one
// thread (k = 0..R-1): S_m = DFT_R^+ (H)[k] with the tap partial sums
// H_c = sum_{q = c mod R} w_q exp(2 pi i t q / N), the phases taken from the
// thread's row of the table eps (exp(2 pi i t q / N), q = 0..kEpsRow-1; the
// negative taps use their conjugates).
template <typename T, int R>
__device__ __forceinline__ void pair_symbol(const cx<T> *eps, const T *w, cx<T> (&H)[R]) {
    cx<T> e[kEpsRow];
    load_row<T, kEpsRow>(eps, e);
    static_for<0, R>([&](auto cc) { H[decltype(cc)::value] = cx<T>{(T)0, (T)0}; });
    static_for<0, kTaps>([&](auto qc) {
        constexpr int qi = decltype(qc)::value;
        constexpr int q = qi - kDMax;
        constexpr int c = ((q % R) + R) % R;
        constexpr int aq = q < 0 ? -q : q;
        const T wq = w[qi];
        if constexpr (q == 0) {
            H[c].re += wq;
        } else if constexpr (q > 0) {
            H[c].re = fma_t<T>(wq, e[aq].re, H[c].re);
            H[c].im = fma_t<T>(wq, e[aq].im, H[c].im);
        } else {
            H[c].re = fma_t<T>(wq, e[aq].re, H[c].re);
            H[c].im = fma_t<T>(-wq, e[aq].im, H[c].im);
        }
    });
    dft<T, 1, R>(H);
}

// The packed product of one line pair: on entry v[r] = z[t + r TPF] with
// z = uA + i uB; on exit Y[i] = y[t + TPF kpos(i)], y = IFFT(P Z + Q conj(Z_{N-m}))
// = (kernel A applied to uA) + i (kernel B applied to uB), unshifted.
// The symbol of the fractional-shift kernel for the modes m = t + k TPF is
//   S_m = sum_q w_q exp(2 pi i m q / N) = DFT_R^+ (H)[k],
//   H_c = sum_{q = c mod R} w_q exp(2 pi i t q / N),
// evaluated for the combined weights wP and wQ.  For B-splines (iden not
// null) the packed product of mode m is divided by the collocation symbol:
// Y_m *= iden[m].  All threads of the block must call this (it contains
// block barriers); WAVE: the pair's threads are contiguous lanes of one wave,
// and only that wave's threads must call it together.
template <typename T, int N, bool RELOAD_TW, bool WAVE = false, int R = fft_regs(N)>
__device__ __forceinline__ void pair_transform(cx<T> (&v)[R], cx<T> (&Y)[R], int t, T *lre, T *lim,
                                               const cx<T> *__restrict__ tw,
                                               const cx<T> *eps,
                                               const T *wP, const T *wQ,
                                               const T *__restrict__ iden) {
    using F = Fft<T, N>;
    constexpr int TPF = F::TPF;
    static_assert(R == F::R, "register count");

    F::template run<-1, WAVE>(v, t, lre, lim, tw);  // v[i] = Z[t + TPF kpos(i)]

    auto symbol = [&](const T *w, cx<T>(&H)[R]) { pair_symbol<T, R>(eps, w, H); };

    if constexpr (TPF > 1) {
        // Z to LDS at its natural position for the partner exchange.
        xsync<WAVE>();
        const int pt = F::pad(t);
        static_for<0, R>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int C = TPF * F::kpos(i);
            const int idx = (TPF % 16 == 0) ? F::template pad_add<C>(pt) : F::pad(t + C);
            lre[idx] = v[i].re;
            lim[idx] = v[i].im;
        });
        {
            cx<T> H[R];
            symbol(wP, H);
            static_for<0, R>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int k = F::kpos(i);
                Y[k] = cmul(H[k], v[i]);
            });
        }
        xsync<WAVE>();
        {
            cx<T> H[R];
            symbol(wQ, H);
            // partner index of m = t + k TPF is N - m = tp + (R - 1 - k) TPF for
            // t > 0 (tp = TPF - t) and (R - k) TPF mod N for t = 0.
            const int ptp = F::pad(TPF - t);
            static_for<0, R>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                constexpr int C1 = (R - 1 - k) * TPF;
                constexpr int C0 = ((R - k) % R) * TPF;
                const int idx = t == 0 ? F::pad(C0)
                                       : ((TPF % 16 == 0) ? F::template pad_add<C1>(ptp)
                                                          : F::pad(TPF - t + C1));
                const cx<T> Wk = cx<T>{lre[idx], -lim[idx]};
                Y[k] = Y[k] + cmul(H[k], Wk);
            });
        }
    } else {
        xsync<WAVE>();  // weights visible
        cx<T> H[R];
        symbol(wP, H);
        static_for<0, R>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int k = F::kpos(i);
            Y[k] = cmul(H[k], v[i]);
        });
        symbol(wQ, H);
        static_for<0, R>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int k = F::kpos(i);
            constexpr int ip = F::kinv((N - k) & (N - 1));
            Y[k] = Y[k] + cmul(H[k], cx<T>{v[ip].re, -v[ip].im});
        });
    }
    if (iden) {
        static_for<0, R>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const T sc = iden[t + k * TPF];
            Y[k].re *= sc;
            Y[k].im *= sc;
        });
    }

    // RELOAD_TW: re-read the twiddle rows instead of keeping the forward
    // pass's rows live in registers (for kernels with a tight register budget).
    if constexpr (RELOAD_TW) F::template run<1, WAVE>(Y, t, lre, lim, opaque(tw));
    else F::template run<1, WAVE>(Y, t, lre, lim, tw);  // Y[i] = y[t + TPF kpos(i)]
}

// Two applications of the packed kernel with a source term between them,
// composed in Fourier space.  On entry v[r] = z[t + r TPF] (z = uA + i uB)
// and, with SRC, s[r] = zs[t + r TPF] (zs = sA + i sB, each line's source at
// the positions its first result would be stored to); on exit
// Y[i] = y[t + TPF kpos(i)] with
//   y = IFFT(K (K Z + Zs)),  K X = P X_m + Q conj(X_{N-m}),
// formed from the thread's own modes and their partners N - m alone, as the
// symbols of real kernels satisfy P_{N-m} = conj(P_m) (likewise Q):
//   (K X)_m = P X_m + Q conj(X_{N-m}),  conj((K X)_{N-m}) = Q X_m + P conj(X_{N-m}).
// The scale 1/N of the inverse transform is in wP, wQ, hence the factor N on
// the inner application.  lre2, lim2: a second pair of exchange arrays (for
// zs).
template <typename T, int N, bool SRC, bool WAVE = false, int R = fft_regs(N)>
__device__ __forceinline__ void pair_transform2(cx<T> (&v)[R], cx<T> (&s)[R], cx<T> (&Y)[R], int t, T *lre,
                                                T *lim, T *lre2, T *lim2, const cx<T> *__restrict__ tw,
                                                const cx<T> *eps, const T *wP, const T *wQ,
                                                const T *__restrict__ iden) {
    using F = Fft<T, N>;
    constexpr int TPF = F::TPF;
    static_assert(R == F::R, "register count");

    // v[i] = Z[t + TPF kpos(i)], s[i] = Zs[t + TPF kpos(i)]
    if constexpr (SRC) F::template run2<-1, WAVE>(v, s, t, lre, lim, lre2, lim2, tw);
    else F::template run<-1, WAVE>(v, t, lre, lim, tw);

    auto symbol = [&](const T *w, cx<T>(&H)[R]) { pair_symbol<T, R>(eps, w, H); };

    if constexpr (TPF > 1) {
        // Z (and Zs) to LDS at their natural positions for the partner exchange
        xsync<WAVE>();
        const int pt = F::pad(t);
        static_for<0, R>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int C = TPF * F::kpos(i);
            const int idx = (TPF % 16 == 0) ? F::template pad_add<C>(pt) : F::pad(t + C);
            lre[idx] = v[i].re;
            lim[idx] = v[i].im;
            if constexpr (SRC) {
                lre2[idx] = s[i].re;
                lim2[idx] = s[i].im;
            }
        });
    } else {
        xsync<WAVE>();  // weights visible
    }
    cx<T> HP[R], HQ[R];
    symbol(wP, HP);
    symbol(wQ, HQ);
    if (iden) {
        static_for<0, R>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const T sc = iden[t + k * TPF];
            HP[k].re *= sc;
            HP[k].im *= sc;
            HQ[k].re *= sc;
            HQ[k].im *= sc;
        });
    }
    if constexpr (TPF > 1) xsync<WAVE>();
    const int ptp = F::pad(TPF - t);
    static_for<0, R>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int k = F::kpos(i);
        // partner of m = t + k TPF: N - m = tp + (R - 1 - k) TPF for t > 0
        // (tp = TPF - t), (R - k) TPF mod N for t = 0
        cx<T> Zp, Sp;
        if constexpr (TPF > 1) {
            constexpr int C1 = (R - 1 - k) * TPF;
            constexpr int C0 = ((R - k) % R) * TPF;
            const int idx = t == 0 ? F::pad(C0)
                                   : ((TPF % 16 == 0) ? F::template pad_add<C1>(ptp) : F::pad(TPF - t + C1));
            Zp = cx<T>{lre[idx], -lim[idx]};
            if constexpr (SRC) Sp = cx<T>{lre2[idx], -lim2[idx]};
        } else {
            constexpr int ip = F::kinv((N - k) & (N - 1));
            Zp = cx<T>{v[ip].re, -v[ip].im};
            if constexpr (SRC) Sp = cx<T>{s[ip].re, -s[ip].im};
        }
        // inner application U = N (P Z + Q conj(Z_{N-m})) + Zs and its value at
        // the partner, conjugated, W = N (Q Z + P conj(Z_{N-m})) + conj(Zs_{N-m});
        // then y = P U + Q W
        const cx<T> P = HP[k], Q = HQ[k];
        constexpr T n1 = (T)N;
        cx<T> U = cmac(cmul(P, v[i]), Q, Zp);
        cx<T> W = cmac(cmul(Q, v[i]), P, Zp);
        if constexpr (SRC) {
            U = cx<T>{fma_t<T>(n1, U.re, s[i].re), fma_t<T>(n1, U.im, s[i].im)};
            W = cx<T>{fma_t<T>(n1, W.re, Sp.re), fma_t<T>(n1, W.im, Sp.im)};
        } else {
            U = cx<T>{n1 * U.re, n1 * U.im};
            W = cx<T>{n1 * W.re, n1 * W.im};
        }
        Y[k] = cmac(cmul(P, U), Q, W);
    });

    F::template run<1, WAVE>(Y, t, lre, lim, tw);  // Y[i] = y[t + TPF kpos(i)]
}

// KIND 0: v-advection by tau = b.a[sim] with field E (lines are x-columns of
// f, length nv).  KIND 1: x-advection by dt = b.a[sim] (lines are v-rows of
// the transposed copy g, length nx).  KIND 2: two v-advections by tau in a
// row with the same E (the closing half step of one Strang step and the
// opening one of the next): the first result, source term included, goes
// through LDS instead of f, in the same FP32 or FP64 values a store and a
// reload would give.  KIND 3: the same two v-advections composed in Fourier
// space (pair_transform2: forward transforms of the lines and of the first
// step's source, one inverse), stored with twice the integer shift; equal to
// KIND 2 up to rounding.
//
// Two real lines A, B are packed as z = uA + i uB and transformed together.
// With beta = b + s (b integer, s in [0,1)), the circulant A of Section 1.2 is
// the cyclic shift by b composed with the kernel w_q(s), q = -d..d+1 (Lagrange,
// or B-spline taps followed by the division by the collocation symbol).
// The kernel is applied in Fourier space through its symbol and the shift by
// b is applied exactly on the store (index j -> j - b mod N).
template <typename T, int N>
struct Sweep {
    using F = Fft<T, N>;
    static constexpr int PPB = 256 / F::TPF;  // line pairs per 256-thread block
    // LDS: the pairs' exchange arrays, then their weights
    static constexpr int SMEM = PPB * 2 * F::LDSN + PPB * 2 * kTaps;
    // KIND 2 in FP32 also keeps line A's delta-f source values of each pair
    // between its two half steps (PPB N = 4096 values, 16 KB) where 3 blocks
    // per CU still fit the 160 KB of LDS (lines of 256 points or more)
    static constexpr bool SRC_CACHE = sizeof(T) == 4 && 3 * (SMEM + PPB * N) * (int)sizeof(T) <= 160 * 1024;
    static constexpr int SMEM2 = SMEM + (SRC_CACHE ? PPB * N : 0);
    // KIND 3: a second pair of exchange arrays per line pair (lines of more
    // than 16 points, whose transforms exchange through LDS)
    static constexpr int SMEM3 = SMEM + (F::TPF > 1 ? PPB * 2 * F::LDSN : 0);
    // KIND 3 has a kernel for FP32 lines (the library runs FP64 sims with
    // KIND 2); elsewhere it stands for two KIND 0 launches
    static constexpr bool COMPOSED = sizeof(T) == 4 && SMEM3 * (int)sizeof(T) <= 160 * 1024;
};

// Block blk of sim `sim` of the batch; smem holds Sweep<T, N>::SMEM values
// (KIND 2: SMEM2).
// CACHE_SRC: KIND 2 may keep line A's source values in smem past SMEM (the
// mixed-length kernel, whose LDS is sized for its shortest lines, does not).
template <typename T, int N, int KIND, bool CACHE_SRC = Sweep<T, N>::SRC_CACHE>
__device__ __forceinline__ void sweep_body(const SweepBatch &b, int sim, int blk, T *smem) {
    using F = Fft<T, N>;
    constexpr int R = F::R, TPF = F::TPF, PPB = Sweep<T, N>::PPB;
    T(*lds)[2][F::LDSN] = reinterpret_cast<T(*)[2][F::LDSN]>(smem);
    T(*wsh)[2][kTaps] = reinterpret_cast<T(*)[2][kTaps]>(smem + PPB * 2 * F::LDSN);

    const SimDev &S = *b.s[sim];
    constexpr bool VS = KIND != 1;  // a v-sweep
    const int nlines = VS ? S.nx : S.nv;
    const int npairs = nlines >> 1;
    if (blk * PPB >= npairs) return;  // whole block idle

    const int slot = threadIdx.x / TPF;
    const int t = threadIdx.x % TPF;
    const int pair = blk * PPB + slot;
    const bool active = pair < npairs;
    const int lineA = active ? 2 * pair : 0;
    const int lineB = lineA + 1;
    T *lre = lds[slot][0];
    T *lim = lds[slot][1];
    T *srcA = smem + Sweep<T, N>::SMEM + slot * N;  // KIND 2 FP32: line A's source values
    const cx<T> *tw = (const cx<T> *)(VS ? S.tw_v : S.tw_x);
    const cx<T> *eps = (const cx<T> *)(VS ? S.eps_v : S.eps_x) + t * kEpsRow;
    // One pair per block: a descriptor per line (uniform base).  Otherwise one
    // for the sim's array, with the line's offset in the byte offset.
    constexpr unsigned LB = N * sizeof(T);  // bytes per line
    const T *data = (const T *)(VS ? S.f : S.g);
    __amdgpu_buffer_rsrc_t rA, rB;
    unsigned oA, oB;
    if constexpr (PPB == 1) {
        rA = buf_rsrc(data + (size_t)lineA * N, LB);  // slot 0 for every thread
        rB = buf_rsrc(data + (size_t)lineB * N, LB);
        oA = oB = 0;
    } else {
        rA = rB = buf_rsrc(data, (unsigned)nlines * LB);
        oA = (unsigned)lineA * LB;
        oB = oA + LB;
    }

    // Shift of each line, FP64: v-sweep beta = -tau E_i / dv, x-sweep
    // beta = -v_j dt / dx.
    const double arg = b.a[sim];
    double EA = 0.0, EB = 0.0, betaA, betaB;
    if constexpr (VS) {
        // E - E_app when the sim is driven, else E (the field solve then
        // leaves Eeff unwritten)
        const double *Ev = S.drv_sc ? S.Eeff : S.E;
        EA = Ev[lineA];
        EB = Ev[lineB];
        betaA = -arg * EA * S.inv_dv;
        betaB = -arg * EB * S.inv_dv;
    } else {
        betaA = -(S.vmin + lineA * S.dv) * arg * S.inv_dx;
        betaB = -(S.vmin + lineB * S.dv) * arg * S.inv_dx;
    }
    long long bA, bB;
    double sA, sB;
    split_shift(betaA, bA, sA);
    split_shift(betaB, bB, sB);
    if constexpr (PPB == 1) {
        // the same in every lane: keep them in scalar registers for the store
        bA = uniform_ll(bA);
        bB = uniform_ll(bB);
        EA = uniform_d(EA);
        EB = uniform_d(EB);
    }
    // FP64 4096-point lines: the four-wave digit transform of pair4096.hpp
    // (measured faster there; for FP32 the radix-16 Stockham transform below
    // is)
    constexpr bool kP4k = N == 4096 && sizeof(T) == 8;
    static_assert(!kP4k || (PPB == 1 && TPF == 256), "one 4096-point pair per 256-thread block");
    pair_weights<T, N, TPF>(S.d, S.interp, sA, sB, t, wsh[slot][0], wsh[slot][1], kP4k ? 0.5 : 1.0);

    // Load the two lines packed as z = uA + i uB (a slot past the last pair
    // reads lines 0 and 1 and stores nothing).
    cx<T> v[R];
    {
        const unsigned tb = (unsigned)t * sizeof(T);
        static_for<0, R>([&](auto rc) {
            constexpr unsigned r = decltype(rc)::value;
            v[r] = cx<T>{buf_load<T>(rA, oA + tb, r * TPF * sizeof(T)),
                         buf_load<T>(rB, oB + tb, r * TPF * sizeof(T))};
        });
    }

    // Y[i] holds the result at position t + TPF kpos(i) (kP4k: kpos(i) = i)
    cx<T> Y[R];
    const T *iden = (const T *)(VS ? S.iden_v : S.iden_x);
    // (KIND 2 gives the second transform opaque copies of the tables and of
    // t, so that it reads the tables and forms its LDS addresses again
    // instead of keeping the first transform's values live)
    auto transform = [&](const cx<T> *twp, const cx<T> *epsp, int tt) {
        if constexpr (kP4k) {
            const cx<T> *eps0 = epsp - tt * kEpsRow;
            {
                cx<T> w[16];
                p4k_col_row<T>(twp, tt, w);
                p4k_fwd_col<T>(v, tt, lre, lim, w);
            }
            __syncthreads();
            p4k_lanes<T>(__builtin_amdgcn_readfirstlane(tt >> 6), tt & 63, lre, lim, LoadRows<T>{twp, eps0},
                         wsh[0][0], iden);
            __syncthreads();
            {
                cx<T> w[16];
                p4k_col_row<T>(opaque(twp), tt, w);  // re-read, not kept live
                p4k_inv_col<T>(Y, tt, lre, lim, w);
            }
        } else {
            // a line pair of at most 1024 points is one wave's contiguous lanes
            pair_transform<T, N, (sizeof(T) == 8), (TPF <= 64)>(v, Y, tt, lre, lim, twp, epsp, wsh[slot][0],
                                                                wsh[slot][1], iden);
        }
    };
    auto out = [&](auto kc) -> const cx<T> & {
        constexpr int k = decltype(kc)::value;
        if constexpr (kP4k) return Y[k];
        else return Y[F::kinv(k)];
    };

    if constexpr (KIND == 3) {
        // u2 = shift_2b(K (K u0 + shift_-b s)) + s: the source s of each line
        // taken at the positions j - b of the first step's store, the result
        // stored at j - 2b with s added there.
        static_assert(Sweep<T, N>::COMPOSED && !kP4k, "no composed kernel for these lines");
        constexpr bool WAVE = TPF <= 64;
        T *lre2 = smem + Sweep<T, N>::SMEM + slot * 2 * F::LDSN;
        T *lim2 = lre2 + F::LDSN;
        cx<T> s[R];
        if (S.deltaf) {
            {
                T sa[R];
                line_source<T, N, R, TPF>(S, arg * EA, bA, t, sa);
                static_for<0, R>([&](auto rc) { s[decltype(rc)::value].re = sa[decltype(rc)::value]; });
            }
            {
                T sb[R];
                line_source<T, N, R, TPF>(S, arg * EB, bB, t, sb);
                static_for<0, R>([&](auto rc) { s[decltype(rc)::value].im = sb[decltype(rc)::value]; });
            }
            pair_transform2<T, N, true, WAVE>(v, s, Y, t, lre, lim, lre2, lim2, tw, eps, wsh[slot][0],
                                              wsh[slot][1], iden);
        } else {
            pair_transform2<T, N, false, WAVE>(v, s, Y, t, lre, lim, lre2, lim2, tw, eps, wsh[slot][0],
                                               wsh[slot][1], iden);
        }
        if (!active) return;
        store_pair<T, N, R, TPF, VS, 0>(S, arg * EA, arg * EB, 2 * bA, 2 * bB, t, rA, oA, rB, oB, out);
        return;
    }
    transform(tw, eps, t);
    if constexpr (KIND == 2) {
        // The first half step's result to LDS at its positions in the line,
        // then back in the load layout v[r] = z[t + r TPF] for the second.
        // The pair's threads are one wave for lines of at most 1024 points.
        constexpr bool WAVE = !kP4k && TPF <= 64;
        xsync<WAVE>();
        emit_pair<T, N, R, TPF, true, (CACHE_SRC ? 1 : 0)>(
            S, arg * EA, arg * EB, bA, bB, t, out,
            [&](unsigned pos, T x) { lre[F::pad((int)(pos / sizeof(T)))] = x; },
            [&](unsigned pos, T x) { lim[F::pad((int)(pos / sizeof(T)))] = x; }, srcA);
        xsync<WAVE>();
        static_for<0, R>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            const int i = F::pad(t + r * TPF);
            v[r] = cx<T>{lre[i], lim[i]};
        });
        if constexpr (kP4k) __syncthreads();  // reads done before the digit transform writes
        transform(opaque(tw), opaque(eps), opaque(t));
    }

    if (!active) return;

    // (KIND 2: positions formed again, not kept live from the staging above;
    // line A's source values from the staging's cache)
    constexpr int CACHE = (KIND == 2 && CACHE_SRC) ? 2 : 0;
    store_pair<T, N, R, TPF, VS, CACHE>(S, arg * EA, arg * EB, bA, bB, KIND == 2 ? opaque(t) : t, rA, oA, rB,
                                        oB, out, srcA);
}

// One line length per launch: blockIdx.y = sim, blockIdx.x = block.
template <typename T, int N, int KIND>
__global__ __launch_bounds__(256, (KIND == 3 ? 2 : (sizeof(T) == 4 && N >= 32 ? 3 : 1))) void sweep_kernel(
    const SweepBatch b) {
    __shared__ T smem[KIND == 3 ? Sweep<T, N>::SMEM3 : KIND == 2 ? Sweep<T, N>::SMEM2 : Sweep<T, N>::SMEM];
    sweep_body<T, N, KIND>(b, (int)blockIdx.y, (int)blockIdx.x, smem);
}

// Sim of block bid in a launch over mixed line lengths (m.first ascending,
// m.first[0] = 0): the number of j in 1 .. n-1 with first[j] <= bid, two
// candidates j per lane of the wave, counted with two ballots.  All 64 lanes
// of the wave must call it.
static_assert(kMaxSweepBatch <= 128, "two candidate sims per lane");
__device__ __forceinline__ int mixed_sim(const SweepBatch &b, const SweepMap &m, int bid) {
    const int j = (int)(threadIdx.x & 63) + 1, j2 = j + 64;
    const bool le = j < b.n && m.first[j] <= bid;
    const bool le2 = j2 < b.n && m.first[j2] <= bid;
    return __builtin_amdgcn_readfirstlane(__popcll(__ballot(le)) + __popcll(__ballot(le2)));
}

// x-advection by dt = b.a[sim] directly on the v-fastest layout f[nx][nv]
// (N = nx): a block owns the x-lines j0 .. j0 + B - 1, i.e. the tile
// f[0..N)[j0..j0+B), and runs the packed line-pair transform on B / 2 pairs
// at once.  Loads go straight to registers: the B / 2 threads that share a
// position t read the row's B contiguous values together.  The shifted
// results are staged through LDS and stored as 16-byte row segments.  Tiles
// are ordered so that the blocks sharing cache lines (neighbouring j0) run
// on the same XCD at the same time.
template <typename T, int N>
struct Fused {
    using F = Fft<T, N>;
    // Threads per block and the minimum waves per SIMD they are compiled
    // for.  Short lines take small blocks (3 waves per SIMD for FP32, up to
    // 168 VGPRs, no spills) while keeping 8 or more lines per tile (32 bytes
    // or more of each row); longer lines need larger blocks for tiles that
    // wide: 2048 points 512 threads (8 lines), 4096 points 1024 threads
    // (8 lines, at most 128 VGPRs).  FP64: 256 threads up to 2048 points.
    static constexpr int TB = sizeof(T) == 4 ? (N > 2048 ? 1024 : (N == 2048 ? 512 : 256))
                                             : (N >= 4096 ? 512 : 256);
    static constexpr int WAVES = sizeof(T) == 4 ? (N <= 1024 ? 3 : (N == 2048 ? 2 : 1))
                                                : (N >= 256 ? 2 : 1);  // short FP64 lines: LDS-bound
    static constexpr int PPB = TB / F::TPF;     // line pairs per block
    static constexpr int B = 2 * PPB;           // lines per block
    static constexpr int VEC = 16 / sizeof(T);  // elements per 16-byte vector
    static constexpr int VPR = B / VEC;         // vectors per tile row
    static constexpr int SKEW = sizeof(T) == 4 ? (VPR >= 16 ? 1 : 16 / VPR) : 8;
    static constexpr int LDSP = F::LDSN + SKEW; // per-array stride (bank skew)
    static constexpr int ITER = N * VPR / TB;   // tile vectors per thread
    static constexpr int SMEM = PPB * 2 * LDSP + PPB * 2 * kTaps;
};

template <typename T, int N>
constexpr int kFusedThreads = Fused<T, N>::TB;

// Block hb of sim `sim`; smem holds Fused<T, N>::SMEM values.
template <typename T, int N>
__device__ __forceinline__ void xsweep_body(const SweepBatch &b, int sim, int hb, T *smem) {
    using F = Fft<T, N>;
    using C = Fused<T, N>;
    constexpr int R = F::R, TPF = F::TPF;
    T *lds = smem;
    T(*wsh)[2][kTaps] = reinterpret_cast<T(*)[2][kTaps]>(smem + C::PPB * 2 * C::LDSP);

    const SimDev &S = *b.s[sim];
    const int nv = S.nv;
    const int ntiles = nv / C::B;
    if (hb >= ntiles) return;  // whole block idle
    const int tile = (ntiles % 8 == 0) ? (hb % 8) * (ntiles / 8) + hb / 8 : hb;
    const int j0 = tile * C::B;
    T *f = (T *)S.f;
    const int tid = threadIdx.x;

    // Shifts and weights first, while no tile data is live in registers.
    // Pairs are the fastest-varying part of the thread index, so the PPB
    // threads with the same t read one row's 2 PPB contiguous values.
    const int slot = tid % C::PPB;
    const int t = tid / C::PPB;
    const int lineA = j0 + 2 * slot, lineB = lineA + 1;
    const double dt = b.a[sim];
    long long bA, bB;
    double sA, sB;
    split_shift(-(S.vmin + lineA * S.dv) * dt * S.inv_dx, bA, sA);
    split_shift(-(S.vmin + lineB * S.dv) * dt * S.inv_dx, bB, sB);
    pair_weights<T, N, TPF>(S.d, S.interp, sA, sB, t, wsh[slot][0], wsh[slot][1]);

    // The pair's two lines straight into registers: v[r] = z[t + r TPF],
    // z = u_lineA + i u_lineB, one 2-value load per row.
    cx<T> v[R];
    {
        typedef T v2t __attribute__((ext_vector_type(2)));
        const gmem<v2t> *src = (const gmem<v2t> *)(f + (size_t)t * nv + lineA);
        static_for<0, R>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            const v2t z = src[(size_t)r * TPF * (nv / 2)];
            v[r] = cx<T>{z.x, z.y};
        });
    }

    T *lre = lds + (2 * slot) * C::LDSP;
    T *lim = lre + C::LDSP;
    const cx<T> *tw = (const cx<T> *)S.tw_x;
    const cx<T> *eps = (const cx<T> *)S.eps_x + t * kEpsRow;

    cx<T> Y[R];
    // FP32 lines up to 512 points keep the twiddle rows in registers (measured
    // faster there); longer lines and FP64 re-read them to stay unspilled.
    pair_transform<T, N, !(sizeof(T) == 4 && N <= 512)>(v, Y, t, lre, lim, tw, eps, wsh[slot][0],
                                                         wsh[slot][1], (const T *)S.iden_x);

    // Shifted result back to LDS: unshifted index j goes to position (j - b) mod N.
    __syncthreads();
    {
        const int p0A = (t - (int)(bA & (N - 1))) & (N - 1);
        const int p0B = (t - (int)(bB & (N - 1))) & (N - 1);
        static_for<0, R>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            constexpr int i = F::kinv(k);
            lre[F::pad((p0A + k * TPF) & (N - 1))] = Y[i].re;
            lim[F::pad((p0B + k * TPF) & (N - 1))] = Y[i].im;
        });
    }
    __syncthreads();

    // Rows of the tile back to f, and the tile's share of rho = int f dv: the
    // FP64 sum of each row's B values in a fixed order (a thread's VEC values
    // pairwise, then xor-shuffles over the VPR neighbouring lanes that hold
    // the row, which leave the same sum in each of them) -> part[tile][row].
    static_assert(C::TB % 64 == 0 && 64 % C::VPR == 0, "a row's vectors sit in one wave");
    gmem<double> *part = as_global(S.part) + (size_t)tile * N;
    static_for<0, C::ITER>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const int q = tid + k * C::TB;
        const int row = q / C::VPR, cv = q % C::VPR;
        T *dst = f + (size_t)row * nv + j0 + cv * C::VEC;
        const int pr = F::pad(row);
        T e[C::VEC];
        static_for<0, C::VEC>([&](auto ec) {
            constexpr int el = decltype(ec)::value;
            e[el] = lds[(cv * C::VEC + el) * C::LDSP + pr];
        });
        double sum;
        if constexpr (sizeof(T) == 4) {
            *reinterpret_cast<float4 *>(dst) = float4{e[0], e[1], e[2], e[3]};
            sum = ((double)e[0] + (double)e[1]) + ((double)e[2] + (double)e[3]);
        } else {
            *reinterpret_cast<double2 *>(dst) = double2{e[0], e[1]};
            sum = e[0] + e[1];
        }
        static_for<0, ilog2(C::VPR)>([&](auto oc) { sum += xor_lane<1 << decltype(oc)::value>(sum); });
        if (cv == 0) part[row] = sum;
    });
}

template <typename T, int N>
__global__ __launch_bounds__((kFusedThreads<T, N>), (Fused<T, N>::WAVES)) void xsweep_fused_kernel(const SweepBatch b) {
    __shared__ T smem[Fused<T, N>::SMEM];
    xsweep_body<T, N>(b, (int)blockIdx.y, (int)blockIdx.x, smem);
}
// ----------------------------------------------------------------- rho

// rho_i = dv sum_p part[p][i] + feq_const for the kRhoCols columns
// i = c0 .. c0 + kRhoCols - 1, by G * kRhoCols threads, in a fixed order: row
// group g sums rows p = g, g + G, g + 2G, ... in turn, then the G group sums
// are added pairwise.  Each group reads kRhoCols * 8 contiguous bytes per row;
// a thread requests its rows DEPTH at a time before adding them.  red holds
// G * kRhoCols doubles; all threads of the block must call it.
template <int G, int DEPTH>
__device__ __forceinline__ void rho_columns(const SimDev &S, int c0, double *red) {
    static_assert((G & (G - 1)) == 0, "G is a power of two");
    const int tx = threadIdx.x % kRhoCols, g = threadIdx.x / kRhoCols;
    const int i = c0 + tx;
    const int np = S.nparts, nx = S.nx;
    const gmem<double> *part = as_global(S.part) + i;
    double acc = 0.0;
    if (i < nx) {
        for (int p0 = g; p0 < np; p0 += DEPTH * G) {
            double x[DEPTH];
            static_for<0, DEPTH>([&](auto uc) {
                constexpr int u = decltype(uc)::value;
                const int p = p0 + u * G;
                x[u] = p < np ? part[(size_t)p * nx] : 0.0;
            });
            static_for<0, DEPTH>([&](auto uc) { acc += x[decltype(uc)::value]; });
        }
    }
    red[g * kRhoCols + tx] = acc;
    for (int h = G / 2; h > 0; h /= 2) {
        __syncthreads();
        if (g < h) red[g * kRhoCols + tx] += red[(g + h) * kRhoCols + tx];
    }
    if (g == 0 && i < nx) as_global(S.rho)[i] = S.dv * red[tx] + S.feq_const;
}

// ----------------------------------------------------------------- field solve

// One block per sim, TPF = N/16 threads (N = nx).  rho_hat = FFT(rho) gives
// the diagnostics (rho_hat_0 .. rho_hat_7) and, for the Fourier solve,
// E_hat_m = rho_hat_m / (i k_m) with E_hat_0 = E_hat_{N/2} = 0 (Section 3.2),
// E = iFFT.  The trapezoidal solve integrates rho - mean (zero_mean) or
// rho - 1 from E_0 = 0 and, with zero_mean, subtracts the mean of E
// (Section 3.2).  Writes E, the advecting field E - E_app(t) and the step's
// diagnostics record.
template <int N>
constexpr int kFieldThreads = Fft<double, N>::TPF;

template <int N>
struct Field {
    using F = Fft<double, N>;
    static constexpr int TPF = F::TPF;
    static constexpr int NW = (TPF + 63) / 64;  // waves in the block
    // LDS (doubles): lre, lim, red, scan, modes, bad flag
    static constexpr int SMEM = 2 * F::LDSN + NW + TPF + 16 + 1;
};

// Field solve of sim `sim` by threads t = 0 .. TPF - 1 (all of them must call
// it); smem holds Field<N>::SMEM doubles.
template <int N>
__device__ __forceinline__ void field_body(const Batch &b, int sim, double *smem) {
    using F = Fft<double, N>;
    constexpr int R = F::R, TPF = F::TPF;
    constexpr int NW = Field<N>::NW;
    constexpr int WL = TPF < 64 ? TPF : 64;
    double *lre = smem, *lim = smem + F::LDSN;
    double *red = lim + F::LDSN;
    double *scan = red + NW;
    double(*modes)[2] = reinterpret_cast<double(*)[2]>(scan + TPF);
    int *bad = reinterpret_cast<int *>(scan + TPF + 16);

    const SimDev &S = *b.s[sim];
    const int t = threadIdx.x;
    const cx<double> *tab = (const cx<double> *)S.tw_x64;
    if (t == 0) bad[0] = 0;
    if (t < 8) modes[t][0] = modes[t][1] = 0.0;

    // block sum in a fixed order: xor-shuffles in each wave, then the waves
    auto block_sum = [&](double x) {
        for (int off = WL / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, WL);
        if constexpr (NW > 1) {
            __syncthreads();
            if ((t & 63) == 0) red[t >> 6] = x;
            __syncthreads();
            x = red[0];
            for (int wv = 1; wv < NW; ++wv) x += red[wv];
        }
        return x;
    };

    const gmem<double> *rho = as_global(S.rho);
    cx<double> v[R];
    static_for<0, R>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        v[r] = cx<double>{rho[t + r * TPF], 0.0};
    });
    // All twiddles of both transforms, requested together with rho (6 of
    // every 16 table entries; the block is latency-bound on this fetch).
    typename F::Rows rows;
    F::load_rows_sparse(t, tab, rows);
    // 1/(N k_m) for this thread's modes, requested now so that the loads
    // overlap the forward transform (Fourier solve only).
    double ik[R];
    if (S.poisson != VOG_POISSON_TRAPEZOID) {
        const gmem<double> *invk = as_global(S.invk);
        static_for<0, R>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            ik[k] = invk[t + TPF * k];
        });
    }
    F::template run<-1>(v, t, lre, lim, rows);

    // rho_hat_0 .. rho_hat_7 (unnormalised here).
    static_for<0, R>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const int m = t + TPF * F::kpos(i);
        if (m < 8) {
            modes[m][0] = v[i].re;
            modes[m][1] = v[i].im;
        }
    });

    double e[R];  // E at positions t + TPF kpos(i)
    if (S.poisson == VOG_POISSON_TRAPEZOID) {
        __syncthreads();  // modes visible
        const double mean = S.zero_mean ? modes[0][0] / (double)N : 1.0;
        // Contiguous chunk j = t R .. t R + R - 1 of rho~ = rho - mean and the
        // increments dx (rho~_j + rho~_{j+1}) / 2 for j < N - 1.
        double acc = 0.0, loc[R];
        double rj = rho[t * R] - mean;
        static_for<0, R>([&](auto jc) {
            constexpr int jj = decltype(jc)::value;
            const int j = t * R + jj;
            loc[jj] = acc;  // sum of the chunk's increments before j
            const double rn = (j + 1 < N) ? rho[j + 1] - mean : 0.0;
            if (j + 1 < N) acc += S.dx * 0.5 * (rj + rn);
            rj = rn;
        });
        scan[t] = acc;
        __syncthreads();
        if (t == 0) {
            double run = 0.0;
            for (int k = 0; k < TPF; ++k) {
                const double c = scan[k];
                scan[k] = run;
                run += c;
            }
        }
        __syncthreads();
        const double off = scan[t];
        double esum = 0.0;
        static_for<0, R>([&](auto jc) {
            constexpr int jj = decltype(jc)::value;
            loc[jj] += off;
            esum += loc[jj];
        });
        const double emean = S.zero_mean ? block_sum(esum) / (double)N : 0.0;
        // back to the strided ownership used below: through LDS
        __syncthreads();
        static_for<0, R>([&](auto jc) {
            constexpr int jj = decltype(jc)::value;
            lre[F::pad(t * R + jj)] = loc[jj] - emean;
        });
        __syncthreads();
        static_for<0, R>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            e[i] = lre[F::pad(t + TPF * F::kpos(i))];
        });
    } else {
        // E_hat_m = rho_hat_m / (i k_m) = (Im rho_hat_m, -Re rho_hat_m) / k_m with
        // the table invk[m] = 1 / (N k_m) (0 for m = 0, m = N/2, or a zero field;
        // 1/N is the scale of the inverse transform).
        cx<double> Y[R];
        static_for<0, R>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int k = F::kpos(i);
            Y[k] = cx<double>{v[i].im * ik[k], -v[i].re * ik[k]};
        });
        F::template run<1>(Y, t, lre, lim, rows);
        static_for<0, R>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            e[i] = Y[i].re;
        });
    }

    double e2 = 0.0;
    bool finite = true;
    // drive: E_app(t, x_j) = damp sin(k x_j - dph) from the table of
    // sin(k x_j), cos(k x_j) (all of this thread's entries requested before
    // any store) and one sincos of dph
    const double damp = b.drv_amp[sim];
    double app[R];
    if (damp != 0.0) {
        double sph, cph;
        sincos(b.drv_ph[sim], &sph, &cph);
        typedef double v2d __attribute__((ext_vector_type(2)));
        const gmem<v2d> *sc = as_global(reinterpret_cast<const v2d *>(S.drv_sc));
        v2d w[R];
        static_for<0, R>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            w[i] = sc[t + TPF * F::kpos(i)];
        });
        static_for<0, R>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            app[i] = damp * (w[i].x * cph - w[i].y * sph);
        });
    } else {
        static_for<0, R>([&](auto ic) { app[decltype(ic)::value] = 0.0; });
    }
    static_for<0, R>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const int j = t + TPF * F::kpos(i);
        const double ej = S.field_zero ? 0.0 : e[i];
        as_global(S.E)[j] = ej;
        if (S.drv_sc) as_global(S.Eeff)[j] = ej - app[i];
        e2 = fma(ej, ej, e2);
        finite = finite && isfinite(ej);
    });
    if (!finite) bad[0] = 1;
    e2 = block_sum(e2);
    if constexpr (NW == 1) __syncthreads();  // modes and bad visible to thread 0
    if (t == 0) {
        const double invn = 1.0 / (double)N;
        vog_diag d;
        d.step = b.step[sim];
        d.t = b.t[sim];
        d.normE = sqrt(S.dx * e2);
        d.rho0 = modes[0][0] * invn;
        d.abs_rho1 = sqrt(modes[1][0] * modes[1][0] + modes[1][1] * modes[1][1]) * invn;
        for (int m = 1; m < 8; ++m)
            d.abs_rho_modes[m - 1] =
                m < N ? sqrt(modes[m][0] * modes[m][0] + modes[m][1] * modes[m][1]) * invn : 0.0;
        d.l2 = __builtin_nan("");
        d.energy = __builtin_nan("");
        d.finite = bad[0] ? 0 : 1;
        d.reserved = 0;
        S.ring[d.step % kRingCap] = d;
    }
}

template <int N>
__global__ __launch_bounds__(kFieldThreads<N>) void field_kernel(const Batch b) {
    __shared__ double smem[Field<N>::SMEM];
    field_body<N>(b, (int)blockIdx.x, smem);
}
}  // namespace vog
