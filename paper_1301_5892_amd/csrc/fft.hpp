// Batched LDS-resident complex FFT for gfx950 (wave64), FP32 and FP64.
//
// One transform of length N (a power of two, 8 <= N <= 4096) is carried by
// TPF = N / R threads that each hold R = min(N, 16) complex values in
// registers.  The transform is a Stockham autosort sequence of passes of
// radix 16 (the last pass takes the remaining factor 2, 4, 8 or 16); every
// pass works on registers, and consecutive passes exchange data through LDS
// (structure-of-arrays, one padding slot per 16 elements, so that every LDS
// address is a per-thread base plus a compile-time offset).
//
// Layouts (t = thread index within the transform, 0 <= t < TPF):
//   input:  register r holds element t + r * TPF            (r < R)
//   output: register i holds frequency t + TPF * kpos(i)    (i < R)
// kpos is a compile-time permutation fixed by the last pass radix.
//
// Twiddles of pass p >= 1 (sub-transform length NS = 16^p, radix RP) come
// from a table with one row of 16 entries per k < NS:
//   row k, entry r = exp(+2 pi i r k / (NS RP))   (conjugated when forward),
// built in FP64 on the host and rounded to the storage precision.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>
#include <utility>

namespace vog {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cmul_conj(cx<T> a, cx<T> b) {  // a * conj(b)
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// Pass structure shared by the kernels and the host table builder.
constexpr int fft_regs(int n) { return n < 16 ? n : 16; }
constexpr int fft_npass(int n) { return (ilog2(n) + 3) / 4; }
constexpr int fft_radix(int n, int p) {
    return p == fft_npass(n) - 1 ? n / ipow(16, fft_npass(n) - 1) : 16;
}
constexpr int fft_ns(int p) { return ipow(16, p); }
// Offset (in complex entries) of the twiddle rows of pass p (p >= 1).
constexpr int fft_tw_off(int n, int p) { return p <= 1 ? 0 : fft_tw_off(n, p - 1) + 16 * fft_ns(p - 1); }
constexpr int fft_tw_total(int n) { return fft_npass(n) <= 1 ? 16 : fft_tw_off(n, fft_npass(n)); }
constexpr int kEpsRow = 10;  // entries per thread row of the symbol table (q = 0 .. 9)

// cos(2 pi j / 16), j = 0..15; sin(2 pi j / 16) = cos(2 pi (j - 4) / 16).
constexpr double kCos16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};

// a * exp(DIR * 2 pi i K / R) for a compile-time K and R dividing 16.
template <typename T, int DIR, int K, int R>
__device__ __forceinline__ cx<T> twc(cx<T> a) {
    constexpr int j = (((K % R) + R) % R) * (16 / R);
    if constexpr (j == 0) {
        return a;
    } else if constexpr (j == 8) {
        return {-a.re, -a.im};
    } else if constexpr (j == 4) {  // exp(DIR i pi/2) = DIR i
        if constexpr (DIR > 0) return {-a.im, a.re};
        else return {a.im, -a.re};
    } else if constexpr (j == 12) {  // exp(DIR i 3pi/2) = -DIR i
        if constexpr (DIR > 0) return {a.im, -a.re};
        else return {-a.im, a.re};
    } else {
        constexpr T c = (T)kCos16[j];
        constexpr T s = (T)(DIR * kCos16[(j + 12) % 16]);
        return {a.re * c - a.im * s, a.re * s + a.im * c};
    }
}

// In-register DFT of length R (2, 4, 8 or 16), natural order in and out:
// v[k] <- sum_n v[n] exp(DIR 2 pi i n k / R).
template <typename T, int DIR, int R>
__device__ __forceinline__ void dft(cx<T> *v) {
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 2) {
        cx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    } else if constexpr (R == 4) {
        cx<T> a0 = v[0] + v[2], a1 = v[0] - v[2], a2 = v[1] + v[3];
        cx<T> a3 = twc<T, DIR, 1, 4>(v[1] - v[3]);
        v[0] = a0 + a2;
        v[2] = a0 - a2;
        v[1] = a1 + a3;
        v[3] = a1 - a3;
    } else {
        constexpr int H = R / 2;
        cx<T> e[H], o[H];
        static_for<0, H>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            e[k] = v[2 * k];
            o[k] = v[2 * k + 1];
        });
        dft<T, DIR, H>(e);
        dft<T, DIR, H>(o);
        static_for<0, H>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            cx<T> tt = twc<T, DIR, k, R>(o[k]);
            v[k] = e[k] + tt;
            v[k + H] = e[k] - tt;
        });
    }
}

// Returns p unchanged but opaque to the optimiser: loads through the result
// cannot be merged with, or hoisted above, loads through p.
template <typename P>
__device__ __forceinline__ P opaque(P p) {
    asm volatile("" : "+v"(p));
    return p;
}

// Loads entries [0, n) of a table row (n even, row 16-byte aligned).  The
// tables live in global memory: the loads are global ones (a flat load would
// also count as an LDS access).
template <typename T, int NE>
__device__ __forceinline__ void load_row(const cx<T> *__restrict__ row, cx<T> (&out)[NE]) {
    if constexpr (sizeof(T) == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        typedef __attribute__((address_space(1))) const f4 gf4;
        gf4 *p = (gf4 *)row;
        static_for<0, NE / 2>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const f4 q = p[i];
            out[2 * i] = cx<T>{q.x, q.y};
            out[2 * i + 1] = cx<T>{q.z, q.w};
        });
    } else {
        typedef T d2 __attribute__((ext_vector_type(2)));
        typedef __attribute__((address_space(1))) const d2 gd2;
        gd2 *p = (gd2 *)row;
        static_for<0, NE>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const d2 q = p[i];
            out[i] = cx<T>{q.x, q.y};
        });
    }
}

// Synchronisation of the threads of one transform around an LDS exchange.
// WAVE: they are contiguous lanes of a single wave, which executes its LDS
// operations in order, so ordering the wave's own accesses is enough;
// otherwise the whole block waits.
template <bool WAVE>
__device__ __forceinline__ void xsync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <typename T, int N>
struct Fft {
    static_assert(N >= 8 && N <= 4096 && (N & (N - 1)) == 0, "N must be a power of two in [8, 4096]");
    static constexpr int R = fft_regs(N);
    static constexpr int TPF = N / R;
    static constexpr int NPASS = fft_npass(N);
    static constexpr int LAST = fft_radix(N, NPASS - 1);
    static constexpr int LDSN = N + N / 16;  // padded SoA length

    static constexpr int radix(int p) { return fft_radix(N, p); }
    static constexpr int ns(int p) { return fft_ns(p); }
    // frequency index (in units of TPF, offset t) held by register i after the last pass
    static constexpr int kpos(int i) { return i / LAST + (i % LAST) * (R / LAST); }
    static constexpr int kinv(int k) {  // register index holding position k
        for (int i = 0; i < R; ++i)
            if (kpos(i) == k) return i;
        return -1;
    }
    static __device__ __forceinline__ int pad(int i) { return i + (i >> 4); }
    // pad(x + C) given px = pad(x), for a compile-time C that is a multiple of 16
    // (or any C when the caller knows x + C stays inside x's 16-block).
    template <int C>
    static __device__ __forceinline__ int pad_add(int px) { return px + C + C / 16; }

    // One radix pass on registers (twiddles, then DFT of each group).
    template <int DIR, int P>
    static __device__ __forceinline__ void pass(cx<T> (&v)[R], int t, const cx<T> *__restrict__ tw) {
        constexpr int RP = radix(P), NS = ns(P);
        static_for<0, R / RP>([&](auto uc) {
            constexpr int u = decltype(uc)::value;
            if constexpr (NS > 1) {
                const int k = (t + u * TPF) & (NS - 1);
                cx<T> w[RP];
                load_row<T, RP>(tw + fft_tw_off(N, P) + 16 * k, w);
                static_for<1, RP>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    if constexpr (DIR > 0) v[u * RP + r] = cmul(v[u * RP + r], w[r]);
                    else v[u * RP + r] = cmul_conj(v[u * RP + r], w[r]);
                });
            }
            dft<T, DIR, RP>(&v[u * RP]);
        });
    }

    // Stockham exchange after pass P: store in autosort order, reload in the
    // layout of pass P + 1.  All threads of the block must call it (WAVE: all
    // threads of the wave; see xsync).
    template <int P, bool WAVE = false>
    static __device__ __forceinline__ void exchange(cx<T> (&v)[R], int t, T *lre, T *lim) {
        constexpr int RP = radix(P), NS = ns(P), RQ = radix(P + 1);
        xsync<WAVE>();
        static_for<0, R / RP>([&](auto uc) {
            constexpr int u = decltype(uc)::value;
            const int jb = t + u * TPF;
            const int k = jb & (NS - 1);
            // base = (jb / NS) * NS * RP + k; element r sits at base + r * NS.
            // NS == 1: base = 16 jb, pad(base + r) = 17 jb + r.
            // NS >= 16: pad(base + r NS) = pad(base) + 17 r NS / 16.
            const int pb = pad((jb - k) * RP + k);
            static_for<0, RP>([&](auto rc) {
                constexpr int r = decltype(rc)::value;
                const int idx = pb + r * NS + (r * NS) / 16;
                lre[idx] = v[u * RP + r].re;
                lim[idx] = v[u * RP + r].im;
            });
        });
        xsync<WAVE>();
        const int pt = pad(t);
        static_for<0, R / RQ>([&](auto uc) {
            constexpr int u = decltype(uc)::value;
            static_for<0, RQ>([&](auto rc) {
                constexpr int r = decltype(rc)::value;
                constexpr int C = u * TPF + r * (N / RQ);
                int idx;
                if constexpr (TPF % 16 == 0) idx = pad_add<C>(pt);
                else idx = pad(t + C);
                v[u * RQ + r] = cx<T>{lre[idx], lim[idx]};
            });
        });
    }

    // Full transform: X_m = sum_n x_n exp(DIR 2 pi i n m / N), unnormalised.
    template <int DIR, bool WAVE = false>
    static __device__ __forceinline__ void run(cx<T> (&v)[R], int t, T *lre, T *lim,
                                               const cx<T> *__restrict__ tw) {
        static_for<0, NPASS>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            pass<DIR, p>(v, t, tw);
            if constexpr (p + 1 < NPASS) exchange<p, WAVE>(v, t, lre, lim);
        });
    }

    // Two independent transforms of the same length side by side: each pass
    // reads its twiddle rows once for both, and each exchange moves both
    // between one pair of barriers (v through lre/lim, u through lre2/lim2).
    // Per value the arithmetic is that of run().
    template <int DIR, bool WAVE = false>
    static __device__ __forceinline__ void run2(cx<T> (&v)[R], cx<T> (&u)[R], int t, T *lre, T *lim, T *lre2,
                                                T *lim2, const cx<T> *__restrict__ tw) {
        static_for<0, NPASS>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int RP = radix(p), NS = ns(p);
            static_for<0, R / RP>([&](auto uc) {
                constexpr int g = decltype(uc)::value;
                if constexpr (NS > 1) {
                    const int k = (t + g * TPF) & (NS - 1);
                    cx<T> w[RP];
                    load_row<T, RP>(tw + fft_tw_off(N, p) + 16 * k, w);
                    static_for<1, RP>([&](auto rc) {
                        constexpr int r = decltype(rc)::value;
                        if constexpr (DIR > 0) {
                            v[g * RP + r] = cmul(v[g * RP + r], w[r]);
                            u[g * RP + r] = cmul(u[g * RP + r], w[r]);
                        } else {
                            v[g * RP + r] = cmul_conj(v[g * RP + r], w[r]);
                            u[g * RP + r] = cmul_conj(u[g * RP + r], w[r]);
                        }
                    });
                }
                dft<T, DIR, RP>(&v[g * RP]);
                dft<T, DIR, RP>(&u[g * RP]);
            });
            if constexpr (p + 1 < NPASS) {
                constexpr int RQ = radix(p + 1);
                xsync<WAVE>();
                static_for<0, R / RP>([&](auto uc) {
                    constexpr int g = decltype(uc)::value;
                    const int jb = t + g * TPF;
                    const int k = jb & (NS - 1);
                    const int pb = pad((jb - k) * RP + k);
                    static_for<0, RP>([&](auto rc) {
                        constexpr int r = decltype(rc)::value;
                        const int idx = pb + r * NS + (r * NS) / 16;
                        lre[idx] = v[g * RP + r].re;
                        lim[idx] = v[g * RP + r].im;
                        lre2[idx] = u[g * RP + r].re;
                        lim2[idx] = u[g * RP + r].im;
                    });
                });
                xsync<WAVE>();
                const int pt = pad(t);
                static_for<0, R / RQ>([&](auto uc) {
                    constexpr int g = decltype(uc)::value;
                    static_for<0, RQ>([&](auto rc) {
                        constexpr int r = decltype(rc)::value;
                        constexpr int C = g * TPF + r * (N / RQ);
                        int idx;
                        if constexpr (TPF % 16 == 0) idx = pad_add<C>(pt);
                        else idx = pad(t + C);
                        v[g * RQ + r] = cx<T>{lre[idx], lim[idx]};
                        u[g * RQ + r] = cx<T>{lre2[idx], lim2[idx]};
                    });
                });
            }
        });
    }

    // The twiddles every pass of thread t uses, held in registers: pass p
    // (p >= 1) group u takes row (t + u TPF) mod NS(p), entries 0 .. RP-1, at
    // w[p - 1][u RP ..].  The same rows serve both directions (forward
    // passes multiply by their conjugates).  For kernels that run few blocks,
    // where a table load inside each pass would be waited for in full.
    struct Rows {
        cx<T> w[NPASS > 1 ? NPASS - 1 : 1][R];
    };
    static __device__ __forceinline__ void load_rows(int t, const cx<T> *__restrict__ tw, Rows &rw) {
        static_for<1, NPASS>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int RP = radix(p), NS = ns(p);
            static_for<0, R / RP>([&](auto uc) {
                constexpr int u = decltype(uc)::value;
                const int k = (t + u * TPF) & (NS - 1);
                cx<T> w[RP];
                load_row<T, RP>(tw + fft_tw_off(N, p) + 16 * k, w);
                static_for<0, RP>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    rw.w[p - 1][u * RP + r] = w[r];
                });
            });
        });
    }
    // The same rows from the exact table entries r = 1, 2, 3 and 4, 8, 12
    // only: entry r = 4a + b (a, b > 0) is formed as entry 4a times entry b,
    // one rounding from two rounded factors.  6 of every 16 entries are
    // read; for kernels whose time goes to fetching the table.
    static __device__ __forceinline__ void load_rows_sparse(int t, const cx<T> *__restrict__ tw, Rows &rw) {
        typedef T v2 __attribute__((ext_vector_type(2)));
        typedef __attribute__((address_space(1))) const v2 gv2;
        static_for<1, NPASS>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int RP = radix(p), NS = ns(p);
            static_for<0, R / RP>([&](auto uc) {
                constexpr int u = decltype(uc)::value;
                const int k = (t + u * TPF) & (NS - 1);
                gv2 *row = (gv2 *)(tw + fft_tw_off(N, p) + 16 * k);
                cx<T> *w = &rw.w[p - 1][u * RP];
                w[0] = cx<T>{(T)1, (T)0};
                static_for<1, RP>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    if constexpr (r < 4 || r % 4 == 0) {
                        const v2 q = row[r];
                        w[r] = cx<T>{q.x, q.y};
                    }
                });
                static_for<5, RP>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    if constexpr (r % 4 != 0) w[r] = cmul(w[r - r % 4], w[r % 4]);
                });
            });
        });
    }

    template <int DIR>
    static __device__ __forceinline__ void run(cx<T> (&v)[R], int t, T *lre, T *lim, const Rows &rw) {
        static_for<0, NPASS>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int RP = radix(p);
            static_for<0, R / RP>([&](auto uc) {
                constexpr int u = decltype(uc)::value;
                if constexpr (p > 0) {
                    static_for<1, RP>([&](auto rc) {
                        constexpr int r = decltype(rc)::value;
                        const cx<T> w = rw.w[p - 1][u * RP + r];
                        if constexpr (DIR > 0) v[u * RP + r] = cmul(v[u * RP + r], w);
                        else v[u * RP + r] = cmul_conj(v[u * RP + r], w);
                    });
                }
                dft<T, DIR, RP>(&v[u * RP]);
            });
            if constexpr (p + 1 < NPASS) exchange<p>(v, t, lre, lim);
        });
    }
};

}  // namespace vog
