#pragma once
// Packed transform of a pair of 4096-point real lines (z = uA + i uB) by the
// 256 threads of four waves, in three radix-16 digit passes:
//
//   n = 256 n1 + t,  t = 16 ta + tb;     m = k1 + 16 k2a + 256 k2b,
//   X_m = sum_tb W16^{tb k2b} W256^{tb k2a} sum_ta W16^{ta k2a}
//           [ W4096^{t k1} sum_n1 W16^{n1 k1} z_n ],     W_L = exp(-2 pi i / L).
//
// Column phase: thread t holds z[t + 256 r] (r = 0..15), runs the n1 digit
// and the twiddle W4096^{t k1}, and writes its 16 values to LDS slot
// slot(k1), column t.  One block barrier.  Lane phase: wave w owns the four
// slots 4w .. 4w+3; lane (s, x) (s = lane / 16, x = lane % 16) of slot
// 4w + s runs the ta digit, an exchange among the 16 lanes of its slot, the
// tb digit, and ends holding X at m0 + 256 k2b, m0 = k1 + 16 x.  The k1 of a
// wave's slots are closed under k1 -> -k1 (mod 16), so the Hermitian partner
// N - m of every mode is in the same wave and reaches it with ds_bpermute.
// The symbol product, the inverse tb and ta digits and the write back to the
// slots follow in the same wave.  One block barrier.  Column phase: thread t
// reads its column, applies W4096^{-t k1} and runs the k1 digit, ending with
// y[t + 256 n1] in register n1.  Only two block barriers per line pair; the
// in-wave exchanges need no barrier (a wave runs its LDS operations in
// order).
//
// Symbol (Section 1.2): with the pair's combined weights c_q = (wP_q + i wQ_q)
// / 2, wP = (wA + wB) / (2N), wQ = (wA - wB) / (2N), one length-16 DFT per
// lane gives C_m = sum_q c_q exp(2 pi i m q / N) at its 16 modes
// (C_{m0 + 256 k} = DFT16+(H)[k], H_c = sum_{q = c mod 16} c_q exp(2 pi i m0 q / N)).
// With the partner's C_{N-m}: P_m = C_m + conj(C_{N-m}) and
// i Q_m = C_m - conj(C_{N-m}) are the symbols of wP and wQ, and
// Y_m = P_m Z_m + Q_m conj(Z_{N-m}) is (kernel A applied to uA) + i (kernel B
// applied to uB) in Fourier space.
//
// Twiddle tables are those of the radix-16 Stockham FFT of fft.hpp:
//   tw + 16 k,        k < 16:  exp(+2 pi i r k / 256),  r = 0..15
//   tw + 256 + 16 k,  k < 256: exp(+2 pi i r k / 4096), r = 0..15.

#include "addr.hpp"
#include "fft.hpp"

namespace vog {

template <typename T>
struct P4k {
    static constexpr int N = 4096;
    static constexpr int SP = 272;  // slot pitch: 256 columns + 16 (slots start 16 banks apart)
    static constexpr int REGION = 2 * 16 * SP;  // LDS values per line pair: re[16][SP], im[16][SP]
    // k1 held by slot s (four bits each).  Slots 2j, 2j+1 hold k1 and -k1,
    // except slots 0 and 1 (k1 = 0 and 8, each its own negative).
    //   slots:  0  1  2  3 | 4  5  6  7 | 8  9 10 11 | 12 13 14 15
    //   k1:     0  8  4 12 | 1 15  2 14 | 3 13  5 11 |  6 10  7  9
    static constexpr uint64_t kK1 = 0x97A6B5D3E2F1C480ull;
    static constexpr int k1_of(int s) { return (int)((kK1 >> (4 * s)) & 15); }
    static constexpr int slot_of(int k1) {
        for (int s = 0; s < 16; ++s)
            if (k1_of(s) == k1) return s;
        return -1;
    }
};
static_assert(P4k<float>::k1_of(0) == 0 && P4k<float>::k1_of(1) == 8 && P4k<float>::k1_of(2) == 4 &&
                  P4k<float>::k1_of(3) == 12 && P4k<float>::k1_of(4) == 1 && P4k<float>::k1_of(5) == 15 &&
                  P4k<float>::k1_of(15) == 9,
              "slot table");

// A value the same in every lane, moved to scalar registers.
template <typename T>
__device__ __forceinline__ T uniform_t(T x) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, x);
        return __builtin_bit_cast(T, addr_join(__builtin_amdgcn_readfirstlane(addr_lo(u)),
                                               __builtin_amdgcn_readfirstlane(addr_hi(u))));
    }
}

// Cross-lane read within the wave: value x of lane (addr / 4).
template <typename T>
__device__ __forceinline__ T bperm(int addr, T x) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, x)));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, x);
        return __builtin_bit_cast(T, addr_join(__builtin_amdgcn_ds_bpermute(addr, addr_lo(u)),
                                               __builtin_amdgcn_ds_bpermute(addr, addr_hi(u))));
    }
}

// Twiddle row of column t: exp(+2 pi i t k / 4096), k = 0..15.
template <typename T>
__device__ __forceinline__ void p4k_col_row(const cx<T> *__restrict__ tw, int t, cx<T> (&w)[16]) {
    load_row<T, 16>(tw + 256 + 16 * t, w);
}

// Forward column phase: on entry v[r] = z[t + 256 r]; the n1 digit, the
// twiddle W4096^{t k1} (w: the row of column t), then value k1 to slot(k1),
// column t.
template <typename T>
__device__ __forceinline__ void p4k_fwd_col(cx<T> (&v)[16], int t, T *lre, T *lim, const cx<T> (&w)[16]) {
    using P = P4k<T>;
    dft<T, -1, 16>(v);
    static_for<1, 16>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        v[k] = cmul_conj(v[k], w[k]);
    });
    static_for<0, 16>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int s = P::slot_of(k);
        lre[s * P::SP + t] = v[k].re;
        lim[s * P::SP + t] = v[k].im;
    });
}

// Inverse column phase: reads column t of every slot, applies W4096^{-t k1}
// (w: the row of column t) and the k1 digit; on exit v[n1] = y[t + 256 n1].
template <typename T>
__device__ __forceinline__ void p4k_inv_col(cx<T> (&v)[16], int t, const T *lre, const T *lim,
                                            const cx<T> (&w)[16]) {
    using P = P4k<T>;
    static_for<0, 16>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int s = P::slot_of(k);
        v[k] = cx<T>{lre[s * P::SP + t], lim[s * P::SP + t]};
    });
    static_for<1, 16>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        v[k] = cmul(v[k], w[k]);
    });
    dft<T, 1, 16>(v);
}

// The lane phase's table rows, read where they are used (`again`: re-read
// instead of kept live).
template <typename T>
struct LoadRows {
    const cx<T> *tw, *eps;
    __device__ void row256(int x, cx<T> (&r)[16], bool again) const {
        load_row<T, 16>((again ? opaque(tw) : tw) + 16 * x, r);  // exp(2 pi i x k / 256)
    }
    __device__ void epsrow(int m0, cx<T> (&e)[kEpsRow]) const { load_row<T, kEpsRow>(eps + m0 * kEpsRow, e); }
};

// Lane phase of wave w (0..3), lane l (0..63), between the two block
// barriers.  rows: the twiddle row exp(2 pi i x k / 256) of the lane's digit
// x and the symbol row exp(2 pi i m0 q / N), q = 0..9, of its m0 (LoadRows).
// wpq: the pair's 18 values wP_q / 2 then 18 values wQ_q / 2 (q = -8..9),
// the same in every lane.  iden: 1 / collocation symbol of the B-spline per
// mode, or null.
template <typename T, typename Rows>
__device__ __forceinline__ void p4k_lanes(int w, int l, T *lre, T *lim, const Rows &rows, const T *wpq,
                                          const T *__restrict__ iden) {
    using P = P4k<T>;
    const int sp = l >> 4, x = l & 15;
    const int s = 4 * w + sp;
    const int k1 = (int)((P::kK1 >> (4 * s)) & 15);
    T *sre = lre + s * P::SP;
    T *sim = lim + s * P::SP;

    // ta digit: v[ta] = value (k1, t = 16 ta + x)
    cx<T> v[16];
    static_for<0, 16>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        v[i] = cx<T>{sre[16 * i + x], sim[16 * i + x]};
    });
    dft<T, -1, 16>(v);
    {
        cx<T> r[16];
        rows.row256(x, r, false);  // exp(2 pi i x k2a / 256)
        static_for<1, 16>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            v[k] = cmul_conj(v[k], r[k]);
        });
    }
    // exchange within the slot's 16 lanes: lane tb's value k2a to lane k2a
    xsync<true>();
    static_for<0, 16>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        sre[17 * x + k] = v[k].re;
        sim[17 * x + k] = v[k].im;
    });
    xsync<true>();
    static_for<0, 16>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        v[i] = cx<T>{sre[17 * i + x], sim[17 * i + x]};
    });
    dft<T, -1, 16>(v);  // v[k2b] = X[m0 + 256 k2b]
    const int m0 = k1 + 16 * x;

    // symbol C at the lane's modes
    cx<T> C[16];
    {
        cx<T> e[kEpsRow];
        rows.epsrow(m0, e);
        static_for<0, 16>([&](auto cc) { C[decltype(cc)::value] = cx<T>{(T)0, (T)0}; });
        static_for<0, kTaps>([&](auto qc) {
            constexpr int qi = decltype(qc)::value;
            constexpr int q = qi - kDMax;
            constexpr int c = q & 15;
            constexpr int aq = q < 0 ? -q : q;
            // the pair's weights, the same in every lane: scalar registers
            const T a = uniform_t<T>(wpq[qi]), b = uniform_t<T>(wpq[kTaps + qi]);
            if constexpr (q == 0) {
                C[c].re += a;
                C[c].im += b;
            } else if constexpr (q > 0) {  // (a + i b)(e.re + i e.im)
                C[c].re = fma_t<T>(a, e[aq].re, fma_t<T>(-b, e[aq].im, C[c].re));
                C[c].im = fma_t<T>(a, e[aq].im, fma_t<T>(b, e[aq].re, C[c].im));
            } else {  // (a + i b)(e.re - i e.im)
                C[c].re = fma_t<T>(a, e[aq].re, fma_t<T>(b, e[aq].im, C[c].re));
                C[c].im = fma_t<T>(-a, e[aq].im, fma_t<T>(b, e[aq].re, C[c].im));
            }
        });
        dft<T, 1, 16>(C);
    }

    // Hermitian partner: mode N - (m0 + 256 k) = m0' + 256 (15 - k) with
    // m0' = 256 - m0 in lane (slot of -k1, x'), x' = 15 - x (k1 != 0) or
    // (16 - x) mod 16 (k1 = 0).  Slot pairs differ in bit 0, except slots 0, 1.
    const int sq = (s < 2) ? sp : (sp ^ 1);
    const int xq = (k1 == 0) ? ((16 - x) & 15) : (15 - x);
    const int pa = (16 * sq + xq) * 4;
    // Modes k and 15 - k are done together: both partner values are fetched
    // before either register is overwritten.  The lane with m0 = 0 (wave 0
    // only) pairs k with (16 - k) mod 16 inside itself; it parks its X and C
    // in its slot (whose exchange data is consumed) and reads them back.
    auto ymode = [&](const cx<T> &c, const cx<T> &cp, const cx<T> &z, const cx<T> &zp) {
        const cx<T> Pm{c.re + cp.re, c.im - cp.im};
        const cx<T> Qm{c.im + cp.im, cp.re - c.re};  // (C - conj Cp) / i
        T yr = Pm.re * z.re;
        yr = fma_t<T>(-Pm.im, z.im, yr);
        yr = fma_t<T>(Qm.re, zp.re, yr);
        yr = fma_t<T>(Qm.im, zp.im, yr);
        T yi = Pm.re * z.im;
        yi = fma_t<T>(Pm.im, z.re, yi);
        yi = fma_t<T>(Qm.im, zp.re, yi);
        yi = fma_t<T>(-Qm.re, zp.im, yi);
        return cx<T>{yr, yi};
    };
    auto product = [&](auto zc) {
        constexpr bool ZERO = decltype(zc)::value;
        const bool self0 = ZERO && m0 == 0;
        if constexpr (ZERO) {
            if (self0) {
                static_for<0, 16>([&](auto kc) {
                    constexpr int k = decltype(kc)::value;
                    sre[k] = v[k].re;
                    sim[k] = v[k].im;
                    sre[16 + k] = C[k].re;
                    sim[16 + k] = C[k].im;
                });
            }
        }
        static_for<0, 8>([&](auto jc) {
            constexpr int a = decltype(jc)::value, b = 15 - a;
            // two pairs of modes in flight at a time (register pressure)
            if constexpr (a % 2 == 0) __builtin_amdgcn_sched_barrier(0);
            cx<T> zpa{bperm<T>(pa, v[b].re), bperm<T>(pa, v[b].im)};
            cx<T> zpb{bperm<T>(pa, v[a].re), bperm<T>(pa, v[a].im)};
            cx<T> cpa{bperm<T>(pa, C[b].re), bperm<T>(pa, C[b].im)};
            cx<T> cpb{bperm<T>(pa, C[a].re), bperm<T>(pa, C[a].im)};
            if constexpr (ZERO) {
                if (self0) {
                    constexpr int ia = (16 - a) & 15, ib = (16 - b) & 15;
                    zpa = cx<T>{sre[ia], sim[ia]};
                    zpb = cx<T>{sre[ib], sim[ib]};
                    cpa = cx<T>{sre[16 + ia], sim[16 + ia]};
                    cpb = cx<T>{sre[16 + ib], sim[16 + ib]};
                }
            }
            v[a] = ymode(C[a], cpa, v[a], zpa);
            v[b] = ymode(C[b], cpb, v[b], zpb);
        });
    };
    if (__builtin_amdgcn_readfirstlane(w) == 0) product(std::true_type{});
    else product(std::false_type{});
    if (iden) {
        // (through a descriptor: one lane offset, the mode stride as a constant)
        const __amdgpu_buffer_rsrc_t ri = buf_rsrc(iden, (unsigned)(P::N * sizeof(T)));
        static_for<0, 16>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const T sc = buf_load<T>(ri, (unsigned)m0 * sizeof(T), (unsigned)(256 * k * sizeof(T)));
            v[k].re *= sc;
            v[k].im *= sc;
        });
    }

    // inverse tb digit: v[tb] for the lane's (k1, k2a = x), twiddle exp(2 pi i tb x / 256)
    dft<T, 1, 16>(v);
    {
        cx<T> r[16];
        rows.row256(x, r, true);
        static_for<1, 16>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            v[k] = cmul(v[k], r[k]);
        });
    }
    // exchange within the slot: lane k2a's value tb to lane tb
    xsync<true>();
    static_for<0, 16>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        sre[17 * x + k] = v[k].re;
        sim[17 * x + k] = v[k].im;
    });
    xsync<true>();
    static_for<0, 16>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        v[i] = cx<T>{sre[17 * i + x], sim[17 * i + x]};
    });
    dft<T, 1, 16>(v);  // v[ta]: value (k1, t = 16 ta + x)
    xsync<true>();
    static_for<0, 16>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        sre[16 * i + x] = v[i].re;
        sim[16 * i + x] = v[i].im;
    });
}

}  // namespace vog
