// Host runtime of libvog: configuration checks, workspace layout, FP64
// tables, the stream-ordered step driver with grouped launches, readout,
// checkpointing and kernel timing.  Implements include/vog.h.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fft.hpp"
#include "vog_internal.hpp"

using namespace vog;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(VOG_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// exp(i pi k / n) for k < 2n, FP64, with the angle reduced to the first
// octant so that symmetric entries are exact mirrors of each other.
void unit_roots(int n, std::vector<double> &re, std::vector<double> &im) {
    const int m = 2 * n;  // period
    re.resize(m);
    im.resize(m);
    for (int k = 0; k < m; ++k) {
        // angle = 2 pi k / m; use k mod m in eighths of a turn
        long long num = (long long)k * 8;  // angle in units of (2 pi / 8) is num / m
        int oct = (int)(num / m);
        long long rem = num % m;  // within octant, fraction rem / m of pi/4
        // reflect to first octant
        double a;
        int o = oct;
        if (o % 2 == 0) a = (M_PI / 4.0) * ((double)rem / m);
        else a = (M_PI / 4.0) * ((double)(m - rem) / m);
        double c = cos(a), s = sin(a);
        double x, y;
        switch (o) {
            case 0: x = c; y = s; break;
            case 1: x = s; y = c; break;
            case 2: x = -s; y = c; break;
            case 3: x = -c; y = s; break;
            case 4: x = -c; y = -s; break;
            case 5: x = -s; y = -c; break;
            case 6: x = s; y = -c; break;
            default: x = c; y = -s; break;
        }
        re[k] = x;
        im[k] = y;
    }
}

struct Layout {
    size_t f, g, E, Eeff, part, rho, mom, tw_x, tw_v, eps_x, eps_v, tw_x64, invk, iden_x, iden_v,
        feq_g, feq64, drv_sc, ring, dev, total;
};

bool prec_fp64(const vog_config &c) {
    return c.precision == VOG_FP64_PLAIN || c.precision == VOG_FP64_DELTAF;
}

bool prec_deltaf(const vog_config &c) {
    return c.precision == VOG_FP32_DELTAF || c.precision == VOG_FP64_DELTAF;
}

// B^k(j) at the integers j = 0 .. k+1 of the uniform B-spline of degree k
// on [0, k+1), from the degree recurrence B^p(x) = x/p B^{p-1}(x) +
// (p+1-x)/p B^{p-1}(x-1) (Section 1.2), FP64.
std::vector<double> bspline_at_integers(int k) {
    std::vector<double> b(k + 2, 0.0), nb(k + 2, 0.0);
    b[0] = 1.0;  // B^0 is the indicator of [0, 1): B^0(j) = [j == 0]
    for (int p = 1; p <= k; ++p) {
        for (int j = 0; j <= k + 1; ++j) {
            const double x = (double)j;
            nb[j] = x / p * b[j] + (j > 0 ? (p + 1 - x) / p * b[j - 1] : 0.0);
        }
        b.swap(nb);
    }
    return b;
}

// 1 / D_m, m < n, for B-spline interpolation of degree k = 2d+1 on n nodes:
// the collocation circulant has the symbol e^{-i theta (d+1)} D_m with
// D_m = sum_{j=1..k} B^k(j) cos(theta_m (j - d - 1)), theta_m = 2 pi m / n,
// which is real and positive for odd k.  The sweep multiplies the packed
// product by 1 / D_m; the phase e^{i theta (d+1)} is folded into the taps
// w_q = B^k(d + 1 - q + s), q = -d .. d+1.
std::vector<double> bspline_inverse_symbol(int n, int k) {
    const int d = (k - 1) / 2;
    const std::vector<double> bj = bspline_at_integers(k);
    std::vector<double> re, im;
    unit_roots(n, re, im);  // exp(i pi l / n), l < 2n
    std::vector<double> out(n);
    for (int m = 0; m < n; ++m) {
        double acc = 0.0;
        for (int j = 1; j <= k; ++j) {
            const long long a = (long long)m * (j - d - 1);
            const long long r = ((a % n) + n) % n;
            acc += bj[j] * re[2 * r];
        }
        out[m] = 1.0 / acc;
    }
    return out;
}

// How the x-sweep reaches the x-lines of the v-fastest array f[nx][nv]:
// tiles of whole x-lines staged through LDS when a tile fits the grid,
// otherwise a transposed copy.
enum XMode { X_TRANSPOSED = 0, X_TILED = 1 };

XMode xsweep_mode(const vog_config &c) {
    const int B = fused_lines_per_block(prec_fp64(c), c.nx);
    return (B > 0 && c.nv >= B) ? X_TILED : X_TRANSPOSED;
}

bool uses_fused_xsweep(const vog_config &c) { return xsweep_mode(c) != X_TRANSPOSED; }

// Rows of velocity partial sums feeding rho: one per tile of the x-sweep on
// the v-fastest layout, one per 64 velocities of the x -> v transpose.
int rho_parts(const vog_config &c) {
    return uses_fused_xsweep(c) ? c.nv / fused_lines_per_block(prec_fp64(c), c.nx)
                                : (c.nv + kTile - 1) / kTile;
}

Layout layout_of(const vog_config &c) {
    const size_t es = prec_fp64(c) ? 8 : 4;
    const size_t cells = (size_t)c.nx * c.nv;
    const bool spline = c.interp == VOG_INTERP_BSPLINE;
    const int nparts = rho_parts(c);
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    L.f = take(cells * es);
    L.g = take(uses_fused_xsweep(c) ? 0 : cells * es);
    L.E = take(sizeof(double) * c.nx);
    L.Eeff = take(sizeof(double) * c.nx);
    L.part = take(sizeof(double) * c.nx * (size_t)nparts);
    L.rho = take(sizeof(double) * c.nx);
    L.mom = take(sizeof(double) * 2 * c.nx);
    L.tw_x = take(2 * es * fft_tw_total(c.nx));
    L.tw_v = take(2 * es * fft_tw_total(c.nv));
    L.eps_x = take(2 * es * kEpsRow * (c.nx / fft_regs(c.nx)));
    L.eps_v = take(2 * es * kEpsRow * (c.nv / fft_regs(c.nv)));
    L.tw_x64 = take(2 * sizeof(double) * fft_tw_total(c.nx));
    L.invk = take(sizeof(double) * c.nx);
    L.iden_x = take(spline ? es * c.nx : 0);
    L.iden_v = take(spline ? es * c.nv : 0);
    L.feq_g = take(es * VOG_MAX_FEQ * c.nv);
    L.feq64 = take(sizeof(double) * c.nv);
    L.drv_sc = take(c.drive_emax != 0.0 ? 2 * sizeof(double) * c.nx : 0);
    L.ring = take(sizeof(vog_diag) * kRingCap);
    L.dev = take(sizeof(SimDev));
    L.total = off;
    return L;
}

struct EventPair {
    hipEvent_t a, b;
};

}  // namespace

struct vog_sim {
    vog_config cfg;
    Layout lay;
    hipStream_t stream;
    int device;
    bool owns;
    char *ws;
    SimDev host_dev;       // host copy of the device constants
    const SimDev *dev;     // device address
    std::vector<double> feq64;  // f_eq(v_j), FP64
    // Host copies of the tables uploaded by vog_create, kept until the copies
    // are known to be done (the next synchronisation), so that creating a sim
    // does not wait for work already queued on the stream.
    std::deque<std::vector<char>> staging;
    int64_t step;
    double t;
    int64_t diag_read;     // records consumed by vog_get_diag
    bool fp64;
    bool fused;            // x-sweep directly on the v-fastest layout
    int xmode;             // XMode
    // profiling
    bool prof;
    std::vector<EventPair> ev[VOG_NUM_KINDS];
    size_t ev_used[VOG_NUM_KINDS];
    double ms[VOG_NUM_KINDS];
    int64_t launches[VOG_NUM_KINDS];
};

namespace {

int validate(const vog_config *c) {
    if (!c) return fail(VOG_EINVAL, "config is NULL");
    if (!is_pow2(c->nx) || c->nx < VOG_MIN_N || c->nx > VOG_MAX_N)
        return fail(VOG_EINVAL, "nx must be a power of two in [8, 4096]");
    if (!is_pow2(c->nv) || c->nv < VOG_MIN_N || c->nv > VOG_MAX_N)
        return fail(VOG_EINVAL, "nv must be a power of two in [8, 4096]");
    if (!(c->L > 0.0) || !isfinite(c->L)) return fail(VOG_EINVAL, "L must be finite and > 0");
    if (!(c->vmin < c->vmax) || !isfinite(c->vmin) || !isfinite(c->vmax))
        return fail(VOG_EINVAL, "need finite vmin < vmax");
    if (c->degree < 1 || c->degree > VOG_MAX_DEGREE || c->degree % 2 == 0)
        return fail(VOG_EINVAL, "degree must be odd in [1, 17]");
    if (c->degree > c->nx - 1 || c->degree > c->nv - 1)
        return fail(VOG_EINVAL, "degree must be <= min(nx, nv) - 1");
    if (c->precision != VOG_FP64_PLAIN && c->precision != VOG_FP32_DELTAF &&
        c->precision != VOG_FP64_DELTAF && c->precision != VOG_FP32_PLAIN)
        return fail(VOG_EINVAL, "unknown precision");
    if (c->interp != VOG_INTERP_LAGRANGE && c->interp != VOG_INTERP_BSPLINE)
        return fail(VOG_EINVAL, "unknown interpolation");
    if (c->merge_v != 0 && c->merge_v != 1) return fail(VOG_EINVAL, "merge_v must be 0 or 1");
    if (c->bitwise_steps != 0 && c->bitwise_steps != 1)
        return fail(VOG_EINVAL, "bitwise_steps must be 0 or 1");
    if (c->poisson != VOG_POISSON_FOURIER && c->poisson != VOG_POISSON_TRAPEZOID)
        return fail(VOG_EINVAL, "unknown Poisson solver");
    if (c->zero_mean != 0 && c->zero_mean != 1) return fail(VOG_EINVAL, "zero_mean must be 0 or 1");
    if (!isfinite(c->drive_emax)) return fail(VOG_EINVAL, "drive_emax must be finite");
    if (c->drive_emax != 0.0) {
        const double p[6] = {c->drive_k, c->drive_omega, c->drive_t0, c->drive_tl, c->drive_tr, 0.0};
        for (int k = 0; k < 5; ++k)
            if (!isfinite(p[k])) return fail(VOG_EINVAL, "drive parameters must be finite");
        if (!(c->drive_twl > 0.0) || !(c->drive_twr > 0.0) || !isfinite(c->drive_twl) ||
            !isfinite(c->drive_twr))
            return fail(VOG_EINVAL, "drive widths must be finite and > 0");
        const double eps = 0.5 * (tanh((c->drive_t0 - c->drive_tl) / c->drive_twl) -
                                  tanh((c->drive_t0 - c->drive_tr) / c->drive_twr));
        if (!(fabs(1.0 - eps) > 1e-12)) return fail(VOG_EINVAL, "drive envelope is already on at t0");
    }
    if (c->field != VOG_FIELD_SELF_CONSISTENT && c->field != VOG_FIELD_ZERO)
        return fail(VOG_EINVAL, "unknown field mode");
    if (c->n_feq < 1 || c->n_feq > VOG_MAX_FEQ) return fail(VOG_EINVAL, "n_feq must be in [1, 4]");
    for (int g = 0; g < c->n_feq; ++g) {
        if (!isfinite(c->feq_a[g]) || !isfinite(c->feq_c[g]) || !(c->feq_sigma[g] > 0.0) ||
            !isfinite(c->feq_sigma[g]))
            return fail(VOG_EINVAL, "f_eq components need finite a, c and sigma > 0");
    }
    if (c->moments_every < 0) return fail(VOG_EINVAL, "moments_every must be >= 0");
    return VOG_OK;
}

// Drive of Section 4.3: emax k a(t) and the phase omega t at time t.
void drive_at(const vog_config &c, double t, double *amp, double *phase) {
    if (c.drive_emax == 0.0) {
        *amp = 0.0;
        *phase = 0.0;
        return;
    }
    const double eps = 0.5 * (tanh((c.drive_t0 - c.drive_tl) / c.drive_twl) -
                              tanh((c.drive_t0 - c.drive_tr) / c.drive_twr));
    const double br = 0.5 * (tanh((t - c.drive_tl) / c.drive_twl) - tanh((t - c.drive_tr) / c.drive_twr));
    *amp = c.drive_emax * c.drive_k * (br - eps) / (1.0 - eps);
    *phase = c.drive_omega * t;
}

double feq_at(const vog_config &c, double v) {
    double acc = 0.0;
    for (int g = 0; g < c.n_feq; ++g) {
        const double z = (v - c.feq_c[g]) / c.feq_sigma[g];
        acc += c.feq_a[g] * exp(-0.5 * z * z);
    }
    return acc;
}

int upload(void *dst, const void *src, size_t bytes, hipStream_t st) {
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    return VOG_OK;
}

// Twiddle rows of the FFT passes p >= 1 (layout of fft.hpp): row k of pass p
// holds exp(+2 pi i r k / (NS RP)), r < 16 (entries r >= RP are 1).
template <typename T>
std::vector<T> twiddle_rows(int n) {
    std::vector<double> re, im;
    unit_roots(n, re, im);
    std::vector<T> out(2 * (size_t)fft_tw_total(n), (T)0);
    for (size_t k = 0; k < out.size(); k += 2) out[k] = (T)1;
    for (int p = 1; p < fft_npass(n); ++p) {
        const int NS = fft_ns(p), RP = fft_radix(n, p);
        const int scale = 2 * (n / (NS * RP));
        for (int k = 0; k < NS; ++k)
            for (int r = 0; r < RP; ++r) {
                const int idx = (r * k * scale) % (2 * n);
                const size_t at = 2 * ((size_t)fft_tw_off(n, p) + 16 * (size_t)k + r);
                out[at] = (T)re[idx];
                out[at + 1] = (T)im[idx];
            }
    }
    return out;
}

// Symbol table: row t < n / 16 holds exp(2 pi i t q / n), q < 10.
template <typename T>
std::vector<T> eps_rows(int n) {
    std::vector<double> re, im;
    unit_roots(n, re, im);
    const int rows = n / fft_regs(n);
    std::vector<T> out(2 * (size_t)rows * kEpsRow);
    for (int t = 0; t < rows; ++t)
        for (int q = 0; q < kEpsRow; ++q) {
            const int idx = (int)((2LL * t * q) % (2 * n));
            out[2 * ((size_t)t * kEpsRow + q)] = (T)re[idx];
            out[2 * ((size_t)t * kEpsRow + q) + 1] = (T)im[idx];
        }
    return out;
}


// Copies bytes into a host buffer owned by the sim and queues their upload
// (the buffer lives until the sim's next synchronisation).
int stage(vog_sim *s, char *dst, const void *src, size_t bytes) {
    s->staging.emplace_back((const char *)src, (const char *)src + bytes);
    return upload(dst, s->staging.back().data(), bytes, s->stream);
}

template <typename T>
int stage_vec(vog_sim *s, char *dst, const std::vector<T> &v) {
    return stage(s, dst, v.data(), v.size() * sizeof(T));
}

// Profiling helpers: events around one grouped launch of a kind.
void prof_begin(vog_sim *s, int kind, EventPair **pp) {
    *pp = nullptr;
    if (!s->prof) return;
    auto &v = s->ev[kind];
    if (s->ev_used[kind] == v.size()) {
        EventPair e;
        if (hipEventCreate(&e.a) != hipSuccess) return;
        if (hipEventCreate(&e.b) != hipSuccess) {
            (void)hipEventDestroy(e.a);
            return;
        }
        v.push_back(e);
    }
    EventPair *p = &v[s->ev_used[kind]++];
    (void)hipEventRecord(p->a, s->stream);
    *pp = p;
}

void prof_end(vog_sim *s, EventPair *p) {
    if (p) (void)hipEventRecord(p->b, s->stream);
}

int collect_profile(vog_sim *s) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (int k = 0; k < VOG_NUM_KINDS; ++k) {
        for (size_t i = 0; i < s->ev_used[k]; ++i) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, s->ev[k][i].a, s->ev[k][i].b));
            s->ms[k] += ms;
            s->launches[k] += 1;
        }
        s->ev_used[k] = 0;
    }
    return VOG_OK;
}

// Launch helpers over groups of sims that share a kernel instantiation.
struct Group {
    std::vector<vog_sim *> sims;
    std::vector<double> arg;
};

// Chunks of up to B's capacity (Batch: kMaxBatch, SweepBatch: kMaxSweepBatch).
template <typename B = Batch, typename Fn>
int for_chunks(const Group &g, Fn &&fn) {
    constexpr size_t cap = sizeof(B::s) / sizeof(B::s[0]);
    for (size_t base = 0; base < g.sims.size(); base += cap) {
        B b{};
        b.n = (int)std::min<size_t>(cap, g.sims.size() - base);
        for (int k = 0; k < b.n; ++k) {
            b.s[k] = g.sims[base + k]->dev;
            b.a[k] = g.arg.empty() ? 0.0 : g.arg[base + k];
        }
        int rc = fn(b, base);
        if (rc != VOG_OK) return rc;
    }
    return VOG_OK;
}

int check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VOG_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return VOG_OK;
}

// Sweeps of all sims (tau or dt per sim).  vsweep: v-advection on the
// v-fastest layout (vv = 2: two v-advections by tau in a row in one launch,
// transformed in turn; vv = 3: the two composed in Fourier space).
// Otherwise x-advection: fused = true selects the sims whose x-sweep runs on
// the v-fastest layout, fused = false the others (which work on the
// transposed copy).
int run_sweep(vog_sim *lead, const std::vector<vog_sim *> &sims, const std::vector<double> &arg,
              bool vsweep, bool fused = false, int vv = 0) {
    if (vv == 2) {
        // FP64 4096-point v-lines: the two-in-one kernel needs more than 256
        // VGPRs (one wave per SIMD instead of two), so those sims take two
        // launches of the single-step kernel, which give the same values.
        std::vector<vog_sim *> split, rest;
        std::vector<double> as, ar;
        for (size_t k = 0; k < sims.size(); ++k) {
            const bool sp = sims[k]->fp64 && sims[k]->cfg.nv == 4096;
            (sp ? split : rest).push_back(sims[k]);
            (sp ? as : ar).push_back(arg[k]);
        }
        if (!split.empty()) {
            for (int i = 0; i < 2; ++i) {
                const int rc = run_sweep(lead, split, as, true);
                if (rc != VOG_OK) return rc;
            }
            return rest.empty() ? VOG_OK : run_sweep(lead, rest, ar, true, false, 2);
        }
    }
    const int vkind = vv;                                  // sweep kind of a v-sweep launch
    const Kind pkind = vv != 0 ? K_SWEEP_VV : K_SWEEP_V;  // its profile kind
    std::map<std::pair<int, int>, Group> groups;  // (fp64, line length)
    for (size_t k = 0; k < sims.size(); ++k) {
        vog_sim *s = sims[k];
        if (!vsweep && s->fused != fused) continue;
        // key: (precision and x-sweep mode, line length)
        auto key = std::make_pair((int)s->fp64 + 2 * (vsweep ? 0 : s->xmode), vsweep ? s->cfg.nv : s->cfg.nx);
        groups[key].sims.push_back(s);
        groups[key].arg.push_back(arg[k]);
    }
    // FP32 groups of different line lengths that one launch covers: merged
    // when there are two or more of them (a single length keeps its own kernel).
    auto mixable = [&](const std::pair<int, int> &key) {
        const bool fp64 = (key.first & 1) != 0;
        const int xmode = key.first / 2;
        return !fp64 && (vsweep || xmode == X_TILED) && sweep_mixed_ok(vsweep, key.second);
    };
    Group mixed;
    {
        std::vector<std::pair<int, int>> keys;
        for (auto &kv : groups)
            if (mixable(kv.first)) keys.push_back(kv.first);
        if (keys.size() >= 2) {
            for (auto it = keys.rbegin(); it != keys.rend(); ++it) {  // longest lines first
                Group &g = groups[*it];
                mixed.sims.insert(mixed.sims.end(), g.sims.begin(), g.sims.end());
                mixed.arg.insert(mixed.arg.end(), g.arg.begin(), g.arg.end());
                groups.erase(*it);
            }
        }
    }
    if (!mixed.sims.empty()) {
        int rc = for_chunks<SweepBatch>(mixed, [&](const SweepBatch &b, size_t base) {
            SweepMap m{};
            for (int k = 0; k < b.n; ++k) {
                const vog_sim *s = mixed.sims[base + k];
                const int n = vsweep ? s->cfg.nv : s->cfg.nx;
                m.lgn[k] = ilog2(n);
                m.first[k + 1] = m.first[k] + sweep_blocks_mixed(vsweep, n, vsweep ? s->cfg.nx : s->cfg.nv);
            }
            EventPair *p;
            prof_begin(lead, vsweep ? pkind : K_SWEEP_X, &p);
            launch_sweep_mixed(vsweep ? vkind : 1, b, m, lead->stream);
            prof_end(lead, p);
            return check_launch();
        });
        if (rc != VOG_OK) return rc;
    }
    for (auto &kv : groups) {
        const bool fp64 = (kv.first.first & 1) != 0;
        const int xmode = kv.first.first / 2;
        SweepFn fn = vsweep              ? sweep_launcher(fp64, kv.first.second, vkind)
                      : xmode == X_TILED ? fused_xsweep_launcher(fp64, kv.first.second)
                                         : sweep_launcher(fp64, kv.first.second, 1);
        if (!fn) return fail(VOG_EINVAL, "no sweep kernel for this line length");
        int rc = for_chunks<SweepBatch>(kv.second, [&](const SweepBatch &b, size_t base) {
            int maxl = 0;
            for (int k = 0; k < b.n; ++k) {
                const vog_sim *s = kv.second.sims[base + k];
                maxl = std::max(maxl, vsweep ? s->cfg.nx : s->cfg.nv);
            }
            EventPair *p;
            prof_begin(lead, vsweep ? pkind : K_SWEEP_X, &p);
            fn(b, maxl, lead->stream);
            prof_end(lead, p);
            return check_launch();
        });
        if (rc != VOG_OK) return rc;
    }
    return VOG_OK;
}

int run_transpose(vog_sim *lead, const std::vector<vog_sim *> &sims, bool to_v) {
    std::map<int, Group> groups;
    for (vog_sim *s : sims)
        if (!s->fused) groups[(int)s->fp64].sims.push_back(s);
    for (auto &kv : groups) {
        int rc = for_chunks(kv.second, [&](const Batch &b, size_t base) {
            int maxt = 0;
            for (int k = 0; k < b.n; ++k) {
                const vog_sim *s = kv.second.sims[base + k];
                const int tiles = ((s->cfg.nx + kTile - 1) / kTile) * ((s->cfg.nv + kTile - 1) / kTile);
                maxt = std::max(maxt, tiles);
            }
            EventPair *p;
            prof_begin(lead, to_v ? K_T_XV : K_T_VX, &p);
            launch_transpose(kv.first != 0, to_v, b, maxt, lead->stream);
            prof_end(lead, p);
            return check_launch();
        });
        if (rc != VOG_OK) return rc;
    }
    return VOG_OK;
}

// rho from the partial velocity sums the x-advection left (tiled x-sweep or
// x -> v transpose).
int run_rho_reduce(vog_sim *lead, const std::vector<vog_sim *> &sims) {
    Group g;
    g.sims = sims;
    return for_chunks<SweepBatch>(g, [&](const SweepBatch &b, size_t base) {
        int maxnx = 0;
        for (int k = 0; k < b.n; ++k) maxnx = std::max(maxnx, g.sims[base + k]->cfg.nx);
        EventPair *p;
        prof_begin(lead, K_RHO, &p);
        launch_rho_reduce(b, maxnx, lead->stream);
        prof_end(lead, p);
        return check_launch();
    });
}

// Field solve (Poisson, E, diagnostics record) for all sims.
int run_field(vog_sim *lead, const std::vector<vog_sim *> &sims, const std::vector<int64_t> &stepno,
              const std::vector<double> &tnow) {
    // nx -> indices; every nx of at most 1024 points goes to key 0, the
    // one-wave kernel that covers all of them (also for a single sim, so that a
    // sim gives the same bits alone and in a batch).
    std::map<int, std::vector<size_t>> groups;
    for (size_t k = 0; k < sims.size(); ++k) {
        const int nx = sims[k]->cfg.nx;
        groups[field_mixed_ok(nx) ? 0 : nx].push_back(k);
    }
    if (groups.count(0)) {  // longest lines first
        std::vector<size_t> &g = groups[0];
        std::stable_sort(g.begin(), g.end(),
                         [&](size_t a, size_t c) { return sims[a]->cfg.nx > sims[c]->cfg.nx; });
    }
    for (auto &kv : groups) {
        LaunchFn fn = kv.first == 0 ? nullptr : field_launcher(kv.first);
        if (kv.first != 0 && !fn) return fail(VOG_EINVAL, "no field kernel for this nx");
        const auto &idx = kv.second;
        for (size_t base = 0; base < idx.size(); base += kMaxBatch) {
            Batch b{};
            BlockMap m{};
            b.n = (int)std::min<size_t>(kMaxBatch, idx.size() - base);
            for (int k = 0; k < b.n; ++k) {
                const size_t i = idx[base + k];
                b.s[k] = sims[i]->dev;
                b.step[k] = stepno[i];
                b.t[k] = tnow[i];
                drive_at(sims[i]->cfg, tnow[i], &b.drv_amp[k], &b.drv_ph[k]);
                m.first[k + 1] = k + 1;
                m.lgn[k] = ilog2(sims[i]->cfg.nx);
            }
            EventPair *p;
            prof_begin(lead, K_FIELD, &p);
            if (fn) fn(b, 0, lead->stream);
            else launch_field_mixed(b, m, lead->stream);
            prof_end(lead, p);
            int rc = check_launch();
            if (rc != VOG_OK) return rc;
        }
    }
    return VOG_OK;
}

// rho = int f dv straight from the v-fastest layout.
int run_rho_v(vog_sim *lead, const std::vector<vog_sim *> &sims) {
    std::map<int, Group> groups;
    for (vog_sim *s : sims) groups[(int)s->fp64].sims.push_back(s);
    for (auto &kv : groups) {
        int rc = for_chunks(kv.second, [&](const Batch &b, size_t base) {
            int maxnx = 0;
            for (int k = 0; k < b.n; ++k) maxnx = std::max(maxnx, kv.second.sims[base + k]->cfg.nx);
            EventPair *p;
            prof_begin(lead, K_RHO, &p);
            launch_rho_v(kv.first != 0, b, maxnx, lead->stream);
            prof_end(lead, p);
            return check_launch();
        });
        if (rc != VOG_OK) return rc;
    }
    return VOG_OK;
}

int run_moments(vog_sim *lead, const std::vector<vog_sim *> &sims, const std::vector<int64_t> &stepno) {
    std::map<int, std::vector<size_t>> groups;
    for (size_t k = 0; k < sims.size(); ++k) groups[(int)sims[k]->fp64].push_back(k);
    for (auto &kv : groups) {
        const auto &idx = kv.second;
        for (size_t base = 0; base < idx.size(); base += kMaxBatch) {
            Batch b{};
            b.n = (int)std::min<size_t>(kMaxBatch, idx.size() - base);
            int maxnx = 0;
            for (int k = 0; k < b.n; ++k) {
                const size_t i = idx[base + k];
                b.s[k] = sims[i]->dev;
                b.step[k] = stepno[i];
                maxnx = std::max(maxnx, sims[i]->cfg.nx);
            }
            EventPair *p;
            prof_begin(lead, K_MOMENTS, &p);
            launch_moments(kv.first != 0, b, maxnx, lead->stream);
            prof_end(lead, p);
            int rc = check_launch();
            if (rc != VOG_OK) return rc;
        }
    }
    return VOG_OK;
}

// Recompute E from the current f (v layout) and write a record for the
// current step number.
int field_from_f(vog_sim *s) {
    std::vector<vog_sim *> one{s};
    int rc = run_rho_v(s, one);
    if (rc != VOG_OK) return rc;
    std::vector<int64_t> st{s->step};
    std::vector<double> tt{s->t};
    return run_field(s, one, st, tt);
}

// x-advection of all sims by dt; with_rho also leaves rho = int f dv.
int x_advection(vog_sim *lead, const std::vector<vog_sim *> &sims, const std::vector<double> &dt,
                bool with_rho) {
    int rc;
    if ((rc = run_sweep(lead, sims, dt, false, true)) != VOG_OK) return rc;
    if ((rc = run_transpose(lead, sims, false)) != VOG_OK) return rc;
    if ((rc = run_sweep(lead, sims, dt, false, false)) != VOG_OK) return rc;
    if ((rc = run_transpose(lead, sims, true)) != VOG_OK) return rc;
    if (!with_rho) return VOG_OK;
    return run_rho_reduce(lead, sims);
}

int device_guard(vog_sim *s) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != s->device) HIP_TRY(hipSetDevice(s->device));
    return VOG_OK;
}

// nsteps Strang steps (Section 1.1) of every sim, one grouped launch per
// kernel kind and line length.  Between two steps of one call, the closing
// half step of the first and the opening half step of the second share the
// field: sims with merge_v replace them by one advection by dt (a different
// scheme, opt-in); the others run both in one launch, except where the
// moments need the full time level in between: FP32 sims composed in Fourier
// space (sweep kind 3, the same scheme up to rounding), FP64 sims and those
// with bitwise_steps transformed in turn (kind 2, the arithmetic of two
// launches).
int step_sims(const std::vector<vog_sim *> &sims, const std::vector<double> &dt, int nsteps) {
    vog_sim *lead = sims[0];
    std::vector<int64_t> stepno(sims.size());
    std::vector<double> tnow(sims.size());
    std::vector<char> opened(sims.size(), 0);  // opening half step already done
    for (int n = 0; n < nsteps; ++n) {
        const bool last = n == nsteps - 1;
        std::vector<vog_sim *> open, once, twice, comp, msims;  // see below
        std::vector<double> half, tau_once, tau_twice, tau_comp;
        std::vector<int64_t> mstep;
        for (size_t k = 0; k < sims.size(); ++k) {
            stepno[k] = sims[k]->step + 1;
            tnow[k] = sims[k]->t + dt[k];
            const bool merge = sims[k]->cfg.merge_v != 0;
            if (!opened[k]) {  // starts this step with a half step
                open.push_back(sims[k]);
                half.push_back(0.5 * dt[k]);
            }
            // moments after this step; merged sims hold a full time level
            // only after a call's last step
            const int every = sims[k]->cfg.moments_every;
            const bool due = every > 0 && stepno[k] % every == 0 && (!merge || last);
            if (due) {
                msims.push_back(sims[k]);
                mstep.push_back(stepno[k]);
            }
            if (merge && !last) {  // closing and next opening half step as one by dt
                once.push_back(sims[k]);
                tau_once.push_back(dt[k]);
            } else if (!last && !due) {  // closing and next opening half step, one launch
                const bool bitwise = sims[k]->fp64 || sims[k]->cfg.bitwise_steps != 0;
                (bitwise ? twice : comp).push_back(sims[k]);
                (bitwise ? tau_twice : tau_comp).push_back(0.5 * dt[k]);
            } else {
                once.push_back(sims[k]);
                tau_once.push_back(0.5 * dt[k]);
            }
            opened[k] = !last && (merge || !due);
        }
        int rc;
        if (!open.empty() && (rc = run_sweep(lead, open, half, true)) != VOG_OK) return rc;
        if ((rc = x_advection(lead, sims, dt, true)) != VOG_OK) return rc;
        if ((rc = run_field(lead, sims, stepno, tnow)) != VOG_OK) return rc;
        if (!once.empty() && (rc = run_sweep(lead, once, tau_once, true)) != VOG_OK) return rc;
        if (!twice.empty() && (rc = run_sweep(lead, twice, tau_twice, true, false, 2)) != VOG_OK)
            return rc;
        if (!comp.empty() && (rc = run_sweep(lead, comp, tau_comp, true, false, 3)) != VOG_OK)
            return rc;
        if (!msims.empty() && (rc = run_moments(lead, msims, mstep)) != VOG_OK) return rc;
        for (size_t k = 0; k < sims.size(); ++k) {
            sims[k]->step = stepno[k];
            sims[k]->t = tnow[k];
        }
    }
    return VOG_OK;
}

}  // namespace

extern "C" {

void vog_config_default(vog_config *c) {
    if (!c) return;
    memset(c, 0, sizeof(*c));
    c->nx = 64;
    c->nv = 128;
    c->L = 4.0 * M_PI;
    c->vmin = -6.0;
    c->vmax = 6.0;
    c->degree = 17;
    c->precision = VOG_FP64_PLAIN;
    c->poisson = VOG_POISSON_FOURIER;
    c->field = VOG_FIELD_SELF_CONSISTENT;
    c->n_feq = 1;
    c->feq_a[0] = 1.0 / sqrt(2.0 * M_PI);
    c->feq_c[0] = 0.0;
    c->feq_sigma[0] = 1.0;
    c->moments_every = 0;
    c->zero_mean = 1;
}

int vog_config_validate(const vog_config *c) { return validate(c); }

size_t vog_workspace_bytes(const vog_config *c) {
    if (validate(c) != VOG_OK) return 0;
    return layout_of(*c).total;
}

int vog_create(const vog_config *c, void *dev_workspace, size_t bytes, void *hip_stream, vog_sim **out) {
    if (!out) return fail(VOG_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(c);
    if (rc != VOG_OK) return rc;
    const Layout L = layout_of(*c);
    if (dev_workspace) {
        if (bytes < L.total) return fail(VOG_ENOMEM, "workspace smaller than vog_workspace_bytes");
        if (((uintptr_t)dev_workspace & 255u) != 0) return fail(VOG_EINVAL, "workspace must be 256-byte aligned");
    }
    vog_sim *s = new (std::nothrow) vog_sim();
    if (!s) return fail(VOG_ENOMEM, "host allocation failed");
    s->cfg = *c;
    s->lay = L;
    s->stream = (hipStream_t)hip_stream;
    s->fp64 = prec_fp64(*c);
    s->fused = uses_fused_xsweep(*c);
    s->xmode = xsweep_mode(*c);
    s->step = 0;
    s->t = 0.0;
    s->diag_read = 0;
    s->prof = false;
    for (int k = 0; k < VOG_NUM_KINDS; ++k) {
        s->ev_used[k] = 0;
        s->ms[k] = 0.0;
        s->launches[k] = 0;
    }
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(VOG_EDEVICE, "hipGetDevice failed");
    }
    if (dev_workspace) {
        s->ws = (char *)dev_workspace;
        s->owns = false;
    } else {
        void *p = nullptr;
        if (hipMalloc(&p, L.total) != hipSuccess) {
            (void)hipGetLastError();
            delete s;
            return fail(VOG_ENOMEM, "hipMalloc of the workspace failed");
        }
        s->ws = (char *)p;
        s->owns = true;
    }

    const bool fp64 = s->fp64;
    const int nx = c->nx, nv = c->nv;
    const double dv = (c->vmax - c->vmin) / nv;
    SimDev &D = s->host_dev;
    memset(&D, 0, sizeof(D));
    D.f = s->ws + L.f;
    D.g = s->fused ? nullptr : s->ws + L.g;
    D.E = (double *)(s->ws + L.E);
    D.Eeff = (double *)(s->ws + L.Eeff);
    D.part = (double *)(s->ws + L.part);
    D.rho = (double *)(s->ws + L.rho);
    D.mom = (double *)(s->ws + L.mom);
    D.tw_x = s->ws + L.tw_x;
    D.tw_v = s->ws + L.tw_v;
    D.eps_x = s->ws + L.eps_x;
    D.eps_v = s->ws + L.eps_v;
    D.tw_x64 = (const double *)(s->ws + L.tw_x64);
    D.iden_x = c->interp == VOG_INTERP_BSPLINE ? s->ws + L.iden_x : nullptr;
    D.iden_v = c->interp == VOG_INTERP_BSPLINE ? s->ws + L.iden_v : nullptr;
    D.interp = c->interp;
    D.invk = (const double *)(s->ws + L.invk);
    D.drv_sc = c->drive_emax != 0.0 ? (const double *)(s->ws + L.drv_sc) : nullptr;
    D.feq_g = s->ws + L.feq_g;
    D.feq64 = (const double *)(s->ws + L.feq64);
    D.ring = (vog_diag *)(s->ws + L.ring);
    D.nx = nx;
    D.nv = nv;
    D.d = (c->degree - 1) / 2;
    D.deltaf = prec_deltaf(*c);
    D.field_zero = c->field == VOG_FIELD_ZERO;
    D.n_feq = c->n_feq;
    D.nparts = rho_parts(*c);
    D.poisson = c->poisson;
    D.zero_mean = c->zero_mean;
    D.fp64 = fp64;
    D.L = c->L;
    D.vmin = c->vmin;
    D.dx = c->L / nx;
    D.dv = dv;
    D.inv_dx = nx / c->L;
    D.inv_dv = 1.0 / dv;
    for (int g = 0; g < VOG_MAX_FEQ; ++g) {
        D.feq_c[g] = g < c->n_feq ? c->feq_c[g] : 0.0;
        D.feq_inv_s2[g] = g < c->n_feq ? 1.0 / (c->feq_sigma[g] * c->feq_sigma[g]) : 0.0;
    }
    s->feq64.resize(nv);
    double feq_sum = 0.0;
    for (int j = 0; j < nv; ++j) {
        s->feq64[j] = feq_at(*c, c->vmin + j * dv);
        feq_sum += s->feq64[j];
    }
    D.feq_const = D.deltaf ? dv * feq_sum : 0.0;
    s->dev = (const SimDev *)(s->ws + L.dev);

    // Host tables (FP64, rounded to the storage precision).
    std::vector<double> fg64((size_t)VOG_MAX_FEQ * nv, 0.0);
    for (int g = 0; g < c->n_feq; ++g)
        for (int j = 0; j < nv; ++j) {
            const double z = (c->vmin + j * dv - c->feq_c[g]) / c->feq_sigma[g];
            fg64[(size_t)g * nv + j] = c->feq_a[g] * exp(-0.5 * z * z);
        }

    auto bail = [&](int code) {
        vog_destroy(s);
        return code;
    };
    launch_fill(s->ws, L.total, s->stream);
    if ((rc = check_launch()) != VOG_OK) return bail(rc);
    // The tables are uploaded from copies the sim owns (stage), so nothing here
    // waits for work already queued on the stream.
    const std::vector<double> tw64x = twiddle_rows<double>(nx);
    const std::vector<double> tw64v = twiddle_rows<double>(nv);
    const std::vector<double> ep64x = eps_rows<double>(nx);
    const std::vector<double> ep64v = eps_rows<double>(nv);
    std::vector<float> tw32x, tw32v, ep32x, ep32v, fg32, id32x, id32v;
    std::vector<double> id64x, id64v;
    if (c->interp == VOG_INTERP_BSPLINE) {
        id64x = bspline_inverse_symbol(nx, c->degree);
        id64v = bspline_inverse_symbol(nv, c->degree);
        if (fp64) {
            if ((rc = stage_vec(s, s->ws + L.iden_x, id64x)) != VOG_OK) return bail(rc);
            if ((rc = stage_vec(s, s->ws + L.iden_v, id64v)) != VOG_OK) return bail(rc);
        } else {
            id32x.assign(id64x.begin(), id64x.end());
            id32v.assign(id64v.begin(), id64v.end());
            if ((rc = stage_vec(s, s->ws + L.iden_x, id32x)) != VOG_OK) return bail(rc);
            if ((rc = stage_vec(s, s->ws + L.iden_v, id32v)) != VOG_OK) return bail(rc);
        }
    }
    if (fp64) {
        if ((rc = stage_vec(s, s->ws + L.tw_x, tw64x)) != VOG_OK) return bail(rc);
        if ((rc = stage_vec(s, s->ws + L.tw_v, tw64v)) != VOG_OK) return bail(rc);
        if ((rc = stage_vec(s, s->ws + L.eps_x, ep64x)) != VOG_OK) return bail(rc);
        if ((rc = stage_vec(s, s->ws + L.eps_v, ep64v)) != VOG_OK) return bail(rc);
        if ((rc = stage_vec(s, s->ws + L.feq_g, fg64)) != VOG_OK) return bail(rc);
    } else {
        tw32x = twiddle_rows<float>(nx);
        tw32v = twiddle_rows<float>(nv);
        ep32x = eps_rows<float>(nx);
        ep32v = eps_rows<float>(nv);
        fg32.assign(fg64.begin(), fg64.end());
        if ((rc = stage_vec(s, s->ws + L.tw_x, tw32x)) != VOG_OK) return bail(rc);
        if ((rc = stage_vec(s, s->ws + L.tw_v, tw32v)) != VOG_OK) return bail(rc);
        if ((rc = stage_vec(s, s->ws + L.eps_x, ep32x)) != VOG_OK) return bail(rc);
        if ((rc = stage_vec(s, s->ws + L.eps_v, ep32v)) != VOG_OK) return bail(rc);
        if ((rc = stage_vec(s, s->ws + L.feq_g, fg32)) != VOG_OK) return bail(rc);
    }
    if ((rc = stage_vec(s, s->ws + L.tw_x64, tw64x)) != VOG_OK) return bail(rc);
    // 1 / (nx k_m) for the Fourier field solve: k_m = 2 pi mt / L with mt the
    // signed mode index; modes 0 and nx/2 (and every mode for a zero field) get 0.
    std::vector<double> invk(nx, 0.0);
    if (c->field == VOG_FIELD_SELF_CONSISTENT)
        for (int m = 1; m < nx; ++m) {
            if (2 * m == nx) continue;
            const int mt = 2 * m < nx ? m : m - nx;
            invk[m] = 1.0 / ((double)nx * (2.0 * M_PI * (double)mt / c->L));
        }
    if ((rc = stage_vec(s, s->ws + L.invk, invk)) != VOG_OK) return bail(rc);
    if ((rc = stage_vec(s, s->ws + L.feq64, s->feq64)) != VOG_OK) return bail(rc);
    if (c->drive_emax != 0.0) {
        // E_app(t, x_j) = amp(t) (sin(k x_j) cos(omega t) - cos(k x_j) sin(omega t))
        std::vector<double> sc(2 * (size_t)nx);
        for (int j = 0; j < nx; ++j) {
            sc[2 * j] = sin(c->drive_k * (j * D.dx));
            sc[2 * j + 1] = cos(c->drive_k * (j * D.dx));
        }
        if ((rc = stage_vec(s, s->ws + L.drv_sc, sc)) != VOG_OK) return bail(rc);
    }
    if ((rc = stage(s, s->ws + L.dev, &D, sizeof(D))) != VOG_OK) return bail(rc);
    *out = s;
    return VOG_OK;
}

int vog_init_perturbed(vog_sim *s, int nmodes, const double *amp, const double *kx, const double *phase) {
    if (!s) return fail(VOG_EINVAL, "sim is NULL");
    if (nmodes < 0 || nmodes > 8) return fail(VOG_EINVAL, "nmodes must be in [0, 8]");
    if (nmodes > 0 && (!amp || !kx || !phase)) return fail(VOG_EINVAL, "mode arrays are NULL");
    for (int m = 0; m < nmodes; ++m)
        if (!isfinite(amp[m]) || !isfinite(kx[m]) || !isfinite(phase[m]))
            return fail(VOG_EINVAL, "mode parameters must be finite");
    int rc = device_guard(s);
    if (rc != VOG_OK) return rc;
    launch_init(s->fp64, s->dev, s->cfg.nx * s->cfg.nv, nmodes, amp, kx, phase, s->stream);
    if ((rc = check_launch()) != VOG_OK) return rc;
    s->step = 0;
    s->t = 0.0;
    s->diag_read = 0;
    launch_fill(s->host_dev.ring, sizeof(vog_diag) * kRingCap, s->stream);
    return field_from_f(s);
}

int vog_set_f(vog_sim *s, const double *host_f) {
    if (!s || !host_f) return fail(VOG_EINVAL, "NULL argument");
    int rc = device_guard(s);
    if (rc != VOG_OK) return rc;
    const int nx = s->cfg.nx, nv = s->cfg.nv;
    const size_t cells = (size_t)nx * nv;
    const bool df = s->host_dev.deltaf;
    if (s->fp64) {
        std::vector<double> buf(cells);
        for (size_t k = 0; k < cells; ++k) buf[k] = host_f[k] - (df ? s->feq64[k % nv] : 0.0);
        HIP_TRY(hipMemcpyAsync(s->host_dev.f, buf.data(), cells * 8, hipMemcpyHostToDevice, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    } else {
        std::vector<float> buf(cells);
        for (size_t k = 0; k < cells; ++k) buf[k] = (float)(host_f[k] - (df ? s->feq64[k % nv] : 0.0));
        HIP_TRY(hipMemcpyAsync(s->host_dev.f, buf.data(), cells * 4, hipMemcpyHostToDevice, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    s->step = 0;
    s->t = 0.0;
    s->diag_read = 0;
    launch_fill(s->host_dev.ring, sizeof(vog_diag) * kRingCap, s->stream);
    return field_from_f(s);
}

int vog_get_raw(vog_sim *s, void *host_buf, size_t bytes, int *elem_bytes) {
    if (!s || !host_buf) return fail(VOG_EINVAL, "NULL argument");
    const size_t es = s->fp64 ? 8 : 4;
    const size_t need = (size_t)s->cfg.nx * s->cfg.nv * es;
    if (bytes < need) return fail(VOG_EINVAL, "host buffer too small");
    int rc = device_guard(s);
    if (rc != VOG_OK) return rc;
    HIP_TRY(hipMemcpyAsync(host_buf, s->host_dev.f, need, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (elem_bytes) *elem_bytes = (int)es;
    return VOG_OK;
}

int vog_get_f(vog_sim *s, double *host_f) {
    if (!s || !host_f) return fail(VOG_EINVAL, "NULL argument");
    const int nx = s->cfg.nx, nv = s->cfg.nv;
    const size_t cells = (size_t)nx * nv;
    const bool df = s->host_dev.deltaf;
    int rc;
    if (s->fp64) {
        if ((rc = vog_get_raw(s, host_f, cells * 8, nullptr)) != VOG_OK) return rc;
        if (df)
            for (size_t k = 0; k < cells; ++k) host_f[k] += s->feq64[k % nv];
    } else {
        std::vector<float> buf(cells);
        if ((rc = vog_get_raw(s, buf.data(), cells * 4, nullptr)) != VOG_OK) return rc;
        for (size_t k = 0; k < cells; ++k) host_f[k] = (double)buf[k] + (df ? s->feq64[k % nv] : 0.0);
    }
    return VOG_OK;
}

int vog_get_E(vog_sim *s, double *host_E) {
    if (!s || !host_E) return fail(VOG_EINVAL, "NULL argument");
    int rc = device_guard(s);
    if (rc != VOG_OK) return rc;
    HIP_TRY(hipMemcpyAsync(host_E, s->host_dev.E, sizeof(double) * s->cfg.nx, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return VOG_OK;
}

int vog_set_E(vog_sim *s, const double *host_E) {
    if (!s || !host_E) return fail(VOG_EINVAL, "NULL argument");
    int rc = device_guard(s);
    if (rc != VOG_OK) return rc;
    const int nx = s->cfg.nx;
    std::vector<double> eff(host_E, host_E + nx);
    double amp, ph;
    drive_at(s->cfg, s->t, &amp, &ph);
    if (amp != 0.0) {  // the form the field solve uses
        const double cph = cos(ph), sph = sin(ph);
        for (int i = 0; i < nx; ++i) {
            const double kx = s->cfg.drive_k * (i * s->host_dev.dx);
            eff[i] -= amp * (sin(kx) * cph - cos(kx) * sph);
        }
    }
    HIP_TRY(hipMemcpyAsync(s->host_dev.E, host_E, sizeof(double) * nx, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->host_dev.Eeff, eff.data(), sizeof(double) * nx, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return VOG_OK;
}

int vog_step(vog_sim *s, double dt, int nsteps) {
    if (!s) return fail(VOG_EINVAL, "sim is NULL");
    return vog_step_batch(&s, 1, &dt, nsteps);
}

int vog_step_batch(vog_sim *const *sims, int nsims, const double *dt, int nsteps) {
    if (!sims || nsims <= 0 || !dt) return fail(VOG_EINVAL, "empty batch");
    if (nsteps < 0) return fail(VOG_EINVAL, "nsteps must be >= 0");
    std::vector<vog_sim *> v(sims, sims + nsims);
    std::vector<double> d(dt, dt + nsims);
    for (int k = 0; k < nsims; ++k) {
        if (!v[k]) return fail(VOG_EINVAL, "NULL sim in batch");
        if (!(d[k] > 0.0) || !isfinite(d[k])) return fail(VOG_EINVAL, "dt must be finite and > 0");
        if (v[k]->stream != v[0]->stream || v[k]->device != v[0]->device)
            return fail(VOG_EINVAL, "all sims of a batch must share the stream and device of sims[0]");
    }
    std::vector<vog_sim *> sorted = v;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        return fail(VOG_EINVAL, "a sim appears twice in the batch");
    if (nsteps == 0) return VOG_OK;
    int rc = device_guard(v[0]);
    if (rc != VOG_OK) return rc;
    return step_sims(v, d, nsteps);
}

int vog_sweep(vog_sim *s, int which, double arg) {
    if (!s) return fail(VOG_EINVAL, "sim is NULL");
    if (which < 0 || which > 2) return fail(VOG_EINVAL, "which must be 0, 1 or 2");
    if (which < 2 && !isfinite(arg)) return fail(VOG_EINVAL, "arg must be finite");
    int rc = device_guard(s);
    if (rc != VOG_OK) return rc;
    std::vector<vog_sim *> one{s};
    std::vector<double> a{arg};
    if (which == 0) return run_sweep(s, one, a, true);
    if (which == 1) return x_advection(s, one, a, false);
    return field_from_f(s);
}

int vog_get_diag(vog_sim *s, vog_diag *out, int cap, int *n) {
    if (!s || !n || (cap > 0 && !out)) return fail(VOG_EINVAL, "NULL argument");
    *n = 0;
    int rc = device_guard(s);
    if (rc != VOG_OK) return rc;
    HIP_TRY(hipStreamSynchronize(s->stream));
    const int64_t first = std::max(s->diag_read, s->step - (int64_t)kRingCap + 1);
    int64_t count = s->step - first + 1;
    if (count <= 0) return VOG_OK;
    if (count > cap) count = cap;
    // records first .. first+count-1 sit in at most two contiguous pieces of the ring
    const int64_t head = first % kRingCap;
    const int64_t n1 = std::min<int64_t>(count, kRingCap - head);
    HIP_TRY(hipMemcpy(out, s->host_dev.ring + head, sizeof(vog_diag) * n1, hipMemcpyDeviceToHost));
    if (count > n1)
        HIP_TRY(hipMemcpy(out + n1, s->host_dev.ring, sizeof(vog_diag) * (count - n1),
                          hipMemcpyDeviceToHost));
    *n = (int)count;
    s->diag_read = first + count;
    return VOG_OK;
}

size_t vog_state_bytes(const vog_sim *s) {
    if (!s) return 0;
    const size_t es = s->fp64 ? 8 : 4;
    return 16 + (size_t)s->cfg.nx * s->cfg.nv * es + 2 * sizeof(double) * s->cfg.nx;
}

int vog_get_state(vog_sim *s, void *host_buf, size_t bytes) {
    if (!s || !host_buf) return fail(VOG_EINVAL, "NULL argument");
    if (bytes < vog_state_bytes(s)) return fail(VOG_EINVAL, "buffer smaller than vog_state_bytes");
    int rc = device_guard(s);
    if (rc != VOG_OK) return rc;
    const size_t fb = (size_t)s->cfg.nx * s->cfg.nv * (s->fp64 ? 8 : 4);
    char *p = (char *)host_buf;
    memcpy(p, &s->step, 8);
    memcpy(p + 8, &s->t, 8);
    HIP_TRY(hipMemcpyAsync(p + 16, s->host_dev.f, fb, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(p + 16 + fb, s->host_dev.E, sizeof(double) * s->cfg.nx, hipMemcpyDeviceToHost, s->stream));
    // the advecting field: E - E_app for driven sims, E itself for the others
    // (whose field solve leaves Eeff unwritten)
    const double *eff = s->host_dev.drv_sc ? s->host_dev.Eeff : s->host_dev.E;
    HIP_TRY(hipMemcpyAsync(p + 16 + fb + sizeof(double) * s->cfg.nx, eff, sizeof(double) * s->cfg.nx,
                           hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return VOG_OK;
}

int vog_set_state(vog_sim *s, const void *host_buf, size_t bytes) {
    if (!s || !host_buf) return fail(VOG_EINVAL, "NULL argument");
    if (bytes < vog_state_bytes(s)) return fail(VOG_EINVAL, "buffer smaller than vog_state_bytes");
    int rc = device_guard(s);
    if (rc != VOG_OK) return rc;
    const size_t fb = (size_t)s->cfg.nx * s->cfg.nv * (s->fp64 ? 8 : 4);
    const char *p = (const char *)host_buf;
    int64_t st;
    double tt;
    memcpy(&st, p, 8);
    memcpy(&tt, p + 8, 8);
    if (st < 0 || !isfinite(tt)) return fail(VOG_EINVAL, "corrupt state header");
    HIP_TRY(hipMemcpyAsync(s->host_dev.f, p + 16, fb, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->host_dev.E, p + 16 + fb, sizeof(double) * s->cfg.nx, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->host_dev.Eeff, p + 16 + fb + sizeof(double) * s->cfg.nx,
                           sizeof(double) * s->cfg.nx, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->step = st;
    s->t = tt;
    s->diag_read = st + 1;
    return VOG_OK;
}

int vog_get_time(const vog_sim *s, int64_t *step, double *t) {
    if (!s) return fail(VOG_EINVAL, "sim is NULL");
    if (step) *step = s->step;
    if (t) *t = s->t;
    return VOG_OK;
}

int vog_sync(vog_sim *s) {
    if (!s) return fail(VOG_EINVAL, "sim is NULL");
    int rc = device_guard(s);
    if (rc != VOG_OK) return rc;
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->staging.clear();
    if (s->step > 0 && s->host_dev.field_zero == 0) {
        vog_diag d;
        HIP_TRY(hipMemcpy(&d, s->host_dev.ring + (s->step % kRingCap), sizeof(d), hipMemcpyDeviceToHost));
        if (d.step == s->step && !d.finite) return fail(VOG_ENONFINITE, "field is not finite");
    }
    return VOG_OK;
}

int vog_sync_batch(vog_sim *const *sims, int nsims, int *status) {
    if (!sims || nsims < 1 || !status) return fail(VOG_EINVAL, "NULL argument or nsims < 1");
    for (int k = 0; k < nsims; ++k) {
        if (!sims[k]) return fail(VOG_EINVAL, "sim is NULL");
        if (sims[k]->device != sims[0]->device || sims[k]->stream != sims[0]->stream)
            return fail(VOG_EINVAL, "sims of a batch must share the device and stream");
    }
    vog_sim *lead = sims[0];
    int rc = device_guard(lead);
    if (rc != VOG_OK) return rc;
    // one flag buffer of kMaxBatch ints per device, kept for the process
    static std::mutex mu;
    static std::map<int, int *> bufs;
    std::lock_guard<std::mutex> g(mu);
    int *&flags = bufs[lead->device];
    if (!flags && hipMalloc((void **)&flags, sizeof(int) * kMaxBatch) != hipSuccess) {
        flags = nullptr;
        return fail(VOG_ENOMEM, "flag buffer allocation failed");
    }
    std::vector<int> host(nsims, 1);
    for (int base = 0; base < nsims; base += kMaxBatch) {
        Batch b{};
        b.n = std::min(kMaxBatch, nsims - base);
        for (int k = 0; k < b.n; ++k) {
            b.s[k] = sims[base + k]->dev;
            b.step[k] = sims[base + k]->step;
        }
        launch_finite_gather(b, flags, lead->stream);
        if ((rc = check_launch()) != VOG_OK) return rc;
        HIP_TRY(hipMemcpyAsync(host.data() + base, flags, sizeof(int) * b.n, hipMemcpyDeviceToHost,
                               lead->stream));
    }
    HIP_TRY(hipStreamSynchronize(lead->stream));
    for (int k = 0; k < nsims; ++k) {
        sims[k]->staging.clear();
        status[k] = host[k] ? VOG_OK : VOG_ENONFINITE;
    }
    return VOG_OK;
}

int vog_sync_batch_noalloc(vog_sim *const *sims, int nsims, int *status) {
    if (!sims || nsims < 1 || !status) return fail(VOG_EINVAL, "NULL argument or nsims < 1");
    if (nsims > VOG_NOALLOC_MAX_SIMS) return fail(VOG_EINVAL, "nsims exceeds VOG_NOALLOC_MAX_SIMS");
    for (int k = 0; k < nsims; ++k) {
        if (!sims[k]) return fail(VOG_EINVAL, "sim is NULL");
        if (sims[k]->device != sims[0]->device || sims[k]->stream != sims[0]->stream)
            return fail(VOG_EINVAL, "sims of a batch must share the device and stream");
    }
    vog_sim *lead = sims[0];
    int rc = device_guard(lead);
    if (rc != VOG_OK) return rc;
    static std::mutex mu;  // calls through this entry point share the array
    std::lock_guard<std::mutex> g(mu);
    int *flags = noalloc_flags(lead->device);
    if (!flags) return fail(VOG_EDEVICE, "address of the library's flag array not found");
    // every flag 0 .. nsims-1 is written by the gathers before the copy reads it
    for (int base = 0; base < nsims; base += kMaxBatch) {
        Batch b{};
        b.n = std::min(kMaxBatch, nsims - base);
        for (int k = 0; k < b.n; ++k) {
            b.s[k] = sims[base + k]->dev;
            b.step[k] = sims[base + k]->step;
        }
        launch_finite_gather(b, flags + base, lead->stream);
        if ((rc = check_launch()) != VOG_OK) return rc;
    }
    HIP_TRY(hipMemcpyAsync(status, flags, sizeof(int) * (size_t)nsims, hipMemcpyDeviceToHost, lead->stream));
    HIP_TRY(hipStreamSynchronize(lead->stream));
    for (int k = 0; k < nsims; ++k) {
        sims[k]->staging.clear();
        status[k] = status[k] ? VOG_OK : VOG_ENONFINITE;
    }
    return VOG_OK;
}

void vog_destroy(vog_sim *s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    for (int k = 0; k < VOG_NUM_KINDS; ++k)
        for (auto &e : s->ev[k]) {
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
    if (s->owns && s->ws) (void)hipFree(s->ws);
    delete s;
}

const char *vog_strerror(int code) {
    switch (code) {
        case VOG_OK: return "ok";
        case VOG_EINVAL: return "invalid argument";
        case VOG_ENOMEM: return "out of memory";
        case VOG_EDEVICE: return "device error";
        case VOG_ENONFINITE: return "non-finite field";
        case VOG_EBUSY: return "busy";
        default: return "unknown error";
    }
}

const char *vog_last_error(void) { return g_last_error.c_str(); }

int vog_profile_enable(vog_sim *s, int on) {
    if (!s) return fail(VOG_EINVAL, "sim is NULL");
    if (on) {
        int rc = collect_profile(s);
        if (rc != VOG_OK) return rc;
        for (int k = 0; k < VOG_NUM_KINDS; ++k) {
            s->ms[k] = 0.0;
            s->launches[k] = 0;
        }
    }
    s->prof = on != 0;
    return VOG_OK;
}

int vog_profile_read(vog_sim *s, double *ms, int64_t *launches, int nkinds) {
    if (!s) return fail(VOG_EINVAL, "sim is NULL");
    int rc = collect_profile(s);
    if (rc != VOG_OK) return rc;
    for (int k = 0; k < nkinds && k < VOG_NUM_KINDS; ++k) {
        if (ms) ms[k] = s->ms[k];
        if (launches) launches[k] = s->launches[k];
    }
    return VOG_OK;
}

const char *vog_build_info(void) {
    return "libvog gfx950: radix-16 Stockham LDS FFT, paired real lines, integer-shift store, "
           "x-sweep on the v-fastest layout (XCD-ordered line tiles), rho row sums, "
           "v half-steps between steps composed in Fourier space (FP32)";
}

}  // extern "C"
