// Internal structures shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vog.h"

namespace vog {

constexpr int kDMax = 8;                 // Lagrange 2d+1 with d <= 8
constexpr int kTaps = 2 * kDMax + 2;     // 18 stencil offsets q = -8 .. 9
constexpr int kMaxBatch = 64;            // sims per grouped launch (field solve, reductions)
constexpr int kMaxSweepBatch = 128;      // sims per grouped sweep launch
constexpr int kRingCap = 4096;           // diagnostics records kept per sim
constexpr int kTile = 64;                // transpose tile edge
constexpr int kRhoCols = 16;             // x-columns per block of the partial-row reduction

// Per-sim constants and device pointers, stored in the sim's workspace.
// Written once at creation; kernels read it through a pointer.
struct SimDev {
    void *f;            // [nx][nv]  f or delta f, storage precision (v fastest)
    void *g;            // [nv][nx]  transposed copy used by the x-sweep
    double *E;          // [nx]      self-consistent field at the current time level
    double *Eeff;       // [nx]      advecting field E - E_app at the current time level
                        //           (driven sims only; the others advect with E)
    double *part;       // [nparts][nx] partial velocity sums: one row per tile of the
                        // tiled x-sweep, or per 64 velocities of the x -> v transpose
    double *rho;        // [nx]      charge density rho_i = int f dv
    double *mom;        // [nx][2]   per-line moment sums
    const void *tw_x;   // FFT twiddle rows for length nx, storage precision (re, im)
    const void *tw_v;   // FFT twiddle rows for length nv
    const void *eps_x;  // [nx / 16][10] exp(2 pi i t q / nx), symbol table for the x-sweep
    const void *eps_v;  // [nv / 16][10] exp(2 pi i t q / nv)
    const double *tw_x64;  // FP64 twiddle rows for length nx (field solve)
    const void *iden_x; // [nx] 1 / collocation symbol of the B-spline, storage precision (else null)
    const void *iden_v; // [nv]
    const double *invk;    // [nx] 1 / (nx k_m), k_m = 2 pi mt / L; 0 at m = 0, nx/2 (field solve)
    const void *feq_g;  // [n_feq][nv] component values f_g(v_j), storage precision
    const double *feq64;    // [nv] f_eq(v_j), FP64
    const double *drv_sc;   // [nx][2] sin(k x_j), cos(k x_j) of the drive wavenumber (else null)
    vog_diag *ring;     // [kRingCap]
    int nx, nv, d, deltaf, field_zero, n_feq, nparts, fp64, poisson, zero_mean, interp;
    double L, vmin, dx, dv, inv_dx, inv_dv;
    double feq_c[VOG_MAX_FEQ], feq_inv_s2[VOG_MAX_FEQ];
    double feq_const;   // dv * sum_j f_eq(v_j) (delta f), else 0
};

// Kernel argument of a grouped launch: up to kMaxBatch sims, each with its
// own scalar argument (dt or tau) and step bookkeeping.
struct Batch {
    int n;
    int pad_;
    const SimDev *s[kMaxBatch];
    double a[kMaxBatch];      // tau (v-sweep), dt (x-sweep)
    double t[kMaxBatch];      // time after the step (field solve)
    int64_t step[kMaxBatch];  // step number after the step (field solve)
    double drv_amp[kMaxBatch];  // emax k a(t) of the drive at t (field solve)
    double drv_ph[kMaxBatch];   // omega t (field solve)
};

// Kernel argument of a grouped sweep launch: up to kMaxSweepBatch sims, each
// with its tau (v-sweep) or dt (x-sweep).  Smaller than Batch, so that one
// launch covers twice as many sims within the 4 KB of kernel arguments.
struct SweepBatch {
    int n;
    int pad_;
    const SimDev *s[kMaxSweepBatch];
    double a[kMaxSweepBatch];
};

// Blocks of one launch over sims whose lines have different lengths: sim k
// owns the blocks first[k] .. first[k+1] - 1 and its lines have 2^lgn[k]
// points.
template <int CAP>
struct BlockMapT {
    int first[CAP + 1];
    int lgn[CAP];
};
using BlockMap = BlockMapT<kMaxBatch>;        // field solves
using SweepMap = BlockMapT<kMaxSweepBatch>;   // sweeps

enum Kind {
    K_SWEEP_V = 0, K_SWEEP_X = 1, K_T_VX = 2, K_T_XV = 3, K_FIELD = 4, K_MOMENTS = 5, K_RHO = 6,
    K_SWEEP_VV = 7
};

// Host-side launchers (defined in kernels.hip).
using LaunchFn = void (*)(const Batch &, int max_lines, hipStream_t);
using SweepFn = void (*)(const SweepBatch &, int max_lines, hipStream_t);
// kind 0: v-sweep, 1: x-sweep on the transposed copy, 2: two v half-steps
SweepFn sweep_launcher(bool fp64, int n, int kind);
// x-sweep on the v-fastest layout: lines per block (0 if not available) and launcher.
int fused_lines_per_block(bool fp64, int nx);
SweepFn fused_xsweep_launcher(bool fp64, int nx);
void launch_transpose(bool fp64, bool to_v, const Batch &b, int max_tiles, hipStream_t st);
LaunchFn field_launcher(int nx);  // nx = 2048, 4096
// One launch of FP32 v-sweeps (lines of 64 .. 4096 points) or FP32 x-sweeps on
// the v-fastest layout (64 .. 1024 points) over sims of mixed line lengths.
// Blocks per sim: sweep_blocks_mixed(vsweep, n, lines) for lines of n points
// (v-sweep: lines = nx; x-sweep: lines = nv).
int sweep_blocks_mixed(bool vsweep, int n, int lines);
bool sweep_mixed_ok(bool vsweep, int n);
// kind 0: v-sweeps, 1: x-sweeps, 2: two v half-steps (blocks as for 0)
void launch_sweep_mixed(int kind, const SweepBatch &b, const SweepMap &m, hipStream_t st);
// One launch of field solves over sims of 8 .. 1024 points in x, of one or
// several lengths (block k = sim k, m.lgn[k] = log2 nx).
bool field_mixed_ok(int nx);
void launch_field_mixed(const Batch &b, const BlockMap &m, hipStream_t st);
void launch_rho_v(bool fp64, const Batch &b, int max_nx, hipStream_t st);
void launch_rho_reduce(const SweepBatch &b, int max_nx, hipStream_t st);
void launch_moments(bool fp64, const Batch &b, int max_nx, hipStream_t st);
void launch_init(bool fp64, const SimDev *s, int cells, int nmodes, const double *amp,
                 const double *kx, const double *ph, hipStream_t st);
void launch_fill(void *p, size_t bytes, hipStream_t st);
// out[k] = 0 if sim k's diagnostics record of step b.step[k] says its field
// is not finite, else 1 (k < b.n).
void launch_finite_gather(const Batch &b, int *out, hipStream_t st);
// Device address of the library's fixed flag array (kNoAllocFlags ints) on
// `device`, which must be the current device; null if it cannot be found.
constexpr int kNoAllocFlags = VOG_NOALLOC_MAX_SIMS;
constexpr int kMaxDevices = 64;
int *noalloc_flags(int device);

}  // namespace vog
