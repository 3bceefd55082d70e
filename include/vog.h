/*
 * vog.h -- C ABI of libvog, a gfx950 (MI355X) implementation of the
 * semi-Lagrangian 1D x 1D Vlasov-Poisson split step of Mehrenberger et al.,
 * "Vlasov on GPU (VOG project)".
 *
 * Model (Introduction, eqs. (1)-(2)): df/dt + v df/dx + E df/dv = 0 with
 * dE/dx = int f dv - 1 and a zero-mean E, periodic in x on [0, L), and
 * periodic in v on [vmin, vmax) (Introduction: the velocity box is taken
 * periodic so that the v-advection is also circulant).
 *
 * Grid: x_i = i L / nx (i < nx) as in Section 1.2; v_j = vmin + j dv with
 * dv = (vmax - vmin) / nv (j < nv).  Host-visible f arrays are FP64 with
 * layout f[i * nv + j] (v fastest), nx * nv values.
 *
 * Conventions for every call:
 *   - Return 0 (VOG_OK) on success or a negative VOG_E* code; a message with
 *     details is available from vog_last_error() on the calling thread.
 *     Nothing is thrown across the ABI.
 *   - Host pointer arguments are read or written during the call only and
 *     are never retained.  The caller owns every host buffer.
 *   - Calls on one sim are not thread-safe; different sims may be used from
 *     different threads.
 *   - Device work is enqueued on the stream given to vog_create (a
 *     hipStream_t passed as void*; NULL means the null stream).  Calls that
 *     return data to the host synchronise that stream first.
 */
#ifndef VOG_H
#define VOG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define VOG_OK          0
#define VOG_EINVAL     -1  /* invalid argument or configuration */
#define VOG_ENOMEM     -2  /* workspace too small or device allocation failed */
#define VOG_EDEVICE    -3  /* a HIP runtime call failed */
#define VOG_ENONFINITE -4  /* the field of a sim became NaN or Inf */
#define VOG_EBUSY      -5  /* sim is not in a state that allows the call */

/* --------------------------------------------------------------- settings */
#define VOG_FP64_PLAIN   0  /* f stored and advected in FP64 */
#define VOG_FP32_DELTAF  1  /* delta f = f - f_eq stored and advected in FP32 (Section 3.1) */
#define VOG_FP64_DELTAF  2  /* delta f in FP64 */
#define VOG_FP32_PLAIN   3  /* f stored and advected in FP32 without the delta-f split: the
                               single-precision variant the paper compares against (Section 4.1) */

#define VOG_INTERP_LAGRANGE 0  /* Lagrange 2d+1 interpolation (Section 1.2) */
#define VOG_INTERP_BSPLINE  1  /* B-spline interpolation of odd degree k = 2d+1 (Section 1.2):
                                  A = M C^{-1}, C the collocation circulant */

#define VOG_POISSON_FOURIER   0  /* Fourier solve, mode 0 set to zero (Section 3.2) */
#define VOG_POISSON_TRAPEZOID 1  /* trapezoidal rule, with or without the zero-mean step (Section 3.2) */

#define VOG_FIELD_SELF_CONSISTENT 0
#define VOG_FIELD_ZERO            1  /* E held at zero: free streaming */

#define VOG_MAX_FEQ    4
#define VOG_MAX_DEGREE 17   /* odd degree 2d+1 with d <= 8: LAG17 (Section 4), B-splines up to degree 17 */
#define VOG_MIN_N      8
#define VOG_MAX_N      4096

typedef struct vog_config {
    int nx, nv;          /* powers of two in [8, 4096] */
    double L;            /* x in [0, L), L > 0 */
    double vmin, vmax;   /* vmin < vmax */
    int degree;          /* odd interpolation degree 2d+1, 1 <= degree <= min(17, nx-1, nv-1) */
    int precision;       /* VOG_FP64_PLAIN, VOG_FP32_DELTAF, VOG_FP64_DELTAF or VOG_FP32_PLAIN */
    int poisson;         /* VOG_POISSON_FOURIER or VOG_POISSON_TRAPEZOID */
    int field;           /* VOG_FIELD_SELF_CONSISTENT or VOG_FIELD_ZERO */
    /* f_eq(v) = sum_g feq_a[g] exp(-(v - feq_c[g])^2 / (2 feq_sigma[g]^2)),
     * 1 <= n_feq <= 4, feq_sigma > 0.  It is the background of
     * vog_init_perturbed and, for the delta-f precisions, the equilibrium of
     * Section 3.1.  Default: the unit Maxwellian. */
    int n_feq;
    double feq_a[VOG_MAX_FEQ], feq_c[VOG_MAX_FEQ], feq_sigma[VOG_MAX_FEQ];
    /* L2 norm and total energy (Section 4.2) are computed every
     * moments_every steps (0: never). */
    int moments_every;
    /* Trapezoidal solve only: 1 subtracts the mean of rho and of E (the
     * zero-mean modification of Section 3.2); 0 uses rho - 1 and E as
     * integrated from E_0 = 0. */
    int zero_mean;
    /* External drive of the KEEN-wave test (Section 4.3):
     *   E_app(t, x) = drive_emax drive_k a(t) sin(drive_k x - drive_omega t),
     *   a(t) = (0.5 (tanh((t - tl)/twl) - tanh((t - tr)/twr)) - eps) / (1 - eps),
     * eps the same bracket at t0.  The v-advection uses E - E_app (the first
     * half step at t^n, the second at t^{n+1}).  drive_emax = 0: no drive;
     * otherwise twl, twr > 0 and drive_k, drive_omega finite. */
    double drive_emax, drive_k, drive_omega, drive_t0, drive_tl, drive_tr, drive_twl, drive_twr;
    /* VOG_INTERP_LAGRANGE or VOG_INTERP_BSPLINE; both use the same 2d+2
     * taps per line, B-splines also divide by the collocation symbol. */
    int interp;
    /* 1: inside one vog_step / vog_step_batch call, the v half-step that
     * ends step n and the one that starts step n+1 (same field
     * E^{n+1} - E_app(t^{n+1})) run as one v-advection by dt (Section 1.1):
     * 2 sweeps per step instead of 3.  Every call still starts and ends
     * with a half step, so f is at a full time level between calls; results
     * differ from the unmerged scheme at the interpolation-error level and
     * depend on how a run is cut into calls.  L2 and energy are computed on
     * the last step of a call only. */
    int merge_v;
    /* Without merge_v, the closing v half-step of step n and the opening one
     * of step n+1 inside one call run in one launch.  0 (default): in the
     * FP32 precisions the two are composed in Fourier space (the kernel's
     * symbol applied twice, the first step's source term transformed beside
     * the lines, one inverse transform; Section 1.2 applied twice), which is
     * the same scheme with different rounding: results depend at the
     * rounding level on how a run is cut into calls (each cut closes and
     * reopens with single half steps).  1: the two half steps are transformed
     * one after the other, and f, E and the diagnostics of a call of n steps
     * are bitwise those of n single-step calls.  FP64 sims always behave as
     * with 1. */
    int bitwise_steps;
} vog_config;

/* One record per time step, written on the device by the field solve. */
typedef struct vog_diag {
    int64_t step;      /* step index n+1 of the state after the step */
    double t;          /* time after the step */
    double normE;      /* ||E||_2 = (dx sum_i E_i^2)^{1/2} (Section 4.1) */
    double rho0;       /* rho_hat_0 = (1/nx) sum_i rho_i: the mass (Section 4.1) */
    double abs_rho1;   /* |rho_hat_1|, rho_hat_m = (1/nx) sum_i rho_i e^{-2 pi i m i/nx} */
    double l2;         /* dx dv sum f^2, or NaN when not computed for this step */
    double energy;     /* dx dv sum f v^2/2 + dx/2 sum E^2 (Section 4.2), or NaN */
    int32_t finite;    /* 1 if every E_i is finite */
    int32_t reserved;
    double abs_rho_modes[7]; /* |rho_hat_m| for m = 1..7 (the mode history of Section 4.3) */
} vog_diag;

typedef struct vog_sim vog_sim;

/* Fills *cfg with a 64 x 128 weak-Landau-sized default: L = 4 pi,
 * v in [-6, 6), degree 17, FP64_PLAIN, Fourier Poisson, unit Maxwellian. */
void vog_config_default(vog_config *cfg);

/* Checks every field of *cfg; VOG_OK or VOG_EINVAL. */
int vog_config_validate(const vog_config *cfg);

/* Exact number of device bytes a sim of this configuration uses (f, a
 * transposed scratch copy when the x-sweep cannot run on the v-fastest
 * layout (nx < 64 or nv smaller than one tile of x-lines), field, partial
 * sums, tables, diagnostics ring).  Returns 0 for an invalid configuration. */
size_t vog_workspace_bytes(const vog_config *cfg);

/* Creates a sim on the current HIP device.  dev_workspace: device memory of
 * at least vog_workspace_bytes(cfg) bytes, 256-byte aligned, owned by the
 * caller, which must keep it alive until vog_destroy; or NULL, in which case
 * the library allocates and owns it.  hip_stream: the hipStream_t all work of
 * this sim is enqueued on (borrowed, must outlive the sim).  The state is
 * zero until vog_init_perturbed, vog_set_f or vog_set_state.  The tables are
 * uploaded asynchronously from copies the library keeps, so the call does not
 * wait for work already queued on the stream. */
int vog_create(const vog_config *cfg, void *dev_workspace, size_t bytes,
               void *hip_stream, vog_sim **out);

/* f0(x, v) = (1 + sum_m amp[m] cos(kx[m] x + phase[m])) f_eq(v), computed on
 * the device (the Landau and bump-on-tail initial data of Sections 4.1-4.2),
 * 0 <= nmodes <= 8.  Delta-f precisions store f0 - f_eq.  Then computes E^0
 * from f0 (Section 2: initial density, then the field) and resets the step
 * counter, the time and the diagnostics ring. */
int vog_init_perturbed(vog_sim *sim, int nmodes, const double *amp, const double *kx,
                       const double *phase);

/* Copies a full FP64 f (layout above: the distribution on the periodic
 * Nx x Nv phase-space grid of the Introduction and Section 1.2) to the
 * device; delta-f precisions store f - f_eq rounded to the storage precision
 * (Section 3.1).  Recomputes E from f (Section 2: density, then field) and
 * resets step counter, time and diagnostics.  host_f: nx*nv FP64 values,
 * owned by the caller and not retained.  VOG_EINVAL for a NULL argument. */
int vog_set_f(vog_sim *sim, const double *host_f);

/* Copies the current full f (the phase-space grid of Section 1.2, layout
 * above) to host FP64, f_eq added back for delta f (Section 3.1).  host_f:
 * nx*nv FP64 values, owned by the caller.  Synchronises the sim's stream.
 * VOG_EINVAL for a NULL argument. */
int vog_get_f(vog_sim *sim, double *host_f);

/* Copies the stored array (f or delta f, storage precision, same layout) to
 * host; elem_bytes receives 4 or 8.  host_buf holds nx*nv*elem_bytes bytes. */
int vog_get_raw(vog_sim *sim, void *host_buf, size_t bytes, int *elem_bytes);

/* Copies the self-consistent E at the current time level (nx FP64 values at
 * the nodes x_i = i dx; the field of the Poisson equation of Section 3.2 that
 * the time loop of Section 2 updates every step) to host.  host_E: owned by
 * the caller.  Synchronises the sim's stream.  VOG_EINVAL for a NULL
 * argument. */
int vog_get_E(vog_sim *sim, double *host_E);

/* Replaces E (nx FP64 values) without touching f; the advecting field becomes
 * E - E_app at the current time.  Used to drive a single v-advection with a
 * chosen field. */
int vog_set_E(vog_sim *sim, const double *host_E);

/* Enqueues nsteps Strang steps of size dt (Section 1.1):
 *   v-advection by dt/2 with E^n, x-advection by dt, field update
 *   E^{n+1} from rho = int f dv, v-advection by dt/2 with E^{n+1};
 * the last half step is not merged with the next step's first unless the
 * configuration sets merge_v.  Each constant advection is the circulant
 * product A u of Section 1.2 (Lagrange 2d+1 or B-spline coefficients),
 * applied as FFT -> multiply by the diagonal of A in Fourier space ->
 * inverse FFT.  With a drive, the v-advections use E - E_app.  Between two
 * steps of one call the closing half step and the next opening one run in
 * one launch, composed in Fourier space for FP32 sims unless the
 * configuration sets bitwise_steps (then, and for FP64 sims, f, E and the
 * diagnostics records are bitwise those of nsteps calls of one step).  The
 * same sequence of calls always gives the same bits.  Asynchronous: returns
 * after enqueueing.
 * dt > 0 and finite, nsteps >= 0 (0: no-op). */
int vog_step(vog_sim *sim, double dt, int nsteps);

/* nsteps Strang steps (Section 1.1, the time loop of Section 2) for nsims
 * sims at once, sim k with step dt[k], with
 * grouped launches of up to 128 sims per sweep and 64 per field solve: one
 * per kernel type and line length, and
 * for FP32 sims one per sweep covering all their line lengths (v-lines of
 * 64..4096 points, x-lines of 64..1024).  Every sim must use the stream of
 * sims[0], and no sim may appear twice.  Each sim's result is bitwise
 * identical to vog_step on that sim alone. */
int vog_step_batch(vog_sim *const *sims, int nsims, const double *dt, int nsteps);

/* Single sweeps, for testing the pieces of the step on their own:
 * which = 0: v-advection by tau = arg with the current E (Section 1.1, steps
 * 1 and 3; delta-f update of Section 3.1 for delta-f precisions);
 * which = 1: x-advection by dt = arg (step 2);
 * which = 2: recompute E from the current f (field update).
 * The step counter is not advanced. */
int vog_sweep(vog_sim *sim, int which, double arg);

/* Copies the diagnostics records written since the previous call (at most
 * cap, oldest first) to out; *n receives the count.  Records older than the
 * ring capacity (4096 steps) are dropped. */
int vog_get_diag(vog_sim *sim, vog_diag *out, int cap, int *n);

/* Checkpoint: the stored array, E, the advecting field, step counter and
 * time, bitwise. */
size_t vog_state_bytes(const vog_sim *sim);
int vog_get_state(vog_sim *sim, void *host_buf, size_t bytes);
int vog_set_state(vog_sim *sim, const void *host_buf, size_t bytes);

/* Step counter and time of the enqueued state. */
int vog_get_time(const vog_sim *sim, int64_t *step, double *t);

/* Waits for all work enqueued for the sim; VOG_ENONFINITE if the last
 * recorded field was not finite. */
int vog_sync(vog_sim *sim);

/* vog_sync for several sims that share one device and stream (a batch of
 * vog_step_batch): waits for the stream once and sets status[k] to VOG_OK or
 * VOG_ENONFINITE for sims[k], read from every sim's last diagnostics record
 * with one gather launch and one copy per up to 64 sims.  status: host
 * array of nsims ints, written on success.  The gather uses a small device
 * buffer the library allocates once per device; calls on one device are
 * serialised.  VOG_EINVAL for a NULL argument, nsims < 1 or sims that do not
 * share the device and stream. */
int vog_sync_batch(vog_sim *const *sims, int nsims, int *status);

/* vog_sync_batch without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as vog_sync_batch;
 * the flags are gathered into a fixed array of VOG_NOALLOC_MAX_SIMS ints in
 * the library's own device memory (one per GPU, held until the process
 * ends), every flag written before it is read.  nsims above
 * VOG_NOALLOC_MAX_SIMS is rejected with VOG_EINVAL.  Calls that overlap on
 * one GPU share that array and race; the library serialises calls made
 * through it, other users of the array must not overlap with them. */
#define VOG_NOALLOC_MAX_SIMS 1024
int vog_sync_batch_noalloc(vog_sim *const *sims, int nsims, int *status);

void vog_destroy(vog_sim *sim);

const char *vog_strerror(int code);
const char *vog_last_error(void);

/* Kernel timing with HIP events recorded on the sim's stream around every
 * launch of the sim (or of a batch led by it).  Kinds: 0 v-sweep, 1 x-sweep,
 * 2 transpose v->x, 3 transpose x->v with rho partial sums, 4 field solve,
 * 5 moments, 6 rho reduction, 7 two v half-steps in one launch (the closing
 * half-step of a step and the opening one of the next, Section 1.1).
 * vog_profile_read synchronises and returns, per kind, the summed
 * milliseconds and the number of launches since profiling was enabled. */
#define VOG_NUM_KINDS 8
int vog_profile_enable(vog_sim *sim, int on);
int vog_profile_read(vog_sim *sim, double *ms, int64_t *launches, int nkinds);

/* Library build identification (kernel variant string). */
const char *vog_build_info(void);

#ifdef __cplusplus
}
#endif
#endif /* VOG_H */
