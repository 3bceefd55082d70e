/*
 * CPU FP64 oracle for the 1D x 1D Vlasov-Poisson split step.
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, by the smoke check and by
 * the benchmark's CPU-baseline leg, never by the product library.
 *
 * What it computes, and where the paper defines it:
 *   - Strang splitting v(dt/2) -> x(dt) -> field update -> v(dt/2)
 *     (Section 1.1, steps 1-3; the last half step is merged with the next
 *     step's first one only when merge_v is set).
 *   - Each constant advection u_i <- pi u(x_i - c dt) as the circulant
 *     product A u with A = C(a_0 .. a_{N-1}) (Section 1.2, eq. of matrix A),
 *     beta = -c dt / dx = b + s with b integer and s in [0, 1), and the
 *     Lagrange 2d+1 coefficients a_{b+j} = prod_{k != j} (s - k) / (j - k),
 *     j = -d .. d+1.  Here the product is evaluated directly, as the sum over
 *     the 2d+2 nonzero entries of each row; no FFT is used.
 *   - The delta-f v-advection (Section 3.1): the advected perturbation plus
 *     f_eq(v - tau E) - f_eq(v), f_eq evaluated, not interpolated.
 *   - rho_i = dv sum_j f_ij (rectangle rule on the periodic v grid) and the
 *     Fourier Poisson solve with mode 0 set to zero (Section 3.2), which
 *     gives a zero-mean E.  The Nyquist mode is also set to zero.
 *   - Diagnostics of Section 4: ||E||_2, the mass rho_hat_0, |rho_hat_1|,
 *     the L2 norm of f and the total energy.
 *   - Variants: the trapezoidal field solve with or without the zero-mean
 *     modification (Section 3.2), the external drive of the KEEN-wave
 *     test (Section 4.3), which enters the v-advection as E - E_app, the
 *     B-spline interpolation A = M C^{-1} (Section 1.2) with the spline
 *     coefficients from a dense LU solve, and merged v half-steps
 *     (Section 1.1).
 */
#include "vp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double ORC_PI = 3.14159265358979323846264338327950288;

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static long wrap(long i, long n) {
    long r = i % n;
    return r < 0 ? r + n : r;
}

/* Lagrange 2d+1 coefficients (Section 1.2): w[j + d] for j = -d .. d+1. */
void orc_lagrange_weights(int d, double s, double *w) {
    for (int j = -d; j <= d + 1; ++j) {
        double p = 1.0;
        for (int k = -d; k <= d + 1; ++k)
            if (k != j) p *= (s - (double)k) / (double)(j - k);
        w[j + d] = p;
    }
}

/* beta = b + s with b integer and s in [0, 1) (Section 1.2). */
void orc_split_shift(double beta, long *b, double *s) {
    double fb = floor(beta);
    double r = beta - fb;
    if (r >= 1.0) { /* beta - floor(beta) rounded up to 1 */
        r = 0.0;
        fb += 1.0;
    }
    *b = (long)fb;
    *s = r;
}

/* First row a_0 .. a_{n-1} of the circulant matrix A (Section 1.2):
 * a_{(b+j) mod n} = w_j, all other entries zero. */
void orc_circulant_row(int n, int d, double beta, double *a) {
    long b;
    double s;
    double w[64];
    orc_split_shift(beta, &b, &s);
    orc_lagrange_weights(d, s, w);
    for (int k = 0; k < n; ++k) a[k] = 0.0;
    for (int j = -d; j <= d + 1; ++j) a[wrap(b + j, n)] += w[j + d];
}

/* out = A u for one line: out_i = sum_k A_{ik} u_k = sum_j w_j u_{(i+b+j) mod n}. */
static void advect_strided(int n, int d, long b, const double *w,
                           const double *u, long us, double *out, long os) {
    for (long i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int j = -d; j <= d + 1; ++j) acc += w[j + d] * u[wrap(i + b + j, n) * us];
        out[i * os] = acc;
    }
}

void orc_advect_line(int n, int d, double beta, const double *u, double *out) {
    long b;
    double s;
    double w[64];
    orc_split_shift(beta, &b, &s);
    orc_lagrange_weights(d, s, w);
    advect_strided(n, d, b, w, u, 1, out, 1);
}

/* ------------------------------------------------------------ B-splines */

/* B^k_0(x) on the unit mesh x_i = i, from the degree recurrence of
 * Section 1.2:
 *   B^0_0 = indicator of [0, 1),
 *   B^p_i(x) = (x - i)/p B^{p-1}_i(x) + (1 - (x - i - 1)/p) B^{p-1}_{i+1}(x).
 * B^k_0(x) needs B^{k-1}_0 and B^{k-1}_1 at x, which need B^{k-2}_{0..2}, and
 * so on down to B^0_{0..k}; level p keeps B^p_i(x) for i = 0 .. k - p. */
double orc_bspline(int k, double x) {
    double b[64];
    for (int i = 0; i <= k; ++i) b[i] = (x >= i && x < i + 1) ? 1.0 : 0.0;
    for (int p = 1; p <= k; ++p)
        for (int i = 0; i <= k - p; ++i)
            b[i] = (x - i) / p * b[i] + (1.0 - (x - i - 1.0) / p) * b[i + 1];
    return b[0];
}

/* Collocation matrix of the periodic spline interpolation on n nodes,
 * C = circulant(0, .., 0, B^k_0(x_1), .., B^k_0(x_k)) of Section 1.2:
 * the spline sum_l c_l B^k_0(x - l) takes the value sum_l c_l B^k_0(i - l)
 * at node i.  Factored in place as P C = L U (partial pivoting). */
static void bspline_collocation_lu(int n, int k, double *a, int *piv) {
    for (long i = 0; i < n; ++i)
        for (long l = 0; l < n; ++l) a[i * n + l] = 0.0;
    for (long i = 0; i < n; ++i)
        for (int j = 1; j <= k; ++j) a[i * n + wrap(i - j, n)] += orc_bspline(k, (double)j);
    for (int col = 0; col < n; ++col) {
        int p = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(a[(long)r * n + col]) > fabs(a[(long)p * n + col])) p = r;
        piv[col] = p;
        if (p != col)
            for (int l = 0; l < n; ++l) {
                double t = a[(long)col * n + l];
                a[(long)col * n + l] = a[(long)p * n + l];
                a[(long)p * n + l] = t;
            }
        for (int r = col + 1; r < n; ++r) {
            double m = a[(long)r * n + col] / a[(long)col * n + col];
            a[(long)r * n + col] = m;
            for (int l = col + 1; l < n; ++l) a[(long)r * n + l] -= m * a[(long)col * n + l];
        }
    }
}

/* Solves C x = rhs with the factors above; x may alias rhs. */
static void lu_solve(int n, const double *a, const int *piv, const double *rhs, double *x) {
    if (x != rhs) memcpy(x, rhs, sizeof(double) * n);
    /* the factorization swapped whole rows, multipliers included: permute
     * the right-hand side first, then substitute */
    for (int col = 0; col < n; ++col) {
        int p = piv[col];
        if (p != col) {
            double t = x[col];
            x[col] = x[p];
            x[p] = t;
        }
    }
    for (int col = 0; col < n; ++col)
        for (int r = col + 1; r < n; ++r) x[r] -= a[(long)r * n + col] * x[col];
    for (int r = n - 1; r >= 0; --r) {
        double acc = x[r];
        for (int l = r + 1; l < n; ++l) acc -= a[(long)r * n + l] * x[l];
        x[r] = acc / a[(long)r * n + r];
    }
}

/* One line of the B-spline advection A = M C^{-1} (Section 1.2): the spline
 * coefficients c solve C c = u, and the spline is evaluated at the feet
 * x_i + beta = x_{i+b} + s, where it equals
 *   sum_{j=0}^{k} B^k_0(x_{j+s}) c_{i+b-j}   (the entries m_{b-j} of M).
 * u and out are strided; work holds n doubles. */
static void bspline_line(int n, int k, long b, double s, const double *lu, const int *piv,
                         const double *u, long us, double *out, long os, double *work) {
    double m[64];
    for (int j = 0; j <= k; ++j) m[j] = orc_bspline(k, j + s);
    for (int i = 0; i < n; ++i) work[i] = u[(long)i * us];
    lu_solve(n, lu, piv, work, work);
    for (long i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int j = 0; j <= k; ++j) acc += m[j] * work[wrap(i + b - j, n)];
        out[i * os] = acc;
    }
}

void orc_advect_line_bspline(int n, int k, double beta, const double *u, double *out) {
    long b;
    double s;
    double *lu = (double *)malloc(sizeof(double) * (size_t)n * n);
    int *piv = (int *)malloc(sizeof(int) * n);
    double *work = (double *)malloc(sizeof(double) * n);
    orc_split_shift(beta, &b, &s);
    bspline_collocation_lu(n, k, lu, piv);
    bspline_line(n, k, b, s, lu, piv, u, 1, out, 1, work);
    free(lu);
    free(piv);
    free(work);
}

static double dx_of(const orc_cfg *c) { return c->L / c->nx; }
static double dv_of(const orc_cfg *c) { return (c->vmax - c->vmin) / c->nv; }
static double v_of(const orc_cfg *c, int j) { return c->vmin + j * dv_of(c); }
static double x_of(const orc_cfg *c, int i) { return i * dx_of(c); }

/* f_eq(v) = sum_g a_g exp(-(v - c_g)^2 / (2 sigma_g^2)); the unit Maxwellian of
 * Section 3.1 is one term with a = 1/sqrt(2 pi), c = 0, sigma = 1. */
double orc_feq(const orc_cfg *c, double v) {
    double acc = 0.0;
    for (int g = 0; g < c->n_feq; ++g) {
        double z = (v - c->feq_c[g]) / c->feq_sigma[g];
        acc += c->feq_a[g] * exp(-0.5 * z * z);
    }
    return acc;
}

/* f0 = (1 + sum_m amp_m cos(kx_m x + phase_m)) f_eq(v); delta f stores f0 - f_eq. */
void orc_init(const orc_cfg *c, int nmodes, const double *amp, const double *kx,
              const double *phase, double *f) {
    for (int i = 0; i < c->nx; ++i) {
        double p = 0.0;
        for (int m = 0; m < nmodes; ++m) p += amp[m] * cos(kx[m] * x_of(c, i) + phase[m]);
        for (int j = 0; j < c->nv; ++j) {
            double fe = orc_feq(c, v_of(c, j));
            f[(long)i * c->nv + j] = c->deltaf ? p * fe : (1.0 + p) * fe;
        }
    }
}

/* Lines of one sweep: nl lines of length n, line l starting at base + l ls
 * with element stride es; beta(l) gives the normalized shift of line l. */
typedef double (*beta_fn)(const orc_cfg *c, const double *E, double arg, int l);

static double beta_x(const orc_cfg *c, const double *E, double dt, int j) {
    (void)E;
    return -v_of(c, j) * dt / dx_of(c);
}

static double beta_v(const orc_cfg *c, const double *E, double tau, int i) {
    const double Ei = c->field_zero ? 0.0 : E[i];
    return -Ei * tau / dv_of(c);
}

static void advect_lines(const orc_cfg *c, int n, int nl, long ls, long es, beta_fn beta,
                         const double *E, double arg, const double *f, double *out) {
    const int d = (c->degree - 1) / 2;
    double *lu = NULL;
    int *piv = NULL;
    if (c->interp == 1) {
        lu = (double *)malloc(sizeof(double) * (size_t)n * n);
        piv = (int *)malloc(sizeof(int) * n);
        bspline_collocation_lu(n, c->degree, lu, piv);
    }
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * n);
#pragma omp for schedule(static)
        for (int l = 0; l < nl; ++l) {
            long b;
            double s;
            double w[64];
            orc_split_shift(beta(c, E, arg, l), &b, &s);
            if (c->interp == 1) {
                bspline_line(n, c->degree, b, s, lu, piv, f + l * ls, es, out + l * ls, es, work);
            } else {
                orc_lagrange_weights(d, s, w);
                advect_strided(n, d, b, w, f + l * ls, es, out + l * ls, es);
            }
        }
        free(work);
    }
    free(lu);
    free(piv);
}

/* x-advection by dt (Section 1.1, step 2): line j (fixed v_j) is advected
 * with speed v_j, beta = -v_j dt / dx. */
void orc_advect_x(const orc_cfg *c, double dt, const double *f, double *out) {
    advect_lines(c, c->nx, c->nv, 1, c->nv, beta_x, NULL, dt, f, out);
}

/* v-advection by tau with field E (Section 1.1, steps 1 and 3): line i (fixed
 * x_i) is advected with speed E_i, beta = -E_i tau / dv.  delta f form
 * (Section 3.1): the advected perturbation plus f_eq(v - tau E_i) - f_eq(v),
 * f_eq evaluated. */
void orc_advect_v(const orc_cfg *c, const double *E, double tau, const double *f, double *out) {
    advect_lines(c, c->nv, c->nx, c->nv, 1, beta_v, E, tau, f, out);
    if (c->deltaf) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < c->nx; ++i) {
            const double Ei = c->field_zero ? 0.0 : E[i];
            double *o = out + (long)i * c->nv;
            for (int j = 0; j < c->nv; ++j) {
                double v = v_of(c, j);
                o[j] += orc_feq(c, v - tau * Ei) - orc_feq(c, v);
            }
        }
    }
}

/* rho_i = dv sum_j f_ij, the velocity integral by the rectangle rule on the
 * periodic grid; in delta f form dv sum_j (delta f_ij + f_eq(v_j)). */
void orc_rho(const orc_cfg *c, const double *f, double *rho) {
    const double dv = dv_of(c);
    double feq_sum = 0.0;
    if (c->deltaf)
        for (int j = 0; j < c->nv; ++j) feq_sum += orc_feq(c, v_of(c, j));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < c->nx; ++i) {
        double acc = 0.0;
        for (int j = 0; j < c->nv; ++j) acc += f[(long)i * c->nv + j];
        rho[i] = dv * (acc + feq_sum);
    }
}

/* Fourier Poisson solve dE/dx = rho - mean(rho) by direct DFT (Section 3.2):
 * rho_hat_m = sum_i rho_i e^{-2 pi i m i / nx}; E_hat_0 = E_hat_{nx/2} = 0,
 * E_hat_m = rho_hat_m / (i k_m), k_m = 2 pi mt / L with mt the signed index;
 * E_i = Re (1/nx) sum_m E_hat_m e^{+2 pi i m i / nx}. */
void orc_poisson(const orc_cfg *c, const double *rho, double *E) {
    const int n = c->nx;
    double *cs = (double *)malloc(sizeof(double) * 2 * n);
    double *sn = cs + n;
    double *Er = (double *)malloc(sizeof(double) * 2 * n);
    double *Ei = Er + n;
    for (int k = 0; k < n; ++k) {
        cs[k] = cos(2.0 * ORC_PI * k / n);
        sn[k] = sin(2.0 * ORC_PI * k / n);
    }
#pragma omp parallel for schedule(static)
    for (int m = 0; m < n; ++m) {
        double re = 0.0, im = 0.0;
        for (int i = 0; i < n; ++i) {
            long k = ((long)m * i) % n;
            re += rho[i] * cs[k];
            im -= rho[i] * sn[k];
        }
        if (m == 0 || 2 * m == n) {
            Er[m] = 0.0;
            Ei[m] = 0.0;
        } else {
            int mt = (2 * m < n) ? m : m - n;
            double km = 2.0 * ORC_PI * mt / c->L;
            /* (re + i im) / (i km) = (im - i re) / km */
            Er[m] = im / km;
            Ei[m] = -re / km;
        }
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int m = 0; m < n; ++m) {
            long k = ((long)m * i) % n;
            acc += Er[m] * cs[k] - Ei[m] * sn[k];
        }
        E[i] = acc / n;
    }
    free(cs);
    free(Er);
}

/* Trapezoidal field solve (Section 3.2): rho~ = rho - mean(rho) (zero_mean)
 * or rho - 1; E~_0 = 0, E~_{k+1} = E~_k + dx (rho~_k + rho~_{k+1}) / 2 for
 * k = 0 .. nx-2; with zero_mean, E = E~ - mean(E~), else E = E~. */
static void poisson_trapezoid(const orc_cfg *c, const double *rho, double *E) {
    const int n = c->nx;
    const double dx = dx_of(c);
    double mean = 1.0;
    if (c->zero_mean) {
        mean = 0.0;
        for (int i = 0; i < n; ++i) mean += rho[i];
        mean /= n;
    }
    E[0] = 0.0;
    for (int k = 0; k + 1 < n; ++k)
        E[k + 1] = E[k] + dx * 0.5 * ((rho[k] - mean) + (rho[k + 1] - mean));
    if (c->zero_mean) {
        double em = 0.0;
        for (int i = 0; i < n; ++i) em += E[i];
        em /= n;
        for (int i = 0; i < n; ++i) E[i] -= em;
    }
}

/* E from rho with the configured solve (zero for free streaming). */
void orc_solve(const orc_cfg *c, const double *rho, double *E) {
    if (c->field_zero)
        for (int i = 0; i < c->nx; ++i) E[i] = 0.0;
    else if (c->poisson == 1)
        poisson_trapezoid(c, rho, E);
    else
        orc_poisson(c, rho, E);
}

void orc_field(const orc_cfg *c, const double *f, double *E, double *rho) {
    orc_rho(c, f, rho);
    orc_solve(c, rho, E);
}

/* Drive envelope (Section 4.3):
 * a(t) = (0.5 (tanh((t - tL)/twL) - tanh((t - tR)/twR)) - eps) / (1 - eps),
 * eps the same bracket at t0, so that a(t0) = 0. */
double orc_drive_amplitude(const orc_cfg *c, double t) {
    double eps = 0.5 * (tanh((c->drive_t0 - c->drive_tl) / c->drive_twl) -
                        tanh((c->drive_t0 - c->drive_tr) / c->drive_twr));
    double br = 0.5 * (tanh((t - c->drive_tl) / c->drive_twl) - tanh((t - c->drive_tr) / c->drive_twr));
    return (br - eps) / (1.0 - eps);
}

/* E_app(t, x) = emax k a(t) sin(k x - omega t). */
double orc_drive(const orc_cfg *c, double t, double x) {
    if (c->drive_emax == 0.0) return 0.0;
    return c->drive_emax * c->drive_k * orc_drive_amplitude(c, t) *
           sin(c->drive_k * x - c->drive_omega * t);
}

/* |rho_hat_m| for m = 1 .. nmodes, rho_hat_m = (1/nx) sum_i rho_i e^{-2 pi i m i / nx}. */
void orc_rho_modes(const orc_cfg *c, const double *rho, int nmodes, double *abs_modes) {
    const int n = c->nx;
    for (int m = 1; m <= nmodes; ++m) {
        double re = 0.0, im = 0.0;
        for (int i = 0; i < n; ++i) {
            long k = ((long)m * i) % n;
            re += rho[i] * cos(2.0 * ORC_PI * k / n);
            im -= rho[i] * sin(2.0 * ORC_PI * k / n);
        }
        abs_modes[m - 1] = sqrt(re * re + im * im) / n;
    }
}

/* v-advection with the field E - E_app(t, x_i). */
static void advect_v_driven(const orc_cfg *c, const double *E, double t, double tau,
                            const double *f, double *out, double *Etot) {
    for (int i = 0; i < c->nx; ++i)
        Etot[i] = (c->field_zero ? 0.0 : E[i]) - orc_drive(c, t, x_of(c, i));
    orc_cfg cc = *c;
    cc.field_zero = 0;
    orc_advect_v(&cc, Etot, tau, f, out);
}

/* v-advection by tau with the field E - E_app(t, x_i) (plain E without a
 * drive). */
static void advect_v_at(const orc_cfg *c, const double *E, double t, double tau,
                        const double *f, double *out, double *Etot) {
    if (c->drive_emax != 0.0) advect_v_driven(c, E, t, tau, f, out, Etot);
    else orc_advect_v(c, E, tau, f, out);
}

/* One Strang step (Section 1.1) from time t.  f, E hold f^n, E^n on entry
 * and f^{n+1}, E^{n+1} on exit; rho receives the density the new field was
 * solved from; tmp has nx*nv doubles.  With a drive, the first half step
 * uses E^n - E_app(t^n) and the second E^{n+1} - E_app(t^{n+1}). */
void orc_step(const orc_cfg *c, double t, double dt, double *f, double *E, double *rho, double *tmp) {
    const long cells = (long)c->nx * c->nv;
    double *Etot = (double *)malloc(sizeof(double) * c->nx);
    advect_v_at(c, E, t, 0.5 * dt, f, tmp, Etot);
    orc_advect_x(c, dt, tmp, f);
    orc_field(c, f, E, rho);
    advect_v_at(c, E, t + dt, 0.5 * dt, f, tmp, Etot);
    memcpy(f, tmp, sizeof(double) * cells);
    free(Etot);
}

/* ||E||_2 = (dx sum E^2)^{1/2}; rho_hat_0 = mean rho; |rho_hat_1| with
 * rho_hat_m = (1/nx) sum_i rho_i e^{-2 pi i m i / nx}. */
void orc_diag_field(const orc_cfg *c, const double *rho, const double *E, double *out3) {
    const int n = c->nx;
    double e2 = 0.0, r0 = 0.0, r1r = 0.0, r1i = 0.0;
    for (int i = 0; i < n; ++i) {
        e2 += E[i] * E[i];
        r0 += rho[i];
        r1r += rho[i] * cos(2.0 * ORC_PI * i / n);
        r1i -= rho[i] * sin(2.0 * ORC_PI * i / n);
    }
    out3[0] = sqrt(dx_of(c) * e2);
    out3[1] = r0 / n;
    out3[2] = sqrt(r1r * r1r + r1i * r1i) / n;
}

/* L2 = dx dv sum f^2 and total energy = dx dv sum f v^2 / 2 + dx/2 sum E^2
 * (Section 4.2), with f the full distribution (f_eq added back for delta f). */
void orc_diag_moments(const orc_cfg *c, const double *f, const double *E, double *out2) {
    const double dx = dx_of(c), dv = dv_of(c);
    double l2 = 0.0, ek = 0.0, ee = 0.0;
    for (int i = 0; i < c->nx; ++i) {
        for (int j = 0; j < c->nv; ++j) {
            double v = v_of(c, j);
            double fij = f[(long)i * c->nv + j] + (c->deltaf ? orc_feq(c, v) : 0.0);
            l2 += fij * fij;
            ek += fij * v * v;
        }
        ee += E[i] * E[i];
    }
    out2[0] = dx * dv * l2;
    out2[1] = 0.5 * dx * dv * ek + 0.5 * dx * ee;
}

/* nsteps Strang steps from time t0; diag (3 doubles per step, may be NULL)
 * receives ||E^{n+1}||_2, rho_hat_0 and |rho_hat_1| after each step. */
/* nsteps Strang steps from time t0.  With merge_v, the half step that ends
 * step n and the half step that starts step n+1 use the same field
 * E^{n+1} - E_app(t^{n+1}), so they are applied as one v-advection by dt
 * (Section 1.1); the run still starts and ends with a half step, so f is at
 * a full time level on return. */
void orc_run(const orc_cfg *c, double t0, double dt, int nsteps, double *f, double *E, double *diag) {
    const long cells = (long)c->nx * c->nv;
    double *tmp = (double *)malloc(sizeof(double) * cells);
    double *rho = (double *)malloc(sizeof(double) * c->nx);
    double *Etot = (double *)malloc(sizeof(double) * c->nx);
    for (int n = 0; n < nsteps; ++n) {
        const double t = t0 + n * dt;
        if (!c->merge_v) {
            orc_step(c, t, dt, f, E, rho, tmp);
        } else {
            if (n == 0) {
                advect_v_at(c, E, t, 0.5 * dt, f, tmp, Etot);
                memcpy(f, tmp, sizeof(double) * cells);
            }
            orc_advect_x(c, dt, f, tmp);
            orc_field(c, tmp, E, rho);
            advect_v_at(c, E, t + dt, n == nsteps - 1 ? 0.5 * dt : dt, tmp, f, Etot);
        }
        if (diag) orc_diag_field(c, rho, E, diag + 3L * n);
    }
    free(tmp);
    free(rho);
    free(Etot);
}
