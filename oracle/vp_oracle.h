/*
 * CPU FP64 oracle for the 1D x 1D Vlasov-Poisson split step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU-baseline timing can check the HIP library against a
 * plain, slow, obviously correct computation.  The product path never links,
 * loads or calls it.  It shares no code, header, table or constant with the
 * HIP library.
 *
 * Every advection is the direct circulant product of the paper's Lagrange
 * 2d+1 interpolation, or of its B-spline interpolation by a dense solve of
 * the collocation system (Section 1.2): no FFT is used anywhere.  The Poisson
 * solve is a direct O(Nx^2) DFT with mode 0 (and the Nyquist mode) set to
 * zero (Section 3.2, Fourier variant).
 *
 * Layout of f: f[ix * nv + jv], v fastest.  x_i = i L / nx for i < nx,
 * v_j = vmin + j (vmax - vmin) / nv for j < nv (both periodic).
 */
#ifndef VP_ORACLE_H
#define VP_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_FEQ 4

typedef struct {
    int nx, nv;
    double L, vmin, vmax;
    int degree;        /* odd, 2d+1 */
    int deltaf;        /* 0: f is stored and advected; 1: delta f = f - f_eq */
    int field_zero;    /* 1: E is held at zero (free streaming) */
    int n_feq;
    double feq_a[ORC_MAX_FEQ], feq_c[ORC_MAX_FEQ], feq_sigma[ORC_MAX_FEQ];
    int poisson;       /* 0: Fourier; 1: trapezoidal rule */
    int zero_mean;     /* trapezoidal only: 1 subtracts mean(rho) and mean(E) */
    /* external drive E_app(t, x) = emax k a(t) sin(k x - omega t) (Section 4.3);
     * emax = 0 switches it off */
    double drive_emax, drive_k, drive_omega, drive_t0, drive_tl, drive_tr, drive_twl, drive_twr;
    int interp;        /* 0: Lagrange 2d+1; 1: B-spline of degree k = degree (Section 1.2) */
    int merge_v;       /* 1: orc_run merges the v half-steps of consecutive steps (Section 1.1) */
} orc_cfg;

int orc_num_threads(void);
void orc_set_num_threads(int n);

void orc_lagrange_weights(int d, double s, double *w);
void orc_split_shift(double beta, long *b, double *s);
void orc_circulant_row(int n, int d, double beta, double *a);
void orc_advect_line(int n, int d, double beta, const double *u, double *out);

double orc_bspline(int k, double x);
void orc_advect_line_bspline(int n, int k, double beta, const double *u, double *out);

double orc_feq(const orc_cfg *c, double v);
void orc_init(const orc_cfg *c, int nmodes, const double *amp, const double *kx,
              const double *phase, double *f);

void orc_advect_x(const orc_cfg *c, double dt, const double *f, double *out);
void orc_advect_v(const orc_cfg *c, const double *E, double tau, const double *f, double *out);
void orc_rho(const orc_cfg *c, const double *f, double *rho);
void orc_poisson(const orc_cfg *c, const double *rho, double *E);
void orc_solve(const orc_cfg *c, const double *rho, double *E);
void orc_field(const orc_cfg *c, const double *f, double *E, double *rho);

double orc_drive_amplitude(const orc_cfg *c, double t);
double orc_drive(const orc_cfg *c, double t, double x);
void orc_step(const orc_cfg *c, double t, double dt, double *f, double *E, double *rho, double *tmp);
void orc_run(const orc_cfg *c, double t0, double dt, int nsteps, double *f, double *E, double *diag);
void orc_rho_modes(const orc_cfg *c, const double *rho, int nmodes, double *abs_modes);

void orc_diag_field(const orc_cfg *c, const double *rho, const double *E, double *out3);
void orc_diag_moments(const orc_cfg *c, const double *f, const double *E, double *out2);

#ifdef __cplusplus
}
#endif
#endif
