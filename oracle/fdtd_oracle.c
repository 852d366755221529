/*
 * FP64 CPU oracle for the two-dimensional TMz (S-polarisation) and TEz
 * (P-polarisation) FDTD method of
 * "Full-Wave Optical Modeling of Leaf Internal Light Scattering Dynamics with
 * Potential Applications for Early Detection of Foliar Fungal Disease"
 * (Lee & Na, arXiv 2512.17132).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant generator with the GPU library.
 *
 * Conventions (SI units, written in the paper's own notation):
 *   - Yee lattice of Sec. 2.3: Ez at cell centres ((i+1/2)h, (j+1/2)h), Hx on
 *     the bottom edge ((i+1/2)h, jh), Hy on the left edge (ih, (j+1/2)h).
 *     Arrays are row-major [j][i], x fastest, i in [0,nx), j in [0,ny), j = 0 at
 *     the bottom.  Light enters at the top and travels towards -y (Sec. 2.1).
 *   - Time stepping of Sec. 2.3, eqs. 18-20, in the paper's order: the
 *     electric field lives at half-integer times, so step n advances
 *     Ez^{n-1/2} -> Ez^{n+1/2} with H^n, then H^n -> H^{n+1} with Ez^{n+1/2}.
 *   - Periodic x by index wrapping (Sec. 2.4, eq. 22).
 *   - Absorbing layers at top and bottom: convolutional PML (one of the PML
 *     variants Sec. 2.4 lists) with polynomial sigma grading.  Behind them the
 *     tangential H is zero (Hx = 0 on the rows y = 0 and y = ny*h).
 *   - TF/SF plane wave of Sec. 2.5 on one horizontal line: Ez rows j <= j_src
 *     are total field, Hx rows j >= j_src+1 and Ez rows j > j_src are
 *     scattered field.  The incident fields come from a 1D auxiliary vacuum
 *     grid with the same h and dt (orc_incident).
 *   - Monitors of Sec. 2.6, eqs. 29-34, with a least-squares tone fit and
 *     discrete-flux order weights (orc_spectra).
 *
 *   - Dispersive labels (Sec. 2.2's Lorentz-Drude alternative): polarisation
 *     ADEs, a pulsed source and multi-frequency monitors (orc_run_ade; in TEz
 *     orc_run_te_ade, where an edge's permittivity is the mean of its two
 *     cells').
 *
 * Readings of places where the paper is garbled or silent are listed at each
 * function.  Every function is a literal loop nest; nothing is tiled, fused or
 * reordered.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* SI constants.  c is exact; mu0 is the CODATA 2018 value; eps0 = 1/(mu0 c^2). */
static const double ORC_C0 = 299792458.0;
static const double ORC_MU0 = 1.25663706212e-6;
static const double ORC_PI = 3.14159265358979323846;

static double orc_eps0(void) { return 1.0 / (ORC_MU0 * ORC_C0 * ORC_C0); }
static double orc_eta0(void) { return ORC_MU0 * ORC_C0; }

/* Problem description shared by every oracle entry point. */
typedef struct {
    int32_t nx, ny;        /* cells; x periodic, y includes both absorbing layers */
    int32_t n_pml;         /* CPML cells at the bottom and at the top            */
    int32_t j_src;         /* last total-field Ez row of the TF/SF line          */
    int32_t j_ref;         /* reflection monitor row (scattered-field region)    */
    int32_t j_trn;         /* transmission monitor row (below the structure)     */
    int32_t n_steps;       /* time steps in a full run                            */
    int32_t dft_start;     /* first step whose Ez^{n+1/2} enters the monitors    */
    int32_t aux_pad;       /* 1D grid: vacuum cells on each side of the TF/SF row */
    int32_t aux_pml;       /* 1D grid: absorbing cells at each end               */
    int32_t aux_src_off;   /* 1D grid: source cell above the TF/SF row           */
    int32_t literal_orders;/* 1: paper-literal R/T (continuous cutoff, unit weights) */
    int32_t polarization;  /* 0: TMz (S), fields Ez, Hx, Hy; 1: TEz (P), fields Hz, Ex, Ey */
    double h;              /* grid spacing, m                                     */
    double courant;        /* S = c dt sqrt(2)/h, in (0,1]                         */
    double lambda0;        /* vacuum wavelength, m                                */
    double ramp_periods;   /* raised-cosine ramp length in source periods         */
    double cpml_order;     /* polynomial grading order m                          */
    double cpml_sigma_fac; /* sigma_max = fac*(m+1)/(eta0*h)                      */
    double cpml_alpha_fac; /* alpha_max = fac*omega*eps0                          */
    double cpml_kappa_max; /* kappa at the outer edge                             */
} orc_problem;

/* ------------------------------------------------------------------------- */
/* Time step and material coefficients                                       */
/* ------------------------------------------------------------------------- */

/* CFL bound of Sec. 2.3: dt <= 1/(c sqrt(1/h^2 + 1/h^2)) = h/(c sqrt 2); the run
 * uses the fraction S of it. */
double orc_time_step(double h, double courant)
{
    return courant / (ORC_C0 * sqrt(1.0 / (h * h) + 1.0 / (h * h)));
}

double orc_omega(const orc_problem* p) { return 2.0 * ORC_PI * ORC_C0 / p->lambda0; }

/* Eqs. 1-2: eps_r = n^2 - k^2, sigma = 2 omega eps0 n k.  Eq. 17: Ce and the
 * curl coefficient.  Reading: eq. 17's Ch lacks the factor dt/(eps0 eps_r) that
 * eqs. 15 and 18 need for dimensional consistency, so the curl coefficient is
 *   Cb = (dt/(eps0 eps_r)) / (1 + sigma dt/(2 eps0 eps_r)),
 * and the E update is Ez <- Ce Ez + Cb [ (dHy - dHx)/h ].
 * out = {eps_r, sigma, Ce, Cb}. */
void orc_material(double n, double k, double omega, double dt, double out[4])
{
    const double eps0 = orc_eps0();
    const double eps_r = n * n - k * k;
    const double sigma = 2.0 * omega * eps0 * n * k;
    const double loss = sigma * dt / (2.0 * eps0 * eps_r);
    out[0] = eps_r;
    out[1] = sigma;
    out[2] = (1.0 - loss) / (1.0 + loss);
    out[3] = (dt / (eps0 * eps_r)) / (1.0 + loss);
}

/* Same coefficients from (eps_r, sigma) directly; used for per-pixel eps_r. */
void orc_material_eps(double eps_r, double sigma, double dt, double out[2])
{
    const double eps0 = orc_eps0();
    const double loss = sigma * dt / (2.0 * eps0 * eps_r);
    out[0] = (1.0 - loss) / (1.0 + loss);
    out[1] = (dt / (eps0 * eps_r)) / (1.0 + loss);
}

/* Per-pixel (Ce, Cb) from a label map and a per-label (n,k) table. */
void orc_pixel_coefficients(const orc_problem* p, const uint8_t* labels, int32_t n_labels,
                            const double* nk, double* ce, double* cb)
{
    const double dt = orc_time_step(p->h, p->courant);
    const double omega = orc_omega(p);
    const size_t ncell = (size_t)p->nx * (size_t)p->ny;
    for (size_t c = 0; c < ncell; ++c) {
        const int L = labels[c];
        double m[4];
        (void)n_labels;
        orc_material(nk[2 * L], nk[2 * L + 1], omega, dt, m);
        ce[c] = m[2];
        cb[c] = m[3];
    }
}

/* ------------------------------------------------------------------------- */
/* Convolutional PML coefficients                                            */
/* ------------------------------------------------------------------------- */

/* Recursive-convolution PML (the paper uses split-field PML and gives no
 * parameters; the convolutional form is one of the alternatives it lists).
 * A field sample at depth rho (cells, measured from the inner face of the
 * layer towards the outer wall, 0 <= rho <= d) gets
 *   sigma = sigma_max (rho/d)^m,  kappa = 1 + (kappa_max-1)(rho/d)^m,
 *   alpha = alpha_max (1 - rho/d),
 *   b = exp(-(sigma/kappa + alpha) dt/eps0),
 *   c = sigma (b - 1) / (sigma kappa + kappa^2 alpha).
 * out = {b, c, 1/kappa}.  rho <= 0 means outside the layer: {0, 0, 1}. */
static void orc_cpml_at(const orc_problem* p, double rho, int32_t d, double out[3])
{
    if (rho <= 0.0 || d <= 0) {
        out[0] = 0.0; out[1] = 0.0; out[2] = 1.0;
        return;
    }
    const double eps0 = orc_eps0();
    const double dt = orc_time_step(p->h, p->courant);
    const double m = p->cpml_order;
    const double x = rho / (double)d;
    const double sigma_max = p->cpml_sigma_fac * (m + 1.0) / (orc_eta0() * p->h);
    const double alpha_max = p->cpml_alpha_fac * orc_omega(p) * eps0;
    const double sigma = sigma_max * pow(x, m);
    const double kappa = 1.0 + (p->cpml_kappa_max - 1.0) * pow(x, m);
    const double alpha = alpha_max * (1.0 - x);
    const double b = exp(-(sigma / kappa + alpha) * dt / eps0);
    const double c = (sigma > 0.0) ? sigma * (b - 1.0) / (sigma * kappa + kappa * kappa * alpha) : 0.0;
    out[0] = b;
    out[1] = c;
    out[2] = 1.0 / kappa;
}

/* Depth of an Ez sample (y = j+1/2) and of an Hx sample (y = j) in the layers
 * of a column of ny cells with d-cell layers at both ends. */
static double orc_depth_ez(int32_t j, int32_t ny, int32_t d)
{
    const double y = j + 0.5;
    if (y < d) return d - y;
    if (y > ny - d) return y - (ny - d);
    return 0.0;
}
static double orc_depth_hx(int32_t j, int32_t ny, int32_t d)
{
    const double y = j;
    if (y < d) return d - y;
    if (y > ny - d) return y - (ny - d);
    return 0.0;
}

/* Profile arrays for the 2D grid: per row j, {b, c, 1/kappa} for Ez and Hx. */
void orc_cpml_profiles(const orc_problem* p, double* ez_prof, double* hx_prof)
{
    for (int32_t j = 0; j < p->ny; ++j) {
        orc_cpml_at(p, orc_depth_ez(j, p->ny, p->n_pml), p->n_pml, &ez_prof[3 * j]);
        orc_cpml_at(p, orc_depth_hx(j, p->ny, p->n_pml), p->n_pml, &hx_prof[3 * j]);
    }
}

/* ------------------------------------------------------------------------- */
/* Incident plane wave (Sec. 2.5)                                            */
/* ------------------------------------------------------------------------- */

/* Source envelope: raised-cosine ramp over ramp_periods periods, then 1. */
static double orc_ramp(const orc_problem* p, double t)
{
    const double tr = p->ramp_periods * p->lambda0 / ORC_C0;
    if (tr <= 0.0 || t >= tr) return 1.0;
    if (t <= 0.0) return 0.0;
    return 0.5 * (1.0 - cos(ORC_PI * t / tr));
}

/* The normally incident wave of Sec. 2.5 is produced by a 1D vacuum Yee grid
 * with the same h and dt.  At normal incidence an x-uniform field on the 2D
 * grid obeys exactly this 1D recurrence, so the TF/SF line leaks nothing.
 *
 * 1D grid: cells k in [0, M), M = 2*(aux_pml + aux_pad) + 1; cell k is 2D row
 * j = k + (j_src - aux_pml - aux_pad).  E1[k] at y = k+1/2, H1[k] at y = k with
 * H1[0] = H1[M] = 0.  Both ends carry aux_pml absorbing cells graded like the
 * 2D layers.  A soft source adds ramp(t) sin(omega t), t = (n+1/2) dt, to the
 * cell aux_src_off above the TF/SF row after each E update, so the wave that
 * reaches the TF/SF row travels towards -y.
 *
 * Recorded per step n:  h_inc[n] = H1 on edge j_src+1 at time n (used by the
 * E update of step n);  e_inc[n] = E1 at row j_src at time n+1/2 (used by the
 * H update of step n and as the incident reference of the monitors). */
int orc_incident(const orc_problem* p, double* e_inc, double* h_inc)
{
    const int32_t P = p->aux_pml, pad = p->aux_pad;
    const int32_t M = 2 * (P + pad) + 1;
    const int32_t ks = P + pad;          /* TF/SF row in the 1D grid */
    const int32_t ksrc = ks + p->aux_src_off;
    if (P < 1 || pad < 2 || p->aux_src_off < 1 || ksrc >= M - P) return -1;
    const double eps0 = orc_eps0();
    const double dt = orc_time_step(p->h, p->courant);
    const double omega = orc_omega(p);
    double* e1 = calloc((size_t)M, sizeof(double));
    double* h1 = calloc((size_t)M + 1, sizeof(double));
    double* pe = calloc((size_t)M, sizeof(double));
    double* ph = calloc((size_t)M + 1, sizeof(double));
    double* pre = malloc(sizeof(double) * 3 * (size_t)M);
    double* prh = malloc(sizeof(double) * 3 * ((size_t)M + 1));
    if (!e1 || !h1 || !pe || !ph || !pre || !prh) {
        free(e1); free(h1); free(pe); free(ph); free(pre); free(prh);
        return -2;
    }
    for (int32_t k = 0; k < M; ++k) orc_cpml_at(p, orc_depth_ez(k, M, P), P, &pre[3 * k]);
    for (int32_t k = 0; k <= M; ++k) orc_cpml_at(p, orc_depth_hx(k, M, P), P, &prh[3 * k]);

    for (int32_t n = 0; n < p->n_steps; ++n) {
        h_inc[n] = h1[ks + 1];
        /* E update (vacuum: Ce = 1, Cb = dt/eps0) */
        for (int32_t k = 0; k < M; ++k) {
            const double dh = h1[k + 1] - h1[k];
            double term = dh * pre[3 * k + 2] / p->h;
            if (pre[3 * k + 1] != 0.0) {
                pe[k] = pre[3 * k] * pe[k] + pre[3 * k + 1] * dh / p->h;
                term += pe[k];
            }
            e1[k] += (dt / eps0) * (-term);
        }
        {
            const double t = (n + 0.5) * dt;
            e1[ksrc] += orc_ramp(p, t) * sin(omega * t);
        }
        e_inc[n] = e1[ks];
        /* H update on interior edges; the end edges stay zero */
        for (int32_t k = 1; k < M; ++k) {
            const double de = e1[k] - e1[k - 1];
            double term = de * prh[3 * k + 2] / p->h;
            if (prh[3 * k + 1] != 0.0) {
                ph[k] = prh[3 * k] * ph[k] + prh[3 * k + 1] * de / p->h;
                term += ph[k];
            }
            h1[k] -= (dt / ORC_MU0) * term;
        }
    }
    free(e1); free(h1); free(pe); free(ph); free(pre); free(prh);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Time stepping (Sec. 2.3-2.6)                                              */
/* ------------------------------------------------------------------------- */

#define IDX(j, i) ((size_t)(j) * (size_t)nx + (size_t)(i))

/* One Ez update (eq. 18 with reading: the two Hx edges that bound the Ez cell
 * are y = jh and y = (j+1)h; the printed indices j and j-1 are one row low).
 * ez_hist, when given, receives Ez after the update. */
static void orc_update_e(const orc_problem* p, const double* ce, const double* cb,
                         const double* prof_e, double h_inc_n,
                         double* ez, const double* hx, const double* hy, double* pez)
{
    const int32_t nx = p->nx, ny = p->ny;
    const double h = p->h;
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ny; ++j) {
        const double b = prof_e[3 * j], c = prof_e[3 * j + 1], ik = prof_e[3 * j + 2];
        for (int32_t i = 0; i < nx; ++i) {
            const double hx_top = (j + 1 < ny) ? hx[IDX(j + 1, i)] : 0.0; /* Hx = 0 on y = ny h */
            const double hx_bot = hx[IDX(j, i)];                           /* row 0 holds zeros   */
            const double dhx = hx_top - hx_bot;
            const int32_t ir = (i + 1 == nx) ? 0 : i + 1;                 /* periodic wrap       */
            const double dhy = hy[IDX(j, ir)] - hy[IDX(j, i)];
            double curl = dhy / h - ik * dhx / h;
            if (c != 0.0) {
                pez[IDX(j, i)] = b * pez[IDX(j, i)] + c * dhx / h;
                curl -= pez[IDX(j, i)];
            }
            if (j == p->j_src) curl -= h_inc_n / h;   /* TF/SF: Hx above is scattered */
            ez[IDX(j, i)] = ce[IDX(j, i)] * ez[IDX(j, i)] + cb[IDX(j, i)] * curl;
        }
    }
}

/* Hx and Hy updates (eqs. 19-20; Hy wraps periodically, eq. 22). */
static void orc_update_h(const orc_problem* p, const double* prof_h, double e_inc_n,
                         const double* ez, double* hx, double* hy, double* phx)
{
    const int32_t nx = p->nx, ny = p->ny;
    const double h = p->h;
    const double dt = orc_time_step(p->h, p->courant);
    const double k = dt / ORC_MU0;
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ny; ++j) {
        const double b = prof_h[3 * j], c = prof_h[3 * j + 1], ik = prof_h[3 * j + 2];
        for (int32_t i = 0; i < nx; ++i) {
            if (j > 0) {
                const double de = ez[IDX(j, i)] - ez[IDX(j - 1, i)];
                double term = ik * de / h;
                if (c != 0.0) {
                    phx[IDX(j, i)] = b * phx[IDX(j, i)] + c * de / h;
                    term += phx[IDX(j, i)];
                }
                if (j == p->j_src + 1) term += e_inc_n / h;   /* TF/SF: Ez below is total */
                hx[IDX(j, i)] -= k * term;
            }
            const int32_t il = (i == 0) ? nx - 1 : i - 1;      /* periodic wrap */
            hy[IDX(j, i)] += k * (ez[IDX(j, i)] - ez[IDX(j, il)]) / h;
        }
    }
}

/* Run steps [n_begin, n_end) from the state passed in (fields in SI units,
 * psi arrays full-size and zero outside the layers).  mon[4][nx] receives the
 * running DFT sums of eqs. 29-30 on the two monitor rows:
 *   mon[0] += Ez(j_ref) cos(w t), mon[1] += Ez(j_ref) sin(w t),
 *   mon[2] += Ez(j_trn) cos(w t), mon[3] += Ez(j_trn) sin(w t),  t = (n+1/2) dt,
 * for every step n >= dft_start.  If ez_hist is given it receives Ez after
 * each step: ez_hist[(n - n_begin)][ny][nx]. */
int orc_run(const orc_problem* p, const double* ce, const double* cb,
            const double* e_inc, const double* h_inc,
            double* ez, double* hx, double* hy, double* pez, double* phx,
            int32_t n_begin, int32_t n_end, double* mon, double* ez_hist)
{
    const int32_t nx = p->nx, ny = p->ny;
    const double dt = orc_time_step(p->h, p->courant);
    const double omega = orc_omega(p);
    double* prof_e = malloc(sizeof(double) * 3 * (size_t)ny);
    double* prof_h = malloc(sizeof(double) * 3 * (size_t)ny);
    if (!prof_e || !prof_h) { free(prof_e); free(prof_h); return -2; }
    orc_cpml_profiles(p, prof_e, prof_h);
    for (int32_t i = 0; i < nx; ++i) hx[IDX(0, i)] = 0.0;

    for (int32_t n = n_begin; n < n_end; ++n) {
        orc_update_e(p, ce, cb, prof_e, h_inc ? h_inc[n] : 0.0, ez, hx, hy, pez);
        orc_update_h(p, prof_h, e_inc ? e_inc[n] : 0.0, ez, hx, hy, phx);
        if (mon && n >= p->dft_start) {
            const double t = (n + 0.5) * dt;
            const double cw = cos(omega * t), sw = sin(omega * t);
            for (int32_t i = 0; i < nx; ++i) {
                mon[0 * (size_t)nx + i] += ez[IDX(p->j_ref, i)] * cw;
                mon[1 * (size_t)nx + i] += ez[IDX(p->j_ref, i)] * sw;
                mon[2 * (size_t)nx + i] += ez[IDX(p->j_trn, i)] * cw;
                mon[3 * (size_t)nx + i] += ez[IDX(p->j_trn, i)] * sw;
            }
        }
        if (ez_hist) memcpy(ez_hist + (size_t)(n - n_begin) * nx * ny, ez, sizeof(double) * (size_t)nx * ny);
    }
    free(prof_e);
    free(prof_h);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Reflectance and transmittance (Sec. 2.6)                                  */
/* ------------------------------------------------------------------------- */

/* Gram matrix of the tone fit over the monitor window: g = {sum c^2, sum c s, sum s^2}. */
/* Time of the monitored field after step n: Ez^{n+1/2} in TMz, Ex^{n+1} in TEz. */
static double orc_sample_time(const orc_problem* p, int32_t n, double dt)
{
    return (p->polarization ? n + 1.0 : n + 0.5) * dt;
}

void orc_gram(const orc_problem* p, double g[3])
{
    const double dt = orc_time_step(p->h, p->courant);
    const double omega = orc_omega(p);
    g[0] = g[1] = g[2] = 0.0;
    for (int32_t n = p->dft_start; n < p->n_steps; ++n) {
        const double t = orc_sample_time(p, n, dt);
        const double cw = cos(omega * t), sw = sin(omega * t);
        g[0] += cw * cw;
        g[1] += cw * sw;
        g[2] += sw * sw;
    }
}

/* Reading of the paper's "DFT after steady state": a sampled tone
 * E(t) = a cos(wt) + b sin(wt) over a finite window is recovered exactly by
 * least squares, (a, b) = G^{-1} (sum E c, sum E s); the complex amplitude is
 * F = a + i b.  A plain DFT would leak for a window that is not a whole number
 * of periods. */
static void orc_tone(const double g[3], double sc, double ss, double* re, double* im)
{
    const double det = g[0] * g[2] - g[1] * g[1];
    *re = (g[2] * sc - g[1] * ss) / det;
    *im = (-g[1] * sc + g[0] * ss) / det;
}

/* Discrete propagation data of Bloch order m (eqs. 31-32, discrete reading).
 * For the Yee scheme the dispersion relation of order m in vacuum is
 *   sin^2(ky h/2) = (sin(w dt/2)/S1)^2 - sin^2(pi m/nx),  S1 = c dt/h.
 * The order propagates when the right side lies in (0,1); returns sin(ky h)
 * (the discrete flux carried per unit |E_m|^2), or 0 when evanescent. */
static double orc_order_flux(const orc_problem* p, int32_t m)
{
    const double dt = orc_time_step(p->h, p->courant);
    const double s1 = ORC_C0 * dt / p->h;
    const double s = sin(orc_omega(p) * dt / 2.0) / s1;
    const double sx = sin(ORC_PI * (double)m / (double)p->nx);
    const double q = s * s - sx * sx;
    if (q <= 0.0 || q >= 1.0) return 0.0;
    if (p->polarization) {
        /* TEz, monitored field Ex on an edge row.  In vacuum the Ex update gives
         * E_m = (S1 sin(ky h/2)/sin(w dt/2)) B_m for a Hz order of amplitude B_m,
         * and the conserved discrete Wronskian of the Hz equation carries
         * |B_m|^2 sin(ky h); per unit |E_m|^2 that is proportional to
         * cot(ky h/2) = sqrt((1 - q)/q). */
        return sqrt((1.0 - q) / q);
    }
    return sin(2.0 * asin(sqrt(q)));
}

/* Paper-literal cutoff (Sec. 2.6): order m propagates when k0^2 - kx_m^2 > 0. */
static int orc_order_literal(const orc_problem* p, int32_t m)
{
    const double k0 = 2.0 * ORC_PI / p->lambda0;
    const double kx = 2.0 * ORC_PI * (double)m / ((double)p->nx * p->h);
    return k0 * k0 - kx * kx > 0.0;
}

/* Bloch amplitudes and R, T, A (eqs. 31-34).
 * mon: the [4][nx] sums of orc_run; inc_sc, inc_ss: the same sums over e_inc.
 * out[0..2] = R, T, A.  Optional per-order outputs (index m + nx/2 for
 * m in [-(nx-1)/2, nx/2]): order_w (weight, 0 if not propagating),
 * ref_pow = |F_ref,m|^2/|F_inc|^2, trn_pow likewise.
 * Reading: R and T sum the orders with discrete flux weights
 * w_m = sin(ky_m h)/sin(ky_0 h), so that R + T = 1 holds exactly for lossless
 * structures once several orders propagate; literal_orders = 1 gives the
 * printed unit weights and continuous cutoff instead. */
int orc_spectra(const orc_problem* p, const double* mon, double inc_sc, double inc_ss,
                double out[3], double* order_w, double* ref_pow, double* trn_pow)
{
    const int32_t nx = p->nx;
    double g[3];
    orc_gram(p, g);
    if (g[0] * g[2] - g[1] * g[1] <= 0.0) return -1;
    double fi_re, fi_im;
    orc_tone(g, inc_sc, inc_ss, &fi_re, &fi_im);
    const double finc2 = fi_re * fi_re + fi_im * fi_im;
    if (!(finc2 > 0.0)) return -1;
    const double flux0 = orc_order_flux(p, 0);
    double R = 0.0, T = 0.0;
    const int32_t m_lo = -(nx - 1) / 2, m_hi = nx / 2;
    for (int32_t m = m_lo; m <= m_hi; ++m) {
        double w;
        if (p->literal_orders) w = orc_order_literal(p, m) ? 1.0 : 0.0;
        else w = orc_order_flux(p, m) / flux0;
        double pr = 0.0, pt = 0.0;
        if (w > 0.0 || ref_pow || trn_pow) {
            /* F_m = (1/nx) sum_i F_i exp(-2 pi i m i/nx), F_i from the tone fit */
            double rr = 0, ri = 0, tr = 0, ti = 0;
            for (int32_t i = 0; i < nx; ++i) {
                const double ph = -2.0 * ORC_PI * (double)(((int64_t)m * i) % nx) / (double)nx;
                const double cp = cos(ph), sp = sin(ph);
                double a, b;
                orc_tone(g, mon[i], mon[nx + i], &a, &b);
                rr += a * cp - b * sp;
                ri += a * sp + b * cp;
                orc_tone(g, mon[2 * nx + i], mon[3 * nx + i], &a, &b);
                tr += a * cp - b * sp;
                ti += a * sp + b * cp;
            }
            rr /= nx; ri /= nx; tr /= nx; ti /= nx;
            pr = (rr * rr + ri * ri) / finc2;
            pt = (tr * tr + ti * ti) / finc2;
        }
        R += w * pr;
        T += w * pt;
        if (order_w) order_w[m - m_lo] = w;
        if (ref_pow) ref_pow[m - m_lo] = pr;
        if (trn_pow) trn_pow[m - m_lo] = pt;
    }
    out[0] = R;
    out[1] = T;
    out[2] = 1.0 - R - T;
    return 0;
}

/* Incident-reference sums over the monitor window: {sum e_inc c, sum e_inc s}. */
void orc_incident_sums(const orc_problem* p, const double* e_inc, double out[2])
{
    const double dt = orc_time_step(p->h, p->courant);
    const double omega = orc_omega(p);
    out[0] = out[1] = 0.0;
    for (int32_t n = p->dft_start; n < p->n_steps; ++n) {
        const double t = orc_sample_time(p, n, dt);
        out[0] += e_inc[n] * cos(omega * t);
        out[1] += e_inc[n] * sin(omega * t);
    }
}

/* ------------------------------------------------------------------------- */
/* TEz (P polarisation), Sec. 2.2 and eqs. 14-16                             */
/* ------------------------------------------------------------------------- */
/*
 * Lattice: Hz at cell centres ((i+1/2)h, (j+1/2)h), array hz[j][i]; Ex on the
 * bottom edge ((i+1/2)h, jh), array ex[j][i]; Ey on the left edge
 * (ih, (j+1/2)h), array ey[j][i].  Ex = 0 on the rows y = 0 and y = ny h
 * (electric walls behind the absorbing layers); Ey wraps in x (eq. 22).
 * Time stepping in the paper's TEz order: step n advances Hz^{n-1/2} ->
 * Hz^{n+1/2} with E^n (eq. 14), then E^n -> E^{n+1} with Hz^{n+1/2}
 * (eqs. 15-16, with the same reading of the curl coefficient as eq. 17).
 * Materials sit on the edges.  Reading: the paper does not say how an edge
 * between two cells of different material is coefficiented; eps_r and sigma
 * are the arithmetic means of the two cells'.
 * TF/SF on the same horizontal line: Hz rows j <= j_src total field, Ex edges
 * j >= j_src+1 and Hz rows j > j_src scattered field.
 */

/* Per-edge (Ce, Cb) of Ex (bottom edge of cell (i,j), cells (i,j-1) and (i,j);
 * row 0 is the wall and gets Ce = 1, Cb = 0) and of Ey (left edge of cell (i,j),
 * cells (i-1,j) and (i,j), periodic). */
void orc_edge_coefficients(const orc_problem* p, const uint8_t* labels, int32_t n_labels,
                           const double* nk, double* cex, double* cbx, double* cey, double* cby)
{
    const int32_t nx = p->nx, ny = p->ny;
    const double dt = orc_time_step(p->h, p->courant);
    const double omega = orc_omega(p);
    (void)n_labels;
    for (int32_t j = 0; j < ny; ++j)
        for (int32_t i = 0; i < nx; ++i) {
            double a[4], b[4], m[2];
            const int La = labels[IDX(j, i)];
            orc_material(nk[2 * La], nk[2 * La + 1], omega, dt, a);
            if (j == 0) {
                cex[IDX(j, i)] = 1.0;
                cbx[IDX(j, i)] = 0.0;
            } else {
                const int Lb = labels[IDX(j - 1, i)];
                orc_material(nk[2 * Lb], nk[2 * Lb + 1], omega, dt, b);
                orc_material_eps(0.5 * (a[0] + b[0]), 0.5 * (a[1] + b[1]), dt, m);
                cex[IDX(j, i)] = m[0];
                cbx[IDX(j, i)] = m[1];
            }
            const int32_t il = (i == 0) ? nx - 1 : i - 1;
            const int Lc = labels[IDX(j, il)];
            orc_material(nk[2 * Lc], nk[2 * Lc + 1], omega, dt, b);
            orc_material_eps(0.5 * (a[0] + b[0]), 0.5 * (a[1] + b[1]), dt, m);
            cey[IDX(j, i)] = m[0];
            cby[IDX(j, i)] = m[1];
        }
}

/* Incident wave for TEz from a 1D vacuum grid in the TEz order: Hz1[k] at
 * y = k+1/2, Ex1[k] at y = k (Ex1[0] = Ex1[M] = 0), absorbing cells at both
 * ends.  A soft source adds ramp(t) sin(omega t), t = (n+1) dt, to the edge
 * aux_src_off + 1 above the TF/SF edge after each E update.
 * Recorded per step n:  e_inc[n] = Ex1 on edge j_src+1 at time (n+1) dt (the
 * value the Hz update of step n+1 needs, and the incident reference of the
 * monitors);  h_inc[n] = Hz1 on row j_src at time n+1/2 (used by the E update
 * of step n). */
static int orc_incident_te_drive(const orc_problem* p, int pulse, double tau, double t0, double* e_inc,
                                 double* h_inc)
{
    const int32_t P = p->aux_pml, pad = p->aux_pad;
    const int32_t M = 2 * (P + pad) + 1;
    const int32_t ks = P + pad;              /* TF/SF cell in the 1D grid */
    const int32_t ksrc = ks + 1 + p->aux_src_off;
    if (P < 1 || pad < 2 || p->aux_src_off < 1 || ksrc >= M - P) return -1;
    const double eps0 = orc_eps0();
    const double dt = orc_time_step(p->h, p->courant);
    const double omega = orc_omega(p);
    double* hz1 = calloc((size_t)M, sizeof(double));
    double* ex1 = calloc((size_t)M + 1, sizeof(double));
    double* phz = calloc((size_t)M, sizeof(double));
    double* pex = calloc((size_t)M + 1, sizeof(double));
    double* prc = malloc(sizeof(double) * 3 * (size_t)M);
    double* pre = malloc(sizeof(double) * 3 * ((size_t)M + 1));
    if (!hz1 || !ex1 || !phz || !pex || !prc || !pre) {
        free(hz1); free(ex1); free(phz); free(pex); free(prc); free(pre);
        return -2;
    }
    for (int32_t k = 0; k < M; ++k) orc_cpml_at(p, orc_depth_ez(k, M, P), P, &prc[3 * k]);
    for (int32_t k = 0; k <= M; ++k) orc_cpml_at(p, orc_depth_hx(k, M, P), P, &pre[3 * k]);
    for (int32_t n = 0; n < p->n_steps; ++n) {
        /* Hz update (eq. 14 without the x term) */
        for (int32_t k = 0; k < M; ++k) {
            const double de = ex1[k + 1] - ex1[k];
            double term = de * prc[3 * k + 2] / p->h;
            if (prc[3 * k + 1] != 0.0) {
                phz[k] = prc[3 * k] * phz[k] + prc[3 * k + 1] * de / p->h;
                term += phz[k];
            }
            hz1[k] -= (dt / ORC_MU0) * (-term);
        }
        h_inc[n] = hz1[ks];
        /* Ex update on interior edges (eq. 15, vacuum) */
        for (int32_t k = 1; k < M; ++k) {
            const double dh = hz1[k] - hz1[k - 1];
            double term = dh * pre[3 * k + 2] / p->h;
            if (pre[3 * k + 1] != 0.0) {
                pex[k] = pre[3 * k] * pex[k] + pre[3 * k + 1] * dh / p->h;
                term += pex[k];
            }
            ex1[k] += (dt / eps0) * term;
        }
        {
            const double t = (n + 1.0) * dt;
            if (pulse) {
                const double x = (t - t0) / tau;
                ex1[ksrc] += exp(-x * x) * sin(omega * (t - t0));
            } else {
                ex1[ksrc] += orc_ramp(p, t) * sin(omega * t);
            }
        }
        e_inc[n] = ex1[ks + 1];
    }
    free(hz1); free(ex1); free(phz); free(pex); free(prc); free(pre);
    return 0;
}

int orc_incident_te(const orc_problem* p, double* e_inc, double* h_inc)
{
    return orc_incident_te_drive(p, 0, 0.0, 0.0, e_inc, h_inc);
}

/* The TEz incident wave of a broadband run: the 1D grid of orc_incident_te
 * driven by exp(-((t - t0)/tau)^2) sin(w0 (t - t0)), w0 = 2 pi c / lambda0, at
 * the same source edge and times t = (n+1) dt.  Recorded like orc_incident_te. */
int orc_incident_pulse_te(const orc_problem* p, double tau, double t0, double* e_inc, double* h_inc)
{
    if (!(tau > 0.0)) return -1;
    return orc_incident_te_drive(p, 1, tau, t0, e_inc, h_inc);
}

/* Run TEz steps [n_begin, n_end) from the state passed in (SI units; psi
 * arrays full-size, zero outside the layers: phz for the dEx/dy term of the Hz
 * update at y = j+1/2, pex for the dHz/dy term of the Ex update at y = j).
 * mon[4][nx]: sums of Ex on the edge rows j_ref and j_trn times cos/sin(w t),
 * t = (n+1) dt, for steps n >= dft_start. */
int orc_run_te(const orc_problem* p, const double* cex, const double* cbx, const double* cey,
               const double* cby, const double* e_inc, const double* h_inc,
               double* hz, double* ex, double* ey, double* phz, double* pex,
               int32_t n_begin, int32_t n_end, double* mon)
{
    const int32_t nx = p->nx, ny = p->ny;
    const double h = p->h;
    const double dt = orc_time_step(p->h, p->courant);
    const double omega = orc_omega(p);
    const double kh = dt / ORC_MU0;
    double* prof_c = malloc(sizeof(double) * 3 * (size_t)ny);   /* at y = j+1/2 */
    double* prof_e = malloc(sizeof(double) * 3 * (size_t)ny);   /* at y = j     */
    if (!prof_c || !prof_e) { free(prof_c); free(prof_e); return -2; }
    orc_cpml_profiles(p, prof_c, prof_e);
    for (int32_t i = 0; i < nx; ++i) ex[IDX(0, i)] = 0.0;

    for (int32_t n = n_begin; n < n_end; ++n) {
        const double ex_inc_n = (e_inc && n > 0) ? e_inc[n - 1] : 0.0;   /* Ex_inc at time n dt */
        /* Hz update, eq. 14 */
#pragma omp parallel for schedule(static)
        for (int32_t j = 0; j < ny; ++j) {
            const double b = prof_c[3 * j], c = prof_c[3 * j + 1], ik = prof_c[3 * j + 2];
            for (int32_t i = 0; i < nx; ++i) {
                const double ex_top = (j + 1 < ny) ? ex[IDX(j + 1, i)] : 0.0;   /* Ex = 0 on y = ny h */
                const double dex = ex_top - ex[IDX(j, i)];
                double term_y = ik * dex / h;
                if (c != 0.0) {
                    phz[IDX(j, i)] = b * phz[IDX(j, i)] + c * dex / h;
                    term_y += phz[IDX(j, i)];
                }
                if (j == p->j_src) term_y += ex_inc_n / h;                  /* TF/SF: Ex above is scattered */
                const int32_t ir = (i + 1 == nx) ? 0 : i + 1;                 /* periodic wrap */
                const double dey = ey[IDX(j, ir)] - ey[IDX(j, i)];
                hz[IDX(j, i)] -= kh * (dey / h - term_y);
            }
        }
        /* Ex and Ey updates, eqs. 15-16 */
#pragma omp parallel for schedule(static)
        for (int32_t j = 0; j < ny; ++j) {
            const double b = prof_e[3 * j], c = prof_e[3 * j + 1], ik = prof_e[3 * j + 2];
            for (int32_t i = 0; i < nx; ++i) {
                if (j > 0) {
                    const double dhz = hz[IDX(j, i)] - hz[IDX(j - 1, i)];
                    double term = ik * dhz / h;
                    if (c != 0.0) {
                        pex[IDX(j, i)] = b * pex[IDX(j, i)] + c * dhz / h;
                        term += pex[IDX(j, i)];
                    }
                    if (j == p->j_src + 1 && h_inc) term += h_inc[n] / h;     /* TF/SF: Hz below is total */
                    ex[IDX(j, i)] = cex[IDX(j, i)] * ex[IDX(j, i)] + cbx[IDX(j, i)] * term;
                }
                const int32_t il = (i == 0) ? nx - 1 : i - 1;                 /* periodic wrap */
                ey[IDX(j, i)] = cey[IDX(j, i)] * ey[IDX(j, i)] - cby[IDX(j, i)] * (hz[IDX(j, i)] - hz[IDX(j, il)]) / h;
            }
        }
        if (mon && n >= p->dft_start) {
            const double t = (n + 1.0) * dt;
            const double cw = cos(omega * t), sw = sin(omega * t);
            for (int32_t i = 0; i < nx; ++i) {
                mon[0 * (size_t)nx + i] += ex[IDX(p->j_ref, i)] * cw;
                mon[1 * (size_t)nx + i] += ex[IDX(p->j_ref, i)] * sw;
                mon[2 * (size_t)nx + i] += ex[IDX(p->j_trn, i)] * cw;
                mon[3 * (size_t)nx + i] += ex[IDX(p->j_trn, i)] * sw;
            }
        }
    }
    free(prof_c);
    free(prof_e);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Discrete adjoint                                                          */
/* ------------------------------------------------------------------------- */

/* Gradient of L = dL_dR * R + dL_dT * T with respect to the four monitor sums.
 * R = sum_m w_m |F_m|^2/|F_inc|^2 with F_m linear in the sums, so
 * dR/dSc_i = (2/(nx |F_inc|^2)) Re[(G11 + i G21) U_i],
 * dR/dSs_i = (2/(nx |F_inc|^2)) Re[(G12 + i G22) U_i],
 * U_i = sum_m w_m conj(F_m) exp(-2 pi i m i/nx), G = Gram^{-1}.
 * The incident sums do not depend on the materials. */
int orc_spectra_grad(const orc_problem* p, const double* mon, double inc_sc, double inc_ss,
                     double dL_dR, double dL_dT, double* dmon)
{
    const int32_t nx = p->nx;
    double g[3];
    orc_gram(p, g);
    const double det = g[0] * g[2] - g[1] * g[1];
    if (det <= 0.0) return -1;
    const double gi11 = g[2] / det, gi12 = -g[1] / det, gi22 = g[0] / det;
    double fi_re, fi_im;
    orc_tone(g, inc_sc, inc_ss, &fi_re, &fi_im);
    const double finc2 = fi_re * fi_re + fi_im * fi_im;
    const double flux0 = orc_order_flux(p, 0);
    const int32_t m_lo = -(nx - 1) / 2, m_hi = nx / 2;
    for (int32_t line = 0; line < 2; ++line) {
        const double* sc = mon + (size_t)(2 * line) * nx;
        const double* ss = mon + (size_t)(2 * line + 1) * nx;
        const double scale = (line == 0 ? dL_dR : dL_dT) * 2.0 / ((double)nx * finc2);
        for (int32_t i = 0; i < nx; ++i) { dmon[(2 * line) * (size_t)nx + i] = 0; dmon[(2 * line + 1) * (size_t)nx + i] = 0; }
        for (int32_t m = m_lo; m <= m_hi; ++m) {
            const double w = p->literal_orders ? (orc_order_literal(p, m) ? 1.0 : 0.0)
                                               : orc_order_flux(p, m) / flux0;
            if (w <= 0.0) continue;
            double fr = 0, fim = 0;
            for (int32_t i = 0; i < nx; ++i) {
                const double ph = -2.0 * ORC_PI * (double)(((int64_t)m * i) % nx) / (double)nx;
                double a, b;
                orc_tone(g, sc[i], ss[i], &a, &b);
                fr += a * cos(ph) - b * sin(ph);
                fim += a * sin(ph) + b * cos(ph);
            }
            fr /= nx; fim /= nx;
            for (int32_t i = 0; i < nx; ++i) {
                const double ph = -2.0 * ORC_PI * (double)(((int64_t)m * i) % nx) / (double)nx;
                /* w conj(F_m) e^{i ph} */
                const double ur = w * (fr * cos(ph) + fim * sin(ph));
                const double ui = w * (fr * sin(ph) - fim * cos(ph));
                /* Re[(G11 + i G21) U] and Re[(G12 + i G22) U] */
                dmon[(2 * line) * (size_t)nx + i] += scale * (gi11 * ur - gi12 * ui);
                dmon[(2 * line + 1) * (size_t)nx + i] += scale * (gi12 * ur - gi22 * ui);
            }
        }
    }
    return 0;
}

/* Transpose of one step with no sources: maps the adjoint state after step n
 * (lez, lhx, lhy, lpez, lphx) to the adjoint state before it.  Each forward
 * assignment is transposed, in reverse order:
 *   H update  Hy += k (Ez_i - Ez_{i-1});  Hx -= k (dEz/kappa_h + psi_h);
 *             psi_h = b_h psi_h + c_h dEz/h
 *   E update  psi_e = b_e psi_e + c_e dHx/h;  Ez = Ce Ez + Cb curl.
 * If gce/gcb are given, they accumulate dL/dCe = lambda_E^{n+1/2} Ez^{n-1/2}
 * and dL/dCb = lambda_E^{n+1/2} curl^n, where curl^n is recovered from the
 * stored Ez before (ez_old) and after (ez_new) the step. */
void orc_step_adjoint(const orc_problem* p, const double* ce, const double* cb,
                      double* lez, double* lhx, double* lhy, double* lpez, double* lphx,
                      const double* ez_old, const double* ez_new, double* gce, double* gcb)
{
    const int32_t nx = p->nx, ny = p->ny;
    const double h = p->h;
    const double dt = orc_time_step(p->h, p->courant);
    const double k = dt / ORC_MU0;
    double* prof_e = malloc(sizeof(double) * 3 * (size_t)ny);
    double* prof_h = malloc(sizeof(double) * 3 * (size_t)ny);
    double* lcurl = malloc(sizeof(double) * (size_t)nx * ny);
    orc_cpml_profiles(p, prof_e, prof_h);

    /* --- transpose of the H update --- */
    /* Hy(j,i) += k (Ez(j,i) - Ez(j,i-1))/h */
    for (int32_t j = 0; j < ny; ++j)
        for (int32_t i = 0; i < nx; ++i) {
            const int32_t il = (i == 0) ? nx - 1 : i - 1;
            lez[IDX(j, i)] += k * lhy[IDX(j, i)] / h;
            lez[IDX(j, il)] -= k * lhy[IDX(j, i)] / h;
        }
    /* Hx(j) -= k (ik dE/h + psi_h(j)),  psi_h(j) = b psi_h(j) + c dE/h,  dE = Ez(j) - Ez(j-1) */
    for (int32_t j = 1; j < ny; ++j) {
        const double b = prof_h[3 * j], c = prof_h[3 * j + 1], ik = prof_h[3 * j + 2];
        for (int32_t i = 0; i < nx; ++i) {
            double lde = -k * ik * lhx[IDX(j, i)] / h;
            if (c != 0.0) {
                const double lpsi_new = lphx[IDX(j, i)] - k * lhx[IDX(j, i)];
                lde += c * lpsi_new / h;
                lphx[IDX(j, i)] = b * lpsi_new;
            }
            lez[IDX(j, i)] += lde;
            lez[IDX(j - 1, i)] -= lde;
        }
    }
    /* --- transpose of the E update --- */
    for (int32_t j = 0; j < ny; ++j)
        for (int32_t i = 0; i < nx; ++i) {
            const double le = lez[IDX(j, i)];
            if (gce) {
                const double curl = (ez_new[IDX(j, i)] - ce[IDX(j, i)] * ez_old[IDX(j, i)]) / cb[IDX(j, i)];
                gce[IDX(j, i)] += le * ez_old[IDX(j, i)];
                gcb[IDX(j, i)] += le * curl;
            }
            lcurl[IDX(j, i)] = cb[IDX(j, i)] * le;
            lez[IDX(j, i)] = ce[IDX(j, i)] * le;
        }
    for (int32_t j = 0; j < ny; ++j) {
        const double b = prof_e[3 * j], c = prof_e[3 * j + 1], ik = prof_e[3 * j + 2];
        for (int32_t i = 0; i < nx; ++i) {
            const double lc = lcurl[IDX(j, i)];
            const int32_t ir = (i + 1 == nx) ? 0 : i + 1;
            /* curl = (Hy(i+1) - Hy(i))/h - ik dHx/h - psi_e_new */
            lhy[IDX(j, ir)] += lc / h;
            lhy[IDX(j, i)] -= lc / h;
            double ldhx = -ik * lc / h;
            if (c != 0.0) {
                const double lpsi_new = lpez[IDX(j, i)] - lc;
                ldhx += c * lpsi_new / h;
                lpez[IDX(j, i)] = b * lpsi_new;
            }
            /* dHx = Hx(j+1) - Hx(j); Hx on rows 0 and ny is held at zero */
            if (j + 1 < ny) lhx[IDX(j + 1, i)] += ldhx;
            if (j > 0) lhx[IDX(j, i)] -= ldhx;
        }
    }
    for (int32_t i = 0; i < nx; ++i) lhx[IDX(0, i)] = 0.0;
    free(prof_e);
    free(prof_h);
    free(lcurl);
}

/* Reverse sweep over a whole run from zero initial fields.
 * ez_hist: Ez after every step, [n_steps][ny][nx] (from orc_run).
 * dmon: dL/d(monitor sums) as produced by orc_spectra_grad.
 * gce, gcb: per-pixel dL/dCe and dL/dCb (accumulated, caller zeroes). */
int orc_adjoint(const orc_problem* p, const double* ce, const double* cb,
                const double* ez_hist, const double* dmon, double* gce, double* gcb)
{
    const int32_t nx = p->nx, ny = p->ny;
    const size_t ncell = (size_t)nx * ny;
    const double dt = orc_time_step(p->h, p->courant);
    const double omega = orc_omega(p);
    double* lez = calloc(ncell, sizeof(double));
    double* lhx = calloc(ncell, sizeof(double));
    double* lhy = calloc(ncell, sizeof(double));
    double* lpez = calloc(ncell, sizeof(double));
    double* lphx = calloc(ncell, sizeof(double));
    double* zero = calloc(ncell, sizeof(double));
    if (!lez || !lhx || !lhy || !lpez || !lphx || !zero) {
        free(lez); free(lhx); free(lhy); free(lpez); free(lphx); free(zero);
        return -2;
    }
    for (int32_t n = p->n_steps - 1; n >= 0; --n) {
        /* transpose of the monitor accumulation of step n */
        if (n >= p->dft_start) {
            const double t = (n + 0.5) * dt;
            const double cw = cos(omega * t), sw = sin(omega * t);
            for (int32_t i = 0; i < nx; ++i) {
                lez[IDX(p->j_ref, i)] += dmon[i] * cw + dmon[nx + i] * sw;
                lez[IDX(p->j_trn, i)] += dmon[2 * (size_t)nx + i] * cw + dmon[3 * (size_t)nx + i] * sw;
            }
        }
        const double* ez_new = ez_hist + (size_t)n * ncell;
        const double* ez_old = (n > 0) ? ez_hist + (size_t)(n - 1) * ncell : zero;
        orc_step_adjoint(p, ce, cb, lez, lhx, lhy, lpez, lphx, ez_old, ez_new, gce, gcb);
    }
    free(lez); free(lhx); free(lhy); free(lpez); free(lphx); free(zero);
    return 0;
}

/* Chain rule from per-pixel (dL/dCe, dL/dCb) to
 *   grad_nk[L][2] = (dL/dn_L, dL/dk_L)   for every label L, and
 *   grad_eps[px]  = dL/d eps_r(px) at fixed sigma(px).
 * With a = sigma dt/(2 eps0 eps_r) = omega dt n k/eps_r:
 *   Ce = (1-a)/(1+a),  Cb = dt/(eps0 eps_r (1+a)),
 *   deps_r/dn = 2n, deps_r/dk = -2k,
 *   da/dn = omega dt k/eps_r - 2 n a/eps_r,  da/dk = omega dt n/eps_r + 2 k a/eps_r,
 *   dCe/dx = -2/(1+a)^2 da/dx,  dCb/dx = -Cb (deps_r/dx / eps_r + da/dx/(1+a));
 * at fixed sigma, da/deps_r = -a/eps_r. */
void orc_grad_chain(const orc_problem* p, const uint8_t* labels, int32_t n_labels, const double* nk,
                    const double* gce, const double* gcb, double* grad_nk, double* grad_eps)
{
    const double dt = orc_time_step(p->h, p->courant);
    const double omega = orc_omega(p);
    const size_t ncell = (size_t)p->nx * p->ny;
    for (int32_t L = 0; L < n_labels; ++L) { grad_nk[2 * L] = 0; grad_nk[2 * L + 1] = 0; }
    for (size_t c = 0; c < ncell; ++c) {
        const int32_t L = labels[c];
        const double n = nk[2 * L], k = nk[2 * L + 1];
        double m[4];
        orc_material(n, k, omega, dt, m);
        const double eps_r = m[0], cbv = m[3];
        const double a = omega * dt * n * k / eps_r;
        const double da_dn = omega * dt * k / eps_r - 2.0 * n * a / eps_r;
        const double da_dk = omega * dt * n / eps_r + 2.0 * k * a / eps_r;
        const double dce_da = -2.0 / ((1.0 + a) * (1.0 + a));
        const double dce_dn = dce_da * da_dn, dce_dk = dce_da * da_dk;
        const double dcb_dn = -cbv * (2.0 * n / eps_r + da_dn / (1.0 + a));
        const double dcb_dk = -cbv * (-2.0 * k / eps_r + da_dk / (1.0 + a));
        grad_nk[2 * L] += gce[c] * dce_dn + gcb[c] * dcb_dn;
        grad_nk[2 * L + 1] += gce[c] * dce_dk + gcb[c] * dcb_dk;
        if (grad_eps) {
            const double da_de = -a / eps_r;
            const double dce_de = dce_da * da_de;
            const double dcb_de = -cbv * (1.0 / eps_r + da_de / (1.0 + a));
            grad_eps[c] = gce[c] * dce_de + gcb[c] * dcb_de;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Dispersive media and broadband runs (Sec. 2.2)                             */
/* ------------------------------------------------------------------------- */
/*
 * Sec. 2.2 names the alternative to one monochromatic run per wavelength: a
 * Lorentz-Drude model of each material, carried in the time domain by
 * auxiliary differential equations for polarisation currents, and a broadband
 * source whose response is Fourier-analysed afterwards.  Model of a label
 * (e^{-i w t} convention, so an absorbing medium has Im eps > 0):
 *   eps(w) = eps_inf + i sigma/(w eps0) + sum_p a_p / (w_p^2 - w^2 - i g_p w),
 * a_p = d_eps_p w_p^2 for a Lorentz pole; a Drude term is the pole w_p = 0 with
 * a_p = w_D^2.  Each pole's polarisation P_p obeys
 *   d2P/dt2 + g_p dP/dt + w_p^2 P = eps0 a_p E,
 * and Ampere's law becomes
 *   eps0 eps_inf dE/dt + sigma E + sum_p dP_p/dt = curl H.
 * Discretisation (central differences around the time of E^{n-1/2}):
 *   P^{n+1/2} = alpha P^{n-1/2} + xi P^{n-3/2} + zeta E^{n-1/2},
 *   alpha = (2 - w_p^2 dt^2)/(1 + g dt/2), xi = (g dt/2 - 1)/(1 + g dt/2),
 *   zeta = eps0 a_p dt^2/(1 + g dt/2),
 * then E^{n+1/2} = Ce E^{n-1/2} + Cb [curl H^n - sum_p (P^{n+1/2} - P^{n-1/2})/dt]
 * with Ce, Cb of eq. 17 (reading R1) at eps_r = eps_inf.
 * model layout per label: eps_inf, sigma, then (a_p, w_p, g_p) per pole.
 * out per label: Ce, Cb, then (alpha, xi, zeta) per pole.
 */
void orc_ade_coefficients(const orc_problem* p, int32_t n_labels, int32_t n_poles, const double* model,
                          double* out)
{
    const double dt = orc_time_step(p->h, p->courant);
    const int32_t w_in = 2 + 3 * n_poles;
    for (int32_t L = 0; L < n_labels; ++L) {
        const double* m = model + (size_t)L * w_in;
        double* o = out + (size_t)L * w_in;
        orc_material_eps(m[0], m[1], dt, o);
        for (int32_t q = 0; q < n_poles; ++q) {
            const double a = m[2 + 3 * q], wp = m[3 + 3 * q], g = m[4 + 3 * q];
            const double den = 1.0 + 0.5 * g * dt;
            o[2 + 3 * q] = (2.0 - wp * wp * dt * dt) / den;
            o[3 + 3 * q] = (0.5 * g * dt - 1.0) / den;
            o[4 + 3 * q] = orc_eps0() * a * dt * dt / den;
        }
    }
}

/* Broadband incident wave: the 1D vacuum grid of orc_incident driven by the
 * Gaussian-modulated sinusoid exp(-((t - t0)/tau)^2) sin(w0 (t - t0)),
 * w0 = 2 pi c / lambda0, added at the same source cell and times.  Recorded
 * like orc_incident. */
int orc_incident_pulse(const orc_problem* p, double tau, double t0, double* e_inc, double* h_inc)
{
    const int32_t P = p->aux_pml, pad = p->aux_pad;
    const int32_t M = 2 * (P + pad) + 1;
    const int32_t ks = P + pad;
    const int32_t ksrc = ks + p->aux_src_off;
    if (P < 1 || pad < 2 || p->aux_src_off < 1 || ksrc >= M - P || !(tau > 0.0)) return -1;
    const double eps0 = orc_eps0();
    const double dt = orc_time_step(p->h, p->courant);
    const double omega = orc_omega(p);
    double* e1 = calloc((size_t)M, sizeof(double));
    double* h1 = calloc((size_t)M + 1, sizeof(double));
    double* pe = calloc((size_t)M, sizeof(double));
    double* ph = calloc((size_t)M + 1, sizeof(double));
    double* pre = malloc(sizeof(double) * 3 * (size_t)M);
    double* prh = malloc(sizeof(double) * 3 * ((size_t)M + 1));
    if (!e1 || !h1 || !pe || !ph || !pre || !prh) {
        free(e1); free(h1); free(pe); free(ph); free(pre); free(prh);
        return -2;
    }
    for (int32_t k = 0; k < M; ++k) orc_cpml_at(p, orc_depth_ez(k, M, P), P, &pre[3 * k]);
    for (int32_t k = 0; k <= M; ++k) orc_cpml_at(p, orc_depth_hx(k, M, P), P, &prh[3 * k]);

    for (int32_t n = 0; n < p->n_steps; ++n) {
        h_inc[n] = h1[ks + 1];
        for (int32_t k = 0; k < M; ++k) {
            const double dh = h1[k + 1] - h1[k];
            double term = dh * pre[3 * k + 2] / p->h;
            if (pre[3 * k + 1] != 0.0) {
                pe[k] = pre[3 * k] * pe[k] + pre[3 * k + 1] * dh / p->h;
                term += pe[k];
            }
            e1[k] += (dt / eps0) * (-term);
        }
        {
            const double t = (n + 0.5) * dt, x = (t - t0) / tau;
            e1[ksrc] += exp(-x * x) * sin(omega * (t - t0));
        }
        e_inc[n] = e1[ks];
        for (int32_t k = 1; k < M; ++k) {
            const double de = e1[k] - e1[k - 1];
            double term = de * prh[3 * k + 2] / p->h;
            if (prh[3 * k + 1] != 0.0) {
                ph[k] = prh[3 * k] * ph[k] + prh[3 * k + 1] * de / p->h;
                term += ph[k];
            }
            h1[k] -= (dt / ORC_MU0) * term;
        }
    }
    free(e1); free(h1); free(pe); free(ph); free(pre); free(prh);
    return 0;
}

/* TMz run with dispersive labels: the steps of orc_run with the polarisation
 * update in front of each Ez update.  coef: per-label output of
 * orc_ade_coefficients.  pol: [n_poles][2][ny][nx] = (P^{n-1/2}, P^{n-3/2}) of
 * each pole, updated in place.  mon: [n_freqs][4][nx] sums of Ez cos(w_f t),
 * Ez sin(w_f t) on j_ref and j_trn, t = (n+1/2) dt, for every step
 * n >= dft_start, w_f = 2 pi c / lambdas[f]. */
int orc_run_ade(const orc_problem* p, const uint8_t* labels, int32_t n_poles, const double* coef,
                const double* e_inc, const double* h_inc, double* ez, double* hx, double* hy, double* pez,
                double* phx, double* pol, int32_t n_begin, int32_t n_end, int32_t n_freqs,
                const double* lambdas, double* mon)
{
    const int32_t nx = p->nx, ny = p->ny;
    const size_t plane = (size_t)nx * (size_t)ny;
    const int32_t w_c = 2 + 3 * n_poles;
    const double h = p->h;
    const double dt = orc_time_step(p->h, p->courant);
    double* prof_e = malloc(sizeof(double) * 3 * (size_t)ny);
    double* prof_h = malloc(sizeof(double) * 3 * (size_t)ny);
    if (!prof_e || !prof_h) { free(prof_e); free(prof_h); return -2; }
    orc_cpml_profiles(p, prof_e, prof_h);
    for (int32_t i = 0; i < nx; ++i) hx[IDX(0, i)] = 0.0;

    for (int32_t n = n_begin; n < n_end; ++n) {
        const double h_inc_n = h_inc ? h_inc[n] : 0.0;
#pragma omp parallel for schedule(static)
        for (int32_t j = 0; j < ny; ++j) {
            const double b = prof_e[3 * j], c = prof_e[3 * j + 1], ik = prof_e[3 * j + 2];
            for (int32_t i = 0; i < nx; ++i) {
                const double* cf = coef + (size_t)labels[IDX(j, i)] * w_c;
                /* polarisation at n+1/2 from E^{n-1/2} */
                double dpol = 0.0;
                for (int32_t q = 0; q < n_poles; ++q) {
                    double* pc = pol + ((size_t)2 * q) * plane;
                    double* pp = pol + ((size_t)2 * q + 1) * plane;
                    const double pn = cf[2 + 3 * q] * pc[IDX(j, i)] + cf[3 + 3 * q] * pp[IDX(j, i)]
                                      + cf[4 + 3 * q] * ez[IDX(j, i)];
                    dpol += pn - pc[IDX(j, i)];
                    pp[IDX(j, i)] = pc[IDX(j, i)];
                    pc[IDX(j, i)] = pn;
                }
                const double hx_top = (j + 1 < ny) ? hx[IDX(j + 1, i)] : 0.0;
                const double hx_bot = hx[IDX(j, i)];
                const double dhx = hx_top - hx_bot;
                const int32_t ir = (i + 1 == nx) ? 0 : i + 1;
                const double dhy = hy[IDX(j, ir)] - hy[IDX(j, i)];
                double curl = dhy / h - ik * dhx / h;
                if (c != 0.0) {
                    pez[IDX(j, i)] = b * pez[IDX(j, i)] + c * dhx / h;
                    curl -= pez[IDX(j, i)];
                }
                if (j == p->j_src) curl -= h_inc_n / h;
                ez[IDX(j, i)] = cf[0] * ez[IDX(j, i)] + cf[1] * (curl - dpol / dt);
            }
        }
        orc_update_h(p, prof_h, e_inc ? e_inc[n] : 0.0, ez, hx, hy, phx);
        if (mon && n >= p->dft_start) {
            const double t = (n + 0.5) * dt;
            for (int32_t f = 0; f < n_freqs; ++f) {
                const double w = 2.0 * ORC_PI * ORC_C0 / lambdas[f];
                const double cw = cos(w * t), sw = sin(w * t);
                double* mf = mon + (size_t)f * 4 * nx;
                for (int32_t i = 0; i < nx; ++i) {
                    mf[0 * (size_t)nx + i] += ez[IDX(p->j_ref, i)] * cw;
                    mf[1 * (size_t)nx + i] += ez[IDX(p->j_ref, i)] * sw;
                    mf[2 * (size_t)nx + i] += ez[IDX(p->j_trn, i)] * cw;
                    mf[3 * (size_t)nx + i] += ez[IDX(p->j_trn, i)] * sw;
                }
            }
        }
    }
    free(prof_e);
    free(prof_h);
    return 0;
}

/* R, T, A at one monitor wavelength of a broadband run.  The field has decayed
 * by the end of the run, so the sums of orc_run_ade are its Fourier transform:
 * F_i = sum_n Ez_i(t_n) e^{i w t_n} = (sum E cos) + i (sum E sin), no tone fit.
 * inc_re, inc_im: the same transform of the incident wave on the TF/SF row.
 * Orders, cutoff and flux weights are those of orc_spectra at this wavelength. */
int orc_spectra_pulse(const orc_problem* p, double lambda, const double* mon_f, double inc_re, double inc_im,
                      double out[3])
{
    const int32_t nx = p->nx;
    orc_problem q = *p;
    q.lambda0 = lambda;
    const double finc2 = inc_re * inc_re + inc_im * inc_im;
    if (!(finc2 > 0.0)) return -1;
    const double flux0 = orc_order_flux(&q, 0);
    if (!(flux0 > 0.0)) return -1;
    double R = 0.0, T = 0.0;
    const int32_t m_lo = -(nx - 1) / 2, m_hi = nx / 2;
    for (int32_t m = m_lo; m <= m_hi; ++m) {
        const double w = orc_order_flux(&q, m) / flux0;
        if (!(w > 0.0)) continue;
        double rr = 0, ri = 0, tr = 0, ti = 0;
        for (int32_t i = 0; i < nx; ++i) {
            const double ph = -2.0 * ORC_PI * (double)(((int64_t)m * i) % nx) / (double)nx;
            const double cp = cos(ph), sp = sin(ph);
            const double a = mon_f[i], b = mon_f[nx + i], c = mon_f[2 * nx + i], d = mon_f[3 * nx + i];
            rr += a * cp - b * sp;
            ri += a * sp + b * cp;
            tr += c * cp - d * sp;
            ti += c * sp + d * cp;
        }
        rr /= nx; ri /= nx; tr /= nx; ti /= nx;
        R += w * (rr * rr + ri * ri) / finc2;
        T += w * (tr * tr + ti * ti) / finc2;
    }
    out[0] = R;
    out[1] = T;
    out[2] = 1.0 - R - T;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* TEz with dispersive labels                                                */
/* ------------------------------------------------------------------------- */

/* Edge coefficients of a dispersive TEz run.  An Ex or Ey edge separates two
 * cells; its permittivity is the arithmetic mean of theirs at every frequency
 * (the edge rule of the monochromatic TEz path, reading R14, applied to
 * eps(w) = eps_inf + i sigma/(w eps0) + chi(w)).  So the edge's Ce, Cb of
 * eq. 17 come from the mean eps_inf and the mean sigma, and its polarisation is
 * half the sum of the two cells' pole responses to the edge field
 * (orc_run_te_ade).  Row 0 of Ex is the wall: Ce = 1, Cb = 0.
 * model layout per label: eps_inf, sigma, then (a_p, w_p, g_p) per pole. */
void orc_edge_model_coefficients(const orc_problem* p, const uint8_t* labels, int32_t n_poles,
                                 const double* model, double* cex, double* cbx, double* cey, double* cby)
{
    const int32_t nx = p->nx, ny = p->ny, w = 2 + 3 * n_poles;
    const double dt = orc_time_step(p->h, p->courant);
    for (int32_t j = 0; j < ny; ++j)
        for (int32_t i = 0; i < nx; ++i) {
            double m[2];
            const double* a = model + (size_t)labels[IDX(j, i)] * w;
            if (j == 0) {
                cex[IDX(j, i)] = 1.0;
                cbx[IDX(j, i)] = 0.0;
            } else {
                const double* b = model + (size_t)labels[IDX(j - 1, i)] * w;
                orc_material_eps(0.5 * (a[0] + b[0]), 0.5 * (a[1] + b[1]), dt, m);
                cex[IDX(j, i)] = m[0];
                cbx[IDX(j, i)] = m[1];
            }
            const int32_t il = (i == 0) ? nx - 1 : i - 1;
            const double* c = model + (size_t)labels[IDX(j, il)] * w;
            orc_material_eps(0.5 * (a[0] + c[0]), 0.5 * (a[1] + c[1]), dt, m);
            cey[IDX(j, i)] = m[0];
            cby[IDX(j, i)] = m[1];
        }
}

/* One edge's polarisation step: for each of the two cells beside the edge
 * (labels la, lb) and each pole, P^{n+1} = alpha P^n + xi P^{n-1} + zeta E^n
 * (E and P at integer times in TEz); returns the edge's dP/dt times dt, i.e.
 * half the sum of both cells' increments.  st: [2 sides][n_poles][2] planes
 * at offset o, plane size `plane`. */
static double orc_edge_pol(const double* coef, int32_t w_c, int32_t n_poles, int la, int lb, double e_old,
                           double* st, size_t plane, size_t o)
{
    double dpol = 0.0;
    for (int32_t s = 0; s < 2; ++s) {
        const double* cf = coef + (size_t)(s == 0 ? la : lb) * w_c;
        for (int32_t q = 0; q < n_poles; ++q) {
            double* pc = st + ((size_t)(s * n_poles + q) * 2) * plane;
            double* pp = pc + plane;
            const double pn = cf[2 + 3 * q] * pc[o] + cf[3 + 3 * q] * pp[o] + cf[4 + 3 * q] * e_old;
            dpol += 0.5 * (pn - pc[o]);
            pp[o] = pc[o];
            pc[o] = pn;
        }
    }
    return dpol;
}

/* TEz run with dispersive labels: the steps of orc_run_te with each edge's
 * polarisation updated from its E^n before the E update,
 *   E^{n+1} = Ce E^n + Cb [curl H^{n+1/2} - (P_edge^{n+1} - P_edge^n)/dt].
 * coef: per-label output of orc_ade_coefficients (only the pole terms are
 * used); cex..cby: orc_edge_model_coefficients.  polx, poly: the Ex and Ey
 * edges' polarisation, [2 sides][n_poles][2][ny][nx] = (P^n, P^{n-1}) of each
 * side's pole (side 0: the cell (i, j); side 1: the cell below for Ex, to the
 * left for Ey).  mon: [n_freqs][4][nx] sums of Ex cos(w_f t), Ex sin(w_f t)
 * on the edge rows j_ref and j_trn, t = (n+1) dt, for steps n >= dft_start. */
int orc_run_te_ade(const orc_problem* p, const uint8_t* labels, int32_t n_poles, const double* coef,
                   const double* cex, const double* cbx, const double* cey, const double* cby,
                   const double* e_inc, const double* h_inc, double* hz, double* ex, double* ey,
                   double* phz, double* pex, double* polx, double* poly, int32_t n_begin, int32_t n_end,
                   int32_t n_freqs, const double* lambdas, double* mon)
{
    const int32_t nx = p->nx, ny = p->ny;
    const size_t plane = (size_t)nx * (size_t)ny;
    const int32_t w_c = 2 + 3 * n_poles;
    const double h = p->h;
    const double dt = orc_time_step(p->h, p->courant);
    const double kh = dt / ORC_MU0;
    double* prof_c = malloc(sizeof(double) * 3 * (size_t)ny);
    double* prof_e = malloc(sizeof(double) * 3 * (size_t)ny);
    if (!prof_c || !prof_e) { free(prof_c); free(prof_e); return -2; }
    orc_cpml_profiles(p, prof_c, prof_e);
    for (int32_t i = 0; i < nx; ++i) ex[IDX(0, i)] = 0.0;

    for (int32_t n = n_begin; n < n_end; ++n) {
        const double ex_inc_n = (e_inc && n > 0) ? e_inc[n - 1] : 0.0;
        /* Hz update, eq. 14 (no material) */
#pragma omp parallel for schedule(static)
        for (int32_t j = 0; j < ny; ++j) {
            const double b = prof_c[3 * j], c = prof_c[3 * j + 1], ik = prof_c[3 * j + 2];
            for (int32_t i = 0; i < nx; ++i) {
                const double ex_top = (j + 1 < ny) ? ex[IDX(j + 1, i)] : 0.0;
                const double dex = ex_top - ex[IDX(j, i)];
                double term_y = ik * dex / h;
                if (c != 0.0) {
                    phz[IDX(j, i)] = b * phz[IDX(j, i)] + c * dex / h;
                    term_y += phz[IDX(j, i)];
                }
                if (j == p->j_src) term_y += ex_inc_n / h;
                const int32_t ir = (i + 1 == nx) ? 0 : i + 1;
                const double dey = ey[IDX(j, ir)] - ey[IDX(j, i)];
                hz[IDX(j, i)] -= kh * (dey / h - term_y);
            }
        }
        /* polarisation, then Ex and Ey, eqs. 15-16 */
#pragma omp parallel for schedule(static)
        for (int32_t j = 0; j < ny; ++j) {
            const double b = prof_e[3 * j], c = prof_e[3 * j + 1], ik = prof_e[3 * j + 2];
            for (int32_t i = 0; i < nx; ++i) {
                const int la = labels[IDX(j, i)];
                if (j > 0) {
                    const double dpol = orc_edge_pol(coef, w_c, n_poles, la, labels[IDX(j - 1, i)], ex[IDX(j, i)],
                                                     polx, plane, IDX(j, i));
                    const double dhz = hz[IDX(j, i)] - hz[IDX(j - 1, i)];
                    double term = ik * dhz / h;
                    if (c != 0.0) {
                        pex[IDX(j, i)] = b * pex[IDX(j, i)] + c * dhz / h;
                        term += pex[IDX(j, i)];
                    }
                    if (j == p->j_src + 1 && h_inc) term += h_inc[n] / h;
                    ex[IDX(j, i)] = cex[IDX(j, i)] * ex[IDX(j, i)] + cbx[IDX(j, i)] * (term - dpol / dt);
                }
                const int32_t il = (i == 0) ? nx - 1 : i - 1;
                const double dpol = orc_edge_pol(coef, w_c, n_poles, la, labels[IDX(j, il)], ey[IDX(j, i)], poly,
                                                 plane, IDX(j, i));
                ey[IDX(j, i)] = cey[IDX(j, i)] * ey[IDX(j, i)]
                                + cby[IDX(j, i)] * (-(hz[IDX(j, i)] - hz[IDX(j, il)]) / h - dpol / dt);
            }
        }
        if (mon && n >= p->dft_start) {
            const double t = (n + 1.0) * dt;
            for (int32_t f = 0; f < n_freqs; ++f) {
                const double w = 2.0 * ORC_PI * ORC_C0 / lambdas[f];
                const double cw = cos(w * t), sw = sin(w * t);
                double* mf = mon + (size_t)f * 4 * nx;
                for (int32_t i = 0; i < nx; ++i) {
                    mf[0 * (size_t)nx + i] += ex[IDX(p->j_ref, i)] * cw;
                    mf[1 * (size_t)nx + i] += ex[IDX(p->j_ref, i)] * sw;
                    mf[2 * (size_t)nx + i] += ex[IDX(p->j_trn, i)] * cw;
                    mf[3 * (size_t)nx + i] += ex[IDX(p->j_trn, i)] * sw;
                }
            }
        }
    }
    free(prof_c);
    free(prof_e);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (timing on a given number of host
 * cores); n < 1 is ignored. */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

double orc_c0(void) { return ORC_C0; }
double orc_mu0(void) { return ORC_MU0; }
double orc_eta0_value(void) { return orc_eta0(); }
