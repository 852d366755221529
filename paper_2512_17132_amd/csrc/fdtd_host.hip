// Host orchestration of the gfx950 FDTD library: the C ABI of include/fdtd.h.
//
// Host work is limited to O(ny + n_steps + orders) set-up and post-processing
// in FP64: per-label coefficients (eqs. 1-2, 17), absorbing-layer profiles,
// the incident-field table of the TF/SF line (a 1D vacuum Yee grid, Sec. 2.5),
// monitor phasors, and the final tone fit / flux-weighted order sums of
// Sec. 2.6.  Every per-cell and per-step operation runs in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fdtd.h"
#include "fdtd_adjoint.h"
#include "fdtd_device.h"
#include "fdtd_kernels.h"
#include "fdtd_host.h"

using namespace fdtd;

namespace {

thread_local std::string g_create_error;

constexpr double kPi = 3.14159265358979323846;
constexpr double kC0 = 299792458.0;   // m/s, exact
constexpr double kMu0 = 1.25663706212e-6;   // H/m (CODATA 2018)

// Absorbing layers: polynomial grading of order 3, sigma_max = 0.8 (m+1)/(eta0 h),
// kappa_max = 1, alpha_max = 0.05 omega eps0.  In normalised form
// sigma dt/eps0 = 0.8 (m+1) S1 x^m and alpha dt/eps0 = 0.05 omega dt (1 - x).
constexpr double kPmlOrder = 3.0;
constexpr double kPmlSigmaFac = 0.8;
constexpr double kPmlAlphaFac = 0.05;
constexpr double kPmlKappaMax = 1.0;
// 1D incident-field grid: absorbing cells at each end, vacuum cells on each
// side of the TF/SF row, source cell above the TF/SF row.
constexpr int kAuxPml = 128;
constexpr int kAuxPad = 64;
constexpr int kAuxSrcOff = 16;

struct PmlCoef {
    double b, c, ik;
};

// depth (in cells) of a sample at height y inside a column of n cells with
// d-cell layers at both ends; 0 outside the layers
double layer_depth(double y, int n, int d) {
    if (y < d) return d - y;
    if (y > n - d) return y - (n - d);
    return 0.0;
}

PmlCoef pml_coef(double depth, int d, double s1, double wdt) {
    if (depth <= 0.0) return {0.0, 0.0, 1.0};
    const double x = depth / d;
    const double xm = std::pow(x, kPmlOrder);
    const double sig = kPmlSigmaFac * (kPmlOrder + 1.0) * s1 * xm;
    const double kap = 1.0 + (kPmlKappaMax - 1.0) * xm;
    const double alp = kPmlAlphaFac * wdt * (1.0 - x);
    const double b = std::exp(-(sig / kap + alp));
    const double c = sig * (b - 1.0) / (sig * kap + kap * kap * alp);
    return {b, c, 1.0 / kap};
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

int fdtd_fail(fdtd_ctx* c, int code, const std::string& msg) {
    if (c)
        c->err = msg;
    else
        g_create_error = msg;
    return code;
}
static int fail(fdtd_ctx* c, int code, const std::string& msg) { return fdtd_fail(c, code, msg); }

#define HIPCHK(ctx, expr) FDTD_HIPCHK(ctx, expr)

// ---------------------------------------------------------------------------
// Set-up helpers
// ---------------------------------------------------------------------------

// Incident fields on the TF/SF line from a 1D vacuum Yee grid with the same
// h and dt (normalised units).  Cells k in [0, M) with M = 2 (P + pad) + 1; the
// TF/SF row is k_s = P + pad.  Absorbing layers of P cells at both ends; the
// soft source adds source(n), the drive at t = (n + 1/2) dt, to the cell
// k_s + 16 after each E update.
template <class Source>
static void incident_grid(HostInst& h, int n_steps, Source&& source) {
    const int P = kAuxPml, pad = kAuxPad;
    const int M = 2 * (P + pad) + 1;
    const int ks = P + pad, ksrc = ks + kAuxSrcOff;
    std::vector<double> e(M, 0.0), hh(M + 1, 0.0), pe(M, 0.0), ph(M + 1, 0.0);
    std::vector<PmlCoef> ce(M), ch(M + 1);
    for (int k = 0; k < M; ++k) ce[k] = pml_coef(layer_depth(k + 0.5, M, P), P, h.s1, h.wdt);
    for (int k = 0; k <= M; ++k) ch[k] = pml_coef(layer_depth(k, M, P), P, h.s1, h.wdt);
    h.e_inc.assign(n_steps, 0.0);
    h.h_inc.assign(n_steps, 0.0);
    for (int n = 0; n < n_steps; ++n) {
        h.h_inc[n] = hh[ks + 1];
        for (int k = 0; k < M; ++k) {
            const double dh = hh[k + 1] - hh[k];
            double t = dh * ce[k].ik;
            if (ce[k].c != 0.0) {
                pe[k] = ce[k].b * pe[k] + ce[k].c * dh;
                t += pe[k];
            }
            e[k] -= h.s1 * t;
        }
        e[ksrc] += source(n);
        h.e_inc[n] = e[ks];
        for (int k = 1; k < M; ++k) {
            const double de = e[k] - e[k - 1];
            double t = de * ch[k].ik;
            if (ch[k].c != 0.0) {
                ph[k] = ch[k].b * ph[k] + ch[k].c * de;
                t += ph[k];
            }
            hh[k] -= h.s1 * t;
        }
    }
}

// Monochromatic drive: ramp(t) sin(omega t), raised-cosine ramp over
// ramp_periods periods.
static void incident_table(HostInst& h, int n_steps, double ramp_periods) {
    const double ramp_phase = 2.0 * kPi * ramp_periods;  // omega * T_ramp
    incident_grid(h, n_steps, [&](int n) {
        const double phase = h.wdt * (n + 0.5);
        const double ramp = (phase >= ramp_phase || ramp_phase <= 0.0) ? 1.0 : 0.5 * (1.0 - std::cos(kPi * phase / ramp_phase));
        return ramp * std::sin(phase);
    });
}

// Broadband drive: exp(-((t - t0)/tau)^2) sin(omega0 (t - t0)), omega0 of lambda0.
static void incident_table_pulse(HostInst& h, int n_steps) {
    const double dt = h.s1 * h.dx / kC0;
    incident_grid(h, n_steps, [&](int n) {
        const double t = (n + 0.5) * dt, x = (t - h.t0) / h.tau;
        return std::exp(-x * x) * std::sin(h.wdt * (t - h.t0) / dt);
    });
}

// Incident fields for TEz from a 1D vacuum grid in the TEz order (Hz at
// cells, Ex on edges; Hz first, eq. 14, then Ex, eq. 15).  The soft source
// adds source(n), the drive at t = (n+1) dt, to the edge 16 above the TF/SF
// edge.  Recorded: e_inc[n] = Ex on edge j_src + 1 at (n+1) dt; h_inc[n] = H~z on
// row j_src at (n+1/2) dt.
template <class Source>
static void incident_grid_te(HostInst& h, int n_steps, Source&& source) {
    const int P = kAuxPml, pad = kAuxPad;
    const int M = 2 * (P + pad) + 1;
    const int ks = P + pad, ksrc = ks + 1 + kAuxSrcOff;
    std::vector<double> hz(M, 0.0), ex(M + 1, 0.0), pc(M, 0.0), pe(M + 1, 0.0);
    std::vector<PmlCoef> cc(M), ce(M + 1);
    for (int k = 0; k < M; ++k) cc[k] = pml_coef(layer_depth(k + 0.5, M, P), P, h.s1, h.wdt);
    for (int k = 0; k <= M; ++k) ce[k] = pml_coef(layer_depth(k, M, P), P, h.s1, h.wdt);
    h.e_inc.assign(n_steps, 0.0);
    h.h_inc.assign(n_steps, 0.0);
    for (int n = 0; n < n_steps; ++n) {
        for (int k = 0; k < M; ++k) {
            const double de = ex[k + 1] - ex[k];
            double t = de * cc[k].ik;
            if (cc[k].c != 0.0) {
                pc[k] = cc[k].b * pc[k] + cc[k].c * de;
                t += pc[k];
            }
            hz[k] += h.s1 * t;
        }
        h.h_inc[n] = hz[ks];
        for (int k = 1; k < M; ++k) {
            const double dh = hz[k] - hz[k - 1];
            double t = dh * ce[k].ik;
            if (ce[k].c != 0.0) {
                pe[k] = ce[k].b * pe[k] + ce[k].c * dh;
                t += pe[k];
            }
            ex[k] += h.s1 * t;
        }
        ex[ksrc] += source(n);
        h.e_inc[n] = ex[ks + 1];
    }
}

// Monochromatic TEz drive: ramp(t) sin(omega t) at t = (n+1) dt.
static void incident_table_te(HostInst& h, int n_steps, double ramp_periods) {
    const double ramp_phase = 2.0 * kPi * ramp_periods;
    incident_grid_te(h, n_steps, [&](int n) {
        const double phase = h.wdt * (n + 1.0);
        const double ramp = (phase >= ramp_phase || ramp_phase <= 0.0) ? 1.0 : 0.5 * (1.0 - std::cos(kPi * phase / ramp_phase));
        return ramp * std::sin(phase);
    });
}

// Broadband TEz drive: exp(-((t - t0)/tau)^2) sin(omega0 (t - t0)) at t = (n+1) dt.
static void incident_table_pulse_te(HostInst& h, int n_steps) {
    const double dt = h.s1 * h.dx / kC0;
    incident_grid_te(h, n_steps, [&](int n) {
        const double t = (n + 1.0) * dt, x = (t - h.t0) / h.tau;
        return std::exp(-x * x) * std::sin(h.wdt * (t - h.t0) / dt);
    });
}

// Polarisation state of one field set, in float planes [ny][pitch]: TMz two
// per pole (P^{n+1/2}, P^{n-1/2}), stored as one float2 plane per pole; TEz
// eight per pole (two per pole for each of the two cells beside an edge, for
// Ex and for Ey edges), stored as one float2 plane per edge, side and pole.
// Poles are padded to kMaxPoles.
static int n_pol_planes(int pol) { return (pol ? 8 : 2) * kMaxPoles; }

// Bytes of one field set of an instance as fdtd_create lays it out: Ez, Hx,
// Hy ([ny][pitch] FP32 each), the two absorbing-layer arrays ([2 n_pml + 1]
// [pitch] each) and, for a broadband instance, its polarisation planes, every
// piece aligned to 256 bytes.  The kernels address a set with 32-bit buffer
// offsets and switch a lane's store off with the offset kDropOffset, which the
// hardware discards only while the set's byte count does not exceed it.
static size_t set_layout_bytes(int nx, int ny, int n_pml, bool broadband, int pol) {
    const size_t pitch = (size_t)(nx + 63) / 64 * 64;
    const size_t f = (size_t)ny * pitch * 4, p = (size_t)(2 * n_pml + 1) * pitch * 4;
    size_t b = 3 * align256(f) + 2 * align256(p);
    if (broadband) b += align256((size_t)n_pol_planes(pol) * f);
    return b;
}

// Time of the monitored field after step n, in units of dt: Ez^{n+1/2} (TMz),
// Ex^{n+1} (TEz).
double fdtd_sample_offset(int pol) { return pol ? 1.0 : 0.5; }

// Propagating Bloch orders (discrete dispersion of the Yee scheme) and their
// flux weights w_m = sin(ky_m h)/sin(ky_0 h); paper-literal mode: |m| < Lx/lambda
// with unit weights.
// Propagating orders of instance h at the wavelength lambda (omega dt = wdt)
// and their flux weights relative to order 0.
static void order_set_at(const HostInst& h, double wdt, double lambda, bool literal, std::vector<int>& orders,
                         std::vector<double>& weights) {
    orders.clear();
    weights.clear();
    const double s = std::sin(0.5 * wdt) / h.s1;
    // flux per unit |E_m|^2 of the monitored field: sin(ky h) for Ez (TMz);
    // cot(ky h / 2) for Ex (TEz), from the discrete Wronskian of the Hz equation
    auto flux = [&](int m) {
        const double sx = std::sin(kPi * m / h.nx);
        const double q = s * s - sx * sx;
        if (q <= 0.0 || q >= 1.0) return 0.0;
        if (h.pol) return std::sqrt((1.0 - q) / q);
        return std::sin(2.0 * std::asin(std::sqrt(q)));
    };
    const double f0 = flux(0);
    const int m_lo = -(h.nx - 1) / 2, m_hi = h.nx / 2;
    for (int m = m_lo; m <= m_hi; ++m) {
        double w;
        if (literal)
            w = (std::fabs((double)m) < h.nx * h.dx / lambda) ? 1.0 : 0.0;
        else
            w = f0 > 0 ? flux(m) / f0 : 0.0;
        if (w > 0.0) {
            orders.push_back(m);
            weights.push_back(w);
        }
    }
}

static void order_set(HostInst& h, bool literal) { order_set_at(h, h.wdt, h.lambda0, literal, h.orders, h.weights); }

static int validate(const fdtd_instance* in, int n_inst, const fdtd_opts* o) {
    if (!in || n_inst < 1 || !o) return fail(nullptr, FDTD_E_INVAL, "null input or n_inst < 1");
    if (o->n_steps < 1) return fail(nullptr, FDTD_E_INVAL, "n_steps must be >= 1");
    if (o->t_block < 0 || o->t_block > kMaxTBlock || (o->t_block > 8 && o->t_block % 2))
        return fail(nullptr, FDTD_E_INVAL, "t_block must be 0..8, 10 or 12");
    if (o->band_rows < 0 || o->band_rows > (1 << 20)) return fail(nullptr, FDTD_E_INVAL, "band_rows out of range");
    if (o->kernel < 0 || o->kernel > 1) return fail(nullptr, FDTD_E_INVAL, "kernel must be 0 or 1");
    if (o->adj_t_block < 0 || o->adj_t_block > kMaxAdjTBlock || (o->adj_t_block > 8 && (o->adj_t_block & 1)))
        return fail(nullptr, FDTD_E_INVAL, "adj_t_block must be in 0..8, 10 or 12");
    if (o->checkpoint_every < -1) return fail(nullptr, FDTD_E_INVAL, "checkpoint_every must be >= -1");
    if (o->special_rows < 0 || o->special_rows > kSpecialBand)
        return fail(nullptr, FDTD_E_INVAL, "special_rows must be in 0..16");
    if (o->adj_band_rows < 0 || o->adj_band_rows > (1 << 20))
        return fail(nullptr, FDTD_E_INVAL, "adj_band_rows out of range");
    if (o->bulk_columns != 0 && o->bulk_columns != 64 && o->bulk_columns != kWgColumns)
        return fail(nullptr, FDTD_E_INVAL, "bulk_columns must be 0, 64 or 256");
    for (int q = 0; q < n_inst; ++q) {
        const fdtd_instance& a = in[q];
        char buf[256];
        auto bad = [&](int code, const char* what) {
            snprintf(buf, sizeof buf, "instance %d: %s", q, what);
            return fail(nullptr, code, buf);
        };
        const bool broadband = a.n_freqs != 0;
        if (a.nx < 1 || a.nx > 65536) return bad(FDTD_E_INVAL, "nx must be in 1..65536");
        if (a.n_steps < 0 || a.n_steps > o->n_steps) return bad(FDTD_E_INVAL, "n_steps must be in 0..opts.n_steps");
        if (a.n_freqs < 0 || a.n_freqs > kMaxFreqs) return bad(FDTD_E_INVAL, "n_freqs must be in 0..256");
        {
            const int n = a.n_steps > 0 ? a.n_steps : o->n_steps;
            const int dft = o->dft_start > 0 ? o->dft_start : (broadband ? 0 : n - n / 2);
            if (dft > n - 2) return bad(FDTD_E_INVAL, "monitor window needs at least 2 steps");
        }
        if (a.n_pml < 1 || a.n_pml > kMaxPml) return bad(FDTD_E_INVAL, "n_pml must be in 1..64");
        if (a.ny < 2 * a.n_pml + 8 || a.ny > (1 << 20)) return bad(FDTD_E_INVAL, "ny must be in 2*n_pml+8..2^20");
        if (a.n_labels < 1 || a.n_labels > kMaxLabels) return bad(FDTD_E_INVAL, "n_labels must be in 1..256");
        if (a.polarization != 0 && a.polarization != 1) return bad(FDTD_E_INVAL, "polarization must be 0 (TMz) or 1 (TEz)");
        if (a.polarization == 1 && a.n_labels > kPairStride)
            return bad(FDTD_E_INVAL, "TEz instances take at most 16 labels (pair table of edge materials)");
        if (broadband) {
            if (a.n_poles < 0 || a.n_poles > kMaxPoles) return bad(FDTD_E_INVAL, "n_poles must be in 0..2");
            if (a.n_labels > kMaxLabelsBB) return bad(FDTD_E_INVAL, "broadband runs take at most 64 labels");
            if (!a.model || !a.lambdas) return bad(FDTD_E_INVAL, "broadband run without model or lambdas");
            if (!(a.pulse_tau > 0.0) || !std::isfinite(a.pulse_tau) || !(a.pulse_t0 >= 0.0) || !std::isfinite(a.pulse_t0))
                return bad(FDTD_E_INVAL, "pulse_tau must be positive and pulse_t0 >= 0");
        }
        if (set_layout_bytes(a.nx, a.ny, a.n_pml, broadband, a.polarization) > (size_t)kDropOffset)
            return bad(FDTD_E_INVAL, "instance too large: one field set must not exceed 2 GiB");
        if (!(a.dx > 0.0) || !std::isfinite(a.dx)) return bad(FDTD_E_INVAL, "dx must be positive");
        if (!(a.courant > 0.0) || a.courant > 1.0) return bad(FDTD_E_INVAL, "Courant number must be in (0, 1]");
        if (!(a.lambda0 > 0.0) || !std::isfinite(a.lambda0)) return bad(FDTD_E_INVAL, "lambda0 must be positive");
        const double s1 = a.courant / std::sqrt(2.0);
        const double wdt = 2.0 * kPi * s1 * a.dx / a.lambda0;
        if (!(std::sin(0.5 * wdt) / s1 < 1.0) || wdt >= kPi) return bad(FDTD_E_INVAL, "wavelength below the grid cutoff");
        if (broadband) {
            for (int f = 0; f < a.n_freqs; ++f) {
                const double wf = 2.0 * kPi * s1 * a.dx / a.lambdas[f];
                if (!(a.lambdas[f] > 0.0) || !std::isfinite(a.lambdas[f]) || !(std::sin(0.5 * wf) / s1 < 1.0) || wf >= kPi)
                    return bad(FDTD_E_INVAL, "monitor wavelength not positive or below the grid cutoff");
            }
        }
        if (!(a.n_pml + 1 <= a.j_trn && a.j_trn < a.j_src && a.j_src < a.j_ref && a.j_ref < a.ny - a.n_pml - 1))
            return bad(FDTD_E_INVAL, "rows must satisfy n_pml+1 <= j_trn < j_src < j_ref < ny-n_pml-1");
        if (!a.labels || (!broadband && !a.nk)) return bad(FDTD_E_INVAL, "null labels or nk");
        const int w_model = 2 + 3 * a.n_poles;
        // a label is vacuum when it is the (n, k) = (1, 0) of a monochromatic
        // run, or eps_inf = 1, sigma = 0 and no pole strength in a broadband run
        std::vector<char> vacuum(a.n_labels, 0);
        for (int L = 0; L < a.n_labels; ++L) {
            if (broadband) {
                const double* m = a.model + (size_t)L * w_model;
                for (int k = 0; k < w_model; ++k)
                    if (!std::isfinite(m[k])) return bad(FDTD_E_MATERIAL, "non-finite model parameter");
                if (m[0] < 1.0) return bad(FDTD_E_MATERIAL, "eps_inf must be >= 1");
                if (m[1] < 0.0) return bad(FDTD_E_MATERIAL, "sigma must be >= 0");
                bool none = m[0] == 1.0 && m[1] == 0.0;
                for (int p = 0; p < a.n_poles; ++p) {
                    const double ap = m[2 + 3 * p], wp = m[3 + 3 * p], gp = m[4 + 3 * p];
                    if (ap < 0.0 || wp < 0.0 || gp < 0.0) return bad(FDTD_E_MATERIAL, "pole parameters must be >= 0");
                    const double dt = s1 * a.dx / kC0;
                    if (wp * dt > 1.0) return bad(FDTD_E_MATERIAL, "pole frequency above 1/dt");
                    none = none && ap == 0.0;
                }
                vacuum[L] = none;
            } else {
                const double n = a.nk[2 * L], k = a.nk[2 * L + 1];
                if (!std::isfinite(n) || !std::isfinite(k) || n <= 0.0) return bad(FDTD_E_MATERIAL, "non-finite or non-positive n");
                if (k < 0.0) return bad(FDTD_E_MATERIAL, "k must be >= 0");
                if (n * n - k * k < 1.0) return bad(FDTD_E_MATERIAL, "eps_r = n^2 - k^2 must be >= 1");
                vacuum[L] = n == 1.0 && k == 0.0;
            }
        }
        const size_t cells = (size_t)a.nx * a.ny;
        for (size_t c = 0; c < cells; ++c)
            if (a.labels[c] >= a.n_labels) return bad(FDTD_E_MATERIAL, "label >= n_labels");
        for (int j = 0; j < a.ny; ++j) {
            if (j > a.j_trn && j < a.j_src) continue;
            const uint8_t* row = a.labels + (size_t)j * a.nx;
            for (int i = 0; i < a.nx; ++i)
                if (!vacuum[row[i]]) return bad(FDTD_E_MATERIAL, "rows outside (j_trn, j_src) must be vacuum (n=1, k=0)");
        }
    }
    {
        int longest = 0;
        for (int q = 0; q < n_inst; ++q) longest = std::max(longest, in[q].n_steps > 0 ? in[q].n_steps : o->n_steps);
        if (longest != o->n_steps) return fail(nullptr, FDTD_E_INVAL, "the longest instance must run opts.n_steps steps");
    }
    return FDTD_OK;
}

// Events that only time work on one stream (profiling and the autotuner).  A
// default event ends its record with a system-scope fence, a writeback and
// invalidation of L2 that slows the launches after it (by 6 % per step on the
// TMz dicot at K = 10 and 30 % on its TEz form at one band height); these
// events skip it, which their only use, hipEventElapsedTime after a stream
// synchronisation, does not need.
constexpr unsigned kTimingEvent = hipEventDisableSystemFence;

// Work items of one (K, band) configuration.  Rows whose K-row halo reaches
// an absorbing layer, a domain edge or the TF/SF line, and the monitor rows,
// are cut into thin "special" bands (kSpecialBand rows) run by the kernel
// variant with every row-dependent branch; the interior [jb, jt) is cut into
// bands of B rows run by the branch-free variant.
//
// m selects the instances: those whose run is at least m steps long (the ones a
// launch starting before step m advances).
// Host side of a work list: the items in launch order (special TMz, TEz,
// broadband TMz, broadband TEz; then lean in the same order) and their counts
// in L (L.d unset).
static void build_items(const fdtd_ctx* c, int K, int B, int m, std::vector<WorkItem>& v, ItemList& L) {
    v.clear();
    std::vector<WorkItem> lean, v_te, lean_te, v_bb, lean_bb, v_bt, lean_bt, wg, wg_te;
    int64_t lean_cells = 0;
    const int V = kWave - 2 * K;
    const int Vwg = kWgColumns - 2 * K;
    for (int q = 0; q < (int)c->inst.size(); ++q) {
        const HostInst& h = c->inst[q];
        if (h.n_steps < m) continue;
        std::vector<WorkItem>& vs = h.n_freqs ? (h.pol ? v_bt : v_bb) : (h.pol ? v_te : v);
        std::vector<WorkItem>& vl = h.n_freqs ? (h.pol ? lean_bt : lean_bb) : (h.pol ? lean_te : lean);
        const int ns = (h.nx + V - 1) / V;
        const int jb = std::min(h.ny, std::max(h.n_pml + 1, h.j_trn + 1) + K);
        const int jt = std::max(jb, std::min(h.ny - h.n_pml - 1, h.j_src) - K);
        auto add = [&](int j0, int j1, bool special) {
            for (int s = 0; s < ns; ++s) {
                WorkItem w{};
                w.inst = q;
                w.x0 = s * V;
                w.j0 = j0;
                w.j1 = j1;
                w.special = special ? 1 : 0;
                (special ? vs : vl).push_back(w);
            }
        };
        for (int j0 = 0; j0 < jb; j0 += c->SB) add(j0, std::min(jb, j0 + c->SB), true);
        for (int j0 = jb; j0 < jt; j0 += B) add(j0, std::min(jt, j0 + B), false);
        if (!h.n_freqs)
            for (int j0 = jb; j0 < jt; j0 += B)
                for (int x0 = 0; x0 < h.nx; x0 += Vwg) {
                    WorkItem w{};
                    w.inst = q;
                    w.x0 = x0;
                    w.j0 = j0;
                    w.j1 = std::min(jt, j0 + B);
                    (h.pol ? wg_te : wg).push_back(w);
                }
        lean_cells += (int64_t)(jt - jb) * h.nx;
        for (int j0 = jt; j0 < h.ny; j0 += c->SB) add(j0, std::min(h.ny, j0 + c->SB), true);
    }
    // order: special TMz, TEz, broadband TMz, broadband TEz; then lean in the same order
    L = ItemList{};
    L.n_special_te = (int)v_te.size();
    L.n_lean_te = (int)lean_te.size();
    L.n_special_bb = (int)v_bb.size();
    L.n_lean_bb = (int)lean_bb.size();
    L.n_special_bt = (int)v_bt.size();
    L.n_lean_bt = (int)lean_bt.size();
    v.insert(v.end(), v_te.begin(), v_te.end());
    v.insert(v.end(), v_bb.begin(), v_bb.end());
    v.insert(v.end(), v_bt.begin(), v_bt.end());
    lean.insert(lean.end(), lean_te.begin(), lean_te.end());
    lean.insert(lean.end(), lean_bb.begin(), lean_bb.end());
    lean.insert(lean.end(), lean_bt.begin(), lean_bt.end());
    L.n_special = (int)v.size();
    L.n_lean = (int)lean.size();
    L.lean_cells = lean_cells;
    v.insert(v.end(), lean.begin(), lean.end());
    L.wg = (int)v.size();
    L.n_lean_wg = (int)wg.size();
    v.insert(v.end(), wg.begin(), wg.end());
    L.wg_te = (int)v.size();
    L.n_lean_wg_te = (int)wg_te.size();
    v.insert(v.end(), wg_te.begin(), wg_te.end());
}

static ItemList* item_list(fdtd_ctx* c, int K, int B, int m) {
    auto key = std::make_tuple(K, B, c->SB, m);
    auto it = c->items.find(key);
    if (it != c->items.end()) return &it->second;
    std::vector<WorkItem> v;
    ItemList L;
    build_items(c, K, B, m, v, L);
    if (!v.empty()) {
        if (hipMalloc(&L.d, sizeof(WorkItem) * v.size()) != hipSuccess) return nullptr;
        if (hipMemcpy(L.d, v.data(), sizeof(WorkItem) * v.size(), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    }
    return &(c->items[key] = L);
}

static int zero_state(fdtd_ctx* c) {
    for (auto& h : c->inst) {
        const InstDev& d = h.dev;
        const size_t f = (size_t)h.ny * h.pitch, p = (size_t)(2 * h.n_pml + 1) * h.pitch;
        for (int b = 0; b < 2; ++b) {
            HIPCHK(c, launch_fill(d.ez[b], f, 0.f, c->stream));
            HIPCHK(c, launch_fill(d.hx[b], f, 0.f, c->stream));
            HIPCHK(c, launch_fill(d.hy[b], f, 0.f, c->stream));
            HIPCHK(c, launch_fill(d.pe[b], p, 0.f, c->stream));
            HIPCHK(c, launch_fill(d.ph[b], p, 0.f, c->stream));
        }
        HIPCHK(c, launch_fill(d.mon, (size_t)8 * h.pitch * std::max(1, h.n_freqs), 0.f, c->stream));
        if (h.n_freqs)
            for (int b = 0; b < 2; ++b)
                HIPCHK(c, launch_fill((float*)((char*)d.ez[b] + d.off_pol), (size_t)n_pol_planes(h.pol) * h.ny * h.pitch, 0.f,
                                      c->stream));
        HIPCHK(c, launch_fill_i32(d.status, 1, 0, c->stream));
    }
    for (auto& h : c->inst) h.cur_end = 0;
    c->cur = 0;
    c->step = 0;
    c->adj.recorded = false;
    return FDTD_OK;
}

// ---------------------------------------------------------------------------
// Stepping
// ---------------------------------------------------------------------------

// Smallest run length above `step`: a launch that starts at `step` advances
// exactly the instances whose run is at least this long, and must end by it.
static int active_end(const fdtd_ctx* c, int step) {
    int m = INT_MAX;
    for (auto& h : c->inst)
        if (h.n_steps > step) m = std::min(m, h.n_steps);
    return m;
}

// The launches that advance `n` steps from `step` with K steps per launch:
// f(first step, steps, m) for each, m selecting the instances it advances.
template <class F>
static void plan_launches(const fdtd_ctx* c, int step, int n, int K, F&& f) {
    const int end = step + n;
    while (step < end) {
        const int m = active_end(c, step);
        const int k = fdtd_launch_steps(K, std::min(end, m) - step);
        f(step, k, m);
        step += k;
    }
}

// Records the field set of every instance whose run ends at the current step.
static void mark_ends(fdtd_ctx* c) {
    for (auto& h : c->inst)
        if (h.n_steps == c->step) h.cur_end = c->cur;
}

// One launch of k steps from the current step over the instances whose run is
// at least m steps long.
static int launch_items(fdtd_ctx* c, int k, int m, const ItemList* L, bool allow_timing);

static int enqueue_launch(fdtd_ctx* c, int k, int B, int m) {
    ItemList* L = item_list(c, k, B, m);
    if (!L) return fail(c, FDTD_E_NOMEM, "work-item list allocation failed");
    return launch_items(c, k, m, L, true);
}

// The launches of one step block over the items of L (L->d a device copy of
// the list build_items makes): special items on the auxiliary stream, lean
// items on the context's stream, joined before the next block.
static int launch_items(fdtd_ctx* c, int k, int m, const ItemList* L, bool allow_timing) {
    // The few special items (thin bands near the layers, the source line and
    // the monitors) are latency-bound: run them on the auxiliary stream,
    // concurrently with the lean items, and join before the next launch.  A
    // context holding broadband TEz instances keeps to its own stream: with
    // the special launch concurrent on the auxiliary stream, replays of a
    // captured run of such a context have differed from direct launches in
    // the last bits.  There the broadband TEz special items share one kernel
    // launch with their lean items, and the other kinds' special items run
    // ahead of the lean launches.
    const int ns_tm = L->n_special - L->n_special_te - L->n_special_bb - L->n_special_bt;
    const int nl_tm = L->n_lean - L->n_lean_te - L->n_lean_bb - L->n_lean_bt;
    const int ns_rest = L->n_special - L->n_special_bt;
    const bool overlap = !c->has_bt;
    hipStream_t ss = overlap ? c->aux : c->stream;
    auto monitors = [&](hipStream_t st) -> int {
        for (auto& h : c->inst)
            if (h.n_freqs && h.n_steps >= m) HIPCHK(c, launch_monitor_bb(h.dev, c->step, k, st));
        return FDTD_OK;
    };
    if (ns_rest > 0) {
        const WorkItem* d = L->d;
        if (overlap) {
            HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
            HIPCHK(c, hipStreamWaitEvent(c->aux, c->ev_fork, 0));
        }
        HIPCHK(c, launch_tblock(k, true, c->d_insts, d, ns_tm, c->step, c->cur, ss));
        d += ns_tm;
        HIPCHK(c, launch_tblock_te(k, true, c->d_insts, d, L->n_special_te, c->step, c->cur, ss));
        d += L->n_special_te;
        HIPCHK(c, launch_tblock_bb(k, true, c->d_insts, d, L->n_special_bb, c->step, c->cur, ss));
        if (overlap) {
            if (L->n_special_bb > 0) {
                const int rc = monitors(ss);
                if (rc != FDTD_OK) return rc;
            }
            HIPCHK(c, hipEventRecord(c->ev_join, c->aux));
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = allow_timing && c->prof && L->n_lean > 0 && (c->prof_seen++ % c->prof) == 0;
    if (timed) {
        HIPCHK(c, hipEventCreateWithFlags(&e0, kTimingEvent));
        HIPCHK(c, hipEventCreateWithFlags(&e1, kTimingEvent));
        HIPCHK(c, hipEventRecord(e0, c->stream));
    }
    HIPCHK(c, fdtd_launch_bulk_tm(c, k, c->d_insts, L, c->step, c->cur, c->stream));
    HIPCHK(c, fdtd_launch_bulk_te(c, k, c->d_insts, L, c->step, c->cur, c->stream));
    const WorkItem* d = L->d + L->n_special + nl_tm + L->n_lean_te;
    HIPCHK(c, launch_tblock_bb(k, false, c->d_insts, d, L->n_lean_bb, c->step, c->cur, c->stream));
    d += L->n_lean_bb;
    HIPCHK(c, launch_tblock_bt(k, c->d_insts, L->d + ns_rest, L->n_special_bt, d, L->n_lean_bt, c->step, c->cur,
                               c->stream));
    if (timed) {
        HIPCHK(c, hipEventRecord(e1, c->stream));
        c->ev.emplace_back(e0, e1);
        c->ev_cells.push_back(L->lean_cells);
    }
    if (!overlap && L->n_special_bb + L->n_special_bt > 0) {
        // the monitor rows' fields of this launch are in the capture slots
        const int rc = monitors(c->stream);
        if (rc != FDTD_OK) return rc;
    }
    if (ns_rest > 0 && overlap) HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
    c->cur ^= 1;
    c->step += k;
    mark_ends(c);
    return FDTD_OK;
}

ItemList* fdtd_item_list(fdtd_ctx* c, int K, int B) { return item_list(c, K, B, active_end(c, 0)); }

hipError_t fdtd_launch_bulk_tm(const fdtd_ctx* c, int k, const InstDev* insts, const ItemList* L, int n0, int cur,
                               hipStream_t s, bool rec, int hslot0) {
    if (c->W == kWgColumns) return launch_tblock_wg(k, insts, L->d + L->wg, L->n_lean_wg, n0, cur, s, rec, hslot0);
    const int nl_tm = L->n_lean - L->n_lean_te - L->n_lean_bb - L->n_lean_bt;
    return launch_tblock(k, false, insts, L->d + L->n_special, nl_tm, n0, cur, s, rec, hslot0);
}

hipError_t fdtd_launch_bulk_te(const fdtd_ctx* c, int k, const InstDev* insts, const ItemList* L, int n0, int cur,
                               hipStream_t s) {
    if (c->W == kWgColumns) return launch_tblock_te_wg(k, insts, L->d + L->wg_te, L->n_lean_wg_te, cur, s);
    const int nl_tm = L->n_lean - L->n_lean_te - L->n_lean_bb - L->n_lean_bt;
    return launch_tblock_te(k, false, insts, L->d + L->n_special + nl_tm, L->n_lean_te, n0, cur, s);
}

int fdtd_inst_cur(const fdtd_ctx* c, int q) {
    const HostInst& h = c->inst[q];
    return c->step >= h.n_steps ? h.cur_end : c->cur;
}

int fdtd_enqueue_steps(fdtd_ctx* c, int n_steps, int K, int B) {
    if (c->opts.kernel == 1) {
        // A broadband instance's monitored steps leave their field in capture
        // slots; the monitor kernel adds up to kMaxTBlock of them at a time,
        // and whatever is pending at the end of the call.
        const size_t ni = c->inst.size();
        std::vector<int> pend(ni, 0), pend_n0(ni, 0);
        auto flush = [&](size_t q) -> int {
            if (pend[q] > 0) HIPCHK(c, launch_monitor_bb(c->inst[q].dev, pend_n0[q], pend[q], c->stream));
            pend[q] = 0;
            return FDTD_OK;
        };
        for (int done = 0; done < n_steps; ++done) {
            for (size_t q = 0; q < ni; ++q) {
                HostInst& h = c->inst[q];
                if (h.n_steps <= c->step) continue;
                hipEvent_t e0 = nullptr, e1 = nullptr;
                const bool timed = c->prof && (c->prof_seen++ % c->prof) == 0;
                if (timed) {
                    HIPCHK(c, hipEventCreateWithFlags(&e0, kTimingEvent));
                    HIPCHK(c, hipEventCreateWithFlags(&e1, kTimingEvent));
                    HIPCHK(c, hipEventRecord(e0, c->stream));
                }
                if (h.n_freqs) {
                    const bool mon = c->step >= h.dev.dft_start;
                    if (mon && pend[q] == 0) pend_n0[q] = c->step;
                    HIPCHK(c, launch_plain_step_broadband(h.dev, c->step, c->cur, mon ? pend[q] : 0, c->stream));
                    if (mon && ++pend[q] == kMaxTBlock) {
                        const int rc = flush(q);
                        if (rc != FDTD_OK) return rc;
                    }
                } else {
                    HIPCHK(c, launch_plain_step(h.dev, c->step, c->cur, c->stream));
                }
                if (timed) {
                    HIPCHK(c, hipEventRecord(e1, c->stream));
                    c->ev.emplace_back(e0, e1);
                    c->ev_cells.push_back((int64_t)h.cells());
                }
            }
            c->step += 1;   // the plain kernels update one field set in place
            mark_ends(c);
        }
        for (size_t q = 0; q < ni; ++q) {
            const int rc = flush(q);
            if (rc != FDTD_OK) return rc;
        }
        return FDTD_OK;
    }
    int rc = FDTD_OK;
    plan_launches(c, c->step, n_steps, K, [&](int, int k, int m) {
        if (rc == FDTD_OK) rc = enqueue_launch(c, k, B, m);
    });
    return rc;
}
static int ensure_config(fdtd_ctx* c) {
    if (c->K > 0 && c->B > 0) return FDTD_OK;
    c->K = c->opts.t_block > 0 ? c->opts.t_block : 0;
    c->B = c->opts.band_rows > 0 ? c->opts.band_rows : 0;
    c->SB = c->opts.special_rows > 0 ? c->opts.special_rows : kSpecialBand;
    if (c->opts.kernel == 1) {
        c->K = 1;
        c->B = 1;
        return FDTD_OK;
    }
    if (c->K == 0 || c->B == 0) {
        double rate = 0;
        const int rc = fdtd_autotune(c, 0, &rate);
        if (rc != FDTD_OK) return rc;
    }
    return FDTD_OK;
}

// ---------------------------------------------------------------------------
// Stepping without allocation
// ---------------------------------------------------------------------------

// Work-item lists of fdtd_step_noalloc: a fixed array in device memory, one
// per device, held until the process ends (kNoallocItems x 32 bytes = 1 MiB).
// Host code never names it directly: hipGetSymbolAddress gives each device's
// address once, with that device current, and only that address is passed
// to copies and kernels.
constexpr int kNoallocItems = 32768;
static __device__ __align__(256) WorkItem scratch[kNoallocItems];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static WorkItem* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (looked up on the first call
// for that device), or null with a message in c->err.
static WorkItem* scratch_on(fdtd_ctx* c, int device) {
    if (device < 0 || device >= kMaxDevices) {
        fail(c, FDTD_E_HIP, "device index beyond the library's table of devices");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[device]) return g_scratch_ptr[device];
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) {
        fail(c, FDTD_E_HIP, "hipGetDevice failed");
        return nullptr;
    }
    if (prev != device && hipSetDevice(device) != hipSuccess) {
        fail(c, FDTD_E_HIP, "hipSetDevice failed");
        return nullptr;
    }
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess || !ptr) {
        fail(c, FDTD_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        return nullptr;
    }
    g_scratch_ptr[device] = (WorkItem*)ptr;
    return g_scratch_ptr[device];
}

// Launch shapes the autotuner has chosen, shared by the contexts of the
// process so that a context whose instances repeat an earlier context's
// layout on the same kind of device starts without trials.  The key holds the
// device's architecture and compute-unit count; per instance, the grid, the
// absorbing-layer depth, the source and monitor rows (they decide which bands
// take the special kernel) and the kind of run; and the options that narrow
// the search (fixed steps per launch, band rows, special rows, bulk columns,
// graph replay), so that a shape chosen under them is not handed to a context
// free of them.  Contexts on different host threads may tune at once: every
// access holds the lock.
static std::mutex g_tune_mutex;
struct TunedShape {
    int K, B, SB;
    bool graph_faster = true;
    int W = 64;
};
static std::map<std::string, TunedShape> g_tune_cache;

static std::string tune_key(const fdtd_ctx* c) {
    std::string key;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess)
        key = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + ":";
    else
        key = "device" + std::to_string(c->device) + ":";
    for (auto& h : c->inst)
        key += std::to_string(h.nx) + "x" + std::to_string(h.ny) + "p" + std::to_string(h.n_pml) + "r" +
               std::to_string(h.j_trn) + "," + std::to_string(h.j_src) + "," + std::to_string(h.j_ref) +
               (h.n_freqs ? "b" + std::to_string(h.n_poles) : std::string()) + (h.pol ? "e;" : "m;");
    const fdtd_opts& o = c->opts;
    key += "|" + std::to_string(o.t_block) + "," + std::to_string(o.band_rows) + "," + std::to_string(o.special_rows) +
           "," + std::to_string(o.bulk_columns) + "," + std::to_string(o.use_graph);
    return key;
}

static bool tune_lookup(const std::string& key, TunedShape& shape) {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tune_cache.find(key);
    if (it == g_tune_cache.end()) return false;
    shape = it->second;
    return true;
}

static void tune_store(const std::string& key, TunedShape shape) {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_cache[key] = shape;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char* fdtd_strerror(int code) {
    switch (code) {
        case FDTD_OK: return "ok";
        case FDTD_E_INVAL: return "invalid argument";
        case FDTD_E_MATERIAL: return "invalid material or label map";
        case FDTD_E_NOMEM: return "out of memory";
        case FDTD_E_HIP: return "HIP runtime error";
        case FDTD_E_STATE: return "call out of order";
        case FDTD_E_UNSTABLE: return "non-finite monitor sum";
        default: return "unknown status";
    }
}

const char* fdtd_last_error(const fdtd_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int fdtd_create(const fdtd_instance* in, int32_t n_inst, const fdtd_opts* opts_in, void* stream, fdtd_ctx** out) {
    g_create_error.clear();
    if (!out) return fail(nullptr, FDTD_E_INVAL, "out is null");
    int rc = validate(in, n_inst, opts_in);
    if (rc != FDTD_OK) return rc;
    std::unique_ptr<fdtd_ctx> c(new (std::nothrow) fdtd_ctx());
    if (!c) return fail(nullptr, FDTD_E_NOMEM, "host allocation failed");
    c->opts = *opts_in;
    c->W = opts_in->bulk_columns > 0 ? opts_in->bulk_columns : 64;
    fdtd_opts& o = c->opts;
    if (!(o.ramp_periods > 0.0)) o.ramp_periods = 5.0;
    // checkpoint_every = -1 is resolved by the first recorded run, once the
    // launch shape is known

    // host tables
    c->inst.resize(n_inst);
    for (int q = 0; q < n_inst; ++q) {
        const fdtd_instance& a = in[q];
        HostInst& h = c->inst[q];
        h.nx = a.nx;
        h.ny = a.ny;
        h.pitch = (a.nx + 63) / 64 * 64;
        h.n_pml = a.n_pml;
        h.j_src = a.j_src;
        h.j_ref = a.j_ref;
        h.j_trn = a.j_trn;
        h.n_labels = a.n_labels;
        h.pol = a.polarization;
        h.n_freqs = a.n_freqs;
        c->has_bt = c->has_bt || (a.n_freqs && a.polarization);
        c->has_mono = c->has_mono || !a.n_freqs;
        h.n_steps = a.n_steps > 0 ? a.n_steps : o.n_steps;
        // a broadband run transforms the whole record; a monochromatic one fits
        // the tone over the last half
        h.dft_start = o.dft_start > 0 ? o.dft_start : (h.n_freqs ? 0 : h.n_steps - h.n_steps / 2);
        h.dx = a.dx;
        h.courant = a.courant;
        h.lambda0 = a.lambda0;
        h.s1 = a.courant / std::sqrt(2.0);
        h.wdt = 2.0 * kPi * h.s1 * a.dx / a.lambda0;
        h.labels.assign(a.labels, a.labels + h.cells());
        if (h.n_freqs) {
            h.n_poles = a.n_poles;
            h.model.assign(a.model, a.model + (size_t)a.n_labels * (2 + 3 * a.n_poles));
            h.lambdas.assign(a.lambdas, a.lambdas + a.n_freqs);
            h.tau = a.pulse_tau;
            h.t0 = a.pulse_t0;
            if (h.pol)
                incident_table_pulse_te(h, h.n_steps);
            else
                incident_table_pulse(h, h.n_steps);
            h.f_orders.resize(h.n_freqs);
            h.f_weights.resize(h.n_freqs);
            for (int f = 0; f < h.n_freqs; ++f)
                order_set_at(h, 2.0 * kPi * h.s1 * h.dx / h.lambdas[f], h.lambdas[f], o.literal_orders != 0,
                             h.f_orders[f], h.f_weights[f]);
        } else {
            h.nk.assign(a.nk, a.nk + 2 * a.n_labels);
            if (h.pol)
                incident_table_te(h, h.n_steps, o.ramp_periods);
            else
                incident_table(h, h.n_steps, o.ramp_periods);
            order_set(h, o.literal_orders != 0);
        }
    }
    // Gram matrix of the tone fit: identical for every instance only if they
    // share omega dt; it is therefore computed per instance in fdtd_spectra.

    // device memory: one slab, carved per instance
    std::vector<size_t> off;
    size_t total = 0;
    auto take = [&](size_t bytes) {
        off.push_back(total);
        total += align256(bytes);
    };
    for (auto& h : c->inst) {
        // psi arrays: the 2 n_pml layer rows and one spare row that the
        // streaming kernel reads and writes for rows outside the layers
        const size_t f = (size_t)h.ny * h.pitch * 4, p = (size_t)(2 * h.n_pml + 1) * h.pitch * 4;
        for (int b = 0; b < 2; ++b) {
            take(f); take(f); take(f); take(p); take(p);
            if (h.n_freqs) take((size_t)n_pol_planes(h.pol) * f);   // polarisation planes
        }
        take((size_t)h.ny * h.pitch);                    // labels
        take(sizeof(float2) * kMaxLabels);               // coef
        take(sizeof(float4) * h.ny);                     // prof_e
        take(sizeof(float4) * h.ny);                     // prof_h
        const size_t nf = std::max(1, h.n_freqs);
        take(sizeof(float2) * h.n_steps);                // inc
        take(sizeof(float2) * h.n_steps * nf);           // phasor
        take((size_t)8 * h.pitch * 4 * nf);              // monitors
        take(256);                                       // status
        if (h.n_freqs) {
            take(sizeof(float4) * kMaxPoles * kMaxLabels);               // pole coefficients
            take((size_t)2 * kMaxTBlock * h.pitch * 4);                  // monitor-row captures
        }
    }
    c->slab_bytes = total;
    int dev = 0;
    HIPCHK(nullptr, hipGetDevice(&dev));
    c->device = dev;
    if (hipMalloc(&c->slab, total) != hipSuccess) {
        (void)hipGetLastError();
        return fail(nullptr, FDTD_E_NOMEM, "device allocation of " + std::to_string(total) + " bytes failed");
    }
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        HIPCHK(nullptr, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    // auxiliary stream (default priority) for the special work items, and the
    // fork/join events that order it against the main stream
    HIPCHK(nullptr, hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    HIPCHK(nullptr, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIPCHK(nullptr, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    size_t k = 0;
    std::vector<InstDev> devs(n_inst);
    for (int q = 0; q < n_inst; ++q) {
        HostInst& h = c->inst[q];
        InstDev& d = h.dev;
        char* pol_planes = nullptr;
        for (int b = 0; b < 2; ++b) {
            d.ez[b] = (float*)(c->slab + off[k++]);
            d.hx[b] = (float*)(c->slab + off[k++]);
            d.hy[b] = (float*)(c->slab + off[k++]);
            d.pe[b] = (float*)(c->slab + off[k++]);
            d.ph[b] = (float*)(c->slab + off[k++]);
            if (h.n_freqs) {
                char* pp = c->slab + off[k++];
                if (b == 0) pol_planes = pp;
            }
        }
        uint8_t* lab = (uint8_t*)(c->slab + off[k++]);
        float2* coef = (float2*)(c->slab + off[k++]);
        float4* pre = (float4*)(c->slab + off[k++]);
        float4* prh = (float4*)(c->slab + off[k++]);
        float2* inc = (float2*)(c->slab + off[k++]);
        float2* pha = (float2*)(c->slab + off[k++]);
        d.mon = (float*)(c->slab + off[k++]);
        d.hist = nullptr;
        d.status = (int*)(c->slab + off[k++]);
        d.n_freqs = h.n_freqs;
        d.n_poles = 0;
        d.poles = nullptr;
        d.off_pol = 0;
        d.cap = nullptr;
        float4* poles = nullptr;
        if (h.n_freqs) {
            poles = (float4*)(c->slab + off[k++]);
            d.poles = poles;
            d.cap = (float*)(c->slab + off[k++]);
            d.n_poles = kMaxPoles;   // poles beyond h.n_poles have zero coefficients
        }
        d.lab = lab;
        d.coef = coef;
        d.prof_e = pre;
        d.prof_h = prh;
        d.inc = inc;
        d.phasor = pha;
        d.nx = h.nx;
        d.ny = h.ny;
        d.pitch = h.pitch;
        d.n_pml = h.n_pml;
        d.j_src = h.j_src;
        d.j_ref = h.j_ref;
        d.j_trn = h.j_trn;
        d.dft_start = h.dft_start;
        d.n_labels = h.n_labels;
        d.pol = h.pol;
        d.n_coef = h.pol ? kPairTable : h.n_labels;
        d.s1 = (float)h.s1;
        d.off_hx = (unsigned)((char*)d.hx[0] - (char*)d.ez[0]);
        d.off_hy = (unsigned)((char*)d.hy[0] - (char*)d.ez[0]);
        d.off_pe = (unsigned)((char*)d.pe[0] - (char*)d.ez[0]);
        d.off_ph = (unsigned)((char*)d.ph[0] - (char*)d.ez[0]);
        d.set_bytes = (unsigned)((char*)d.ph[0] - (char*)d.ez[0] + align256((size_t)(2 * h.n_pml + 1) * h.pitch * 4));
        if (h.n_freqs) {
            // the polarisation planes follow the layer rows inside each set
            d.off_pol = (unsigned)(pol_planes - (char*)d.ez[0]);
            d.set_bytes = d.off_pol + (unsigned)align256((size_t)n_pol_planes(h.pol) * h.ny * h.pitch * 4);
        }
        if (d.set_bytes != set_layout_bytes(h.nx, h.ny, h.n_pml, h.n_freqs != 0, h.pol))
            return fail(nullptr, FDTD_E_INVAL, "internal error: field-set layout differs from its validated size");

        // labels, padded rows
        std::vector<uint8_t> lp((size_t)h.ny * h.pitch, 0);
        for (int j = 0; j < h.ny; ++j) memcpy(&lp[(size_t)j * h.pitch], &h.labels[(size_t)j * h.nx], h.nx);
        HIPCHK(nullptr, hipMemcpy(lab, lp.data(), lp.size(), hipMemcpyHostToDevice));
        // coefficients (eqs. 1-2, 17 in normalised form): per label for TMz;
        // for TEz per pair of labels an edge separates, from the means of eps_r
        // and sigma dt/eps0 = 2 n k omega dt
        std::vector<float2> cf(kMaxLabels, make_float2(1.f, 0.f));
        auto coef_of = [&](double eps, double sdt) {   // sdt = sigma dt / eps0
            const double a = 0.5 * sdt / eps;
            return make_float2((float)((1.0 - a) / (1.0 + a)), (float)(h.s1 / (eps * (1.0 + a))));
        };
        auto eps_of = [&](int L) { return h.nk[2 * L] * h.nk[2 * L] - h.nk[2 * L + 1] * h.nk[2 * L + 1]; };
        auto sdt_of = [&](int L) { return 2.0 * h.nk[2 * L] * h.nk[2 * L + 1] * h.wdt; };
        if (h.n_freqs) {
            // broadband: Ce, Cb at (eps_inf, sigma); per pole the recursion
            // P^{n+1/2} = alpha P^{n-1/2} + xi P^{n-3/2} + zeta E^{n-1/2} of
            // P'' + g P' + w_p^2 P = a E (P normalised by eps0) by central
            // differences, and Cp = 1/(eps_inf (1 + a)) of the E update's
            // -Cp (P^{n+1/2} - P^{n-1/2})
            const int w = 2 + 3 * h.n_poles;
            const double dt = h.s1 * h.dx / kC0;
            std::vector<float4> pt4((size_t)kMaxPoles * kMaxLabels, make_float4(0.f, 0.f, 0.f, 0.f));
            for (int L = 0; L < h.n_labels; ++L) {
                const double* m = &h.model[(size_t)L * w];
                const double sdt = m[1] * h.s1 * h.dx * kMu0 * kC0;   // sigma dt / eps0
                cf[L] = coef_of(m[0], sdt);
                const double cp = 1.0 / (m[0] * (1.0 + 0.5 * sdt / m[0]));
                // poles beyond the instance's own: zero coefficients (their
                // polarisation stays 0), Cp kept for the record
                for (int p = h.n_poles; p < kMaxPoles; ++p)
                    pt4[(size_t)p * kMaxLabels + L] = make_float4(0.f, 0.f, 0.f, (float)cp);
                for (int p = 0; p < h.n_poles; ++p) {
                    const double ap = m[2 + 3 * p], wp = m[3 + 3 * p], g = m[4 + 3 * p];
                    const double den = 1.0 + 0.5 * g * dt;
                    pt4[(size_t)p * kMaxLabels + L] =
                        make_float4((float)((2.0 - wp * wp * dt * dt) / den), (float)((0.5 * g * dt - 1.0) / den),
                                    (float)(ap * dt * dt / den), (float)cp);
                }
            }
            if (h.pol) {
                // TEz: an edge's (Ce, Cb) from the mean eps_inf and the mean
                // sigma of the two cells it separates (its polarisation is half
                // the sum of theirs, in k_plain_te_e_ade)
                for (int La = 0; La < h.n_labels; ++La)
                    for (int Lb = 0; Lb < h.n_labels; ++Lb) {
                        const double* ma = &h.model[(size_t)La * w];
                        const double* mb = &h.model[(size_t)Lb * w];
                        const double sdt = 0.5 * (ma[1] + mb[1]) * h.s1 * h.dx * kMu0 * kC0;
                        cf[La * kPairStride + Lb] = coef_of(0.5 * (ma[0] + mb[0]), sdt);
                    }
            }
            HIPCHK(nullptr, hipMemcpy(poles, pt4.data(), sizeof(float4) * pt4.size(), hipMemcpyHostToDevice));
        } else if (h.pol == 0) {
            for (int L = 0; L < h.n_labels; ++L) cf[L] = coef_of(eps_of(L), sdt_of(L));
        } else {
            for (int La = 0; La < h.n_labels; ++La)
                for (int Lb = 0; Lb < h.n_labels; ++Lb)
                    cf[La * kPairStride + Lb] = coef_of(0.5 * (eps_of(La) + eps_of(Lb)), 0.5 * (sdt_of(La) + sdt_of(Lb)));
        }
        HIPCHK(nullptr, hipMemcpy(coef, cf.data(), sizeof(float2) * kMaxLabels, hipMemcpyHostToDevice));
        // absorbing-layer profiles at Ez rows (y = j + 1/2) and Hx rows (y = j)
        std::vector<float4> pe(h.ny), ph(h.ny);
        for (int j = 0; j < h.ny; ++j) {
            PmlCoef a = pml_coef(layer_depth(j + 0.5, h.ny, h.n_pml), h.n_pml, h.s1, h.wdt);
            PmlCoef b = pml_coef(j == 0 ? 0.0 : layer_depth(j, h.ny, h.n_pml), h.n_pml, h.s1, h.wdt);
            pe[j] = make_float4((float)a.b, (float)a.c, (float)a.ik, 0.f);
            ph[j] = make_float4((float)b.b, (float)b.c, (float)b.ik, 0.f);
        }
        HIPCHK(nullptr, hipMemcpy(pre, pe.data(), sizeof(float4) * h.ny, hipMemcpyHostToDevice));
        HIPCHK(nullptr, hipMemcpy(prh, ph.data(), sizeof(float4) * h.ny, hipMemcpyHostToDevice));
        // incident table and phasors
        const int nf = std::max(1, h.n_freqs);
        std::vector<float2> it(h.n_steps), pt((size_t)h.n_steps * nf);
        h.inc_c = h.inc_s = 0.0;
        if (h.n_freqs) {
            h.f_inc_re.assign(h.n_freqs, 0.0);
            h.f_inc_im.assign(h.n_freqs, 0.0);
        }
        for (int n = 0; n < h.n_steps; ++n) {
            // .y feeds the centre-field update of row j_src, .x the edge update
            // of edge j_src + 1: TMz (E_inc(n+1/2), H~x_inc(n)), TEz (H~z_inc(n+1/2),
            // Ex_inc(n))
            if (h.pol == 0)
                it[n] = make_float2((float)h.e_inc[n], (float)h.h_inc[n]);
            else
                it[n] = make_float2((float)h.h_inc[n], n > 0 ? (float)h.e_inc[n - 1] : 0.f);
            if (h.n_freqs) {
                // the transform of the monitored Ez^{n+1/2} (TEz: Ex^{n+1}) at
                // every monitor wavelength, and of the incident wave over the
                // same window
                for (int f = 0; f < h.n_freqs; ++f) {
                    const double ph_ = 2.0 * kPi * h.s1 * h.dx / h.lambdas[f] * (n + fdtd_sample_offset(h.pol));
                    pt[(size_t)n * nf + f] = make_float2((float)std::cos(ph_), (float)std::sin(ph_));
                    if (n >= h.dft_start) {
                        h.f_inc_re[f] += h.e_inc[n] * std::cos(ph_);
                        h.f_inc_im[f] += h.e_inc[n] * std::sin(ph_);
                    }
                }
                continue;
            }
            const double ph_ = h.wdt * (n + fdtd_sample_offset(h.pol));
            pt[n] = make_float2((float)std::cos(ph_), (float)std::sin(ph_));
            if (n >= h.dft_start) {
                h.inc_c += h.e_inc[n] * std::cos(ph_);
                h.inc_s += h.e_inc[n] * std::sin(ph_);
            }
        }
        HIPCHK(nullptr, hipMemcpy(inc, it.data(), sizeof(float2) * h.n_steps, hipMemcpyHostToDevice));
        HIPCHK(nullptr, hipMemcpy(pha, pt.data(), sizeof(float2) * pt.size(), hipMemcpyHostToDevice));
        devs[q] = d;
    }
    HIPCHK(nullptr, hipMalloc(&c->d_insts, sizeof(InstDev) * n_inst));
    HIPCHK(nullptr, hipMemcpy(c->d_insts, devs.data(), sizeof(InstDev) * n_inst, hipMemcpyHostToDevice));
    // projection requests: (instance, monitor block, m) for every propagating
    // order; a broadband instance's block of wavelength f and line l is 2f + l
    for (int q = 0; q < n_inst; ++q) {
        HostInst& h = c->inst[q];
        h.proj_begin = c->proj.size();
        if (h.n_freqs) {
            for (int f = 0; f < h.n_freqs; ++f)
                for (int line = 0; line < 2; ++line)
                    for (int m : h.f_orders[f]) c->proj.push_back(ProjItem{q, 2 * f + line, m, 0});
        } else {
            for (int line = 0; line < 2; ++line)
                for (int m : h.orders) c->proj.push_back(ProjItem{q, line, m, 0});
        }
        h.proj_count = c->proj.size() - h.proj_begin;
    }
    if (!c->proj.empty()) {
        HIPCHK(nullptr, hipMalloc(&c->d_proj, sizeof(ProjItem) * c->proj.size()));
        HIPCHK(nullptr, hipMemcpy(c->d_proj, c->proj.data(), sizeof(ProjItem) * c->proj.size(), hipMemcpyHostToDevice));
        HIPCHK(nullptr, hipMalloc(&c->d_proj_out, sizeof(double) * 4 * c->proj.size()));
    }
    rc = zero_state(c.get());
    if (rc != FDTD_OK) return fail(nullptr, rc, c->err);
    HIPCHK(nullptr, hipStreamSynchronize(c->stream));
    *out = c.release();
    return FDTD_OK;
}

void fdtd_destroy(fdtd_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    for (auto& kv : c->items) (void)hipFree(kv.second.d);
    for (auto& e : c->ev) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    adjoint_free(c);
    (void)hipFree(c->d_proj);
    (void)hipFree(c->d_proj_out);
    (void)hipFree(c->d_insts);
    (void)hipFree(c->slab);
    if (c->aux) {
        (void)hipStreamSynchronize(c->aux);
        (void)hipStreamDestroy(c->aux);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

int fdtd_reset(fdtd_ctx* c) {
    if (!c) return FDTD_E_INVAL;
    return zero_state(c);
}

int fdtd_steps_done(const fdtd_ctx* c, int32_t* n) {
    if (!c || !n) return FDTD_E_INVAL;
    *n = c->step;
    return FDTD_OK;
}

int fdtd_step(fdtd_ctx* c, int32_t n) {
    if (!c) return FDTD_E_INVAL;
    if (n < 0 || c->step + n > c->opts.n_steps) return fail(c, FDTD_E_INVAL, "step count past n_steps");
    int rc = ensure_config(c);
    if (rc != FDTD_OK) return rc;
    return fdtd_enqueue_steps(c, n, c->K, c->B);
}

int fdtd_step_noalloc(fdtd_ctx* c, int32_t n) {
    if (!c) return FDTD_E_INVAL;
    if (n < 0 || c->step + n > c->opts.n_steps) return fail(c, FDTD_E_INVAL, "step count past n_steps");
    const int prof = c->prof;
    if (c->opts.kernel == 1) {   // the plain sweeps use no work list
        c->K = c->B = 1;
        c->prof = 0;
        const int rc = fdtd_enqueue_steps(c, n, 1, 1);
        c->prof = prof;
        return rc;
    }
    if (c->K <= 0 || c->B <= 0) {
        if (c->opts.t_block > 0 && c->opts.band_rows > 0) {
            c->K = c->opts.t_block;
            c->B = c->opts.band_rows;
        } else {
            return fail(c, FDTD_E_STATE,
                        "no launch shape: set opts.t_block and opts.band_rows, or tune or step the context first");
        }
    }
    // every list this call launches must fit the array
    int rc = FDTD_OK;
    std::vector<std::tuple<int, int, int, int>> keys;
    plan_launches(c, c->step, n, c->K, [&](int, int k, int m) {
        const auto key = std::make_tuple(k, c->B, c->SB, m);
        auto it = c->host_items.find(key);
        if (it == c->host_items.end()) {
            auto& e = c->host_items[key];
            build_items(c, k, c->B, m, e.first, e.second);
            it = c->host_items.find(key);
        }
        if (it->second.first.size() > (size_t)kNoallocItems && rc == FDTD_OK)
            rc = fail(c, FDTD_E_INVAL, "a launch needs " + std::to_string(it->second.first.size()) +
                                           " work items, above the " + std::to_string(kNoallocItems) +
                                           " of the fixed array (use fdtd_step)");
        keys.push_back(key);
    });
    if (rc != FDTD_OK || keys.empty()) return rc;
    WorkItem* dev_items = scratch_on(c, c->device);
    if (!dev_items) return FDTD_E_HIP;
    // stage a list when it differs from the previous launch's in this call
    // (stream order keeps each copy behind the launches that read the array
    // before it; the special items' stream is joined at every launch)
    const std::tuple<int, int, int, int>* staged = nullptr;
    for (const auto& key : keys) {
        auto& e = c->host_items[key];
        if (!staged || *staged != key) {
            if (!e.first.empty())
                HIPCHK(c, hipMemcpyAsync(dev_items, e.first.data(), sizeof(WorkItem) * e.first.size(),
                                         hipMemcpyHostToDevice, c->stream));
            staged = &key;
        }
        ItemList L = e.second;
        L.d = dev_items;
        rc = launch_items(c, std::get<0>(key), std::get<3>(key), &L, false);
        if (rc != FDTD_OK) return rc;
    }
    return FDTD_OK;
}

int fdtd_run(fdtd_ctx* c, int32_t record) {
    if (!c) return FDTD_E_INVAL;
    int rc = ensure_config(c);
    if (rc != FDTD_OK) return rc;
    if (record) return adjoint_record_run(c);
    const int remaining = c->opts.n_steps - c->step;
    if (remaining <= 0) return FDTD_OK;
    // a full run from step 0 replays a captured graph of all launches
    if (c->opts.use_graph && c->graph_faster && c->step == 0 && c->cur == 0 && !c->prof && c->opts.kernel == 0) {
        if (!c->graph || c->graph_K != c->K || c->graph_B != c->B || c->graph_SB != c->SB || c->graph_W != c->W) {
            if (c->graph) {
                (void)hipGraphExecDestroy(c->graph);
                c->graph = nullptr;
            }
            // build every work-item list before capture (capture cannot allocate)
            bool ok = true;
            plan_launches(c, 0, remaining, c->K, [&](int, int k, int m) { ok = ok && item_list(c, k, c->B, m); });
            if (!ok) return fail(c, FDTD_E_NOMEM, "work-item list allocation failed");
            hipGraph_t g = nullptr;
            HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            rc = fdtd_enqueue_steps(c, remaining, c->K, c->B);
            hipError_t e = hipStreamEndCapture(c->stream, &g);
            c->step = 0;
            c->cur = 0;
            if (rc != FDTD_OK) return rc;
            if (e != hipSuccess) return fail(c, FDTD_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return fail(c, FDTD_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
            c->graph_K = c->K;
            c->graph_W = c->W;
            c->graph_B = c->B;
            c->graph_SB = c->SB;
        }
        HIPCHK(c, hipGraphLaunch(c->graph, c->stream));
        // replay the bookkeeping of the captured sequence
        plan_launches(c, 0, remaining, c->K, [&](int s, int k, int) {
            c->cur ^= 1;
            c->step = s + k;
            mark_ends(c);
        });
        return FDTD_OK;
    }
    return fdtd_enqueue_steps(c, remaining, c->K, c->B);
}

int fdtd_spectra(fdtd_ctx* c, double* R, double* T, double* A) {
    if (!c) return FDTD_E_INVAL;
    std::vector<std::vector<double>> fre, fim;
    std::vector<double> finc2;
    int rc = fdtd_order_amplitudes(c, fre, fim, finc2);
    if (rc != FDTD_OK) return rc;
    for (size_t q = 0; q < c->inst.size(); ++q) {
        const HostInst& h = c->inst[q];
        if (h.n_freqs) {   // see fdtd_broadband_spectra
            const double nan = std::nan("");
            if (R) R[q] = nan;
            if (T) T[q] = nan;
            if (A) A[q] = nan;
            continue;
        }
        const size_t no = h.orders.size();
        double Rq = 0.0, Tq = 0.0;
        for (size_t o = 0; o < no; ++o) {
            Rq += h.weights[o] * (fre[q][o] * fre[q][o] + fim[q][o] * fim[q][o]) / finc2[q];
            Tq += h.weights[o] * (fre[q][no + o] * fre[q][no + o] + fim[q][no + o] * fim[q][no + o]) / finc2[q];
        }
        if (R) R[q] = Rq;
        if (T) T[q] = Tq;
        if (A) A[q] = 1.0 - Rq - Tq;
    }
    return FDTD_OK;
}

int fdtd_broadband_spectra(fdtd_ctx* c, int32_t inst, double* R, double* T, double* A) {
    if (!c || inst < 0 || inst >= (int)c->inst.size()) return FDTD_E_INVAL;
    const HostInst& h = c->inst[inst];
    if (!h.n_freqs) return fail(c, FDTD_E_INVAL, "fdtd_broadband_spectra covers broadband instances");
    if (c->step != c->opts.n_steps) return fail(c, FDTD_E_STATE, "the run has not reached n_steps");
    const size_t np = h.proj_count;
    std::vector<double> po(4 * np);
    int status = 0;
    if (np) {
        HIPCHK(c, launch_project(c->d_insts, c->d_proj + h.proj_begin, (int)np, c->d_proj_out + 4 * h.proj_begin,
                                 c->stream));
        HIPCHK(c, hipMemcpyAsync(po.data(), c->d_proj_out + 4 * h.proj_begin, sizeof(double) * 4 * np,
                                 hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(&status, h.dev.status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (status) return fail(c, FDTD_E_UNSTABLE, "instance " + std::to_string(inst) + ": non-finite monitor sum");
    // the monitor sums are the transform F_i = S_cos,i + i S_sin,i itself (no
    // tone fit); the projection gives, per order, the cosine-sum and sine-sum
    // projections (c_re, c_im, s_re, s_im), so F_m = (c_re - s_im + i (c_im + s_re))/nx
    size_t p = 0;
    for (int f = 0; f < h.n_freqs; ++f) {
        const double finc2 = h.f_inc_re[f] * h.f_inc_re[f] + h.f_inc_im[f] * h.f_inc_im[f];
        const size_t no = h.f_orders[f].size();
        double pw[2] = {0.0, 0.0};
        for (int line = 0; line < 2; ++line)
            for (size_t o = 0; o < no; ++o, ++p) {
                const double* v = &po[4 * p];
                const double re = (v[0] - v[3]) / h.nx, im = (v[1] + v[2]) / h.nx;
                pw[line] += h.f_weights[f][o] * (re * re + im * im) / finc2;
            }
        if (R) R[f] = pw[0];
        if (T) T[f] = pw[1];
        if (A) A[f] = 1.0 - pw[0] - pw[1];
    }
    return FDTD_OK;
}

int fdtd_combine_spectra(const double* R, const double* T, int32_t n_runs, const int32_t* group, int32_t n_groups,
                         double* R_out, double* T_out, double* A_out) {
    g_create_error.clear();
    if (!R || !T || !group || n_runs < 1 || n_groups < 1)
        return fail(nullptr, FDTD_E_INVAL, "null input, n_runs < 1 or n_groups < 1");
    std::vector<double> sr(n_groups, 0.0), st(n_groups, 0.0);
    std::vector<int64_t> cnt(n_groups, 0);
    for (int32_t i = 0; i < n_runs; ++i) {
        const int32_t g = group[i];
        if (g < 0 || g >= n_groups) return fail(nullptr, FDTD_E_INVAL, "run " + std::to_string(i) + ": group out of range");
        if (!std::isfinite(R[i]) || !std::isfinite(T[i]))
            return fail(nullptr, FDTD_E_INVAL, "run " + std::to_string(i) + ": non-finite R or T");
        sr[g] += R[i];
        st[g] += T[i];
        ++cnt[g];
    }
    for (int32_t g = 0; g < n_groups; ++g)
        if (!cnt[g]) return fail(nullptr, FDTD_E_INVAL, "group " + std::to_string(g) + " has no runs");
    for (int32_t g = 0; g < n_groups; ++g) {
        const double r = sr[g] / (double)cnt[g], t = st[g] / (double)cnt[g];
        if (R_out) R_out[g] = r;
        if (T_out) T_out[g] = t;
        if (A_out) A_out[g] = 1.0 - r - t;
    }
    return FDTD_OK;
}

int fdtd_orders(fdtd_ctx* c, int32_t inst, int32_t max_orders, int32_t* m, double* w, double* ref_pow,
                double* trn_pow, int32_t* n_orders) {
    if (!c || inst < 0 || inst >= (int)c->inst.size() || max_orders < 0) return FDTD_E_INVAL;
    if (c->inst[inst].n_freqs) return fail(c, FDTD_E_INVAL, "fdtd_orders covers monochromatic instances");
    std::vector<std::vector<double>> fre, fim;
    std::vector<double> finc2;
    int rc = fdtd_order_amplitudes(c, fre, fim, finc2);
    if (rc != FDTD_OK) return rc;
    const HostInst& h = c->inst[inst];
    const int no = (int)h.orders.size();
    if (n_orders) *n_orders = no;
    for (int o = 0; o < std::min(no, max_orders); ++o) {
        if (m) m[o] = h.orders[o];
        if (w) w[o] = h.weights[o];
        if (ref_pow) ref_pow[o] = (fre[inst][o] * fre[inst][o] + fim[inst][o] * fim[inst][o]) / finc2[inst];
        if (trn_pow)
            trn_pow[o] = (fre[inst][no + o] * fre[inst][no + o] + fim[inst][no + o] * fim[inst][no + o]) / finc2[inst];
    }
    return FDTD_OK;
}

int fdtd_fields(fdtd_ctx* c, int32_t inst, float* ez, float* hx, float* hy) {
    if (!c || inst < 0 || inst >= (int)c->inst.size()) return FDTD_E_INVAL;
    HostInst& h = c->inst[inst];
    float* dst[3] = {ez, hx, hy};
    const int cur = fdtd_inst_cur(c, inst);
    float* src[3] = {h.dev.ez[cur], h.dev.hx[cur], h.dev.hy[cur]};
    for (int f = 0; f < 3; ++f)
        if (dst[f])
            HIPCHK(c, hipMemcpy2DAsync(dst[f], sizeof(float) * h.nx, src[f], sizeof(float) * h.pitch, sizeof(float) * h.nx,
                                       h.ny, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return FDTD_OK;
}

int fdtd_monitors(fdtd_ctx* c, int32_t inst, double* mon) {
    if (!c || !mon || inst < 0 || inst >= (int)c->inst.size()) return FDTD_E_INVAL;
    HostInst& h = c->inst[inst];
    const int nf = std::max(1, h.n_freqs);
    std::vector<float> m((size_t)8 * h.pitch * nf);
    HIPCHK(c, hipMemcpyAsync(m.data(), h.dev.mon, sizeof(float) * m.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int f = 0; f < nf; ++f)
        for (int line = 0; line < 2; ++line)
            for (int cs = 0; cs < 2; ++cs)
                for (int i = 0; i < h.nx; ++i) {
                    const float* b = &m[(size_t)(2 * f + line) * 4 * h.pitch];
                    mon[((size_t)4 * f + 2 * line + cs) * h.nx + i] =
                        (double)b[(size_t)(2 * cs) * h.pitch + i] - (double)b[(size_t)(2 * cs + 1) * h.pitch + i];
                }
    return FDTD_OK;
}

int fdtd_set_fields(fdtd_ctx* c, int32_t inst, const float* ez, const float* hx, const float* hy, const float* psi_ez,
                    const float* psi_hx) {
    if (!c || inst < 0 || inst >= (int)c->inst.size()) return FDTD_E_INVAL;
    HostInst& h = c->inst[inst];
    const float* srcs[3] = {ez, hx, hy};
    const int cur = fdtd_inst_cur(c, inst);
    float* dsts[3] = {h.dev.ez[cur], h.dev.hx[cur], h.dev.hy[cur]};
    std::vector<float> tmp;
    for (int f = 0; f < 3; ++f) {
        if (!srcs[f]) continue;
        tmp.assign(srcs[f], srcs[f] + h.cells());
        if (f == 1)
            for (int i = 0; i < h.nx; ++i) tmp[i] = 0.f;
        HIPCHK(c, hipMemcpy2DAsync(dsts[f], sizeof(float) * h.pitch, tmp.data(), sizeof(float) * h.nx, sizeof(float) * h.nx,
                                   h.ny, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    const float* ps[2] = {psi_ez, psi_hx};
    float* pd[2] = {h.dev.pe[cur], h.dev.ph[cur]};
    for (int f = 0; f < 2; ++f) {
        if (!ps[f]) continue;
        std::vector<float> rows((size_t)2 * h.n_pml * h.pitch, 0.f);
        for (int j = 0; j < h.ny; ++j) {
            const bool layer = f == 0 ? (j < h.n_pml || j >= h.ny - h.n_pml)
                                      : ((j >= 1 && j < h.n_pml) || j > h.ny - h.n_pml);
            if (!layer) continue;
            const int r = j < h.n_pml ? j : j - h.ny + 2 * h.n_pml;
            memcpy(&rows[(size_t)r * h.pitch], ps[f] + (size_t)j * h.nx, sizeof(float) * h.nx);
        }
        HIPCHK(c, hipMemcpyAsync(pd[f], rows.data(), sizeof(float) * rows.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return FDTD_OK;
}

int fdtd_get_config(const fdtd_ctx* c, int32_t* kernel, int32_t* t_block, int32_t* band_rows, int32_t* items,
                    int64_t* device_bytes, int64_t* lean_cells, int32_t* special_rows, int32_t* bulk_columns) {
    if (!c) return FDTD_E_INVAL;
    if (special_rows) *special_rows = c->SB;
    if (bulk_columns) *bulk_columns = c->W;
    const auto key = std::make_tuple(c->K, c->B, c->SB, active_end(c, 0));
    if (lean_cells) {
        auto it = c->items.find(key);
        *lean_cells = it == c->items.end() ? 0 : it->second.lean_cells;
        if (c->opts.kernel == 1) {
            *lean_cells = 0;
            for (auto& h : c->inst) *lean_cells += (int64_t)h.cells();
        }
    }
    if (kernel) *kernel = c->opts.kernel;
    if (t_block) *t_block = c->K;
    if (band_rows) *band_rows = c->B;
    if (items) {
        auto it = c->items.find(key);
        *items = it == c->items.end() ? 0 : it->second.n();
    }
    if (device_bytes) *device_bytes = (int64_t)c->slab_bytes + adjoint_bytes(c);
    return FDTD_OK;
}

int fdtd_autotune(fdtd_ctx* c, int32_t trial_steps, double* best_rate) {
    if (!c) return FDTD_E_INVAL;
    if (c->opts.kernel == 1) {   // the plain sweeps have no launch shape to tune
        c->K = c->B = 1;
        c->tuned = true;
        if (best_rate) *best_rate = 0;
        return FDTD_OK;
    }
    if (c->step != 0) {
        int rc = zero_state(c);
        if (rc != FDTD_OK) return rc;
    }
    size_t cells = 0;
    for (auto& h : c->inst) cells += h.cells();
    const std::string key = tune_key(c);
    const int fixK = c->opts.t_block, fixB = c->opts.band_rows, fixSB = c->opts.special_rows;
    const int fixW = c->opts.bulk_columns;
    if (trial_steps <= 0) {
        TunedShape shape;
        if (tune_lookup(key, shape)) {
            c->K = fixK > 0 ? fixK : shape.K;
            c->B = fixB > 0 ? fixB : shape.B;
            c->SB = fixSB > 0 ? fixSB : shape.SB;
            c->W = fixW > 0 ? fixW : shape.W;
            c->graph_faster = shape.graph_faster;
            if (best_rate) *best_rate = 0;
            return FDTD_OK;
        }
        // about 4e9 cell-updates per candidate (at most 240 steps), at least
        // two launches of the largest K
        trial_steps = (int)std::min<double>(240.0, std::max(2.0 * kMaxTBlock, 4e9 / (double)std::max<size_t>(cells, 1)));
    }
    trial_steps = std::min(trial_steps, c->opts.n_steps);
    std::vector<int> Ks, Bs;
    // broadband TEz carries 16 pole values per row and level, which leaves
    // its streaming kernel short of registers above a few steps per launch
    if (fixK > 0) Ks = {fixK}; else if (c->has_bt) Ks = {3, 4, 5, 6}; else Ks = {4, 6, 8, 10, 12};
    if (fixB > 0) Bs = {fixB}; else Bs = {16, 32, 64, 96, 128, 192, 256, 512};
    // bulk items of one wave or of one workgroup: the workgroup's waves
    // exchange their edge columns instead of recomputing them, which saves
    // arithmetic on large grids but needs grids wide enough to fill the device
    std::vector<int> Ws;
    if (fixW > 0) Ws = {fixW}; else if (c->has_mono) Ws = {64, kWgColumns}; else Ws = {64};
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreateWithFlags(&e0, kTimingEvent));
    HIPCHK(c, hipEventCreateWithFlags(&e1, kTimingEvent));
    const int prof = c->prof;
    c->prof = 0;
    // time of `steps` steps of configuration (K, B) from a zeroed state, best
    // of `reps` trials (the first launch of a configuration builds its list)
    auto trial = [&](int K, int B, int steps, int reps, double& best_ms) -> int {
        best_ms = 1e30;
        for (int rep = 0; rep < reps; ++rep) {
            int rc = zero_state(c);
            if (rc != FDTD_OK) return rc;
            rc = fdtd_enqueue_steps(c, std::min(K, steps), K, B);
            if (rc != FDTD_OK) return rc;
            // whole launches only, so that no K is charged a short tail launch
            int n = std::min(steps, c->opts.n_steps - c->step);
            if (n >= K) n -= n % K;
            if (n <= 0) return FDTD_OK;
            HIPCHK(c, hipEventRecord(e0, c->stream));
            rc = fdtd_enqueue_steps(c, n, K, B);
            if (rc != FDTD_OK) return rc;
            HIPCHK(c, hipEventRecord(e1, c->stream));
            HIPCHK(c, hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
            best_ms = std::min(best_ms, (double)ms / n);
        }
        return FDTD_OK;
    };
    // stage 1: every (K, B), best of two short trials, with 16-row special
    // bands (or the fixed height); stage 2: the three fastest again with three
    // times the steps, each with special bands of 4, 8, 12 and 16 rows.  Thinner
    // special bands put more, shorter waves on the rows next to the layers,
    // the source line and the monitors, which pays where those waves set the
    // launch period (small grids), and costs halo work where they run hidden
    // behind the bulk kernel.
    std::vector<int> SBs;
    if (fixSB > 0) SBs = {fixSB}; else SBs = {4, 8, 12, kSpecialBand};
    c->SB = fixSB > 0 ? fixSB : kSpecialBand;
    std::vector<std::pair<double, TunedShape>> ranked;
    for (int W : Ws)
        for (int K : Ks)
            for (int B : Bs) {
                c->W = W;
                double ms;
                int rc = trial(K, B, trial_steps, 2, ms);
                if (rc != FDTD_OK) return rc;
                TunedShape t{K, B, c->SB};
                t.W = W;
                ranked.push_back({ms, t});
            }
    auto faster = [](const std::pair<double, TunedShape>& a, const std::pair<double, TunedShape>& b) {
        return a.first < b.first;
    };
    std::stable_sort(ranked.begin(), ranked.end(), faster);
    if (ranked.size() > 1 || SBs.size() > 1) {
        const size_t top = std::min<size_t>(3, ranked.size());
        std::vector<std::pair<double, TunedShape>> second;
        for (size_t k = 0; k < top; ++k)
            for (int sb : SBs) {
                c->SB = sb;
                c->W = ranked[k].second.W;
                double ms;
                int rc = trial(ranked[k].second.K, ranked[k].second.B, 3 * trial_steps, 2, ms);
                if (rc != FDTD_OK) return rc;
                TunedShape t = ranked[k].second;
                t.SB = sb;
                second.push_back({ms, t});
            }
        std::stable_sort(second.begin(), second.end(), faster);
        ranked = second;
    }
    // Graph replay of the chosen shape against direct launches: replay
    // removes launch gaps, which pays on small grids, but its kernel nodes
    // end with a cache flush that costs the bulk kernel its L2 hits on large
    // ones (most in TEz).  fdtd_run replays a graph only if it measured faster.
    c->graph_faster = true;
    if (c->opts.use_graph) {
        const TunedShape cand = ranked[0].second;
        c->SB = cand.SB;
        c->W = cand.W;
        double g_ms = 1e30;
        int rc = zero_state(c);
        if (rc != FDTD_OK) return rc;
        rc = fdtd_enqueue_steps(c, std::min(cand.K, 3 * trial_steps), cand.K, cand.B);
        if (rc != FDTD_OK) return rc;
        int n = std::min(3 * trial_steps, c->opts.n_steps - c->step);
        if (n >= cand.K) n -= n % cand.K;
        if (n > 0) {
            // every list the captured launches use exists before the capture
            bool ok = true;
            plan_launches(c, c->step, n, cand.K, [&](int, int k, int m) { ok = ok && item_list(c, k, cand.B, m); });
            if (!ok) return fail(c, FDTD_E_NOMEM, "work-item list allocation failed");
            hipGraph_t g = nullptr;
            HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            rc = fdtd_enqueue_steps(c, n, cand.K, cand.B);
            const hipError_t e = hipStreamEndCapture(c->stream, &g);
            if (rc != FDTD_OK) return rc;
            if (e != hipSuccess) return fail(c, FDTD_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
            hipGraphExec_t ge = nullptr;
            const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ei != hipSuccess) return fail(c, FDTD_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
            // timing only: each replay repeats the captured steps on whatever
            // state the previous one left (the scheme keeps it bounded); the
            // context is zeroed below
            for (int rep = 0; rep < 3; ++rep) {
                HIPCHK(c, hipEventRecord(e0, c->stream));
                HIPCHK(c, hipGraphLaunch(ge, c->stream));
                HIPCHK(c, hipEventRecord(e1, c->stream));
                HIPCHK(c, hipEventSynchronize(e1));
                float ms = 0;
                HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
                if (rep > 0) g_ms = std::min(g_ms, (double)ms / n);
            }
            (void)hipGraphExecDestroy(ge);
        }
        c->graph_faster = g_ms < ranked[0].first;
    }
    c->prof = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const TunedShape bs = ranked[0].second;
    const double best = (double)cells / (ranked[0].first * 1e-3);
    c->K = bs.K;
    c->B = bs.B;
    c->SB = bs.SB;
    c->W = bs.W;
    c->tuned = true;
    TunedShape stored = bs;
    stored.graph_faster = c->graph_faster;
    tune_store(key, stored);
    if (best_rate) *best_rate = best;
    return zero_state(c);
}

int fdtd_set_profiling(fdtd_ctx* c, int32_t enable) {
    if (!c) return FDTD_E_INVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto& e : c->ev) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    c->ev.clear();
    c->ev_cells.clear();
    c->prof = enable > 0 ? enable : 0;
    c->prof_seen = 0;
    return FDTD_OK;
}

int fdtd_kernel_time(fdtd_ctx* c, double* total_ms, int64_t* launches) {
    if (!c) return FDTD_E_INVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double t = 0;
    for (auto& e : c->ev) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, e.first, e.second));
        t += ms;
    }
    if (total_ms) *total_ms = t;
    if (launches) *launches = (int64_t)c->ev.size();
    return FDTD_OK;
}

}  // extern "C"

// Gram matrix of the least-squares tone fit over samples t = (n + off) dt,
// n in [n0, n1): {sum cos^2, sum cos sin, sum sin^2}.
void fdtd_gram(double wdt, int n0, int n1, double g[3], double off) {
    g[0] = g[1] = g[2] = 0.0;
    for (int n = n0; n < n1; ++n) {
        const double ph = wdt * (n + off);
        const double cs = std::cos(ph), sn = std::sin(ph);
        g[0] += cs * cs;
        g[1] += cs * sn;
        g[2] += sn * sn;
    }
}

// Tone-fit Bloch amplitudes (eqs. 29-32): the projection kernel gives, per
// (instance, line, m), sum_i S_i exp(-2 pi i m i/nx) for the cosine and sine
// sums S; the least-squares fit (a, b) = G^-1 (S_c, S_s) is linear, so it is
// applied after projecting, and F_m = (a_m + i b_m)/nx.
int fdtd_order_amplitudes(fdtd_ctx* c, std::vector<std::vector<double>>& f_re, std::vector<std::vector<double>>& f_im,
                          std::vector<double>& finc2) {
    if (c->step != c->opts.n_steps) return fdtd_fail(c, FDTD_E_STATE, "the run has not reached n_steps");
    const size_t np = c->proj.size();
    if (np) FDTD_HIPCHK(c, launch_project(c->d_insts, c->d_proj, (int)np, c->d_proj_out, c->stream));
    std::vector<double> po(4 * np);
    std::vector<int> status(c->inst.size());
    if (np)
        FDTD_HIPCHK(c, hipMemcpyAsync(po.data(), c->d_proj_out, sizeof(double) * 4 * np, hipMemcpyDeviceToHost, c->stream));
    for (size_t q = 0; q < c->inst.size(); ++q)
        FDTD_HIPCHK(c, hipMemcpyAsync(&status[q], c->inst[q].dev.status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    FDTD_HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t q = 0; q < c->inst.size(); ++q)
        if (status[q]) return fdtd_fail(c, FDTD_E_UNSTABLE, "instance " + std::to_string(q) + ": non-finite monitor sum");
    f_re.assign(c->inst.size(), {});
    f_im.assign(c->inst.size(), {});
    finc2.assign(c->inst.size(), 0.0);
    for (size_t q = 0; q < c->inst.size(); ++q) {
        const HostInst& h = c->inst[q];
        if (h.n_freqs) continue;
        size_t p = h.proj_begin;
        double g[3];
        fdtd_gram(h.wdt, h.dft_start, h.n_steps, g, fdtd_sample_offset(h.pol));
        const double det = g[0] * g[2] - g[1] * g[1];
        const double i11 = g[2] / det, i12 = -g[1] / det, i22 = g[0] / det;
        const double fa = i11 * h.inc_c + i12 * h.inc_s, fb = i12 * h.inc_c + i22 * h.inc_s;
        finc2[q] = fa * fa + fb * fb;
        const size_t no = h.orders.size();
        f_re[q].assign(2 * no, 0.0);
        f_im[q].assign(2 * no, 0.0);
        for (int line = 0; line < 2; ++line)
            for (size_t o = 0; o < no; ++o, ++p) {
                const double* v = &po[4 * p];
                const double ar = i11 * v[0] + i12 * v[2], ai = i11 * v[1] + i12 * v[3];
                const double br = i12 * v[0] + i22 * v[2], bi = i12 * v[1] + i22 * v[3];
                f_re[q][line * no + o] = (ar - bi) / h.nx;
                f_im[q][line * no + o] = (ai + br) / h.nx;
            }
    }
    return FDTD_OK;
}
