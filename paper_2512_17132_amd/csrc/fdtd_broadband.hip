// gfx950 kernels of broadband runs (Sec. 2.2's Lorentz-Drude alternative to
// one monochromatic run per wavelength): the TMz E sweep with per-label
// polarisation currents and monitors at many wavelengths.  The H sweep is the
// monochromatic one.
#include "fdtd_device.h"
#include "fdtd_kernels.h"

namespace fdtd {

// One step's E sweep of a broadband instance, in place on field set 0, one
// thread per cell.  Each pole's polarisation (normalised P/eps0) advances
// first, from the Ez it is about to replace:
//   P^{n+1/2} = alpha P^{n-1/2} + xi P^{n-3/2} + zeta Ez^{n-1/2},
// and the E update loses Cp times the sum of the increments P^{n+1/2} - P^{n-1/2}
// (Ampere's law with eps_inf in Ce, Cb and the poles' dP/dt as a current).
// The monitor rows add Ez^{n+1/2} (cos, sin)(omega_f (n+1/2) dt) to the Kahan
// sums of every monitor wavelength f.
__global__ __launch_bounds__(256) void k_plain_e_ade(InstDev d, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const size_t o = (size_t)j * d.pitch + i;
    const size_t plane = (size_t)d.ny * d.pitch;
    const int ir = (i + 1 == d.nx) ? 0 : i + 1;
    const float hx_c = d.hx[0][o];
    const float hx_u = (j + 1 < d.ny) ? d.hx[0][o + d.pitch] : 0.0f;
    const float hy_c = d.hy[0][o];
    const float hy_r = d.hy[0][(size_t)j * d.pitch + ir];
    const int L = d.lab[o];
    const float2 cf = d.coef[L];
    const float e_old = d.ez[0][o];
    float dpol = 0.0f, cp = 0.0f;
    for (int q = 0; q < d.n_poles; ++q) {
        const float4 pq = d.poles[q * kMaxLabels + L];
        float* pc = d.pstate + (size_t)(2 * q) * plane;
        float* pp = pc + plane;
        const float p_c = pc[o], p_p = pp[o];
        const float p_n = __fmaf_rn(pq.x, p_c, __fmaf_rn(pq.y, p_p, pq.z * e_old));
        dpol += p_n - p_c;
        pp[o] = p_c;
        pc[o] = p_n;
        cp = pq.w;
    }
    const bool pml = is_pml_e(j, d.ny, d.n_pml);
    float pe = 0.0f;
    float4 pr = make_float4(0.f, 0.f, 1.f, 0.f);
    size_t po = 0;
    if (pml) {
        po = (size_t)psi_row(j, d.ny, d.n_pml) * d.pitch + i;
        pe = d.pe[0][po];
        pr = d.prof_e[j];
    }
    const float e = upd_e(e_old, cf.x, cf.y, hy_c, hy_r, hx_c, hx_u, pml, pr, pe, j == d.j_src, d.inc[n].y) - cp * dpol;
    d.ez[0][o] = e;
    if (pml) d.pe[0][po] = pe;
    if (n >= d.dft_start && (j == d.j_ref || j == d.j_trn)) {
        const int line = (j == d.j_ref) ? 0 : 1;
        const float2* ph = d.phasor + (size_t)n * d.n_freqs;
        bool finite = true;
        for (int f = 0; f < d.n_freqs; ++f) {
            float* m = d.mon + (size_t)(2 * f + line) * 4 * d.pitch;
            const float2 w = ph[f];
            float s0 = m[i], c0 = m[d.pitch + i], s1 = m[2 * d.pitch + i], c1 = m[3 * d.pitch + i];
            kahan_add(s0, c0, e * w.x);
            kahan_add(s1, c1, e * w.y);
            m[i] = s0;
            m[d.pitch + i] = c0;
            m[2 * d.pitch + i] = s1;
            m[3 * d.pitch + i] = c1;
            finite = finite && __builtin_isfinite(s0) && __builtin_isfinite(s1);
        }
        if (!finite) *d.status = 1;
    }
}

hipError_t launch_plain_step_broadband(const InstDev& d, int n, hipStream_t s) {
    dim3 grid((d.nx + 255) / 256, d.ny);
    k_plain_e_ade<<<grid, 256, 0, s>>>(d, n);
    return launch_plain_h(d, n, 0, s);
}

}  // namespace fdtd
