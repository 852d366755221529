// Discrete adjoint of the TMz FDTD run: the exact transpose of the forward
// recurrence, stepped backwards in time over checkpointed segments.
//
// Lossy FDTD is not time-reversible, so the forward states the gradient needs
// (Ez before and after every step) are recomputed segment by segment from
// checkpoints stored during a recorded forward run.  The loss is
// L = sum_i dL_dR[i] R_i + dL_dT[i] T_i; its sensitivity to the monitor sums
// is injected on the monitor rows at every step of the window, and the
// per-pixel sensitivities to the update coefficients (Ce, Cb) are reduced per
// label and chained to (n, k) on the host, or mapped to eps_r per pixel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fdtd.h"
#include "fdtd_adjoint.h"
#include "fdtd_device.h"
#include "fdtd_host.h"
#include "fdtd_kernels.h"

using namespace fdtd;

namespace {

constexpr double kPi = 3.14159265358979323846;

struct AdjDev {
    float* lez;
    float* lhx;
    float* lhy;
    float* lpe;
    float* lph;
    float* t0;   // delta per Hx edge
    float* t1;   // mu per Ez cell
    float* t2;   // nu per Ez cell
    float* gce;
    float* gcb;
    const float* src;     // [2][2][pitch]
    const float* e_old;   // Ez^{n-1/2}
    const float* e_new;   // Ez^{n+1/2}
};

// --- plain transposed sweeps (one thread per cell, three launches per step) ---

__global__ __launch_bounds__(256) void k_adj_delta(InstDev d, AdjDev a) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const size_t o = (size_t)j * d.pitch + i;
    float delta = 0.f;
    if (j > 0) {
        const bool pml = is_pml_h(j, d.ny, d.n_pml);
        float lph = 0.f;
        float4 pr = make_float4(0.f, 0.f, 1.f, 0.f);
        size_t po = 0;
        if (pml) {
            po = (size_t)psi_row(j, d.ny, d.n_pml) * d.pitch + i;
            lph = a.lph[po];
            pr = d.prof_h[j];
        }
        delta = adj_delta(a.lhx[o], lph, pml, pr, d.s1);
        if (pml) a.lph[po] = lph;
    }
    a.t0[o] = delta;
}

__global__ __launch_bounds__(256) void k_adj_e(InstDev d, AdjDev a, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const size_t o = (size_t)j * d.pitch + i;
    const int ir = (i + 1 == d.nx) ? 0 : i + 1;
    float le = a.lez[o];
    if (n >= d.dft_start) {
        const float2 ph = d.phasor[n];
        if (j == d.j_ref) le = le + __fmaf_rn(a.src[i], ph.x, a.src[d.pitch + i] * ph.y);
        if (j == d.j_trn) le = le + __fmaf_rn(a.src[2 * d.pitch + i], ph.x, a.src[3 * d.pitch + i] * ph.y);
    }
    const float dj = a.t0[o];
    const float dj1 = (j + 1 < d.ny) ? a.t0[o + d.pitch] : 0.f;
    const float dly = a.lhy[(size_t)j * d.pitch + ir] - a.lhy[o];
    const float av = (le + (dj - dj1)) - d.s1 * dly;
    const float2 cf = d.coef[d.lab[o]];
    const float eo = a.e_old[o], en = a.e_new[o];
    a.gce[o] = __fmaf_rn(av, eo, a.gce[o]);
    a.gcb[o] = __fmaf_rn(av, (en - cf.x * eo) / cf.y, a.gcb[o]);
    const float mu = cf.y * av;
    const bool pml = is_pml_e(j, d.ny, d.n_pml);
    float lpe = 0.f;
    float4 pr = make_float4(0.f, 0.f, 1.f, 0.f);
    size_t po = 0;
    if (pml) {
        po = (size_t)psi_row(j, d.ny, d.n_pml) * d.pitch + i;
        lpe = a.lpe[po];
        pr = d.prof_e[j];
    }
    const float nu = adj_nu(mu, lpe, pml, pr);
    if (pml) a.lpe[po] = lpe;
    a.lez[o] = cf.x * av;
    a.t1[o] = mu;
    a.t2[o] = nu;
}

__global__ __launch_bounds__(256) void k_adj_h(InstDev d, AdjDev a) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const size_t o = (size_t)j * d.pitch + i;
    const int il = (i == 0) ? d.nx - 1 : i - 1;
    if (j > 0) a.lhx[o] = a.lhx[o] + (a.t2[o] - a.t2[o - d.pitch]);
    a.lhy[o] = a.lhy[o] - (a.t1[o] - a.t1[(size_t)j * d.pitch + il]);
}

// Per-label sums of gCe and gCb in FP64 (block reduction in LDS, then atomics).
__global__ __launch_bounds__(256) void k_label_sums(InstDev d, const float* __restrict__ gce,
                                                    const float* __restrict__ gcb, double* __restrict__ out) {
    __shared__ double acc[kMaxLabels][2];
    for (int k = threadIdx.x; k < d.n_labels; k += 256) acc[k][0] = acc[k][1] = 0.0;
    __syncthreads();
    const int j = blockIdx.y;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < d.nx; i += gridDim.x * 256) {
        const size_t o = (size_t)j * d.pitch + i;
        const int L = d.lab[o];
        atomicAdd(&acc[L][0], (double)gce[o]);
        atomicAdd(&acc[L][1], (double)gcb[o]);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < d.n_labels; k += 256) {
        if (acc[k][0] != 0.0) atomicAdd(&out[2 * k], acc[k][0]);
        if (acc[k][1] != 0.0) atomicAdd(&out[2 * k + 1], acc[k][1]);
    }
}

// dL/d eps_r per pixel at fixed sigma: gCe dCe/deps + gCb dCb/deps, with the
// per-label derivatives in `deriv` ([n_labels][2]); output row-major, no pitch.
__global__ __launch_bounds__(256) void k_eps_grad(InstDev d, const float* __restrict__ gce,
                                                  const float* __restrict__ gcb, const float2* __restrict__ deriv,
                                                  float* __restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const size_t o = (size_t)j * d.pitch + i;
    const float2 dv = deriv[d.lab[o]];
    out[(size_t)j * d.nx + i] = __fmaf_rn(gce[o], dv.x, gcb[o] * dv.y);
}

int copy_state(fdtd_ctx* c, int q, int from_cur, float* dst, bool to_store) {
    HostInst& h = c->inst[q];
    const size_t f = (size_t)h.ny * h.pitch, p = (size_t)2 * h.n_pml * h.pitch;
    float* parts[5] = {h.dev.ez[from_cur], h.dev.hx[from_cur], h.dev.hy[from_cur], h.dev.pe[from_cur], h.dev.ph[from_cur]};
    const size_t sizes[5] = {f, f, f, p, p};
    size_t off = 0;
    for (int k = 0; k < 5; ++k) {
        if (to_store)
            FDTD_HIPCHK(c, hipMemcpyAsync(dst + off, parts[k], sizes[k] * 4, hipMemcpyDeviceToDevice, c->stream));
        else
            FDTD_HIPCHK(c, hipMemcpyAsync(parts[k], dst + off, sizes[k] * 4, hipMemcpyDeviceToDevice, c->stream));
        off += sizes[k];
    }
    return FDTD_OK;
}

int ensure_alloc(fdtd_ctx* c) {
    AdjointState& A = c->adj;
    const int N = c->opts.n_steps;
    const int every = c->opts.checkpoint_every;
    if (every <= 0) return fdtd_fail(c, FDTD_E_STATE, "checkpoint_every = 0: the run cannot be differentiated");
    const int n_ckpt = (N + every - 1) / every;
    if (A.slab && A.every == every && A.n_ckpt == n_ckpt) return FDTD_OK;
    if (A.slab) {
        (void)hipFree(A.slab);
        A.slab = nullptr;
    }
    A.every = every;
    A.n_ckpt = n_ckpt;
    A.inst.assign(c->inst.size(), AdjointInst{});
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    size_t total = 0;
    std::vector<size_t> off;
    for (auto& h : c->inst) {
        const size_t f = (size_t)h.ny * h.pitch * 4, p = (size_t)2 * h.n_pml * h.pitch * 4;
        const size_t st = 3 * f + 2 * p;
        for (size_t b : {f, f, f, p, p, f, f, f, f, f, (size_t)4 * h.pitch * 4, st * n_ckpt,
                         f * (size_t)(every + 1), st, sizeof(double) * 2 * kMaxLabels}) {
            off.push_back(total);
            total += al(b);
        }
    }
    if (hipMalloc(&A.slab, total) != hipSuccess) {
        (void)hipGetLastError();
        return fdtd_fail(c, FDTD_E_NOMEM, "adjoint allocation of " + std::to_string(total) + " bytes failed");
    }
    A.bytes = total;
    size_t k = 0;
    for (size_t q = 0; q < c->inst.size(); ++q) {
        AdjointInst& a = A.inst[q];
        HostInst& h = c->inst[q];
        float** ptrs[] = {&a.lez, &a.lhx, &a.lhy, &a.lpe, &a.lph, &a.tmp0, &a.tmp1, &a.tmp2, &a.gce, &a.gcb, &a.src,
                          &a.ckpt, &a.seg, &a.fin};
        for (float** pp : ptrs) *pp = (float*)(A.slab + off[k++]);
        a.lsum = (double*)(A.slab + off[k++]);
        a.state_floats = (size_t)3 * h.ny * h.pitch + (size_t)4 * h.n_pml * h.pitch;
    }
    return FDTD_OK;
}

}  // namespace

int adjoint_record_run(fdtd_ctx* c) {
    if (c->step != 0) return fdtd_fail(c, FDTD_E_STATE, "a recorded run must start at step 0 (call fdtd_reset)");
    int rc = ensure_alloc(c);
    if (rc != FDTD_OK) return rc;
    AdjointState& A = c->adj;
    const int N = c->opts.n_steps;
    for (int s = 0; s < A.n_ckpt; ++s) {
        for (size_t q = 0; q < c->inst.size(); ++q) {
            rc = copy_state(c, (int)q, c->cur, A.inst[q].ckpt + (size_t)s * A.inst[q].state_floats, true);
            if (rc != FDTD_OK) return rc;
        }
        const int len = std::min(A.every, N - s * A.every);
        rc = fdtd_enqueue_steps(c, len, c->K, c->B);
        if (rc != FDTD_OK) return rc;
    }
    A.recorded = true;
    return FDTD_OK;
}

void adjoint_free(fdtd_ctx* c) {
    if (c->adj.slab) (void)hipFree(c->adj.slab);
    c->adj.slab = nullptr;
}

int64_t adjoint_bytes(const fdtd_ctx* c) { return (int64_t)c->adj.bytes; }

extern "C" int fdtd_backward(fdtd_ctx* c, const double* dL_dR, const double* dL_dT, double* grad_nk,
                             float* grad_eps_pixel) {
    if (!c || !dL_dR) return FDTD_E_INVAL;
    AdjointState& A = c->adj;
    const int N = c->opts.n_steps;
    if (!A.recorded || c->step != N) return fdtd_fail(c, FDTD_E_STATE, "fdtd_backward needs a completed fdtd_run(ctx, 1)");
    // tone-fit amplitudes of every propagating order
    std::vector<std::vector<double>> fre, fim;
    std::vector<double> finc2;
    int rc = fdtd_order_amplitudes(c, fre, fim, finc2);
    if (rc != FDTD_OK) return rc;
    hipStream_t s = c->stream;
    const int n_inst = (int)c->inst.size();
    // save the final state; the segment replays overwrite the field buffers
    for (int q = 0; q < n_inst; ++q) {
        rc = copy_state(c, q, c->cur, A.inst[q].fin, true);
        if (rc != FDTD_OK) return rc;
    }
    std::vector<AdjDev> ad(n_inst);
    for (int q = 0; q < n_inst; ++q) {
        HostInst& h = c->inst[q];
        AdjointInst& a = A.inst[q];
        // dL/d(monitor sums): for line l with weight wl and G = Gram^-1,
        // dR/dSc_i = (2 wl/(nx |F_inc|^2)) Re[(G11 + i G12) U_i],
        // dR/dSs_i = (2 wl/(nx |F_inc|^2)) Re[(G12 + i G22) U_i],
        // U_i = sum_m w_m conj(F_m) exp(-2 pi i m i/nx).
        double g[3];
        fdtd_gram(h.wdt, c->opts.dft_start, N, g);
        const double det = g[0] * g[2] - g[1] * g[1];
        const double i11 = g[2] / det, i12 = -g[1] / det, i22 = g[0] / det;
        std::vector<float> src((size_t)4 * h.pitch, 0.f);
        const int no = (int)h.orders.size();
        for (int line = 0; line < 2; ++line) {
            const double wl = line == 0 ? dL_dR[q] : (dL_dT ? dL_dT[q] : 0.0);
            if (wl == 0.0) continue;
            const double scale = 2.0 * wl / (h.nx * finc2[q]);
            for (int i = 0; i < h.nx; ++i) {
                double ur = 0, ui = 0;
                for (int o = 0; o < no; ++o) {
                    const long long mm = ((long long)h.orders[o] % h.nx + h.nx) % h.nx;
                    const double ph = -2.0 * kPi * (double)((mm * i) % h.nx) / h.nx;
                    const double fr = fre[q][line * no + o], fi = fim[q][line * no + o];
                    const double cp = std::cos(ph), sp = std::sin(ph);
                    // w conj(F) e^{i ph}
                    ur += h.weights[o] * (fr * cp + fi * sp);
                    ui += h.weights[o] * (fr * sp - fi * cp);
                }
                src[(size_t)(2 * line) * h.pitch + i] = (float)(scale * (i11 * ur - i12 * ui));
                src[(size_t)(2 * line + 1) * h.pitch + i] = (float)(scale * (i12 * ur - i22 * ui));
            }
        }
        FDTD_HIPCHK(c, hipMemcpyAsync(a.src, src.data(), sizeof(float) * src.size(), hipMemcpyHostToDevice, s));
        const size_t f = (size_t)h.ny * h.pitch, p = (size_t)2 * h.n_pml * h.pitch;
        for (float* z : {a.lez, a.lhx, a.lhy, a.gce, a.gcb}) FDTD_HIPCHK(c, launch_fill(z, f, 0.f, s));
        for (float* z : {a.lpe, a.lph}) FDTD_HIPCHK(c, launch_fill(z, p, 0.f, s));
        ad[q] = AdjDev{a.lez, a.lhx, a.lhy, a.lpe, a.lph, a.tmp0, a.tmp1, a.tmp2, a.gce, a.gcb, a.src, nullptr, nullptr};
        FDTD_HIPCHK(c, hipStreamSynchronize(s));
    }
    // reverse sweep over the checkpoint segments
    for (int seg = A.n_ckpt - 1; seg >= 0; --seg) {
        const int s0 = seg * A.every, s1 = std::min(N, s0 + A.every);
        for (int q = 0; q < n_inst; ++q) {
            HostInst& h = c->inst[q];
            AdjointInst& a = A.inst[q];
            InstDev dn = h.dev;           // replay without touching the monitors
            dn.dft_start = 0x7fffffff;
            rc = copy_state(c, q, 0, a.ckpt + (size_t)seg * a.state_floats, false);
            if (rc != FDTD_OK) return rc;
            const size_t f = (size_t)h.ny * h.pitch;
            FDTD_HIPCHK(c, hipMemcpyAsync(a.seg, h.dev.ez[0], f * 4, hipMemcpyDeviceToDevice, s));
            for (int n = s0; n < s1; ++n) {
                FDTD_HIPCHK(c, launch_plain_step(dn, n, 0, s));
                FDTD_HIPCHK(c, hipMemcpyAsync(a.seg + (size_t)(n - s0 + 1) * f, h.dev.ez[0], f * 4,
                                              hipMemcpyDeviceToDevice, s));
            }
            dim3 grid((h.nx + 255) / 256, h.ny);
            for (int n = s1 - 1; n >= s0; --n) {
                AdjDev x = ad[q];
                x.e_old = a.seg + (size_t)(n - s0) * f;
                x.e_new = a.seg + (size_t)(n - s0 + 1) * f;
                k_adj_delta<<<grid, 256, 0, s>>>(h.dev, x);
                k_adj_e<<<grid, 256, 0, s>>>(h.dev, x, n);
                k_adj_h<<<grid, 256, 0, s>>>(h.dev, x);
                FDTD_HIPCHK(c, hipGetLastError());
            }
        }
    }
    // per-label sums and chain rule; per-pixel eps_r gradient
    size_t pix_off = 0;
    size_t lab_off = 0;
    for (int q = 0; q < n_inst; ++q) {
        HostInst& h = c->inst[q];
        AdjointInst& a = A.inst[q];
        FDTD_HIPCHK(c, hipMemsetAsync(a.lsum, 0, sizeof(double) * 2 * kMaxLabels, s));
        dim3 grid(std::max(1, std::min(16, (h.nx + 255) / 256)), h.ny);
        k_label_sums<<<grid, 256, 0, s>>>(h.dev, a.gce, a.gcb, a.lsum);
        FDTD_HIPCHK(c, hipGetLastError());
        std::vector<double> ls(2 * kMaxLabels);
        FDTD_HIPCHK(c, hipMemcpyAsync(ls.data(), a.lsum, sizeof(double) * 2 * kMaxLabels, hipMemcpyDeviceToHost, s));
        FDTD_HIPCHK(c, hipStreamSynchronize(s));
        std::vector<float2> deps(kMaxLabels, make_float2(0.f, 0.f));
        for (int L = 0; L < h.n_labels; ++L) {
            const double n = h.nk[2 * L], k = h.nk[2 * L + 1];
            const double eps = n * n - k * k;
            const double av = n * k * h.wdt / eps;
            const double cb = h.s1 / (eps * (1.0 + av));
            const double dce_da = -2.0 / ((1.0 + av) * (1.0 + av));
            const double da_dn = h.wdt * k / eps - 2.0 * n * av / eps;
            const double da_dk = h.wdt * n / eps + 2.0 * k * av / eps;
            const double dcb_dn = -cb * (2.0 * n / eps + da_dn / (1.0 + av));
            const double dcb_dk = -cb * (-2.0 * k / eps + da_dk / (1.0 + av));
            if (grad_nk) {
                grad_nk[lab_off + 2 * L] = ls[2 * L] * dce_da * da_dn + ls[2 * L + 1] * dcb_dn;
                grad_nk[lab_off + 2 * L + 1] = ls[2 * L] * dce_da * da_dk + ls[2 * L + 1] * dcb_dk;
            }
            const double da_de = -av / eps;
            deps[L] = make_float2((float)(dce_da * da_de), (float)(-cb * (1.0 / eps + da_de / (1.0 + av))));
        }
        if (grad_eps_pixel) {
            float2* d_deps = (float2*)a.tmp0;  // scratch: tmp0 is free after the sweep
            FDTD_HIPCHK(c, hipMemcpyAsync(d_deps, deps.data(), sizeof(float2) * kMaxLabels, hipMemcpyHostToDevice, s));
            dim3 grid2((h.nx + 255) / 256, h.ny);
            k_eps_grad<<<grid2, 256, 0, s>>>(h.dev, a.gce, a.gcb, d_deps, grad_eps_pixel + pix_off);
            FDTD_HIPCHK(c, hipGetLastError());
        }
        pix_off += h.cells();
        lab_off += 2 * (size_t)h.n_labels;
    }
    // restore the final forward state
    for (int q = 0; q < n_inst; ++q) {
        rc = copy_state(c, q, 0, A.inst[q].fin, false);
        if (rc != FDTD_OK) return rc;
    }
    c->cur = 0;
    FDTD_HIPCHK(c, hipStreamSynchronize(s));
    return FDTD_OK;
}
