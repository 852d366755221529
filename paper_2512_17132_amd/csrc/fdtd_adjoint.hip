// Discrete adjoint of the TMz FDTD run: the exact transpose of the forward
// recurrence, stepped backwards in time over checkpointed segments.
//
// Lossy FDTD is not time-reversible, so the forward states the gradient needs
// (Ez before and after every step) are recomputed segment by segment from
// checkpoints stored during a recorded forward run: a replay of the segment
// with the recording variant of the streaming kernel writes Ez of every step
// to a segment history, and the transposed steps then run backwards over it.
// The loss is L = sum_i dL_dR[i] R_i + dL_dT[i] T_i; its sensitivity to the
// monitor sums is injected on the monitor rows at every step of the window,
// and the per-pixel sensitivities to the update coefficients (Ce, Cb) are
// reduced per label and chained to (n, k) on the host, or mapped to eps_r per
// pixel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/fdtd.h"
#include "fdtd_adjoint.h"
#include "fdtd_device.h"
#include "fdtd_host.h"
#include "fdtd_kernels.h"

using namespace fdtd;

namespace {

constexpr double kPi = 3.14159265358979323846;
// 8 steps per launch: on the 1024 x 2048 monocot (8000 steps) the backward
// took 55.3 ms at 8, 57.9 at 10, 87.0 at 12 and 71.3 at 6
constexpr int kAdjDefaultTBlock = 8;

// rows per work item of the streaming adjoint kernel: the option, else the
// height tune_adj_band chose, else the forward's
int adj_band(const fdtd_ctx* c) {
    if (c->opts.adj_band_rows > 0) return c->opts.adj_band_rows;
    return c->adj.band > 0 ? c->adj.band : c->B;
}

// ---------------------------------------------------------------------------
// Plain transposed sweeps (one thread per cell, three launches per step, in
// place on lambda set 0): the adjoint of the plain forward kernels.
// ---------------------------------------------------------------------------

struct PlainAdj {
    float* lez;
    float* lhx;
    float* lhy;
    float* lpe;
    float* lph;
    float* t0;   // delta per Hx edge
    float* t1;   // mu per Ez cell
    float* t2;   // nu per Ez cell
    float* ga;
    float* gb;
    const float* src;     // [2][2][pitch]
    const float* e_old;   // Ez^{n-1/2}
    const float* e_new;   // Ez^{n+1/2}
};

__global__ __launch_bounds__(256) void k_adj_delta(InstDev d, PlainAdj a) {
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

__global__ __launch_bounds__(256) void k_adj_e(InstDev d, PlainAdj a, int n) {
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
    a.ga[o] = __fmaf_rn(av, eo, a.ga[o]);
    a.gb[o] = __fmaf_rn(av, __fmaf_rn(-cf.x, eo, en), a.gb[o]);
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

__global__ __launch_bounds__(256) void k_adj_h(InstDev d, PlainAdj a) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const size_t o = (size_t)j * d.pitch + i;
    const int il = (i == 0) ? d.nx - 1 : i - 1;
    if (j > 0) a.lhx[o] = a.lhx[o] + (a.t2[o] - a.t2[o - d.pitch]);
    a.lhy[o] = a.lhy[o] - (a.t1[o] - a.t1[(size_t)j * d.pitch + il]);
}

// ---------------------------------------------------------------------------
// Streaming transposed kernel with temporal blocking.
//
// The transposed step has the forward step's stencil shape (an E-like phase
// reading row j+1 and column i+1 of the input state, then an H-like phase
// reading row j-1 and column i-1 of the new values), so it runs in the same
// register pipeline as the forward kernel: one wave per work item (64
// periodic columns, 64 - 2K of them written, and a band of rows), walking the
// rows upwards; level t applies the transpose of step n_top - t + 1 to row
// r - t while row r is read.  Besides the lambda fields, every row carries
// its two gradient sums down the pipeline, each level adding its step's
// contribution, and every level reads Ez^{n-1/2} of its row and step from the
// segment history (prefetched one row ahead); Ez^{n+1/2} is the level above's
// Ez^{n-1/2}, handed down with the row.
// ---------------------------------------------------------------------------

struct AdjSlot {
    float le, lhx, lhy, ce, cb, lpe, lph, ga, gb, ehi, nu;
};

struct AdjLds {
    RowTab rows[kTabRows];      // profiles of every row the item touches (.w unused)
    float2 phasor[kMaxTBlock];  // of step n_top - t + 1 for level t
};

template <int K, bool SPECIAL>
__device__ __forceinline__ void adj_band(const InstDev& dref, const AdjDevT& aref, const WorkItem& w, int n_top,
                                         int lcur, int hslot_top, int lane, const float2* __restrict__ coef_lds,
                                         const AdjLds* __restrict__ sp) {
    const int nx = dref.nx, ny = dref.ny, pitch = dref.pitch;
    const float s1 = dref.s1;
    const int n_pml = SPECIAL ? dref.n_pml : 0;
    const int j_ref = dref.j_ref, j_trn = dref.j_trn, dft_start = dref.dft_start;
    const unsigned off_pe = dref.off_pe, off_ph = dref.off_ph, set_bytes = dref.set_bytes;
    const unsigned rowb = (unsigned)pitch * 4u;
    const unsigned plane_b = (unsigned)ny * rowb;
    const size_t plane = (size_t)ny * pitch;
    int col = w.x0 - K + lane;
    col %= nx;
    if (col < 0) col += nx;
    const bool valid_col = (lane >= K) && (lane < kWave - K) && (w.x0 + lane - K < nx);
    const bool c1 = lcur != 0;
    const __amdgpu_buffer_rsrc_t rin = make_rsrc(c1 ? aref.lset[1] : aref.lset[0], set_bytes);
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(c1 ? aref.lset[0] : aref.lset[1], set_bytes);
    const __amdgpu_buffer_rsrc_t rlab = make_rsrc(dref.lab, (unsigned)ny * (unsigned)pitch);
    const __amdgpu_buffer_rsrc_t rga = make_rsrc(aref.ga, plane_b);
    const __amdgpu_buffer_rsrc_t rgb = make_rsrc(aref.gb, plane_b);
    const unsigned vo = (unsigned)col * 4u, vl = (unsigned)col;
    const unsigned ohx = dref.off_hx, ohy = dref.off_hy;
    const float* __restrict__ hist = aref.hist;

    // adjoint sources of the two monitor rows: every item whose rows reach a
    // monitor row applies them there (they change the state, not only sums)
    float sr0 = 0.f, sr1 = 0.f, st0 = 0.f, st1 = 0.f;
    if (SPECIAL) {
        const float* __restrict__ src = aref.src;
        sr0 = gld(src, col);
        sr1 = gld(src, pitch + col);
        st0 = gld(src, 2 * pitch + col);
        st1 = gld(src, 3 * pitch + col);
    }

    AdjSlot S[K + 1][2];
#pragma unroll
    for (int t = 0; t <= K; ++t)
#pragma unroll
        for (int p = 0; p < 2; ++p) S[t][p] = AdjSlot{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

    const int r_begin = SPECIAL ? max(0, w.j0 - K) : w.j0 - K;
    const int r_end = w.j1 + K;

    // level-0 ring: lambda state, gradient sums, label, and Ez^{n_top+1/2}
    float l_le[2], l_lhx[2], l_lhy[2], l_lpe[2], l_lph[2], l_ga[2], l_gb[2], l_eh[2];
    int l_lab[2];
    const float* __restrict__ hist_top = hist + (size_t)(hslot_top + 1) * plane;
    auto fetch = [&](int r, int q) {
        const int rr = min(r, ny - 1);
        const unsigned so = (unsigned)rr * rowb;
        l_le[q] = buf_ld(rin, vo, so);
        l_lhx[q] = buf_ld(rin, vo, so + ohx);
        l_lhy[q] = buf_ld(rin, vo, so + ohy);
        l_lab[q] = buf_ld_u8(rlab, vl, (unsigned)rr * (unsigned)pitch);
        l_ga[q] = buf_ld(rga, vo, so);
        l_gb[q] = buf_ld(rgb, vo, so);
        l_eh[q] = gld(hist_top, (size_t)rr * pitch + col);
        if (SPECIAL) {
            l_lpe[q] = buf_ld(rin, vo, off_pe + (unsigned)psi_slot_e(rr, ny, n_pml) * rowb);
            l_lph[q] = buf_ld(rin, vo, off_ph + (unsigned)psi_slot_h(rr, ny, n_pml) * rowb);
        } else {
            l_lpe[q] = l_lph[q] = 0.f;
        }
    };
    // history ring of level t: Ez^{n_t - 1/2} of row j, slot (j - r_begin) & 1
    // relative to the level's first row r_begin - t
    float h_lo[K + 1][2];
    auto hfetch = [&](int t, int j, int q) {
        const int rr = min(max(j, 0), ny - 1);
        h_lo[t][q] = gld(hist, (size_t)(hslot_top - t + 1) * plane + (size_t)rr * pitch + col);
    };
    l_le[1] = l_lhx[1] = l_lhy[1] = l_lpe[1] = l_lph[1] = l_ga[1] = l_gb[1] = l_eh[1] = 0.f;
    l_lab[1] = 0;
    fetch(r_begin, 0);
#pragma unroll
    for (int t = 1; t <= K; ++t) {
        h_lo[t][0] = h_lo[t][1] = 0.f;
        hfetch(t, r_begin - t, t & 1);
    }

    auto iteration = [&](int r, auto P_) {
        constexpr int P = decltype(P_)::value;
        const RowTab* const rt = SPECIAL ? sp->rows + (r - r_begin) : nullptr;
#pragma unroll
        for (int t = 1; t <= K; ++t) {
            const int j = r - t;
            const int hq = (P ^ t) & 1;  // history ring slot of row j for level t
            AdjSlot pv;
            float up_lhx, up_lph;
            if (t == 1) {
                const float2 cf = coef_lds[l_lab[P ^ 1]];
                pv = AdjSlot{vcopy(l_le[P ^ 1]), vcopy(l_lhx[P ^ 1]), vcopy(l_lhy[P ^ 1]), cf.x, cf.y,
                             SPECIAL ? vcopy(l_lpe[P ^ 1]) : 0.f, SPECIAL ? vcopy(l_lph[P ^ 1]) : 0.f,
                             vcopy(l_ga[P ^ 1]), vcopy(l_gb[P ^ 1]), vcopy(l_eh[P ^ 1]), 0.f};
                up_lhx = l_lhx[P];
                up_lph = SPECIAL ? l_lph[P] : 0.f;
                fetch(r + 1, P ^ 1);
            } else {
                pv = S[t - 1][P ^ 1];
                up_lhx = S[t - 1][P].lhx;
                up_lph = S[t - 1][P].lph;
            }
            const float e_lo = h_lo[t][hq];
            const float e_hi = pv.ehi;
            hfetch(t, j + 1, hq ^ 1);
            const int n = n_top - t + 1;
            float le = pv.le;
            float lph = pv.lph, lpe = pv.lpe;
            float delta, delta_up;
            if (SPECIAL) {
                if (n >= dft_start) {
                    const float2 ph = sp->phasor[t - 1];
                    const float add_r = __fmaf_rn(sr0, ph.x, sr1 * ph.y);
                    const float add_t = __fmaf_rn(st0, ph.x, st1 * ph.y);
                    le = (j == j_ref) ? le + add_r : le;
                    le = (j == j_trn) ? le + add_t : le;
                }
                // branch-free form of adj_delta for row j and row j + 1: rows
                // outside the layers read the neutral profile (b = c = 0,
                // 1/kappa = 1), which reproduces the plain value
                const int ju = j + 1;
                const float4 prh = rt[K - t].h;
                const float4 pru = rt[K - t + 1].h;
                const float g = -s1 * pv.lhx;
                const float lt = lph + g;
                delta = __fmaf_rn(prh.z, g, prh.y * lt);
                lph = prh.x * lt;
                delta = (j > 0) ? delta : 0.f;   // Hx(0) is the wall
                const float gu = -s1 * up_lhx;
                delta_up = __fmaf_rn(pru.z, gu, pru.y * (up_lph + gu));
                delta_up = (ju < ny) ? delta_up : 0.f;   // no edge above the top row
            } else {
                delta = -s1 * pv.lhx;
                delta_up = -s1 * up_lhx;
            }
            const float lhy_r = from_right(pv.lhy);
            const float a = (le + (delta - delta_up)) - s1 * (lhy_r - pv.lhy);
            const float ga = __fmaf_rn(a, e_lo, pv.ga);
            const float gb = __fmaf_rn(a, __fmaf_rn(-pv.ce, e_lo, e_hi), pv.gb);
            const float le_new = pv.ce * a;
            const float mu = pv.cb * a;
            float nu;
            if (SPECIAL) {
                const float4 pre = rt[K - t].e;
                const float lt = lpe - mu;
                nu = __fmaf_rn(pre.z, mu, -(pre.y * lt));
                lpe = pre.x * lt;
            } else {
                nu = mu;
            }
            const float nu_below = S[t][P ^ 1].nu;
            float lhx_new = pv.lhx + (nu - nu_below);
            if (SPECIAL) lhx_new = (j > 0) ? lhx_new : pv.lhx;
            const float mu_l = from_left(mu);
            const float lhy_new = pv.lhy - (mu - mu_l);
            S[t][P] = AdjSlot{le_new, lhx_new, lhy_new, pv.ce, pv.cb, lpe, lph, ga, gb, e_lo, nu};
            if (t == K) {
                // owned cells only; other lanes and rows are dropped
                const bool owned = SPECIAL ? (j >= w.j0 && j < w.j1) : (j >= w.j0);
                const unsigned vs = (owned && valid_col) ? vo : kDropOffset;
                const unsigned so = (unsigned)j * rowb;
                buf_st(rout, vs, so, le_new);
                buf_st(rout, vs, so + ohx, lhx_new);
                buf_st(rout, vs, so + ohy, lhy_new);
                buf_st(rga, vs, so, ga);
                buf_st(rgb, vs, so, gb);
                if (SPECIAL) {
                    buf_st(rout, vs, off_pe + (unsigned)psi_slot_e(j, ny, n_pml) * rowb, lpe);
                    buf_st(rout, vs, off_ph + (unsigned)psi_slot_h(j, ny, n_pml) * rowb, lph);
                }
            }
        }
    };

    int r = r_begin;
    for (; r + 1 < r_end; r += 2) {
        iteration(r, std::integral_constant<int, 0>{});
        iteration(r + 1, std::integral_constant<int, 1>{});
    }
    if (r < r_end) iteration(r, std::integral_constant<int, 0>{});
}

template <int K, bool SPECIAL>
__global__ __launch_bounds__(256) void k_adj_tblock(const InstDev* __restrict__ insts, const AdjDevT* __restrict__ adjs,
                                                    const WorkItem* __restrict__ items, int n_items, int n_top,
                                                    int lcur, int hslot_top) {
    __shared__ float2 coef_lds[4][kMaxLabels];
    __shared__ AdjLds sp_lds[SPECIAL ? 4 : 1];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int it = xcd_item(wave);
    if (it >= n_items) return;
    const WorkItem w = items[it];
    const InstDev* __restrict__ dp = insts + w.inst;
    AdjLds* sp = &sp_lds[SPECIAL ? wave : 0];
    if (SPECIAL) {
        stage_rows(dp, w, K, sp->rows, lane);
        if (lane < K) sp->phasor[lane] = dp->phasor[n_top - lane];
    }
    stage_coef(dp, coef_lds[wave], lane);
    adj_band<K, SPECIAL>(*dp, adjs[w.inst], w, n_top, lcur, hslot_top, lane, coef_lds[wave], sp);
}

hipError_t launch_adj_tblock(int K, bool special, const InstDev* insts, const AdjDevT* adjs, const WorkItem* items,
                             int n_items, int n_top, int lcur, int hslot_top, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    const int blocks = ((n_items + 3) / 4 + 7) / 8 * 8;  // multiple of 8 for the XCD remap
    switch (K) {
#define FDTD_ADJ_CASE(k)                                                                                     \
    case k:                                                                                                  \
        if (special)                                                                                         \
            k_adj_tblock<k, true><<<blocks, 256, 0, s>>>(insts, adjs, items, n_items, n_top, lcur, hslot_top);  \
        else                                                                                                 \
            k_adj_tblock<k, false><<<blocks, 256, 0, s>>>(insts, adjs, items, n_items, n_top, lcur, hslot_top); \
        break;
        FDTD_ADJ_CASE(1)
        FDTD_ADJ_CASE(2)
        FDTD_ADJ_CASE(3)
        FDTD_ADJ_CASE(4)
        FDTD_ADJ_CASE(5)
        FDTD_ADJ_CASE(6)
        FDTD_ADJ_CASE(7)
        FDTD_ADJ_CASE(8)
        FDTD_ADJ_CASE(10)
        FDTD_ADJ_CASE(12)
#undef FDTD_ADJ_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reductions after the sweep
// ---------------------------------------------------------------------------

// Per-label sums of dL/dCe = ga and dL/dCb = gb / Cb in FP64, in a fixed
// order so that the result does not depend on scheduling: one wave per row
// walks the row in 64-column chunks; within a chunk it takes the labels
// present one at a time (the first remaining lane's label), sums that label's
// lanes with a fixed butterfly and adds the sum to the row's LDS total.  The
// row totals go to rows[j][label][2]; k_label_total adds them in row order.
__global__ __launch_bounds__(64) void k_label_rows(InstDev d, const float* __restrict__ ga,
                                                   const float* __restrict__ gb, double* __restrict__ rows) {
    __shared__ double acc[kMaxLabels][2];
    const int lane = threadIdx.x;
    for (int k = lane; k < d.n_labels; k += 64) acc[k][0] = acc[k][1] = 0.0;
    __syncthreads();
    const int j = blockIdx.x;
    for (int i0 = 0; i0 < d.nx; i0 += 64) {
        const int i = i0 + lane;
        int L = -1;
        double a = 0.0, b = 0.0;
        if (i < d.nx) {
            const size_t o = (size_t)j * d.pitch + i;
            L = d.lab[o];
            a = (double)ga[o];
            b = (double)gb[o] / (double)d.coef[L].y;
        }
        bool left = L >= 0;
        while (__any(left)) {
            // the label of the lowest lane still to be summed
            const unsigned long long m = __ballot(left);
            const int L0 = __shfl(L, __ffsll((long long)m) - 1);
            const bool mine = left && L == L0;
            double sa = mine ? a : 0.0, sb = mine ? b : 0.0;
            for (int w = 32; w >= 1; w >>= 1) {
                sa += __shfl_xor(sa, w);
                sb += __shfl_xor(sb, w);
            }
            if (lane == 0) {
                acc[L0][0] += sa;
                acc[L0][1] += sb;
            }
            left = left && !mine;
        }
    }
    __syncthreads();
    for (int k = lane; k < d.n_labels; k += 64) {
        rows[((size_t)j * d.n_labels + k) * 2] = acc[k][0];
        rows[((size_t)j * d.n_labels + k) * 2 + 1] = acc[k][1];
    }
}

// out[2 L + c] = sum over rows j, in order, of rows[j][L][c].
__global__ __launch_bounds__(256) void k_label_total(InstDev d, const double* __restrict__ rows,
                                                     double* __restrict__ out) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= 2 * d.n_labels) return;
    double s = 0.0;
    for (int j = 0; j < d.ny; ++j) s += rows[(size_t)j * 2 * d.n_labels + t];
    out[t] = s;
}

// dL/d eps_r per pixel at fixed sigma: dL/dCe dCe/deps + dL/dCb dCb/deps, with
// the per-label derivatives in `deriv` ([n_labels][2]); output row-major, no
// pitch.
__global__ __launch_bounds__(256) void k_eps_grad(InstDev d, const float* __restrict__ ga,
                                                  const float* __restrict__ gb, const float2* __restrict__ deriv,
                                                  float* __restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const size_t o = (size_t)j * d.pitch + i;
    const int L = d.lab[o];
    const float2 dv = deriv[L];
    out[(size_t)j * d.nx + i] = __fmaf_rn(ga[o], dv.x, (gb[o] / d.coef[L].y) * dv.y);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// copies one instance's field set `cur` to (to_store) or from a set-sized
// buffer: one contiguous region per set
int copy_state(fdtd_ctx* c, int q, int cur, float* buf, bool to_store) {
    HostInst& h = c->inst[q];
    const size_t bytes = h.dev.set_bytes;
    if (to_store)
        FDTD_HIPCHK(c, hipMemcpyAsync(buf, h.dev.ez[cur], bytes, hipMemcpyDeviceToDevice, c->stream));
    else
        FDTD_HIPCHK(c, hipMemcpyAsync(h.dev.ez[cur], buf, bytes, hipMemcpyDeviceToDevice, c->stream));
    return FDTD_OK;
}

// Checkpoint spacing of checkpoint_every = -1: about sqrt(N) steps (the
// memory of checkpoints and of one segment's history balance there), moved to
// the nearest multiple of both launch lengths when one lies within a factor
// 1.5 of sqrt(N), so that a segment's replay and transposed steps are whole
// launches (a short tail launch costs nearly as much as a full one on a grid
// whose launches are latency-bound).
int auto_checkpoint_every(const fdtd_ctx* c) {
    const int N = c->opts.n_steps;
    const double root = std::sqrt((double)N);
    const int base = std::max(1, (int)std::lround(root));
    if (c->opts.kernel == 1) return base;
    const int adjK = c->opts.adj_t_block > 0 ? c->opts.adj_t_block : kAdjDefaultTBlock;
    const int L = std::lcm(std::max(1, c->K), adjK);
    const int m = std::max(1, (int)std::lround(root / L)) * L;
    return (m <= 1.5 * root && m >= root / 1.5 && m <= N) ? m : base;
}

// Device bytes of the Ez history of a whole run (one segment of n_steps).
static size_t full_history_bytes(const fdtd_ctx* c) {
    size_t b = 0;
    for (auto& h : c->inst) b += (((size_t)h.ny * h.pitch * 4 * ((size_t)c->opts.n_steps + 1)) + 255) & ~size_t(255);
    return b;
}

int ensure_alloc(fdtd_ctx* c) {
    AdjointState& A = c->adj;
    const int N = c->opts.n_steps;
    int every = c->opts.checkpoint_every;
    if (every == 0) return fdtd_fail(c, FDTD_E_STATE, "checkpoint_every = 0: the run cannot be differentiated");
    if (every < 0) {
        // the whole run's Ez history when it takes at most half the device
        // memory free to the adjoint (what is free plus what its current
        // buffers hold, which a new choice would release): the backward then
        // replays nothing.  Else about sqrt(N)-step segments.
        size_t free_b = 0, total_b = 0;
        const bool fits = c->opts.kernel == 0 && hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
                          full_history_bytes(c) <= (free_b + (A.slab ? A.bytes : 0)) / 2;
        every = fits ? N : auto_checkpoint_every(c);
    }
    every = std::min(every, N);
    const int n_ckpt = (N + every - 1) / every;
    const bool full = every == N && c->opts.kernel == 0;
    if (A.slab && A.every == every && A.n_ckpt == n_ckpt && A.full == full) return FDTD_OK;
    if (A.slab) {
        if (A.graph) (void)hipGraphExecDestroy(A.graph);
        A.graph = nullptr;
        (void)hipFree(A.slab);
        A.slab = nullptr;
    }
    A.full = full;
    A.every = every;
    A.n_ckpt = n_ckpt;
    A.band = 0;   // chosen again by the next backward
    const int n_inst = (int)c->inst.size();
    A.inst.assign(n_inst, AdjointInst{});
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    size_t total = 0;
    std::vector<size_t> off;
    auto take = [&](size_t b) {
        off.push_back(total);
        total += al(b);
    };
    for (auto& h : c->inst) {
        const size_t f = (size_t)h.ny * h.pitch * 4;
        const size_t st = h.dev.set_bytes;
        take(st);                            // lambda set 0
        take(st);                            // lambda set 1
        take(f); take(f); take(f);           // plain-sweep scratch
        take(f); take(f);                    // ga, gb
        take((size_t)4 * h.pitch * 4);       // src
        take(st * n_ckpt);                   // checkpoints
        take(f * (size_t)(every + 1));       // segment history
        take(st);                            // final state
        take(sizeof(double) * 2 * kMaxLabels);
        take(sizeof(double) * 2 * (size_t)h.n_labels * h.ny);   // per-row label sums
    }
    take(sizeof(InstDev) * n_inst);
    take(sizeof(InstDev) * n_inst);
    take(sizeof(AdjDevT) * n_inst);
    if (hipMalloc(&A.slab, total) != hipSuccess) {
        (void)hipGetLastError();
        return fdtd_fail(c, FDTD_E_NOMEM, "adjoint allocation of " + std::to_string(total) + " bytes failed");
    }
    A.bytes = total;
    size_t k = 0;
    std::vector<InstDev> rec(n_inst), recm(n_inst);
    std::vector<AdjDevT> adj(n_inst);
    for (int q = 0; q < n_inst; ++q) {
        AdjointInst& a = A.inst[q];
        HostInst& h = c->inst[q];
        float** ptrs[] = {&a.lset[0], &a.lset[1], &a.tmp0, &a.tmp1, &a.tmp2, &a.ga, &a.gb, &a.src,
                          &a.ckpt, &a.seg, &a.fin};
        for (float** pp : ptrs) *pp = (float*)(A.slab + off[k++]);
        a.lsum = (double*)(A.slab + off[k++]);
        a.rowsum = (double*)(A.slab + off[k++]);
        a.set_floats = h.dev.set_bytes / 4;
        rec[q] = h.dev;                    // replay: monitors off, history on
        rec[q].dft_start = INT_MAX;
        rec[q].hist = a.seg;
        recm[q] = h.dev;                   // single-segment recorded run: monitors and history on
        recm[q].hist = a.seg;
        adj[q] = AdjDevT{{a.lset[0], a.lset[1]}, a.ga, a.gb, a.seg, a.src};
    }
    A.d_rec = (InstDev*)(A.slab + off[k++]);
    A.d_recm = (InstDev*)(A.slab + off[k++]);
    A.d_adj = (AdjDevT*)(A.slab + off[k++]);
    FDTD_HIPCHK(c, hipMemcpyAsync(A.d_rec, rec.data(), sizeof(InstDev) * n_inst, hipMemcpyHostToDevice, c->stream));
    FDTD_HIPCHK(c, hipMemcpyAsync(A.d_recm, recm.data(), sizeof(InstDev) * n_inst, hipMemcpyHostToDevice, c->stream));
    FDTD_HIPCHK(c, hipMemcpyAsync(A.d_adj, adj.data(), sizeof(AdjDevT) * n_inst, hipMemcpyHostToDevice, c->stream));
    FDTD_HIPCHK(c, hipStreamSynchronize(c->stream));
    return FDTD_OK;
}

// Forward steps [s0, s1) of every instance from the state in field set 0,
// writing Ez^{n+1/2} of each step n to history slot n - s0 + 1.  Leaves the
// state in set c->cur.  insts: the replay descriptors (monitors off), or the
// recorded run's (monitors on) for the single-segment form.
int enqueue_replay(fdtd_ctx* c, int s0, int s1, const InstDev* insts) {
    AdjointState& A = c->adj;
    hipStream_t s = c->stream;
    c->cur = 0;
    if (c->opts.kernel == 1) {
        for (size_t q = 0; q < c->inst.size(); ++q) {
            const HostInst& h = c->inst[q];
            InstDev dn = h.dev;
            dn.dft_start = INT_MAX;
            const size_t f = (size_t)h.ny * h.pitch;
            for (int n = s0; n < s1; ++n) {
                FDTD_HIPCHK(c, launch_plain_step(dn, n, 0, s));
                FDTD_HIPCHK(c, hipMemcpyAsync(A.inst[q].seg + (size_t)(n - s0 + 1) * f, h.dev.ez[0], f * 4,
                                              hipMemcpyDeviceToDevice, s));
            }
        }
        return FDTD_OK;
    }
    for (int n = s0; n < s1;) {
        const int k = fdtd_launch_steps(c->K, s1 - n);
        ItemList* L = fdtd_item_list(c, k, c->B);
        if (!L) return fdtd_fail(c, FDTD_E_NOMEM, "work-item list allocation failed");
        if (L->n_special > 0) {
            FDTD_HIPCHK(c, hipEventRecord(c->ev_fork, s));
            FDTD_HIPCHK(c, hipStreamWaitEvent(c->aux, c->ev_fork, 0));
            FDTD_HIPCHK(c, launch_tblock(k, true, insts, L->d, L->n_special, n, c->cur, c->aux, true, n - s0 + 1));
            FDTD_HIPCHK(c, hipEventRecord(c->ev_join, c->aux));
        }
        FDTD_HIPCHK(c, fdtd_launch_bulk_tm(c, k, insts, L, n, c->cur, s, true, n - s0 + 1));
        if (L->n_special > 0) FDTD_HIPCHK(c, hipStreamWaitEvent(s, c->ev_join, 0));
        c->cur ^= 1;
        n += k;
    }
    return FDTD_OK;
}

// Transposed steps s1 - 1 down to s0 over the segment history.
int launch_adj_block(fdtd_ctx* c, int k, int B, int n_top, int s0);
int tune_adj_band(fdtd_ctx* c);

int enqueue_adjoint(fdtd_ctx* c, int s0, int s1) {
    AdjointState& A = c->adj;
    hipStream_t s = c->stream;
    if (c->opts.kernel == 1) {
        for (size_t q = 0; q < c->inst.size(); ++q) {
            const HostInst& h = c->inst[q];
            AdjointInst& a = A.inst[q];
            const InstDev& d = h.dev;
            const size_t f = (size_t)h.ny * h.pitch;
            float* base = a.lset[0];
            PlainAdj x{base, (float*)((char*)base + d.off_hx), (float*)((char*)base + d.off_hy),
                       (float*)((char*)base + d.off_pe), (float*)((char*)base + d.off_ph), a.tmp0, a.tmp1, a.tmp2,
                       a.ga, a.gb, a.src, nullptr, nullptr};
            dim3 grid((h.nx + 255) / 256, h.ny);
            for (int n = s1 - 1; n >= s0; --n) {
                x.e_old = a.seg + (size_t)(n - s0) * f;
                x.e_new = a.seg + (size_t)(n - s0 + 1) * f;
                k_adj_delta<<<grid, 256, 0, s>>>(d, x);
                k_adj_e<<<grid, 256, 0, s>>>(d, x, n);
                k_adj_h<<<grid, 256, 0, s>>>(d, x);
                FDTD_HIPCHK(c, hipGetLastError());
            }
        }
        return FDTD_OK;
    }
    const int K = c->opts.adj_t_block > 0 ? c->opts.adj_t_block : kAdjDefaultTBlock;
    for (int n_top = s1 - 1; n_top >= s0;) {
        const int k = fdtd_launch_steps(K, n_top - s0 + 1);
        const int rc = launch_adj_block(c, k, adj_band(c), n_top, s0);
        if (rc != FDTD_OK) return rc;
        n_top -= k;
    }
    return FDTD_OK;
}

// One launch of the streaming transposed kernel: k steps down from n_top
// (segment start s0) with bands of B rows; special items on the auxiliary
// stream, joined before the next launch.
int launch_adj_block(fdtd_ctx* c, int k, int B, int n_top, int s0) {
    AdjointState& A = c->adj;
    hipStream_t s = c->stream;
    ItemList* L = fdtd_item_list(c, k, B);
    if (!L) return fdtd_fail(c, FDTD_E_NOMEM, "work-item list allocation failed");
    if (L->n_special > 0) {
        FDTD_HIPCHK(c, hipEventRecord(c->ev_fork, s));
        FDTD_HIPCHK(c, hipStreamWaitEvent(c->aux, c->ev_fork, 0));
        FDTD_HIPCHK(c, launch_adj_tblock(k, true, c->d_insts, A.d_adj, L->d, L->n_special, n_top, A.lcur, n_top - s0,
                                         c->aux));
        FDTD_HIPCHK(c, hipEventRecord(c->ev_join, c->aux));
    }
    FDTD_HIPCHK(c, launch_adj_tblock(k, false, c->d_insts, A.d_adj, L->d + L->n_special, L->n_lean, n_top, A.lcur,
                                     n_top - s0, s));
    if (L->n_special > 0) FDTD_HIPCHK(c, hipStreamWaitEvent(s, c->ev_join, 0));
    A.lcur ^= 1;
    return FDTD_OK;
}

// Chooses the streaming adjoint kernel's band height (unless
// opts.adj_band_rows fixes it) by timing a few launches over the first
// segment's history at each candidate height.  The transposed kernel carries
// more per cell than the forward one, so on grids where its launches are
// latency-bound thinner bands than the forward's (more, shorter waves) can
// pay.  Works on zeroed lambda sets and gradient sums, which fdtd_backward
// zeroes again before its sweep.
int tune_adj_band(fdtd_ctx* c) {
    AdjointState& A = c->adj;
    if (c->opts.adj_band_rows > 0 || c->opts.kernel == 1 || A.band > 0) return FDTD_OK;
    hipStream_t s = c->stream;
    for (size_t q = 0; q < c->inst.size(); ++q) {
        const HostInst& h = c->inst[q];
        AdjointInst& a = A.inst[q];
        for (float* z : {a.lset[0], a.lset[1]}) FDTD_HIPCHK(c, launch_fill(z, h.dev.set_bytes / 4, 0.f, s));
        for (float* z : {a.ga, a.gb, a.src}) FDTD_HIPCHK(c, launch_fill(z, z == a.src ? 4 * (size_t)h.pitch
                                                                                       : (size_t)h.ny * h.pitch, 0.f, s));
    }
    const int K = c->opts.adj_t_block > 0 ? c->opts.adj_t_block : kAdjDefaultTBlock;
    const int k = fdtd_launch_steps(K, A.every);
    hipEvent_t e0, e1;
    FDTD_HIPCHK(c, hipEventCreate(&e0));
    FDTD_HIPCHK(c, hipEventCreate(&e1));
    double best = 1e30;
    int best_B = c->B;
    for (int B : {16, 32, 48, 64, 96, 128, 192, 256}) {
        A.lcur = 0;
        int rc = launch_adj_block(c, k, B, k - 1, 0);   // builds the list, warms up
        if (rc != FDTD_OK) return rc;
        FDTD_HIPCHK(c, hipEventRecord(e0, s));
        for (int rep = 0; rep < 3 && rc == FDTD_OK; ++rep) rc = launch_adj_block(c, k, B, k - 1, 0);
        if (rc != FDTD_OK) return rc;
        FDTD_HIPCHK(c, hipEventRecord(e1, s));
        FDTD_HIPCHK(c, hipEventSynchronize(e1));
        float ms = 0;
        FDTD_HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
            best = ms;
            best_B = B;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    A.band = best_B;
    A.lcur = 0;
    return FDTD_OK;
}

}  // namespace

// The reverse sweep over the checkpoint segments: per segment, restore its
// checkpoint into field set 0, replay it forward recording Ez, then step the
// transposed recurrence back through it.
static int enqueue_sweep_direct(fdtd_ctx* c) {
    AdjointState& A = c->adj;
    const int N = c->opts.n_steps;
    A.lcur = 0;
    for (int seg = A.n_ckpt - 1; seg >= 0; --seg) {
        const int s0 = seg * A.every, s1 = std::min(N, s0 + A.every);
        if (!A.full) {   // the single segment's history was written by the recorded run
            for (int q = 0; q < (int)c->inst.size(); ++q) {
                HostInst& h = c->inst[q];
                AdjointInst& a = A.inst[q];
                int rc = copy_state(c, q, 0, a.ckpt + (size_t)seg * a.set_floats, false);
                if (rc != FDTD_OK) return rc;
                FDTD_HIPCHK(c, hipMemcpyAsync(a.seg, h.dev.ez[0], (size_t)h.ny * h.pitch * 4, hipMemcpyDeviceToDevice,
                                              c->stream));
            }
            int rc = enqueue_replay(c, s0, s1, A.d_rec);
            if (rc != FDTD_OK) return rc;
        }
        int rc = enqueue_adjoint(c, s0, s1);
        if (rc != FDTD_OK) return rc;
    }
    return FDTD_OK;
}

// The reverse sweep, replayed from a captured graph when opts.use_graph is
// set and graph replay measured faster for the forward launches (captured on
// first use, and again after the launch shape or the adjoint's buffers
// change): the sweep is a few thousand short launches and copies on a small
// grid, whose issue gaps the graph removes.  The sweep's
// inputs (the adjoint source, the zeroed lambda sets and gradient sums) are
// written before it, outside the graph.
static int enqueue_sweep(fdtd_ctx* c) {
    AdjointState& A = c->adj;
    if (!c->opts.use_graph || !c->graph_faster || c->opts.kernel == 1) return enqueue_sweep_direct(c);
    const int adjK = c->opts.adj_t_block > 0 ? c->opts.adj_t_block : kAdjDefaultTBlock;
    if (!A.graph || A.graph_K != c->K || A.graph_B != c->B || A.graph_SB != c->SB || A.graph_W != c->W ||
        A.graph_adjK != adjK || A.graph_adjB != adj_band(c) || A.graph_slab != A.slab) {
        if (A.graph) {
            (void)hipGraphExecDestroy(A.graph);
            A.graph = nullptr;
        }
        // every work-item list the sweep launches exists before the capture
        // (a capture cannot allocate)
        const int N = c->opts.n_steps;
        for (int seg = A.n_ckpt - 1; seg >= 0; --seg) {
            const int s0 = seg * A.every, s1 = std::min(N, s0 + A.every);
            for (int n = s0; n < s1 && !A.full;) {
                const int k = fdtd_launch_steps(c->K, s1 - n);
                if (!fdtd_item_list(c, k, c->B)) return fdtd_fail(c, FDTD_E_NOMEM, "work-item list allocation failed");
                n += k;
            }
            for (int n_top = s1 - 1; n_top >= s0;) {
                const int k = fdtd_launch_steps(adjK, n_top - s0 + 1);
                if (!fdtd_item_list(c, k, adj_band(c)))
                    return fdtd_fail(c, FDTD_E_NOMEM, "work-item list allocation failed");
                n_top -= k;
            }
        }
        hipGraph_t g = nullptr;
        FDTD_HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue_sweep_direct(c);
        const hipError_t e = hipStreamEndCapture(c->stream, &g);
        if (rc != FDTD_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fdtd_fail(c, FDTD_E_HIP, std::string("adjoint graph capture: ") + hipGetErrorString(e));
        const hipError_t ei = hipGraphInstantiate(&A.graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            A.graph = nullptr;
            return fdtd_fail(c, FDTD_E_HIP, std::string("adjoint graph instantiate: ") + hipGetErrorString(ei));
        }
        A.graph_K = c->K;
        A.graph_W = c->W;
        A.graph_B = c->B;
        A.graph_SB = c->SB;
        A.graph_adjK = adjK;
        A.graph_adjB = adj_band(c);
        A.graph_slab = A.slab;
    }
    A.lcur = 0;
    FDTD_HIPCHK(c, hipGraphLaunch(A.graph, c->stream));
    return FDTD_OK;
}

int adjoint_record_run(fdtd_ctx* c) {
    if (c->step != 0) return fdtd_fail(c, FDTD_E_STATE, "a recorded run must start at step 0 (call fdtd_reset)");
    for (size_t q = 0; q < c->inst.size(); ++q) {
        if (c->inst[q].pol != 0 || c->inst[q].n_freqs)
            return fdtd_fail(c, FDTD_E_INVAL,
                             "instance " + std::to_string(q) + ": the adjoint covers monochromatic TMz instances only");
        if (c->inst[q].n_steps != c->opts.n_steps)
            return fdtd_fail(c, FDTD_E_INVAL, "instance " + std::to_string(q) + ": the adjoint needs every instance to run opts.n_steps steps");
    }
    int rc = ensure_alloc(c);
    if (rc != FDTD_OK) return rc;
    AdjointState& A = c->adj;
    const int N = c->opts.n_steps;
    if (A.full) {
        // the whole run with the recording kernels: Ez of every step to the
        // history (slot 0: the initial state), monitors as in any run
        for (size_t q = 0; q < c->inst.size(); ++q) {
            const HostInst& h = c->inst[q];
            FDTD_HIPCHK(c, hipMemcpyAsync(A.inst[q].seg, h.dev.ez[c->cur], (size_t)h.ny * h.pitch * 4,
                                          hipMemcpyDeviceToDevice, c->stream));
        }
        rc = enqueue_replay(c, 0, N, A.d_recm);
        if (rc != FDTD_OK) return rc;
        c->step = N;
        for (auto& h : c->inst) h.cur_end = c->cur;
        A.recorded = true;
        return FDTD_OK;
    }
    for (int s = 0; s < A.n_ckpt; ++s) {
        for (size_t q = 0; q < c->inst.size(); ++q) {
            rc = copy_state(c, (int)q, c->cur, A.inst[q].ckpt + (size_t)s * A.inst[q].set_floats, true);
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
    if (c->adj.graph) (void)hipGraphExecDestroy(c->adj.graph);
    c->adj.graph = nullptr;
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
    rc = tune_adj_band(c);
    if (rc != FDTD_OK) return rc;
    // save the final state; the segment replays overwrite the field buffers
    for (int q = 0; q < n_inst; ++q) {
        rc = copy_state(c, q, c->cur, A.inst[q].fin, true);
        if (rc != FDTD_OK) return rc;
    }
    std::vector<std::vector<float>> srcs(n_inst);
    for (int q = 0; q < n_inst; ++q) {
        HostInst& h = c->inst[q];
        AdjointInst& a = A.inst[q];
        // dL/d(monitor sums): for line l with weight wl and G = Gram^-1,
        // dR/dSc_i = (2 wl/(nx |F_inc|^2)) Re[(G11 + i G12) U_i],
        // dR/dSs_i = (2 wl/(nx |F_inc|^2)) Re[(G12 + i G22) U_i],
        // U_i = sum_m w_m conj(F_m) exp(-2 pi i m i/nx).
        double g[3];
        fdtd_gram(h.wdt, h.dft_start, N, g, fdtd_sample_offset(h.pol));
        const double det = g[0] * g[2] - g[1] * g[1];
        const double i11 = g[2] / det, i12 = -g[1] / det, i22 = g[0] / det;
        std::vector<float>& src = srcs[q];
        src.assign((size_t)4 * h.pitch, 0.f);
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
        const size_t f = (size_t)h.ny * h.pitch;
        for (float* z : {a.lset[0], a.lset[1]}) FDTD_HIPCHK(c, launch_fill(z, h.dev.set_bytes / 4, 0.f, s));
        for (float* z : {a.ga, a.gb}) FDTD_HIPCHK(c, launch_fill(z, f, 0.f, s));
    }
    rc = enqueue_sweep(c);
    if (rc != FDTD_OK) return rc;
    // per-label sums and chain rule; per-pixel eps_r gradient
    size_t pix_off = 0;
    size_t lab_off = 0;
    for (int q = 0; q < n_inst; ++q) {
        HostInst& h = c->inst[q];
        AdjointInst& a = A.inst[q];
        k_label_rows<<<h.ny, 64, 0, s>>>(h.dev, a.ga, a.gb, a.rowsum);
        k_label_total<<<(2 * h.n_labels + 255) / 256, 256, 0, s>>>(h.dev, a.rowsum, a.lsum);
        FDTD_HIPCHK(c, hipGetLastError());
        std::vector<double> ls(2 * kMaxLabels, 0.0);
        FDTD_HIPCHK(c, hipMemcpyAsync(ls.data(), a.lsum, sizeof(double) * 2 * h.n_labels, hipMemcpyDeviceToHost, s));
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
            k_eps_grad<<<grid2, 256, 0, s>>>(h.dev, a.ga, a.gb, d_deps, grad_eps_pixel + pix_off);
            FDTD_HIPCHK(c, hipGetLastError());
        }
        pix_off += h.cells();
        lab_off += 2 * (size_t)h.n_labels;
    }
    // restore the final forward state into set 0, which then holds every
    // instance's state (all of them ended at step N)
    for (int q = 0; q < n_inst; ++q) {
        rc = copy_state(c, q, 0, A.inst[q].fin, false);
        if (rc != FDTD_OK) return rc;
        c->inst[q].cur_end = 0;
    }
    c->cur = 0;
    FDTD_HIPCHK(c, hipStreamSynchronize(s));
    return FDTD_OK;
}
