// gfx950 kernels of the TMz FDTD path: plain per-step E and H sweeps, the
// temporally blocked streaming kernel, Bloch projection of the monitors, and
// small utility kernels.  All cell arithmetic goes through fdtd_device.h.
#include <type_traits>

#include "fdtd_device.h"
#include "fdtd_kernels.h"

namespace fdtd {

// ---------------------------------------------------------------------------
// Plain sweeps: one E launch and one H launch per step, in place, one thread
// per cell.  The reference GPU path of the scheme (Sec. 2.3 eqs. 18-20).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_plain_e(InstDev d, int n, int cur) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const size_t o = (size_t)j * d.pitch + i;
    const int ir = (i + 1 == d.nx) ? 0 : i + 1;
    const float hx_c = d.hx[cur][o];
    const float hx_u = (j + 1 < d.ny) ? d.hx[cur][o + d.pitch] : 0.0f;
    const float hy_c = d.hy[cur][o];
    const float hy_r = d.hy[cur][(size_t)j * d.pitch + ir];
    const float2 cf = d.coef[d.lab[o]];
    const bool pml = is_pml_e(j, d.ny, d.n_pml);
    float pe = 0.0f;
    float4 pr = make_float4(0.f, 0.f, 1.f, 0.f);
    size_t po = 0;
    if (pml) {
        po = (size_t)psi_row(j, d.ny, d.n_pml) * d.pitch + i;
        pe = d.pe[cur][po];
        pr = d.prof_e[j];
    }
    const float e = upd_e(d.ez[cur][o], cf.x, cf.y, hy_c, hy_r, hx_c, hx_u, pml, pr, pe, j == d.j_src, d.inc[n].y);
    d.ez[cur][o] = e;
    if (pml) d.pe[cur][po] = pe;
    if (n >= d.dft_start) {
        if (j == d.j_ref) monitor_add(d, 0, i, e, d.phasor[n]);
        if (j == d.j_trn) monitor_add(d, 1, i, e, d.phasor[n]);
    }
}

__global__ __launch_bounds__(256) void k_plain_h(InstDev d, int n, int cur) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const size_t o = (size_t)j * d.pitch + i;
    const float* ez = d.ez[cur];
    const float e_c = ez[o];
    if (j > 0) {
        const bool pml = is_pml_h(j, d.ny, d.n_pml);
        float ph = 0.0f;
        float4 pr = make_float4(0.f, 0.f, 1.f, 0.f);
        size_t po = 0;
        if (pml) {
            po = (size_t)psi_row(j, d.ny, d.n_pml) * d.pitch + i;
            ph = d.ph[cur][po];
            pr = d.prof_h[j];
        }
        d.hx[cur][o] = upd_hx(d.hx[cur][o], e_c, ez[o - d.pitch], d.s1, pml, pr, ph, j == d.j_src + 1, d.inc[n].x);
        if (pml) d.ph[cur][po] = ph;
    }
    const int il = (i == 0) ? d.nx - 1 : i - 1;
    d.hy[cur][o] = upd_hy(d.hy[cur][o], e_c, ez[(size_t)j * d.pitch + il], d.s1);
}

// ---------------------------------------------------------------------------
// Streaming kernel with temporal blocking.
//
// Each wavefront owns a work item: 64 consecutive columns (periodic) of one
// instance, of which the middle 64 - 2K are written, and a band of output rows
// [j0, j1).  It walks the rows upwards.  Level t of the pipeline advances the
// fields of row r - t from step n0 + t - 1 to step n0 + t while row r is read
// from memory, so one pass over the band performs K steps.  A level needs, from
// the level below it, row j (all fields) and row j+1 (Hx), and from itself row
// j-1 (Ez); every level therefore keeps two row slots in registers, written
// alternately on even and odd iterations.  The x neighbours Hy(i+1) and
// Ez(i-1) come from the adjacent lanes through DPP wave shifts; each level
// invalidates one lane at each end, hence the 2K halo columns.  Rows of the
// band's K-row halo above and below are recomputed, not exchanged.
// ---------------------------------------------------------------------------

struct Slot {
    float e, hx, hy, ce, cb, pe, ph;
};

template <int K, bool PML>
__device__ __forceinline__ void tblock_body(const InstDev& d, const WorkItem& w, int n0, int cur, int lane,
                                            const float2* __restrict__ coef_lds) {
    const int nx = d.nx, ny = d.ny, pitch = d.pitch;
    int col = w.x0 - K + lane;
    col %= nx;
    if (col < 0) col += nx;
    const bool valid_col = (lane >= K) && (lane < kWave - K) && (w.x0 + lane - K < nx);
    // select, not index: a runtime index into the descriptor would force it
    // into scratch memory
    const bool c1 = cur != 0;
    const float* __restrict__ ez_in = c1 ? d.ez[1] : d.ez[0];
    const float* __restrict__ hx_in = c1 ? d.hx[1] : d.hx[0];
    const float* __restrict__ hy_in = c1 ? d.hy[1] : d.hy[0];
    const float* __restrict__ pe_in = c1 ? d.pe[1] : d.pe[0];
    const float* __restrict__ ph_in = c1 ? d.ph[1] : d.ph[0];
    float* __restrict__ ez_out = c1 ? d.ez[0] : d.ez[1];
    float* __restrict__ hx_out = c1 ? d.hx[0] : d.hx[1];
    float* __restrict__ hy_out = c1 ? d.hy[0] : d.hy[1];
    float* __restrict__ pe_out = c1 ? d.pe[0] : d.pe[1];
    float* __restrict__ ph_out = c1 ? d.ph[0] : d.ph[1];
    const uint8_t* __restrict__ lab = d.lab;

    Slot S[K + 1][2];
#pragma unroll
    for (int t = 0; t <= K; ++t)
#pragma unroll
        for (int p = 0; p < 2; ++p) S[t][p] = Slot{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

    const int r_begin = max(0, w.j0 - K);
    const int r_end = w.j1 + K;

    // prefetch registers for the next level-0 row
    float pf_e = 0.f, pf_hx = 0.f, pf_hy = 0.f, pf_pe = 0.f, pf_ph = 0.f;
    int pf_lab = 0;
    auto fetch = [&](int r) {
        if (r < ny) {
            const size_t o = (size_t)r * pitch + col;
            pf_e = ez_in[o];
            pf_hx = hx_in[o];
            pf_hy = hy_in[o];
            pf_lab = lab[o];
            if (PML) {
                pf_pe = is_pml_e(r, ny, d.n_pml) ? pe_in[(size_t)psi_row(r, ny, d.n_pml) * pitch + col] : 0.f;
                pf_ph = is_pml_h(r, ny, d.n_pml) ? ph_in[(size_t)psi_row(r, ny, d.n_pml) * pitch + col] : 0.f;
            }
        } else {
            pf_e = pf_hx = pf_hy = pf_pe = pf_ph = 0.f;
            pf_lab = 0;
        }
    };
    fetch(r_begin);

    auto iteration = [&](int r, auto P_) {
        constexpr int P = decltype(P_)::value;
        // level 0: row r enters the pipeline
        {
            const float2 cf = coef_lds[pf_lab];
            S[0][P] = Slot{pf_e, pf_hx, pf_hy, cf.x, cf.y, pf_pe, pf_ph};
        }
        fetch(r + 1);
#pragma unroll
        for (int t = 1; t <= K; ++t) {
            const int j = r - t;
            if (j < 0) continue;
            if (j >= ny) {
                S[t][P] = Slot{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                continue;
            }
            const Slot pv = S[t - 1][P ^ 1];     // level t-1, row j
            const float hx_up = S[t - 1][P].hx;  // level t-1, row j+1
            const float e_below = S[t][P ^ 1].e; // level t, row j-1
            const int n = n0 + t - 1;
            const float2 inc = d.inc[n];
            // E
            const bool pml_e = PML && is_pml_e(j, ny, d.n_pml);
            float pe = pv.pe;
            float4 pre = make_float4(0.f, 0.f, 1.f, 0.f);
            if (pml_e) pre = d.prof_e[j];
            const float hy_r = from_right(pv.hy);
            const float e_new = upd_e(pv.e, pv.ce, pv.cb, pv.hy, hy_r, pv.hx, hx_up, pml_e, pre, pe, j == d.j_src, inc.y);
            // Hx
            float hx_new = pv.hx;
            float ph = pv.ph;
            if (j > 0) {
                const bool pml_h = PML && is_pml_h(j, ny, d.n_pml);
                float4 prh = make_float4(0.f, 0.f, 1.f, 0.f);
                if (pml_h) prh = d.prof_h[j];
                hx_new = upd_hx(pv.hx, e_new, e_below, d.s1, pml_h, prh, ph, j == d.j_src + 1, inc.x);
            }
            // Hy
            const float e_left = from_left(e_new);
            const float hy_new = upd_hy(pv.hy, e_new, e_left, d.s1);
            S[t][P] = Slot{e_new, hx_new, hy_new, pv.ce, pv.cb, pe, ph};

            const bool owned = (j >= w.j0) && (j < w.j1);
            if (owned && n >= d.dft_start && (j == d.j_ref || j == d.j_trn) && valid_col)
                monitor_add(d, j == d.j_ref ? 0 : 1, col, e_new, d.phasor[n]);
            if (t == K && owned && valid_col) {
                const size_t o = (size_t)j * pitch + col;
                ez_out[o] = e_new;
                hx_out[o] = hx_new;
                hy_out[o] = hy_new;
                if (PML) {
                    if (is_pml_e(j, ny, d.n_pml)) pe_out[(size_t)psi_row(j, ny, d.n_pml) * pitch + col] = pe;
                    if (is_pml_h(j, ny, d.n_pml)) ph_out[(size_t)psi_row(j, ny, d.n_pml) * pitch + col] = ph;
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

template <int K>
__global__ __launch_bounds__(256) void k_tblock(const InstDev* __restrict__ insts, const WorkItem* __restrict__ items,
                                                int n_items, int n0, int cur) {
    __shared__ float2 coef_lds[4][kMaxLabels];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    // XCD-aware order: consecutive workgroups land on different XCDs, so give
    // each XCD a contiguous run of work items (neighbouring strips and bands,
    // whose halos then hit in the same L2).
    const int nblk = gridDim.x;
    const int b = blockIdx.x;
    const int per_xcd = (nblk + 7) / 8;
    const int xcd = b % 8, local = b / 8;
    int blk = xcd * per_xcd + local;
    // with nblk not a multiple of 8 the remap is not a bijection on its tail;
    // fall back to the identity there
    if ((nblk & 7) != 0) blk = b;
    const int it = __builtin_amdgcn_readfirstlane(blk * 4 + wave);
    if (it >= n_items) return;
    const WorkItem w = items[it];
    const InstDev d = insts[w.inst];
    // Each wave stages its own instance's coefficient table in its own LDS
    // slice; LDS instructions of one wave execute in order, so only a
    // compiler-level barrier is needed before the lanes read each other's
    // entries.  (No workgroup barrier: waves past the end of the item list
    // have already returned.)
    for (int k = lane; k < d.n_labels; k += kWave) coef_lds[wave][k] = d.coef[k];
    __builtin_amdgcn_wave_barrier();
    if (w.pml)
        tblock_body<K, true>(d, w, n0, cur, lane, coef_lds[wave]);
    else
        tblock_body<K, false>(d, w, n0, cur, lane, coef_lds[wave]);
}

// ---------------------------------------------------------------------------
// Bloch projection of the monitor sums (eq. 31-32): for each (instance, line,
// order m), sum_i S_i exp(-2 pi i m i / nx) for the cosine and sine sums, in
// FP64.  One workgroup per request.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_project(const InstDev* __restrict__ insts, const ProjItem* __restrict__ items,
                                                 double* __restrict__ out) {
    __shared__ double red[4][4];
    const ProjItem q = items[blockIdx.x];
    const InstDev& d = insts[q.inst];
    const float* m = d.mon + (size_t)q.line * 4 * d.pitch;
    double cr = 0, ci = 0, sr = 0, si = 0;
    const long long mm = ((q.m % d.nx) + d.nx) % d.nx;
    for (int i = threadIdx.x; i < d.nx; i += 256) {
        const double vc = (double)m[i] - (double)m[d.pitch + i];
        const double vs = (double)m[2 * d.pitch + i] - (double)m[3 * d.pitch + i];
        const long long k = (mm * i) % d.nx;
        double sn, cs;
        sincospi(2.0 * (double)k / (double)d.nx, &sn, &cs);
        // exp(-i phi) = cos phi - i sin phi
        cr += vc * cs;
        ci -= vc * sn;
        sr += vs * cs;
        si -= vs * sn;
    }
    for (int off = 32; off > 0; off >>= 1) {
        cr += __shfl_down(cr, off);
        ci += __shfl_down(ci, off);
        sr += __shfl_down(sr, off);
        si += __shfl_down(si, off);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        red[wave][0] = cr;
        red[wave][1] = ci;
        red[wave][2] = sr;
        red[wave][3] = si;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const double v = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
        out[(size_t)blockIdx.x * 4 + threadIdx.x] = v;
    }
}

// ---------------------------------------------------------------------------
// Utilities
// ---------------------------------------------------------------------------

__global__ void k_fill(float* __restrict__ p, size_t n, float v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_i32(int* __restrict__ p, size_t n, int v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// Streaming copy, 16 B per lane, for measuring attainable HBM bandwidth.
__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from the host orchestration unit)
// ---------------------------------------------------------------------------

hipError_t launch_plain_step(const InstDev& d, int n, int cur, hipStream_t s) {
    dim3 grid((d.nx + 255) / 256, d.ny);
    k_plain_e<<<grid, 256, 0, s>>>(d, n, cur);
    k_plain_h<<<grid, 256, 0, s>>>(d, n, cur);
    return hipGetLastError();
}

hipError_t launch_tblock(int K, const InstDev* insts, const WorkItem* items, int n_items, int n0, int cur,
                         hipStream_t s) {
    const int blocks = (n_items + 3) / 4;
    switch (K) {
#define FDTD_TB_CASE(k)                                                      \
    case k:                                                                  \
        k_tblock<k><<<blocks, 256, 0, s>>>(insts, items, n_items, n0, cur); \
        break;
        FDTD_TB_CASE(1)
        FDTD_TB_CASE(2)
        FDTD_TB_CASE(3)
        FDTD_TB_CASE(4)
        FDTD_TB_CASE(5)
        FDTD_TB_CASE(6)
        FDTD_TB_CASE(7)
        FDTD_TB_CASE(8)
#undef FDTD_TB_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_project(const InstDev* insts, const ProjItem* items, int n_items, double* out, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    k_project<<<n_items, 256, 0, s>>>(insts, items, out);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, size_t n, float v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_fill<<<(unsigned)blocks, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, size_t n, int v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_fill_i32<<<(unsigned)blocks, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 16;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_copy<<<(unsigned)blocks, 256, 0, s>>>((const float4*)src, (float4*)dst, n);
    return hipGetLastError();
}

}  // namespace fdtd
