// gfx950 kernels of the FDTD path: plain per-step sweeps and the temporally
// blocked streaming kernel for TMz and for TEz, Bloch projection of the
// monitors, and small utility kernels.  All cell arithmetic goes through fdtd_device.h.
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

// Plain TEz sweeps (eqs. 14-16): the Hz launch, then the Ex/Ey launch, in
// place, one thread per cell.  Hz, Ex, Ey live in the ez, hx, hy arrays; the
// cell-row psi (dEx/dy term of Hz) in pe, the edge-row psi (dHz/dy term of
// Ex) in ph.  The monitors record Ex^{n+1} of the edge rows j_ref, j_trn.
__global__ __launch_bounds__(256) void k_plain_te_h(InstDev d, int n, int cur) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const size_t o = (size_t)j * d.pitch + i;
    const int ir = (i + 1 == d.nx) ? 0 : i + 1;
    const float ex_c = d.hx[cur][o];
    const float ex_u = (j + 1 < d.ny) ? d.hx[cur][o + d.pitch] : 0.0f;   // Ex = 0 on the top wall
    const float ey_c = d.hy[cur][o];
    const float ey_r = d.hy[cur][(size_t)j * d.pitch + ir];
    const bool pml = is_pml_e(j, d.ny, d.n_pml);
    float pc = 0.0f;
    float4 pr = make_float4(0.f, 0.f, 1.f, 0.f);
    size_t po = 0;
    if (pml) {
        po = (size_t)psi_row(j, d.ny, d.n_pml) * d.pitch + i;
        pc = d.pe[cur][po];
        pr = d.prof_e[j];
    }
    d.ez[cur][o] = upd_hz(d.ez[cur][o], ey_c, ey_r, ex_c, ex_u, d.s1, pml, pr, pc, j == d.j_src, d.inc[n].y);
    if (pml) d.pe[cur][po] = pc;
}

__global__ __launch_bounds__(256) void k_plain_te_e(InstDev d, int n, int cur) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const size_t o = (size_t)j * d.pitch + i;
    const float* hz = d.ez[cur];
    const int la = d.lab[o];
    if (j > 0) {
        const float2 cf = d.coef[pair_index(d.lab[o - d.pitch], la)];
        const bool pml = is_pml_h(j, d.ny, d.n_pml);
        float pe = 0.0f;
        float4 pr = make_float4(0.f, 0.f, 1.f, 0.f);
        size_t po = 0;
        if (pml) {
            po = (size_t)psi_row(j, d.ny, d.n_pml) * d.pitch + i;
            pe = d.ph[cur][po];
            pr = d.prof_h[j];
        }
        const float ex = upd_ex(d.hx[cur][o], cf.x, cf.y, hz[o], hz[o - d.pitch], pml, pr, pe, j == d.j_src + 1,
                                d.inc[n].x);
        d.hx[cur][o] = ex;
        if (pml) d.ph[cur][po] = pe;
        if (n >= d.dft_start) {
            if (j == d.j_ref) monitor_add(d, 0, i, ex, d.phasor[n]);
            if (j == d.j_trn) monitor_add(d, 1, i, ex, d.phasor[n]);
        }
    }
    const int il = (i == 0) ? d.nx - 1 : i - 1;
    const size_t ol = (size_t)j * d.pitch + il;
    const float2 cy = d.coef[pair_index(d.lab[ol], la)];
    d.hy[cur][o] = upd_ey(d.hy[cur][o], cy.x, cy.y, hz[o], hz[ol]);
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

// Rows [j0, j1) of a work item, K steps.  SPECIAL items (thin bands near the
// absorbing layers, the TF/SF line and the monitor rows) run the full update
// on every row, with the row table above; all other items run a branch-free
// pipeline without layers, sources or monitors.
//
// Register layout: level 0 is a two-slot ring of raw rows straight from
// memory (l_*[r & 1] holds row r); levels 1..K keep two computed row slots
// each (S[t][r & 1]).  Row r + 1 is loaded into the ring slot that row r - 1
// leaves once level 1 has copied it out, so every load writes the register
// the loop carries and no in-flight load is ever copied (a copy would stall
// the wave until the load returns).
//
// REC (the adjoint's forward replay) also writes Ez^{n+1/2} of every level's
// owned cells to history slot hslot0 + t - 1 (hslot0: the slot of step n0).
template <int K, bool SPECIAL, bool REC>
__device__ __forceinline__ void tblock_band(const InstDev& dref, const WorkItem& w, int n0, int cur, int hslot0,
                                            int lane, const float2* __restrict__ coef_lds,
                                            const SpecialLds* __restrict__ sp) {
    // Descriptor fields in registers: the stores below could alias the
    // descriptor as far as the compiler knows, which would otherwise make it
    // reload every field after every store.
    const int nx = dref.nx, ny = dref.ny, pitch = dref.pitch;
    const float s1 = dref.s1;
    const int n_pml = SPECIAL ? dref.n_pml : 0;
    const int j_ref = dref.j_ref, j_trn = dref.j_trn, dft_start = dref.dft_start;
    const unsigned off_pe = dref.off_pe, off_ph = dref.off_ph, set_bytes = dref.set_bytes;
    float* const mon = dref.mon;
    int* const status = dref.status;
    float* const hist = dref.hist;
    const size_t plane = (size_t)ny * pitch;
    const unsigned rowb = (unsigned)pitch * 4u;
    const unsigned plane_b = (unsigned)ny * rowb;
    int col = w.x0 - K + lane;
    col %= nx;
    if (col < 0) col += nx;
    const bool valid_col = (lane >= K) && (lane < kWave - K) && (w.x0 + lane - K < nx);
    const bool c1 = cur != 0;
    const __amdgpu_buffer_rsrc_t rin = make_rsrc(c1 ? dref.ez[1] : dref.ez[0], set_bytes);
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(c1 ? dref.ez[0] : dref.ez[1], set_bytes);
    const __amdgpu_buffer_rsrc_t rlab = make_rsrc(dref.lab, (unsigned)ny * (unsigned)pitch);
    const unsigned vo = (unsigned)col * 4u, vl = (unsigned)col;
    const unsigned ohx = dref.off_hx, ohy = dref.off_hy;

    // Monitor rows owned by this item: Ez of the row at every level is
    // captured in registers and added to the Kahan sums after the sweep, in
    // step order.
    const bool own_ref = SPECIAL && w.j0 <= j_ref && j_ref < w.j1;
    const bool own_trn = SPECIAL && w.j0 <= j_trn && j_trn < w.j1;
    float cap_r[K + 1], cap_t[K + 1];
#pragma unroll
    for (int t = 0; t <= K; ++t) cap_r[t] = cap_t[t] = 0.f;

    Slot S[K + 1][2];  // S[0] unused: level 0 lives in the load ring
#pragma unroll
    for (int t = 0; t <= K; ++t)
#pragma unroll
        for (int p = 0; p < 2; ++p) S[t][p] = Slot{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

    const int r_begin = SPECIAL ? max(0, w.j0 - K) : w.j0 - K;
    const int r_end = w.j1 + K;

    float l_e[2], l_hx[2], l_hy[2], l_pe[2], l_ph[2];
    int l_lab[2];
    auto fetch = [&](int r, int q) {
        // rows past the top are read from row ny - 1 (in bounds); their values
        // never reach a row of the domain (Hx above the top row is forced to 0)
        const int rr = min(r, ny - 1);
        const unsigned so = (unsigned)rr * rowb;
        l_e[q] = buf_ld(rin, vo, so);
        l_hx[q] = buf_ld(rin, vo, so + ohx);
        l_hy[q] = buf_ld(rin, vo, so + ohy);
        l_lab[q] = buf_ld_u8(rlab, vl, (unsigned)rr * (unsigned)pitch);
        if (SPECIAL) {
            // the spare psi row stands in for rows outside the layers; the
            // value read there is finite and multiplied by a zero profile
            l_pe[q] = buf_ld(rin, vo, off_pe + (unsigned)psi_slot_e(rr, ny, n_pml) * rowb);
            l_ph[q] = buf_ld(rin, vo, off_ph + (unsigned)psi_slot_h(rr, ny, n_pml) * rowb);
        } else {
            l_pe[q] = l_ph[q] = 0.f;
        }
    };
    l_e[1] = l_hx[1] = l_hy[1] = l_pe[1] = l_ph[1] = 0.f;
    l_lab[1] = 0;
    fetch(r_begin, 0);

    auto iteration = [&](int r, auto P_) {
        constexpr int P = decltype(P_)::value;
        const RowTab* const rt = SPECIAL ? sp->rows + (r - r_begin) : nullptr;
#pragma unroll
        for (int t = 1; t <= K; ++t) {
            // In special bands some levels run on rows outside the domain
            // (j < 0 at the bottom, j >= ny at the top).  Their values never
            // reach a domain row: Hx(0) is never updated, and Hx above the top
            // row is taken as 0.
            const int j = r - t;
            Slot pv;        // level t-1, row j
            float hx_up;    // level t-1, row j+1
            if (t == 1) {
                // copy the ring slot of row r - 1, then reuse it for row r + 1
                // (the copies keep the arithmetic, whose accumulating
                // instructions overwrite an operand, out of the load targets)
                const float2 cf = coef_lds[l_lab[P ^ 1]];
                pv = Slot{vcopy(l_e[P ^ 1]), vcopy(l_hx[P ^ 1]), vcopy(l_hy[P ^ 1]), cf.x, cf.y,
                          SPECIAL ? vcopy(l_pe[P ^ 1]) : 0.f, SPECIAL ? vcopy(l_ph[P ^ 1]) : 0.f};
                hx_up = l_hx[P];
                fetch(r + 1, P ^ 1);
            } else {
                pv = S[t - 1][P ^ 1];
                hx_up = S[t - 1][P].hx;
            }
            if (SPECIAL) hx_up = (j + 1 < ny) ? hx_up : 0.f;   // magnetic wall above the top row
            const float e_below = S[t][P ^ 1].e;  // level t, row j-1
            const float hy_r = from_right(pv.hy);
            float pe = pv.pe, ph = pv.ph;
            float e_new, hx_new;
            const float4 none = make_float4(0.f, 0.f, 1.f, 0.f);
            if (SPECIAL) {
                // Branch-free form of upd_e/upd_hx: rows outside the layers read
                // the neutral profile (b = c = 0, 1/kappa = 1) and rows off the
                // TF/SF line a zero source flag, which reproduces the plain
                // update exactly (up to the sign of an exact zero, which no
                // later add, mul or fma can turn into a nonzero value).
                const float2 inc = sp->inc[t - 1];
                const float4 pre = rt[K - t].e;
                const float4 prh = rt[K - t].h;
                const float dhx = hx_up - pv.hx;
                const float dhy = hy_r - pv.hy;
                pe = __fmaf_rn(pre.x, pe, pre.y * dhx);
                const float te = __fmaf_rn(dhx, pre.z, pe) + pre.w * inc.y;
                e_new = __fmaf_rn(pv.ce, pv.e, pv.cb * (dhy - te));
                const float de = e_new - e_below;
                ph = __fmaf_rn(prh.x, ph, prh.y * de);
                const float th = __fmaf_rn(de, prh.z, ph) + prh.w * inc.x;
                hx_new = (j > 0) ? __fmaf_rn(-s1, th, pv.hx) : pv.hx;   // Hx(0) is the wall
                cap_r[t] = (j == j_ref) ? e_new : cap_r[t];
                cap_t[t] = (j == j_trn) ? e_new : cap_t[t];
            } else {
                e_new = upd_e(pv.e, pv.ce, pv.cb, pv.hy, hy_r, pv.hx, hx_up, false, none, pe, false, 0.f);
                hx_new = upd_hx(pv.hx, e_new, e_below, s1, false, none, ph, false, 0.f);
            }
            const float e_left = from_left(e_new);
            const float hy_new = upd_hy(pv.hy, e_new, e_left, s1);
            S[t][P] = Slot{e_new, hx_new, hy_new, pv.ce, pv.cb, pe, ph};
            if (REC) {
                // history slot of this level's step: a resource per slot (a
                // whole segment can exceed 32-bit offsets)
                const __amdgpu_buffer_rsrc_t rh = make_rsrc(hist + (size_t)(hslot0 + t - 1) * plane, plane_b);
                const unsigned vh = (j >= w.j0 && j < w.j1 && valid_col) ? vo : kDropOffset;
                buf_st(rh, vh, (unsigned)j * rowb, e_new);
            }
            if (t == K) {
                // owned cells only
                const bool owned = SPECIAL ? (j >= w.j0 && j < w.j1) : (j >= w.j0);
                const unsigned so = (unsigned)j * rowb;
                if (!SPECIAL && !REC) {
                    // the bulk kernel keeps a masked store: with it the
                    // compiler fits the pipeline in 72 VGPRs (7 waves per SIMD),
                    // which measures faster than the branch-free form
                    if (owned && valid_col) {
                        buf_st(rout, vo, so, e_new);
                        buf_st(rout, vo, so + ohx, hx_new);
                        buf_st(rout, vo, so + ohy, hy_new);
                    }
                } else {
                    // other lanes and rows are dropped (no branch)
                    const unsigned vs = (owned && valid_col) ? vo : kDropOffset;
                    buf_st(rout, vs, so, e_new);
                    buf_st(rout, vs, so + ohx, hx_new);
                    buf_st(rout, vs, so + ohy, hy_new);
                    if (SPECIAL) {
                        buf_st(rout, vs, off_pe + (unsigned)psi_slot_e(j, ny, n_pml) * rowb, pe);
                        buf_st(rout, vs, off_ph + (unsigned)psi_slot_h(j, ny, n_pml) * rowb, ph);
                    }
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

    if (SPECIAL) {
        // Kahan sums of the owned monitor rows, in step order
        auto accumulate = [&](float* m, const float (&cap)[K + 1]) {
            float a0 = gld(m, col), a1 = gld(m, pitch + col), a2 = gld(m, 2 * pitch + col), a3 = gld(m, 3 * pitch + col);
#pragma unroll
            for (int t = 1; t <= K; ++t) {
                if (n0 + t - 1 >= dft_start) {
                    const float2 phs = sp->phasor[t - 1];
                    kahan_add(a0, a1, cap[t] * phs.x);
                    kahan_add(a2, a3, cap[t] * phs.y);
                }
            }
            if (valid_col) {
                gst(m, col, a0);
                gst(m, pitch + col, a1);
                gst(m, 2 * pitch + col, a2);
                gst(m, 3 * pitch + col, a3);
                if (!__builtin_isfinite(a0) || !__builtin_isfinite(a2)) gst_i32(status, 1);
            }
        };
        if (own_ref) accumulate(mon, cap_r);
        if (own_trn) accumulate(mon + (size_t)4 * pitch, cap_t);
    }
}

template <int K, bool SPECIAL, bool REC>
__global__ __launch_bounds__(256) void k_tblock(const InstDev* __restrict__ insts, const WorkItem* __restrict__ items,
                                                int n_items, int n0, int cur, int hslot0) {
    __shared__ float2 coef_lds[4][kMaxLabels];
    __shared__ SpecialLds sp_lds[SPECIAL ? 4 : 1];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int it = xcd_item(wave);
    if (it >= n_items) return;
    const WorkItem w = items[it];
    const InstDev* __restrict__ dp = insts + w.inst;
    SpecialLds* sp = &sp_lds[SPECIAL ? wave : 0];
    if (SPECIAL) {
        stage_rows(dp, w, K, sp->rows, lane);
        if (lane < K) {
            sp->inc[lane] = dp->inc[n0 + lane];
            sp->phasor[lane] = dp->phasor[n0 + lane];
        }
    }
    stage_coef(dp, coef_lds[wave], lane);
    tblock_band<K, SPECIAL, REC>(*dp, w, n0, cur, hslot0, lane, coef_lds[wave], sp);
}

// ---------------------------------------------------------------------------
// Bulk TMz items as workgroup items.  The four waves of a workgroup take 256
// consecutive columns [x0 - K, x0 - K + 256) (periodic) of one band and walk
// its rows together, each wave 64 of them as in tblock_band.  A row
// iteration runs in two phases: Ez and Hx of every level, whose one x
// neighbour, Hy(i+1), lane 63 takes from the wave on its right; then Hy of
// every level, whose Ez(i-1) lane 0 takes from the wave on its left.  Those
// edge values cross through LDS, each crossing behind a workgroup barrier,
// so that only the workgroup's outer K columns on each side are recomputed
// halo: 256 - 2K columns owned per 256 computed, where a wave that
// recomputes its own halo owns 64 - 2K of 64.  The phases reorder no
// arithmetic: every value is the one tblock_band computes.
// ---------------------------------------------------------------------------

constexpr int kWgWaves = 4;
constexpr int kWgCols = kWgWaves * kWave;
static_assert(kWgCols == kWgColumns, "the host lays bulk TMz items out kWgColumns wide");

// value of lane l+1 (l-1), the end lane taking `edge` instead
__device__ __forceinline__ float from_right_or(float v, float edge) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                                 __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_left_or(float v, float edge) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                                 __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}

// The exchange slots first: their addresses then fit the immediate offsets of
// the LDS instructions.
struct WgLds {
    float hy[kWgWaves][kMaxTBlock];      // lane 0's Hy of levels 0..K-1, for the wave on the left
    float e[kWgWaves][kMaxTBlock + 1];   // lane 63's Ez of levels 1..K, for the wave on the right
    float2 coef[kMaxLabels];             // the instance's (Ce, Cb)
};

// A workgroup barrier that orders LDS accesses only: the global loads in
// flight (the next rows) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int K, bool REC>
__device__ __forceinline__ void tblock_band_wg(const InstDev& dref, const WorkItem& w, int n0, int cur, int hslot0,
                                               int wave, int lane, WgLds* __restrict__ lds) {
    const int nx = dref.nx, ny = dref.ny, pitch = dref.pitch;
    const float s1 = dref.s1;
    const unsigned set_bytes = dref.set_bytes;
    float* const hist = dref.hist;
    const size_t plane = (size_t)ny * pitch;
    const unsigned rowb = (unsigned)pitch * 4u;
    const unsigned plane_b = (unsigned)ny * rowb;
    const int g = wave * kWave + lane;   // column of the workgroup
    int col = w.x0 - K + g;
    col %= nx;
    if (col < 0) col += nx;
    const bool valid_col = (g >= K) && (g < kWgCols - K) && (w.x0 + g - K < nx);
    const bool c1 = cur != 0;
    const __amdgpu_buffer_rsrc_t rin = make_rsrc(c1 ? dref.ez[1] : dref.ez[0], set_bytes);
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(c1 ? dref.ez[0] : dref.ez[1], set_bytes);
    const __amdgpu_buffer_rsrc_t rlab = make_rsrc(dref.lab, (unsigned)ny * (unsigned)pitch);
    const unsigned vo = (unsigned)col * 4u, vl = (unsigned)col;
    const unsigned ohx = dref.off_hx, ohy = dref.off_hy;
    const float2* __restrict__ coef = lds->coef;
    // the neighbours' edge values (the outer waves read their own: their end
    // lanes are halo)
    const float* xhy_r = lds->hy[wave + 1 < kWgWaves ? wave + 1 : wave];
    const float* xe_l = lds->e[wave > 0 ? wave - 1 : wave];
    float* const xhy_w = lds->hy[wave];
    float* const xe_w = lds->e[wave];

    Slot S[K + 1][2];  // S[0] unused: level 0 lives in the load ring
#pragma unroll
    for (int t = 0; t <= K; ++t)
#pragma unroll
        for (int p = 0; p < 2; ++p) S[t][p] = Slot{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

    const int r_begin = w.j0 - K;
    const int r_end = w.j1 + K;

    float l_e[2], l_hx[2], l_hy[2];
    int l_lab[2];
    auto fetch = [&](int r, int q) {
        const int rr = min(r, ny - 1);
        const unsigned so = (unsigned)rr * rowb;
        l_e[q] = buf_ld(rin, vo, so);
        l_hx[q] = buf_ld(rin, vo, so + ohx);
        l_hy[q] = buf_ld(rin, vo, so + ohy);
        l_lab[q] = buf_ld_u8(rlab, vl, (unsigned)rr * (unsigned)pitch);
    };
    l_e[1] = l_hx[1] = l_hy[1] = 0.f;
    l_lab[1] = 0;
    fetch(r_begin, 0);

    const float4 none = make_float4(0.f, 0.f, 1.f, 0.f);
    auto iteration = [&](int r, auto P_) {
        constexpr int P = decltype(P_)::value;
        float hy0;   // Hy of level 0 (row r - 1), for the Hy phase
        // Ez and Hx of every level
#pragma unroll
        for (int t = 1; t <= K; ++t) {
            const int j = r - t;
            Slot pv;        // level t-1, row j
            float hx_up;    // level t-1, row j+1
            if (t == 1) {
                const float2 cf = coef[l_lab[P ^ 1]];
                pv = Slot{vcopy(l_e[P ^ 1]), vcopy(l_hx[P ^ 1]), vcopy(l_hy[P ^ 1]), cf.x, cf.y, 0.f, 0.f};
                hy0 = pv.hy;
                hx_up = l_hx[P];
                fetch(r + 1, P ^ 1);
            } else {
                pv = S[t - 1][P ^ 1];
                hx_up = S[t - 1][P].hx;
            }
            const float e_below = S[t][P ^ 1].e;  // level t, row j-1
            const float hy_r = from_right_or(pv.hy, xhy_r[t - 1]);
            float pe = 0.f, ph = 0.f;
            const float e_new = upd_e(pv.e, pv.ce, pv.cb, pv.hy, hy_r, pv.hx, hx_up, false, none, pe, false, 0.f);
            const float hx_new = upd_hx(pv.hx, e_new, e_below, s1, false, none, ph, false, 0.f);
            S[t][P].e = e_new;
            S[t][P].hx = hx_new;
            S[t][P].ce = pv.ce;
            S[t][P].cb = pv.cb;
            if (REC) {
                const __amdgpu_buffer_rsrc_t rh = make_rsrc(hist + (size_t)(hslot0 + t - 1) * plane, plane_b);
                const unsigned vh = (j >= w.j0 && j < w.j1 && valid_col) ? vo : kDropOffset;
                buf_st(rh, vh, (unsigned)j * rowb, e_new);
            }
        }
        if (lane == kWave - 1) {
#pragma unroll
            for (int t = 1; t <= K; ++t) xe_w[t] = S[t][P].e;
        }
        lds_barrier();
        // Hy of every level
#pragma unroll
        for (int t = 1; t <= K; ++t) {
            const int j = r - t;
            const float hy_old = (t == 1) ? hy0 : S[t - 1][P ^ 1].hy;
            const float e_c = S[t][P].e;
            const float e_left = from_left_or(e_c, xe_l[t]);
            const float hy_new = upd_hy(hy_old, e_c, e_left, s1);
            S[t][P].hy = hy_new;
            if (t == K && j >= w.j0 && valid_col) {
                const unsigned so = (unsigned)j * rowb;
                buf_st(rout, vo, so, e_c);
                buf_st(rout, vo, so + ohx, S[t][P].hx);
                buf_st(rout, vo, so + ohy, hy_new);
            }
        }
        // Hy of levels 0..K-1 at this row, which the next iteration's Ez
        // phase reads one level up (level 0: the row just read)
        if (lane == 0) {
            xhy_w[0] = l_hy[P];
#pragma unroll
            for (int t = 2; t <= K; ++t) xhy_w[t - 1] = S[t - 1][P].hy;
        }
        lds_barrier();
    };

    int r = r_begin;
    for (; r + 1 < r_end; r += 2) {
        iteration(r, std::integral_constant<int, 0>{});
        iteration(r + 1, std::integral_constant<int, 1>{});
    }
    if (r < r_end) iteration(r, std::integral_constant<int, 0>{});
}

// One workgroup per item; the XCD remap of xcd_item at workgroup level.
template <int K, bool REC>
__global__ __launch_bounds__(256) void k_tblock_wg(const InstDev* __restrict__ insts,
                                                   const WorkItem* __restrict__ items, int n_items, int n0, int cur,
                                                   int hslot0) {
    __shared__ WgLds lds;
    const int per_xcd = gridDim.x >> 3;
    const int it = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (it >= n_items) return;   // the whole workgroup
    const WorkItem w = items[it];
    const InstDev* __restrict__ dp = insts + w.inst;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (int k = threadIdx.x; k < dp->n_coef; k += kWgCols) lds.coef[k] = dp->coef[k];
    if (threadIdx.x < kWgWaves * kMaxTBlock) (&lds.hy[0][0])[threadIdx.x] = 0.f;
    __syncthreads();
    tblock_band_wg<K, REC>(*dp, w, n0, cur, hslot0, wave, lane, &lds);
}

// ---------------------------------------------------------------------------
// Streaming kernel for TEz.  The pipeline of tblock_band with the TEz updates:
// level t advances Hz of row r - t (from Ex, Ey of the level below, rows j
// and j + 1, and Ey of the lane to the right), then Ex of that row (from the
// new Hz of rows j and j - 1) and Ey (from the new Hz of the lane to the
// left).  The per-edge coefficients of a cell depend on its label and on the
// labels of the cells below and to the left; level 1 looks them up once per
// row in the pair table and every level carries them with the row.
// ---------------------------------------------------------------------------

struct SlotTE {
    float hz, ex, ey, cex, cbx, cey, cby, pc, pe;
};

template <int K, bool SPECIAL>
__device__ __forceinline__ void tblock_band_te(const InstDev& dref, const WorkItem& w, int n0, int cur, int lane,
                                               const float2* __restrict__ coef_lds,
                                               const SpecialLds* __restrict__ sp) {
    const int nx = dref.nx, ny = dref.ny, pitch = dref.pitch;
    const float s1 = dref.s1;
    const int n_pml = SPECIAL ? dref.n_pml : 0;
    const int j_ref = dref.j_ref, j_trn = dref.j_trn, dft_start = dref.dft_start;
    const unsigned off_pe = dref.off_pe, off_ph = dref.off_ph, set_bytes = dref.set_bytes;
    float* const mon = dref.mon;
    int* const status = dref.status;
    const unsigned rowb = (unsigned)pitch * 4u;
    int col = w.x0 - K + lane;
    col %= nx;
    if (col < 0) col += nx;
    const bool valid_col = (lane >= K) && (lane < kWave - K) && (w.x0 + lane - K < nx);
    const bool c1 = cur != 0;
    const __amdgpu_buffer_rsrc_t rin = make_rsrc(c1 ? dref.ez[1] : dref.ez[0], set_bytes);
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(c1 ? dref.ez[0] : dref.ez[1], set_bytes);
    const __amdgpu_buffer_rsrc_t rlab = make_rsrc(dref.lab, (unsigned)ny * (unsigned)pitch);
    const unsigned vo = (unsigned)col * 4u, vl = (unsigned)col;
    const unsigned ohx = dref.off_hx, ohy = dref.off_hy;

    const bool own_ref = SPECIAL && w.j0 <= j_ref && j_ref < w.j1;
    const bool own_trn = SPECIAL && w.j0 <= j_trn && j_trn < w.j1;
    float cap_r[K + 1], cap_t[K + 1];
#pragma unroll
    for (int t = 0; t <= K; ++t) cap_r[t] = cap_t[t] = 0.f;

    SlotTE S[K + 1][2];
#pragma unroll
    for (int t = 0; t <= K; ++t)
#pragma unroll
        for (int p = 0; p < 2; ++p) S[t][p] = SlotTE{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

    const int r_begin = SPECIAL ? max(0, w.j0 - K) : w.j0 - K;
    const int r_end = w.j1 + K;

    float l_hz[2], l_ex[2], l_ey[2], l_pc[2], l_pe[2];
    int l_lab[2];
    auto fetch = [&](int r, int q) {
        const int rr = min(r, ny - 1);
        const unsigned so = (unsigned)rr * rowb;
        l_hz[q] = buf_ld(rin, vo, so);
        l_ex[q] = buf_ld(rin, vo, so + ohx);
        l_ey[q] = buf_ld(rin, vo, so + ohy);
        l_lab[q] = buf_ld_u8(rlab, vl, (unsigned)rr * (unsigned)pitch);
        if (SPECIAL) {
            l_pc[q] = buf_ld(rin, vo, off_pe + (unsigned)psi_slot_e(rr, ny, n_pml) * rowb);
            l_pe[q] = buf_ld(rin, vo, off_ph + (unsigned)psi_slot_h(rr, ny, n_pml) * rowb);
        } else {
            l_pc[q] = l_pe[q] = 0.f;
        }
    };
    l_hz[1] = l_ex[1] = l_ey[1] = l_pc[1] = l_pe[1] = 0.f;
    l_lab[1] = 0;
    fetch(r_begin, 0);
    int lab_prev[2] = {0, 0};   // label of the row level 1 handled on the last even / odd iteration

    auto iteration = [&](int r, auto P_) {
        constexpr int P = decltype(P_)::value;
        const RowTab* const rt = SPECIAL ? sp->rows + (r - r_begin) : nullptr;
#pragma unroll
        for (int t = 1; t <= K; ++t) {
            const int j = r - t;
            SlotTE pv;       // level t-1, row j
            float ex_up;     // level t-1, row j+1
            if (t == 1) {
                const int la = vcopy_i(l_lab[P ^ 1]);
                const int lb = lab_prev[P ^ 1];          // row j - 1
                const int ll = from_left_i(la);           // row j, column i - 1
                lab_prev[P] = la;
                const float2 cx = coef_lds[pair_index(lb, la)];
                const float2 cy = coef_lds[pair_index(ll, la)];
                pv = SlotTE{vcopy(l_hz[P ^ 1]), vcopy(l_ex[P ^ 1]), vcopy(l_ey[P ^ 1]), cx.x, cx.y, cy.x, cy.y,
                            SPECIAL ? vcopy(l_pc[P ^ 1]) : 0.f, SPECIAL ? vcopy(l_pe[P ^ 1]) : 0.f};
                ex_up = l_ex[P];
                fetch(r + 1, P ^ 1);
            } else {
                pv = S[t - 1][P ^ 1];
                ex_up = S[t - 1][P].ex;
            }
            if (SPECIAL) ex_up = (j + 1 < ny) ? ex_up : 0.f;   // electric wall above the top row
            const float hz_below = S[t][P ^ 1].hz;          // level t, row j-1
            const float ey_r = from_right(pv.ey);
            float pc = pv.pc, pe = pv.pe;
            float hz_new, ex_new;
            const float4 none = make_float4(0.f, 0.f, 1.f, 0.f);
            if (SPECIAL) {
                // branch-free upd_hz/upd_ex: neutral profiles outside the layers,
                // zero TF/SF flags off the source rows (exact up to the sign of
                // an exact zero)
                const float2 inc = sp->inc[t - 1];
                const float4 prc = rt[K - t].e;
                const float4 pre = rt[K - t].h;
                const float dex = ex_up - pv.ex;
                const float dey = ey_r - pv.ey;
                pc = __fmaf_rn(prc.x, pc, prc.y * dex);
                const float tc = __fmaf_rn(dex, prc.z, pc) + prc.w * inc.y;
                hz_new = __fmaf_rn(-s1, dey - tc, pv.hz);
                const float dh = hz_new - hz_below;
                pe = __fmaf_rn(pre.x, pe, pre.y * dh);
                const float te = __fmaf_rn(dh, pre.z, pe) + pre.w * inc.x;
                ex_new = (j > 0) ? __fmaf_rn(pv.cex, pv.ex, pv.cbx * te) : pv.ex;   // Ex(0) is the wall
                cap_r[t] = (j == j_ref) ? ex_new : cap_r[t];
                cap_t[t] = (j == j_trn) ? ex_new : cap_t[t];
            } else {
                hz_new = upd_hz(pv.hz, pv.ey, ey_r, pv.ex, ex_up, s1, false, none, pc, false, 0.f);
                ex_new = upd_ex(pv.ex, pv.cex, pv.cbx, hz_new, hz_below, false, none, pe, false, 0.f);
            }
            const float hz_left = from_left(hz_new);
            const float ey_new = upd_ey(pv.ey, pv.cey, pv.cby, hz_new, hz_left);
            S[t][P] = SlotTE{hz_new, ex_new, ey_new, pv.cex, pv.cbx, pv.cey, pv.cby, pc, pe};
            if (t == K) {
                const bool owned = SPECIAL ? (j >= w.j0 && j < w.j1) : (j >= w.j0);
                const unsigned vs = (owned && valid_col) ? vo : kDropOffset;
                const unsigned so = (unsigned)j * rowb;
                buf_st(rout, vs, so, hz_new);
                buf_st(rout, vs, so + ohx, ex_new);
                buf_st(rout, vs, so + ohy, ey_new);
                if (SPECIAL) {
                    buf_st(rout, vs, off_pe + (unsigned)psi_slot_e(j, ny, n_pml) * rowb, pc);
                    buf_st(rout, vs, off_ph + (unsigned)psi_slot_h(j, ny, n_pml) * rowb, pe);
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

    if (SPECIAL) {
        auto accumulate = [&](float* m, const float (&cap)[K + 1]) {
            float a0 = gld(m, col), a1 = gld(m, pitch + col), a2 = gld(m, 2 * pitch + col), a3 = gld(m, 3 * pitch + col);
#pragma unroll
            for (int t = 1; t <= K; ++t) {
                if (n0 + t - 1 >= dft_start) {
                    const float2 phs = sp->phasor[t - 1];
                    kahan_add(a0, a1, cap[t] * phs.x);
                    kahan_add(a2, a3, cap[t] * phs.y);
                }
            }
            if (valid_col) {
                gst(m, col, a0);
                gst(m, pitch + col, a1);
                gst(m, 2 * pitch + col, a2);
                gst(m, 3 * pitch + col, a3);
                if (!__builtin_isfinite(a0) || !__builtin_isfinite(a2)) gst_i32(status, 1);
            }
        };
        if (own_ref) accumulate(mon, cap_r);
        if (own_trn) accumulate(mon + (size_t)4 * pitch, cap_t);
    }
}

template <int K, bool SPECIAL>
__global__ __launch_bounds__(256) void k_tblock_te(const InstDev* __restrict__ insts,
                                                   const WorkItem* __restrict__ items, int n_items, int n0, int cur) {
    // TEz special waves start only as bulk waves leave their SIMD (their
    // registers do not fit beside four bulk waves) and end after the bulk
    // kernel, so they set the launch period: give them issue priority
    if (SPECIAL) __builtin_amdgcn_s_setprio(3);
    __shared__ float2 coef_lds[4][kMaxLabels];
    __shared__ SpecialLds sp_lds[SPECIAL ? 4 : 1];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int it = xcd_item(wave);
    if (it >= n_items) return;
    const WorkItem w = items[it];
    const InstDev* __restrict__ dp = insts + w.inst;
    SpecialLds* sp = &sp_lds[SPECIAL ? wave : 0];
    if (SPECIAL) {
        stage_rows(dp, w, K, sp->rows, lane);
        if (lane < K) {
            sp->inc[lane] = dp->inc[n0 + lane];
            sp->phasor[lane] = dp->phasor[n0 + lane];
        }
    }
    stage_coef(dp, coef_lds[wave], lane);
    tblock_band_te<K, SPECIAL>(*dp, w, n0, cur, lane, coef_lds[wave], sp);
}

// ---------------------------------------------------------------------------
// Bulk TEz items as workgroup items: the scheme of tblock_band_wg with the
// TEz updates.  Phase one advances Hz (whose Ey(i+1) lane 63 takes from the
// wave on its right) and Ex of every level, phase two Ey (whose Hz(i-1) lane
// 0 takes from the wave on its left).  The label of the cell to the left,
// which selects the Ey edge's coefficients, crosses the same way once per row.
// ---------------------------------------------------------------------------

struct WgLdsTe {
    float ey[kWgWaves][kMaxTBlock];      // lane 0's Ey of levels 0..K-1, for the wave on the left
    float hz[kWgWaves][kMaxTBlock + 1];  // lane 63's Hz of levels 1..K, for the wave on the right
    int lab[kWgWaves];                   // lane 63's label of the row just read
    float2 coef[kPairTable];             // the instance's edge (Ce, Cb) pair table
};

__device__ __forceinline__ int from_left_or_i(int v, int edge) {
    return __builtin_amdgcn_update_dpp(edge, v, 0x138, 0xf, 0xf, false);
}

template <int K>
__device__ __forceinline__ void tblock_band_te_wg(const InstDev& dref, const WorkItem& w, int cur, int wave, int lane,
                                                  WgLdsTe* __restrict__ lds) {
    const int nx = dref.nx, ny = dref.ny, pitch = dref.pitch;
    const float s1 = dref.s1;
    const unsigned set_bytes = dref.set_bytes;
    const unsigned rowb = (unsigned)pitch * 4u;
    const int g = wave * kWave + lane;   // column of the workgroup
    int col = w.x0 - K + g;
    col %= nx;
    if (col < 0) col += nx;
    const bool valid_col = (g >= K) && (g < kWgCols - K) && (w.x0 + g - K < nx);
    const bool c1 = cur != 0;
    const __amdgpu_buffer_rsrc_t rin = make_rsrc(c1 ? dref.ez[1] : dref.ez[0], set_bytes);
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(c1 ? dref.ez[0] : dref.ez[1], set_bytes);
    const __amdgpu_buffer_rsrc_t rlab = make_rsrc(dref.lab, (unsigned)ny * (unsigned)pitch);
    const unsigned vo = (unsigned)col * 4u, vl = (unsigned)col;
    const unsigned ohx = dref.off_hx, ohy = dref.off_hy;
    const float2* __restrict__ coef = lds->coef;
    const int wr = wave + 1 < kWgWaves ? wave + 1 : wave, wl = wave > 0 ? wave - 1 : wave;
    const float* xey_r = lds->ey[wr];
    const float* xhz_l = lds->hz[wl];
    const int* xlab_l = &lds->lab[wl];
    float* const xey_w = lds->ey[wave];
    float* const xhz_w = lds->hz[wave];
    int* const xlab_w = &lds->lab[wave];

    SlotTE S[K + 1][2];
#pragma unroll
    for (int t = 0; t <= K; ++t)
#pragma unroll
        for (int p = 0; p < 2; ++p) S[t][p] = SlotTE{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

    const int r_begin = w.j0 - K;
    const int r_end = w.j1 + K;

    float l_hz[2], l_ex[2], l_ey[2];
    int l_lab[2];
    auto fetch = [&](int r, int q) {
        const int rr = min(r, ny - 1);
        const unsigned so = (unsigned)rr * rowb;
        l_hz[q] = buf_ld(rin, vo, so);
        l_ex[q] = buf_ld(rin, vo, so + ohx);
        l_ey[q] = buf_ld(rin, vo, so + ohy);
        l_lab[q] = buf_ld_u8(rlab, vl, (unsigned)rr * (unsigned)pitch);
    };
    l_hz[1] = l_ex[1] = l_ey[1] = 0.f;
    l_lab[1] = 0;
    fetch(r_begin, 0);
    int lab_prev[2] = {0, 0};   // label of the row level 1 handled on the last even / odd iteration

    const float4 none = make_float4(0.f, 0.f, 1.f, 0.f);
    auto iteration = [&](int r, auto P_) {
        constexpr int P = decltype(P_)::value;
        float ey0;   // Ey of level 0 (row r - 1), for the Ey phase
        // Hz and Ex of every level
#pragma unroll
        for (int t = 1; t <= K; ++t) {
            SlotTE pv;       // level t-1, row j
            float ex_up;     // level t-1, row j+1
            if (t == 1) {
                const int la = vcopy_i(l_lab[P ^ 1]);
                const int lb = lab_prev[P ^ 1];              // row j - 1
                const int ll = from_left_or_i(la, *xlab_l);   // row j, column i - 1
                lab_prev[P] = la;
                const float2 cx = coef[pair_index(lb, la)];
                const float2 cy = coef[pair_index(ll, la)];
                pv = SlotTE{vcopy(l_hz[P ^ 1]), vcopy(l_ex[P ^ 1]), vcopy(l_ey[P ^ 1]), cx.x, cx.y, cy.x, cy.y, 0.f, 0.f};
                ey0 = pv.ey;
                ex_up = l_ex[P];
                fetch(r + 1, P ^ 1);
            } else {
                pv = S[t - 1][P ^ 1];
                ex_up = S[t - 1][P].ex;
            }
            const float hz_below = S[t][P ^ 1].hz;          // level t, row j-1
            const float ey_r = from_right_or(pv.ey, xey_r[t - 1]);
            float pc = 0.f, pe = 0.f;
            const float hz_new = upd_hz(pv.hz, pv.ey, ey_r, pv.ex, ex_up, s1, false, none, pc, false, 0.f);
            const float ex_new = upd_ex(pv.ex, pv.cex, pv.cbx, hz_new, hz_below, false, none, pe, false, 0.f);
            S[t][P].hz = hz_new;
            S[t][P].ex = ex_new;
            S[t][P].cex = pv.cex;
            S[t][P].cbx = pv.cbx;
            S[t][P].cey = pv.cey;
            S[t][P].cby = pv.cby;
        }
        if (lane == kWave - 1) {
#pragma unroll
            for (int t = 1; t <= K; ++t) xhz_w[t] = S[t][P].hz;
        }
        lds_barrier();
        // Ey of every level
#pragma unroll
        for (int t = 1; t <= K; ++t) {
            const int j = r - t;
            const float ey_old = (t == 1) ? ey0 : S[t - 1][P ^ 1].ey;
            const float hz_c = S[t][P].hz;
            const float hz_left = from_left_or(hz_c, xhz_l[t]);
            const float ey_new = upd_ey(ey_old, S[t][P].cey, S[t][P].cby, hz_c, hz_left);
            S[t][P].ey = ey_new;
            if (t == K && j >= w.j0 && valid_col) {
                const unsigned so = (unsigned)j * rowb;
                buf_st(rout, vo, so, hz_c);
                buf_st(rout, vo, so + ohx, S[t][P].ex);
                buf_st(rout, vo, so + ohy, ey_new);
            }
        }
        // Ey of levels 0..K-1 at this row and the row's label, for the next
        // iteration
        if (lane == 0) {
            xey_w[0] = l_ey[P];
#pragma unroll
            for (int t = 2; t <= K; ++t) xey_w[t - 1] = S[t - 1][P].ey;
        }
        if (lane == kWave - 1) *xlab_w = l_lab[P];
        lds_barrier();
    };

    int r = r_begin;
    for (; r + 1 < r_end; r += 2) {
        iteration(r, std::integral_constant<int, 0>{});
        iteration(r + 1, std::integral_constant<int, 1>{});
    }
    if (r < r_end) iteration(r, std::integral_constant<int, 0>{});
}

template <int K>
__global__ __launch_bounds__(256) void k_tblock_te_wg(const InstDev* __restrict__ insts,
                                                      const WorkItem* __restrict__ items, int n_items, int cur) {
    __shared__ WgLdsTe lds;
    const int per_xcd = gridDim.x >> 3;
    const int it = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (it >= n_items) return;   // the whole workgroup
    const WorkItem w = items[it];
    const InstDev* __restrict__ dp = insts + w.inst;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (int k = threadIdx.x; k < dp->n_coef; k += kWgCols) lds.coef[k] = dp->coef[k];
    if (threadIdx.x < kWgWaves * kMaxTBlock) (&lds.ey[0][0])[threadIdx.x] = 0.f;
    if (threadIdx.x < kWgWaves) lds.lab[threadIdx.x] = 0;
    __syncthreads();
    tblock_band_te_wg<K>(*dp, w, cur, wave, lane, &lds);
}

hipError_t launch_tblock_te_wg(int K, const InstDev* insts, const WorkItem* items, int n_items, int cur,
                               hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    const int blocks = (n_items + 7) / 8 * 8;  // one item per workgroup; a multiple of 8 for the XCD remap
    switch (K) {
#define FDTD_TEWG_CASE(k)                                                                  \
    case k:                                                                                \
        k_tblock_te_wg<k><<<blocks, kWgCols, 0, s>>>(insts, items, n_items, cur);          \
        break;
        FDTD_TEWG_CASE(1)
        FDTD_TEWG_CASE(2)
        FDTD_TEWG_CASE(3)
        FDTD_TEWG_CASE(4)
        FDTD_TEWG_CASE(5)
        FDTD_TEWG_CASE(6)
        FDTD_TEWG_CASE(7)
        FDTD_TEWG_CASE(8)
        FDTD_TEWG_CASE(10)
        FDTD_TEWG_CASE(12)
#undef FDTD_TEWG_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
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

hipError_t launch_plain_h(const InstDev& d, int n, int cur, hipStream_t s) {
    dim3 grid((d.nx + 255) / 256, d.ny);
    k_plain_h<<<grid, 256, 0, s>>>(d, n, cur);
    return hipGetLastError();
}

hipError_t launch_plain_te_h(const InstDev& d, int n, int cur, hipStream_t s) {
    dim3 grid((d.nx + 255) / 256, d.ny);
    k_plain_te_h<<<grid, 256, 0, s>>>(d, n, cur);
    return hipGetLastError();
}

hipError_t launch_plain_step(const InstDev& d, int n, int cur, hipStream_t s) {
    dim3 grid((d.nx + 255) / 256, d.ny);
    if (d.pol == 0) {
        k_plain_e<<<grid, 256, 0, s>>>(d, n, cur);
        k_plain_h<<<grid, 256, 0, s>>>(d, n, cur);
    } else {
        k_plain_te_h<<<grid, 256, 0, s>>>(d, n, cur);
        k_plain_te_e<<<grid, 256, 0, s>>>(d, n, cur);
    }
    return hipGetLastError();
}

hipError_t launch_tblock_te(int K, bool special, const InstDev* insts, const WorkItem* items, int n_items, int n0,
                            int cur, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    const int blocks = ((n_items + 3) / 4 + 7) / 8 * 8;  // multiple of 8 for the XCD remap
    switch (K) {
#define FDTD_TE_CASE(k)                                                                    \
    case k:                                                                                \
        if (special)                                                                       \
            k_tblock_te<k, true><<<blocks, 256, 0, s>>>(insts, items, n_items, n0, cur);   \
        else                                                                               \
            k_tblock_te<k, false><<<blocks, 256, 0, s>>>(insts, items, n_items, n0, cur);  \
        break;
        FDTD_TE_CASE(1)
        FDTD_TE_CASE(2)
        FDTD_TE_CASE(3)
        FDTD_TE_CASE(4)
        FDTD_TE_CASE(5)
        FDTD_TE_CASE(6)
        FDTD_TE_CASE(7)
        FDTD_TE_CASE(8)
        FDTD_TE_CASE(10)
        FDTD_TE_CASE(12)
#undef FDTD_TE_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tblock(int K, bool special, const InstDev* insts, const WorkItem* items, int n_items, int n0,
                         int cur, hipStream_t s, bool rec, int hslot0) {
    if (n_items == 0) return hipSuccess;
    const int blocks = ((n_items + 3) / 4 + 7) / 8 * 8;  // multiple of 8 for the XCD remap
    switch (K) {
#define FDTD_TB_LAUNCH(k, sp, rc) k_tblock<k, sp, rc><<<blocks, 256, 0, s>>>(insts, items, n_items, n0, cur, hslot0)
#define FDTD_TB_CASE(k)                                                         \
    case k:                                                                     \
        if (rec) {                                                              \
            if (special)                                                        \
                FDTD_TB_LAUNCH(k, true, true);                                  \
            else                                                                \
                FDTD_TB_LAUNCH(k, false, true);                                 \
        } else {                                                                \
            if (special)                                                        \
                FDTD_TB_LAUNCH(k, true, false);                                 \
            else                                                                \
                FDTD_TB_LAUNCH(k, false, false);                                \
        }                                                                       \
        break;
        FDTD_TB_CASE(1)
        FDTD_TB_CASE(2)
        FDTD_TB_CASE(3)
        FDTD_TB_CASE(4)
        FDTD_TB_CASE(5)
        FDTD_TB_CASE(6)
        FDTD_TB_CASE(7)
        FDTD_TB_CASE(8)
        FDTD_TB_CASE(10)
        FDTD_TB_CASE(12)
#undef FDTD_TB_CASE
#undef FDTD_TB_LAUNCH
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tblock_wg(int K, const InstDev* insts, const WorkItem* items, int n_items, int n0, int cur,
                            hipStream_t s, bool rec, int hslot0) {
    if (n_items == 0) return hipSuccess;
    const int blocks = (n_items + 7) / 8 * 8;  // one item per workgroup; a multiple of 8 for the XCD remap
    switch (K) {
#define FDTD_WG_CASE(k)                                                                                  \
    case k:                                                                                              \
        if (rec)                                                                                         \
            k_tblock_wg<k, true><<<blocks, kWgCols, 0, s>>>(insts, items, n_items, n0, cur, hslot0);     \
        else                                                                                             \
            k_tblock_wg<k, false><<<blocks, kWgCols, 0, s>>>(insts, items, n_items, n0, cur, hslot0);    \
        break;
        FDTD_WG_CASE(1)
        FDTD_WG_CASE(2)
        FDTD_WG_CASE(3)
        FDTD_WG_CASE(4)
        FDTD_WG_CASE(5)
        FDTD_WG_CASE(6)
        FDTD_WG_CASE(7)
        FDTD_WG_CASE(8)
        FDTD_WG_CASE(10)
        FDTD_WG_CASE(12)
#undef FDTD_WG_CASE
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
