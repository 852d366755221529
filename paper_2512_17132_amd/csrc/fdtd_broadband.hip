// gfx950 kernels of broadband runs (Sec. 2.2's Lorentz-Drude alternative to
// one monochromatic run per wavelength): the TMz update with per-label
// polarisation currents and the TEz update with per-edge polarisations, each
// as plain sweeps and as a temporally blocked streaming kernel; and the
// monitor kernel that adds captured monitor-row fields to the Kahan sums of
// every wavelength.
#include <type_traits>

#include "fdtd_device.h"
#include "fdtd_kernels.h"

namespace fdtd {

static_assert(kMaxPoles == 2, "pole activity is carried as two bits per label");

// Polarisations of a TMz broadband instance in field set `cur`: one float2
// plane [ny][pitch] per pole p (plane p), (P_p^{n-1/2}, P_p^{n-3/2}) per cell,
// so that one pole's state moves in one 8-byte access and a pole whose drive
// zeta is zero (its state stays 0) need not move at all.
__device__ __forceinline__ float2* pol_tm(const InstDev& d, int cur) {
    return (float2*)((char*)d.ez[cur] + d.off_pol);
}

// 8-byte buffer accesses (lane offset in bytes; kDropOffset turns a store off
// and makes a load return zeros)
typedef float v2f __attribute__((ext_vector_type(2)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));
__device__ __forceinline__ v2f buf_ld2(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(v2f, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void buf_st2(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, v2f v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), r, (int)voff, (int)soff, 0);
}

// Labels whose pole p is driven (zeta != 0), as bit L of a wave-uniform mask:
// a pole with zeta = 0 starts at zero and stays there (alpha 0 + xi 0 + 0 E is
// +0 for finite E), so the streaming kernels neither load nor store its state.
// Lane L (< n_labels <= 64) tests label L.
__device__ __forceinline__ uint64_t driven_labels(const InstDev* __restrict__ d, int p, int lane) {
    const bool on = lane < d->n_labels && d->poles[p * kMaxLabels + lane].z != 0.0f;
    return __ballot(on);
}

// Keeps a monitored field value e (column i, line 0: reflection, 1:
// transmission) in capture slot `slot` of InstDev::cap; k_monitor_bb adds a
// run of consecutive slots to the Kahan sums of every monitor wavelength.
__device__ __forceinline__ void monitor_keep(const InstDev& d, int line, int slot, int i, float e) {
    d.cap[(size_t)(line * kMaxTBlock + slot) * d.pitch + i] = e;
}

// One step's E sweep of a broadband instance, in place on field set `cur`, one
// thread per cell.  Each pole's polarisation (normalised P/eps0) advances
// first, from the Ez it is about to replace:
//   P^{n+1/2} = alpha P^{n-1/2} + xi P^{n-3/2} + zeta Ez^{n-1/2},
// and the E update loses Cp times the sum of the increments P^{n+1/2} - P^{n-1/2}
// (Ampere's law with eps_inf in Ce, Cb and the poles' dP/dt as a current).
// The monitor rows keep Ez^{n+1/2} in capture slot `slot` for k_monitor_bb.
__global__ __launch_bounds__(256) void k_plain_e_ade(InstDev d, int n, int cur, int slot) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const size_t o = (size_t)j * d.pitch + i;
    const int ir = (i + 1 == d.nx) ? 0 : i + 1;
    const float hx_c = d.hx[cur][o];
    const float hx_u = (j + 1 < d.ny) ? d.hx[cur][o + d.pitch] : 0.0f;
    const float hy_c = d.hy[cur][o];
    const float hy_r = d.hy[cur][(size_t)j * d.pitch + ir];
    const int L = d.lab[o];
    const float2 cf = d.coef[L];
    const float e_old = d.ez[cur][o];
    float2* const pl = pol_tm(d, cur);
    const size_t plane = (size_t)d.ny * d.pitch;
    const float2 p0 = pl[o], p1 = pl[plane + o];
    const float4 q0 = d.poles[L], q1 = d.poles[kMaxLabels + L];
    const float n0 = __fmaf_rn(q0.x, p0.x, __fmaf_rn(q0.y, p0.y, q0.z * e_old));
    const float n1 = __fmaf_rn(q1.x, p1.x, __fmaf_rn(q1.y, p1.y, q1.z * e_old));
    float dpol = 0.0f;
    dpol += n0 - p0.x;
    dpol += n1 - p1.x;
    pl[o] = make_float2(n0, p0.x);
    pl[plane + o] = make_float2(n1, p1.x);
    const float cp = q1.w;
    const bool pml = is_pml_e(j, d.ny, d.n_pml);
    float pe = 0.0f;
    float4 pr = make_float4(0.f, 0.f, 1.f, 0.f);
    size_t po = 0;
    if (pml) {
        po = (size_t)psi_row(j, d.ny, d.n_pml) * d.pitch + i;
        pe = d.pe[cur][po];
        pr = d.prof_e[j];
    }
    const float e =
        upd_e(e_old, cf.x, cf.y, hy_c, hy_r, hx_c, hx_u, pml, pr, pe, j == d.j_src, d.inc[n].y) - cp * dpol;
    d.ez[cur][o] = e;
    if (pml) d.pe[cur][po] = pe;
    if (n >= d.dft_start && (j == d.j_ref || j == d.j_trn)) monitor_keep(d, j == d.j_ref ? 0 : 1, slot, i, e);
}

// TEz with dispersive labels: an Ex or Ey edge's permittivity is the mean of
// its two cells' at every frequency.  Its (Ce, Cb) therefore come from the
// pair table (mean eps_inf and sigma), and its polarisation is half the sum of
// both cells' pole responses to the edge field, each cell's recursion
//   P^{n+1} = alpha P^n + xi P^{n-1} + zeta E^n
// (E and P at integer times in TEz) with that cell's coefficients.  The E
// update loses Cp (P_edge^{n+1} - P_edge^n) with Cp = Cb/S1, since both equal
// 1/(eps_inf (1 + a)) up to the factor S1 of the normalised curl.
// Polarisations of set `cur`: one float2 plane [ny][pitch] per edge, side and
// pole, plane (edge * 2 + side) * kMaxPoles + p, holding (P_p^n, P_p^{n-1}).
// Edge 0 is Ex, 1 is Ey; side 0 is the cell (i, j), side 1 the cell below (Ex)
// or to the left (Ey).

// One side's poles: advances them and returns the sum of their increments.
__device__ __forceinline__ float side_pol_step(const InstDev& d, int cur, int edge, int side, int L, float e_old,
                                               size_t o) {
    const size_t plane = (size_t)d.ny * d.pitch;
    float2* pl = (float2*)((char*)d.ez[cur] + d.off_pol) + (size_t)(edge * 2 + side) * kMaxPoles * plane;
    const float2 p0 = pl[o], p1 = pl[plane + o];
    const float4 q0 = d.poles[L], q1 = d.poles[kMaxLabels + L];
    const float n0 = __fmaf_rn(q0.x, p0.x, __fmaf_rn(q0.y, p0.y, q0.z * e_old));
    const float n1 = __fmaf_rn(q1.x, p1.x, __fmaf_rn(q1.y, p1.y, q1.z * e_old));
    float s = 0.0f;
    s += n0 - p0.x;
    s += n1 - p1.x;
    pl[o] = make_float2(n0, p0.x);
    pl[plane + o] = make_float2(n1, p1.x);
    return s;
}

// The edge's increment 0.5 (S_a + S_b).  When both cells carry the same label
// their poles see the same drive from the same zero start, so S_b = S_a and
// the edge takes S_a exactly (0.5 (S + S) = S in floating point); side 1's
// planes of such an edge are never read or written.
__device__ __forceinline__ float edge_pol_step(const InstDev& d, int cur, int edge, int la, int lb, float e_old,
                                               size_t o) {
    const float sa = side_pol_step(d, cur, edge, 0, la, e_old, o);
    if (lb == la) return sa;
    const float sb = side_pol_step(d, cur, edge, 1, lb, e_old, o);
    return 0.5f * (sa + sb);
}

// One step's E sweep of a broadband TEz instance (after k_plain_te_h), in
// place on set `cur`; the monitor edge rows keep Ex^{n+1} in capture slot
// `slot` for k_monitor_bb.
__global__ __launch_bounds__(256) void k_plain_te_e_ade(InstDev d, int n, int cur, int slot) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx) return;
    const size_t o = (size_t)j * d.pitch + i;
    const float* hz = d.ez[cur];
    const float inv_s1 = 1.0f / d.s1;
    const int la = d.lab[o];
    if (j > 0) {
        const int lb = d.lab[o - d.pitch];
        const float2 cf = d.coef[pair_index(lb, la)];
        const float e_old = d.hx[cur][o];
        const float dpol = edge_pol_step(d, cur, 0, la, lb, e_old, o);
        const bool pml = is_pml_h(j, d.ny, d.n_pml);
        float pe = 0.0f;
        float4 pr = make_float4(0.f, 0.f, 1.f, 0.f);
        size_t po = 0;
        if (pml) {
            po = (size_t)psi_row(j, d.ny, d.n_pml) * d.pitch + i;
            pe = d.ph[cur][po];
            pr = d.prof_h[j];
        }
        const float ex = upd_ex(e_old, cf.x, cf.y, hz[o], hz[o - d.pitch], pml, pr, pe, j == d.j_src + 1,
                                d.inc[n].x) - cf.y * inv_s1 * dpol;
        d.hx[cur][o] = ex;
        if (pml) d.ph[cur][po] = pe;
        if (n >= d.dft_start && (j == d.j_ref || j == d.j_trn)) monitor_keep(d, j == d.j_ref ? 0 : 1, slot, i, ex);
    }
    const int il = (i == 0) ? d.nx - 1 : i - 1;
    const size_t ol = (size_t)j * d.pitch + il;
    const int ll = d.lab[ol];
    const float2 cy = d.coef[pair_index(ll, la)];
    const float e_old = d.hy[cur][o];
    const float dpol = edge_pol_step(d, cur, 1, la, ll, e_old, o);
    d.hy[cur][o] = upd_ey(e_old, cy.x, cy.y, hz[o], hz[ol]) - cy.y * inv_s1 * dpol;
}

hipError_t launch_plain_step_broadband(const InstDev& d, int n, int cur, int slot, hipStream_t s) {
    if (slot < 0 || slot >= kMaxTBlock) return hipErrorInvalidValue;
    dim3 grid((d.nx + 255) / 256, d.ny);
    if (d.pol) {
        const hipError_t e = launch_plain_te_h(d, n, cur, s);
        if (e != hipSuccess) return e;
        k_plain_te_e_ade<<<grid, 256, 0, s>>>(d, n, cur, slot);
        return hipGetLastError();
    }
    k_plain_e_ade<<<grid, 256, 0, s>>>(d, n, cur, slot);
    return launch_plain_h(d, n, cur, s);
}

// ---------------------------------------------------------------------------
// Streaming kernel of broadband instances: the register pipeline of the TMz
// streaming kernel (one wave per 64-column strip and band of rows, level t
// advancing row r - t while row r is read, two row slots per level, DPP
// neighbours, K-row and K-column halos recomputed) with each row also
// carrying its label and the polarisations of its poles.  (Ce, Cb) and the
// pole coefficients come from per-wave LDS tables at every level.  Labels are
// read one row ahead of the fields, so that a row's pole states load with its
// fields and only the driven poles of each cell's label (driven_labels) move
// between HBM and registers; the others are zero and stay zero.  Special
// items capture Ez of the monitor rows at every level and add them to the
// Kahan sums of every monitor wavelength after the sweep (k_monitor_bb, one
// thread per column, wavelength and line).
// ---------------------------------------------------------------------------

// A row slot: fields, layer states, the byte offset of the row's label record
// in the LDS table (low 16 bits; bit 16 + p set where the label drives pole
// p), and each pole's P^{n-1/2}, P^{n-3/2}.
struct SlotBB {
    float e, hx, hy, pe, ph;
    int rec;
    float pc[kMaxPoles], pp[kMaxPoles];
};

// Per-label LDS record: (Ce, Cb, Cp, 0), then (alpha, xi, zeta, 0) of each
// pole; one address per row, the three reads at immediate offsets.
struct BBLds {
    float4 rec[kMaxLabelsBB][1 + kMaxPoles];
};
constexpr int kRecBytes = (int)sizeof(float4) * (1 + kMaxPoles);

template <int K, bool SPECIAL>
__device__ __forceinline__ void tblock_band_bb(const InstDev& dref, const WorkItem& w, int n0, int cur, int lane,
                                               const BBLds* __restrict__ tab, const SpecialLds* __restrict__ sp,
                                               uint64_t drv0, uint64_t drv1) {
    const int nx = dref.nx, ny = dref.ny, pitch = dref.pitch;
    const float s1 = dref.s1;
    const int n_pml = SPECIAL ? dref.n_pml : 0;
    const int j_ref = dref.j_ref, j_trn = dref.j_trn;
    const unsigned off_pe = dref.off_pe, off_ph = dref.off_ph, off_pol = dref.off_pol, set_bytes = dref.set_bytes;
    const unsigned rowb = (unsigned)pitch * 4u;
    const unsigned rowb2 = (unsigned)pitch * 8u;   // a row of a float2 pole plane
    const unsigned plane2 = (unsigned)ny * rowb2;   // one pole plane
    int col = w.x0 - K + lane;
    col %= nx;
    if (col < 0) col += nx;
    const bool valid_col = (lane >= K) && (lane < kWave - K) && (w.x0 + lane - K < nx);
    const bool c1 = cur != 0;
    const __amdgpu_buffer_rsrc_t rin = make_rsrc(c1 ? dref.ez[1] : dref.ez[0], set_bytes);
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(c1 ? dref.ez[0] : dref.ez[1], set_bytes);
    const __amdgpu_buffer_rsrc_t rlab = make_rsrc(dref.lab, (unsigned)ny * (unsigned)pitch);
    const unsigned vo = (unsigned)col * 4u, vl = (unsigned)col, vo2 = (unsigned)col * 8u;
    const unsigned ohx = dref.off_hx, ohy = dref.off_hy;

    const bool own_ref = SPECIAL && w.j0 <= j_ref && j_ref < w.j1;
    const bool own_trn = SPECIAL && w.j0 <= j_trn && j_trn < w.j1;
    float cap_r[K + 1], cap_t[K + 1];
#pragma unroll
    for (int t = 0; t <= K; ++t) cap_r[t] = cap_t[t] = 0.f;

    SlotBB S[K + 1][2];
#pragma unroll
    for (int t = 0; t <= K; ++t)
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            S[t][p].e = S[t][p].hx = S[t][p].hy = S[t][p].pe = S[t][p].ph = 0.f;
            S[t][p].rec = 0;
#pragma unroll
            for (int q = 0; q < kMaxPoles; ++q) S[t][p].pc[q] = S[t][p].pp[q] = 0.f;
        }

    const int r_begin = SPECIAL ? max(0, w.j0 - K) : w.j0 - K;
    const int r_end = w.j1 + K;

    // two row slots of fields, pole states and label records (slot q holds
    // the row after next while the other feeds level 1), and two of labels,
    // read a row ahead of the rest
    float l_e[2], l_hx[2], l_hy[2], l_pe[2], l_ph[2], l_pc[2][kMaxPoles], l_pp[2][kMaxPoles];
    int l_lab[2], l_rec[2];
    auto fetch_lab = [&](int r) { return buf_ld_u8(rlab, vl, (unsigned)min(r, ny - 1) * (unsigned)pitch); };
    auto fetch = [&](int r, int q) {
        const int rr = min(r, ny - 1);
        const unsigned so = (unsigned)rr * rowb;
        l_e[q] = buf_ld(rin, vo, so);
        l_hx[q] = buf_ld(rin, vo, so + ohx);
        l_hy[q] = buf_ld(rin, vo, so + ohy);
        if (SPECIAL) {
            l_pe[q] = buf_ld(rin, vo, off_pe + (unsigned)psi_slot_e(rr, ny, n_pml) * rowb);
            l_ph[q] = buf_ld(rin, vo, off_ph + (unsigned)psi_slot_h(rr, ny, n_pml) * rowb);
        } else {
            l_pe[q] = l_ph[q] = 0.f;
        }
    };
    // label record and pole states of row r, whose label is lab, into slot q:
    // driven poles only
    auto fetch_poles = [&](int r, int lab, int q) {
        const int rr = min(r, ny - 1);
        const unsigned d0 = (unsigned)(drv0 >> lab) & 1u, d1 = (unsigned)(drv1 >> lab) & 1u;
        l_rec[q] = lab * kRecBytes | (int)(d0 << 16) | (int)(d1 << 17);
        const unsigned so = off_pol + (unsigned)rr * rowb2;
        const v2f q0 = buf_ld2(rin, d0 ? vo2 : kDropOffset, so);
        const v2f q1 = buf_ld2(rin, d1 ? vo2 : kDropOffset, so + plane2);
        l_pc[q][0] = q0.x;
        l_pp[q][0] = q0.y;
        l_pc[q][1] = q1.x;
        l_pp[q][1] = q1.y;
    };
    l_e[1] = l_hx[1] = l_hy[1] = l_pe[1] = l_ph[1] = 0.f;
    l_rec[1] = 0;
#pragma unroll
    for (int p = 0; p < kMaxPoles; ++p) l_pc[1][p] = l_pp[1][p] = 0.f;
    {
        const int lab0 = fetch_lab(r_begin);
        l_lab[1] = fetch_lab(r_begin + 1);
        l_lab[0] = 0;
        fetch(r_begin, 0);
        fetch_poles(r_begin, lab0, 0);
    }

    auto iteration = [&](int r, auto P_) {
        constexpr int P = decltype(P_)::value;
        const RowTab* const rt = SPECIAL ? sp->rows + (r - r_begin) : nullptr;
#pragma unroll
        for (int t = 1; t <= K; ++t) {
            const int j = r - t;
            SlotBB pv;
            float hx_up;
            if (t == 1) {
                pv.e = vcopy(l_e[P ^ 1]);
                pv.hx = vcopy(l_hx[P ^ 1]);
                pv.hy = vcopy(l_hy[P ^ 1]);
                pv.pe = SPECIAL ? vcopy(l_pe[P ^ 1]) : 0.f;
                pv.ph = SPECIAL ? vcopy(l_ph[P ^ 1]) : 0.f;
                pv.rec = vcopy_i(l_rec[P ^ 1]);
#pragma unroll
                for (int p = 0; p < kMaxPoles; ++p) {
                    pv.pc[p] = vcopy(l_pc[P ^ 1][p]);
                    pv.pp[p] = vcopy(l_pp[P ^ 1][p]);
                }
                hx_up = l_hx[P];
                // the label of row r + 1 arrived during the last iteration;
                // row r + 2's is read first, ahead of this iteration's fields
                const int lab1 = vcopy_i(l_lab[P ^ 1]);
                l_lab[P] = fetch_lab(r + 2);
                fetch(r + 1, P ^ 1);
                fetch_poles(r + 1, lab1, P ^ 1);
                // keep this row's loads ahead of the levels' arithmetic
                __builtin_amdgcn_sched_barrier(0);
            } else {
                pv = S[t - 1][P ^ 1];
                hx_up = S[t - 1][P].hx;
            }
            if (SPECIAL) hx_up = (j + 1 < ny) ? hx_up : 0.f;
            const float e_below = S[t][P ^ 1].e;
            const float hy_r = from_right(pv.hy);
            // polarisation of the row's poles, from the Ez it replaces
            const float4* const rec = (const float4*)((const char*)&tab->rec[0][0] + (pv.rec & 0xffff));
            const float4 cf4 = rec[0];
            const float2 cf = make_float2(cf4.x, cf4.y);
            const float cp = cf4.z;
            float dpol = 0.f;
            SlotBB nw;
#pragma unroll
            for (int p = 0; p < kMaxPoles; ++p) {
                const float4 pq = rec[1 + p];
                const float pn = __fmaf_rn(pq.x, pv.pc[p], __fmaf_rn(pq.y, pv.pp[p], pq.z * pv.e));
                dpol += pn - pv.pc[p];
                nw.pp[p] = pv.pc[p];
                nw.pc[p] = pn;
            }
            float pe = pv.pe, ph = pv.ph;
            float e_new, hx_new;
            const float4 none = make_float4(0.f, 0.f, 1.f, 0.f);
            if (SPECIAL) {
                const float2 inc = sp->inc[t - 1];
                const float4 pre = rt[K - t].e;
                const float4 prh = rt[K - t].h;
                const float dhx = hx_up - pv.hx;
                const float dhy = hy_r - pv.hy;
                pe = __fmaf_rn(pre.x, pe, pre.y * dhx);
                const float te = __fmaf_rn(dhx, pre.z, pe) + pre.w * inc.y;
                e_new = __fmaf_rn(cf.x, pv.e, cf.y * (dhy - te)) - cp * dpol;
                const float de = e_new - e_below;
                ph = __fmaf_rn(prh.x, ph, prh.y * de);
                const float th = __fmaf_rn(de, prh.z, ph) + prh.w * inc.x;
                hx_new = (j > 0) ? __fmaf_rn(-s1, th, pv.hx) : pv.hx;
                cap_r[t] = (j == j_ref) ? e_new : cap_r[t];
                cap_t[t] = (j == j_trn) ? e_new : cap_t[t];
            } else {
                e_new = upd_e(pv.e, cf.x, cf.y, pv.hy, hy_r, pv.hx, hx_up, false, none, pe, false, 0.f) - cp * dpol;
                hx_new = upd_hx(pv.hx, e_new, e_below, s1, false, none, ph, false, 0.f);
            }
            const float e_left = from_left(e_new);
            const float hy_new = upd_hy(pv.hy, e_new, e_left, s1);
            nw.e = e_new;
            nw.hx = hx_new;
            nw.hy = hy_new;
            nw.pe = pe;
            nw.ph = ph;
            nw.rec = pv.rec;
            S[t][P] = nw;
            if (t == K) {
                // owned cells only; other lanes and rows are dropped
                const bool owned = SPECIAL ? (j >= w.j0 && j < w.j1) : (j >= w.j0);
                const unsigned so = (unsigned)j * rowb;
                const unsigned vs = (owned && valid_col) ? vo : kDropOffset;
                buf_st(rout, vs, so, e_new);
                buf_st(rout, vs, so + ohx, hx_new);
                buf_st(rout, vs, so + ohy, hy_new);
                const bool keep = owned && valid_col;
                const unsigned sp2 = off_pol + (unsigned)j * rowb2;
                const v2f q0 = {nw.pc[0], nw.pp[0]};
                const v2f q1 = {nw.pc[1], nw.pp[1]};
                buf_st2(rout, (keep && ((pv.rec >> 16) & 1)) ? vo2 : kDropOffset, sp2, q0);
                buf_st2(rout, (keep && ((pv.rec >> 17) & 1)) ? vo2 : kDropOffset, sp2 + plane2, q1);
                if (SPECIAL) {
                    buf_st(rout, vs, off_pe + (unsigned)psi_slot_e(j, ny, n_pml) * rowb, pe);
                    buf_st(rout, vs, off_ph + (unsigned)psi_slot_h(j, ny, n_pml) * rowb, ph);
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
        // the owned monitor rows' Ez of every level, for k_monitor_bb
        float* const capb = dref.cap;
        auto keep = [&](int line, const float (&cap)[K + 1]) {
            if (!valid_col) return;
#pragma unroll
            for (int t = 1; t <= K; ++t) gst(capb, (size_t)(line * kMaxTBlock + t - 1) * pitch + col, cap[t]);
        };
        if (own_ref) keep(0, cap_r);
        if (own_trn) keep(1, cap_t);
    }
}

// Monitor sums of a broadband instance over K consecutive steps from n0 (one
// streaming launch, or up to kMaxTBlock plain steps): thread (column,
// wavelength f, line) adds the captured field of each step, in step order,
// times that step's phasor of f to its Kahan pairs.
__global__ __launch_bounds__(256) void k_monitor_bb(InstDev d, int n0, int K) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int f = blockIdx.y, line = blockIdx.z;
    if (i >= d.nx) return;
    float* m = d.mon + (size_t)(2 * f + line) * 4 * d.pitch;
    float s0 = m[i], c0 = m[d.pitch + i], s1 = m[2 * d.pitch + i], c1 = m[3 * d.pitch + i];
    for (int t = 0; t < K; ++t) {
        const int n = n0 + t;
        if (n < d.dft_start) continue;
        const float e = d.cap[(size_t)(line * kMaxTBlock + t) * d.pitch + i];
        const float2 w = d.phasor[(size_t)n * d.n_freqs + f];
        kahan_add(s0, c0, e * w.x);
        kahan_add(s1, c1, e * w.y);
    }
    m[i] = s0;
    m[d.pitch + i] = c0;
    m[2 * d.pitch + i] = s1;
    m[3 * d.pitch + i] = c1;
    if (!__builtin_isfinite(s0) || !__builtin_isfinite(s1)) *d.status = 1;
}

hipError_t launch_monitor_bb(const InstDev& d, int n0, int K, hipStream_t s) {
    dim3 grid((d.nx + 255) / 256, d.n_freqs, 2);
    k_monitor_bb<<<grid, 256, 0, s>>>(d, n0, K);
    return hipGetLastError();
}

template <int K, bool SPECIAL>
// The lean kernel of up to 8 steps per launch fits 128 registers, which
// lets 4 waves share a SIMD; without the hint it takes a few more.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(!SPECIAL && K <= 8 ? 4 : 1))) void k_tblock_bb(const InstDev* __restrict__ insts, const WorkItem* __restrict__ items,
                                                   int n_items, int n0, int cur) {
    __shared__ BBLds tab_lds[4];
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
        if (lane < K) sp->inc[lane] = dp->inc[n0 + lane];
    }
    BBLds* tab = &tab_lds[wave];
    const int nl = dp->n_labels, np = dp->n_poles;   // np == kMaxPoles
    for (int k = lane; k < nl; k += kWave) {
        const float2 c = dp->coef[k];
        // Cp is the same for every pole of a label; a label without poles has
        // no current to subtract
        const float cp = dp->poles[k].w;
        tab->rec[k][0] = make_float4(c.x, c.y, cp, 0.f);
        for (int p = 0; p < kMaxPoles; ++p)
            tab->rec[k][1 + p] = p < np ? dp->poles[p * kMaxLabels + k] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const uint64_t drv0 = driven_labels(dp, 0, lane), drv1 = driven_labels(dp, 1, lane);
    __builtin_amdgcn_wave_barrier();
    tblock_band_bb<K, SPECIAL>(*dp, w, n0, cur, lane, tab, sp, drv0, drv1);
}

hipError_t launch_tblock_bb(int K, bool special, const InstDev* insts, const WorkItem* items, int n_items, int n0,
                            int cur, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    const int blocks = ((n_items + 3) / 4 + 7) / 8 * 8;  // multiple of 8 for the XCD remap
    switch (K) {
#define FDTD_BB_CASE(k)                                                                    \
    case k:                                                                                \
        if (special)                                                                       \
            k_tblock_bb<k, true><<<blocks, 256, 0, s>>>(insts, items, n_items, n0, cur);   \
        else                                                                               \
            k_tblock_bb<k, false><<<blocks, 256, 0, s>>>(insts, items, n_items, n0, cur);  \
        break;
        FDTD_BB_CASE(1)
        FDTD_BB_CASE(2)
        FDTD_BB_CASE(3)
        FDTD_BB_CASE(4)
        FDTD_BB_CASE(5)
        FDTD_BB_CASE(6)
        FDTD_BB_CASE(7)
        FDTD_BB_CASE(8)
        FDTD_BB_CASE(10)
        FDTD_BB_CASE(12)
#undef FDTD_BB_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Streaming kernel of broadband TEz instances: the TEz pipeline of
// k_tblock_te (level t advances Hz of row r - t, then Ex and Ey) with the
// edge polarisations of k_plain_te_e_ade evaluated in the same order.  Per
// level a row carries Hz, Ex, Ey, one register of packed labels and the pole
// states of both sides of its Ex and Ey edges (16 values); the edge (Ce, Cb)
// and each side's pole coefficients are read from per-wave LDS tables at every
// level rather than carried, to keep the per-level state small.  The side-1
// state of an edge (the second cell's poles) exists only where the two cells
// differ in label, and a pole's state only where its cell's label drives it
// (driven_labels): other lanes load such a state through the dropped offset
// (zero, the value it keeps forever) and store nothing.  A row's pole states
// are loaded one iteration before level 1 needs them, into one load set.
// ---------------------------------------------------------------------------

// A row slot: fields, layer states, the packed labels
//   la | lb << 4 | la << 8 | ll << 12 | da << 16 | db << 18 | dl << 20
// (la the cell's label, lb the cell below's, ll the cell to the left's, so that
// the low byte is the Ex edge's pair index and the next byte the Ey edge's;
// da, db, dl their driven-pole bits, bit p for pole p), and the pole states
// (P_0^n, P_0^{n-1}, P_1^n, P_1^{n-1}) of each edge side: x0, x1 (Ex, sides 0
// and 1), y0, y1 (Ey).
struct SlotBT {
    float hz, ex, ey, pc, pe;
    int pk;
    float x0[4], x1[4], y0[4], y1[4];
};

// Pole records of a broadband TEz run per label: (alpha, xi, zeta, -) of each
// pole; at most kPairStride labels.
struct BTLds {
    float2 coef[kPairTable];
    float4 pole[kPairStride][kMaxPoles];
};

// One side's poles driven by the edge's old field: the new state in n, the sum
// of the two increments returned (side_pol_step's arithmetic, in its order).
__device__ __forceinline__ float side_step(const float4 q0, const float4 q1, const float (&p)[4], float e_old,
                                           float (&n)[4]) {
    const float n0 = __fmaf_rn(q0.x, p[0], __fmaf_rn(q0.y, p[1], q0.z * e_old));
    const float n1 = __fmaf_rn(q1.x, p[2], __fmaf_rn(q1.y, p[3], q1.z * e_old));
    float s = 0.0f;
    s += n0 - p[0];
    s += n1 - p[2];
    n[0] = n0;
    n[1] = p[0];
    n[2] = n1;
    n[3] = p[2];
    return s;
}

// An edge's polarisation increment (edge_pol_step): side 0 with label a,
// side 1 with label b where b differs; the side-1 state is left as it is
// where the labels agree.
__device__ __forceinline__ float edge_step(const BTLds* __restrict__ tab, int a, int b, const float (&p0)[4],
                                           const float (&p1)[4], float e_old, float (&n0)[4], float (&n1)[4]) {
    const float sa = side_step(tab->pole[a][0], tab->pole[a][1], p0, e_old, n0);
    float m[4];
    const float sb = side_step(tab->pole[b][0], tab->pole[b][1], p1, e_old, m);
    const bool two = a != b;
#pragma unroll
    for (int k = 0; k < 4; ++k) n1[k] = two ? m[k] : p1[k];
    return two ? 0.5f * (sa + sb) : sa;
}

// edge_step where no edge of the wave has a second cell that drives a pole:
// every side-1 state is +0 and stays so, and side 1's increment is +0 (as
// side_step computes it with zeta = 0), so only side 0 is evaluated and the
// mean is taken with that +0.
__device__ __forceinline__ float edge_step_side0(const BTLds* __restrict__ tab, int a, int b, const float (&p0)[4],
                                                 const float (&p1)[4], float e_old, float (&n0)[4], float (&n1)[4]) {
    const float sa = side_step(tab->pole[a][0], tab->pole[a][1], p0, e_old, n0);
    const float sb = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) n1[k] = p1[k];
    return a != b ? 0.5f * (sa + sb) : sa;
}

template <int K, bool SPECIAL>
__device__ __forceinline__ void tblock_band_bt(const InstDev& dref, const WorkItem& w, int n0, int cur, int lane,
                                               const BTLds* __restrict__ tab, const SpecialLds* __restrict__ sp,
                                               unsigned drv0, unsigned drv1) {
    const int nx = dref.nx, ny = dref.ny, pitch = dref.pitch;
    const float s1 = dref.s1;
    const float inv_s1 = 1.0f / s1;
    const int n_pml = SPECIAL ? dref.n_pml : 0;
    const int j_ref = dref.j_ref, j_trn = dref.j_trn;
    const unsigned off_pe = dref.off_pe, off_ph = dref.off_ph, off_pol = dref.off_pol, set_bytes = dref.set_bytes;
    const unsigned rowb = (unsigned)pitch * 4u;
    const unsigned rowb2 = (unsigned)pitch * 8u;           // a row of a float2 pole plane
    const unsigned plane = (unsigned)ny * rowb2;            // one pole plane
    int col = w.x0 - K + lane;
    col %= nx;
    if (col < 0) col += nx;
    const bool valid_col = (lane >= K) && (lane < kWave - K) && (w.x0 + lane - K < nx);
    const bool c1 = cur != 0;
    const __amdgpu_buffer_rsrc_t rin = make_rsrc(c1 ? dref.ez[1] : dref.ez[0], set_bytes);
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(c1 ? dref.ez[0] : dref.ez[1], set_bytes);
    const __amdgpu_buffer_rsrc_t rlab = make_rsrc(dref.lab, (unsigned)ny * (unsigned)pitch);
    const unsigned vo = (unsigned)col * 4u, vl = (unsigned)col, vo2 = (unsigned)col * 8u;
    const unsigned ohx = dref.off_hx, ohy = dref.off_hy;

    const bool own_ref = SPECIAL && w.j0 <= j_ref && j_ref < w.j1;
    const bool own_trn = SPECIAL && w.j0 <= j_trn && j_trn < w.j1;
    float cap_r[K + 1], cap_t[K + 1];
#pragma unroll
    for (int t = 0; t <= K; ++t) cap_r[t] = cap_t[t] = 0.f;

    SlotBT S[K + 1][2];
#pragma unroll
    for (int t = 0; t <= K; ++t)
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            S[t][p].hz = S[t][p].ex = S[t][p].ey = S[t][p].pc = S[t][p].pe = 0.f;
            S[t][p].pk = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) S[t][p].x0[k] = S[t][p].x1[k] = S[t][p].y0[k] = S[t][p].y1[k] = 0.f;
        }

    const int r_begin = SPECIAL ? max(0, w.j0 - K) : w.j0 - K;
    const int r_end = w.j1 + K;

    // fields and label of the row after next; pole states of the next row
    float l_hz[2], l_ex[2], l_ey[2], l_pc[2], l_pe[2];
    int l_lab[2];
    float l_x0[4], l_x1[4], l_y0[4], l_y1[4];
    int l_pk = 0;
    int lab_last = 0;   // label of the row whose poles were loaded last
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
    // pole states of row r, whose label is la (the row below's was lab_last)
    auto driven = [&](int l) { return (int)(((drv0 >> l) & 1u) | (((drv1 >> l) & 1u) << 1)); };
    // plane of edge e (0: Ex, 1: Ey), side s, pole p
    auto pl_off = [&](int e, int s, int p) { return (unsigned)((e * 2 + s) * kMaxPoles + p) * plane; };
    auto fetch_poles = [&](int r, int la) {
        const int rr = min(r, ny - 1);
        const int lb = lab_last;
        const int ll = from_left_i(la);
        lab_last = la;
        const int da = driven(la), db = la != lb ? driven(lb) : 0, dl = la != ll ? driven(ll) : 0;
        l_pk = la | (lb << 4) | (la << 8) | (ll << 12) | (da << 16) | (db << 18) | (dl << 20);
        const unsigned so = off_pol + (unsigned)rr * rowb2;
        auto ld = [&](int e, int s, int p, int on, float* dst) {
            const v2f v = buf_ld2(rin, on ? vo2 : kDropOffset, so + pl_off(e, s, p));
            dst[2 * p] = v.x;
            dst[2 * p + 1] = v.y;
        };
#pragma unroll
        for (int p = 0; p < kMaxPoles; ++p) {
            ld(0, 0, p, (da >> p) & 1, l_x0);
            ld(0, 1, p, (db >> p) & 1, l_x1);
            ld(1, 0, p, (da >> p) & 1, l_y0);
            ld(1, 1, p, (dl >> p) & 1, l_y1);
        }
    };
    l_hz[1] = l_ex[1] = l_ey[1] = l_pc[1] = l_pe[1] = 0.f;
    l_lab[1] = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) l_x0[k] = l_x1[k] = l_y0[k] = l_y1[k] = 0.f;
    fetch(r_begin, 0);

    auto iteration = [&](int r, auto P_) {
        constexpr int P = decltype(P_)::value;
        const RowTab* const rt = SPECIAL ? sp->rows + (r - r_begin) : nullptr;
#pragma unroll
        for (int t = 1; t <= K; ++t) {
            const int j = r - t;
            SlotBT pv;       // level t-1, row j
            float ex_up;     // level t-1, row j+1
            if (t == 1) {
                pv.hz = vcopy(l_hz[P ^ 1]);
                pv.ex = vcopy(l_ex[P ^ 1]);
                pv.ey = vcopy(l_ey[P ^ 1]);
                pv.pc = SPECIAL ? vcopy(l_pc[P ^ 1]) : 0.f;
                pv.pe = SPECIAL ? vcopy(l_pe[P ^ 1]) : 0.f;
                pv.pk = vcopy_i(l_pk);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    pv.x0[k] = vcopy(l_x0[k]);
                    pv.x1[k] = vcopy(l_x1[k]);
                    pv.y0[k] = vcopy(l_y0[k]);
                    pv.y1[k] = vcopy(l_y1[k]);
                }
                ex_up = l_ex[P];
                fetch_poles(r, vcopy_i(l_lab[P]));
                fetch(r + 1, P ^ 1);
            } else {
                pv = S[t - 1][P ^ 1];
                ex_up = S[t - 1][P].ex;
            }
            if (SPECIAL) ex_up = (j + 1 < ny) ? ex_up : 0.f;   // electric wall above the top row
            const float hz_below = S[t][P ^ 1].hz;          // level t, row j-1
            const float ey_r = from_right(pv.ey);
            const int la = pv.pk & 15, lb = (pv.pk >> 4) & 15, ll = (pv.pk >> 12) & 15;
            const float2 cx = tab->coef[pv.pk & 0xff];          // pair (lb, la)
            const float2 cy = tab->coef[(pv.pk >> 8) & 0xff];   // pair (ll, la)
            SlotBT nw;
            float dpx = 0.f, dpy = 0.f;
            const int drv = (pv.pk >> 16) & 63;   // da | db << 2 | dl << 4
            if (__builtin_amdgcn_ballot_w64((drv >> 2) != 0) != 0) {
                dpx = edge_step(tab, la, lb, pv.x0, pv.x1, pv.ex, nw.x0, nw.x1);
                dpy = edge_step(tab, la, ll, pv.y0, pv.y1, pv.ey, nw.y0, nw.y1);
            } else if (__builtin_amdgcn_ballot_w64(drv != 0) != 0) {
                dpx = edge_step_side0(tab, la, lb, pv.x0, pv.x1, pv.ex, nw.x0, nw.x1);
                dpy = edge_step_side0(tab, la, ll, pv.y0, pv.y1, pv.ey, nw.y0, nw.y1);
            } else {
                // no cell of this wave's row drives a pole: every side state
                // is +0 and stays so, and the increments are +0 as computed;
                // the states are passed on as they are, so that the copies
                // run on this path only
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    nw.x0[k] = pv.x0[k];
                    nw.x1[k] = pv.x1[k];
                    nw.y0[k] = pv.y0[k];
                    nw.y1[k] = pv.y1[k];
                }
            }
            float pc = pv.pc, pe = pv.pe;
            float hz_new, ex_new;
            const float4 none = make_float4(0.f, 0.f, 1.f, 0.f);
            if (SPECIAL) {
                // branch-free upd_hz/upd_ex as in the TEz streaming kernel
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
                // Ex(0) is the wall: neither it nor its poles advance
                if (j > 0) {
                    ex_new = __fmaf_rn(cx.x, pv.ex, cx.y * te) - cx.y * inv_s1 * dpx;
                } else {
                    ex_new = pv.ex;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        nw.x0[k] = pv.x0[k];
                        nw.x1[k] = pv.x1[k];
                    }
                }
                cap_r[t] = (j == j_ref) ? ex_new : cap_r[t];
                cap_t[t] = (j == j_trn) ? ex_new : cap_t[t];
            } else {
                hz_new = upd_hz(pv.hz, pv.ey, ey_r, pv.ex, ex_up, s1, false, none, pc, false, 0.f);
                ex_new = upd_ex(pv.ex, cx.x, cx.y, hz_new, hz_below, false, none, pe, false, 0.f) - cx.y * inv_s1 * dpx;
            }
            const float hz_left = from_left(hz_new);
            const float ey_new = upd_ey(pv.ey, cy.x, cy.y, hz_new, hz_left) - cy.y * inv_s1 * dpy;
            nw.hz = hz_new;
            nw.ex = ex_new;
            nw.ey = ey_new;
            nw.pc = pc;
            nw.pe = pe;
            nw.pk = pv.pk;
            S[t][P] = nw;
            if (t == K) {
                // owned cells only; other lanes and rows are dropped, and so are
                // the side-1 states of edges between cells of one label
                const bool owned = SPECIAL ? (j >= w.j0 && j < w.j1) : (j >= w.j0);
                const bool keep = owned && valid_col;
                const unsigned vs = keep ? vo : kDropOffset;
                const unsigned so = (unsigned)j * rowb;
                buf_st(rout, vs, so, hz_new);
                buf_st(rout, vs, so + ohx, ex_new);
                buf_st(rout, vs, so + ohy, ey_new);
                // driven poles only (the side-1 bits are clear where the
                // labels agree)
                const unsigned sp2 = off_pol + (unsigned)j * rowb2;
                const int da = (pv.pk >> 16) & 3, db = (pv.pk >> 18) & 3, dl = (pv.pk >> 20) & 3;
                auto st = [&](int e, int s, int p, int on, const float* src) {
                    const v2f v = {src[2 * p], src[2 * p + 1]};
                    buf_st2(rout, (keep && on) ? vo2 : kDropOffset, sp2 + pl_off(e, s, p), v);
                };
#pragma unroll
                for (int p = 0; p < kMaxPoles; ++p) {
                    st(0, 0, p, (da >> p) & 1, nw.x0);
                    st(0, 1, p, (db >> p) & 1, nw.x1);
                    st(1, 0, p, (da >> p) & 1, nw.y0);
                    st(1, 1, p, (dl >> p) & 1, nw.y1);
                }
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
        // the owned monitor rows' Ex of every level, for k_monitor_bb
        float* const capb = dref.cap;
        auto keep = [&](int line, const float (&cap)[K + 1]) {
            if (!valid_col) return;
#pragma unroll
            for (int t = 1; t <= K; ++t) gst(capb, (size_t)(line * kMaxTBlock + t - 1) * pitch + col, cap[t]);
        };
        if (own_ref) keep(0, cap_r);
        if (own_trn) keep(1, cap_t);
    }
}

// Blocks of the special items in a broadband TEz launch: a multiple of 8.
__host__ __device__ __forceinline__ int bt_special_blocks(int n_special) { return ((n_special + 3) / 4 + 7) / 8 * 8; }

// One launch of broadband TEz items, each wave on the code path of its item's
// kind (the branch is uniform per wave).  Both paths need about the same
// registers, so sharing the kernel costs no occupancy, and the few special
// items (the bands at the absorbing layers, the source and the monitor rows)
// run in the slots the lean items leave free instead of ahead of them.  The
// special items take the first blocks in dispatch order, which go round-robin
// over the XCDs; the lean items take the rest, grouped by XCD as in xcd_item.
template <int K>
__global__ __launch_bounds__(256) void k_tblock_bt(const InstDev* __restrict__ insts,
                                                   const WorkItem* __restrict__ special, int n_special,
                                                   const WorkItem* __restrict__ lean, int n_lean, int n0, int cur) {
    __shared__ BTLds tab_lds[4];
    __shared__ SpecialLds sp_lds[4];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int sb = bt_special_blocks(n_special);
    const bool is_special = (int)blockIdx.x < sb;
    int it;
    if (is_special) {
        it = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + wave);
        if (it >= n_special) return;
    } else {
        const int lb = (int)blockIdx.x - sb;
        const int per_xcd = ((int)gridDim.x - sb) >> 3;
        it = __builtin_amdgcn_readfirstlane(((lb & 7) * per_xcd + (lb >> 3)) * 4 + wave);
        if (it >= n_lean) return;
    }
    const WorkItem w = is_special ? special[it] : lean[it];
    const InstDev* __restrict__ dp = insts + w.inst;
    SpecialLds* sp = &sp_lds[wave];
    if (is_special) {
        stage_rows(dp, w, K, sp->rows, lane);
        if (lane < K) sp->inc[lane] = dp->inc[n0 + lane];
    }
    BTLds* tab = &tab_lds[wave];
    for (int k = lane; k < kPairTable; k += kWave) tab->coef[k] = dp->coef[k];
    const int nl = dp->n_labels;   // <= kPairStride for TEz
    if (lane < kPairStride) {
        const bool ok = lane < nl;
        tab->pole[lane][0] = ok ? dp->poles[lane] : make_float4(0.f, 0.f, 0.f, 0.f);
        tab->pole[lane][1] = ok ? dp->poles[kMaxLabels + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const unsigned drv0 = (unsigned)driven_labels(dp, 0, lane), drv1 = (unsigned)driven_labels(dp, 1, lane);
    __builtin_amdgcn_wave_barrier();
    if (is_special)
        tblock_band_bt<K, true>(*dp, w, n0, cur, lane, tab, sp, drv0, drv1);
    else
        tblock_band_bt<K, false>(*dp, w, n0, cur, lane, tab, sp, drv0, drv1);
}

hipError_t launch_tblock_bt(int K, const InstDev* insts, const WorkItem* special, int n_special, const WorkItem* lean,
                            int n_lean, int n0, int cur, hipStream_t s) {
    if (n_special + n_lean == 0) return hipSuccess;
    const int blocks = bt_special_blocks(n_special) + ((n_lean + 3) / 4 + 7) / 8 * 8;
    switch (K) {
#define FDTD_BT_CASE(k)                                                                                     \
    case k:                                                                                                 \
        k_tblock_bt<k><<<blocks, 256, 0, s>>>(insts, special, n_special, lean, n_lean, n0, cur);            \
        break;
        FDTD_BT_CASE(1)
        FDTD_BT_CASE(2)
        FDTD_BT_CASE(3)
        FDTD_BT_CASE(4)
        FDTD_BT_CASE(5)
        FDTD_BT_CASE(6)
        FDTD_BT_CASE(7)
        FDTD_BT_CASE(8)
        FDTD_BT_CASE(10)
        FDTD_BT_CASE(12)
#undef FDTD_BT_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fdtd
