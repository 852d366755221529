// Internal device-side definitions of the gfx950 FDTD library.
//
// Units on the device are normalised: H~ = eta0 H, S1 = c dt / h.  The TMz
// updates of eqs. 18-20 then read
//   Ez  <- Ce Ez + Cb [ (Hy(i+1) - Hy(i)) - ((Hx(j+1) - Hx(j))/kappa_e + psi_e) ]
//   Hx  <- Hx - S1 [ (Ez(j) - Ez(j-1))/kappa_h + psi_h ]
//   Hy  <- Hy + S1 [ Ez(i) - Ez(i-1) ]
// with Ce = (1-a)/(1+a), Cb = S1/(eps_r (1+a)), a = sigma dt/(2 eps0 eps_r)
// (eq. 17 with its curl factor restored), and in absorbing-layer rows
//   psi_e <- b_e psi_e + c_e (Hx(j+1) - Hx(j)),  psi_h <- b_h psi_h + c_h (Ez(j) - Ez(j-1)).
// Every kernel evaluates a cell through the functions below, with explicit
// fused multiply-adds and contraction disabled elsewhere, so all kernels give
// bit-identical fields.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdtd {

constexpr int kWave = 64;       // CDNA wavefront
constexpr int kMaxLabels = 256;
constexpr int kMaxPoles = 2;     // dispersive poles per label (broadband runs)
constexpr int kMaxFreqs = 256;   // monitor wavelengths of a broadband run
constexpr int kMaxLabelsBB = 64; // labels of a broadband run (per-wave LDS tables)
constexpr int kMaxTBlock = 12;  // steps per launch of the streaming kernel
constexpr int kMaxPml = 64;     // absorbing-layer cells per side
constexpr int kSpecialBand = 16;  // rows per work item near layers, source and monitors
// TEz edge coefficients: (Ce, Cb) of the edge between cells of labels (a, b),
// averaged materials, at coef[a * kPairStride + b]; instances with more labels
// than kPairStride are rejected for TEz.
constexpr int kPairStride = 16;
constexpr int kPairTable = kPairStride * kPairStride;

// Per-instance device descriptor (all pointers device memory).
struct InstDev {
    float* ez[2];
    float* hx[2];
    float* hy[2];
    float* pe[2];          // psi of Ez on the 2*n_pml layer rows, [2*n_pml][pitch]
    float* ph[2];          // psi of Hx on the layer rows
    const uint8_t* lab;    // [ny][pitch]
    const float2* coef;    // [n_labels]: (Ce, Cb)
    const float4* prof_e;  // [ny]: (b, c, 1/kappa, 0) at Ez rows
    const float4* prof_h;  // [ny]: at Hx rows
    const float2* inc;     // [n_steps]: (E_inc at row j_src, time n+1/2; H~x_inc at edge j_src+1, time n)
    const float2* phasor;  // [n_steps][max(1, n_freqs)]: (cos, sin)(omega_f (n+1/2) dt)
    float* mon;            // [max(1, n_freqs)][2 lines][4][pitch]: sum_c, comp_c, sum_s, comp_s
    int* status;           // non-zero once a monitor sum is non-finite
    int nx, ny, pitch, n_pml;
    int j_src, j_ref, j_trn, dft_start;
    int n_labels;
    float s1;
    // Each ping-pong set is one contiguous region starting at ez[b]: byte
    // offsets of hx, hy, pe, ph inside it and its total size (< 2^31 bytes),
    // for 32-bit buffer addressing.
    unsigned off_hx, off_hy, off_pe, off_ph, set_bytes;
    int pol;               // 0: TMz (fields Ez, Hx, Hy); 1: TEz (Hz, Ex, Ey in the same arrays)
    int n_coef;            // entries of coef: n_labels (TMz) or kPairTable (TEz)
    int n_freqs;           // 0: monochromatic run; >= 1: broadband run at n_freqs wavelengths
    // Ez history of a checkpoint segment ([slot][ny][pitch]), written by the
    // recording variant of the streaming kernel during the adjoint's forward
    // replay; null otherwise.
    float* hist;
    // Broadband runs: per-label pole coefficients [kMaxPoles][kMaxLabels]
    // (alpha, xi, zeta, Cp) of P^{n+1/2} = alpha P^{n-1/2} + xi P^{n-3/2} +
    // zeta Ez^{n-1/2} (P normalised by eps0) and the E update's
    // -Cp (P^{n+1/2} - P^{n-1/2}); and the polarisations at byte offset
    // off_pol of each field set, float2 planes [ny][pitch] holding one pole's
    // two time levels: TMz, one plane per pole (the cell's); TEz, one per
    // edge (Ex, Ey), side and pole.
    const float4* poles;
    unsigned off_pol;
    int n_poles;
    // the monitored field of the two monitor rows at every level of the last
    // streaming launch, or of the pending plain steps, [2 lines][kMaxTBlock]
    // [pitch], for the separate monitor kernel
    float* cap;
};

// Per-instance device descriptor of the discrete adjoint (the transposed
// recurrence shares InstDev's geometry, tables and set layout).
struct AdjDevT {
    float* lset[2];       // ping-pong lambda sets, laid out like the field sets
    float* ga;            // [ny][pitch]: sum_n a^n Ez^{n-1/2}            (= dL/dCe)
    float* gb;            // [ny][pitch]: sum_n a^n (Ez^{n+1/2} - Ce Ez^{n-1/2})  (= Cb dL/dCb)
    const float* hist;    // Ez history of the current segment, [slot][ny][pitch]
    const float* src;     // [2 lines][2][pitch]: dL/d(cosine sum), dL/d(sine sum)
};

// One wave's share of a launch of the streaming kernel: output columns
// [x0, x0 + 64 - 2K) (clipped at nx) and output rows [j0, j1) of one instance.
struct WorkItem {
    int inst;
    int x0;
    int j0;
    int j1;
    int special;  // the band's K-row halo reaches an absorbing layer, the TF/SF
                  // line or a domain edge, or the band owns a monitor row
    int _pad[3];
};

// Bloch projection request: one (instance, monitor line, order m).
struct ProjItem {
    int inst;
    int line;
    int m;
    int _pad;
};

__device__ __forceinline__ bool is_pml_e(int j, int ny, int n_pml) { return j < n_pml || j >= ny - n_pml; }
__device__ __forceinline__ bool is_pml_h(int j, int ny, int n_pml) {
    return (j >= 1 && j < n_pml) || j > ny - n_pml;
}
// Row of the psi arrays holding layer row j (valid for rows where is_pml_* holds).
__device__ __forceinline__ int psi_row(int j, int ny, int n_pml) { return j < n_pml ? j : j - ny + 2 * n_pml; }
// Row of the psi arrays the streaming kernels use for row j: the layer row,
// or the spare row 2 n_pml (never read back as state) for any other row, so
// that their psi loads and stores need no branch.
__device__ __forceinline__ int psi_slot_e(int j, int ny, int n_pml) {
    const int r = j < n_pml ? j : j - ny + 2 * n_pml;
    return ((j < n_pml) | (j >= ny - n_pml)) ? r : 2 * n_pml;
}
__device__ __forceinline__ int psi_slot_h(int j, int ny, int n_pml) {
    const int r = j < n_pml ? j : j - ny + 2 * n_pml;
    return (((j >= 1) & (j < n_pml)) | (j > ny - n_pml)) ? r : 2 * n_pml;
}

// Ez update of one cell (eq. 18).  hx_c = Hx(j), hx_u = Hx(j+1) (0 above the
// top row), hy_c = Hy(i), hy_r = Hy(i+1).  In a layer row pe is updated in
// place.  On the TF/SF row the incident Hx of the edge above is added, since
// that edge belongs to the scattered-field region.
__device__ __forceinline__ float upd_e(float ez, float ce, float cb, float hy_c, float hy_r, float hx_c,
                                       float hx_u, bool pml, float4 pr, float& pe, bool src, float hinc) {
    const float dhx = hx_u - hx_c;
    const float dhy = hy_r - hy_c;
    float t;
    if (pml) {
        pe = __fmaf_rn(pr.x, pe, pr.y * dhx);
        t = __fmaf_rn(dhx, pr.z, pe);
    } else {
        t = dhx;
    }
    if (src) t = t + hinc;
    return __fmaf_rn(ce, ez, cb * (dhy - t));
}

// Hx update of one edge (eq. 19), j >= 1.  e_c = Ez(j), e_d = Ez(j-1).  On the
// first scattered-field edge the incident Ez of the total-field row below is
// removed.
__device__ __forceinline__ float upd_hx(float hx, float e_c, float e_d, float s1, bool pml, float4 pr,
                                        float& ph, bool src, float einc) {
    const float de = e_c - e_d;
    float t;
    if (pml) {
        ph = __fmaf_rn(pr.x, ph, pr.y * de);
        t = __fmaf_rn(de, pr.z, ph);
    } else {
        t = de;
    }
    if (src) t = t + einc;
    return __fmaf_rn(-s1, t, hx);
}

// Hy update of one edge (eq. 20); e_l = Ez(i-1) with periodic wrap (eq. 22).
// The difference is formed as -(e_l - e_c): the same IEEE value as e_c - e_l
// up to the sign of an exact zero, with the shifted operand first so that a
// cross-lane move folds into the subtraction.
__device__ __forceinline__ float upd_hy(float hy, float e_c, float e_l, float s1) {
    return __fmaf_rn(s1, -(e_l - e_c), hy);
}

// TEz updates (eqs. 14-16) in the same normalised units, H~z = eta0 Hz:
//   Hz <- Hz - S1 [ (Ey(i+1) - Ey(i)) - ((Ex(j+1) - Ex(j))/kappa + psi) ]
//   Ex <- Ce Ex + Cb [ (Hz(j) - Hz(j-1))/kappa + psi ],  Ey <- Ce Ey + Cb (Hz(i-1) - Hz(i))
// with per-edge (Ce, Cb) of the averaged materials.  Hz uses the absorbing-
// layer profile of the cell rows (y = j + 1/2), Ex that of the edge rows
// (y = j).  On the TF/SF row j_src the incident Ex of the edge above is
// added to the Hz update; on edge j_src + 1 the incident Hz of the row below
// is added to the Ex update.
__device__ __forceinline__ float upd_hz(float hz, float ey_c, float ey_r, float ex_c, float ex_u, float s1,
                                        bool pml, float4 pr, float& pc, bool src, float exinc) {
    const float dex = ex_u - ex_c;
    const float dey = ey_r - ey_c;
    float t;
    if (pml) {
        pc = __fmaf_rn(pr.x, pc, pr.y * dex);
        t = __fmaf_rn(dex, pr.z, pc);
    } else {
        t = dex;
    }
    if (src) t = t + exinc;
    return __fmaf_rn(-s1, dey - t, hz);
}
__device__ __forceinline__ float upd_ex(float ex, float ce, float cb, float hz_c, float hz_d, bool pml, float4 pr,
                                        float& pe, bool src, float hzinc) {
    const float dh = hz_c - hz_d;
    float t;
    if (pml) {
        pe = __fmaf_rn(pr.x, pe, pr.y * dh);
        t = __fmaf_rn(dh, pr.z, pe);
    } else {
        t = dh;
    }
    if (src) t = t + hzinc;
    return __fmaf_rn(ce, ex, cb * t);
}
// hz_l = Hz(i-1) (periodic); the shifted operand first so that the cross-lane
// move folds into the subtraction.
__device__ __forceinline__ float upd_ey(float ey, float ce, float cb, float hz_c, float hz_l) {
    return __fmaf_rn(ce, ey, cb * (hz_l - hz_c));
}
__device__ __forceinline__ int pair_index(int la, int lb) { return la * kPairStride + lb; }

// Compensated (Kahan) accumulation of one monitor term.
__device__ __forceinline__ void kahan_add(float& sum, float& comp, float x) {
    const float y = x - comp;
    const float t = sum + y;
    comp = (t - sum) - y;
    sum = t;
}

// Adds Ez^{n+1/2} * (cos, sin) to the monitor sums of line `line`, column i.
__device__ __forceinline__ void monitor_add(const InstDev& d, int line, int i, float e, float2 ph) {
    float* m = d.mon + (size_t)line * 4 * d.pitch;
    float s0 = m[i], c0 = m[d.pitch + i], s1 = m[2 * d.pitch + i], c1 = m[3 * d.pitch + i];
    kahan_add(s0, c0, e * ph.x);
    kahan_add(s1, c1, e * ph.y);
    m[i] = s0;
    m[d.pitch + i] = c0;
    m[2 * d.pitch + i] = s1;
    m[3 * d.pitch + i] = c1;
    if (!__builtin_isfinite(s0) || !__builtin_isfinite(s1)) *d.status = 1;
}

// Buffer-resource addressing: a uniform base (SGPRs) plus a per-lane 32-bit
// offset and a uniform 32-bit row offset.  gfx9-family resource word 3.
// A raw buffer access whose lane offset is not below the resource's record
// count is discarded by the hardware (stores) or reads 0 (loads); every buffer
// here is below 2 GiB, so kDropOffset as a lane offset turns a store off for
// that lane without a branch, which keeps the stores of the streaming kernels
// in the same basic block as the arithmetic around them.
constexpr int kBufWord3 = 0x00020000;
constexpr unsigned kDropOffset = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufWord3);
}
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ int buf_ld_u8(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return (int)__builtin_amdgcn_raw_buffer_load_b8(r, (int)voff, (int)soff, 0);
}

// Global-memory access through an address-space-1 pointer: a global_load /
// global_store rather than a flat one, whose possible LDS target would make
// the compiler wait for every outstanding load before the next use.
typedef __attribute__((address_space(1))) float gfloat;
__device__ __forceinline__ float gld(const float* p, size_t i) { return ((const gfloat*)p)[i]; }
__device__ __forceinline__ void gst(float* p, size_t i, float v) { ((gfloat*)p)[i] = v; }
__device__ __forceinline__ void gst_i32(int* p, int v) { *((__attribute__((address_space(1))) int*)p) = v; }

// A register copy the compiler cannot coalesce away (early-clobber output):
// used to move a loaded row out of the load-ring register before the ring
// register receives the next row.  ALU only.
__device__ __forceinline__ float vcopy(float x) {
    float y;
    asm volatile("v_mov_b32 %0, %1" : "=&v"(y) : "v"(x));
    return y;
}
__device__ __forceinline__ int vcopy_i(int x) {
    int y;
    asm volatile("v_mov_b32 %0, %1" : "=&v"(y) : "v"(x));
    return y;
}

// Cross-lane moves inside a wavefront (DPP wave shifts).  Lane l receives the
// value of lane l+1 (from_right) or l-1 (from_left); the end lanes, whose
// source lane does not exist, read 0 (bound_ctrl), which lets the move fold
// into the instruction that consumes it.
__device__ __forceinline__ float from_right(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_left(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ int from_left_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true); }

// Per-wave LDS row table of the special (near-layer) items of the streaming
// kernels.  rows[k] describes row r_begin - K + k of the item (every row any level of the item touches):
// absorbing-layer profile (b, c, 1/kappa) of its Ez and its Hx, neutral
// (0, 0, 1) outside the layers and outside the domain, and in .w a 0/1 flag
// that selects the TF/SF correction (Ez on row j_src, Hx on edge j_src + 1).
// Level t of iteration r reads entry (r - r_begin) + (K - t), an immediate
// offset from a per-iteration base, so no level computes a row index.
struct RowTab {
    float4 e;
    float4 h;
};
constexpr int kTabRows = kSpecialBand + 3 * kMaxTBlock;

// Per-wave LDS tables of the special kernels: the row table, and the
// incident values and monitor phasors of the launch's K steps.
struct SpecialLds {
    RowTab rows[kTabRows];
    float2 inc[kMaxTBlock];
    float2 phasor[kMaxTBlock];
};

// Fills the row table of work item w (K steps per launch) from the instance's
// profile arrays; one row per lane.  Rows of a special item number at most
// kSpecialBand + 3K.
__device__ __forceinline__ void stage_rows(const InstDev* __restrict__ dp, const WorkItem& w, int K,
                                           RowTab* __restrict__ rows, int lane) {
    const int ny = dp->ny, j_src = dp->j_src;
    const int jlo = max(0, w.j0 - K) - K;
    const int nrows = (w.j1 + K) - jlo;
    for (int k = lane; k < nrows; k += kWave) {
        const int j = jlo + k;
        float4 e = make_float4(0.f, 0.f, 1.f, 0.f), h = e;
        if (j >= 0 && j < ny) {
            e = dp->prof_e[j];
            h = dp->prof_h[j];
        }
        e.w = (j == j_src) ? 1.f : 0.f;
        h.w = (j == j_src + 1) ? 1.f : 0.f;
        rows[k] = RowTab{e, h};
    }
}

// XCD-aware order: workgroups are dealt round-robin to the 8 XCDs; the grid
// is a multiple of 8, so this remap is a bijection that hands each XCD a
// contiguous run of work items.  Items are listed band by band, strip by strip
// within a band, so an XCD runs the adjacent strips of a few bands, whose
// shared halo columns then hit in its L2.  Four waves per workgroup, one item
// per wave.
__device__ __forceinline__ int xcd_item(int wave) {
    const int per_xcd = gridDim.x >> 3;
    const int blk = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    return __builtin_amdgcn_readfirstlane(blk * 4 + wave);
}

// Each wave stages its own instance's coefficient table in its own LDS slice;
// LDS instructions of one wave execute in order, so only a compiler-level
// barrier is needed before the lanes read each other's entries.  (No
// workgroup barrier: waves past the end of the item list have returned.)
__device__ __forceinline__ void stage_coef(const InstDev* __restrict__ dp, float2* lds, int lane) {
    const int nl = dp->n_coef;
    const float2* __restrict__ cf = dp->coef;
    for (int k = lane; k < nl; k += kWave) lds[k] = cf[k];
    __builtin_amdgcn_wave_barrier();
}

}  // namespace fdtd

namespace fdtd {

// ---------------------------------------------------------------------------
// Transposed step (discrete adjoint).  The forward step is linear in the
// fields, so its transpose is again a two-phase sweep with the forward's
// stencil shape:
//   E-like phase (reads row j+1 and column i+1):
//     delta(j) = ik_h g + c_h (lph + g),  g = -S1 lHx(j),   lph <- b_h (lph + g)
//     a        = lEz + src + delta(j) - delta(j+1) - S1 (lHy(i+1) - lHy(i))
//     gCe += a Ez^{n-1/2},  gCb += a curl^n,  lEz <- Ce a
//   H-like phase (reads row j-1 and column i-1), with mu = Cb a,
//     nu = ik_e mu - c_e (lpe - mu),  lpe <- b_e (lpe - mu)
//     lHx(j) += nu(j) - nu(j-1),  lHy(i) -= mu(i) - mu(i-1).
// Outside the absorbing layers ik = 1 and c = 0, so delta = g and nu = mu.
// ---------------------------------------------------------------------------

// delta of Hx edge j (j >= 1); updates lph in place on layer rows.
__device__ __forceinline__ float adj_delta(float lhx, float& lph, bool pml, float4 pr, float s1) {
    const float g = -s1 * lhx;
    if (pml) {
        const float lt = lph + g;
        const float d = __fmaf_rn(pr.z, g, pr.y * lt);
        lph = pr.x * lt;
        return d;
    }
    return g;
}

// nu of Ez row j from mu = Cb a; updates lpe in place on layer rows.
__device__ __forceinline__ float adj_nu(float mu, float& lpe, bool pml, float4 pr) {
    if (pml) {
        const float lt = lpe - mu;
        const float v = __fmaf_rn(pr.z, mu, -(pr.y * lt));
        lpe = pr.x * lt;
        return v;
    }
    return mu;
}

}  // namespace fdtd
