// Internal host-side definitions shared by the host units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/fdtd.h"
#include "fdtd_device.h"

struct HostInst {
    int nx, ny, pitch, n_pml, j_src, j_ref, j_trn, n_labels;
    int pol = 0;                  // 0: TMz, 1: TEz
    int n_steps = 0;              // this instance's run length
    int dft_start = 0;            // first monitored step
    int cur_end = 0;              // field set holding the state once the run has ended
    double dx, courant, lambda0;
    double s1, wdt;               // S1 = c dt/h, omega dt
    std::vector<double> nk;       // n_labels * 2
    std::vector<uint8_t> labels;  // ny * nx
    std::vector<double> e_inc;    // n_steps: TMz incident Ez on row j_src at (n+1/2) dt;
                                  //          TEz incident Ex on edge j_src+1 at (n+1) dt
    std::vector<double> h_inc;    // n_steps: TMz incident H~x on edge j_src+1 at n dt;
                                  //          TEz incident H~z on row j_src at (n+1/2) dt
    double inc_c = 0, inc_s = 0;  // incident monitor sums over the window
    std::vector<int> orders;      // propagating Bloch orders
    std::vector<double> weights;  // their flux weights
    // broadband runs (n_freqs > 0): dispersive model, monitor wavelengths and
    // pulse; per monitor wavelength the propagating orders, their weights and
    // the transform of the incident wave over the window
    int n_freqs = 0, n_poles = 0;
    std::vector<double> model;    // n_labels x (2 + 3 n_poles)
    std::vector<double> lambdas;
    double tau = 0.0, t0 = 0.0;
    std::vector<std::vector<int>> f_orders;
    std::vector<std::vector<double>> f_weights;
    std::vector<double> f_inc_re, f_inc_im;
    size_t proj_begin = 0, proj_count = 0;  // this instance's projection requests
    fdtd::InstDev dev;
    size_t cells() const { return (size_t)nx * ny; }
};

// Work items of one (K, band) launch configuration, split into the items that
// take every row-dependent branch (special) and the branch-free rest (lean).
struct ItemList {
    fdtd::WorkItem* d = nullptr;  // special: TMz, TEz, broadband TMz, broadband TEz; then lean, the same
    int n_special = 0;            // both polarisations
    int n_lean = 0;
    int n_special_te = 0;         // the TEz share of each group
    int n_lean_te = 0;
    int n_special_bb = 0;         // the broadband TMz share of each group
    int n_lean_bb = 0;
    int n_special_bt = 0;         // the broadband TEz share of each group
    int n_lean_bt = 0;
    int64_t lean_cells = 0;  // cells the lean items of one launch own
    // the lean monochromatic items again as workgroup items (fdtd::kWgColumns
    // columns each): TMz at d + wg, TEz at d + wg_te.  The forward launches use
    // these when the context's bulk layout is the workgroup one; the adjoint's
    // transposed kernel always uses the per-wave ones
    int wg = 0;
    int n_lean_wg = 0;
    int wg_te = 0;
    int n_lean_wg_te = 0;
    int n() const { return n_special + n_lean; }
};

// Device buffers of the discrete adjoint (allocated on the first recorded run).
struct AdjointInst {
    float* lset[2] = {nullptr, nullptr};  // lambda sets, laid out like the forward's field sets
    float* tmp0 = nullptr;  // per-step scratch rows of the plain transposed sweeps
    float* tmp1 = nullptr;
    float* tmp2 = nullptr;
    float* ga = nullptr;    // accumulated dL/dCe per pixel
    float* gb = nullptr;    // accumulated Cb dL/dCb per pixel
    float* src = nullptr;   // [2 lines][2][pitch]: dL/d(cos sum), dL/d(sin sum)
    float* ckpt = nullptr;  // checkpoints: [n_ckpt][field set]
    float* seg = nullptr;   // Ez history of one segment: [seg_len + 1][ny][pitch]
    float* fin = nullptr;   // final forward state (restored after the sweep)
    double* lsum = nullptr; // per-label sums of gCe and gCb: [n_labels][2]
    double* rowsum = nullptr; // the same sums per row, [ny][n_labels][2], added in row order
    size_t set_floats = 0;  // floats of one field set (checkpoint stride)
};

struct AdjointState {
    bool recorded = false;
    bool full = false;      // one segment whose Ez history the recorded run itself writes: no replays
    int every = 0;          // steps per checkpoint segment
    int n_ckpt = 0;
    size_t bytes = 0;
    char* slab = nullptr;
    std::vector<AdjointInst> inst;
    fdtd::InstDev* d_rec = nullptr;   // replay descriptors: monitors off, Ez history on
    fdtd::InstDev* d_recm = nullptr;  // recorded-run descriptors of the single-segment form: monitors and Ez history on
    fdtd::AdjDevT* d_adj = nullptr;   // adjoint descriptors
    int lcur = 0;                     // lambda set holding the current adjoint state
    int band = 0;                     // rows per work item of the streaming adjoint kernel (0: not chosen)
    // captured reverse sweep (checkpoint restores, segment replays, transposed
    // launches) and the launch shape and buffers it was captured with
    hipGraphExec_t graph = nullptr;
    int graph_K = 0, graph_B = 0, graph_SB = 0, graph_W = 0, graph_adjK = 0, graph_adjB = 0;
    char* graph_slab = nullptr;
};

struct fdtd_ctx {
    std::vector<HostInst> inst;
    fdtd_opts opts;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t aux = nullptr;       // special work items run here, concurrently
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join = nullptr;
    bool has_bt = false;             // holds broadband TEz: one stream, special items in the lean items' kernel
    int device = 0;
    char* slab = nullptr;
    size_t slab_bytes = 0;
    fdtd::InstDev* d_insts = nullptr;
    int cur = 0;   // ping-pong buffer holding the current state
    int step = 0;  // steps done
    // streaming kernel configuration: steps per launch, rows of a bulk band,
    // rows of a special band
    int K = 0, B = 0, SB = fdtd::kSpecialBand;
    int W = 64;            // columns per bulk item of a monochromatic instance: 64 (a wave) or fdtd::kWgColumns (a workgroup)
    bool has_mono = false; // holds monochromatic instances (the only bulk items W applies to)
    bool tuned = false;
    // (K, B, SB, m) -> device work list of the instances whose run is >= m steps
    std::map<std::tuple<int, int, int, int>, ItemList> items;
    // the same key -> host copy of the list and its counts, for the launches
    // of fdtd_step_noalloc, which stage it in the library's fixed device array
    std::map<std::tuple<int, int, int, int>, std::pair<std::vector<fdtd::WorkItem>, ItemList>> host_items;
    // Bloch projection requests and results
    std::vector<fdtd::ProjItem> proj;
    fdtd::ProjItem* d_proj = nullptr;
    double* d_proj_out = nullptr;
    // captured graph of a full run
    hipGraphExec_t graph = nullptr;
    int graph_K = 0, graph_B = 0, graph_SB = 0, graph_W = 0;
    bool graph_faster = true;  // the autotuner's verdict on graph replay of its chosen shape
    // kernel timing
    int prof = 0;          // 0: no kernel timing; N >= 1: every N-th launch is timed
    int64_t prof_seen = 0; // launches since timing was enabled
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;  // around each launch of the bulk kernel
    std::vector<int64_t> ev_cells;                       // cells each timed launch owns
    AdjointState adj;
    std::string err;
};

// Steps of the next streaming launch: at most K and at most `left`, rounded
// down to a step count the kernels are instantiated for (1..8, 10, 12).
inline int fdtd_launch_steps(int K, int left) {
    const int k = K < left ? K : left;
    return (k > 8 && (k & 1)) ? k - 1 : k;
}

// shared helpers (fdtd_host.hip)
int fdtd_fail(fdtd_ctx* c, int code, const std::string& msg);
// the bulk TMz (TEz) items of L in the layout the context launches (c->W),
// with the launcher for them
hipError_t fdtd_launch_bulk_tm(const fdtd_ctx* c, int k, const fdtd::InstDev* insts, const ItemList* L, int n0,
                               int cur, hipStream_t s, bool rec = false, int hslot0 = 0);
hipError_t fdtd_launch_bulk_te(const fdtd_ctx* c, int k, const fdtd::InstDev* insts, const ItemList* L, int n0,
                               int cur, hipStream_t s);
int fdtd_enqueue_steps(fdtd_ctx* c, int n_steps, int K, int B);
// device work list of one (K, band) configuration over every instance (built
// on first use)
ItemList* fdtd_item_list(fdtd_ctx* c, int K, int B);
// field set holding instance q's current state
int fdtd_inst_cur(const fdtd_ctx* c, int q);
void fdtd_gram(double wdt, int n0, int n1, double g[3], double off);
// sample time of the monitored field after step n, in dt, by polarisation
double fdtd_sample_offset(int pol);
// tone-fit amplitudes F_m (complex, per propagating order) of both monitor
// lines of every instance, after the projection kernel; synchronizes
int fdtd_order_amplitudes(fdtd_ctx* c, std::vector<std::vector<double>>& f_re,
                          std::vector<std::vector<double>>& f_im, std::vector<double>& finc2);

#define FDTD_HIPCHK(ctx, expr)                                                                       \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return fdtd_fail(ctx, FDTD_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)
