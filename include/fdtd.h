/*
 * fdtd.h -- C ABI of the MI355X (gfx950) library for the two-dimensional
 * TMz FDTD method of Lee & Na, "Full-Wave Optical Modeling of Leaf Internal
 * Light Scattering Dynamics with Potential Applications for Early Detection of
 * Foliar Fungal Disease" (arXiv 2512.17132).
 *
 * What the library computes (one "instance" = one monochromatic run):
 *   - a segmented leaf cross-section in the xy-plane, light incident along -y,
 *     periodic in x, absorbing layers at top and bottom (Sec. 2.1, 2.4);
 *   - per-label complex index n + ik mapped to eps_r = n^2 - k^2 and
 *     sigma = 2 n k omega eps0 (eqs. 1-2) and to the semi-implicit loss
 *     coefficients of eq. 17;
 *   - leapfrog Yee updates of Ez, Hx, Hy (TMz, S polarisation, eqs. 18-20) or
 *     of Hz, Ex, Ey (TEz, P polarisation, eqs. 14-16, materials of an edge the
 *     mean of its two cells'), with index wrapping in x (eq. 22), convolutional
 *     PML in y, and a TF/SF normally incident plane wave (eqs. 23-28);
 *   - running-DFT monitors on two rows (Ez for TMz, Ex for TEz) and the
 *     Bloch-order reflectance, transmittance and absorptance of eqs. 29-34;
 *   - the discrete adjoint of a TMz run, giving dL/d(n,k) per label and
 *     dL/d eps_r per pixel for L = sum_i (dL/dR_i R_i + dL/dT_i T_i).
 *
 * Conventions shared by every call:
 *   - Arrays are row-major [j][i], x (i) fastest, j = 0 at the bottom of the
 *     domain.  Ez[j][i] sits at the cell centre ((i+1/2)h, (j+1/2)h) and takes
 *     the material labels[j][i]; Hx[j][i] sits on the bottom edge (y = jh),
 *     Hy[j][i] on the left edge (x = ih).  Hx is zero on the rows y = 0 and
 *     y = ny*h (magnetic walls behind the absorbing layers).
 *   - Fields are FP32 on the device.  Magnetic fields are reported in electric
 *     units, H~ = eta0 * H; electric fields in the units of the source (a unit
 *     amplitude sinusoid injected in the incident-field grid).
 *   - Time step dt = S h / (c sqrt 2) (the CFL bound of Sec. 2.3 scaled by S).
 *     TMz step n advances Ez^{n-1/2} -> Ez^{n+1/2} and then H^n -> H^{n+1};
 *     TEz step n advances Hz^{n-1/2} -> Hz^{n+1/2} and then E^n -> E^{n+1}
 *     (the paper's orders).
 *   - TEz uses the same arrays: the "ez" array holds H~z (cell centres), "hx"
 *     holds Ex (bottom edges, zero on the rows y = 0 and y = ny*h: electric
 *     walls) and "hy" holds Ey (left edges).  The psi arrays hold the layer
 *     state of the Hz update (cell rows) and of the Ex update (edge rows).
 *   - The scattered-field region is every row above j_src (Ez rows > j_src and
 *     Hx rows > j_src); the reflection monitor row j_ref lies there and the
 *     transmission monitor row j_trn below the structure.
 *
 * Ownership and threading:
 *   - The caller owns every input; fdtd_create copies what it needs, so inputs
 *     may be freed when it returns.  Outputs go to caller buffers.
 *   - A context owns all of its device memory until fdtd_destroy.
 *   - All device work is enqueued on the HIP stream given to fdtd_create (NULL:
 *     the library creates its own default-priority stream).  Calls that return
 *     host data synchronize that stream.
 *   - One host thread at a time per context; contexts are independent.  The
 *     only state shared between contexts is the autotuner's table of chosen
 *     launch shapes (see fdtd_autotune), which a lock guards.
 *
 * Errors: every int-returning call returns FDTD_OK (0) or a negative
 * FDTD_E_* code, writes no partial outputs on failure, and records a message
 * for fdtd_last_error.  No C++ exception crosses this interface.
 */
#ifndef FDTD_H
#define FDTD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum fdtd_status {
    FDTD_OK = 0,
    FDTD_E_INVAL = -1,     /* bad sizes, Courant number, row order, options      */
    FDTD_E_MATERIAL = -2,  /* eps_r < 1, k < 0, label >= n_labels, non-vacuum row */
    FDTD_E_NOMEM = -3,     /* device or host allocation failed                     */
    FDTD_E_HIP = -4,       /* a HIP runtime call failed                            */
    FDTD_E_STATE = -5,     /* call out of order (spectra before the run ended...)  */
    FDTD_E_UNSTABLE = -6   /* a monitor accumulator became non-finite              */
};

typedef struct fdtd_ctx fdtd_ctx;

/* One run (Sec. 2.1-2.2): monochromatic (n_freqs = 0), TMz or TEz, with a
 * per-label (n, k) table at lambda0; or broadband (n_freqs >= 1, TMz), with a
 * Gaussian-modulated pulse centred on lambda0, dispersive labels described by
 * a Lorentz-Drude model (Sec. 2.2's auxiliary-differential-equation
 * alternative) and monitors at n_freqs wavelengths.
 * Row order must satisfy n_pml + 1 <= j_trn < j_src < j_ref < ny - n_pml - 1;
 * every row j <= j_trn and j >= j_src must be vacuum (n = 1, k = 0; for a
 * broadband run eps_inf = 1, sigma = 0 and no poles): the absorbing layers,
 * the TF/SF line and both monitors assume it. */
typedef struct {
    int32_t nx, ny;          /* cells; 1 <= nx <= 65536, 2*n_pml + 8 <= ny <= 1048576 */
    int32_t n_pml;           /* absorbing cells at the bottom and at the top, 1..64  */
    int32_t j_src;           /* last total-field Ez row of the TF/SF line           */
    int32_t j_ref;           /* reflection monitor row (scattered field)            */
    int32_t j_trn;           /* transmission monitor row (below the structure)      */
    int32_t n_labels;        /* 1..256 (TEz: 1..16; broadband TMz: 1..64)           */
    int32_t polarization;    /* 0: TMz (S; Ez, Hx, Hy; monitors on Ez, Sec. 2.2-2.6);
                                1: TEz (P; Hz, Ex, Ey, eqs. 14-16; monitors on Ex)     */
    int32_t n_steps;         /* this instance's run length, 1..opts.n_steps; 0: opts.n_steps.
                                A shorter instance leaves the batched launches at its own
                                count (its fields stay at that step); its monitor window
                                is the last half of its own run unless opts.dft_start
                                is set (a broadband run's window starts at step 0
                                unless opts.dft_start is set)                          */
    int32_t n_freqs;         /* 0: monochromatic; 1..256: broadband, monitored at lambdas */
    double dx;               /* grid spacing h in metres, > 0                       */
    double courant;          /* S in (0, 1]                                         */
    double lambda0;          /* vacuum wavelength (broadband: the pulse's centre) in
                                metres, above the grid cutoff                          */
    const uint8_t* labels;   /* host, ny*nx, row-major; values < n_labels           */
    const double* nk;        /* monochromatic: host, n_labels*2: (n, k) per label,
                                n^2-k^2 >= 1; ignored by broadband runs                */
    /* Broadband runs only (n_freqs >= 1; ignored otherwise).  Per label
     * eps(w) = eps_inf + i sigma/(w eps0) + sum_p a_p/(w_p^2 - w^2 - i g_p w)
     * (e^{-i w t} convention; a Lorentz pole has a_p = d_eps_p w_p^2, a Drude
     * term is the pole w_p = 0 with a_p = w_D^2).  Each pole's polarisation
     * obeys P'' + g_p P' + w_p^2 P = eps0 a_p E, stepped by central differences
     * next to the E update.  In TEz an edge's permittivity is the mean of its
     * two cells' at every frequency (mean eps_inf and sigma; the polarisation
     * is half the sum of both cells' pole responses to the edge field).
     * Broadband TEz runs in its own streaming kernel, whose per-row state (16
     * pole values per level) keeps it to short launches: a context holding such
     * instances is tuned over 3, 4, 5 and 6 steps per launch, and launches
     * its band items next to the layers, the source and the monitors before,
     * not beside, its other items (when the two ran concurrently, replays of a
     * captured run differed from direct launches in the last bits). */
    int32_t n_poles;         /* poles per label, 0..2                               */
    int32_t _reserved;       /* 0                                                   */
    const double* model;     /* host, n_labels x (2 + 3 n_poles): eps_inf (>= 1),
                                sigma (S/m, >= 0), then per pole a_p ((rad/s)^2, >= 0),
                                w_p (rad/s, >= 0, w_p dt <= 1), g_p (rad/s, >= 0)       */
    const double* lambdas;   /* host, n_freqs monitor wavelengths in metres, above the
                                grid cutoff                                            */
    double pulse_tau;        /* source exp(-((t - t0)/tau)^2) sin(w0 (t - t0)),
                                w0 = 2 pi c/lambda0: tau in seconds, > 0               */
    double pulse_t0;         /* t0 in seconds, >= 0                                 */
} fdtd_instance;

/* Options shared by all instances of a context.  Zero-initialised fields take
 * the documented defaults. */
typedef struct {
    int32_t n_steps;          /* time steps of a full run (the longest instance), >= 1  */
    int32_t dft_start;        /* first step whose Ez^{n+1/2} enters the monitors, for
                                 every instance; <= 0: the last half of each instance's
                                 own run                                                 */
    double ramp_periods;      /* raised-cosine source ramp, in periods; <= 0: 5          */
    int32_t kernel;           /* 0: temporally blocked streaming kernel (default);
                                 1: plain per-step E and H kernels                       */
    int32_t t_block;          /* steps per launch of the streaming kernel, 1..8, 10
                                 or 12; 0: chosen by the autotuner                       */
    int32_t band_rows;        /* rows per work item of the streaming kernel; 0: tuned   */
    int32_t checkpoint_every; /* forward checkpoints for fdtd_backward: 0 none (backward
                                 unavailable); >= n_steps: one segment, whose Ez history
                                 (every step, ny*pitch*4 B each) the recorded run writes
                                 itself, so that the backward replays nothing; -1: that
                                 single segment when its history takes at most half the
                                 device memory free to the adjoint, else checkpoints about
                                 sqrt(n_steps) steps apart, rounded to a multiple of both
                                 launch lengths (forward t_block and adj_t_block) when that
                                 stays within a factor 1.5 of it, so that no segment ends
                                 in a short launch; else that many steps apart (each
                                 backward segment is replayed from its checkpoint)        */
    int32_t literal_orders;   /* 1: paper-literal R/T (continuous cutoff, unit weights) */
    int32_t use_graph;        /* 1: replay full runs from a captured HIP graph (after
                                 fdtd_autotune: only if it timed graph replay of its
                                 shape faster than direct launches)                      */
    int32_t adj_t_block;      /* steps per launch of the streaming adjoint kernel, 1..8,
                                 10 or 12; 0: the library's default                      */
    int32_t special_rows;     /* rows per work item of the streaming kernel's bands next to
                                 the absorbing layers, the TF/SF line and the monitors
                                 (1..16); 0: 16, or the autotuner's choice of 4, 8, 12
                                 or 16 when it runs                                      */
    int32_t adj_band_rows;    /* rows per work item of the streaming adjoint kernel; 0: as
                                 band_rows                                               */
    int32_t bulk_columns;     /* columns per work item of the streaming kernel's bulk bands
                                 of monochromatic instances (TMz and TEz): 64 (one wave,
                                 which recomputes the 2 t_block columns at its edges) or
                                 256 (a workgroup of four waves that exchange their edge
                                 columns through LDS, recomputing only the workgroup's);
                                 0: 64, or the autotuner's choice when it runs. Results
                                 are identical either way                                */
    int32_t _reserved[2];
} fdtd_opts;

/* Creates a context for n_inst instances run together (a batched launch when
 * n_inst > 1; instances may differ in every size).  Validates all inputs,
 * computes per-label coefficients (eqs. 1-2, 17), absorbing-layer profiles, the
 * incident-field table of the TF/SF line (eqs. 23-28, from a 1D vacuum grid with
 * the same h and dt) and the monitor phasors, copies labels and tables to the
 * device, and zeroes all fields.  stream: a hipStream_t or NULL.
 * Returns FDTD_E_INVAL / FDTD_E_MATERIAL on bad input before touching the GPU.
 * *out is set only on success. */
int fdtd_create(const fdtd_instance* inst, int32_t n_inst, const fdtd_opts* opts,
                void* stream, fdtd_ctx** out);

/* Enqueues all remaining steps of the run (to opts.n_steps) on the stream:
 * the leapfrog time loop of Sec. 2.3 (TMz eqs. 18-20, TEz eqs. 14-16), each
 * step with the periodic wrap of eq. 22, the absorbing layers of Sec. 2.4,
 * the TF/SF injection of Sec. 2.5 (eqs. 23-28) and the running-DFT monitor
 * sums of eqs. 29-30.
 * record = 1 also stores the forward checkpoints that fdtd_backward needs
 * (requires opts.checkpoint_every != 0, a run starting at step 0 and TMz
 * instances only: FDTD_E_INVAL otherwise).
 * Asynchronous; errors of the device work surface in the next synchronizing
 * call. */
int fdtd_run(fdtd_ctx* ctx, int32_t record);

/* Enqueues the next n steps (n >= 0, not past opts.n_steps) of the time loop
 * that fdtd_run describes (Sec. 2.3-2.6); FDTD_E_INVAL past the end. */
int fdtd_step(fdtd_ctx* ctx, int32_t n);

/* For callers that cannot allocate device memory during stepping (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * fdtd_step whose streaming launches read their work-item lists from a fixed
 * array in the library's device memory (32768 items, 1 MiB per device, held
 * until the process ends) instead of lists allocated on first use.  It calls
 * no hipMalloc, hipFree or allocating library routine; each launch's list is
 * copied (host to device, on the context's stream) into the array when it
 * differs from the previous launch's.  Fields and monitors are bit-identical
 * to fdtd_step's.  Needs a settled launch shape: opts.t_block and
 * opts.band_rows > 0, or an earlier fdtd_autotune, fdtd_run or fdtd_step on
 * the context (FDTD_E_STATE otherwise); FDTD_E_INVAL, with no step enqueued,
 * when a launch needs more than 32768 work items (use fdtd_step) or n is out
 * of range.  Kernel timing (fdtd_set_profiling) does not cover these launches.
 * The array is shared by every context and host thread using the library on
 * that device and keeps only the last list copied into it: calls that overlap
 * on one device (other streams or threads) race. */
int fdtd_step_noalloc(fdtd_ctx* ctx, int32_t n);

/* Zeroes fields, absorbing-layer state, monitors and the step counter, so the
 * next fdtd_run starts a fresh run with the same inputs.  Asynchronous. */
int fdtd_reset(fdtd_ctx* ctx);

/* Steps completed so far. */
int fdtd_steps_done(const fdtd_ctx* ctx, int32_t* n);

/* Reflectance, transmittance and absorptance of every instance (eqs. 29-34):
 * tone fit of the monitor sums over the window, Bloch projection onto the
 * propagating orders, flux-weighted sums, A = 1 - R - T.  Each output has
 * n_inst entries; any may be NULL.  Synchronizes the stream.
 * FDTD_E_STATE if the run has not reached opts.n_steps; FDTD_E_UNSTABLE if a
 * monitor became non-finite. */
int fdtd_spectra(fdtd_ctx* ctx, double* R, double* T, double* A);

/* Broadband instances: R, T, A at each of the instance's n_freqs monitor
 * wavelengths (n_freqs entries each, any may be NULL).  The monitor sums over
 * the window are the Fourier transform of the monitored field (the pulse must
 * have left the domain by the end of the run); they are projected onto the
 * propagating orders of each wavelength, weighted by the discrete flux and
 * divided by the transform of the incident wave on the TF/SF row.
 * fdtd_spectra reports NaN for broadband instances.  FDTD_E_INVAL for a
 * monochromatic instance; otherwise as fdtd_spectra.  Synchronizes. */
int fdtd_broadband_spectra(fdtd_ctx* ctx, int32_t inst, double* R, double* T, double* A);

/* Per-order detail for one monochromatic instance: for up to max_orders propagating orders,
 * m (Bloch index), w (flux weight) and the reflected / transmitted power of
 * that order relative to the incident power.  *n_orders receives the number of
 * propagating orders (which may exceed max_orders).  Synchronizes. */
int fdtd_orders(fdtd_ctx* ctx, int32_t inst, int32_t max_orders, int32_t* m, double* w,
                double* ref_pow, double* trn_pow, int32_t* n_orders);

/* Host copies of the current fields of one instance, ny*nx floats each
 * (row-major, no padding; the Yee positions of eq. 13 and Sec. 2.3 as in the
 * conventions above: TMz Ez, H~x, H~y; TEz H~z, Ex, Ey); any pointer may be
 * NULL.  Synchronizes. */
int fdtd_fields(fdtd_ctx* ctx, int32_t inst, float* ez, float* hx, float* hy);

/* Host copy of one instance's monitor sums as FP64, [4][nx]:
 * sum Ez(j_ref) cos, sum Ez(j_ref) sin, sum Ez(j_trn) cos, sum Ez(j_trn) sin,
 * each the compensated FP32 sum plus its compensation term; a broadband
 * instance gives n_freqs such blocks, one per monitor wavelength.
 * Synchronizes. */
int fdtd_monitors(fdtd_ctx* ctx, int32_t inst, double* mon);

/* Overwrites the current state of one instance from host arrays (ny*nx floats
 * each, normalised units as in fdtd_fields; psi arrays are the absorbing-layer
 * auxiliary fields on full-size grids and are read only on layer rows; NULL
 * leaves a field unchanged).  Hx rows 0 are forced to zero.  For tests and for
 * restarting from saved state.  Synchronizes. */
int fdtd_set_fields(fdtd_ctx* ctx, int32_t inst, const float* ez, const float* hx,
                    const float* hy, const float* psi_ez, const float* psi_hx);

/* Discrete adjoint of the recorded (TMz) run for L = sum_i dL_dR[i] R_i + dL_dT[i] T_i
 * (dL_dT may be NULL): the gradient of the reflectance and transmittance of
 * eqs. 33-34 with respect to the material inputs of eqs. 1-2, for the
 * inversion that Sec. 5 names as the method's next use.  Recomputes each
 * checkpoint segment forward, then steps the exact transpose of the forward
 * recurrence (eqs. 17-20 with the absorbing layers, the wrap and the TF/SF
 * line) backwards in time.
 * grad_nk (host, sum of n_labels*2 over instances, may be NULL) receives
 * dL/dn, dL/dk per label; grad_eps_pixel (device pointer to sum of ny*nx floats
 * over instances, may be NULL) receives dL/d eps_r per pixel with sigma held
 * fixed.  Requires a completed fdtd_run(ctx, 1).  Synchronizes. */
int fdtd_backward(fdtd_ctx* ctx, const double* dL_dR, const double* dL_dT, double* grad_nk,
                  float* grad_eps_pixel);

/* Averages over groups of runs (Sec. 2.1: the TE and TM results of a point
 * are combined for unpolarised light; Sec. 4 and 4.2: the spectra of the
 * slices of a cross-section and of both polarisations are averaged).  Run i
 * (0 <= i < n_runs), with reflectance R[i] and transmittance T[i] (as from
 * fdtd_spectra or fdtd_broadband_spectra, possibly of several contexts),
 * belongs to group group[i] (0 <= group[i] < n_groups).  For every group g,
 * R_out[g] and T_out[g] are the unweighted means of its members' R and T, summed
 * in run order, and A_out[g] = 1 - R_out[g] - T_out[g] (outputs n_groups each;
 * any may be NULL).  Host arrays; needs no context and no device.
 * FDTD_E_INVAL, with nothing written, for n_runs < 1, n_groups < 1, a null
 * input, a group index out of range, a group without members or a non-finite
 * R or T; the message is read with fdtd_last_error(NULL). */
int fdtd_combine_spectra(const double* R, const double* T, int32_t n_runs, const int32_t* group,
                         int32_t n_groups, double* R_out, double* T_out, double* A_out);

/* Launch configuration in use: kernel, t_block, band_rows, work items per
 * launch (one per wave of 64 columns), device bytes held by the context, the
 * number of cells whose update the bulk kernel (the streaming kernel's
 * branch-free variant, or the plain sweeps) performs per launch, the rows of
 * a special band, and the columns of a bulk work item (opts.bulk_columns).
 * Any pointer may be NULL. */
int fdtd_get_config(const fdtd_ctx* ctx, int32_t* kernel, int32_t* t_block, int32_t* band_rows,
                    int32_t* items, int64_t* device_bytes, int64_t* lean_cells, int32_t* special_rows,
                    int32_t* bulk_columns);

/* Times candidate (t_block, band_rows) pairs of the streaming kernel on this
 * context's instances for trial_steps steps each, with bulk work items of 64
 * and of 256 columns (unless opts.bulk_columns fixes them or the context holds
 * no monochromatic instance), then the three fastest again with
 * special bands of 4, 8, 12 and 16 rows (unless opts.special_rows fixes them),
 * keeps the fastest, and resets the context.  Writes the winner's throughput
 * in cell-updates per second to *best_rate (may be NULL).  Synchronizes.
 * trial_steps <= 0 picks the trial length and first looks the shape up in a
 * process-wide table of earlier choices (kept under a lock, so contexts on
 * different host threads may tune at once), keyed by the device's
 * architecture and compute-unit count, by each instance's grid, layer
 * depth, source and monitor rows and kind of run, and by the options that
 * narrow the search (t_block, band_rows, special_rows, bulk_columns,
 * use_graph); a hit skips the trials (best_rate 0).  fdtd_run and fdtd_step call it that way when opts leave
 * t_block or band_rows at 0. */
int fdtd_autotune(fdtd_ctx* ctx, int32_t trial_steps, double* best_rate);

/* Kernel timing.  enable = 0 turns it off; enable = N >= 1 brackets every N-th
 * launch of the bulk stepping kernel (see fdtd_get_config), starting with the
 * first after this call, by HIP events on the context's stream (N = 1: every
 * launch; a larger N samples the launches, and the events' own cost in the
 * stream falls with it).  fdtd_kernel_time returns the summed event time (ms)
 * and the number of timed launches since enabling; their ratio is the average
 * launch duration.  Timing disables graph replay.  Synchronizes. */
int fdtd_set_profiling(fdtd_ctx* ctx, int32_t enable);
int fdtd_kernel_time(fdtd_ctx* ctx, double* total_ms, int64_t* launches);

/* Frees all device and host memory of the context; NULL is a no-op. */
void fdtd_destroy(fdtd_ctx* ctx);

/* Message of the last failed call on ctx (or of the last failed fdtd_create in
 * this thread when ctx is NULL); valid until the next call on ctx. */
const char* fdtd_last_error(const fdtd_ctx* ctx);

/* Static one-line description of a status code ("unknown status" for any
 * other value). */
const char* fdtd_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* FDTD_H */
