// Host-callable launchers of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "fdtd_device.h"

namespace fdtd {

hipError_t launch_plain_step(const InstDev& d, int n, int cur, hipStream_t s);
// the plain TMz H sweep alone
hipError_t launch_plain_h(const InstDev& d, int n, int cur, hipStream_t s);
// the plain TEz Hz sweep alone
hipError_t launch_plain_te_h(const InstDev& d, int n, int cur, hipStream_t s);
// one step of a broadband instance (InstDev::n_freqs > 0) in place on field
// set cur: the dispersive E and the H sweep; the monitor rows' field goes to
// capture slot `slot` (0 .. kMaxTBlock-1) of InstDev::cap
hipError_t launch_plain_step_broadband(const InstDev& d, int n, int cur, int slot, hipStream_t s);
// monitor sums of a broadband instance over K consecutive steps from n0, whose
// monitor-row fields are in capture slots 0 .. K-1 of InstDev::cap (left by a
// streaming launch's special items or by K plain steps)
hipError_t launch_monitor_bb(const InstDev& d, int n0, int K, hipStream_t s);
// the streaming kernel of broadband TMz instances
hipError_t launch_tblock_bb(int K, bool special, const InstDev* insts, const WorkItem* items, int n_items, int n0,
                            int cur, hipStream_t s);
// the streaming kernel of broadband TEz instances: their special and lean
// items in one launch
hipError_t launch_tblock_bt(int K, const InstDev* insts, const WorkItem* special, int n_special, const WorkItem* lean,
                            int n_lean, int n0, int cur, hipStream_t s);
// The TMz streaming kernel, one item (64 columns) per wave: special, the thin
// bands near the layers, the source and the monitors; otherwise bulk bands.
// rec: the recording variant (Ez of every step to InstDev::hist, slot hslot0
// for step n0).
hipError_t launch_tblock(int K, bool special, const InstDev* insts, const WorkItem* items, int n_items, int n0,
                         int cur, hipStream_t s, bool rec = false, int hslot0 = 0);
// The TMz bulk bands with one item of kWgColumns columns per workgroup, whose
// waves exchange their edge columns (ItemList::wg).
constexpr int kWgColumns = 256;
hipError_t launch_tblock_wg(int K, const InstDev* insts, const WorkItem* items, int n_items, int n0, int cur,
                            hipStream_t s, bool rec = false, int hslot0 = 0);
// the TEz streaming kernel (instances with InstDev::pol == 1)
hipError_t launch_tblock_te(int K, bool special, const InstDev* insts, const WorkItem* items, int n_items, int n0,
                            int cur, hipStream_t s);
// its bulk bands with one item of kWgColumns columns per workgroup (ItemList::wg_te)
hipError_t launch_tblock_te_wg(int K, const InstDev* insts, const WorkItem* items, int n_items, int cur,
                               hipStream_t s);
hipError_t launch_project(const InstDev* insts, const ProjItem* items, int n_items, double* out, hipStream_t s);
hipError_t launch_fill(float* p, size_t n, float v, hipStream_t s);
hipError_t launch_fill_i32(int* p, size_t n, int v, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

}  // namespace fdtd
