// Private host-side definitions shared by the C-ABI sources.
#pragma once

#include <map>
#include <string>
#include <utility>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/swe.h"
#include "swe_device.h"

namespace swe {
hipError_t launch_stage(int stage, bool proj, const Dom &d, const Tiling &T, int parity, double dt_fixed,
                        hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_ensemble(int stage, bool proj, bool w10, bool comp, const EnsMember *mem, const EnsItem *items,
                           EnsCtrl *ec, int parity, int chunk, int nblocks, hipStream_t s, hipEvent_t ev0,
                           hipEvent_t ev1);
hipError_t launch_cfl(const Dom &d, int slot, hipStream_t s);
hipError_t launch_ctrl_reset(Ctrl *c, double t, int slot, hipStream_t s);
hipError_t launch_frame_static(const Dom &d, hipStream_t s);
hipError_t launch_frame_state(const Dom &d, int parity, hipStream_t s);
hipError_t launch_set_t_end(Ctrl *c, double te, hipStream_t s);
hipError_t launch_policy_reset(Ctrl *c, int parity, hipStream_t s);
hipError_t launch_diagnostics(const Dom &d, hipStream_t s);
int stage_waves_per_simd(int stage, bool proj, bool comp);
int ensemble_waves_per_simd(int stage, bool proj, bool comp);

int set_error(int code, const std::string &msg);  // records the message for swe_last_error
// A member destroyed while it still belongs to an ensemble: the ensemble
// drops it and refuses further steps.
void ensemble_forget(swe_ensemble *e, swe_domain *d);
// Device workspace of an ensemble whose members have these (nx, ny) shapes.
size_t ensemble_bytes_for_shapes(const std::vector<std::pair<int, int>> &shapes, int rows_per_wave);

struct Layout {
    size_t eta, hu, hv, eta1, hu1, hv1, eta_lo, hu_lo, hv_lo, eta1_lo, hu1_lo, hv1_lo, Hc, f, north, fghost,
        nghost, alpha, bnd_t, bnd, wind_t, wind, ctrl, partials, total;
};

}  // namespace swe

struct swe_domain {
    swe_params p{};
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    char *ws = nullptr;
    swe::Layout L{};
    swe::Dom dom{};
    swe::Tiling T[2]{};   // per stage
    int wps[2] = {3, 3};  // resident waves per SIMD of each stage kernel
    int parity = 0;
    int max_wind = 0, max_bnd = 0;
    bool has_bnd = false;
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;  // (steps, start parity)
    std::vector<hipGraph_t> graph_objs;
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    int64_t timed_steps = 0;
    int cus = 256;
    swe_ensemble *ensemble = nullptr;  // set while the domain belongs to an ensemble
    hipStream_t own_stream = nullptr;  // the domain's stream outside the ensemble
    // Pinned host staging: device-to-host copies land here (a DMA that is
    // complete once the stream is synchronised) before a plain host copy to
    // the caller's pageable memory.
    swe::Ctrl *pinned_ctrl = nullptr;
    float *pinned_state = nullptr;  // 3 planes of nx*ny, allocated on first use
};
