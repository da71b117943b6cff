// Launch wrappers of the stage kernels for the host-side sanitizer build of
// the C ABI (tests/test_host_sanitized.py): that build leaves the kernel
// source out, and none of the host paths it drives reaches a launch, so
// each wrapper only reports that no device is there.
#include "swe_host.h"

namespace swe {
hipError_t launch_stage(int, bool, const Dom &, const Tiling &, int, double, hipStream_t, hipEvent_t, hipEvent_t)
{
    return hipErrorNoDevice;
}
hipError_t launch_ensemble(int, bool, bool, bool, const EnsMember *, const EnsItem *, EnsCtrl *, int, int, int,
                           hipStream_t, hipEvent_t, hipEvent_t)
{
    return hipErrorNoDevice;
}
hipError_t launch_cfl(const Dom &, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_ctrl_reset(Ctrl *, double, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_frame_static(const Dom &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_frame_state(const Dom &, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_set_t_end(Ctrl *, double, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_policy_reset(Ctrl *, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_diagnostics(const Dom &, hipStream_t) { return hipErrorNoDevice; }
int stage_waves_per_simd(int, bool, bool) { return 4; }
int ensemble_waves_per_simd(int, bool, bool) { return 4; }
}  // namespace swe
