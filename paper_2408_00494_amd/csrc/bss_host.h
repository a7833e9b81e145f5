// bss_host.h -- host-side helpers shared by the context API and the serving runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "../../include/bssmppi.h"
#include "bss_internal.h"

namespace bss {

// Record a formatted message for bss_last_error and return `st`.
bss_status fail(bss_status st, const char* fmt, ...);
// BSS_E_DEVICE with the HIP error string.
bss_status device_fail(hipError_t e, const char* what);
const char* last_error_message();

// Back-off coefficient nu of a risk level (Remark 1): Gaussian upper-tail quantile, or Cantelli's
// sqrt((1 - delta) / delta) when the parameter set selects it.
double gaussian_backoff(double delta);
double backoff_of(const bss_params& p);

ScoreF64 make_score(const bss_params& p);
CarF32 make_car(const bss_params& p);
Car8F32 make_car8(const bss_params& p);
size_t align256(size_t x);

// Descriptor of a parameter set: sizes, Philox key, model and score constants.  Launch shape,
// state fields and buffer pointers are left zero for the caller to fill.
InstanceDesc make_desc(const bss_params& p);

// The sampled controls are repaired (the per-sample shield) unless only the update is repaired.
bool samples_shielded(const bss_params& p);
// Kernel variant flags of an instance (half-space constraints add the CON flag to the plain or
// split variant, or, with the repair or the re-sampling, to the generic one).
bool launch_shield(const bss_params& p);
bool launch_resample(const bss_params& p);
// The automatic shape's eight particles per lane for the repair: the plain shielded variant only
// (the generic one, which the constraints or the re-sampling select, runs out of registers at
// eight).
bool shape_for_shield(const bss_params& p);

// Solve blocks of one instance: (inst, k0) for k0 = 0, 256/L, 2*256/L, ... < K.
void append_blocks(std::vector<BlockDesc>& out, int inst, int K, int lanes);

}  // namespace bss
