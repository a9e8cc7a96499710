// Finite-L_tau correlation estimates from two transforms (qsg_corr_mix.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qsg {

// out[3i + {0, 1, 2}] = sum_e w[3e + {0, 1, 2}] R_e^2 with
// R_e = (1 - w_odd[i]) We[mask[e]] / We[0] + w_odd[i] Wo[mask[e]] / Wo[0],
// for i < n_weights (device arrays; one block per weight).
hipError_t launch_tm_corr_mixed(const double* We, const double* Wo, const uint32_t* mask,
                                const double* w, uint32_t n, const double* w_odd,
                                uint32_t n_weights, double* out, hipStream_t s);

}  // namespace qsg
