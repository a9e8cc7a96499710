// Euclidean-time overlaps of a slot's configuration (paper: App. E); the
// kernel is in qsg_overlaps.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qsg {

// The plane width the kernel supports and the tau values one launch takes
// (passed by value).
constexpr uint32_t kOvMaxL = 32;
constexpr uint32_t kOvMaxTaus = 64;
struct TauList {
    uint32_t n;
    uint32_t t[kOvMaxTaus];
};

// Adds the contributions of n_slots consecutive slots (slot_spins: the first
// one's [L_tau][L][L] words) for taus to out: per slot int64 q2 [64][n],
// q4 [64][n], A [n][L], B [n][L].
hipError_t launch_tau_overlaps(const uint64_t* slot_spins, uint32_t n_slots, uint32_t L,
                               uint32_t Ltau, const TauList& taus, int64_t* out, hipStream_t s);

}  // namespace qsg
