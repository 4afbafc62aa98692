// Structures of the fixed-point potential path (kmc_phifix.hip), shared with
// the host library (kmc_api.cpp).  Not part of the public ABI.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "kmc_internal.h"

namespace kmc {

constexpr int kPhiMaxSites = 2048;  // sites per rail of the fixed-point path

// Potential of every site in fixed point (units of 2^-frac_bits V), kept up
// to date hop by hop, or computed from scratch for every rail (`full` set, or
// a hop list that overflowed).
struct PhiFixArgs {
    const int8_t *occ;         // padded state (bit 0 = occupied)
    const DevInfo *devs;
    const int32_t *rail_dev, *rail_idx;  // global rail -> device, rail within it
    int64_t rails_total;
    const int64_t *kfix;       // [(m+1)][(c+1)] round(K 2^frac_bits), kfix[0][0] = 0
    int32_t cutoff, rail_range;
    int64_t *phi;              // padded layout (off_pad + r pitch + s), or the caller's
                               // layout (off + r L + s) when out_unpadded
    int32_t out_unpadded;
    const uint4 *hops;         // (device, rail, s, dir): dir 0 moves the ion at s up
    const int64_t *hop_count;  // entries appended by the half-step (may exceed hop_cap)
    int64_t hop_cap;
    int32_t full;              // recompute every rail whatever the hop list holds
};

// What the decision kernel needs beyond HopArgs (whose hops / hop_ctl /
// hop_cap receive the accepted hops; the state is updated in place).
struct PhiFixDecide {
    const int64_t *phi;        // padded layout
    int32_t frac_bits;
    int64_t k10;               // K(1, 0) in the same units
};

hipError_t launch_phifix_decide(const HopArgs &a, const PhiFixDecide &x, hipStream_t st);
hipError_t launch_phifix_update(const PhiFixArgs &a, hipStream_t st);
hipError_t launch_phifix_export(const int64_t *phi_pad, int64_t *out, const DevInfo *devs, const int32_t *rail_dev,
                                const int32_t *rail_idx, int64_t rails_total, hipStream_t st);

}  // namespace kmc
