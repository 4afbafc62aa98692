// Open electrodes (kmc_set_electrodes): structures shared by the host library
// (kmc_api.cpp) and the boundary-bond kernel (kmc_electrode.hip).  Not part of
// the public ABI.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "kmc_internal.h"

namespace kmc {

// Reservoirs of one device: the grounded one behind site 0 (virtual site -1)
// and the biased one behind site L-1 (virtual site L).
struct Electrode {
    int32_t open, pad_;
    double ea_ground, mu_ground;   // eV
    double ea_bias, mu_bias;       // eV
};

// One half-step of boundary bonds, after the interior bonds of the same
// half-step (it reads the half-step's snapshot and changes the new state's
// boundary sites only).
struct ElectrodeArgs {
    const int8_t *occ_in;          // padded snapshot of the half-step
    int8_t *occ_out;               // padded new state
    const DevInfo *devs;
    const int32_t *rail_dev, *rail_idx;
    int64_t rails_total;
    const Electrode *el;           // [D]
    const double *knot_t, *knot_v;
    const double *ktab64;
    const float *ktab32;
    int32_t cutoff;
    double beta, c0, alpha, dt;
    uint32_t key0, key1;
    int64_t n;                     // step
    int32_t h;
    int64_t tally_row;             // n - first step of the tally chunk
    int32_t *tally_net, *tally_dec;
    int32_t n_devices;
    HopArgs::LogBuf log;
};

hipError_t launch_electrodes(const ElectrodeArgs &a, bool fp64, hipStream_t st);

}  // namespace kmc
