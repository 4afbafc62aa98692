// Internal structures shared by the host library (kmc_api.cpp) and the HIP
// kernels (kmc_kernels.hip).  Not part of the public ABI.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace kmc {

constexpr int kMaxKnots = 64;
constexpr int kMaxRailRange = 4;
constexpr int kMaxSites = 4096;          // sites per rail
constexpr int kChunkSites = 16;          // sites per lane chunk (one 16-byte load)
constexpr int kBlock = 256;              // threads per workgroup of the hop kernel
constexpr int kTileSites = 4096;         // default padded sites per hop-kernel tile
constexpr int kTallySteps = 1024;        // steps per tally chunk
constexpr int kDeciles = 10;
constexpr int kClasses = 128;            // barrier classes in bits 1..7 of a state byte
constexpr int kLdsTableMax = 2048;       // kernel-table entries kept in LDS

// Per-device description, resident in the workspace.
struct DevInfo {
    int32_t rails, sites, pitch;         // pitch = sites rounded up to 16
    int32_t n_knots;
    int64_t off;                         // unpadded offset (caller layout)
    int64_t off_pad;                     // padded offset (internal buffers)
    int64_t n_set;                       // step at which the protocol was installed
    int64_t row0;                        // global index of the device's first rail
    double ea_min;                       // minimum barrier of the device, eV
    double ea_step;                      // barrier class width: class q covers
                                         // [ea_min + q*ea_step, ...), eV
    double coul_bound;                   // |dE_coul| <= coul_bound for any state, eV
    int32_t n_nbr;                       // distinct rail offsets (incl. 0)
    int8_t nbr_off[2 * kMaxRailRange + 1];   // rail offsets in [-m, m]
    int8_t nbr_dist[2 * kMaxRailRange + 1];  // minimal-image distance per offset
    int32_t pad_;
};

// One workgroup's work: rails [r0, r0 + nr) of device d.
struct Tile {
    int32_t d, r0, nr, pad_;
};

// Tile of the persistent kernel: rails [r0, r0 + nr) of device d, and the
// tiles owning the rails just below and just above it (itself when the device
// is a single tile).
struct PTile {
    int32_t d, r0, nr, prev, next, pad_;
};

constexpr int kPubSlots = 2 * kTallySteps + 1;  // publication slots per tile: one per state of a launch
constexpr int kPMaxBlock = 1024;         // threads per workgroup, persistent kernel
constexpr int kWaveTilesPerWG = 4;       // wave kernel: tiles (one wavefront each) per workgroup
constexpr int kSnapSlots = 64;           // wave kernel: edge-row snapshots per tile in a ring
constexpr int kTicketBuckets = 64;       // wave kernel: end-of-launch counters (one 128-byte line each)
constexpr int kTicketStride = 32;        // uint32 per counter line
constexpr int kTicketWords = (kTicketBuckets + 1) * kTicketStride;  // the buckets, then the total

// Step bookkeeping of one launch, passed by value (the host keeps the step
// counter).
struct Ctl {
    int64_t n_base;        // step index of the launch's first step (chunk start)
    int64_t tally_base;    // step index of row 0 of the tally chunk buffers
    int64_t call_base;     // first step of the current kmc_run_steps call
    int32_t *net_out;      // caller buffers of the current call (may be null)
    int32_t *dec_out;
};

// End of a tally chunk (either a kernel of its own or the tail of the wave
// kernel): the per-step tally deltas of devices [d0, d1) are turned into the
// caller's rows and the running totals.
struct FinishArgs {
    Ctl ctl;
    int32_t *tally_net;        // [kTallySteps][D] net hops per step (cleared here)
    int32_t *tally_dec;        // [kTallySteps][D][10] decile deltas per step (cleared here)
    int64_t *dec_run;          // [D][10] decile counts before the chunk, advanced here
    int64_t *net_total;        // [D] running net-hop totals
    int32_t n_devices, d0, d1, steps;
};

// Recording of the accepted hops of a run of steps, for the score replay:
// the hops of half-step h of step n (n0 <= n < n0 + n_hs / 2) go to list
// 2 (n - n0) + h, cap entries of (device, rail, s, dir) each (dir 0: the ion
// at s moves to s + 1), with the list's count (which may exceed cap: the list
// then overflowed).  buf == nullptr: nothing is recorded.
struct HopRecord {
    uint4 *buf;
    int64_t *count;            // [n_hs]
    int64_t cap, n0, n_hs;
};

// Everything the hop kernel needs, passed by value.
struct HopArgs {
    const int8_t *occ_in;      // padded internal state, read (Jacobi snapshot); one bit per site in the recorded replay
    int8_t *occ_out;           // padded internal state, written
    const DevInfo *devs;
    const Tile *tiles;
    int32_t n_tiles;
    const double *knot_t;      // [D][kMaxKnots]
    const double *knot_v;
    const void *ea;            // null or per-site barrier (float or double)
    const double *ktab64;      // [(m+1)][(c+1)] kernel table, binary64
    const float *ktab32;       // same, rounded once to binary32
    int32_t cutoff, rail_range;
    double ea_scalar, beta, c0, alpha, dt;
    uint32_t key0, key1;
    Ctl ctl;
    int32_t *tally_net;        // [kTallySteps][D]
    int32_t *tally_dec;        // [kTallySteps][D][10]  (deltas)
    int32_t n_devices;
    struct LogBuf { int64_t *count; void *entries; int64_t cap; } log;
    HopRecord record;          // forward kernels: where accepted hops are recorded
    int32_t step_in_chunk;
    int32_t h;
    // score replay only (hop_half_step<..., 1>)
    int64_t n_abs;             // step index of the launch
    double nu0, kappa;
    const void *rec;           // Coulomb part of each candidate bond's dE in the half-step's state,
                               // path precision, [device offset + r L + (s odd ? (L + 1) / 2 : 0) + s / 2]
    uint4 *hops;               // accepted hops of the half-step (device, rail, s, dir), hop_cap entries
    int64_t *hop_ctl;          // [h] entries appended by the half-steps of parity h
    int64_t hop_cap;
    const double *score_w;     // [D] weights of this step's decisions
    double *score_grad;        // [D][4] accumulators (Ea shift, nu0, kappa, alpha)
    // dense-potential decisions only (dense_decide)
    const float *phi;          // [total rails][phi_row] potential of the half-step's snapshot
    int64_t phi_row;
    float k10;                 // K(1, 0) in binary32
    const Tile *dtiles;        // decision tiles: whole rails of one device per workgroup
    int32_t n_dtiles;
    // recorded replay only (replay_logged): the half-step's recorded hops
    const uint4 *rec_hops;
    const int64_t *rec_count;
};

// Coulomb part of every candidate bond's energy change, for the score replay,
// and its recomputation where the accepted hops of a half-step changed it.
struct PhiArgs {
    const int8_t *occ;         // padded state (bit 0 = occupied): read by full recomputations
    int32_t occ_bits;          // 1: occ holds one bit per site (site at padded index i: bit i % 8 of byte i / 8)
    const DevInfo *devs;
    int32_t n_devices;
    const double *ktab64;      // [(m+1)][(c+1)] kernel table
    int32_t cutoff, rail_range;
    double k01;                // K(1, 0) in binary64 (0 when the cutoff is 0)
    void *ec;                  // path precision, [device offset + r L + (s odd ? (L + 1) / 2 : 0) + s / 2]
    const uint4 *hops;         // (device, rail, s, dir): dir 0 moves the ion at s up
    const int64_t *hop_count;  // entries appended by the half-step (may exceed hop_cap)
    int64_t hop_cap;
    int64_t known_count;       // >= 0: the count, known to be at most hop_cap (hop_count is not read)
};

// Dense potential (MFMA): every site's Coulomb potential of one state.
constexpr int kDenseRails = 128;         // rails per workgroup tile of the dense kernel
constexpr int kDenseMaxSites = 1024;     // sites per rail supported by the dense path

struct DenseArgs {
    const int8_t *occ;        // padded internal state (bit 0 = occupied)
    const DevInfo *devs;
    const Tile *tiles;        // rails [r0, r0 + nr) of device d, nr <= kDenseRails
    int32_t n_tiles;
    const void *ktiles;       // [m+1][2 nb - 1][hi, lo][q][64 lanes] 16-byte MFMA B fragments
    int32_t nb;               // 32-site blocks per rail (multiple of 4)
    int32_t rail_range;
    float *phi;               // output rows
    int64_t phi_row;          // floats per output row
    int32_t sites;            // valid sites per row (columns >= sites are not written)
};

// Arguments of the persistent kernel (several steps per launch, each
// workgroup keeps its tile in LDS and talks to its two neighbours only).
struct PArgs {
    int8_t *occ;               // padded state: read at launch start, written at the end
    const DevInfo *devs;
    const PTile *tiles;
    int32_t n_tiles;
    const double *knot_t;
    const double *knot_v;
    const void *ea;
    const double *ktab64;
    const float *ktab32;
    int32_t cutoff, rail_range;
    double ea_scalar, beta, c0, alpha, dt;
    uint32_t key0, key1;
    Ctl ctl;
    int32_t *tally_net;
    int32_t *tally_dec;
    int32_t n_devices;
    HopArgs::LogBuf log;
    HopRecord record;
    uint64_t *pub;             // edge-rail publications, pub_stride words per tile
    int64_t pub_stride;        // block tiles: a slot per state; wave tiles: a word per state, then
                               // the snapshot ring
    uint64_t epoch;
    int32_t n_steps;
    int32_t *status;           // nonzero: a neighbour wait timed out
    int32_t spin_limit;        // polls before a neighbour wait is declared hung (0: at once)
    // wave kernel only: the launch ends its chunk itself.  Every tile also
    // writes its rails to the caller's occupancy (occ_user, unpadded layout),
    // and, when ticket is set, the last tile to finish (counted per bucket of
    // tiles, then over the buckets: kTicketWords counters) runs the chunk's
    // tally finish for the launch's devices [fin.d0, fin.d1) and clears the
    // counters.
    int8_t *occ_user;
    uint32_t *ticket;
    FinishArgs fin;
};

}  // namespace kmc
