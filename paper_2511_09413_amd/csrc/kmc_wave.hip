// Persistent hop-step kernel with one wavefront per tile.
//
// A tile is whole rails of one device that fit one wavefront: each lane owns
// SPL (16 or 32) consecutive sites of a rail for the whole launch and keeps
// their occupancy as bits in a register, with the next lane's first bit (the
// far end of its last bond) beside them, refreshed by a cross-lane move only
// after half-steps that moved ions.  A half-step therefore needs neither an
// LDS round trip nor a workgroup barrier: the Philox words, the candidate test
// and the exact prefilter (against a per-lane bound from the lowest barrier
// class of the lane's sites) stay in registers, and a wavefront vote finds the
// rare half-steps with prefilter survivors.  Only those build an LDS copy of
// the tile's bits (the Jacobi snapshot) and, when a survivor's Coulomb window
// may cross the tile edge, fetch the neighbouring tiles' edge rails.  The
// workgroup is only a container for kWaveTilesPerWG independent tiles; its one
// barrier precedes the loop.
//
// Cross-tile data.  After every half-step a tile stores one 64-bit word for
// the new state into its per-state array: a tag naming the state (launch
// epoch, half-step) and which snapshot holds that state's edge rails.  Only a
// half-step that changed an edge rail stores a new snapshot (64-bit words:
// 32 occupancy bits plus the tag of the snapshot's state) into a ring of
// kSnapSlots slots.  A snapshot serves every state from its own up to the next
// snapshot's; before a tile reuses a slot it waits until both neighbouring
// tiles have published the state at which the slot's snapshot stops serving,
// after which no neighbour can still ask for it.  A reader polls the state
// word, then the snapshot words, until their tags name what it wants.  Every
// wait is for a state no later than the waiter's own, so the tile furthest
// behind never waits; every wait is also bounded: on time-out the kernel raises
// the status flag, all tiles leave their loops and the host reports the error.
//
// Per bond the work is that of hop_half_step: Philox4x32-10 draw, candidate
// test, exact two-stage prefilter, survivor energy (wavefront-cooperative
// window sum in the same order as the other kernels), Arrhenius probability
// and accept test.
#include <type_traits>

#include "kmc_device.h"
#include "kmc_internal.h"

namespace kmc {

namespace {

constexpr int kWaveWin = 64;         // per-step table entries: one per lane

// Values of a tile that only the rare paths need.  They live in LDS and are
// read again where needed, so that they do not hold scalar registers across
// the loop (which would push the loop's own values into spill code).
struct WaveGeo {
    int32_t R, L, P, lpr, nr, m, W32, e, r0, d, prev, next, ti, single, isolated, cutoff;
    int32_t n_nbr, n_knots;
    int8_t nbr_off[2 * kMaxRailRange + 1];
    int8_t nbr_dist[2 * kMaxRailRange + 1];
    int16_t nr_prev, nr_next;  // rails of the neighbour tiles
    int8_t pad_[2];
    int64_t dv_off, off_pad, n_set, n_base, tally_base;
    double coul_bound;
};
static_assert(sizeof(WaveGeo) % 16 == 0, "LDS tiles stay 16-byte aligned");

// A tile's LDS: its rare-path values, per-device and per-step tables and the
// rare-path buffers.
template <int SPL>
struct WaveLds {
    static constexpr int kBand = 4 * SPL + 16;  // 32-bit words of neighbour rails
    WaveGeo geo;
    double cls_a[kClasses];              // exp(-beta (ea_min + q ea_step)) of the tile's device
    double step_v[kWaveWin];             // bias of the steps of the current window
    double step_g[kWaveWin];             // exp(beta (|alpha V| / L + coul_bound) / 2)
    uint32_t snap[64];                   // each lane's bits at the start of a survivor half-step
    uint32_t band[kBand];                // neighbour rails: prev tile's last m, next tile's first m
    int16_t snap_state[kSnapSlots];      // launch-relative state of each ring slot's snapshot
    unsigned char cls[64 * SPL];         // barrier class of every site, rows at the device pitch
};
static_assert(sizeof(WaveLds<16>) % 16 == 0 && sizeof(WaveLds<32>) % 16 == 0, "LDS tiles stay 16-byte aligned");
static_assert(offsetof(WaveLds<16>, cls) % 16 == 0 && offsetof(WaveLds<32>, cls) % 16 == 0,
              "class rows are written as 16-byte vectors");

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// Poll a published word until its tag is `want` (stored in *out); false after
// `limit` polls (raising the status flag; at once for a limit of 0) or once
// another tile has raised it.
__device__ __forceinline__ bool poll_tag(const uint64_t *p, uint32_t want, int32_t *status, int limit, uint64_t *out) {
    for (int spins = 0;; ++spins) {
        if (spins >= limit) {
            __hip_atomic_store(status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        const uint64_t v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(v >> 32) == want) {
            *out = v;
            return true;
        }
        if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        __builtin_amdgcn_s_sleep(2);
    }
}

// The kernel arguments, read again from the argument segment where a rare
// path needs them (scalar loads); the opaque pointer keeps the compiler from
// hoisting those loads out of the loop.
typedef const __attribute__((address_space(4))) PArgs *KArgs;
__device__ __forceinline__ KArgs kargs() {
    KArgs p = (KArgs)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return p;
}
// An LDS object made opaque in the same way (its loads stay LDS loads).
template <typename T>
__device__ __forceinline__ T *lds_opaque(T *p) {
    __attribute__((address_space(3))) T *q = (__attribute__((address_space(3))) T *)p;
    asm volatile("" : "+s"(q));
    return (T *)q;
}
__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t rfl(int64_t v) {
    return (int64_t)(((uint64_t)(uint32_t)rfl((int)((uint64_t)v >> 32)) << 32) | (uint32_t)rfl((int)(uint32_t)v));
}
__device__ __forceinline__ double rfl(double v) { return __longlong_as_double(rfl((int64_t)__double_as_longlong(v))); }

// Philox4x32-10 of the hop words, counter (blk, rail, n, c3), key (k0, k1),
// with its first rounds split by how often their inputs change: blk and rail
// are fixed per lane, c3 = d << 4 | h takes one value per half-step parity, n
// one value per step.  Round i uses the keys k0 + i W0 and k1 + i W1.
//   PhLane (once per launch): what depends on blk and c3 only, for both
//     parities: round 0's product M0 blk and round 1's product M1 x2.
//   PhStep (once per step, shared by both half-steps): round 0's product
//     M1 n, round 1's product M0 x0 and round 2's product M1 x2 (x2 after
//     round 1 does not depend on the parity).
//   ph_words (each half-step): the rest of rounds 1 and 2, then rounds 3 to 9.
// The words equal philox4x32_10(blk, rail, n, c3, k0, k1).  Every array index
// below is a compile-time constant (template recursion or fully unrolled
// loops), so the values stay in registers.
constexpr uint32_t kPhM0 = 0xD2511F53u, kPhM1 = 0xCD9E8D57u, kPhW0 = 0x9E3779B9u, kPhW1 = 0xBB67AE85u;

template <int NB>
struct PhLane {
    uint32_t p[2][NB];  // [h][block] hi(M1 x2) ^ (k0 + W0), x2 = hi(M0 blk) ^ c3 ^ k1 after round 0
    uint32_t q[2][NB];  // [h][block] lo(M1 x2): word x1 after round 1
    uint32_t r[NB];     // lo(M0 blk) ^ (k1 + W1)
};
template <int NB>
struct PhStep {
    uint32_t lo_b0;      // lo(M1 n): word x1 after round 0
    uint32_t lo_a1;      // lo(M0 x0) of round 1: word x3 after round 1
    uint32_t hi_b2[NB];  // M1 x2 of round 2, per block
    uint32_t lo_b2[NB];
};

template <int K, int NB>
__device__ __forceinline__ void ph_lane_init(PhLane<NB> &pl, uint32_t blk0, uint32_t c3, uint32_t k0, uint32_t k1) {
    if constexpr (K < NB) {
        const uint64_t a0 = (uint64_t)kPhM0 * (blk0 + (uint32_t)K);
        const uint64_t b_even = (uint64_t)kPhM1 * ((uint32_t)(a0 >> 32) ^ c3 ^ k1);
        const uint64_t b_odd = (uint64_t)kPhM1 * ((uint32_t)(a0 >> 32) ^ (c3 | 1u) ^ k1);
        pl.p[0][K] = (uint32_t)(b_even >> 32) ^ (k0 + kPhW0);
        pl.q[0][K] = (uint32_t)b_even;
        pl.p[1][K] = (uint32_t)(b_odd >> 32) ^ (k0 + kPhW0);
        pl.q[1][K] = (uint32_t)b_odd;
        pl.r[K] = (uint32_t)a0 ^ (k1 + kPhW1);
        ph_lane_init<K + 1>(pl, blk0, c3, k0, k1);
    }
}
template <int K, int NB>
__device__ __forceinline__ void ph_step_blocks(PhStep<NB> &ps, const PhLane<NB> &pl, uint32_t hi_a1) {
    if constexpr (K < NB) {
        const uint64_t b2 = (uint64_t)kPhM1 * (hi_a1 ^ pl.r[K]);
        ps.hi_b2[K] = (uint32_t)(b2 >> 32);
        ps.lo_b2[K] = (uint32_t)b2;
        ph_step_blocks<K + 1>(ps, pl, hi_a1);
    }
}
template <int NB>
__device__ __forceinline__ void ph_step(PhStep<NB> &ps, const PhLane<NB> &pl, uint32_t rail, uint32_t n,
                                        uint32_t k0) {
    const uint64_t b0 = (uint64_t)kPhM1 * n;
    const uint64_t a1 = (uint64_t)kPhM0 * ((uint32_t)(b0 >> 32) ^ k0 ^ rail);
    ps.lo_b0 = (uint32_t)b0;
    ps.lo_a1 = (uint32_t)a1;
    ph_step_blocks<0>(ps, pl, (uint32_t)(a1 >> 32));
}
template <int H, int N, int NB>
__device__ __forceinline__ void ph_words(uint32_t (&wd)[N], const PhLane<NB> &pl, const PhStep<NB> &ps, uint32_t k0,
                                         uint32_t k1) {
    // all blocks advance round by round; each round key is derived just before
    // its round (the empty asm keeps the compiler from deriving them all at
    // once and holding them in scalar registers)
    uint32_t x0[NB], x1[NB], x2[NB], x3[NB];
    uint32_t kr0 = k0 + 2u * kPhW0, kr1 = k1 + 2u * kPhW1;
#pragma unroll
    for (int K = 0; K < NB; ++K) {
        const uint64_t a2 = (uint64_t)kPhM0 * (pl.p[H][K] ^ ps.lo_b0);
        x0[K] = xor3(ps.hi_b2[K], pl.q[H][K], kr0);
        x1[K] = ps.lo_b2[K];
        x2[K] = xor3((uint32_t)(a2 >> 32), ps.lo_a1, kr1);
        x3[K] = (uint32_t)a2;
    }
#pragma unroll
    for (int round = 3; round < 10; ++round) {
        kr0 += kPhW0;
        kr1 += kPhW1;
        asm volatile("" : "+s"(kr0), "+s"(kr1));
#pragma unroll
        for (int K = 0; K < NB; ++K) {
            const uint64_t m0 = (uint64_t)kPhM0 * x0[K];
            const uint64_t m1 = (uint64_t)kPhM1 * x2[K];
            const uint32_t y0 = xor3((uint32_t)(m1 >> 32), x1[K], kr0);
            const uint32_t y2 = xor3((uint32_t)(m0 >> 32), x3[K], kr1);
            x1[K] = (uint32_t)m1;
            x3[K] = (uint32_t)m0;
            x0[K] = y0;
            x2[K] = y2;
        }
    }
#pragma unroll
    for (int K = 0; K < NB; ++K) {
        wd[4 * K + 0] = x0[K];
        wd[4 * K + 1] = x1[K];
        wd[4 * K + 2] = x2[K];
        wd[4 * K + 3] = x3[K];
    }
}
template <int K, int N>
__device__ __forceinline__ uint32_t min_word(const uint32_t (&wd)[N]) {
    if constexpr (K == N - 1) return wd[K];
    else return min(wd[K], min_word<K + 1>(wd));
}
// word i (runtime index): a select chain
template <int K, int N>
__device__ __forceinline__ uint32_t pick_word(const uint32_t (&wd)[N], int i) {
    if constexpr (K == N - 1) return wd[K];
    else return i == K ? wd[K] : pick_word<K + 1>(wd, i);
}

}  // namespace

template <typename Real, int SPL>
__global__ __launch_bounds__(64 * kWaveTilesPerWG) void hop_wave(PArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int kW = SPL / 2;          // Philox words per lane and half-step (SPL / 8 blocks):
                                         // word b / 2 belongs to the bond at site s0 + b
    constexpr int kNB = SPL / 8;         // Philox blocks per lane and half-step
    constexpr uint32_t kAll = SPL == 32 ? 0xFFFFFFFFu : 0xFFFFu;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: tile data in scalar registers

    const int n_groups = (a.n_tiles + kWaveTilesPerWG - 1) / kWaveTilesPerWG;
    const int ti = tile_of_block(blockIdx.x, n_groups) * kWaveTilesPerWG + wave;
    // the tile and its device, loaded before the barrier that the kernel table
    // needs, so that their latencies overlap the table's
    const PTile tile = a.tiles[ti < a.n_tiles ? ti : 0];
    const DevInfo dvc = a.devs[tile.d];
    const int nr_prev = a.tiles[tile.prev].nr, nr_next = a.tiles[tile.next].nr;
    // the kernel table K(dist, ds), shared by the workgroup's tiles
    {
        const int n_kt = (a.rail_range + 1) * (a.cutoff + 1);
        if (n_kt <= kLdsTableMax) {
            const Real *kt_glob = std::is_same<Real, double>::value ? reinterpret_cast<const Real *>(a.ktab64)
                                                                    : reinterpret_cast<const Real *>(a.ktab32);
            for (int i = threadIdx.x; i < n_kt; i += blockDim.x) reinterpret_cast<Real *>(smem)[i] = kt_glob[i];
        }
    }
    __syncthreads();
    // the tile's LDS (after the kernel table when that is in LDS)
    auto lds_of = [&](KArgs ka) -> WaveLds<SPL> & {
        const int n_kt = (ka->rail_range + 1) * (ka->cutoff + 1);
        const size_t kt_bytes = n_kt <= kLdsTableMax ? (((size_t)n_kt * sizeof(Real) + 15) & ~(size_t)15) : 0;
        return reinterpret_cast<WaveLds<SPL> *>(smem + kt_bytes)[wave];
    };
    WaveLds<SPL> &w = lds_of(kargs());

    if (ti >= a.n_tiles) return;  // no barrier follows

    // ------------------------------------------------------------ set-up
    // Values the loop itself needs stay in registers; the rest goes to w.geo.
    uint32_t bits = 0, valid = 0, rail = 0, r_lane = 0, nbit = 0;
    uint32_t bx = 0;  // 16 sites per lane: bits | nbit << 16
    int s0 = 0, cls_base = 0, d = 0;
    bool isolated = true;
    uint64_t *own = nullptr;
    {
        const DevInfo &dv = dvc;
        const int R = dv.rails, L = dv.sites, P = dv.pitch, m = a.rail_range;
        const int lpr = (P + SPL - 1) / SPL;  // lanes per rail
        const int nr = tile.nr;
        const bool single = tile.prev == ti && tile.next == ti;
        isolated = single || m == 0;  // no rail of another tile is ever read
        d = tile.d;
        own = a.pub + (int64_t)ti * a.pub_stride;  // kPubSlots state words, then the ring
        if (lane == 0) {
            WaveGeo &g = w.geo;
            g.R = R;
            g.L = L;
            g.P = P;
            g.lpr = lpr;
            g.nr = nr;
            g.m = m;
            g.W32 = (P + 31) / 32;              // 32-bit words of a published rail
            g.e = nr < 2 * m ? nr : 2 * m;      // edge rails: the first min(m, nr) and the last m
            g.r0 = tile.r0;
            g.d = tile.d;
            g.prev = tile.prev;
            g.next = tile.next;
            g.nr_prev = (int16_t)nr_prev;
            g.nr_next = (int16_t)nr_next;
            g.ti = ti;
            g.single = single;
            g.isolated = isolated;
            g.cutoff = a.cutoff;
            g.n_nbr = dv.n_nbr;
            g.n_knots = dv.n_knots;
            for (int k = 0; k < 2 * kMaxRailRange + 1; ++k) {
                g.nbr_off[k] = dv.nbr_off[k];
                g.nbr_dist[k] = dv.nbr_dist[k];
            }
            g.dv_off = dv.off;
            g.off_pad = dv.off_pad;
            g.n_set = dv.n_set;
            g.n_base = a.ctl.n_base;
            g.tally_base = a.ctl.tally_base;
            g.coul_bound = dv.coul_bound;
        }
        // the lane's sites, fixed for the launch
        const bool has = lane < nr * lpr;
        const int row = has ? lane / lpr : 0;
        s0 = has ? (lane - row * lpr) * SPL : 0;
        cls_base = row * P;
        rail = (uint32_t)(tile.r0 + row);
        const int last = L - 2 - s0;  // the bond at s0 + b lies inside the rail iff b <= last
        valid = (!has || last < 0) ? 0u : (last >= SPL - 1 ? kAll : ((2u << last) - 1u));

        // load the tile: occupancy bits to registers, barrier classes to LDS
        const int8_t *gstate = a.occ + dv.off_pad + (int64_t)tile.r0 * P;
        if (has) {
#pragma unroll
            for (int c = 0; c < SPL / 16; ++c) {
                if (c == 0 || s0 + 16 * c < P) {
                    const uint4 v = *reinterpret_cast<const uint4 *>(gstate + row * P + s0 + 16 * c);
                    bits |= occ_bits(v) << (16 * c);
                    *reinterpret_cast<uint4 *>(w.cls + row * P + s0 + 16 * c) =
                        make_uint4((v.x >> 1) & 0x7F7F7F7Fu, (v.y >> 1) & 0x7F7F7F7Fu, (v.z >> 1) & 0x7F7F7F7Fu,
                                   (v.w >> 1) & 0x7F7F7F7Fu);
                }
            }
        }
        for (int q = lane; q < kClasses; q += 64) w.cls_a[q] = exp(-a.beta * (dv.ea_min + (double)q * dv.ea_step));
        wave_sync();
        // the next lane's first site (the far end of the lane's last bond);
        // refreshed only after half-steps that moved ions
        nbit = __shfl_down(bits, 1, 64) & 1u;
        bx = bits | (nbit << 16);

        // Stage-0 scale of the lane: every origin of its bonds (sites s0 ..
        // s0 + SPL) has a class >= q_lo, so every exact threshold is at most
        // rho (thr0 + 1) + 2^32 2e-6 with rho = A(q_lo) / A(0); r_lane =
        // ceil(rho 2^32), and the per-step bound is mulhi(thr0, r_lane) +
        // 8600, the addition saturating (the margin covers the widening term,
        // both ceilings and binary64 rounding).  This holds while thr0 is the
        // unclipped threshold: a step whose lowest-class bound reaches 1
        // (thr0 saturated) bounds nothing for the higher classes, and its
        // window adds 2^32 - 1 instead (every word goes to the exact check).
        if (has && last >= 0) {
            int q_lo = kClasses;
            const int s_hi = s0 + SPL < L - 1 ? s0 + SPL : L - 1;
            for (int x = s0; x <= s_hi; ++x) q_lo = min(q_lo, (int)w.cls[row * P + x]);
            const double rho = w.cls_a[q_lo] / w.cls_a[0];
            r_lane = q_lo == 0 ? 0xFFFFFFFFu : (uint32_t)fmin(ceil(rho * 4294967296.0), 4294967295.0);
        }
    }
    PhLane<kNB> phl;
    ph_lane_init<0>(phl, (uint32_t)(s0 >> 3), (uint32_t)d << 4, a.key0, a.key1);
    // the candidate bonds of each parity that lie inside the rail
    const uint32_t valid_e = valid & 0x55555555u, valid_o = valid & 0xAAAAAAAAu;
    // the tile's publication words are written by one lane: keeping their base
    // in a vector register frees two scalar registers for the whole loop
    asm volatile("" : "+v"(own));
    const uint32_t tag_hi = (uint32_t)(a.epoch & 0xFFFFFu) << 12;  // state tag = tag_hi | launch-relative state

    // Per-step tables of the window [kb, kb + 64): lane k holds step kb + k's
    // stage-0 threshold in a register, the bias and g go to LDS.
    uint32_t thr_lane = 0;
    uint32_t t_add = 8600u;  // the stage-0 margin of the window (uniform, kept in a vector register)
    auto refresh = [&](int kb) {
        const KArgs ka = kargs();
        WaveLds<SPL> &wr = *lds_opaque(&w);
        const WaveGeo &g = wr.geo;
        const int dd = rfl(g.d);
        const int64_t k = rfl(g.n_base) - rfl(g.n_set) + kb + lane;
        const double V = protocol_voltage(ka->knot_t + dd * kMaxKnots, ka->knot_v + dd * kMaxKnots, rfl(g.n_knots),
                                          (double)k * ka->dt);
        const double gg = exp(0.5 * ka->beta * (fabs(ka->alpha * V) / (double)rfl(g.L) + rfl(g.coul_bound)));
        wr.step_v[lane] = V;
        wr.step_g[lane] = gg;
        thr_lane = threshold_of(ka->c0, wr.cls_a[0], gg);
        t_add = __ballot(thr_lane == 0xFFFFFFFFu) != 0 ? 0xFFFFFFFFu : 8600u;
        asm volatile("" : "+v"(t_add));
        wave_sync();
    };

    // 32 bits [32 q, 32 q + 32) of tile row r, gathered from the owning lanes;
    // every lane takes part in the cross-lane reads
    auto row_word = [&](int lpr, int r, int q) -> uint32_t {
        if (SPL == 32) return __shfl(bits, r * lpr + q, 64);
        const uint32_t lo = __shfl(bits, r * lpr + 2 * q, 64);
        const uint32_t hi = __shfl(bits, r * lpr + (2 * q + 1 < lpr ? 2 * q + 1 : 2 * q), 64);
        return lo | (2 * q + 1 < lpr ? hi << 16 : 0u);
    };
    // snapshot of the edge rails as state jrel into ring slot `slot`
    auto write_snapshot = [&](const WaveGeo &g, int slot, int64_t jrel) {
        const int w32 = rfl(g.W32), mm = rfl(g.m), ee = rfl(g.e), nrr = rfl(g.nr), lpr = rfl(g.lpr);
        uint64_t *dst = own + kPubSlots + (int64_t)slot * (ee * w32);
        const uint64_t tag = (uint64_t)(tag_hi | (uint32_t)jrel) << 32;
        for (int sr = 0; sr < ee; ++sr)
            for (int q0 = 0; q0 < w32; q0 += 64) {
                const int q = q0 + lane < w32 ? q0 + lane : w32 - 1;
                const uint32_t word = row_word(lpr, sr < mm ? sr : sr + (nrr - ee), q);
                if (q0 + lane < w32)
                    __hip_atomic_store(dst + sr * w32 + q, tag | word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
    };
    // Neighbour rails of state jrel into band: entry idx * W32 + q holds rail
    // offset idx - m (idx < m, from the previous tile) or nr + idx - m (from
    // the next tile).  The lanes take all 2 m W32 words at once (each its own
    // wait for the owning tile's state, then the word of its snapshot), so
    // that the round trips to the other tiles' publications overlap.  Uniform
    // result.
    auto fetch_bands = [&](KArgs ka, WaveLds<SPL> &wr, int64_t jrel) -> bool {
        const WaveGeo &g = wr.geo;
        const int w32 = rfl(g.W32), mm = rfl(g.m), prev = rfl(g.prev), next = rfl(g.next);
        const int nr_p = rfl(g.nr_prev), nr_n = rfl(g.nr_next);
        uint64_t *pub = ka->pub;
        const int64_t stride = ka->pub_stride;
        int32_t *status = ka->status;
        const int limit = ka->spin_limit;
        bool ok = true;
        for (int i = lane; i < 2 * mm * w32; i += 64) {
            const int idx = i / w32, q = i - idx * w32;
            const int T = idx < mm ? prev : next;
            const int nrT = idx < mm ? nr_p : nr_n;
            const int eT = nrT < 2 * mm ? nrT : 2 * mm;
            const int rr = idx < mm ? nrT - mm + idx : idx - mm;  // rail of tile T
            const int sr = rr < mm ? rr : rr - (nrT - eT);        // its row in T's snapshots
            const uint64_t *base = pub + (int64_t)T * stride;
            uint64_t st = 0, v = 0;
            if (ok) ok = poll_tag(base + jrel, tag_hi | (uint32_t)jrel, status, limit, &st);
            if (ok) {
                const int slot = (int)((uint32_t)st >> 12);
                const uint32_t snap_rel = (uint32_t)st & 0xFFFu;
                ok = poll_tag(base + kPubSlots + (int64_t)slot * (eT * w32) + sr * w32 + q, tag_hi | snap_rel,
                              status, limit, &v);
            }
            wr.band[i] = (uint32_t)v;
        }
        return __ballot(!ok) == 0;
    };

    int snap_count = 0;
    uint32_t snap_word = 0;  // ring slot << 12 | launch-relative state of the latest snapshot
    if (!isolated) {
        write_snapshot(w.geo, 0, 0);
        if (lane == 0) {
            w.snap_state[0] = 0;
            __hip_atomic_store(own, (uint64_t)tag_hi << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    // The publication of each new state: lane 0 writes word j of the tile's
    // slots with tag tag_hi | j (an isolated tile writes its words too; no
    // tile reads them, and the store needs no tile-dependent condition).  The
    // address, the tag and the snapshot count live in vector registers (they
    // change every half-step or only on a rare path), which keeps the scalar
    // registers for the loop's own values.
    uint64_t *pub_at = own;
    uint32_t tag_j = tag_hi;
    asm volatile("" : "+v"(tag_j), "+v"(snap_count));

    // One half-step of parity h (a compile-time constant): state js = 2 kstep
    // + h to js + 1 (the first state of a launch is even).  False when a wait
    // for a neighbour failed.
    auto half_step = [&](auto h_c, const int kstep, const PhStep<kNB> &ps) -> bool {
        constexpr int h = decltype(h_c)::value;
        // the state index, needed only on rare paths: derived there from an
        // opaque copy of the step, so that no register holds it across the step
        auto js_now = [&]() -> int {
            int k = kstep;
            asm volatile("" : "+s"(k));
            return 2 * k + h;
        };
        const int kw = kstep & (kWaveWin - 1);

        // candidates: bonds of parity h whose two sites differ
        // (the site after bond b: bit b + 1, or the next lane's first site)
        const uint32_t after = SPL == 32 ? __builtin_amdgcn_alignbit(nbit, bits, 1) : bx >> 1;
        const uint32_t cand = (bits ^ after) & (h ? valid_o : valid_e);

        // Philox words (the key is read from the kernel arguments each
        // half-step, a scalar load, rather than held in scalar registers)
        uint32_t wd[kW];
        {
            const KArgs ka = kargs();
            ph_words<h>(wd, phl, ps, ka->key0, ka->key1);
        }
        // stage 0: the smallest word against the bound of the lane's lowest
        // class; stage 1 (rare): each candidate's word against its origin's
        // exact class threshold
        const uint32_t thr0 = (uint32_t)__builtin_amdgcn_readlane((int)thr_lane, kw);
        const uint32_t t_lane = __builtin_elementwise_add_sat(__umulhi(thr0, r_lane), t_add);
        const uint32_t mn = min_word<0>(wd);
        // the common path decides with one wavefront vote that no lane has a
        // stage-0 word; only then are the survivor bits and their vote formed
        const bool stage1 = mn <= t_lane && cand != 0u;
        uint32_t sv = 0;
        uint64_t any = 0;
        if (__ballot(stage1)) {
            if (stage1) {
                const double c0 = kargs()->c0;
                WaveLds<SPL> &wr = *lds_opaque(&w);
                const double g_step = wr.step_g[kw];
                uint32_t c = cand;
                while (c) {
                    const int b = __builtin_ctz(c);
                    c &= c - 1;
                    const uint32_t x = pick_word<0>(wd, b >> 1);
                    if (x <= t_lane) {
                        const int o = s0 + (((bits >> b) & 1u) ? b : b + 1);
                        if (x <= threshold_of(c0, wr.cls_a[wr.cls[cls_base + o]], g_step)) sv |= 1u << b;
                    }
                }
            }
            any = __ballot(sv != 0u);
        }

        // survivors (rare): one at a time over the whole wavefront
        bool edge_changed = false;
        if (any) {
            const KArgs ka = kargs();
            WaveLds<SPL> &wr = *lds_opaque(&w);
            const WaveGeo &g = wr.geo;
            const int cut = rfl(g.cutoff), Lq = rfl(g.L), lprq = rfl(g.lpr), nrq = rfl(g.nr), mq = rfl(g.m);
            const int w32 = rfl(g.W32), Rq = rfl(g.R), n_nbr = rfl(g.n_nbr), r0 = rfl(g.r0), dd = rfl(g.d);
            const bool single = rfl(g.single) != 0;
            const int64_t n = rfl(g.n_base) + kstep;
            const int n_kt = (ka->rail_range + 1) * (cut + 1);
            const Real *kt = n_kt <= kLdsTableMax ? reinterpret_cast<const Real *>(smem)
                                                  : (std::is_same<Real, double>::value
                                                         ? reinterpret_cast<const Real *>(ka->ktab64)
                                                         : reinterpret_cast<const Real *>(ka->ktab32));
            auto bit_at = [&](int r, int site) -> uint32_t {
                return (wr.snap[r * lprq + site / SPL] >> (site % SPL)) & 1u;
            };
            wr.snap[lane] = bits;
            bool ok = true;
            if (!isolated) ok = fetch_bands(ka, wr, js_now());
            wave_sync();
            if (!ok) return false;
            uint32_t fl = 0;
            uint64_t rest = any;
            while (rest) {
                const int l = __builtin_ctzll(rest);
                rest &= rest - 1;
                uint32_t svl = (uint32_t)__builtin_amdgcn_readlane((int)sv, l);
                const int ls0 = __builtin_amdgcn_readlane(s0, l);
                const int lrow = __builtin_amdgcn_readlane(cls_base, l) / rfl(g.P);
                while (svl) {
                    const int b = __builtin_ctz(svl);
                    svl &= svl - 1;
                    const int s = ls0 + b;
                    const uint32_t word = (uint32_t)__builtin_amdgcn_readlane((int)pick_word<0>(wd, b >> 1), l);
                    const int o = bit_at(lrow, s) ? s : s + 1;
                    const int t = (o == s) ? s + 1 : s;
                    int lo = s - cut, hi = s + 1 + cut;
                    lo = lo < 0 ? 0 : lo;
                    hi = hi > Lq - 1 ? Lq - 1 : hi;
                    Real part = (Real)0;
                    for (int k = 0; k < n_nbr; ++k) {
                        const int off = rfl((int)g.nbr_off[k]);
                        const Real *ktr = kt + rfl((int)g.nbr_dist[k]) * (cut + 1);
                        int rho = lrow + off, band = -1;
                        if (single) {
                            while (rho < 0) rho += Rq;
                            while (rho >= Rq) rho -= Rq;
                        } else if (rho < 0) {
                            band = rho + mq;
                        } else if (rho >= nrq) {
                            band = mq + rho - nrq;
                        }
                        for (int jj = lo + lane; jj <= hi; jj += 64) {
                            uint32_t bit = band < 0 ? bit_at(rho, jj) : (wr.band[band * w32 + (jj >> 5)] >> (jj & 31)) & 1u;
                            if (off == 0 && (jj == o || jj == t)) bit = 0;
                            const int dt_ = t - jj < 0 ? jj - t : t - jj;
                            const int do_ = o - jj < 0 ? jj - o : o - jj;
                            const Real kt_v = dt_ > cut ? (Real)0 : ktr[dt_];
                            const Real ko_v = do_ > cut ? (Real)0 : ktr[do_];
                            part += bit ? (kt_v - ko_v) : (Real)0;
                        }
                    }
#pragma unroll
                    for (int sh_ = 32; sh_ >= 1; sh_ >>= 1) part += __shfl_xor(part, sh_, 64);
                    int acc = 0;
                    if (lane == 0) {
                        const Real alpha_r = (Real)ka->alpha, beta_r = (Real)ka->beta, c0_r = (Real)ka->c0;
                        const Real e_app = ((alpha_r * (Real)wr.step_v[kw]) * (Real)(t - o)) / (Real)Lq;
                        const int srail = r0 + lrow;
                        const Real ea = ka->ea ? reinterpret_cast<const Real *>(ka->ea)[rfl(g.dv_off) + (int64_t)srail * Lq + o]
                                               : (Real)ka->ea_scalar;
                        HopArgs::LogBuf log;
                        log.count = ka->log.count;
                        log.entries = ka->log.entries;
                        log.cap = ka->log.cap;
                        acc = decide_hop<Real>(e_app + part, ea, word, beta_r, c0_r, log, dd, h, n, srail, s);
                        if (acc) {
                            HopRecord rec;
                            rec.buf = ka->record.buf;
                            rec.count = ka->record.count;
                            rec.cap = ka->record.cap;
                            rec.n0 = ka->record.n0;
                            rec.n_hs = ka->record.n_hs;
                            record_hop(rec, dd, h, n, srail, s, o == s ? 0 : 1);
                            const int64_t base = (n - rfl(g.tally_base)) * ka->n_devices + dd;
                            atomicAdd(&ka->tally_net[base], t < o ? 1 : -1);
                            const int qo = (10 * o) / Lq, qt = (10 * t) / Lq;
                            if (qo != qt) {
                                atomicAdd(&ka->tally_dec[base * kDeciles + qo], -1);
                                atomicAdd(&ka->tally_dec[base * kDeciles + qt], 1);
                            }
                        }
                    }
                    acc = __builtin_amdgcn_readfirstlane(acc);
                    if (acc) {
                        if (lane == lrow * lprq + s / SPL) fl ^= 1u << (s % SPL);
                        if (lane == lrow * lprq + (s + 1) / SPL) fl ^= 1u << ((s + 1) % SPL);
                        if (lrow < mq || lrow >= nrq - mq) edge_changed = true;
                    }
                }
            }
            bits ^= fl;
            nbit = __shfl_down(bits, 1, 64) & 1u;
            bx = bits | (nbit << 16);
        }

        // publish the new state js + 1
        ++pub_at;
        ++tag_j;
        if (edge_changed && !isolated) {
            const uint32_t jn = (uint32_t)js_now() + 1u;
            const KArgs ka = kargs();
            WaveLds<SPL> &wr = *lds_opaque(&w);
            const int sc = rfl(snap_count) + 1;
            snap_count = sc;
            const int slot = sc % kSnapSlots;
            if (sc >= kSnapSlots) {
                // the slot's snapshot serves states before the next snapshot's
                const uint32_t need = (uint32_t)wr.snap_state[(slot + 1) % kSnapSlots];
                bool ok = true;
                if (lane < 2) {
                    const int T = lane == 0 ? rfl(wr.geo.prev) : rfl(wr.geo.next);
                    uint64_t v = 0;
                    ok = poll_tag(ka->pub + (int64_t)T * ka->pub_stride + need, tag_hi | need, ka->status, ka->spin_limit, &v);
                }
                if (__ballot(!ok)) return false;
            }
            write_snapshot(wr.geo, slot, jn);
            if (lane == 0) wr.snap_state[slot] = (int16_t)jn;
            snap_word = ((uint32_t)slot << 12) | jn;
        }
        if (lane == 0)
            __hip_atomic_store(pub_at, ((uint64_t)tag_j << 32) | snap_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    };
    // Wave priority.  A SIMD's issue arbiter prefers the older of its waves,
    // so the tiles of the workgroups dispatched first would run ahead and the
    // launch would end with the later ones alone on their SIMDs.  A launch of
    // up to 128 steps lowers each wave's priority by quarters of its steps (a
    // wave ahead yields to the ones behind); a longer one rotates the first
    // place among the workgroups that share a CU (dispatch layers of
    // gridDim / 4 workgroups) every 10.24 us of the real-time clock.
    uint32_t layer = (uint32_t)(((int64_t)blockIdx.x * 4) / (int64_t)gridDim.x);
    asm volatile("" : "+v"(layer));
    auto set_priority = [&](int kstep) {
        const int n = kargs()->n_steps;
        uint32_t pr;
        if (n <= 128) {
            pr = 3u - (uint32_t)(kstep >= (n >> 2)) - (uint32_t)(kstep >= (n >> 1)) - (uint32_t)(kstep >= ((3 * n) >> 2));
        } else {
            const uint32_t slice = (uint32_t)(__builtin_amdgcn_s_memrealtime() >> 10);
            pr = (slice + (uint32_t)__builtin_amdgcn_readfirstlane((int)layer)) & 3u;
        }
        if (pr == 0u) __builtin_amdgcn_s_setprio(0);
        else if (pr == 1u) __builtin_amdgcn_s_setprio(1);
        else if (pr == 2u) __builtin_amdgcn_s_setprio(2);
        else __builtin_amdgcn_s_setprio(3);
    };
    for (int kstep = 0; kstep < a.n_steps; ++kstep) {
        if ((kstep & 1) == 0) set_priority(kstep);
        if ((kstep & (kWaveWin - 1)) == 0) refresh(kstep);
        PhStep<kNB> ps;
        {
            const KArgs ka = kargs();
            const uint32_t n_first = (uint32_t)ka->ctl.n_base;
            ph_step(ps, phl, rail, n_first + (uint32_t)kstep, ka->key0);
        }
        if (!half_step(std::integral_constant<int, 0>{}, kstep, ps)) break;
        if (!half_step(std::integral_constant<int, 1>{}, kstep, ps)) break;
    }

    // write the tile back: the padded state (bits and barrier classes) and the
    // caller's occupancy (unpadded, one byte per site)
    {
        const KArgs ka = kargs();
        const WaveGeo &g = lds_opaque(&w)->geo;
        const int P = rfl(g.P), L = rfl(g.L);
        int8_t *gstate = ka->occ + rfl(g.off_pad) + (int64_t)rfl(g.r0) * P;
        if (lane < rfl(g.nr) * rfl(g.lpr)) {
            const int row = cls_base / P;
            int8_t *urow = ka->occ_user + rfl(g.dv_off) + (int64_t)(rfl(g.r0) + row) * L;
#pragma unroll
            for (int c = 0; c < SPL / 16; ++c) {
                if (c == 0 || s0 + 16 * c < P) {
                    const uint32_t b16 = (bits >> (16 * c)) & 0xFFFFu;
                    const uint4 cv = *reinterpret_cast<const uint4 *>(w.cls + cls_base + s0 + 16 * c);
                    uint4 o;
                    o.x = ((b16 >> 0) & 0xFu) * 0x00204081u & 0x01010101u;
                    o.y = ((b16 >> 4) & 0xFu) * 0x00204081u & 0x01010101u;
                    o.z = ((b16 >> 8) & 0xFu) * 0x00204081u & 0x01010101u;
                    o.w = ((b16 >> 12) & 0xFu) * 0x00204081u & 0x01010101u;
                    const uint4 v = make_uint4(o.x | (cv.x << 1), o.y | (cv.y << 1), o.z | (cv.z << 1), o.w | (cv.w << 1));
                    *reinterpret_cast<uint4 *>(gstate + cls_base + s0 + 16 * c) = v;
                    const int sc = s0 + 16 * c;
                    int8_t *u = urow + sc;
                    if (sc + 16 <= L && (reinterpret_cast<uintptr_t>(u) & 15) == 0) {
                        *reinterpret_cast<uint4 *>(u) = o;
                    } else {
                        for (int k = 0; k < 16 && sc + k < L; ++k) u[k] = (int8_t)((b16 >> k) & 1u);
                    }
                }
            }
        }
    }

    // The last tile to finish ends the chunk (the launch's tally rows and
    // totals), when the host asked for it.  The tallies are only ever touched
    // by device-scope atomics inside the launch: a tile waits until its own
    // have been performed before it counts itself, and the last tile reads
    // them with device-scope atomic loads.  (A device-scope release fence per
    // tile would write back the whole L2 of its XCD.)  Tiles count themselves
    // in kTicketBuckets counters (tile index modulo the bucket count), and the
    // tile that completes a bucket counts the bucket in the total, so that no
    // counter takes more than one atomic per bucket member.
    if (a.ticket) {
        const KArgs ka = kargs();
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const int nt = ka->n_tiles;
        const int b = ti % kTicketBuckets;
        const uint32_t members = (uint32_t)(nt / kTicketBuckets + (b < nt % kTicketBuckets ? 1 : 0));
        const uint32_t buckets = (uint32_t)(nt < kTicketBuckets ? nt : kTicketBuckets);
        uint32_t last = 0;
        if (lane == 0) {
            uint32_t *bucket = ka->ticket + b * kTicketStride;
            uint32_t *total = ka->ticket + kTicketBuckets * kTicketStride;
            if (__hip_atomic_fetch_add(bucket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == members - 1u) {
                __hip_atomic_store(bucket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                if (__hip_atomic_fetch_add(total, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == buckets - 1u) {
                    __hip_atomic_store(total, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    last = 1;
                }
            }
        }
        last = (uint32_t)__builtin_amdgcn_readfirstlane((int)last);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (last) {
            // the tile's class rows are free now: 128 segment sums
            const FinishArgs fin = a.fin;
            finish_tallies_wave(fin, lane, reinterpret_cast<int64_t *>(w.cls));
        }
    }
}

namespace {
const void *wave_fn(int spl, bool fp64) {
    if (spl == 32) return fp64 ? (const void *)hop_wave<double, 32> : (const void *)hop_wave<float, 32>;
    return fp64 ? (const void *)hop_wave<double, 16> : (const void *)hop_wave<float, 16>;
}
}  // namespace

size_t wave_lds_bytes(int spl, int n_kt, bool fp64) {
    const size_t kt = n_kt <= kLdsTableMax ? ((size_t)n_kt * (fp64 ? sizeof(double) : sizeof(float)) + 15) & ~(size_t)15 : 0;
    return kt + kWaveTilesPerWG * (spl == 32 ? sizeof(WaveLds<32>) : sizeof(WaveLds<16>));
}

int wave_band_words(int spl) { return spl == 32 ? WaveLds<32>::kBand : WaveLds<16>::kBand; }

hipError_t launch_wave(const PArgs &a, int spl, size_t lds, bool fp64, hipStream_t st) {
    PArgs args = a;
    void *kargs[] = {&args};
    const int groups = (a.n_tiles + kWaveTilesPerWG - 1) / kWaveTilesPerWG;
    // An ordinary launch: the grid never exceeds what is co-resident (checked
    // by the host), and every neighbour wait is bounded.
    return hipLaunchKernel(wave_fn(spl, fp64), dim3(groups), dim3(64 * kWaveTilesPerWG), kargs, (size_t)lds, st);
}

hipError_t wave_capacity(int spl, size_t lds, bool fp64, int *blocks_per_cu) {
    const void *fn = wave_fn(spl, fp64);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, 64 * kWaveTilesPerWG, lds);
}

}  // namespace kmc
