// The paper's own zone model (SI S2.1, "Step-by-Step Explanation of the
// Markov Chain Monte Carlo Framework"), declared in include/kmc.h as the
// kmc_zone_* calls.
//
// State: the ion-position matrix X [rails][ions] (1-based columns, uint16,
// strictly increasing along a rail).  One kernel launch per step:
//   * the step's table comes from the zone populations before the step: the
//     bias V(t_n), the net drop with the implicit space charge
//     dV_net(z) = V - f (sum_{z'<z} rho_z' - sum_{z'>z} rho_z'),
//     rho_z = N_z - N/Z, the energy gap of Eq. S1, the Boltzmann factor of
//     Eq. S2 and the directional probabilities of Eqs. S3-S4, in binary64
//     (computed by the previous step's last workgroup, or after a state or
//     protocol change by a one-workgroup kernel);
//   * a wavefront takes two rails, a lane two neighbouring ions of a rail:
//     one Philox4x32-10 block gives the lane's four uniforms (right and left
//     trial of each ion), the neighbours' columns come from the adjacent
//     lanes, a move is M_right - M_left with the gap tests of SI S2.1, and two
//     ions aiming at one column both stay;
//   * the new zone populations (added at zone boundaries only: the columns of
//     a rail stay increasing) and the net hops are summed per workgroup in
//     LDS, then into 64 bucket rows by device atomics; the last workgroup to
//     finish (counted per bucket, then over the buckets) sums the buckets
//     into the populations, writes the step's output row, clears the buckets
//     and evaluates the next step's table.
#include "../../include/kmc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kmc_device.h"
#include "kmc_internal.h"

namespace kmc {
kmc_status record_error(kmc_status s, const std::string &msg);
}

namespace {

using kmc::record_error;
using kmc::kMaxKnots;
using kmc::philox4x32_10;
using kmc::protocol_voltage;

constexpr int kZoneMaxZones = 64;
constexpr int kZoneMaxIons = 64;      // two per lane of a 32-lane half-wavefront
constexpr int kZoneBuckets = 64;
constexpr int kZoneBucketStride = 128;  // int64 per bucket row (zones, then net)
constexpr int kZoneBlock = 256;
constexpr int kZoneMaxGrid = 2048;

constexpr int kZonePairsPerIter = 4;  // rail pairs a wavefront loads before computing them

struct ZoneArgs {
    uint16_t *X;                // [rails][ions]
    int32_t rails, ions, sites, zones;
    double p0, kT, hot, v_factor, dt;
    uint32_t key0, key1;
    const double *knot_t, *knot_v;
    int32_t n_knots;
    int64_t n_set;
    int64_t n;                  // absolute step of the launch
    int64_t row;                // output row of the step (n - first step of the call)
    const double *table;        // [2][Z] P_left, P_right of this step
    double *table_next;         // [2][Z] of the next step (written by the last workgroup)
    int64_t *pop_next;          // [Z] zone populations after the step (written by the last workgroup)
    int64_t *bucket;            // [kZoneBuckets][kZoneBucketStride], zero on entry
    uint32_t *ticket;           // [kZoneBuckets + 1] counters, 32 uint32 apart
    int32_t *net_out;           // caller [n_steps] or null
    int32_t *zone_out;          // caller [n_steps][Z] or null
    int64_t *net_total;         // running total of the net hops
};

__device__ __forceinline__ int zone_of(int x, int sites, int zones) {
    return (int)(((int64_t)x * zones + sites - 1) / sites);  // 1-based
}

// The same zone without an integer division: q = (x zones + sites - 1) /
// sites with n = x zones + sites - 1 < 2^23, from a binary32 reciprocal (n is
// exact in binary32 and the product is within one unit of the quotient),
// corrected by one integer test each way.
__device__ __forceinline__ int zone_fast(uint32_t x, uint32_t sites, uint32_t zones, float inv_sites) {
    const uint32_t n = x * zones + sites - 1u;
    uint32_t q = (uint32_t)((float)n * inv_sites);
    q -= q * sites > n ? 1u : 0u;
    q += (q + 1u) * sites <= n ? 1u : 0u;
    return (int)q;
}

// The accept test u <= p of a uniform u = w 2^-32 is w <= floor(p 2^32) for
// the integer w (p 2^32 is exact in binary64): one threshold per zone and
// direction, 0xFFFFFFFF when p >= 1 (every word accepts).
__device__ __forceinline__ uint32_t word_threshold(double p) {
    const double t = floor(p * 4294967296.0);
    return t >= 4294967295.0 ? 0xFFFFFFFFu : (t <= 0.0 ? 0u : (uint32_t)t);
}

// Table entry of zone z for bias V and populations pop (Eqs. S1-S4 with the
// space-charge drop), binary64, the operations in the order of the text.
__device__ inline void zone_entry(int z, int Z, const int64_t *pop, double V, double p0, double kT, double hot,
                                  double v_factor, double *pl_out, double *pr_out) {
    double total = 0.0;
    for (int y = 0; y < Z; ++y) total += (double)pop[y];
    const double mean = total / (double)Z;
    double below = 0.0, above = 0.0;
    for (int y = 0; y < z; ++y) below += (double)pop[y] - mean;
    for (int y = z + 1; y < Z; ++y) above += (double)pop[y] - mean;
    const double dv = V - v_factor * (below - above);
    const double dE = dv * hot;
    const double B = exp(-dE / kT);
    const double pl = p0 / (1.0 + B);
    *pl_out = pl;
    *pr_out = B * pl;
}

__global__ __launch_bounds__(kZoneBlock) void zone_step(ZoneArgs a) {
    __shared__ uint32_t s_tl[kZoneMaxZones], s_tr[kZoneMaxZones];
    __shared__ int32_t s_pop[kZoneMaxZones];
    __shared__ int64_t s_fin[kZoneMaxZones + 1];
    __shared__ int32_t s_net;
    __shared__ double s_v;
    __shared__ uint32_t s_last;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int Z = a.zones;
    if (tid < Z) {
        s_tl[tid] = word_threshold(a.table[tid]);
        s_tr[tid] = word_threshold(a.table[Z + tid]);
        s_pop[tid] = 0;
    }
    if (tid == 0) s_net = 0;
    __syncthreads();
    const uint32_t sites = (uint32_t)a.sites, zones = (uint32_t)Z;
    const float inv_sites = 1.0f / (float)a.sites;

    // ions: a half-wavefront per rail, a lane per two neighbouring ions; a
    // wavefront loads kZonePairsPerIter rail pairs before computing them
    const int half = lane >> 5, l = lane & 31;
    const int j0 = 2 * l, j1 = 2 * l + 1;
    const int64_t pairs = ((int64_t)a.rails + 1) / 2;
    const int64_t tw = (int64_t)gridDim.x * (kZoneBlock / 64), gw = (int64_t)blockIdx.x * (kZoneBlock / 64) + wave;
    int net = 0;
    for (int64_t it = 0; it * kZonePairsPerIter * tw < pairs; ++it) {
        int x0[kZonePairsPerIter], x1[kZonePairsPerIter];
        int64_t rail[kZonePairsPerIter];
#pragma unroll
        for (int k = 0; k < kZonePairsPerIter; ++k) {
            const int64_t pr = (it * kZonePairsPerIter + k) * tw + gw;
            rail[k] = 2 * pr + half;
            const bool ok = pr < pairs && rail[k] < a.rails;
            const uint16_t *row = a.X + rail[k] * a.ions;
            x0[k] = ok && j0 < a.ions ? (int)row[j0] : 0;
            x1[k] = ok && j1 < a.ions ? (int)row[j1] : 0;
        }
#pragma unroll
        for (int k = 0; k < kZonePairsPerIter; ++k) {
            const int64_t pr = (it * kZonePairsPerIter + k) * tw + gw;
            const bool rail_ok = pr < pairs && rail[k] < a.rails;
            const bool h0 = rail_ok && j0 < a.ions, h1 = rail_ok && j1 < a.ions;
            // neighbours: the previous lane's second ion, the next lane's first
            // ion (a virtual ion at column 0 before the first ion and at
            // sites + 1 after the last)
            const int prev_x1 = __shfl_up(x1[k], 1, 32);
            const int next_x0 = __shfl_down(x0[k], 1, 32);
            const bool has_next = j1 + 1 < a.ions && l < 31;
            const int left0 = l == 0 ? 0 : prev_x1;
            const int right0 = h1 ? x1[k] : a.sites + 1;
            const int right1 = has_next ? next_x0 : a.sites + 1;
            // the lane's four uniforms: right and left trial of ions j0 and j1
            const uint4 w = philox4x32_10((uint32_t)l, (uint32_t)rail[k], (uint32_t)a.n, 2u << 1, a.key0, a.key1);
            int m0 = 0, m1 = 0;
            if (h0) {
                const int z = zone_fast((uint32_t)x0[k], sites, zones, inv_sites) - 1;
                const int mr = (w.x <= s_tr[z]) && (right0 - x0[k] > 1);
                const int ml = (w.y <= s_tl[z]) && (x0[k] - left0 > 1);
                m0 = mr - ml;
            }
            if (h1) {
                const int z = zone_fast((uint32_t)x1[k], sites, zones, inv_sites) - 1;
                const int mr = (w.z <= s_tr[z]) && (right1 - x1[k] > 1);
                const int ml = (w.w <= s_tl[z]) && (x1[k] - x0[k] > 1);
                m1 = mr - ml;
            }
            // two ions aiming at one column both stay (such pairs are disjoint)
            const int prev_m1 = __shfl_up(m1, 1, 32);
            const int next_m0 = __shfl_down(m0, 1, 32);
            const bool in_pair = h0 && h1 && m0 == 1 && m1 == -1 && x1[k] - x0[k] == 2;
            const bool with_prev = h0 && l > 0 && prev_m1 == 1 && m0 == -1 && x0[k] - prev_x1 == 2;
            const bool with_next = h1 && has_next && m1 == 1 && next_m0 == -1 && next_x0 - x1[k] == 2;
            if (in_pair || with_prev) m0 = 0;
            if (in_pair || with_next) m1 = 0;
            const int y0 = x0[k] + m0, y1 = x1[k] + m1;
            uint16_t *row = a.X + rail[k] * a.ions;
            if (h0) row[j0] = (uint16_t)y0;
            if (h1) row[j1] = (uint16_t)y1;
            net -= m0 + m1;
            // zone populations after the move: the columns stay increasing, so
            // the ions of a zone are consecutive; zone z holds (index after its
            // last ion) - (index of its first ion), added at the boundaries only
            const int zz0 = h0 ? zone_fast((uint32_t)y0, sites, zones, inv_sites) : 0;
            const int zz1 = h1 ? zone_fast((uint32_t)y1, sites, zones, inv_sites) : 0;
            const int prev_zz1 = __shfl_up(zz1, 1, 32);
            const int next_zz0 = __shfl_down(zz0, 1, 32);
            if (h0) {
                if (j0 > 0 && prev_zz1 != zz0) atomicAdd(&s_pop[zz0 - 1], -j0);
                if (!h1 || zz1 != zz0) atomicAdd(&s_pop[zz0 - 1], j0 + 1);
            }
            if (h1) {
                if (zz0 != zz1) atomicAdd(&s_pop[zz1 - 1], -j1);
                if (!has_next || next_zz0 != zz1) atomicAdd(&s_pop[zz1 - 1], j1 + 1);
            }
        }
    }
    // the workgroup's net hops
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) net += __shfl_xor(net, off, 64);
    if (lane == 0 && net != 0) atomicAdd(&s_net, net);
    __syncthreads();

    // workgroup sums into its bucket row; the last workgroup ends the step
    const int b = blockIdx.x % kZoneBuckets;
    int64_t *brow = a.bucket + (int64_t)b * kZoneBucketStride;
    if (tid < Z && s_pop[tid] != 0) atomicAdd((unsigned long long *)&brow[tid], (unsigned long long)(int64_t)s_pop[tid]);
    if (tid == Z && s_net != 0) atomicAdd((unsigned long long *)&brow[Z], (unsigned long long)(int64_t)s_net);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
        const uint32_t nb = (uint32_t)min((int)gridDim.x, kZoneBuckets);
        const uint32_t members = gridDim.x / kZoneBuckets + ((uint32_t)b < gridDim.x % kZoneBuckets ? 1u : 0u);
        uint32_t last = 0;
        uint32_t *cb = a.ticket + b * 32;
        uint32_t *ct = a.ticket + kZoneBuckets * 32;
        if (__hip_atomic_fetch_add(cb, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == members - 1u) {
            __hip_atomic_store(cb, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (__hip_atomic_fetch_add(ct, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == nb - 1u) {
                __hip_atomic_store(ct, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                last = 1;
            }
        }
        s_last = last;
    }
    __syncthreads();
    if (!s_last) return;
    // the last workgroup: populations after the step, the output row, and the
    // next step's table
    if (tid == 0) s_v = protocol_voltage(a.knot_t, a.knot_v, a.n_knots, (double)(a.n + 1 - a.n_set) * a.dt);
    if (tid <= Z) s_fin[tid] = 0;
    __syncthreads();
    // every thread takes some of the kZoneBuckets x (Z + 1) bucket entries
    for (int e = tid; e < kZoneBuckets * (Z + 1); e += kZoneBlock) {
        const int bb = e / (Z + 1), q = e - bb * (Z + 1);
        int64_t *p = a.bucket + (int64_t)bb * kZoneBucketStride + q;
        const int64_t v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v != 0) {
            __hip_atomic_store(p, (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            atomicAdd((unsigned long long *)&s_fin[q], (unsigned long long)v);
        }
    }
    __syncthreads();
    if (tid <= Z) {
        const int64_t sum = s_fin[tid];
        if (tid < Z) {
            a.pop_next[tid] = sum;
            if (a.zone_out) a.zone_out[a.row * Z + tid] = (int32_t)sum;
        } else {
            if (a.net_out) a.net_out[a.row] = (int32_t)sum;
            *a.net_total += sum;
        }
    }
    __syncthreads();
    if (tid < Z) {
        double pl, pr;
        zone_entry(tid, Z, s_fin, s_v, a.p0, a.kT, a.hot, a.v_factor, &pl, &pr);
        a.table_next[tid] = pl;
        a.table_next[Z + tid] = pr;
    }
}

// The table of the step n from the populations pop (one workgroup).
__global__ void zone_make_table(const int64_t *pop, int Z, const double *knot_t, const double *knot_v, int n_knots,
                                int64_t n, int64_t n_set, double dt, double p0, double kT, double hot,
                                double v_factor, double *table) {
    __shared__ double s_v;
    __shared__ int64_t s_pop[kZoneMaxZones];
    const int tid = threadIdx.x;
    if (tid == 0) s_v = protocol_voltage(knot_t, knot_v, n_knots, (double)(n - n_set) * dt);
    if (tid < Z) s_pop[tid] = pop[tid];
    __syncthreads();
    if (tid < Z) {
        double pl, pr;
        zone_entry(tid, Z, s_pop, s_v, p0, kT, hot, v_factor, &pl, &pr);
        table[tid] = pl;
        table[Z + tid] = pr;
    }
}

// Ion-position matrix from the caller's occupancy (one wavefront per rail):
// the k-th occupied site of a rail becomes column X[k] (1-based).  Rails
// whose ion count differs from `ions` raise *bad.  The populations of the
// zones are added to pop.
__global__ __launch_bounds__(256) void zone_import(const int8_t *occ, uint16_t *X, int rails, int sites, int ions,
                                                  int zones, int64_t *pop, int32_t *bad, int write) {
    __shared__ int32_t s_pop[kZoneMaxZones];
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < kZoneMaxZones) s_pop[threadIdx.x] = 0;
    __syncthreads();
    const int64_t rail = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (rail < rails) {
        const int8_t *src = occ + rail * sites;
        int base = 0;
        for (int s0 = 0; s0 < sites; s0 += 64) {
            const int s = s0 + lane;
            const bool occd = s < sites && src[s] != 0;
            const uint64_t m = __ballot(occd);
            const int rank = base + __popcll(m & ((1ull << lane) - 1ull));
            if (write && occd && rank < ions) {
                X[rail * ions + rank] = (uint16_t)(s + 1);
                atomicAdd(&s_pop[zone_of(s + 1, sites, zones) - 1], 1);
            }
            base += __popcll(m);
        }
        if (lane == 0 && base != ions) atomicExch(bad, 1);
    }
    __syncthreads();
    if (write && threadIdx.x < zones && s_pop[threadIdx.x] != 0)
        atomicAdd((unsigned long long *)&pop[threadIdx.x], (unsigned long long)(int64_t)s_pop[threadIdx.x]);
}

// Caller occupancy from the ion-position matrix (one wavefront per rail).
__global__ __launch_bounds__(256) void zone_export(const uint16_t *X, int8_t *occ, int rails, int sites, int ions) {
    const int lane = threadIdx.x & 63;
    const int64_t rail = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (rail >= rails) return;
    int8_t *dst = occ + rail * sites;
    for (int s = lane; s < sites; s += 64) dst[s] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int j = lane; j < ions; j += 64) dst[(int)X[rail * ions + j] - 1] = 1;
}

__global__ void zone_fill_i64(int64_t *p, int64_t n, int64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

struct ZoneKnots {
    double t[kMaxKnots], v[kMaxKnots];
};
__global__ void zone_set_knots(double *kt, double *kv, ZoneKnots k) {
    const int i = threadIdx.x;
    if (i < kMaxKnots) {
        kt[i] = k.t[i];
        kv[i] = k.v[i];
    }
}

}  // namespace

struct kmc_zone_ctx {
    kmc_zone_params p{};
    int32_t ions = 0;
    unsigned char *ws = nullptr;
    int8_t *occ_user = nullptr;
    hipStream_t stream = nullptr;
    bool poisoned = false;
    int64_t n = 0;              // step counter
    int64_t n_set = 0;          // step of the protocol install
    int32_t n_knots = 1;
    int cur = 0;                // population buffer holding the current state
    // workspace layout
    size_t off_X, off_pop, off_table, off_bucket, off_ticket, off_knots, off_total, off_bad, total;
    template <typename T>
    T *at(size_t off) { return reinterpret_cast<T *>(ws + off); }
};

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

kmc_status zone_validate(const kmc_zone_params *p) {
    if (!p) return record_error(KMC_EINVAL, "params is NULL");
    if (p->rails < 1) return record_error(KMC_EINVAL, "rails must be >= 1");
    if (p->sites < 2 || p->sites > 65534) return record_error(KMC_EUNSUPPORTED, "sites must be in [2, 65534]");
    if (p->zones < 1 || p->zones > kZoneMaxZones) return record_error(KMC_EUNSUPPORTED, "zones must be in [1, 64]");
    if (p->ions_per_rail < 0 || p->ions_per_rail > kZoneMaxIons || p->ions_per_rail > p->sites)
        return record_error(KMC_EUNSUPPORTED, "ions_per_rail must be in [0, min(64, sites)]");
    if (!(std::isfinite(p->p0) && p->p0 >= 0.0 && p->p0 <= 1.0)) return record_error(KMC_EINVAL, "p0 must be in [0, 1]");
    if (!(std::isfinite(p->kT_ev) && p->kT_ev > 0.0)) return record_error(KMC_EINVAL, "kT_ev must be > 0");
    if (!std::isfinite(p->hop_over_thickness)) return record_error(KMC_EINVAL, "hop_over_thickness must be finite");
    if (!std::isfinite(p->v_factor)) return record_error(KMC_EINVAL, "v_factor must be finite");
    if (!(std::isfinite(p->dt_s) && p->dt_s > 0.0)) return record_error(KMC_EINVAL, "dt_s must be > 0");
    if ((int64_t)p->rails * p->ions_per_rail > ((int64_t)1 << 31) - 1)
        return record_error(KMC_EUNSUPPORTED, "more than 2^31 - 1 ions");
    return KMC_OK;
}

void zone_layout(kmc_zone_ctx *c) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    c->off_X = take(sizeof(uint16_t) * (size_t)c->p.rails * (size_t)std::max(c->p.ions_per_rail, 1));
    c->off_pop = take(sizeof(int64_t) * 2 * kZoneMaxZones);
    c->off_table = take(sizeof(double) * 2 * 2 * kZoneMaxZones);
    c->off_bucket = take(sizeof(int64_t) * kZoneBuckets * kZoneBucketStride);
    c->off_ticket = take(sizeof(uint32_t) * (kZoneBuckets + 1) * 32);
    c->off_knots = take(sizeof(double) * 2 * kMaxKnots);
    c->off_total = take(sizeof(int64_t));
    c->off_bad = take(sizeof(int32_t));
    c->total = off;
}

kmc_status zone_hip(kmc_zone_ctx *c, hipError_t e, const char *what) {
    if (e == hipSuccess) return KMC_OK;
    if (c) c->poisoned = true;
    return record_error(KMC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define ZONE_HIP(c, expr)                                     \
    do {                                                      \
        kmc_status s_ = zone_hip((c), (expr), #expr);         \
        if (s_ != KMC_OK) return s_;                          \
    } while (0)

kmc_status zone_usable(kmc_zone_ctx *c) {
    if (!c) return record_error(KMC_EINVAL, "context is NULL");
    if (c->poisoned) return record_error(KMC_ESTATE, "context poisoned by an earlier HIP error");
    return KMC_OK;
}

hipError_t zone_fill(int64_t *p, int64_t n, int64_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zone_fill_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// The table of the current step from the current populations (after a
// state or protocol change; otherwise each step's last workgroup writes it).
kmc_status zone_refresh_table(kmc_zone_ctx *c) {
    const int Z = c->p.zones;
    hipLaunchKernelGGL(zone_make_table, dim3(1), dim3(64), 0, c->stream,
                       c->at<int64_t>(c->off_pop) + c->cur * kZoneMaxZones, Z, c->at<double>(c->off_knots),
                       c->at<double>(c->off_knots) + kMaxKnots, c->n_knots, c->n, c->n_set, c->p.dt_s, c->p.p0,
                       c->p.kT_ev, c->p.hop_over_thickness, c->p.v_factor,
                       c->at<double>(c->off_table) + c->cur * 2 * kZoneMaxZones);
    ZONE_HIP(c, hipGetLastError());
    return KMC_OK;
}

// Read the caller's occupancy into X and the populations of the current
// buffer.  A first pass only counts the ions of every rail (and synchronises),
// so a rejected occupancy leaves the context's state as it was.
kmc_status zone_load(kmc_zone_ctx *c) {
    const int Z = c->p.zones;
    int64_t *pop = c->at<int64_t>(c->off_pop) + c->cur * kZoneMaxZones;
    const dim3 grid((unsigned)((c->p.rails + 3) / 4));
    ZONE_HIP(c, zone_fill(reinterpret_cast<int64_t *>(c->at<int32_t>(c->off_bad)), 1, 0, c->stream));
    hipLaunchKernelGGL(zone_import, grid, dim3(256), 0, c->stream, c->occ_user, c->at<uint16_t>(c->off_X), c->p.rails,
                       c->p.sites, c->p.ions_per_rail, Z, pop, c->at<int32_t>(c->off_bad), 0);
    ZONE_HIP(c, hipGetLastError());
    int32_t bad = 0;
    ZONE_HIP(c, hipMemcpyAsync(&bad, c->at<int32_t>(c->off_bad), sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    ZONE_HIP(c, hipStreamSynchronize(c->stream));
    if (bad) return record_error(KMC_EINVAL, "a rail of the occupancy does not hold ions_per_rail ions");
    ZONE_HIP(c, zone_fill(pop, Z, 0, c->stream));
    hipLaunchKernelGGL(zone_import, grid, dim3(256), 0, c->stream, c->occ_user, c->at<uint16_t>(c->off_X), c->p.rails,
                       c->p.sites, c->p.ions_per_rail, Z, pop, c->at<int32_t>(c->off_bad), 1);
    ZONE_HIP(c, hipGetLastError());
    return zone_refresh_table(c);
}

}  // namespace

extern "C" {

kmc_status kmc_zone_workspace_bytes(const kmc_zone_params *params, size_t *bytes) {
    kmc_status s = zone_validate(params);
    if (s != KMC_OK) return s;
    if (!bytes) return record_error(KMC_EINVAL, "bytes is NULL");
    kmc_zone_ctx c;
    c.p = *params;
    zone_layout(&c);
    *bytes = c.total;
    return KMC_OK;
}

kmc_status kmc_zone_init(const kmc_zone_params *params, int8_t *occ_dev, void *workspace_dev, size_t ws_bytes,
                         void *stream, kmc_zone_ctx **out) {
    kmc_status s = zone_validate(params);
    if (s != KMC_OK) return s;
    if (!out || !occ_dev || !workspace_dev) return record_error(KMC_EINVAL, "out, occ_dev and workspace_dev must not be NULL");
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256 != 0)
        return record_error(KMC_EINVAL, "workspace_dev must be 256-byte aligned");
    kmc_zone_ctx *c = new kmc_zone_ctx();
    c->p = *params;
    zone_layout(c);
    if (ws_bytes < c->total) {
        const size_t need = c->total;
        delete c;
        return record_error(KMC_ETOOSMALL, "workspace too small: need " + std::to_string(need) + " bytes");
    }
    c->ws = static_cast<unsigned char *>(workspace_dev);
    c->occ_user = occ_dev;
    c->stream = static_cast<hipStream_t>(stream);
    auto fail_init = [&](kmc_status st) {
        delete c;
        return st;
    };
    if ((s = zone_hip(c, zone_fill(c->at<int64_t>(c->off_bucket), kZoneBuckets * kZoneBucketStride, 0, c->stream),
                      "clear buckets")) != KMC_OK)
        return fail_init(s);
    if ((s = zone_hip(c, zone_fill(reinterpret_cast<int64_t *>(c->at<uint32_t>(c->off_ticket)), (kZoneBuckets + 1) * 16,
                                   0, c->stream),
                      "clear counters")) != KMC_OK)
        return fail_init(s);
    if ((s = zone_hip(c, zone_fill(c->at<int64_t>(c->off_total), 1, 0, c->stream), "clear total")) != KMC_OK)
        return fail_init(s);
    ZoneKnots k{};
    hipLaunchKernelGGL(zone_set_knots, dim3(1), dim3(64), 0, c->stream, c->at<double>(c->off_knots),
                       c->at<double>(c->off_knots) + kMaxKnots, k);
    if ((s = zone_hip(c, hipGetLastError(), "install 0 V")) != KMC_OK) return fail_init(s);
    if ((s = zone_load(c)) != KMC_OK) return fail_init(s);
    *out = c;
    return KMC_OK;
}

kmc_status kmc_zone_load_occupancy(kmc_zone_ctx *c) {
    kmc_status s = zone_usable(c);
    if (s != KMC_OK) return s;
    return zone_load(c);
}

kmc_status kmc_zone_set_bias_protocol(kmc_zone_ctx *c, const double *t_s, const double *v_volt, int32_t n_knots) {
    kmc_status s = zone_usable(c);
    if (s != KMC_OK) return s;
    if (n_knots < 1 || n_knots > kMaxKnots) return record_error(KMC_EINVAL, "n_knots must be in [1, 64]");
    if (!t_s || !v_volt) return record_error(KMC_EINVAL, "knot arrays are NULL");
    ZoneKnots k{};
    for (int i = 0; i < n_knots; ++i) {
        if (!std::isfinite(t_s[i]) || !std::isfinite(v_volt[i])) return record_error(KMC_EINVAL, "knots must be finite");
        if (i > 0 && t_s[i] < t_s[i - 1]) return record_error(KMC_EINVAL, "knot times must be nondecreasing");
        k.t[i] = t_s[i];
        k.v[i] = v_volt[i];
    }
    hipLaunchKernelGGL(zone_set_knots, dim3(1), dim3(64), 0, c->stream, c->at<double>(c->off_knots),
                       c->at<double>(c->off_knots) + kMaxKnots, k);
    ZONE_HIP(c, hipGetLastError());
    c->n_knots = n_knots;
    c->n_set = c->n;
    return zone_refresh_table(c);
}

kmc_status kmc_zone_run_steps(kmc_zone_ctx *c, int64_t n_steps, int32_t *net_dev, int32_t *zone_dev) {
    kmc_status s = zone_usable(c);
    if (s != KMC_OK) return s;
    if (n_steps < 0) return record_error(KMC_EINVAL, "n_steps < 0");
    if (c->n + n_steps > (int64_t)0xffffffffLL) return record_error(KMC_EUNSUPPORTED, "step counter would reach 2^32");
    if (n_steps == 0) return KMC_OK;
    ZoneArgs a{};
    a.X = c->at<uint16_t>(c->off_X);
    a.rails = c->p.rails;
    a.ions = c->p.ions_per_rail;
    a.sites = c->p.sites;
    a.zones = c->p.zones;
    a.p0 = c->p.p0;
    a.kT = c->p.kT_ev;
    a.hot = c->p.hop_over_thickness;
    a.v_factor = c->p.v_factor;
    a.dt = c->p.dt_s;
    a.key0 = (uint32_t)(c->p.seed & 0xffffffffu);
    a.key1 = (uint32_t)(c->p.seed >> 32);
    a.knot_t = c->at<double>(c->off_knots);
    a.knot_v = a.knot_t + kMaxKnots;
    a.n_knots = c->n_knots;
    a.n_set = c->n_set;
    a.bucket = c->at<int64_t>(c->off_bucket);
    a.ticket = c->at<uint32_t>(c->off_ticket);
    a.net_out = net_dev;
    a.zone_out = zone_dev;
    a.net_total = c->at<int64_t>(c->off_total);
    const int64_t pairs = ((int64_t)c->p.rails + 1) / 2;
    const int64_t per_wg = (int64_t)(kZoneBlock / 64) * kZonePairsPerIter;
    const unsigned grid = (unsigned)std::min<int64_t>((pairs + per_wg - 1) / per_wg, kZoneMaxGrid);
    int64_t *pop = c->at<int64_t>(c->off_pop);
    double *table = c->at<double>(c->off_table);
    for (int64_t k = 0; k < n_steps; ++k) {
        a.n = c->n + k;
        a.row = k;
        a.table = table + c->cur * 2 * kZoneMaxZones;
        a.table_next = table + (1 - c->cur) * 2 * kZoneMaxZones;
        a.pop_next = pop + (1 - c->cur) * kZoneMaxZones;
        hipLaunchKernelGGL(zone_step, dim3(grid), dim3(kZoneBlock), 0, c->stream, a);
        ZONE_HIP(c, hipGetLastError());
        c->cur = 1 - c->cur;
    }
    hipLaunchKernelGGL(zone_export, dim3((unsigned)((c->p.rails + 3) / 4)), dim3(256), 0, c->stream,
                       c->at<uint16_t>(c->off_X), c->occ_user, c->p.rails, c->p.sites, c->p.ions_per_rail);
    ZONE_HIP(c, hipGetLastError());
    c->n += n_steps;
    return KMC_OK;
}

kmc_status kmc_zone_read_positions(kmc_zone_ctx *c, int32_t *X_host, size_t count) {
    kmc_status s = zone_usable(c);
    if (s != KMC_OK) return s;
    if (!X_host) return record_error(KMC_EINVAL, "X_host is NULL");
    const size_t n = (size_t)c->p.rails * (size_t)c->p.ions_per_rail;
    if (count < n) return record_error(KMC_ETOOSMALL, "X_host holds fewer than rails * ions_per_rail entries");
    std::vector<uint16_t> tmp(n);
    if (n > 0) {
        ZONE_HIP(c, hipMemcpyAsync(tmp.data(), c->at<uint16_t>(c->off_X), sizeof(uint16_t) * n, hipMemcpyDeviceToHost,
                                   c->stream));
    }
    ZONE_HIP(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < n; ++i) X_host[i] = tmp[i];
    return KMC_OK;
}

kmc_status kmc_zone_get_step(kmc_zone_ctx *c, int64_t *step) {
    if (!c || !step) return record_error(KMC_EINVAL, "NULL argument");
    *step = c->n;
    return KMC_OK;
}

void kmc_zone_destroy(kmc_zone_ctx *c) {
    if (!c) return;
    if (!c->poisoned) (void)hipStreamSynchronize(c->stream);
    delete c;
}

}  // extern "C"
