// Long-range Coulomb term from a potential kept at every site and updated hop
// by hop (the KMC_PHI_FIXED precision of include/kmc.h).
//
// The potential of site s of rail r is the ion field of main text section 3,
//     phi(r, s) = sum over the distinct rails r' within rail_range and the
//                 sites j of occ(r', j) K(s - j, dist(r, r')),   K(0, 0) = 0,
// and a hop o -> t then has dE_coul = phi(t) - K(1, 0) - phi(o) (the ion at o
// contributes K(1, 0) to phi(t); the definition gives this exactly).  phi is
// held in fixed point: every kernel value is rounded once to an integer
// multiple of 2^-F V (F from the largest |phi| the kernel allows, so that no
// sum overflows 63 bits), and phi is the exact integer sum of those values.
// Integer sums do not depend on their order, so a potential updated by
// thousands of hops in any order equals the one computed from scratch bit
// for bit.
//
// Per half-step:
//   * phifix_decide<h>: one thread per Philox block (the four bonds of
//     parity h in eight sites).  The exact class prefilter of the other hop
//     kernels rejects almost every candidate on its Philox word alone; a
//     survivor reads phi at its two sites and is decided in binary64.  An
//     accepted hop flips its two sites in place (a bond's two sites belong to
//     no other bond of the half-step, and no thread reads a site another
//     thread writes) and is appended to the hop list.
//   * phifix_update: every listed hop adds K(s - t) - K(s - o) to phi on the
//     sites of the distinct rails within rail_range whose window it entered
//     or left (one workgroup per hop, integer atomics).  A half-step with more
//     hops than the list holds recomputes every rail from scratch instead.
#include "kmc_phifix.h"

#include <algorithm>

#include "kmc_device.h"

namespace kmc {

namespace {

constexpr int kPhiBlock = 256;
constexpr int kPhiUpdateGrid = 512;
constexpr int kPhiMaxRails = 2 * kMaxRailRange + 1;

// phi of one rail from scratch.  The ion positions of every neighbour rail
// are compacted into LDS (one wavefront per rail, in site order), then every
// thread sums the kernel over them for its sites.
__device__ void phifix_rail(const PhiFixArgs &a, int64_t grow, uint16_t *pos, int *cnt) {
    const int d = a.rail_dev[grow], r = a.rail_idx[grow];
    const DevInfo &dv = a.devs[d];
    const int L = dv.sites, R = dv.rails, pitch = dv.pitch;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int8_t *src = a.occ + dv.off_pad;
    for (int k = wave; k < dv.n_nbr; k += kPhiBlock / 64) {
        const int rr = ((r + dv.nbr_off[k]) % R + R) % R;
        const int8_t *row = src + (int64_t)rr * pitch;
        uint16_t *out = pos + k * kPhiMaxSites;
        int base = 0;
        for (int s0 = 0; s0 < L; s0 += 64) {
            const int s = s0 + lane;
            const bool occd = s < L && (row[s] & 1);
            const uint64_t m = __ballot(occd);
            if (occd) out[base + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)s;
            base += __popcll(m);
        }
        if (lane == 0) cnt[k] = base;
    }
    __syncthreads();
    const int cs = a.cutoff + 1;
    for (int s = tid; s < L; s += kPhiBlock) {
        int64_t acc = 0;
        for (int k = 0; k < dv.n_nbr; ++k) {
            const int64_t *kt = a.kfix + dv.nbr_dist[k] * cs;
            const uint16_t *p = pos + k * kPhiMaxSites;
            const int nk = cnt[k];
            for (int i = 0; i < nk; ++i) {
                const int ds = abs(s - (int)p[i]);
                acc += ds <= a.cutoff ? kt[ds] : 0;
            }
        }
        const int64_t at = a.out_unpadded ? dv.off + (int64_t)r * L + s : dv.off_pad + (int64_t)r * pitch + s;
        a.phi[at] = acc;
    }
    __syncthreads();  // pos and cnt are reused by the next rail
}

// The change of phi by one hop o -> t of rail r of device d: on every
// distinct rail within rail_range, the sites whose window holds o or t get
// K(s - t) - K(s - o) (K(0, 0) = 0 takes care of the two sites themselves).
// The neighbour rails' rows and distances are staged in LDS first.  The
// additions are atomics that return nothing; since the memory counter also
// waits for them, the kernel values of a batch of kBatch additions are read
// before any of the batch is issued (from the LDS copy of the table when it
// fits, kLdsTable, else from global memory).
constexpr int kBatch = 4;

template <bool kLdsTable>
__device__ void phifix_hop(const PhiFixArgs &a, const int64_t *kt, uint4 hop, int64_t *nb_row, int *nb_dist) {
    const int d = (int)hop.x, r = (int)hop.y, s = (int)hop.z;
    const int o = hop.w == 0u ? s : s + 1, t = hop.w == 0u ? s + 1 : s;
    const DevInfo &dv = a.devs[d];
    const int L = dv.sites, R = dv.rails, n_nbr = dv.n_nbr;
    const int cut = a.cutoff, cs = cut + 1;
    if ((int)threadIdx.x < n_nbr) {
        const int k = threadIdx.x;
        const int rr = ((r + dv.nbr_off[k]) % R + R) % R;
        nb_row[k] = dv.off_pad + (int64_t)rr * dv.pitch;
        nb_dist[k] = dv.nbr_dist[k] * cs;
    }
    __syncthreads();
    int lo = s - cut, hi = s + 1 + cut;
    lo = lo < 0 ? 0 : lo;
    hi = hi > L - 1 ? L - 1 : hi;
    const int span = hi - lo + 1;
    const int work = span * n_nbr;
    unsigned long long *phi = reinterpret_cast<unsigned long long *>(a.phi);
    for (int i0 = threadIdx.x; i0 < work; i0 += kBatch * kPhiBlock) {
        int64_t delta[kBatch], at[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const int i = i0 + j * kPhiBlock;
            delta[j] = 0;
            at[j] = 0;
            if (i < work) {
                const int k = i / span, x = lo + (i - k * span);
                const int64_t *ktr = kt + nb_dist[k];
                const int dt_ = abs(x - t), do_ = abs(x - o);
                delta[j] = (dt_ <= cut ? ktr[dt_] : 0) - (do_ <= cut ? ktr[do_] : 0);
                at[j] = nb_row[k] + x;
            }
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j)
            if (delta[j] != 0) atomicAdd(phi + at[j], (unsigned long long)delta[j]);
    }
    __syncthreads();  // nb_row / nb_dist are rewritten by the next hop
}

__global__ __launch_bounds__(kPhiBlock) void phifix_update(PhiFixArgs a) {
    __shared__ __align__(16) uint16_t pos[kPhiMaxRails * kPhiMaxSites];
    __shared__ int cnt[kPhiMaxRails];
    __shared__ int64_t nb_row[kPhiMaxRails];
    __shared__ int nb_dist[kPhiMaxRails];
    const int64_t count =
        a.full ? 0 : __hip_atomic_load(a.hop_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (a.full || count > a.hop_cap) {
        for (int64_t g = blockIdx.x; g < a.rails_total; g += gridDim.x) phifix_rail(a, g, pos, cnt);
        return;
    }
    if ((int64_t)blockIdx.x >= count) return;
    // the kernel table, staged in LDS (the rail path's position buffer) when it fits
    const int n_kt = (a.rail_range + 1) * (a.cutoff + 1);
    if (n_kt * (int)sizeof(int64_t) <= (int)sizeof(pos)) {
        int64_t *lk = reinterpret_cast<int64_t *>(pos);
        for (int i = threadIdx.x; i < n_kt; i += kPhiBlock) lk[i] = a.kfix[i];
        __syncthreads();
        for (int64_t i = blockIdx.x; i < count; i += gridDim.x) phifix_hop<true>(a, lk, a.hops[i], nb_row, nb_dist);
    } else {
        for (int64_t i = blockIdx.x; i < count; i += gridDim.x)
            phifix_hop<false>(a, a.kfix, a.hops[i], nb_row, nb_dist);
    }
}

// Decisions of half-step H from the fixed-point potential; see the file
// comment.  A workgroup takes a run of consecutive rails of one device
// (tile.r0, tile.nr); bpr = pitch / 8 threads share a rail, so the workgroup
// covers 256 / bpr rails per pass, and every thread loads its next rail's
// block before deciding the current one.  The bias and the stage-0 threshold
// are evaluated once per workgroup, the tallies summed in LDS and added to
// the device's row once.
template <int H>
__global__ __launch_bounds__(kPhiBlock) void phifix_decide(HopArgs a, PhiFixDecide x) {
    __shared__ int32_t tally[1 + kDeciles];  // net hops and decile changes of the run
    __shared__ double v_wg;
    __shared__ uint32_t thr0_wg;
    const int tid = threadIdx.x;
    const int64_t n = a.ctl.n_base + a.step_in_chunk;
    // the previous half-step's list (the other parity) was consumed by its
    // update kernel: clear its count for the next half-step
    if (blockIdx.x == 0 && tid == 0)
        __hip_atomic_store(a.hop_ctl + (1 - H), (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const Tile tile = a.dtiles[blockIdx.x];
    const int d = tile.d;
    const DevInfo &dv = a.devs[d];
    const int L = dv.sites, pitch = dv.pitch, bpr = pitch / 8;
    if (tid <= kDeciles) tally[tid] = 0;
    if (tid == 0) {
        const double V = protocol_voltage(a.knot_t + d * kMaxKnots, a.knot_v + d * kMaxKnots, dv.n_knots,
                                          (double)(n - dv.n_set) * a.dt);
        v_wg = V;
        thr0_wg = class_threshold(a.c0, a.beta, a.alpha, V, L, dv.ea_min, dv.ea_step, dv.coul_bound, 0);
    }
    const int per_pass = kPhiBlock / bpr;
    const int slot = tid / bpr, b = tid - slot * bpr, s0 = 8 * b;
    const int r_end = tile.r0 + tile.nr;
    int8_t *dev_occ = a.occ_out + dv.off_pad;
    auto load = [&](int r, uint2 &v, uint32_t &nxt) {
        const int8_t *row = dev_occ + (int64_t)r * pitch;
        v = *reinterpret_cast<const uint2 *>(row + s0);
        nxt = (H == 1 && s0 + 8 < pitch) ? (uint32_t)(uint8_t)row[s0 + 8] : 0u;
    };
    int r = tile.r0 + slot;
    uint2 v_next = make_uint2(0u, 0u);
    uint32_t nxt_next = 0u;
    if (slot < per_pass && r < r_end) load(r, v_next, nxt_next);
    __syncthreads();
    const double V = v_wg;
    const uint32_t thr0 = thr0_wg;
    const int last = L - 2 - s0;  // bond (s0+k, s0+k+1) exists iff k <= last
    const uint32_t exist = last >= 7 ? 0xFFu : (last < 0 ? 0u : ((2u << last) - 1u));
    for (; slot < per_pass && r < r_end; r += per_pass) {
        const uint2 v = v_next;
        const uint32_t nxt = nxt_next;
        if (r + per_pass < r_end) load(r + per_pass, v_next, nxt_next);
        const uint4 blk = philox4x32_10((uint32_t)b, (uint32_t)r, (uint32_t)n, ((uint32_t)d << 4) | (uint32_t)H,
                                        a.key0, a.key1);
        const uint32_t bits = (((v.x & 0x01010101u) * 0x01020408u) >> 24 & 0xFu) |
                              ((((v.y & 0x01010101u) * 0x01020408u) >> 24 & 0xFu) << 4) | ((nxt & 1u) << 8);
        const uint32_t cand = (bits ^ (bits >> 1)) & (H ? 0xAAu : 0x55u) & exist;
        uint32_t sv = 0;  // bit i: bond i of the block passes stage 0
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (((cand >> (H + 2 * i)) & 1u) && word_of(blk, i) <= thr0) sv |= 1u << i;
        while (sv) {  // rare
            const int i = __builtin_ctz(sv);
            sv &= sv - 1;
            const int k = H + 2 * i, s = s0 + k;
            const bool first = (bits >> k) & 1u;
            const int o = first ? s : s + 1, t = first ? s + 1 : s;
            auto byte_at = [&](int site) {
                const int j = site - s0;
                return j < 8 ? ((j < 4 ? v.x : v.y) >> (8 * (j & 3))) & 0xFFu : nxt;
            };
            const uint32_t ob = byte_at(o), tb = byte_at(t);
            const uint32_t w = word_of(blk, i);
            if (w > class_threshold(a.c0, a.beta, a.alpha, V, L, dv.ea_min, dv.ea_step, dv.coul_bound,
                                    (int)(ob >> 1)))
                continue;
            // phi(t) - K(1, 0) - phi(o), exact in the fixed-point units, then
            // one rounding to binary64
            const int64_t prow = dv.off_pad + (int64_t)r * pitch;
            const int64_t diff = x.phi[prow + t] - x.k10 - x.phi[prow + o];
            const double e_coul = ldexp((double)diff, -x.frac_bits);
            const double e_app = ((a.alpha * V) * (double)(t - o)) / (double)L;
            const double ea = a.ea ? reinterpret_cast<const double *>(a.ea)[dv.off + (int64_t)r * L + o] : a.ea_scalar;
            if (decide_hop<double>(e_app + e_coul, ea, w, a.beta, a.c0, a.log, d, H, n, r, s)) {
                int8_t *row = dev_occ + (int64_t)r * pitch;
                row[o] = (int8_t)(ob ^ 1u);
                row[t] = (int8_t)(tb ^ 1u);
                const int64_t k_hop = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(a.hop_ctl + H), 1ull);
                if (k_hop < a.hop_cap) a.hops[k_hop] = make_uint4((uint32_t)d, (uint32_t)r, (uint32_t)s, first ? 0u : 1u);
                atomicAdd(&tally[0], t < o ? 1 : -1);
                const int qo = (10 * o) / L, qt = (10 * t) / L;
                if (qo != qt) {
                    atomicAdd(&tally[1 + qo], -1);
                    atomicAdd(&tally[1 + qt], 1);
                }
            }
        }
    }
    __syncthreads();
    if (tid <= kDeciles && tally[tid] != 0) {
        const int64_t base = (n - a.ctl.tally_base) * a.n_devices + d;
        atomicAdd(tid == 0 ? &a.tally_net[base] : &a.tally_dec[base * kDeciles + tid - 1], tally[tid]);
    }
}

// The padded potential in the caller's layout (one workgroup per rail, grid-stride).
__global__ __launch_bounds__(kPhiBlock) void phifix_export(const int64_t *phi_pad, int64_t *out, const DevInfo *devs,
                                                          const int32_t *rail_dev, const int32_t *rail_idx,
                                                          int64_t rails_total) {
    for (int64_t g = blockIdx.x; g < rails_total; g += gridDim.x) {
        const DevInfo &dv = devs[rail_dev[g]];
        const int r = rail_idx[g];
        for (int s = threadIdx.x; s < dv.sites; s += kPhiBlock)
            out[dv.off + (int64_t)r * dv.sites + s] = phi_pad[dv.off_pad + (int64_t)r * dv.pitch + s];
    }
}

}  // namespace

hipError_t launch_phifix_decide(const HopArgs &a, const PhiFixDecide &x, hipStream_t st) {
    if (a.h == 0) hipLaunchKernelGGL(phifix_decide<0>, dim3(a.n_dtiles), dim3(kPhiBlock), 0, st, a, x);
    else hipLaunchKernelGGL(phifix_decide<1>, dim3(a.n_dtiles), dim3(kPhiBlock), 0, st, a, x);
    return hipGetLastError();
}

hipError_t launch_phifix_update(const PhiFixArgs &a, hipStream_t st) {
    const int64_t grid = a.full ? std::min<int64_t>(a.rails_total, 65535) : kPhiUpdateGrid;
    hipLaunchKernelGGL(phifix_update, dim3((unsigned)grid), dim3(kPhiBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_phifix_export(const int64_t *phi_pad, int64_t *out, const DevInfo *devs, const int32_t *rail_dev,
                                const int32_t *rail_idx, int64_t rails_total, hipStream_t st) {
    const int64_t grid = std::min<int64_t>(rails_total, 65535);
    hipLaunchKernelGGL(phifix_export, dim3((unsigned)grid), dim3(kPhiBlock), 0, st, phi_pad, out, devs, rail_dev,
                       rail_idx, rails_total);
    return hipGetLastError();
}

}  // namespace kmc
