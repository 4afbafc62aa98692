// Persistent hop-step kernel: one launch runs a chunk of steps.
//
// Each workgroup owns a tile (whole rails of one device) and keeps the tile's
// int8 state in LDS for the whole launch, double-buffered: every half-step
// reads the snapshot buffer and writes the other (Jacobi update of the pair
// checkerboard).  The only data that crosses workgroups are the tile's first
// and last rail_range rails, which the Coulomb windows of the neighbouring
// tiles need.  After each half-step a workgroup publishes those edge rails into
// a ring of kRing slots in global memory and bumps its progress counter; a
// neighbour waits for that counter only when one of its survivors has a window
// reaching into the tile, or when it is about to reuse a ring slot the tile may
// still read.  There is no grid-wide barrier, so a workgroup delayed by a
// survivor evaluation does not stall the chip.
//
// Cross-workgroup data (publications, progress counters) is accessed only with
// relaxed agent-scope atomics, which gfx950 executes as coherent (sc1) loads and
// stores; a writer waits for its stores to complete (s_waitcnt on every
// counter, then a workgroup barrier) before one thread stores the counter, and
// a reader loads the data only after it has observed the counter.  Every wait is bounded: on time-out
// the kernel raises a status flag, every workgroup leaves its loop, and the
// host reports the error.
//
// The per-bond work (Philox4x32-10 draw, candidate test, exact prefilter,
// survivor energy, Arrhenius probability and accept test) is the same as in
// hop_half_step.
#include "kmc_device.h"
#include "kmc_internal.h"

namespace kmc {

constexpr int kSpinLimit = 1 << 20;  // about a second of polling

struct PShared {
    double V;
    int32_t n_surv, n_down, n_up, stop;
    int32_t dec[kDeciles];
    uint32_t wtab[kClasses];
};

__device__ __forceinline__ uint64_t progress_tag(uint64_t epoch, int64_t j) { return (epoch << 40) | (uint64_t)j; }

// Wait until tile t has published state j (completed half-steps < j) in this
// launch.  Returns false when the wait timed out or another workgroup did.
__device__ bool wait_progress(const PArgs &a, int t, int64_t j) {
    const uint64_t want = progress_tag(a.epoch, j);
    int spins = 0;
    while (__hip_atomic_load(&a.progress[(int64_t)t * 8], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
        if (__hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        if (++spins > kSpinLimit) {
            __hip_atomic_store(a.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

template <typename Real>
__global__ __launch_bounds__(kPMaxBlock) void hop_persistent(PArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ PShared sh;

    const int ti = tile_of_block(blockIdx.x, a.n_tiles);
    const PTile tile = a.tiles[ti];
    const DevInfo &dv = a.devs[tile.d];
    const int R = dv.rails, L = dv.sites, P = dv.pitch;
    const int m = a.rail_range;
    const int p16 = P / kChunkSites;
    const int nr = tile.nr;
    const int n_chunks = nr * p16;
    const int cap = nr * P / 2;
    const int tid = threadIdx.x, bdim = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, n_waves = bdim >> 6;
    const bool single = tile.prev == ti && tile.next == ti;

    unsigned char *S0 = smem;
    unsigned char *S1 = smem + nr * P;
    uint32_t *sv_pos = reinterpret_cast<uint32_t *>(smem + 2 * nr * P);
    uint32_t *sv_w = sv_pos + cap;
    Real *sv_ea = reinterpret_cast<Real *>(sv_w + cap);
    Real *kt_lds = sv_ea + cap;
    const int kt_stride = a.cutoff + 1;
    const int n_kt = (m + 1) * kt_stride;
    const bool kt_in_lds = n_kt <= kLdsTableMax;
    const Real *kt_glob = std::is_same<Real, double>::value ? reinterpret_cast<const Real *>(a.ktab64)
                                                            : reinterpret_cast<const Real *>(a.ktab32);
    const Real *kt = kt_in_lds ? kt_lds : kt_glob;
    const int band_words = P / 8;                 // 64-bit words per published rail
    const int slot_words = 2 * m * band_words;    // one ring slot
    const uint64_t epoch = a.epoch;
    const int64_t j0 = 2 * a.ctl->n_base;
    const Real beta_r = (Real)a.beta, c0_r = (Real)a.c0, alpha_r = (Real)a.alpha;

    // load the tile and the kernel table
    int8_t *gstate = a.occ + dv.off_pad + (int64_t)tile.r0 * P;
    for (int c = tid; c < n_chunks; c += bdim) {
        const int row = c / p16, col = c - row * p16;
        *reinterpret_cast<uint4 *>(S0 + row * P + col * kChunkSites) =
            *reinterpret_cast<const uint4 *>(gstate + (int64_t)row * P + col * kChunkSites);
    }
    if (kt_in_lds)
        for (int i = tid; i < n_kt; i += bdim) kt_lds[i] = kt_glob[i];
    if (tid == 0) sh.stop = 0;
    __syncthreads();

    // Publication of the edge rails of `state` as state j, in two parts: the
    // stores are issued at the end of half-step j-1 and completed (s_waitcnt on
    // every counter: a workgroup-scope fence does not wait for global stores on
    // gfx950, then a barrier) during half-step j, just before the progress
    // counter announces state j; the store latency overlaps the Philox work.
    auto publish_issue = [&](const unsigned char *state, int64_t j) {
        uint64_t *slot = a.pub + (int64_t)ti * a.pub_stride + (int64_t)(j % kRing) * slot_words;
        for (int i = tid; i < slot_words; i += bdim) {
            const int b = i / band_words, wd = i - b * band_words;
            const int row = b < m ? b : nr - 2 * m + b;
            const uint64_t word = *reinterpret_cast<const uint64_t *>(state + row * P + wd * 8);
            __hip_atomic_store(slot + i, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    };
    auto publish_complete = [&](int64_t j) {  // contains a workgroup barrier
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0)
            __hip_atomic_store(&a.progress[(int64_t)ti * 8], progress_tag(epoch, j), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    };
    if (!single) {
        publish_issue(S0, j0);
        publish_complete(j0);
    }

    for (int js = 0; js < 2 * a.n_steps; ++js) {
        const int64_t j = j0 + js;
        const int64_t n = j >> 1;
        const int h = (int)(j & 1);
        unsigned char *cur = (js & 1) ? S1 : S0;
        unsigned char *nxt = (js & 1) ? S0 : S1;
        if (h == 0) {
            const double V = protocol_voltage(a.knot_t + tile.d * kMaxKnots, a.knot_v + tile.d * kMaxKnots,
                                              dv.n_knots, (double)(n - dv.n_set) * a.dt);
            for (int q = tid; q < kClasses; q += bdim)
                sh.wtab[q] = class_threshold(a.c0, a.beta, a.alpha, V, L, dv.ea_min, dv.ea_step, dv.coul_bound, q);
            if (tid == 0) {
                sh.V = V;
                sh.n_down = 0;
                sh.n_up = 0;
                for (int q = 0; q < kDeciles; ++q) sh.dec[q] = 0;
            }
        }
        if (tid == 0) {
            sh.n_surv = 0;
            // the slot this half-step will write held state j+1-kRing, which the
            // neighbours read during their half-step j+1-kRing
            const int64_t need = j + 2 - kRing;
            if (!single && need > j0) {
                bool ok = wait_progress(a, tile.prev, need);
                if (ok && tile.next != tile.prev) ok = wait_progress(a, tile.next, need);
                if (!ok) sh.stop = 1;
            }
        }
        for (int c = tid; c < n_chunks; c += bdim) {
            const int off = (c / p16) * P + (c - (c / p16) * p16) * kChunkSites;
            *reinterpret_cast<uint4 *>(nxt + off) = *reinterpret_cast<const uint4 *>(cur + off);
        }
        __syncthreads();
        if (sh.stop) break;

        // candidates, Philox words, exact two-stage prefilter
        const uint32_t thr0 = sh.wtab[0];
        const uint32_t ctr3 = ((uint32_t)tile.d << 4) | (uint32_t)h;
        const uint32_t pmask = h ? 0xAAAAu : 0x5555u;
        for (int c = tid; c < n_chunks; c += bdim) {
            const int row = c / p16;
            const int s0 = (c - row * p16) * kChunkSites;
            const unsigned char *rp = cur + row * P;
            const uint4 v = *reinterpret_cast<const uint4 *>(rp + s0);
            const uint32_t nx = (h && s0 + kChunkSites < P) ? (uint32_t)rp[s0 + kChunkSites] : 0u;
            const uint32_t bits = occ_bits(v) | ((nx & 1u) << 16);
            uint32_t cand = (bits ^ (bits >> 1)) & pmask;
            const int last = L - 2 - s0;
            if (last < 15) cand &= last < 0 ? 0u : ((2u << last) - 1u);
            if (cand == 0) continue;
            const uint32_t rail = (uint32_t)(tile.r0 + row);
            const uint4 blkA = philox4x32_10((uint32_t)(s0 >> 3), rail, (uint32_t)n, ctr3, a.key0, a.key1);
            const uint4 blkB = philox4x32_10((uint32_t)(s0 >> 3) + 1u, rail, (uint32_t)n, ctr3, a.key0, a.key1);
            uint32_t sv = 0;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int bit = h + 2 * jj;
                if (((cand >> bit) & 1u) && word_of(blkA, jj) <= thr0) sv |= 1u << bit;
                if (((cand >> (bit + 8)) & 1u) && word_of(blkB, jj) <= thr0) sv |= 1u << (bit + 8);
            }
            while (sv) {  // rare: the threshold of the origin's barrier class
                const int bit = __builtin_ctz(sv);
                sv &= sv - 1;
                const int ob = ((bits >> bit) & 1u) ? bit : bit + 1;
                const uint32_t obyte = ob < kChunkSites ? (word_of(v, ob >> 2) >> (8 * (ob & 3))) & 0xFFu : nx;
                const uint32_t w = word_of8(blkA, blkB, bit >> 1);
                if (w <= sh.wtab[obyte >> 1]) {
                    const int k = atomicAdd(&sh.n_surv, 1);
                    sv_pos[k] = ((uint32_t)row << 13) | (uint32_t)(s0 + bit);
                    sv_w[k] = w;
                    Real ea;
                    if (a.ea) ea = reinterpret_cast<const Real *>(a.ea)[dv.off + (int64_t)rail * L + s0 + ob];
                    else ea = (Real)a.ea_scalar;
                    sv_ea[k] = ea;
                }
            }
        }
        if (!single && js > 0) {
            publish_complete(j);  // state j (issued at the end of half-step j-1); includes the barrier
        } else {
            __syncthreads();
        }

        // survivors: one wavefront each; window rows from the snapshot in LDS or
        // from the neighbours' publications of state j
        const int n_surv = sh.n_surv;
        const int slot = (int)(j % kRing);
        for (int i = wave; i < n_surv; i += n_waves) {
            const int srow = (int)(sv_pos[i] >> 13), s = (int)(sv_pos[i] & 8191u);
            const unsigned char *rp = cur + srow * P;
            const int o = (rp[s] & 1) ? s : s + 1;
            const int t = (rp[s] & 1) ? s + 1 : s;
            int ok = 1;
            if (!single && lane == 0) {
                if (srow - m < 0) ok = wait_progress(a, tile.prev, j);
                if (ok && srow + m >= nr) ok = wait_progress(a, tile.next, j);
                if (!ok) sh.stop = 1;
            }
            ok = __shfl(ok, 0, 64);
            if (!ok) break;
            int lo = s - a.cutoff, hi = s + 1 + a.cutoff;
            lo = lo < 0 ? 0 : lo;
            hi = hi > L - 1 ? L - 1 : hi;
            Real part = (Real)0;
            for (int k = 0; k < dv.n_nbr; ++k) {
                const int off = dv.nbr_off[k];
                const Real *ktr = kt + dv.nbr_dist[k] * kt_stride;
                int rho = srow + off;
                const unsigned char *lrow = nullptr;
                const uint64_t *prow = nullptr;
                if (single) {
                    rho = ((rho % R) + R) % R;
                    lrow = cur + rho * P;
                } else if (rho >= 0 && rho < nr) {
                    lrow = cur + rho * P;
                } else if (rho < 0) {
                    prow = a.pub + (int64_t)tile.prev * a.pub_stride + (int64_t)slot * slot_words +
                           (2 * m + rho) * band_words;
                } else {
                    prow = a.pub + (int64_t)tile.next * a.pub_stride + (int64_t)slot * slot_words +
                           (rho - nr) * band_words;
                }
                for (int jj = lo + lane; jj <= hi; jj += 64) {
                    uint32_t byte;
                    if (lrow) byte = lrow[jj];
                    else byte = (uint32_t)(__hip_atomic_load(prow + (jj >> 3), __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT) >> (8 * (jj & 7)));
                    int occ = byte & 1;
                    if (off == 0 && (jj == o || jj == t)) occ = 0;
                    const int dt_ = t - jj < 0 ? jj - t : t - jj;
                    const int do_ = o - jj < 0 ? jj - o : o - jj;
                    const Real kt_v = dt_ > a.cutoff ? (Real)0 : ktr[dt_];
                    const Real ko_v = do_ > a.cutoff ? (Real)0 : ktr[do_];
                    part += occ ? (kt_v - ko_v) : (Real)0;
                }
            }
#pragma unroll
            for (int sh_ = 32; sh_ >= 1; sh_ >>= 1) part += __shfl_xor(part, sh_, 64);
            if (lane == 0) {
                const Real e_app = ((alpha_r * (Real)sh.V) * (Real)(t - o)) / (Real)L;
                const int srail = tile.r0 + srow;
                if (decide_hop<Real>(e_app + part, sv_ea[i], sv_w[i], beta_r, c0_r, a.log, tile.d, h, n, srail, s)) {
                    nxt[srow * P + s] ^= 1;
                    nxt[srow * P + s + 1] ^= 1;
                    if (t < o) atomicAdd(&sh.n_down, 1);
                    else atomicAdd(&sh.n_up, 1);
                    const int qo = (10 * o) / L, qt = (10 * t) / L;
                    if (qo != qt) {
                        atomicAdd(&sh.dec[qo], -1);
                        atomicAdd(&sh.dec[qt], 1);
                    }
                }
            }
        }
        __syncthreads();
        if (sh.stop) break;

        if (!single) publish_issue(nxt, j + 1);
        if (h == 1 && tid == 0 && (sh.n_down | sh.n_up)) {
            const int64_t base = (n - a.ctl->tally_base) * a.n_devices + tile.d;
            atomicAdd(&a.tally_net[base], sh.n_down - sh.n_up);
            for (int q = 0; q < kDeciles; ++q)
                if (sh.dec[q]) atomicAdd(&a.tally_dec[base * kDeciles + q], sh.dec[q]);
        }
    }

    // announce the last state, write the tile back (an even number of
    // half-steps ends in S0)
    if (!single && !sh.stop) publish_complete(j0 + 2 * (int64_t)a.n_steps);
    __syncthreads();
    for (int c = tid; c < n_chunks; c += bdim) {
        const int row = c / p16, col = c - row * p16;
        *reinterpret_cast<uint4 *>(gstate + (int64_t)row * P + col * kChunkSites) =
            *reinterpret_cast<const uint4 *>(S0 + row * P + col * kChunkSites);
    }
}

hipError_t launch_persistent(const PArgs &a, int block, size_t lds, bool fp64, hipStream_t st) {
    PArgs args = a;
    void *kargs[] = {&args};
    const void *fn = fp64 ? (const void *)hop_persistent<double> : (const void *)hop_persistent<float>;
    return hipLaunchCooperativeKernel(fn, dim3(a.n_tiles), dim3(block), kargs, (unsigned)lds, st);
}

hipError_t persistent_capacity(int block, size_t lds, bool fp64, int *blocks_per_cu) {
    const void *fn = fp64 ? (const void *)hop_persistent<double> : (const void *)hop_persistent<float>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, block, lds);
}

}  // namespace kmc
