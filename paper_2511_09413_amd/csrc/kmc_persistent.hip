// Persistent hop-step kernel: one launch runs a chunk of up to 1024 steps.
//
// Each workgroup owns a tile (whole rails of one device) and keeps it in LDS
// for the whole launch: the occupancy as bits (double-buffered: every
// half-step reads the snapshot and writes the other buffer, the Jacobi update
// of the pair checkerboard) and the barrier class of every site as a byte.
// One lane owns 16 consecutive sites of a rail for the whole launch, so its
// coordinates and Philox counter words stay in registers.
//
// Only the tile's first and last rail_range rails cross workgroups: the
// Coulomb windows of the neighbouring tiles reach into them.  After every
// half-step the workgroup writes those rails into its own slot for that state
// (a slot per state of the launch, never reused within it) as 64-bit words:
// 32 occupancy bits plus a 32-bit tag naming the state (launch epoch,
// half-step).  Data and tag travel in one store, so a writer never waits; a
// reader that needs a neighbour's rail (a survivor whose window crosses the
// tile edge, which is rare) polls the words it needs until their tags name the
// state it wants.  Nothing else couples the workgroups: there is no grid-wide
// barrier and no slot reuse to guard, so a workgroup waits only when one of its
// survivors needs a neighbour's state that is not published yet.  Every wait
// is bounded: on time-out the kernel raises a status flag, all workgroups leave
// their loops and the host reports the error.  Cross-workgroup words are
// accessed only with relaxed agent-scope atomics, which gfx950 executes as
// coherent (sc1) loads and stores.
//
// Per bond the work is that of hop_half_step: Philox4x32-10 draw, candidate
// test, exact two-stage prefilter, survivor energy (wavefront-cooperative
// window sum), Arrhenius probability and accept test.
#include "kmc_device.h"
#include "kmc_internal.h"

namespace kmc {

constexpr int kStepWin = 128;        // steps of the per-step tables held in LDS

struct PShared {
    int32_t n_surv[2];            // survivors of even / odd half-steps (reset one half-step ahead)
    int32_t n_down, n_up, stop;
    int32_t dec[kDeciles];
};

__device__ __forceinline__ uint32_t pub_tag(uint64_t epoch, int64_t j_rel) {
    return ((uint32_t)(epoch & 0xFFFFFu) << 12) | (uint32_t)j_rel;
}

template <typename Real>
__global__ __launch_bounds__(kPMaxBlock) void hop_persistent(PArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ PShared sh;
    __shared__ double cls_A[kClasses];

    const int ti = tile_of_block(blockIdx.x, a.n_tiles);
    const PTile tile = a.tiles[ti];
    const DevInfo &dv = a.devs[tile.d];
    const int R = dv.rails, L = dv.sites, P = dv.pitch;
    const int m = a.rail_range;
    const int p16 = P / kChunkSites;
    const int W = (P + 63) / 64;             // 64-bit occupancy words per rail in LDS
    const int W32 = (P + 31) / 32;           // 32-bit data words per published rail
    const int nr = tile.nr;
    const int n_chunks = nr * p16;           // <= blockDim.x (host guarantees)
    const int cap = nr * P / 2;
    const int tid = threadIdx.x, bdim = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, n_waves = bdim >> 6;
    const bool single = tile.prev == ti && tile.next == ti;
    const bool isolated = single || a.rail_range == 0;  // no rail of another tile is ever read

    uint64_t *B0 = reinterpret_cast<uint64_t *>(smem);
    uint64_t *B1 = B0 + nr * W;
    unsigned char *cls = reinterpret_cast<unsigned char *>(B1 + nr * W);
    uint32_t *sv_pos = reinterpret_cast<uint32_t *>(cls + nr * P);  // survivors: row << 13 | bond
    Real *kt_lds = reinterpret_cast<Real *>(sv_pos + cap + (cap & 1));
    const int kt_stride = a.cutoff + 1;
    const int n_kt = (m + 1) * kt_stride;
    const bool kt_in_lds = n_kt <= kLdsTableMax;
    // per-step tables, a window of kStepWin steps refreshed half a window
    // ahead: bias V, g = exp(beta (|alpha V|/L + coul_bound)/2) and the
    // stage-0 threshold of step k at index k % kStepWin
    double *step_V = reinterpret_cast<double *>(
        reinterpret_cast<unsigned char *>(kt_lds) + (kt_in_lds ? ((n_kt * (int)sizeof(Real) + 7) & ~7) : 0));
    double *step_g = step_V + kStepWin;
    uint32_t *step_thr0 = reinterpret_cast<uint32_t *>(step_g + kStepWin);
    const Real *kt_glob = std::is_same<Real, double>::value ? reinterpret_cast<const Real *>(a.ktab64)
                                                            : reinterpret_cast<const Real *>(a.ktab32);
    const Real *kt = kt_in_lds ? kt_lds : kt_glob;
    const int slot_words = 2 * m * W32;      // 64-bit words of one ring slot
    const uint64_t epoch = a.epoch;
    const int64_t j0 = 2 * a.ctl.n_base;
    const Real beta_r = (Real)a.beta, c0_r = (Real)a.c0, alpha_r = (Real)a.alpha;

    // the lane's chunk, fixed for the launch
    const bool has_chunk = tid < n_chunks;
    const int row = has_chunk ? tid / p16 : 0;
    const int s0 = has_chunk ? (tid - row * p16) * kChunkSites : 0;
    const int wi = row * W + (s0 >> 6), sb = s0 & 63;
    const uint32_t rail = (uint32_t)(tile.r0 + row);
    const int last = L - 2 - s0;
    const uint32_t valid = last >= 15 ? 0xFFFFu : (last < 0 ? 0u : ((2u << last) - 1u));
    const bool nx_here = sb < 48;                       // bit s0+16 in the same word
    const bool nx_exists = s0 + kChunkSites < P;

    // load the tile: occupancy bits and barrier classes
    int8_t *gstate = a.occ + dv.off_pad + (int64_t)tile.r0 * P;
    for (int i = tid; i < nr * W; i += bdim) B0[i] = 0;  // padding bits stay 0
    __syncthreads();
    if (has_chunk) {
        const uint4 v = *reinterpret_cast<const uint4 *>(gstate + (int64_t)row * P + s0);
        reinterpret_cast<uint16_t *>(B0)[row * W * 4 + (s0 >> 4)] = (uint16_t)occ_bits(v);
        *reinterpret_cast<uint4 *>(cls + row * P + s0) =
            make_uint4((v.x >> 1) & 0x7F7F7F7Fu, (v.y >> 1) & 0x7F7F7F7Fu, (v.z >> 1) & 0x7F7F7F7Fu,
                       (v.w >> 1) & 0x7F7F7F7Fu);
    }
    if (kt_in_lds)
        for (int i = tid; i < n_kt; i += bdim) kt_lds[i] = kt_glob[i];
    for (int q = tid; q < kClasses; q += bdim) cls_A[q] = exp(-a.beta * (dv.ea_min + (double)q * dv.ea_step));
    auto fill_steps = [&](int k_lo, int k_hi) {  // table entries of steps [k_lo, k_hi)
        for (int k = k_lo + tid; k < k_hi && k < a.n_steps; k += bdim) {
            const double V = protocol_voltage(a.knot_t + tile.d * kMaxKnots, a.knot_v + tile.d * kMaxKnots,
                                              dv.n_knots, (double)((j0 >> 1) + k - dv.n_set) * a.dt);
            const double g = exp(0.5 * a.beta * (fabs(a.alpha * V) / (double)L + dv.coul_bound));
            step_V[k % kStepWin] = V;
            step_g[k % kStepWin] = g;
            step_thr0[k % kStepWin] = threshold_of(a.c0, exp(-a.beta * dv.ea_min), g);
        }
    };
    fill_steps(0, kStepWin);
    if (tid == 0) {
        sh.stop = 0;
        sh.n_surv[0] = 0;
        sh.n_surv[1] = 0;
        sh.n_down = 0;
        sh.n_up = 0;
        for (int q = 0; q < kDeciles; ++q) sh.dec[q] = 0;
    }
    __syncthreads();
    for (int i = tid; i < nr * W; i += bdim) B1[i] = B0[i];  // the first half-step writes B1
    __syncthreads();

    // The edge rails of `state` as state j (no wait: tags validate the data).
    // The stores are issued by the last wavefronts: on gfx950 one counter
    // tracks a wavefront's loads and stores, so the first wavefronts, which
    // load the per-step tables, never wait for publication stores.
    const int pub_first = bdim - ((slot_words + 63) / 64) * 64;
    // word i of a slot: 32 bits of edge rail i / W32 (the first m rails, then
    // the last m); when the last wavefronts have a lane per word, each lane's
    // word is fixed for the launch
    const int pub_i = tid - (pub_first > 0 ? pub_first : 0);
    const bool pub_one = pub_first >= 0;
    int pub_w = 0, pub_sh = 0;
    if (pub_one && pub_i >= 0 && pub_i < slot_words) {
        const int b = pub_i / W32, q = pub_i - b * W32;
        pub_w = (b < m ? b : nr - 2 * m + b) * W + (q >> 1);
        pub_sh = 32 * (q & 1);
    }
    auto publish = [&](const uint64_t *state, int64_t j) {
        uint64_t *slot = a.pub + (int64_t)ti * a.pub_stride + (j - j0) * slot_words;
        const uint64_t tag = (uint64_t)pub_tag(epoch, j - j0) << 32;
        if (pub_one) {
            if (pub_i >= 0 && pub_i < slot_words)
                __hip_atomic_store(slot + pub_i, tag | (uint32_t)(state[pub_w] >> pub_sh), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        for (int i = tid; i < slot_words; i += bdim) {
            const int b = i / W32, q = i - b * W32;
            const int rrow = b < m ? b : nr - 2 * m + b;
            const uint32_t data = (uint32_t)(state[rrow * W + (q >> 1)] >> (32 * (q & 1)));
            __hip_atomic_store(slot + i, tag | data, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    };
    // Wait until word `i` of tile t's slot for state j carries state j's tag
    // and store it in *out; false on time-out.
    auto fetch = [&](int t, int64_t j, int i, uint64_t *out) -> bool {
        const uint64_t *w = a.pub + (int64_t)t * a.pub_stride + (j - j0) * slot_words + i;
        const uint32_t want = pub_tag(epoch, j - j0);
        for (int spins = 0;; ++spins) {
            if (spins >= a.spin_limit) {  // declared hung (at once for a limit of 0)
                __hip_atomic_store(a.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
            const uint64_t v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t tag = (uint32_t)(v >> 32);
            if (tag == want) {
                *out = v;
                return true;
            }
            if (__hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
            __builtin_amdgcn_s_sleep(2);
        }
    };
    if (!isolated) publish(B0, j0);

    for (int js = 0; js < 2 * a.n_steps; ++js) {
        const int64_t j = j0 + js;
        const int64_t n = j >> 1;
        const int h = (int)(j & 1);
        const uint64_t *cur = (js & 1) ? B1 : B0;
        uint64_t *nxt = (js & 1) ? B0 : B1;
        const int kstep = js >> 1;
        // The counter of the next half-step is cleared here, before this
        // half-step's barrier: its last readers (the previous half-step) have
        // either passed that half-step's survivor barrier or read a zero.
        if (tid == 0) sh.n_surv[(js + 1) & 1] = 0;

        // candidates, Philox words, exact two-stage prefilter
        if (has_chunk) {
            const uint64_t word = cur[wi];
            uint32_t bits = (uint32_t)(word >> sb) & 0xFFFFu;
            if (h && nx_exists) bits |= (uint32_t)((nx_here ? (word >> (sb + 16)) : cur[wi + 1]) & 1u) << 16;
            const uint32_t cand = (bits ^ (bits >> 1)) & (h ? 0xAAAAu : 0x5555u) & valid;
            {
                // the key enters each half-step opaquely, so that the compiler
                // derives the round keys on the scalar unit here instead of
                // keeping twenty of them live (and spilled) across the loop
                uint32_t k0 = a.key0, k1 = a.key1;
                asm volatile("" : "+s"(k0), "+s"(k1));
                const uint32_t ctr3 = ((uint32_t)tile.d << 4) | (uint32_t)h;
                const uint4 blkA = philox4x32_10((uint32_t)(s0 >> 3), rail, (uint32_t)n, ctr3, k0, k1);
                const uint4 blkB = philox4x32_10((uint32_t)(s0 >> 3) + 1u, rail, (uint32_t)n, ctr3, k0, k1);
                const uint32_t thr0 = step_thr0[kstep % kStepWin];
                // stage 0: the smallest of the eight words against the largest
                // threshold; only then the candidate bonds' words one by one
                const uint32_t mn = min(min(min(blkA.x, blkA.y), min(blkA.z, blkA.w)),
                                        min(min(blkB.x, blkB.y), min(blkB.z, blkB.w)));
                uint32_t sv = 0;
                if (mn <= thr0) {
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) {
                        const int bit = h + 2 * jj;
                        if (((cand >> bit) & 1u) && word_of(blkA, jj) <= thr0) sv |= 1u << bit;
                        if (((cand >> (bit + 8)) & 1u) && word_of(blkB, jj) <= thr0) sv |= 1u << (bit + 8);
                    }
                }
                while (sv) {  // rare: the threshold of the origin's barrier class
                    const int bit = __builtin_ctz(sv);
                    sv &= sv - 1;
                    const int o = s0 + (((bits >> bit) & 1u) ? bit : bit + 1);
                    const uint32_t w = word_of8(blkA, blkB, bit >> 1);
                    if (w <= threshold_of(a.c0, cls_A[cls[row * P + o]], step_g[kstep % kStepWin])) {
                        const int k = atomicAdd(&sh.n_surv[js & 1], 1);
                        sv_pos[k] = ((uint32_t)row << 13) | (uint32_t)(s0 + bit);
                    }
                }
            }
        }
        lds_barrier();
        if (sh.stop) break;
        if (js > 0 && (js % kStepWin) == 0) fill_steps(kstep + kStepWin / 2, kstep + kStepWin);

        // survivors: one wavefront each
        const int n_surv = sh.n_surv[js & 1];
        for (int i = wave; i < n_surv; i += n_waves) {
            const int srow = (int)(sv_pos[i] >> 13), s = (int)(sv_pos[i] & 8191u);
            const int o = ((cur[srow * W + (s >> 6)] >> (s & 63)) & 1u) ? s : s + 1;
            const int t = (o == s) ? s + 1 : s;
            int lo = s - a.cutoff, hi = s + 1 + a.cutoff;
            lo = lo < 0 ? 0 : lo;
            hi = hi > L - 1 ? L - 1 : hi;
            Real part = (Real)0;
            bool ok = true;
            for (int k = 0; k < dv.n_nbr && ok; ++k) {
                const int off = dv.nbr_off[k];
                const Real *ktr = kt + dv.nbr_dist[k] * kt_stride;
                int rho = srow + off;
                int nb = -1, band = 0;
                if (single) rho = ((rho % R) + R) % R;
                else if (rho < 0) { nb = tile.prev; band = 2 * m + rho; }
                else if (rho >= nr) { nb = tile.next; band = rho - nr; }
                for (int jj = lo + lane; jj <= hi; jj += 64) {
                    uint32_t bit;
                    if (nb < 0) {
                        bit = (uint32_t)(cur[rho * W + (jj >> 6)] >> (jj & 63)) & 1u;
                    } else {
                        uint64_t v = 0;
                        if (!fetch(nb, j, band * W32 + (jj >> 5), &v)) {
                            ok = false;
                            break;
                        }
                        bit = (uint32_t)(v >> (jj & 31)) & 1u;
                    }
                    if (off == 0 && (jj == o || jj == t)) bit = 0;
                    const int dt_ = t - jj < 0 ? jj - t : t - jj;
                    const int do_ = o - jj < 0 ? jj - o : o - jj;
                    const Real kt_v = dt_ > a.cutoff ? (Real)0 : ktr[dt_];
                    const Real ko_v = do_ > a.cutoff ? (Real)0 : ktr[do_];
                    part += bit ? (kt_v - ko_v) : (Real)0;
                }
            }
            if (__any(!ok)) {
                if (lane == 0) sh.stop = 1;
                break;
            }
#pragma unroll
            for (int sh_ = 32; sh_ >= 1; sh_ >>= 1) part += __shfl_xor(part, sh_, 64);
            if (lane == 0) {
                const Real e_app = ((alpha_r * (Real)step_V[kstep % kStepWin]) * (Real)(t - o)) / (Real)L;
                const int srail = tile.r0 + srow;
                // the survivor's word and barrier again (rare: cheaper than
                // keeping them for every possible survivor)
                const uint4 blk = philox4x32_10((uint32_t)(s >> 3), (uint32_t)srail, (uint32_t)n,
                                                ((uint32_t)tile.d << 4) | (uint32_t)h, a.key0, a.key1);
                const Real ea = a.ea ? reinterpret_cast<const Real *>(a.ea)[dv.off + (int64_t)srail * L + o]
                                     : (Real)a.ea_scalar;
                if (decide_hop<Real>(e_app + part, ea, word_of(blk, (s >> 1) & 3), beta_r, c0_r, a.log, tile.d, h, n,
                                     srail, s)) {
                    record_hop(a.record, tile.d, h, n, srail, s, o == s ? 0 : 1);
                    atomicXor(reinterpret_cast<unsigned long long *>(&nxt[srow * W + (s >> 6)]), 1ull << (s & 63));
                    atomicXor(reinterpret_cast<unsigned long long *>(&nxt[srow * W + ((s + 1) >> 6)]),
                              1ull << ((s + 1) & 63));
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
        // Only a half-step with survivors (uniform) needs a second barrier: the
        // survivors read `cur` and flip bits of `nxt`.  Otherwise `nxt` is
        // already final (the copy below, made in the previous half-step, was
        // complete at this half-step's first barrier).
        if (n_surv > 0) lds_barrier();

        if (!isolated) publish(nxt, j + 1);
        if (h == 1 && tid == 0) {
            if (sh.n_down | sh.n_up) {
                const int64_t base = (n - a.ctl.tally_base) * a.n_devices + tile.d;
                atomicAdd(&a.tally_net[base], sh.n_down - sh.n_up);
                for (int q = 0; q < kDeciles; ++q)
                    if (sh.dec[q]) atomicAdd(&a.tally_dec[base * kDeciles + q], sh.dec[q]);
            }
            sh.n_down = 0;
            sh.n_up = 0;
            for (int q = 0; q < kDeciles; ++q) sh.dec[q] = 0;
        }
        // `cur` is read by no one any more: it becomes the next half-step's
        // output, starting as a copy of the new state.
        for (int i = tid; i < nr * W; i += bdim) const_cast<uint64_t *>(cur)[i] = nxt[i];
    }

    // write the tile back (an even number of half-steps ends in B0)
    __syncthreads();
    if (has_chunk) {
        const uint32_t bits = (uint32_t)(B0[wi] >> sb) & 0xFFFFu;
        const uint4 c = *reinterpret_cast<const uint4 *>(cls + row * P + s0);
        uint4 v;
        v.x = (((bits >> 0) & 0xFu) * 0x00204081u & 0x01010101u) | (c.x << 1);
        v.y = (((bits >> 4) & 0xFu) * 0x00204081u & 0x01010101u) | (c.y << 1);
        v.z = (((bits >> 8) & 0xFu) * 0x00204081u & 0x01010101u) | (c.z << 1);
        v.w = (((bits >> 12) & 0xFu) * 0x00204081u & 0x01010101u) | (c.w << 1);
        *reinterpret_cast<uint4 *>(gstate + (int64_t)row * P + s0) = v;
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
