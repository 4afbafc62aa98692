// HIP kernels of the rail-KMC hop step for gfx950 (MI355X): the half-step
// kernel (the general path for lattices that are not kept co-resident, and
// the score replay), the replay's per-bond Coulomb parts, and the
// set-up and bookkeeping kernels.  The persistent kernels are in
// kmc_persistent.hip and kmc_wave.hip.
//
// hop_half_step: one launch decides every bond of one parity
// (a half-step of the pair checkerboard) for every device, reading the state
// at the start of the half-step from one buffer and writing the new state to
// the other.  One workgroup owns whole rails of one device ("tile"), one lane
// owns 16 consecutive sites of a rail:
//   1. the lane issues the coalesced 16-byte load of its int8 chunk (and of a
//      chunk of the +-rail_range halo rails), then draws the two Philox4x32-10
//      blocks of its bonds while the loads are in flight; the tile and halo are
//      staged in LDS as the Jacobi snapshot;
//   2. candidate bonds (exactly one of the two sites occupied) are found with
//      bit operations on the 16 occupancy bits;
//   3. an exact prefilter discards every candidate whose Philox word lies above
//      a bound on its hop probability valid for any configuration (telescoping
//      bound on the Coulomb term, a lower bound of the origin's barrier stored
//      as a 7-bit class next to the occupancy bit, the step's bias); the few
//      survivors are queued in LDS;
//   4. survivors get the full energy change from the LDS window (bias drop plus
//      the screened Coulomb sum, paper main text section 3 and SI Eq. S1), the
//      Arrhenius probability with the half-energy barrier shift (main text Eq.
//      hop_rate and Eq. 2), the accept test u < p and the near-threshold log;
//   5. accepted hops are tallied (net hops toward the grounded site 0, decile
//      crossings), applied to the lanes' registers and the tile is written out.
//
// With kScore the same kernel replays a half-step for the score-function
// gradient: the decisions are taken exactly as above (so the replay follows the
// forward trajectory), and in addition every candidate bond gets its hop
// probability from the Coulomb part dE_coul = phi(t) - K(1, 0) - phi(o) of the
// half-step's state (kept per bond, summed in binary64 and rounded once to the
// path precision, recomputed by replay_ec_update where hops changed it) and
// contributes W g (y - p)/(1 - p) to
// the device's four accumulators, g being the log-derivative of p in (Ea shift,
// nu0, kappa, alpha).  The accepted hops go to a global list for the potential
// update.
#include <math.h>

#include <type_traits>

#include "kmc_device.h"
#include "kmc_internal.h"

namespace kmc {

struct HopShared {
    double score[kBlock / 64][4];  // score replay: per-wave partial sums
    double V;
    int32_t n_surv, n_hop, n_down, n_up, n_cand;
    int32_t dec[kDeciles];
    uint32_t wtab[kClasses];  // inclusive Philox-word thresholds per barrier class
};

// ------------------------------------------------------------------------
// The half-step kernel.  H = bond parity.  State bytes: bit 0 = occupied,
// bits 1..7 = barrier class of the site (a lower bound of its barrier used only
// by the prefilter).  One lane per 16-site chunk (a tile has at most kBlock
// chunks).  Dynamic LDS layout:
//   rows   [(nr + 2m) * pitch] bytes : tile rails and halo rails (snapshot)
//   surv   [cap] uint32 (row << 13 | s; bit 31 set once the hop is accepted)
//   ktab   [(m + 1) * (cutoff + 1)] Real, when small enough
// The survivors' Philox words and barriers are read again where they are
// needed (a rare path), which keeps the LDS per workgroup small.
// ------------------------------------------------------------------------
template <typename Real, int H, int kMode>
__global__ __launch_bounds__(kBlock) void hop_half_step(HopArgs a) {
    constexpr bool kScore = kMode == 1;  // score replay
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ HopShared sh;

    const Tile tile = a.tiles[tile_of_block(blockIdx.x, a.n_tiles)];
    const DevInfo &dv = a.devs[tile.d];
    const int R = dv.rails, L = dv.sites, pitch = dv.pitch;
    const int m = a.rail_range;
    const int p16 = pitch / kChunkSites;
    const int n_rows = tile.nr + 2 * m;
    const int n_chunks = tile.nr * p16;
    const int n_halo = 2 * m * p16;
    const int cap = tile.nr * pitch / 2;
    unsigned char *rows = smem;
    uint32_t *surv = reinterpret_cast<uint32_t *>(smem + n_rows * pitch);
    Real *kt_lds = reinterpret_cast<Real *>(surv + cap + (cap & 1));
    const int kt_stride = a.cutoff + 1;
    const int n_kt = (m + 1) * kt_stride;
    const bool kt_in_lds = n_kt <= kLdsTableMax;
    const Real *kt_glob = std::is_same<Real, double>::value ? reinterpret_cast<const Real *>(a.ktab64)
                                                            : reinterpret_cast<const Real *>(a.ktab32);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t n = kScore ? a.n_abs : a.ctl.n_base + a.step_in_chunk;
    const int8_t *src_dev = a.occ_in + dv.off_pad;

    // 1. issue the loads of the lane's chunk and of one halo chunk
    const bool has_chunk = tid < n_chunks;
    const int row = has_chunk ? tid / p16 : 0;
    const int s0 = (tid - row * p16) * kChunkSites;
    uint4 v = make_uint4(0, 0, 0, 0);
    uint32_t nxt = 0;
    if (has_chunk) {
        const int8_t *rp = src_dev + (int64_t)(tile.r0 + row) * pitch;
        v = *reinterpret_cast<const uint4 *>(rp + s0);
        if (H == 1 && s0 + kChunkSites < pitch) nxt = (uint32_t)(uint8_t)rp[s0 + kChunkSites];
    }
    auto halo_lds_row = [&](int i) { const int hr = i / p16; return hr < m ? hr : hr + tile.nr; };
    auto halo_src = [&](int i) {
        const int lr = halo_lds_row(i);
        int rail = tile.r0 - m + lr;
        rail = ((rail % R) + R) % R;
        return src_dev + (int64_t)rail * pitch + (i - (i / p16) * p16) * kChunkSites;
    };
    uint4 hv = make_uint4(0, 0, 0, 0);
    if (tid < n_halo) hv = *reinterpret_cast<const uint4 *>(halo_src(tid));

    // bias of this step and the prefilter thresholds per barrier class
    const double V = protocol_voltage(a.knot_t + tile.d * kMaxKnots, a.knot_v + tile.d * kMaxKnots, dv.n_knots,
                                      (double)(n - dv.n_set) * a.dt);
    for (int q = tid; q < kClasses; q += kBlock)
        sh.wtab[q] = class_threshold(a.c0, a.beta, a.alpha, V, L, dv.ea_min, dv.ea_step, dv.coul_bound, q);
    if (tid == 0) {
        sh.V = V;
        sh.n_surv = 0;
        sh.n_cand = 0;
        sh.n_hop = 0;
        sh.n_down = 0;
        sh.n_up = 0;
        for (int q = 0; q < kDeciles; ++q) sh.dec[q] = 0;
    }
    if (kt_in_lds)
        for (int i = tid; i < n_kt; i += kBlock) kt_lds[i] = kt_glob[i];

    // 2. the two Philox blocks of the chunk (independent of the state)
    const uint32_t ctr3 = ((uint32_t)tile.d << 4) | (uint32_t)H;
    const uint32_t rail = (uint32_t)(tile.r0 + row);
    const uint4 blkA = philox4x32_10((uint32_t)(s0 >> 3), rail, (uint32_t)n, ctr3, a.key0, a.key1);
    const uint4 blkB = philox4x32_10((uint32_t)(s0 >> 3) + 1u, rail, (uint32_t)n, ctr3, a.key0, a.key1);

    // stage the Jacobi snapshot in LDS
    if (has_chunk) *reinterpret_cast<uint4 *>(rows + (m + row) * pitch + s0) = v;
    if (tid < n_halo)
        *reinterpret_cast<uint4 *>(rows + halo_lds_row(tid) * pitch + (tid - (tid / p16) * p16) * kChunkSites) = hv;
    for (int i = tid + kBlock; i < n_halo; i += kBlock)
        *reinterpret_cast<uint4 *>(rows + halo_lds_row(i) * pitch + (i - (i / p16) * p16) * kChunkSites) =
            *reinterpret_cast<const uint4 *>(halo_src(i));
    __syncthreads();

    // 3. candidates and the exact two-stage prefilter
    uint32_t bits = 0, cand_all = 0;
    if (has_chunk) {
        bits = occ_bits(v) | ((nxt & 1u) << 16);
        uint32_t cand = (bits ^ (bits >> 1)) & (H ? 0xAAAAu : 0x5555u);
        const int last = L - 2 - s0;  // bond (s0+k, s0+k+1) exists iff k <= last
        if (last < 15) cand &= last < 0 ? 0u : ((2u << last) - 1u);
        cand_all = cand;
        const uint32_t thr0 = sh.wtab[0];  // the largest threshold (lowest class)
        // stage 0: the smallest candidate word (non-candidates forced to all
        // ones by their sign-extended bit) against the largest threshold
        const uint32_t nc = ~cand;
        auto masked = [&](uint32_t w, int bit) { return w | (uint32_t)__builtin_amdgcn_sbfe((int)nc, bit, 1); };
        const uint32_t mA = min(min(masked(blkA.x, H), masked(blkA.y, H + 2)),
                                min(masked(blkA.z, H + 4), masked(blkA.w, H + 6)));
        const uint32_t mB = min(min(masked(blkB.x, H + 8), masked(blkB.y, H + 10)),
                                min(masked(blkB.z, H + 12), masked(blkB.w, H + 14)));
        uint32_t sv = 0;
        if (min(mA, mB) <= thr0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int bit = H + 2 * j;
                if (((cand >> bit) & 1u) && word_of(blkA, j) <= thr0) sv |= 1u << bit;
                if (((cand >> (bit + 8)) & 1u) && word_of(blkB, j) <= thr0) sv |= 1u << (bit + 8);
            }
        }
        if (sv) {  // rare: compare with the threshold of the origin's class
            while (sv) {
                const int bit = __builtin_ctz(sv);
                sv &= sv - 1;
                const int ob = ((bits >> bit) & 1u) ? bit : bit + 1;   // origin byte in the chunk
                const uint32_t obyte = ob < kChunkSites ? (word_of(v, ob >> 2) >> (8 * (ob & 3))) & 0xFFu : nxt;
                const uint32_t w = word_of8(blkA, blkB, bit >> 1);
                if (w <= sh.wtab[obyte >> 1]) {
                    const int k = atomicAdd(&sh.n_surv, 1);
                    surv[k] = ((uint32_t)row << 13) | (uint32_t)(s0 + bit);
                }
            }
        }
    }
    __syncthreads();

    // 4. full evaluation of the survivors, one wavefront per survivor: every
    //    lane sums a strided subset of the window terms in a fixed order, a
    //    butterfly reduction combines the lanes (the same order on every run).
    const int n_surv = sh.n_surv;
    if (n_surv > 0) {
        const Real alpha_r = (Real)a.alpha, V_r = (Real)sh.V;
        const Real beta_r = (Real)a.beta, c0_r = (Real)a.c0;
        const Real *kt = kt_in_lds ? kt_lds : kt_glob;
        for (int i = wave; i < n_surv; i += kBlock / 64) {
            const int srow = (int)(surv[i] >> 13), s = (int)(surv[i] & 8191u);
            const unsigned char *rp = rows + (m + srow) * pitch;
            const int o = (rp[s] & 1) ? s : s + 1;
            const int t = (rp[s] & 1) ? s + 1 : s;
            int lo = s - a.cutoff, hi = s + 1 + a.cutoff;
            lo = lo < 0 ? 0 : lo;
            hi = hi > L - 1 ? L - 1 : hi;
            Real part = (Real)0;
            for (int k = 0; k < dv.n_nbr; ++k) {
                const int off = dv.nbr_off[k];
                const Real *ktr = kt + dv.nbr_dist[k] * kt_stride;
                const unsigned char *nrow = rows + (m + srow + off) * pitch;
                for (int j = lo + lane; j <= hi; j += 64) {
                    int occ = nrow[j] & 1;
                    if (off == 0 && (j == o || j == t)) occ = 0;
                    const int dt_ = t - j < 0 ? j - t : t - j;
                    const int do_ = o - j < 0 ? j - o : o - j;
                    const Real kt_v = dt_ > a.cutoff ? (Real)0 : ktr[dt_];
                    const Real ko_v = do_ > a.cutoff ? (Real)0 : ktr[do_];
                    part += occ ? (kt_v - ko_v) : (Real)0;
                }
            }
#pragma unroll
            for (int sh_ = 32; sh_ >= 1; sh_ >>= 1) part += __shfl_xor(part, sh_, 64);
            if (lane == 0) {
                const Real e_app = ((alpha_r * V_r) * (Real)(t - o)) / (Real)L;
                const Real dE = e_app + part;
                const int srail = tile.r0 + srow;
                // the survivor's word and its origin's barrier, read again
                const uint4 blk = philox4x32_10((uint32_t)(s >> 3), (uint32_t)srail, (uint32_t)n, ctr3, a.key0, a.key1);
                const uint32_t word = word_of(blk, (s >> 1) & 3);
                const Real ea = a.ea ? reinterpret_cast<const Real *>(a.ea)[dv.off + (int64_t)srail * L + o]
                                     : (Real)a.ea_scalar;
                const bool accept = decide_hop<Real>(dE, ea, word, beta_r, c0_r, a.log, tile.d, H, n, srail, s);
                if (accept) {
                    if (!kScore) record_hop(a.record, tile.d, H, n, srail, s, o == s ? 0 : 1);
                    atomicAdd(&sh.n_hop, 1);
                    surv[i] |= 1u << 31;
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
    }
    if (!kScore && tid == 0 && sh.n_hop > 0) {
        const int64_t k = n - a.ctl.tally_base;
        const int64_t base = k * a.n_devices + tile.d;
        atomicAdd(&a.tally_net[base], sh.n_down - sh.n_up);
        for (int q = 0; q < kDeciles; ++q)
            if (sh.dec[q]) atomicAdd(&a.tally_dec[base * kDeciles + q], sh.dec[q]);
    }

    // 5. apply the accepted hops that touch the lane's chunk, write it out
    uint32_t acc = 0;  // accepted bonds starting in the chunk
    if (has_chunk) {
        if (sh.n_hop > 0) {
            for (int k = 0; k < n_surv; ++k) {
                const uint32_t e = surv[k];
                if (!(e >> 31)) continue;
                const int hr = (int)((e >> 13) & 0x3FFFFu), hs = (int)(e & 8191u);
                if (hr != row) continue;
                if (hs >= s0 && hs < s0 + kChunkSites) {
                    flip_byte(v, hs - s0);
                    acc |= 1u << (hs - s0);
                }
                if (hs + 1 >= s0 && hs + 1 < s0 + kChunkSites) flip_byte(v, hs + 1 - s0);
            }
        }
        *reinterpret_cast<uint4 *>(a.occ_out + dv.off_pad + (int64_t)(tile.r0 + row) * pitch + s0) = v;
    }

    // 6. score replay: every candidate's term W g (y - p)/(1 - p), binary64.
    //    The candidates of the tile are listed in LDS (the survivor list is free
    //    now) and shared round-robin by all lanes.  The Coulomb part of dE,
    //    phi(t) - K(1, 0) - phi(o), is read from the per-bond values of the
    //    half-step's state (summed in binary64, rounded once to the path
    //    precision).  The half-step's accepted hops are appended to the global
    //    list (device, rail, site, direction) from which replay_ec_update
    //    recomputes the bonds they changed before the next half-step.
    if constexpr (kScore) {
        // the count of the previous half-step's list (the other parity) was
        // consumed by its update kernel: clear it for the next half-step
        if (blockIdx.x == 0 && tid == 0)
            __hip_atomic_store(a.hop_ctl + (1 - H), (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int i = tid; i < n_surv; i += kBlock) {
            const uint32_t e = surv[i];
            if (!(e >> 31)) continue;
            const int hr = (int)((e >> 13) & 0x3FFFFu), hs = (int)(e & 8191u);
            const uint32_t dir = (rows[(m + hr) * pitch + hs] & 1) ? 0u : 1u;  // 0: the ion at hs moves up
            const int64_t k = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(a.hop_ctl + H), 1ull);
            if (k < a.hop_cap) a.hops[k] = make_uint4((uint32_t)tile.d, (uint32_t)(tile.r0 + hr), (uint32_t)hs, dir);
        }
        __syncthreads();  // the survivor list becomes the candidate list
        uint32_t *clist = surv;
        {
            // slots of the lane's candidates: a prefix sum over the wavefront
            // and one LDS atomic per wavefront
            const int nc = has_chunk ? __builtin_popcount(cand_all) : 0;
            int pre = nc;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int t = __shfl_up(pre, d, 64);
                if (lane >= d) pre += t;
            }
            int base = 0;
            if (lane == 63) base = atomicAdd(&sh.n_cand, pre);
            int k = __shfl(base, 63, 64) + pre - nc;
            uint32_t cm = has_chunk ? cand_all : 0u;
            while (cm) {
                const int bit = __builtin_ctz(cm);
                cm &= cm - 1;
                const uint32_t dir = ((bits >> bit) & 1u) ? 0u : 1u;  // 0: ion at s moves up
                const uint32_t y = (acc >> bit) & 1u;
                clist[k++] = ((uint32_t)row << 14) | (y << 13) | (dir << 12) | (uint32_t)(s0 + bit);
            }
        }
        __syncthreads();
        const int n_cand = sh.n_cand;
        const Real alpha_r = (Real)a.alpha, V_r = (Real)sh.V;
        const Real beta_r = (Real)a.beta, c0_r = (Real)a.c0;
        const double W = a.score_w[tile.d];
        const double beta = a.beta, V = sh.V;
        // weights of the four log-derivatives, folded once per workgroup:
        // W g = W (-beta), W / nu0, W (-beta / (2 kappa)) dE_coul, W (-beta V / (2 L)) (t - o)
        const double w_ea = W * -beta, w_nu = W * (1.0 / a.nu0);
        const double w_k = W * (-0.5 * beta / a.kappa), w_a = W * (-0.5 * beta * V / (double)L);
        double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
        // four candidates per lane and pass: their loads are issued together
        constexpr int kBatch = 4;
        const Real *ec_of = reinterpret_cast<const Real *>(a.rec);
        const int64_t odd_at = (L + 1) / 2;  // start of the odd bonds in a rail's run
        for (int i0 = tid; i0 < n_cand; i0 += kBatch * kBlock) {
            Real ec_b[kBatch], ea_b[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int i = i0 + u * kBlock;
                ec_b[u] = (Real)0;
                ea_b[u] = (Real)a.ea_scalar;
                if (i < n_cand) {
                    const uint32_t e = clist[i];
                    const int crow = (int)(e >> 14), s = (int)(e & 4095u);
                    const int64_t rail_at = dv.off + (int64_t)(tile.r0 + crow) * L;
                    ec_b[u] = ec_of[rail_at + (H ? odd_at : 0) + (s >> 1)];
                    if (a.ea) {
                        const int o = ((e >> 12) & 1u) ? s + 1 : s;
                        ea_b[u] = reinterpret_cast<const Real *>(a.ea)[rail_at + o];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int i = i0 + u * kBlock;
                if (i >= n_cand) break;
                const uint32_t e = clist[i];
                const int s = (int)(e & 4095u);
                const int dir = (int)((e >> 12) & 1u);
                const uint32_t y = (e >> 13) & 1u;
                const int o = dir ? s + 1 : s, t = dir ? s : s + 1;
                const Real ec = ec_b[u];
                const Real e_app = ((alpha_r * V_r) * (Real)(t - o)) / (Real)L;
                const Real dE = e_app + ec;
                Real p = c0_r * exp_r<Real>(-beta_r * (ea_b[u] + (Real)0.5 * dE));
                p = p < (Real)1 ? p : (Real)1;
                if (p < (Real)1) {
                    const double pd = (double)p;
                    const double ratio = ((double)y - pd) / (1.0 - pd);
                    g0 += w_ea * ratio;
                    g1 += w_nu * ratio;
                    g2 += (w_k * (double)ec) * ratio;
                    g3 += (t > o ? w_a : -w_a) * ratio;
                }
            }
        }
#pragma unroll
        for (int sh_ = 32; sh_ >= 1; sh_ >>= 1) {
            g0 += __shfl_xor(g0, sh_, 64);
            g1 += __shfl_xor(g1, sh_, 64);
            g2 += __shfl_xor(g2, sh_, 64);
            g3 += __shfl_xor(g3, sh_, 64);
        }
        if (lane == 0) {
            sh.score[wave][0] = g0;
            sh.score[wave][1] = g1;
            sh.score[wave][2] = g2;
            sh.score[wave][3] = g3;
        }
        __syncthreads();
        if (tid < 4) {
            double sum = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) sum += sh.score[w][tid];
            if (sum != 0.0) atomicAdd(&a.score_grad[tile.d * 4 + tid], sum);
        }
    }
}

// ------------------------------------------------------------------------
// Bookkeeping kernels
// ------------------------------------------------------------------------

// Caller layout -> padded internal layout: bit 0 = occupied (any nonzero
// byte), bits 1..7 = barrier class floor((Ea - ea_min)/ea_step) clamped to
// [0, 127] (0 without a barrier field); padding bytes cleared.
// The device holding element i of the padded (or unpadded) layout: the last
// device whose offset is <= i (offsets ascend), by bisection.
__device__ __forceinline__ int device_of(const DevInfo *devs, int n_dev, int64_t i, bool padded) {
    int lo = 0, hi = n_dev - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t at = padded ? devs[mid].off_pad : devs[mid].off;
        if (at <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Internal state from the caller's occupancy and per-site barriers: 16 padded
// bytes per thread, always inside one rail (pitch and device offsets are
// multiples of 16), written with one 16-byte store.
template <typename Real>
__global__ __launch_bounds__(256) void import_occupancy(const int8_t *src, int8_t *dst, const DevInfo *devs,
                                                        int n_dev, int64_t total_pad, const Real *ea) {
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16;
    if (i0 >= total_pad) return;
    const int d = device_of(devs, n_dev, i0, true);
    const DevInfo &dv = devs[d];
    const int64_t loc = i0 - dv.off_pad;
    const int r = (int)(loc / dv.pitch), s0 = (int)(loc - (int64_t)r * dv.pitch);
    const int64_t at = dv.off + (int64_t)r * dv.sites + s0;
    const bool classes = ea && dv.ea_step > 0.0;
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (s0 + k < dv.sites) {
            int cls = 0;
            if (classes) {
                const double q = floor(((double)ea[at + k] - dv.ea_min) / dv.ea_step);
                cls = q < 0.0 ? 0 : (q > (double)(kClasses - 1) ? kClasses - 1 : (int)q);
            }
            w[k >> 2] |= (uint32_t)((cls << 1) | (src[at + k] != 0 ? 1 : 0)) << (8 * (k & 3));
        }
    }
    *reinterpret_cast<uint4 *>(dst + i0) = make_uint4(w[0], w[1], w[2], w[3]);
}

// Occupancy bits in the caller's unpadded layout: 16 consecutive output bytes
// per thread (one 16-byte store when dst allows it), walking rails and devices
// from the first byte's position (every device has >= 1 rail of >= 2 sites).
__global__ __launch_bounds__(256) void export_occupancy(const int8_t *src, int8_t *dst, const DevInfo *devs,
                                                        int n_dev, int64_t total) {
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16;
    if (i0 >= total) return;
    int d = device_of(devs, n_dev, i0, false);
    int L = devs[d].sites, R = devs[d].rails, pitch = devs[d].pitch;
    int64_t base = devs[d].off_pad;
    const int64_t loc = i0 - devs[d].off;
    int r = (int)(loc / L), s = (int)(loc - (int64_t)r * L);
    const int n = (int)min((int64_t)16, total - i0);
    uint64_t lo = 0, hi = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k < n) {
            if (s == L) {  // next rail, or the next device's first rail
                s = 0;
                if (++r == R) {
                    ++d;
                    L = devs[d].sites, R = devs[d].rails, pitch = devs[d].pitch;
                    base = devs[d].off_pad;
                    r = 0;
                }
            }
            const uint64_t b = (uint64_t)(src[base + (int64_t)r * pitch + s] & 1);
            if (k < 8) lo |= b << (8 * k);
            else hi |= b << (8 * (k - 8));
            ++s;
        }
    }
    if (n == 16 && ((uintptr_t)dst & 15u) == 0) {
        *reinterpret_cast<uint4 *>(dst + i0) =
            make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
    } else {
        for (int k = 0; k < n; ++k) dst[i0 + k] = (int8_t)((k < 8 ? lo >> (8 * k) : hi >> (8 * (k - 8))) & 1u);
    }
}

// Random placement: floor(f L + 1/2) ions on the sites with the smallest
// (placement word, site) keys.  One workgroup per rail; rank by counting.
__global__ __launch_bounds__(256) void place_ions(int8_t *occ_pad, const DevInfo *devs,
                                                  const int32_t *rail_dev, const int32_t *rail_idx,
                                                  const int32_t *n_ions, uint32_t key0, uint32_t key1) {
    __shared__ uint64_t keys[kMaxSites];
    const int d = rail_dev[blockIdx.x], r = rail_idx[blockIdx.x];
    const DevInfo &dv = devs[d];
    const int L = dv.sites;
    const int nion = n_ions[d];
    for (int s = threadIdx.x; s < L; s += blockDim.x) {
        const uint4 blk = philox4x32_10((uint32_t)(s >> 2), (uint32_t)r, 0u,
                                        ((uint32_t)d << 4) | (1u << 1), key0, key1);
        keys[s] = ((uint64_t)word_of(blk, s & 3) << 32) | (uint32_t)s;
    }
    __syncthreads();
    int8_t *row = occ_pad + dv.off_pad + (int64_t)r * dv.pitch;
    for (int s = threadIdx.x; s < L; s += blockDim.x) {
        const uint64_t ks = keys[s];
        int rank = 0;
        for (int q = 0; q < L; ++q) rank += keys[q] < ks ? 1 : 0;
        row[s] = (int8_t)((row[s] & ~1) | (rank < nion ? 1 : 0));
    }
}

// Order-preserving unsigned key of a double (for atomicMin).
__device__ __forceinline__ unsigned long long order_key(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

template <typename Real>
__global__ void barrier_range(const Real *ea, const DevInfo *devs, unsigned long long *kmin,
                              unsigned long long *kmax) {
    const int d = blockIdx.y;
    const DevInfo &dv = devs[d];
    const int64_t cnt = (int64_t)dv.rails * dv.sites;
    unsigned long long lo = ~0ull, hi = 0ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
         i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long k = order_key((double)ea[dv.off + i]);
        lo = k < lo ? k : lo;
        hi = k > hi ? k : hi;
    }
    atomicMin(&kmin[d], lo);
    atomicMax(&kmax[d], hi);
}

__device__ __forceinline__ double key_value(unsigned long long k) {
    const unsigned long long b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    return __longlong_as_double((long long)b);
}

// ea_min and the class width ea_step = (ea_max - ea_min)/127 of every device.
__global__ void barrier_range_finish(const unsigned long long *kmin, const unsigned long long *kmax,
                                     DevInfo *devs, int n_dev) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n_dev) return;
    const double lo = key_value(kmin[d]), hi = key_value(kmax[d]);
    devs[d].ea_min = lo;
    devs[d].ea_step = hi > lo ? (hi - lo) / (double)(kClasses - 1) : 0.0;
}

// Decile counts of the current state (int64), one workgroup per device.
// Occupied sites per decile of every device, from the padded state; dec_run
// must be zero on entry.  Grid (devices, kDecileBlocks): each thread takes
// 16-site chunks; a chunk touches few deciles, each counted with one popcount.
constexpr int kDecileBlocks = 64;

__global__ __launch_bounds__(256) void count_deciles(const int8_t *occ_pad, const DevInfo *devs,
                                                     unsigned long long *dec_run) {
    __shared__ int cnt[kDeciles];
    const int d = blockIdx.x;
    const DevInfo &dv = devs[d];
    if (threadIdx.x < kDeciles) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int L = dv.sites, cpr = dv.pitch / 16;
    const int64_t chunks = (int64_t)dv.rails * cpr;
    const uint4 *src = reinterpret_cast<const uint4 *>(occ_pad + dv.off_pad);
    for (int64_t c = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; c < chunks;
         c += (int64_t)gridDim.y * blockDim.x) {
        const int s0 = (int)(c % cpr) * 16;
        if (s0 >= L) continue;
        const uint4 v = src[c];
        uint32_t mask = 0;  // bit j: site s0 + j occupied
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) mask |= (((w[k] & 0x01010101u) * 0x01020408u) >> 24 & 0xFu) << (4 * k);
        if (L - s0 < 16) mask &= (1u << (L - s0)) - 1u;
        if (!mask) continue;
        const int s_end = min(s0 + 16, L);
        for (int q = (10 * s0) / L; q <= (10 * (s_end - 1)) / L; ++q) {
            const int lo = max((q * L + 9) / 10, s0), hi = min(((q + 1) * L + 9) / 10, s_end);
            const uint32_t range = ((hi - s0 >= 32 ? 0u : (1u << (hi - s0))) - 1u) & ~((1u << (lo - s0)) - 1u);
            const int n = __popc(mask & range);
            if (n) atomicAdd(&cnt[q], n);
        }
    }
    __syncthreads();
    if (threadIdx.x < kDeciles && cnt[threadIdx.x])
        atomicAdd(&dec_run[d * kDeciles + threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
}

// Install a protocol: knots are passed by value so the update is ordered on the
// stream like every other launch.
struct KnotPack {
    double t[kMaxKnots];
    double v[kMaxKnots];
};

__global__ void set_protocol(double *knot_t, double *knot_v, DevInfo *devs, int d0, int d1,
                             int nk, int64_t n_set, KnotPack kp) {
    const int d = d0 + blockIdx.x;
    if (d >= d1) return;
    for (int i = threadIdx.x; i < kMaxKnots; i += blockDim.x) {
        knot_t[d * kMaxKnots + i] = i < nk ? kp.t[i] : 0.0;
        knot_v[d * kMaxKnots + i] = i < nk ? kp.v[i] : 0.0;
    }
    if (threadIdx.x == 0) {
        devs[d].n_knots = nk;
        devs[d].n_set = n_set;
    }
}

// End of a tally chunk of `steps` steps: per device, prefix-sum the decile
// deltas into absolute counts, accumulate the int64 net total, copy rows to the
// caller's buffers and clear the chunk buffers.  One workgroup per series
// (device, decile or net hops), one thread per step.
static_assert(kTallySteps <= 1024, "finish_chunk scans a chunk in one workgroup");
__global__ __launch_bounds__(1024) void finish_chunk(FinishArgs f) {
    __shared__ int64_t wsum[1024 / 64];
    const int d = f.d0 + blockIdx.x, q = blockIdx.y;  // q == kDeciles: net hops
    const int k = threadIdx.x, lane = k & 63, wave = k >> 6;
    const int n_dev = f.n_devices, steps = f.steps;
    const int64_t row0 = f.ctl.tally_base - f.ctl.call_base;
    int32_t *net_out = f.ctl.net_out;
    int32_t *dec_out = f.ctl.dec_out;
    const int64_t carry = q < kDeciles ? f.dec_run[d * kDeciles + q] : 0;  // read before the barrier
    int64_t x = 0;
    if (k < steps) {
        int32_t *p = q < kDeciles ? &f.tally_dec[((int64_t)k * n_dev + d) * kDeciles + q]
                                  : &f.tally_net[(int64_t)k * n_dev + d];
        x = *p;
        *p = 0;
        if (q == kDeciles && net_out) net_out[(row0 + k) * n_dev + d] = (int32_t)x;
    }
    // inclusive scan: within the wavefront, then over the wavefront totals
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)x, off, 64);
        const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)((uint64_t)x >> 32), off, 64);
        if (lane >= off) x += (int64_t)(((uint64_t)hi << 32) | lo);
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int64_t before = 0, total = 0;
    for (int w = 0; w < 1024 / 64; ++w) {
        if (w < wave) before += wsum[w];
        total += wsum[w];
    }
    if (k < steps && q < kDeciles && dec_out) dec_out[((row0 + k) * n_dev + d) * kDeciles + q] = (int32_t)(carry + before + x);
    if (k == 0) {
        if (q < kDeciles) f.dec_run[d * kDeciles + q] = carry + total;
        else f.net_total[d] += total;
    }
}

__global__ void zero_i32(int32_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void zero_i64(int64_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Plain streaming copy (16 bytes per lane per iteration), for counter calibration.
__global__ void copy_bytes(const uint4 *src, uint4 *dst, int64_t n16) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// ------------------------------------------------------------------------
// Host-side launch wrappers (called from kmc_api.cpp)
// ------------------------------------------------------------------------
static inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// ------------------------------------------------------------------------
// Coulomb part of the energy change of every candidate bond, for the score
// replay (main text section 3: the field of the ions; SI Eq. S1 takes its
// difference between target and origin).  With phi(r, s) the sum over the
// distinct neighbour rails r + off (offsets and minimal-image distances of
// the device, off = 0 included) and the sites j with |s - j| <= cutoff of
// occ(r + off, j) K(|s - j|, dist), the site itself excluded, a candidate bond
// (s, s+1) with its ion at o and the empty site t has
//     ec = phi(t) - K(1, 0) - phi(o) = +-(phi(s + 1) - phi(s)) - K(1, 0).
// It is summed in binary64 in one pass over the bond's window and rounded once
// to the path precision; a bond that is not a candidate holds 0.  The values
// are kept for every bond, split by bond parity so that a half-step reads one
// contiguous run per rail, and recomputed from the new state for every bond
// whose window an accepted hop changed.
// ------------------------------------------------------------------------
__device__ __forceinline__ int64_t bond_index(const DevInfo &dv, int r, int s) {
    return dv.off + (int64_t)r * dv.sites + ((s & 1) ? (dv.sites + 1) / 2 : 0) + (s >> 1);
}

// Occupancy of site j of rail r of the state a.occ (a byte or a bit per site).
__device__ __forceinline__ int occ_site(const PhiArgs &a, const DevInfo &dv, int r, int j) {
    const int64_t at = dv.off_pad + (int64_t)r * dv.pitch + j;
    return a.occ_bits ? (reinterpret_cast<const uint8_t *>(a.occ)[at >> 3] >> (at & 7)) & 1 : a.occ[at] & 1;
}

template <typename Real>
__device__ Real replay_bond_ec(const PhiArgs &a, const DevInfo &dv, int r, int s) {
    const int R = dv.rails, L = dv.sites, cut = a.cutoff;
    const int up = occ_site(a, dv, r, s);
    if (up == occ_site(a, dv, r, s + 1)) return (Real)0;
    const int lo = s - cut < 0 ? 0 : s - cut, hi = s + 1 + cut > L - 1 ? L - 1 : s + 1 + cut;
    double acc = 0.0;  // phi(s + 1) - phi(s)
    for (int k = 0; k < dv.n_nbr; ++k) {
        const int off = dv.nbr_off[k];
        int rr = (r + off) % R;
        rr = rr < 0 ? rr + R : rr;
        const double *kr = a.ktab64 + dv.nbr_dist[k] * (cut + 1);
        for (int j = lo; j <= hi; ++j) {
            if (!occ_site(a, dv, rr, j)) continue;
            const int dt = j < s + 1 ? s + 1 - j : j - s - 1, dO = j < s ? s - j : j - s;
            const double kt = (dt > cut || (off == 0 && j == s + 1)) ? 0.0 : kr[dt];
            const double ko = (dO > cut || (off == 0 && j == s)) ? 0.0 : kr[dO];
            acc += kt - ko;
        }
    }
    return (Real)((up ? acc : -acc) - a.k01);
}

// every bond of every device from the state a.occ
template <typename Real>
__device__ void replay_ec_all(const PhiArgs &a) {
    Real *ec = reinterpret_cast<Real *>(a.ec);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t first = 0;  // bonds of the earlier devices: every device's bonds form one sequence
    for (int d = 0; d < a.n_devices; ++d) {
        const DevInfo &dv = a.devs[d];
        const int nb = dv.sites - 1;
        const int64_t n = (int64_t)dv.rails * nb;
        const int64_t i0 = ((t - first) % stride + stride) % stride;
        first += n;
        for (int64_t i = i0; i < n; i += stride) {
            const int r = (int)(i / nb), s = (int)(i - (int64_t)r * nb);
            ec[bond_index(dv, r, s)] = replay_bond_ec<Real>(a, dv, r, s);
        }
    }
}

// acc + sum over x < n of w[x] dr[x] (w in LDS, 0 or 1; dr the LDS table),
// accumulated in order by binary64 fma; the loads of eight terms are issued
// before their fmas so that their latencies overlap.
__device__ __forceinline__ double window_dot(const uint8_t *w, const double *dr, int n, double acc) {
    int x = 0;
    for (; x + 8 <= n; x += 8) {
        uint32_t b[8];
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            b[u] = w[x + u];
            t[u] = dr[x + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fma((double)b[u], t[u], acc);
    }
    for (; x < n; ++x) acc = fma((double)w[x], dr[x], acc);
    return acc;
}

// The starting values, one workgroup per run of up to 256 bonds of one rail:
// the occupancy of the run's window on every neighbour rail is staged in LDS
// (zero outside the rail), and each lane sums its bond's terms in one pass,
// occ(j) D(dist, j - s + cut) with D the table of K(|s + 1 - j|, dist) -
// K(|s - j|, dist) (the distance-0 row, the bond's own rail, without the self
// terms).  Windows wider than kEcMaxCut fall back to replay_ec_all.
constexpr int kEcRun = 256;
constexpr int kEcMaxCut = 512;

template <typename Real>
__global__ __launch_bounds__(kEcRun) void replay_ec_full(PhiArgs a) {
    const int cut = a.cutoff;
    if (cut > kEcMaxCut) {
        replay_ec_all<Real>(a);
        return;
    }
    Real *ec = reinterpret_cast<Real *>(a.ec);
    // dynamic LDS sized to the window (ec_full_lds): the rows of the run's
    // window on every neighbour rail, then the table of kernel differences
    extern __shared__ __align__(16) unsigned char ec_smem[];
    const int wn = 2 * cut + 2;               // window of a bond: sites s - cut .. s + 1 + cut
    const int width = kEcRun + 2 * cut + 2;   // window of the run: sites b0 - cut .. b0 + kEcRun + cut + 1
    uint8_t *win = ec_smem;                   // row k at k * width
    double *dtab = reinterpret_cast<double *>(ec_smem + ((size_t)(2 * a.rail_range + 1) * width + 15) / 16 * 16);
    for (int i = threadIdx.x; i < (a.rail_range + 1) * wn; i += kEcRun) {
        const int dist = i / wn, x = i - dist * wn;
        const int dt = x - cut - 1 < 0 ? cut + 1 - x : x - cut - 1, dO = x - cut < 0 ? cut - x : x - cut;
        const double *kr = a.ktab64 + dist * (cut + 1);
        const double kt = (dt > cut || (dist == 0 && dt == 0)) ? 0.0 : kr[dt];
        const double ko = (dO > cut || (dist == 0 && dO == 0)) ? 0.0 : kr[dO];
        dtab[i] = kt - ko;
    }
    // the units of every device in one sequence (device by device), dealt to
    // the workgroups in turn, so that no workgroup waits on a small device
    int64_t first = 0;  // the sequence index of the device's first unit
    for (int d = 0; d < a.n_devices; ++d) {
        const DevInfo &dv = a.devs[d];
        const int R = dv.rails, L = dv.sites, nb = L - 1;
        const int runs = (nb + kEcRun - 1) / kEcRun;
        const int64_t units = (int64_t)R * runs;
        int k_own = 0;  // the entry of offset 0 (the bond's own rail)
        for (int k = 0; k < dv.n_nbr; ++k)
            if (dv.nbr_off[k] == 0) k_own = k;
        const int64_t g = gridDim.x;
        const int64_t u0 = (((int64_t)blockIdx.x - first) % g + g) % g;  // this workgroup's first unit here
        first += units;
        for (int64_t u = u0; u < units; u += g) {
            const int r = (int)(u / runs), b0 = (int)(u - (int64_t)r * runs) * kEcRun;
            __syncthreads();  // the table is written; the previous unit's window is no longer read
            for (int k = 0; k < dv.n_nbr; ++k) {
                int rr = (r + dv.nbr_off[k]) % R;
                rr = rr < 0 ? rr + R : rr;
                const int8_t *row = a.occ + dv.off_pad + (int64_t)rr * dv.pitch;
                for (int x = threadIdx.x; x < width; x += kEcRun) {
                    const int j = b0 - cut + x;
                    win[k * width + x] = (j >= 0 && j < L) ? (uint8_t)(row[j] & 1) : (uint8_t)0;
                }
            }
            __syncthreads();
            const int s = b0 + (int)threadIdx.x;
            if (s < nb) {
                const uint8_t *w_own = win + k_own * width + (int)threadIdx.x;  // w[x] is site s - cut + x
                const int up = w_own[cut];
                Real v = (Real)0;
                if (up != w_own[cut + 1]) {
                    double acc = 0.0;
                    for (int k = 0; k < dv.n_nbr; ++k) {
                        const double *dr = dtab + dv.nbr_dist[k] * wn;
                        const uint8_t *w = win + k * width + (int)threadIdx.x;
                        acc = window_dot(w, dr, wn, acc);
                    }
                    v = (Real)((up ? acc : -acc) - a.k01);
                }
                ec[bond_index(dv, r, s)] = v;
            }
        }
    }
}

// Recomputes, from the new state a.occ, every bond whose window the
// half-step's accepted hops changed: for a hop (device, rail r, s, dir; it
// moved the ion between s and s + 1) the bonds j = s - cutoff - 1 .. s + 1 +
// cutoff of each neighbour rail r + off.  One workgroup per hop stages the
// occupancy those bonds' windows read (sites s - 2 cutoff - 1 .. s + 2 cutoff
// + 2 of the rails r - 2m .. r + 2m) in LDS and sums each bond with the table
// of kernel differences, as replay_ec_full does.  Bonds reached from several
// hops are written with the same value.  A list that overflowed (count >
// capacity) is replaced by a recomputation of every bond.  The count is
// cleared by the replay kernel of the next half-step (which appends to the
// other parity's count).
constexpr int kEcUpdMaxCut = 128;

template <typename Real>
__global__ __launch_bounds__(256) void replay_ec_update(PhiArgs a) {
    const int64_t cnt = a.known_count >= 0 ? a.known_count
                                           : __hip_atomic_load(a.hop_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cnt > a.hop_cap) {
        replay_ec_all<Real>(a);
        return;
    }
    Real *ec = reinterpret_cast<Real *>(a.ec);
    const int cut = a.cutoff, m = a.rail_range, w = 2 * cut + 3;  // bonds per rail whose window holds s or s + 1
    if (blockIdx.x >= cnt) return;  // no hop for this workgroup
    if (cut > kEcUpdMaxCut) {  // wide windows: every bond summed from global memory
        for (int64_t i = blockIdx.x; i < cnt; i += gridDim.x) {
            const uint4 e = a.hops[i];
            const int d = (int)e.x, r = (int)e.y, s = (int)e.z;
            const DevInfo &dv = a.devs[d];
            const int R = dv.rails, L = dv.sites;
            for (int q = threadIdx.x; q < dv.n_nbr * w; q += blockDim.x) {
                const int k = q / w, j = s - cut - 1 + (q - k * w);
                if (j < 0 || j > L - 2) continue;
                int rr = (r + dv.nbr_off[k]) % R;
                rr = rr < 0 ? rr + R : rr;
                ec[bond_index(dv, rr, j)] = replay_bond_ec<Real>(a, dv, rr, j);
            }
        }
        return;
    }
    __shared__ uint8_t win[4 * kMaxRailRange + 1][4 * kEcUpdMaxCut + 4];  // row 2m + o: rail r + o
    __shared__ double dtab[(kMaxRailRange + 1) * (2 * kEcUpdMaxCut + 2)];
    const int wn = 2 * cut + 2;     // window of a bond
    const int width = 4 * cut + 4;  // sites s - 2 cut - 1 .. s + 2 cut + 2
    const int n_rows = 4 * m + 1;
    uint4 e_next = a.hops[blockIdx.x];  // the first hop, loaded while the table is built
    for (int i = threadIdx.x; i < (m + 1) * wn; i += blockDim.x) {
        const int dist = i / wn, x = i - dist * wn;
        const int dt = x - cut - 1 < 0 ? cut + 1 - x : x - cut - 1, dO = x - cut < 0 ? cut - x : x - cut;
        const double *kr = a.ktab64 + dist * (cut + 1);
        const double kt = (dt > cut || (dist == 0 && dt == 0)) ? 0.0 : kr[dt];
        const double ko = (dO > cut || (dist == 0 && dO == 0)) ? 0.0 : kr[dO];
        dtab[i] = kt - ko;
    }
    for (int64_t i = blockIdx.x; i < cnt; i += gridDim.x) {
        const uint4 e = e_next;
        if (i + gridDim.x < cnt) e_next = a.hops[i + gridDim.x];
        const int d = (int)e.x, r = (int)e.y, s = (int)e.z;
        const DevInfo &dv = a.devs[d];
        const int R = dv.rails, L = dv.sites;
        const int base = s - 2 * cut - 1;  // site of column 0
        __syncthreads();  // the table is written; the previous hop's window is no longer read
        for (int q = threadIdx.x; q < n_rows * width; q += blockDim.x) {
            const int row = q / width, x = q - row * width, j = base + x;
            int rr = (r + row - 2 * m) % R;
            rr = rr < 0 ? rr + R : rr;
            win[row][x] = (j >= 0 && j < L) ? (uint8_t)occ_site(a, dv, rr, j) : (uint8_t)0;
        }
        __syncthreads();
        // a pair of adjacent lanes per bond, each summing half of every
        // neighbour rail's window (the first half sites j - cut .. j - cut +
        // wn/2 - 1, the second the rest), added once at the end
        const int wh = wn / 2;
        for (int q = threadIdx.x; q < 2 * dv.n_nbr * w; q += blockDim.x) {
            const int hf = q & 1, qb = q >> 1;
            const int kb = qb / w, j = s - cut - 1 + (qb - kb * w);  // bond j on rail r + off(kb)
            const bool inside = j >= 0 && j <= L - 2;
            const int o1 = dv.nbr_off[kb];
            const int col = j - cut - base;  // column of site j - cut
            int up = 0;
            bool cand = false;
            double acc = 0.0;
            if (inside) {
                const uint8_t *w_own = win[2 * m + o1] + col;  // w[x] is site j - cut + x of the bond's rail
                up = w_own[cut];
                cand = up != w_own[cut + 1];
                if (cand) {
                    const int x0 = hf ? wh : 0, nx = hf ? wn - wh : wh;
                    for (int k = 0; k < dv.n_nbr; ++k) {
                        const double *dr = dtab + dv.nbr_dist[k] * wn + x0;
                        const uint8_t *wk = win[2 * m + o1 + dv.nbr_off[k]] + col + x0;
                        acc = window_dot(wk, dr, nx, acc);
                    }
                }
            }
            const double sum = acc + __shfl_xor(acc, 1, 64);  // both lanes of a pair are here
            if (inside && hf == 0) {
                int rr = (r + o1) % R;
                rr = rr < 0 ? rr + R : rr;
                ec[bond_index(dv, rr, j)] = cand ? (Real)((up ? sum : -sum) - a.k01) : (Real)0;
            }
        }
    }
}

template <int kMode>
static hipError_t launch_half_step(const HopArgs &a, size_t lds_bytes, bool fp64, hipStream_t st) {
    const dim3 grid(a.n_tiles), block(kBlock);
    if (fp64) {
        if (a.h == 0) hipLaunchKernelGGL((hop_half_step<double, 0, kMode>), grid, block, lds_bytes, st, a);
        else hipLaunchKernelGGL((hop_half_step<double, 1, kMode>), grid, block, lds_bytes, st, a);
    } else {
        if (a.h == 0) hipLaunchKernelGGL((hop_half_step<float, 0, kMode>), grid, block, lds_bytes, st, a);
        else hipLaunchKernelGGL((hop_half_step<float, 1, kMode>), grid, block, lds_bytes, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_hop(const HopArgs &a, size_t lds_bytes, bool fp64, hipStream_t st) {
    return launch_half_step<0>(a, lds_bytes, fp64, st);
}

hipError_t launch_score(const HopArgs &a, size_t lds_bytes, bool fp64, hipStream_t st) {
    return launch_half_step<1>(a, lds_bytes, fp64, st);
}

hipError_t set_hop_lds_limit(size_t lds_bytes, size_t score_lds_bytes) {
    const void *fns[8] = {(const void *)hop_half_step<double, 0, 0>, (const void *)hop_half_step<double, 1, 0>,
                          (const void *)hop_half_step<float, 0, 0>,  (const void *)hop_half_step<float, 1, 0>,
                          (const void *)hop_half_step<double, 0, 1>, (const void *)hop_half_step<double, 1, 1>,
                          (const void *)hop_half_step<float, 0, 1>,  (const void *)hop_half_step<float, 1, 1>};
    for (int i = 0; i < 8; ++i) {
        const int bytes = (int)(i < 4 ? lds_bytes : score_lds_bytes);
        hipError_t e = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_import(const int8_t *src, int8_t *dst, const DevInfo *devs, int n_dev, int64_t total_pad,
                         const void *ea, bool fp64, hipStream_t st) {
    const dim3 grid(grid_for(total_pad / 16, 256)), block(256);  // total_pad is a multiple of 16
    if (fp64) hipLaunchKernelGGL((import_occupancy<double>), grid, block, 0, st, src, dst, devs, n_dev, total_pad,
                                 (const double *)ea);
    else hipLaunchKernelGGL((import_occupancy<float>), grid, block, 0, st, src, dst, devs, n_dev, total_pad,
                            (const float *)ea);
    return hipGetLastError();
}

hipError_t launch_export(const int8_t *src, int8_t *dst, const DevInfo *devs, int n_dev, int64_t total,
                         hipStream_t st) {
    hipLaunchKernelGGL(export_occupancy, dim3(grid_for((total + 15) / 16, 256)), dim3(256), 0, st, src, dst, devs,
                       n_dev, total);
    return hipGetLastError();
}

hipError_t launch_place(int8_t *occ_pad, const DevInfo *devs, const int32_t *rail_dev, const int32_t *rail_idx,
                        const int32_t *n_ions, int n_rails_total, uint32_t key0, uint32_t key1, hipStream_t st) {
    hipLaunchKernelGGL(place_ions, dim3(n_rails_total), dim3(256), 0, st, occ_pad, devs, rail_dev, rail_idx,
                       n_ions, key0, key1);
    return hipGetLastError();
}

hipError_t launch_barrier_range(const void *ea, bool fp64, DevInfo *devs, int n_dev,
                                unsigned long long *scratch, hipStream_t st) {
    unsigned long long *kmin = scratch, *kmax = scratch + n_dev;
    hipLaunchKernelGGL(fill_u64, dim3(grid_for(n_dev, 256)), dim3(256), 0, st, kmin, (int64_t)n_dev, ~0ull);
    hipLaunchKernelGGL(fill_u64, dim3(grid_for(n_dev, 256)), dim3(256), 0, st, kmax, (int64_t)n_dev, 0ull);
    const dim3 grid(64, n_dev);
    if (fp64) hipLaunchKernelGGL((barrier_range<double>), grid, dim3(256), 0, st, (const double *)ea, devs, kmin, kmax);
    else hipLaunchKernelGGL((barrier_range<float>), grid, dim3(256), 0, st, (const float *)ea, devs, kmin, kmax);
    hipLaunchKernelGGL(barrier_range_finish, dim3(grid_for(n_dev, 256)), dim3(256), 0, st, kmin, kmax, devs, n_dev);
    return hipGetLastError();
}

hipError_t launch_count_deciles(const int8_t *occ_pad, const DevInfo *devs, int n_dev, int64_t *dec_run,
                                hipStream_t st) {
    const int64_t n = (int64_t)n_dev * kDeciles;
    hipLaunchKernelGGL(zero_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dec_run, n);
    hipLaunchKernelGGL(count_deciles, dim3(n_dev, kDecileBlocks), dim3(256), 0, st, occ_pad, devs,
                       reinterpret_cast<unsigned long long *>(dec_run));
    return hipGetLastError();
}

hipError_t launch_set_protocol(double *knot_t, double *knot_v, DevInfo *devs, int d0, int d1, int nk,
                               int64_t n_set, const double *t, const double *v, hipStream_t st) {
    KnotPack kp;
    for (int i = 0; i < kMaxKnots; ++i) {
        kp.t[i] = i < nk ? t[i] : 0.0;
        kp.v[i] = i < nk ? v[i] : 0.0;
    }
    hipLaunchKernelGGL(set_protocol, dim3(d1 - d0), dim3(64), 0, st, knot_t, knot_v, devs, d0, d1, nk, n_set, kp);
    return hipGetLastError();
}

hipError_t launch_finish_chunk(const FinishArgs &f, hipStream_t st) {
    // one workgroup per series (device, decile or net hops), one thread per step
    if (f.steps < 1 || f.steps > 1024 || f.d1 <= f.d0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(finish_chunk, dim3(f.d1 - f.d0, kDeciles + 1), dim3(1024), 0, st, f);
    return hipGetLastError();
}

hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_i32, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_copy_bytes(const void *src, void *dst, size_t bytes, hipStream_t st) {
    const int64_t n16 = (int64_t)(bytes / 16);
    hipLaunchKernelGGL(copy_bytes, dim3(2048), dim3(256), 0, st, (const uint4 *)src, (uint4 *)dst, n16);
    return hipGetLastError();
}

constexpr int kEcGrid = 2048;  // workgroups of the replay's Coulomb-part kernels

hipError_t launch_replay_ec_full(const PhiArgs &a, bool fp64, hipStream_t st) {
    if (a.occ_bits) return hipErrorInvalidValue;  // the start-up reads a byte per site
    // LDS of the window rows and the difference table (none beyond kEcMaxCut,
    // where every bond is summed from global memory)
    const int cut = a.cutoff;
    const size_t lds = cut > kEcMaxCut ? 0
                                       : ((size_t)(2 * a.rail_range + 1) * (kEcRun + 2 * cut + 2) + 15) / 16 * 16 +
                                             sizeof(double) * (size_t)(a.rail_range + 1) * (2 * cut + 2);
    if (fp64) hipLaunchKernelGGL(replay_ec_full<double>, dim3(kEcGrid), dim3(kEcRun), lds, st, a);
    else hipLaunchKernelGGL(replay_ec_full<float>, dim3(kEcGrid), dim3(kEcRun), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_replay_ec_update(const PhiArgs &a, bool fp64, hipStream_t st, int64_t hops_known) {
    // a known hop count (at most the list's capacity) sizes the grid: one
    // workgroup per hop, none when there is none
    if (hops_known == 0) return hipSuccess;
    const int grid = hops_known > 0 && hops_known < kEcGrid ? (int)hops_known : kEcGrid;
    PhiArgs b = a;
    b.known_count = hops_known >= 0 && hops_known <= a.hop_cap ? hops_known : -1;
    if (fp64) hipLaunchKernelGGL(replay_ec_update<double>, dim3(grid), dim3(256), 0, st, b);
    else hipLaunchKernelGGL(replay_ec_update<float>, dim3(grid), dim3(256), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_zero_i64(int64_t *p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_i64, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace kmc
