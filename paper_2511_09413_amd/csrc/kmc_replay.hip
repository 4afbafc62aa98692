// Score replay, one streaming kernel per half-step (kmc_score_replay in
// include/kmc.h; main text Eq. hop_rate and Eq. 2 for the rate law whose
// log-derivatives are summed).
//
// The replay re-takes the forward's decisions and, for every candidate bond,
// adds W g (y - p)/(1 - p) (0 when p = 1) to the device's four sums, g the
// log-derivatives of p with respect to the common barrier shift, nu0, kappa
// and alpha, y the decision and W the step's weight.  p is evaluated with the
// Coulomb part of the bond's energy change kept per bond (the exact window sum
// in binary64 rounded once to the path's precision, maintained by
// replay_ec_full / replay_ec_update), the rest in the path's precision.
//
// A workgroup takes a run of consecutive rails of one device (sixteen passes of
// 256 / (pitch / 8) rails); a thread owns one Philox block (the four bonds of
// the parity in eight sites) per pass, and loads the next pass's occupancy and
// per-bond Coulomb parts before scoring the current one.  Decisions are the
// forward's: the exact class
// prefilter settles almost every candidate as rejected on its word alone; a
// survivor is listed in LDS and decided at the end of its pass with the full
// window sum over the half-step's snapshot, one wavefront per survivor in the same
// order as the hop kernels (lanes strided over the window, then a butterfly),
// so the decision equals the forward's bit for bit.  The kernel never writes
// the snapshot: accepted hops are marked in an LDS flip mask, each pass writes
// its blocks' new state to the other plane, and the hops go to the list from
// which replay_ec_update recomputes the Coulomb parts they changed.  The
// candidates the prefilter rejects (y = 0) are compacted per wavefront in LDS
// before their terms are evaluated, 64 per round.
#include "kmc_device.h"
#include "kmc_internal.h"

namespace kmc {

namespace {

constexpr int kRBlock = 256;
constexpr int kRPasses = 16;
constexpr int kRRing = 2 * kRBlock * 4;  // twice every bond of one pass

// The exponential factor exp(-beta (Ea + dE/2)) of a score term's rate (not
// of a decision), from y2 = 2 Ea + dE and the factor k = score_factor: in
// binary64 as the decisions, exp(y2 (-beta/2)), which rounds -beta (Ea +
// dE/2) exactly as written (the scalings by two are exact); in binary32 the
// hardware's base-2 exponential of y2 k with k = -beta log2(e) / 2 rounded
// once (the constant's and the product's roundings add about |x| eps to the
// relative error of p, the base-2 exponential about one unit).
template <typename Real>
__device__ __forceinline__ Real score_exp(Real y2, Real k);
template <>
__device__ __forceinline__ double score_exp<double>(double y2, double k) { return exp(y2 * k); }
template <>
__device__ __forceinline__ float score_exp<float>(float y2, float k) { return __builtin_amdgcn_exp2f(y2 * k); }
template <typename Real>
__host__ __device__ __forceinline__ Real score_factor(double beta) {
    return std::is_same<Real, double>::value ? (Real)(-0.5 * beta) : (Real)(-0.5 * beta * 1.4426950408889634);
}

// A value every lane holds alike, moved to scalar registers.
__device__ __forceinline__ float uniform(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double uniform(double x) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, (uint64_t)hi << 32 | lo);
}

// x with its sign bit flipped where bit 31 of sign is set.
__device__ __forceinline__ float flip_sign(float x, uint32_t sign) {
    return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, x) ^ sign);
}
__device__ __forceinline__ double flip_sign(double x, uint32_t sign) {
    return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, x) ^ ((uint64_t)sign << 32));
}

template <typename Real>
__device__ __forceinline__ const Real *ktable(const HopArgs &a) {
    return std::is_same<Real, double>::value ? reinterpret_cast<const Real *>(a.ktab64)
                                             : reinterpret_cast<const Real *>(a.ktab32);
}

template <typename Real, int H>
__global__ __launch_bounds__(kRBlock) void replay_stream(HopArgs a) {
    __shared__ double v_wg;
    __shared__ uint32_t wtab[kClasses];             // prefilter threshold of each barrier class
    __shared__ int n_surv;                          // survivors listed so far (the list is a ring)
    __shared__ uint32_t surv[kRRing];               // (rail - r0) << 12 | s
    __shared__ uint32_t flips[kRBlock];             // bit j: byte s0 + j of the thread's block flips
    __shared__ double gsum[kRBlock / 64][4];
    __shared__ Real rec_ec[kRBlock / 64][4 * 64];   // per wavefront: compacted rejected candidates
    __shared__ Real rec_ea[kRBlock / 64][4 * 64];
    __shared__ uint32_t rec_aux[kRBlock / 64][4 * 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const Tile tile = a.dtiles[blockIdx.x];
    const int d = tile.d;
    const DevInfo &dv = a.devs[d];
    const int L = dv.sites, R = dv.rails, pitch = dv.pitch, bpr = pitch / 8;
    const int64_t n = a.n_abs;
    // the count of the previous half-step's list (the other parity) was
    // consumed by its update kernel: clear it for the next half-step
    if (blockIdx.x == 0 && tid == 0)
        __hip_atomic_store(a.hop_ctl + (1 - H), (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid < kClasses) {  // every thread evaluates the step's bias; one class threshold each
        const double V = protocol_voltage(a.knot_t + d * kMaxKnots, a.knot_v + d * kMaxKnots, dv.n_knots,
                                          (double)(n - dv.n_set) * a.dt);
        wtab[tid] = class_threshold(a.c0, a.beta, a.alpha, V, L, dv.ea_min, dv.ea_step, dv.coul_bound, tid);
        if (tid == 0) {
            v_wg = V;
            n_surv = 0;
        }
    }
    flips[tid] = 0u;
    const int per_pass = kRBlock / bpr;
    const int slot = tid / bpr, b = tid - slot * bpr, s0 = 8 * b;
    const bool lane_used = slot < per_pass;
    const int r_end = tile.r0 + tile.nr;
    const int8_t *snap = a.occ_in + dv.off_pad;
    const Real *ec_of = reinterpret_cast<const Real *>(a.rec);
    const int64_t odd_at = (L + 1) / 2;  // start of the odd bonds in a rail's run
    const int last = L - 2 - s0;         // bond (s0+k, s0+k+1) exists iff k <= last
    const uint32_t exist = last >= 7 ? 0xFFu : (last < 0 ? 0u : ((2u << last) - 1u));
    // a pass's occupancy block and the Coulomb parts of its four bonds.  The
    // loads are issued unconditionally (a lane without a block of this pass
    // reads the run's first rail and ignores it; the parts of bonds beyond a
    // rail's end are read from the array's padding or the next run and
    // ignored), so that the memory counter of every lane counts the same
    // loads and the next pass's loads stay in flight while this one is
    // scored.
    const int64_t dev_off = dv.off;
    const int64_t ec_base = dev_off + (H ? odd_at : 0) + 4 * b;
    const int8_t *snap_s0 = snap + s0;
    auto load_pass = [&](int r, uint2 &v, uint32_t &nxt, Real *ec) {
        const int rl = (lane_used && r < r_end) ? r : tile.r0;
        const int8_t *row = snap_s0 + (int64_t)rl * pitch;
        v = *reinterpret_cast<const uint2 *>(row);
        nxt = H == 1 ? (uint32_t)(uint8_t)row[s0 + 8 < pitch ? 8 : 0] : 0u;
        const Real *e = ec_of + ec_base + (int64_t)rl * L;
#pragma unroll
        for (int i = 0; i < 4; ++i) ec[i] = e[i];
    };
    uint2 v_next;
    uint32_t nx_next;
    Real ec_next[4];
    load_pass(tile.r0 + slot, v_next, nx_next, ec_next);
    __syncthreads();
    const double V = v_wg;
    const uint32_t thr0 = wtab[0];  // the largest threshold (lowest class)
    const Real alpha_r = (Real)a.alpha, V_r = (Real)V, beta_r = (Real)a.beta, c0_r = (Real)a.c0;
    const double W = a.score_w[d], beta = a.beta;
    const double w_ea = W * -beta, w_nu = W * (1.0 / a.nu0);
    const double w_k = W * (-0.5 * beta / a.kappa), w_a = W * (-0.5 * beta * V / (double)L);
    // Per thread: S0 = sum of (y - p)/(1 - p) over its candidates (the Ea and
    // nu0 terms are W g times it, g the same for every candidate), S2 = sum of
    // dE_coul (y - p)/(1 - p) and S3 = sum of +-(y - p)/(1 - p) (sign of t - o);
    // the constant factors are applied once at the end.
    double S0 = 0.0, S2 = 0.0, S3 = 0.0;
    // the bias part of dE for a hop toward site L - 1 and toward site 0 (the
    // same expression as the forward's, t - o = +-1)
    const Real e_up = ((alpha_r * V_r) * (Real)1) / (Real)L;
    const Real e_down = ((alpha_r * V_r) * (Real)-1) / (Real)L;
    const Real kf = score_factor<Real>(a.beta);
    // score term of one candidate with its decision y
    auto term = [&](Real ec, Real ea, bool up, uint32_t y) {
        const Real dE = (up ? e_up : e_down) + ec;
        Real p = c0_r * score_exp<Real>((ea + ea) + dE, kf);
        p = p < (Real)1 ? p : (Real)1;
        if (p < (Real)1) {
            // (y - p)/(1 - p) with a reciprocal refined by two Newton steps
            // (within an ulp or two of the rounded quotient; 1 - p lies in (0, 1])
            const double pd = (double)p;
            const double den = 1.0 - pd;
            double rc = __builtin_amdgcn_rcp(den);
            rc = fma(rc, fma(-den, rc, 1.0), rc);
            rc = fma(rc, fma(-den, rc, 1.0), rc);
            const double ratio = ((double)y - pd) * rc;
            S0 += ratio;
            S2 += (double)ec * ratio;
            S3 += up ? ratio : -ratio;
        }
    };
    // the survivors listed in [from, to) of the ring: the forward's decision
    // from the full window sum over the snapshot, one wavefront each, in the
    // hop kernels' order; the score term of each with its decision
    const Real *kt = ktable<Real>(a);
    const int kt_stride = a.cutoff + 1;
    const uint32_t ctr3 = ((uint32_t)d << 4) | (uint32_t)H;
    auto decide_survivors = [&](int from, int to) {
        for (int i = from + wave; i < to; i += kRBlock / 64) {
            const uint32_t e = surv[i & (kRRing - 1)];
            const int rr = tile.r0 + (int)(e >> 12), s = (int)(e & 4095u);
            const int8_t *rp = snap + (int64_t)rr * pitch;
            const bool first = rp[s] & 1;
            const int o = first ? s : s + 1, t = first ? s + 1 : s;
            int lo = s - a.cutoff, hi = s + 1 + a.cutoff;
            lo = lo < 0 ? 0 : lo;
            hi = hi > L - 1 ? L - 1 : hi;
            Real part = (Real)0;
            for (int k = 0; k < dv.n_nbr; ++k) {
                const int off = dv.nbr_off[k];
                const Real *ktr = kt + dv.nbr_dist[k] * kt_stride;
                const int8_t *nrow = snap + (int64_t)(((rr + off) % R + R) % R) * pitch;
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
                const uint4 blk = philox4x32_10((uint32_t)(s >> 3), (uint32_t)rr, (uint32_t)n, ctr3, a.key0, a.key1);
                const uint32_t word = word_of(blk, (s >> 1) & 3);
                const Real ea = a.ea ? reinterpret_cast<const Real *>(a.ea)[dv.off + (int64_t)rr * L + o] : (Real)a.ea_scalar;
                const bool y = decide_hop<Real>(e_app + part, ea, word, beta_r, c0_r, a.log, d, H, n, rr, s);
                const Real ec = ec_of[dv.off + (int64_t)rr * L + (H ? odd_at : 0) + (s >> 1)];
                term(ec, ea, t > o, y ? 1u : 0u);
                if (y) {
                    // flip bytes s and s + 1 in the masks of the threads that own them
                    const int sl = (rr - tile.r0) % per_pass;
                    atomicOr(&flips[sl * bpr + (s >> 3)], 1u << (s & 7));
                    atomicOr(&flips[sl * bpr + ((s + 1) >> 3)], 1u << ((s + 1) & 7));
                    const int64_t kh = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(a.hop_ctl + H), 1ull);
                    if (kh < a.hop_cap) a.hops[kh] = make_uint4((uint32_t)d, (uint32_t)rr, (uint32_t)s, first ? 0u : 1u);
                }
            }
        }
    };
    int listed = 0;  // survivors of the earlier passes (the same value in every thread)
    // wavefront priority lowered by quarters of the passes, as in replay_logged
    __builtin_amdgcn_s_setprio(3);
    for (int p = 0; p < kRPasses; ++p) {
        if (p == kRPasses / 4) __builtin_amdgcn_s_setprio(2);
        if (p == kRPasses / 2) __builtin_amdgcn_s_setprio(1);
        if (p == 3 * kRPasses / 4) __builtin_amdgcn_s_setprio(0);
        const int r = tile.r0 + slot + p * per_pass;
        const bool valid = lane_used && r < r_end;
        const uint2 v = v_next;
        const uint32_t nxt = nx_next;
        Real ec[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) ec[i] = ec_next[i];
        if (p + 1 < kRPasses) load_pass(r + per_pass, v_next, nx_next, ec_next);  // in flight meanwhile
        const uint32_t bits = (((v.x & 0x01010101u) * 0x01020408u) >> 24 & 0xFu) |
                              ((((v.y & 0x01010101u) * 0x01020408u) >> 24 & 0xFu) << 4) | ((nxt & 1u) << 8);
        // (exist drops the last block's bond 7 when site s0 + 8 lies beyond the rail)
        const uint32_t cand = valid ? (bits ^ (bits >> 1)) & (H ? 0xAAu : 0x55u) & exist : 0u;
        int pushed = 0;
        uint32_t rest = 0u;  // bit i: bond i is a candidate rejected by the prefilter (y = 0)
        if (cand) {
            const uint4 blk = philox4x32_10((uint32_t)b, (uint32_t)r, (uint32_t)n, ((uint32_t)d << 4) | (uint32_t)H,
                                            a.key0, a.key1);
            // stage 0 without branches: bit i when bond i is a candidate whose
            // word passes the lowest class's threshold
            uint32_t c4 = 0u, s4 = 0u;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t ci = (cand >> (H + 2 * i)) & 1u;
                c4 |= ci << i;
                s4 |= (ci & (word_of(blk, i) <= thr0 ? 1u : 0u)) << i;
            }
            rest = c4 & ~s4;
            if (s4) {  // rare: the origin's class decides whether it survives
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (!((s4 >> i) & 1u)) continue;
                    const int k = H + 2 * i;
                    const int s = s0 + k;
                    const int o = ((bits >> k) & 1u) ? s : s + 1;
                    const int j = o - s0;
                    const uint32_t ob = j < 8 ? ((j < 4 ? v.x : v.y) >> (8 * (j & 3))) & 0xFFu : nxt;
                    if (word_of(blk, i) <= wtab[ob >> 1]) {
                        // decided (and scored) at the end of the pass
                        const int q = atomicAdd(&n_surv, 1);
                        surv[q & (kRRing - 1)] = ((uint32_t)(r - tile.r0) << 12) | (uint32_t)s;
                        pushed = 1;
                    } else {
                        rest |= 1u << i;
                    }
                }
            }
        }
        // the rejected candidates of the wavefront, compacted: each lane writes
        // its records from its offset among the wavefront's records (a prefix
        // count from three ballots of its count's bits), and the wavefront then
        // scores 64 records per round (a lane's four bond slots would otherwise
        // cost four rounds whenever any lane has a candidate in each)
        {
            const uint32_t cnt = (uint32_t)__builtin_popcount(rest);
            uint32_t at = 0u, total = 0u;
#pragma unroll
            for (int bit = 0; bit < 3; ++bit) {
                const uint64_t bal = __ballot((cnt >> bit) & 1u);
                at += __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))
                      << bit;
                total += (uint32_t)__popcll(bal) << bit;
            }
            uint32_t m = rest;
            while (m) {
                const int i = __builtin_ctz(m);
                m &= m - 1u;
                const uint32_t up = (bits >> (H + 2 * i)) & 1u;  // 1: toward site L-1
                rec_ec[wave][at] = ec[i];
                rec_aux[wave][at] = up;
                if (a.ea) {
                    const int s = s0 + H + 2 * i;
                    rec_ea[wave][at] = reinterpret_cast<const Real *>(a.ea)[dev_off + (int64_t)r * L + (up ? s : s + 1)];
                }
                ++at;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
            for (int j = lane; j < (int)total; j += 64) {
                const Real ea = a.ea ? rec_ea[wave][j] : (Real)a.ea_scalar;
                term(rec_ec[wave][j], ea, rec_aux[wave][j] != 0u, 0u);
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
        }
        uint32_t f = 0u;
        if (__syncthreads_or(pushed)) {  // uniform: the pass had survivors
            const int to = n_surv;
            decide_survivors(listed, to);
            listed = to;
            __syncthreads();  // their flips are in the masks
            f = flips[tid];
            flips[tid] = 0u;
        }
        if (valid) {  // the new state of the pass's block
            uint2 vn = v;
            vn.x ^= ((f & 0xFu) * 0x00204081u) & 0x01010101u;
            vn.y ^= (((f >> 4) & 0xFu) * 0x00204081u) & 0x01010101u;
            *reinterpret_cast<uint2 *>(a.occ_out + dv.off_pad + (int64_t)r * pitch + s0) = vn;
        }
    }
    // the workgroup's four sums, one atomic each
    double g0 = w_ea * S0, g1 = w_nu * S0, g2 = w_k * S2, g3 = w_a * S3;
#pragma unroll
    for (int sh_ = 32; sh_ >= 1; sh_ >>= 1) {
        g0 += __shfl_xor(g0, sh_, 64);
        g1 += __shfl_xor(g1, sh_, 64);
        g2 += __shfl_xor(g2, sh_, 64);
        g3 += __shfl_xor(g3, sh_, 64);
    }
    if (lane == 0) {
        gsum[wave][0] = g0;
        gsum[wave][1] = g1;
        gsum[wave][2] = g2;
        gsum[wave][3] = g3;
    }
    __syncthreads();
    if (tid < 4) {
        double sum = 0.0;
        for (int w = 0; w < kRBlock / 64; ++w) sum += gsum[w][tid];
        if (sum != 0.0) atomicAdd(&a.score_grad[d * 4 + tid], sum);
    }
}

// The recorded replay of one half-step: the decisions are the forward's, read
// from the list of hops it recorded for this half-step, so there is no Philox
// draw, prefilter or window sum; every candidate's term comes from its bond's
// Coulomb part.  The workgroup takes the same runs of rails as replay_stream,
// marks the recorded hops of its rails in LDS, scores its sixteen passes
// (every candidate compacted per wavefront as there), and at the end flips the
// two sites of each of its hops in the state in place: a workgroup reads only
// its own rails, so no other workgroup sees a flip before the launch ends.
// The state is one bit per site (pack_occ_bits), a byte per thread's block of
// eight sites, so that the pass reads an eighth of the bytes it would read as
// a byte per site; the flips are atomic exclusive-ors of 32-bit words, whose
// other bits may belong to other hops or to another workgroup's rails.
constexpr int kLogRec = 64 + 4 * 64;  // a carried partial round and one pass's candidates

// One candidate of the recorded replay: its bond's Coulomb part, and in aux
// kDown (the ion moves toward site 0) and kHopped (the decision).
constexpr uint32_t kDown = 0x80000000u, kHopped = 0x40000000u;
template <typename Real>
struct alignas(2 * sizeof(Real)) LogRec {
    Real ec;
    uint32_t aux;
};

template <typename Real, int H, bool kSiteEa>
__global__ __launch_bounds__(kRBlock, 8) void replay_logged(HopArgs a) {
    __shared__ double v_wg;
    __shared__ uint32_t taken[kRPasses * kRBlock / 4];  // byte (pass, thread): bit j when the bond at s0 + j hopped
    __shared__ double gsum[kRBlock / 64][4];
    // per wavefront: the candidates not yet scored (fewer than 64 carried
    // over from the earlier passes, then the current pass's)
    __shared__ LogRec<Real> rec[kRBlock / 64][kLogRec];
    __shared__ Real rec_ea[kRBlock / 64][kLogRec];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const Tile tile = a.dtiles[blockIdx.x];
    const int d = tile.d;
    const DevInfo &dv = a.devs[d];
    const int L = dv.sites, pitch = dv.pitch, bpr = pitch / 8;
    const int64_t n = a.n_abs;
    // the workspace hop list of the other parity was consumed by its update
    // kernel (a half-step replayed without the recording may follow)
    if (blockIdx.x == 0 && tid == 0)
        __hip_atomic_store(a.hop_ctl + (1 - H), (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid == 0)
        v_wg = protocol_voltage(a.knot_t + d * kMaxKnots, a.knot_v + d * kMaxKnots, dv.n_knots,
                                (double)(n - dv.n_set) * a.dt);
    for (int i = tid; i < kRPasses * kRBlock / 4; i += kRBlock) taken[i] = 0u;
    const int per_pass = kRBlock / bpr;
    const int slot = tid / bpr, b = tid - slot * bpr, s0 = 8 * b;
    const bool lane_used = slot < per_pass;
    const int r_end = tile.r0 + tile.nr;
    const int rowb = pitch / 8;  // bytes per rail (the pitch is a multiple of 16 sites)
    const uint8_t *snap = reinterpret_cast<const uint8_t *>(a.occ_in) + dv.off_pad / 8;
    const Real *ec_of = reinterpret_cast<const Real *>(a.rec);
    const int64_t odd_at = (L + 1) / 2;
    const int last = L - 2 - s0;
    const uint32_t exist = last >= 7 ? 0xFFu : (last < 0 ? 0u : ((2u << last) - 1u));
    const int64_t dev_off = dv.off;
    const int64_t ec_base = dev_off + (H ? odd_at : 0) + 4 * b;
    const uint8_t *snap_b = snap + b;
    // as in replay_stream: unconditional loads, the next pass's in flight
    auto load_pass = [&](int r, uint32_t &v, uint32_t &nxt, Real *ec) {
        const int rl = (lane_used && r < r_end) ? r : tile.r0;
        const uint8_t *row = snap_b + (int64_t)rl * rowb;
        v = row[0];
        nxt = H == 1 ? (uint32_t)row[b + 1 < bpr ? 1 : 0] : 0u;
        const Real *e = ec_of + ec_base + (int64_t)rl * L;
#pragma unroll
        for (int i = 0; i < 4; ++i) ec[i] = e[i];
    };
    uint32_t v_next, nx_next;
    Real ec_next[4];
    load_pass(tile.r0 + slot, v_next, nx_next, ec_next);
    __syncthreads();
    // the recorded hops of this workgroup's rails (the host has checked that
    // the list did not overflow)
    const int64_t n_hops = *a.rec_count;
    auto mine = [&](const uint4 &e) {
        const int rel = (int)e.y - tile.r0;
        return (int)e.x == d && rel >= 0 && rel < tile.nr && (int)e.z >= 0 && (int)e.z + 1 < L;
    };
    for (int64_t i = tid; i < n_hops; i += kRBlock) {
        const uint4 e = a.rec_hops[i];
        if (mine(e)) {
            const int rel = (int)e.y - tile.r0, s = (int)e.z;
            const int pp = rel / per_pass, sl = rel - pp * per_pass;
            const int at = pp * kRBlock + sl * bpr + (s >> 3);
            atomicOr(&taken[at >> 2], 1u << (8 * (at & 3) + (s & 7)));
        }
    }
    __syncthreads();
    const double V = uniform(v_wg);  // the workgroup's values in scalar registers
    const Real alpha_r = (Real)a.alpha, V_r = (Real)V, c0_r = (Real)a.c0;
    const double W = a.score_w[d], beta = a.beta;
    const double w_ea = W * -beta, w_nu = W * (1.0 / a.nu0);
    const double w_k = W * (-0.5 * beta / a.kappa), w_a = W * (-0.5 * beta * V / (double)L);
    // S0, S2, S3 as in replay_stream
    double S0 = 0.0, S2 = 0.0, S3 = 0.0;
    // the bias part of dE toward site L - 1 (the forward's expression; toward
    // site 0 it is exactly its negative), in scalar registers
    const Real e_up = uniform(((alpha_r * V_r) * (Real)1) / (Real)L);
    // per-site barriers (kSiteEa, a.ea not null) or one barrier for all sites
    const Real *ea_of = reinterpret_cast<const Real *>(a.ea);
    const Real ea2_scalar = (Real)a.ea_scalar + (Real)a.ea_scalar;
    const Real kf = score_factor<Real>(a.beta);
    // The term of one candidate, equal bit for bit to replay_stream's: p =
    // c0 score_exp(2 ea + dE), and (y - p)/(1 - p) with the reciprocal refined
    // by Newton steps to within an ulp or two of binary64 (one step from the
    // hardware estimate for a binary32 p, two for binary64).
    auto term = [&](Real ec, Real ea2, uint32_t aux) {
        const uint32_t dn = aux & kDown;
        const Real dE = flip_sign(e_up, dn) + ec;
        const Real p = c0_r * score_exp<Real>(ea2 + dE, kf);
        if (p < (Real)1) {
            const double pd = (double)p;
            const double den = 1.0 - pd;
            double rc = __builtin_amdgcn_rcp(den);
            rc = fma(rc, fma(-den, rc, 1.0), rc);
            if (std::is_same<Real, double>::value) rc = fma(rc, fma(-den, rc, 1.0), rc);
            double ratio = -pd * rc;
            // the decision y = 1 is rare (about one candidate in 1e5): a
            // branch no lane takes costs less than a select on every term
            const bool hop = (aux & kHopped) != 0u;
            if (__builtin_expect(__ballot(hop) != 0, 0)) {
                if (hop) ratio = den * rc;
            }
            S0 += ratio;
            S2 = fma((double)ec, ratio, S2);
            S3 += flip_sign(ratio, dn);
        }
    };
    // scores the wavefront's records [0, n)
    auto score_rounds = [&](uint32_t n) {
        for (int j = lane; j < (int)n; j += 64) {
            const Real ea2 = kSiteEa ? rec_ea[wave][j] : ea2_scalar;
            const LogRec<Real> x = rec[wave][j];
            term(x.ec, ea2, x.aux);
        }
    };
    uint32_t pending = 0u;  // records carried to the next pass (uniform)
    // per lane: the word of the hop table that holds its byte of every pass
    // (pass p at p kRBlock / 4 words further), the byte's place in it, and the
    // candidate mask's fixed part (the parity and the bonds the rail has)
    const uint32_t *taken_at = taken + (tid >> 2);
    const int taken_sh = 8 * (tid & 3);
    const uint32_t par_exist = lane_used ? (H ? 0xAAu : 0x55u) & exist : 0u;
    // The issue arbiter prefers older wavefronts: each wavefront lowers its
    // priority by quarters of its passes, so that the workgroups dispatched
    // later are not left alone on their SIMDs at the end of the launch.
    __builtin_amdgcn_s_setprio(3);
#pragma unroll
    for (int p = 0; p < kRPasses; ++p) {
        if (p == kRPasses / 4) __builtin_amdgcn_s_setprio(2);
        if (p == kRPasses / 2) __builtin_amdgcn_s_setprio(1);
        if (p == 3 * kRPasses / 4) __builtin_amdgcn_s_setprio(0);
        const int r = tile.r0 + slot + p * per_pass;
        const uint32_t bits = v_next | ((nx_next & 1u) << 8);  // bit j: site s0 + j
        Real ec[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) ec[i] = ec_next[i];
        if (p + 1 < kRPasses) load_pass(r + per_pass, v_next, nx_next, ec_next);
        const uint32_t cand = r < r_end ? (bits ^ (bits >> 1)) & par_exist : 0u;
        const uint32_t hopped = (taken_at[p * (kRBlock / 4)] >> taken_sh) & 0xFFu;
        // bit k: the bond hopped; bit k + 1: toward site 0 (k of parity H; the
        // masks keep the other parity's bits out), moved to kHopped and kDown
        const uint32_t par = H ? 0xAAu : 0x55u;
        const uint32_t aux_bits = (hopped & par) | ((~bits & par) << 1);
        // the wavefront's candidates, slot-major (slot i of every lane, in
        // lane order, after those of slots < i), after the carried ones; the
        // slot's ballot is the branch's lane mask
        uint32_t base = pending;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = H + 2 * i;
            const uint64_t bal = __ballot((cand >> k) & 1u);
            if (__builtin_amdgcn_inverse_ballot_w64(bal)) {
                const uint32_t at =
                    __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, base));
                LogRec<Real> x;
                x.ec = ec[i];
                x.aux = aux_bits << (30 - k);  // (the bits below kHopped are not read)
                rec[wave][at] = x;
                if (kSiteEa) {
                    const int s = s0 + k;
                    const Real ea = ea_of[dev_off + (int64_t)r * L + (((bits >> k) & 1u) ? s : s + 1)];
                    rec_ea[wave][at] = ea + ea;
                }
            }
            base += (uint32_t)__popcll(bal);
        }
        // whole rounds of 64 now (all of them after the last pass); the rest
        // moves to the front for the next pass
        const uint32_t upto = p + 1 < kRPasses ? (base & ~63u) : base;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
        score_rounds(upto);
        pending = base - upto;
        if (upto != 0u && (uint32_t)lane < pending) {
            const uint32_t from = upto + (uint32_t)lane;
            const LogRec<Real> x = rec[wave][from];
            const Real ea = kSiteEa ? rec_ea[wave][from] : (Real)0;
            rec[wave][lane] = x;
            if (kSiteEa) rec_ea[wave][lane] = ea;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
    }
    // every pass has read its rails: flip the hops' sites in place
    __syncthreads();
    uint32_t *words = reinterpret_cast<uint32_t *>(a.occ_out);
    for (int64_t i = tid; i < n_hops; i += kRBlock) {
        const uint4 e = a.rec_hops[i];
        if (mine(e)) {
            const int64_t at = dv.off_pad + (int64_t)e.y * pitch + e.z;  // bit of site s
            uint32_t *w0 = words + (at >> 5);
            const int sh = (int)(at & 31);
            // the two sites' bits (other bits of the words may be flipping)
            const uint32_t x0 = __hip_atomic_load(w0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t x1 =
                sh < 31 ? x0 >> 1 : __hip_atomic_load(w0 + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) << 31;
            if (((x0 ^ x1) >> sh) & 1u) {  // a hop moves an ion to an empty site
                if (sh < 31) {
                    atomicXor(w0, 3u << sh);
                } else {
                    atomicXor(w0, 1u << 31);
                    atomicXor(w0 + 1, 1u);
                }
            }
        }
    }
    double g0 = w_ea * S0, g1 = w_nu * S0, g2 = w_k * S2, g3 = w_a * S3;
#pragma unroll
    for (int sh_ = 32; sh_ >= 1; sh_ >>= 1) {
        g0 += __shfl_xor(g0, sh_, 64);
        g1 += __shfl_xor(g1, sh_, 64);
        g2 += __shfl_xor(g2, sh_, 64);
        g3 += __shfl_xor(g3, sh_, 64);
    }
    if (lane == 0) {
        gsum[wave][0] = g0;
        gsum[wave][1] = g1;
        gsum[wave][2] = g2;
        gsum[wave][3] = g3;
    }
    __syncthreads();
    if (tid < 4) {
        double sum = 0.0;
        for (int w = 0; w < kRBlock / 64; ++w) sum += gsum[w][tid];
        if (sum != 0.0) atomicAdd(&a.score_grad[d * 4 + tid], sum);
    }
}

// Sets *flag when the n bytes at x and y differ anywhere.
__global__ void compare_bytes(const int8_t *x, const int8_t *y, int64_t n, int64_t *flag) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool diff = false;
    const bool wide = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15) == 0;
    int64_t done = 0;
    if (wide) {
        const int64_t n16 = n / 16;
        const uint4 *x4 = reinterpret_cast<const uint4 *>(x), *y4 = reinterpret_cast<const uint4 *>(y);
        for (int64_t i = t; i < n16; i += stride) {
            const uint4 u = x4[i], w = y4[i];
            diff |= ((u.x ^ w.x) | (u.y ^ w.y) | (u.z ^ w.z) | (u.w ^ w.w)) != 0u;
        }
        done = n16 * 16;
    }
    for (int64_t i = done + t; i < n; i += stride) diff |= x[i] != y[i];
    if (diff) __hip_atomic_store(flag, (int64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One bit per site from a byte per site (bit 0 = occupied): 16 sites per
// thread, bit i % 8 of byte i / 8 for padded site i.
__global__ __launch_bounds__(256) void pack_occ_bits(const int8_t *src, uint16_t *dst, int64_t n16) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n16) return;
    const uint4 v = reinterpret_cast<const uint4 *>(src)[i];
    auto four = [](uint32_t x) { return ((x & 0x01010101u) * 0x01020408u) >> 24 & 0xFu; };
    dst[i] = (uint16_t)(four(v.x) | four(v.y) << 4 | four(v.z) << 8 | four(v.w) << 12);
}

// The inverse: bit 0 of every byte of dst from the bits, its other bits
// (barrier classes) kept.
__global__ __launch_bounds__(256) void unpack_occ_bits(const uint16_t *src, int8_t *dst, int64_t n16) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n16) return;
    uint4 v = reinterpret_cast<uint4 *>(dst)[i];
    const uint32_t b = src[i];
    auto spread = [](uint32_t q) { return (q & 1u) | (q & 2u) << 7 | (q & 4u) << 14 | (q & 8u) << 21; };
    v.x = (v.x & 0xFEFEFEFEu) | spread(b & 0xFu);
    v.y = (v.y & 0xFEFEFEFEu) | spread(b >> 4 & 0xFu);
    v.z = (v.z & 0xFEFEFEFEu) | spread(b >> 8 & 0xFu);
    v.w = (v.w & 0xFEFEFEFEu) | spread(b >> 12);
    reinterpret_cast<uint4 *>(dst)[i] = v;
}

}  // namespace

// n_pad: padded sites (a multiple of 16); byte planes 16-byte aligned, the
// bit plane 4-byte aligned.
hipError_t launch_pack_occ_bits(const int8_t *src, uint8_t *dst, int64_t n_pad, hipStream_t st) {
    const int64_t n16 = n_pad / 16;
    if (n16 <= 0) return hipSuccess;
    hipLaunchKernelGGL(pack_occ_bits, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, st, src,
                       reinterpret_cast<uint16_t *>(dst), n16);
    return hipGetLastError();
}

hipError_t launch_unpack_occ_bits(const uint8_t *src, int8_t *dst, int64_t n_pad, hipStream_t st) {
    const int64_t n16 = n_pad / 16;
    if (n16 <= 0) return hipSuccess;
    hipLaunchKernelGGL(unpack_occ_bits, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<const uint16_t *>(src), dst, n16);
    return hipGetLastError();
}

hipError_t launch_replay_logged(const HopArgs &a, bool fp64, hipStream_t st) {
    const dim3 grid(a.n_dtiles), block(kRBlock);
    if (fp64) {
        if (a.ea) {
            if (a.h == 0) hipLaunchKernelGGL((replay_logged<double, 0, true>), grid, block, 0, st, a);
            else hipLaunchKernelGGL((replay_logged<double, 1, true>), grid, block, 0, st, a);
        } else {
            if (a.h == 0) hipLaunchKernelGGL((replay_logged<double, 0, false>), grid, block, 0, st, a);
            else hipLaunchKernelGGL((replay_logged<double, 1, false>), grid, block, 0, st, a);
        }
    } else {
        if (a.ea) {
            if (a.h == 0) hipLaunchKernelGGL((replay_logged<float, 0, true>), grid, block, 0, st, a);
            else hipLaunchKernelGGL((replay_logged<float, 1, true>), grid, block, 0, st, a);
        } else {
            if (a.h == 0) hipLaunchKernelGGL((replay_logged<float, 0, false>), grid, block, 0, st, a);
            else hipLaunchKernelGGL((replay_logged<float, 1, false>), grid, block, 0, st, a);
        }
    }
    return hipGetLastError();
}

hipError_t launch_compare_bytes(const int8_t *x, const int8_t *y, int64_t n, int64_t *flag, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t want = (n + 16 * 256 - 1) / (16 * 256);
    const int grid = (int)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(compare_bytes, dim3(grid), dim3(256), 0, st, x, y, n, flag);
    return hipGetLastError();
}

// Rails of one run of the streaming replay (sixteen passes of a 256-thread
// workgroup, pitch / 8 threads per rail), or 0 when a rail is longer than
// one workgroup covers.
int replay_run_rails(int pitch) {
    const int bpr = pitch / 8;
    return bpr > kRBlock ? 0 : kRPasses * (kRBlock / bpr);
}

hipError_t launch_replay_stream(const HopArgs &a, bool fp64, hipStream_t st) {
    const dim3 grid(a.n_dtiles), block(kRBlock);
    if (fp64) {
        if (a.h == 0) hipLaunchKernelGGL((replay_stream<double, 0>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((replay_stream<double, 1>), grid, block, 0, st, a);
    } else {
        if (a.h == 0) hipLaunchKernelGGL((replay_stream<float, 0>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((replay_stream<float, 1>), grid, block, 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace kmc
