// Dense long-range Coulomb potential on the MFMA units of gfx950 (MI355X).
//
// phi(r, s) = sum over rails r' within rail_range (r itself included) and all
// sites j of occ(r', j) K(s - j, dist(r, r')), K(0, 0) = 0: the field of the
// ions that the hop decision adds to the bias (paper main text section 3).
// Written as a product C[rail][s] = sum_k X[rail][k] T[k][s] with k = (dist,
// j):
//   X[rail][(dist, j)] = sum of occ(r', j) over the distinct rails r' at
//     minimal-image distance dist from the rail (0, 1 or 2 ions: exact in
//     BF16); folding the rails at +-dist halves the work;
//   T[(dist, j)][s] = K(s - j, dist), Toeplitz in (j, s) for every dist, so a
//     32 x 32 block of T depends only on (dist, jb - sb): the kernel reads its
//     MFMA fragments from a small table of distinct blocks (L2-resident),
//     each value split as K = hi + lo with hi, lo in BF16 (|K - hi - lo| <=
//     2^-16 |K|); both products accumulate in FP32.
// One workgroup (4 wavefronts) computes 128 rails x 256 sites; a wavefront
// computes 64 rails x 128 sites with v_mfma_f32_32x32x16_bf16, keeps the four
// T blocks of its four 32-site column blocks in registers and slides them
// along the diagonal (one new block per 32-site step of k).  The occupancy rows
// of the workgroup's rails and their +-rail_range halo are staged in LDS; the
// X fragments are built there from the occupancy bytes with byte permutes.
#include <hip/hip_runtime.h>

#include "kmc_device.h"
#include "kmc_internal.h"

namespace kmc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kDenseBlock = 256;  // 4 wavefronts: 2 along rails x 2 along sites

// Eight occupancy-sum bytes (values 0..2) -> eight BF16 values (0, 1.0, 2.0).
__device__ __forceinline__ u32x4 bytes_to_bf16(uint32_t lo4, uint32_t hi4) {
    // byte tables indexed by the value: low and high bytes of BF16 0, 1, 2
    const uint32_t t_lo = 0x00008000u, t_hi = 0x00403F00u;
    const uint32_t l0 = __builtin_amdgcn_perm(0u, t_lo, lo4), h0 = __builtin_amdgcn_perm(0u, t_hi, lo4);
    const uint32_t l1 = __builtin_amdgcn_perm(0u, t_lo, hi4), h1 = __builtin_amdgcn_perm(0u, t_hi, hi4);
    u32x4 r;
    r.x = __builtin_amdgcn_perm(h0, l0, 0x05010400u);
    r.y = __builtin_amdgcn_perm(h0, l0, 0x07030602u);
    r.z = __builtin_amdgcn_perm(h1, l1, 0x05010400u);
    r.w = __builtin_amdgcn_perm(h1, l1, 0x07030602u);
    return r;
}

__global__ __launch_bounds__(kDenseBlock) __attribute__((amdgpu_waves_per_eu(2))) void dense_phi(DenseArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile tile = a.tiles[blockIdx.x];
    const DevInfo &dv = a.devs[tile.d];
    const int R = dv.rails, m = a.rail_range;
    const int Lp = a.nb * 32;
    const int rs = Lp + 8;                   // LDS row stride (bytes), 8 mod 16 against bank conflicts
    const int n_rows = kDenseRails + 2 * m;  // row i = rail r0 - m + i (mod R) while i < nr + 2m
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // stage the occupancy bits of the rows, zero beyond the tile and the row
    const int8_t *src = a.occ + dv.off_pad;
    const int c16 = Lp / 16;
    for (int idx = tid; idx < n_rows * c16; idx += kDenseBlock) {
        const int i = idx / c16, c = idx - i * c16;
        uint2 lo = make_uint2(0, 0), hi = make_uint2(0, 0);
        if (i < tile.nr + 2 * m && c * 16 < dv.pitch) {
            int rail = tile.r0 - m + i;
            rail = ((rail % R) + R) % R;
            const uint4 v = *reinterpret_cast<const uint4 *>(src + (int64_t)rail * dv.pitch + c * 16);
            lo = make_uint2(v.x & 0x01010101u, v.y & 0x01010101u);
            hi = make_uint2(v.z & 0x01010101u, v.w & 0x01010101u);
        }
        *reinterpret_cast<uint2 *>(smem + i * rs + c * 16) = lo;
        *reinterpret_cast<uint2 *>(smem + i * rs + c * 16 + 8) = hi;
    }
    __syncthreads();

    const int wm = wave & 1, wn = wave >> 1;
    const int rail0 = wm * 64;                          // wavefront's first tile rail
    const int sb0 = blockIdx.y * 8 + wn * 4;            // wavefront's first 32-site block
    if (rail0 >= tile.nr || sb0 >= a.nb) return;        // nothing to compute (no barrier follows)

    f32x16 acc[2][4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[mb][t] = f32x16{};

    const int nd = 2 * a.nb - 1;
    const int half = lane >> 5, col = lane & 31;
    // the issue arbiter prefers older wavefronts: each lowers its priority by
    // quarters of its k-steps, so that the workgroups dispatched later are not
    // left alone on their SIMDs at the end of the launch
    const int k_steps = (m + 1) * ((a.nb + 3) / 4);
    int k_done = 0;
    __builtin_amdgcn_s_setprio(3);
    for (int dd = 0; dd <= m; ++dd) {
        // the distinct rails at this minimal-image distance: none, one or two
        int oa = 127, ob = 127;
        for (int k = 0; k < dv.n_nbr; ++k)
            if (dv.nbr_dist[k] == dd) {
                if (oa == 127) oa = dv.nbr_off[k];
                else ob = dv.nbr_off[k];
            }
        if (oa == 127) continue;
        const u32x4 *kt = reinterpret_cast<const u32x4 *>(a.ktiles) + (int64_t)dd * nd * 256 + lane;  // 256 = 2 parts x 2 q x 64 lanes
        auto tile_of = [&](int delta, u32x4 (&b)[2][2]) {
            const u32x4 *p = kt + (int64_t)(delta + a.nb - 1) * 256;
            b[0][0] = p[0];
            b[0][1] = p[64];
            b[1][0] = p[128];
            b[1][1] = p[192];
        };
        // slot[(k - t) & 3] holds the T block of diagonal k - sb0 - t while
        // k-block k is processed (t = 0..3: the wavefront's column blocks).  The
        // block of the next k-step is fetched as soon as its slot is free
        // (after the t = 3 products), a whole k-step ahead of its first use.
        u32x4 slot[4][2][2];
        tile_of(-sb0, slot[0]);
        tile_of(-sb0 - 1, slot[3]);
        tile_of(-sb0 - 2, slot[2]);
        tile_of(-sb0 - 3, slot[1]);
        const unsigned char *rowa0 = smem + (m + rail0 + col + oa) * rs;
        const unsigned char *rowb0 = smem + (m + rail0 + col + (ob == 127 ? 0 : ob)) * rs;
        const bool two = ob != 127;
        for (int jb = 0; jb < a.nb; jb += 4, ++k_done) {
            if (4 * k_done == k_steps) __builtin_amdgcn_s_setprio(2);
            if (2 * k_done == k_steps) __builtin_amdgcn_s_setprio(1);
            if (4 * k_done == 3 * k_steps) __builtin_amdgcn_s_setprio(0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                // X fragments of the two 32-rail blocks, q = 0, 1
                u32x4 xa[2][2];
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const int j = (jb + u) * 32 + q * 16 + half * 8;
                        uint2 va = *reinterpret_cast<const uint2 *>(rowa0 + mb * 32 * rs + j);
                        if (two) {
                            const uint2 vb = *reinterpret_cast<const uint2 *>(rowb0 + mb * 32 * rs + j);
                            va.x += vb.x;
                            va.y += vb.y;
                        }
                        xa[mb][q] = bytes_to_bf16(va.x, va.y);
                    }
                // consecutive products go to different accumulators (no chain
                // of dependent MFMAs); t = 3 first so that its slot can be refilled
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int part = 0; part < 2; ++part)
#pragma unroll
                        for (int mb = 0; mb < 2; ++mb)
                            acc[mb][3] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                __builtin_bit_cast(bf16x8, xa[mb][q]),
                                __builtin_bit_cast(bf16x8, slot[(u + 1) & 3][part][q]), acc[mb][3], 0, 0, 0);
                if (jb + u + 1 < a.nb) tile_of(jb + u + 1 - sb0, slot[(u + 1) & 3]);
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int part = 0; part < 2; ++part)
#pragma unroll
                        for (int t = 0; t < 3; ++t)
#pragma unroll
                            for (int mb = 0; mb < 2; ++mb)
                                acc[mb][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                    __builtin_bit_cast(bf16x8, xa[mb][q]),
                                    __builtin_bit_cast(bf16x8, slot[(u - t) & 3][part][q]), acc[mb][t], 0, 0, 0);
            }
        }
    }

    // epilogue: lane holds column col of every block, rows 8 (r/4) + 4 half + r%4
    const int64_t row0 = dv.row0 + tile.r0;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int s = (sb0 + t) * 32 + col;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int tr = rail0 + mb * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                if (tr < tile.nr && s < a.sites) a.phi[(row0 + tr) * a.phi_row + s] = acc[mb][t][r];
            }
        }
}

// Hop decisions of one half-step from the potential (binary32): one thread per
// Philox block, i.e. the four bonds of parity H starting in sites 8b .. 8b+7 of
// one rail; a workgroup holds whole rails.  dE = alpha V (t - o)/L +
// phi(t) - K(1,0) - phi(o), p = min(nu0 dt exp(-(Ea(o) + dE/2)/kT), 1), accept
// when u < p.  Sites of the thread are written to the new state, including the
// effect of the previous thread's last bond (parity 1 crosses into this
// thread's first site), passed through LDS.
template <int H>
__global__ __launch_bounds__(256) void dense_decide(HopArgs a, int blocks_per_rail) {
    __shared__ uint32_t last_hop[256];
    __shared__ int32_t tally[1 + kDeciles];  // the workgroup's net crossings and decile changes
    __shared__ double v_wg;                  // the bias of the step (one device per workgroup)
    const int tid = threadIdx.x;
    const Tile tile = a.dtiles[blockIdx.x];
    const int d = tile.d;
    const DevInfo &dv = a.devs[d];
    const int64_t n = a.ctl.n_base + a.step_in_chunk;
    const int slot = tid / blocks_per_rail, b = tid - slot * blocks_per_rail;
    const bool active = slot < tile.nr;
    const int r = tile.r0 + slot;
    const int L = dv.sites, s0 = 8 * b;
    // the occupancy and the potential of the block are loaded, and the
    // Philox block drawn, before the barrier that publishes the step's bias,
    // so that their latencies overlap the bias's (blocks without a candidate
    // read their potential needlessly)
    uint2 v = make_uint2(0, 0);
    uint32_t nxt = 0u;
    float4 f0 = make_float4(0.f, 0.f, 0.f, 0.f), f1 = f0;
    float f8 = 0.0f;
    uint4 blk = make_uint4(0u, 0u, 0u, 0u);
    if (active) {
        const int8_t *row = a.occ_in + dv.off_pad + (int64_t)r * dv.pitch;
        v = *reinterpret_cast<const uint2 *>(row + s0);
        nxt = (H == 1 && s0 + 8 < dv.pitch) ? (uint32_t)(uint8_t)row[s0 + 8] : 0u;
        const float *prow = a.phi + (dv.row0 + r) * a.phi_row + s0;
        f0 = *reinterpret_cast<const float4 *>(prow);
        f1 = *reinterpret_cast<const float4 *>(prow + 4);
        f8 = (H == 1 && s0 + 8 < L) ? prow[8] : 0.0f;  // only bond 3 of parity 1 needs it
        blk = philox4x32_10((uint32_t)b, (uint32_t)r, (uint32_t)n, ((uint32_t)d << 4) | (uint32_t)H, a.key0, a.key1);
    }
    if (tid <= kDeciles) tally[tid] = 0;
    if (tid == 0)
        v_wg = protocol_voltage(a.knot_t + d * kMaxKnots, a.knot_v + d * kMaxKnots, dv.n_knots,
                                (double)(n - dv.n_set) * a.dt);
    __syncthreads();
    const double V = v_wg;
    uint32_t hopped = 0;  // bit i: bond i of the block moved
    int8_t *dst = a.occ_out + dv.off_pad + (int64_t)r * dv.pitch + s0;
    if (active) {
        const uint32_t bits = (((v.x & 0x01010101u) * 0x01020408u) >> 24 & 0xFu) |
                              ((((v.y & 0x01010101u) * 0x01020408u) >> 24 & 0xFu) << 4) | ((nxt & 1u) << 8);
        uint32_t cand = (bits ^ (bits >> 1)) & (H ? 0xAAu : 0x55u);
        const int last = L - 2 - s0;  // bond (s0+k, s0+k+1) exists iff k <= last
        if (last < 7) cand &= last < 0 ? 0u : ((2u << last) - 1u);
        if (cand) {
            // potential at site s0 + k, k = 0..8, with k known at compile time
            // (a runtime index would send the nine values through scratch)
            const float ph[9] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w, f8};
            const float alpha_r = (float)a.alpha, V_r = (float)V, beta_r = (float)a.beta, c0_r = (float)a.c0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = H + 2 * i;  // bond (s0 + k, s0 + k + 1)
                if (!((cand >> k) & 1u)) continue;
                const int s = s0 + k;
                const bool first = (bits >> k) & 1u;
                const int o = first ? s : s + 1, t = first ? s + 1 : s;
                const float phi_o = first ? ph[k] : ph[k + 1], phi_t = first ? ph[k + 1] : ph[k];
                const float e_coul = (phi_t - a.k10) - phi_o;
                const float e_app = ((alpha_r * V_r) * (float)(t - o)) / (float)L;
                const float ea = a.ea ? reinterpret_cast<const float *>(a.ea)[dv.off + (int64_t)r * L + o]
                                      : (float)a.ea_scalar;
                if (decide_hop<float>(e_app + e_coul, ea, word_of(blk, i), beta_r, c0_r, a.log, d, H, n, r, s)) {
                    hopped |= 1u << i;
                    atomicAdd(&tally[0], t < o ? 1 : -1);
                    const int qo = (10 * o) / L, qt = (10 * t) / L;
                    if (qo != qt) {
                        atomicAdd(&tally[1 + qo], -1);
                        atomicAdd(&tally[1 + qt], 1);
                    }
                }
            }
        }
    }
    last_hop[tid] = hopped;
    __syncthreads();
    if (tid <= kDeciles && tally[tid] != 0) {  // all rails of the workgroup belong to device d
        const int64_t base = (n - a.ctl.tally_base) * a.n_devices + d;
        atomicAdd(tid == 0 ? &a.tally_net[base] : &a.tally_dec[base * kDeciles + tid - 1], tally[tid]);
    }
    if (!active) return;
    // flip both sites of every bond that moved; bond i starts at 8b + H + 2i
    uint64_t w = (uint64_t)v.x | ((uint64_t)v.y << 32);
    for (int i = 0; i < 4; ++i)
        if ((hopped >> i) & 1u) {
            const int k = H + 2 * i;
            w ^= (uint64_t)1 << (8 * k);
            if (k + 1 < 8) w ^= (uint64_t)1 << (8 * (k + 1));
        }
    if (H == 1 && b > 0 && ((last_hop[tid - 1] >> 3) & 1u)) w ^= 1ull;  // previous block's bond (8b-1, 8b)
    // the state is updated in place: every read of it precedes the barrier
    // above, and a workgroup's rails are its own; only changed blocks are written
    if (w != ((uint64_t)v.x | ((uint64_t)v.y << 32))) *reinterpret_cast<uint2 *>(dst) = make_uint2((uint32_t)w, (uint32_t)(w >> 32));
}

hipError_t launch_dense_decide(const HopArgs &a, int pitch, hipStream_t st) {
    const int bpr = pitch / 8;
    const dim3 grid(a.n_dtiles), block((256 / bpr) * bpr);
    if (a.h == 0) hipLaunchKernelGGL(dense_decide<0>, grid, block, 0, st, a, bpr);
    else hipLaunchKernelGGL(dense_decide<1>, grid, block, 0, st, a, bpr);
    return hipGetLastError();
}

hipError_t launch_dense_phi(const DenseArgs &a, hipStream_t st) {
    const size_t lds = (size_t)(kDenseRails + 2 * a.rail_range) * (a.nb * 32 + 8);
    const dim3 grid(a.n_tiles, (a.nb + 7) / 8), block(kDenseBlock);
    hipLaunchKernelGGL(dense_phi, grid, block, lds, st, a);
    return hipGetLastError();
}

hipError_t set_dense_lds_limit(size_t lds_bytes) {
    return hipFuncSetAttribute((const void *)dense_phi, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

}  // namespace kmc
