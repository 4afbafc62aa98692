// Device-side helpers shared by the HIP kernels of the hop step.
#pragma once
#include <math.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "kmc_internal.h"

namespace kmc {

// ------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  gfx950 has a
// three-input bitwise op; truth table 0x96 is a ^ b ^ c.
// ------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox4x32_10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * x0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t y0 = xor3((uint32_t)(m1 >> 32), x1, k0);
        const uint32_t y2 = xor3((uint32_t)(m0 >> 32), x3, k1);
        x1 = (uint32_t)m1;
        x3 = (uint32_t)m0;
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(x0, x1, x2, x3);
}

__device__ __forceinline__ uint32_t word_of(const uint4 &b, int i) {
    return i == 0 ? b.x : (i == 1 ? b.y : (i == 2 ? b.z : b.w));
}

// Piecewise-linear bias, right-continuous at repeated knot times, constant
// outside the knot range.  Binary64.
__device__ inline double protocol_voltage(const double *t, const double *v, int nk, double t_rel) {
    if (nk <= 0) return 0.0;
    if (t_rel < t[0]) return v[0];
    int k = 0;
    for (int i = 0; i < nk; ++i)
        if (t[i] <= t_rel) k = i;
    if (k == nk - 1) return v[nk - 1];
    const double num = (v[k + 1] - v[k]) * (t_rel - t[k]);
    return v[k] + num / (t[k + 1] - t[k]);
}

template <typename Real>
__device__ __forceinline__ Real exp_r(Real x);
template <>
__device__ __forceinline__ double exp_r<double>(double x) { return exp(x); }
template <>
__device__ __forceinline__ float exp_r<float>(float x) { return expf(x); }

template <typename Real>
__device__ __forceinline__ Real uniform_of(uint32_t w);
template <>
__device__ __forceinline__ double uniform_of<double>(uint32_t w) { return (double)w * 0x1p-32; }
template <>
__device__ __forceinline__ float uniform_of<float>(uint32_t w) { return (float)w * 0x1p-32f; }

// occupancy bits (bit 0 of each byte) of a 16-byte chunk, site k -> bit k
__device__ __forceinline__ uint32_t occ_bits(const uint4 &v) {
    uint32_t bits = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) bits |= (((word_of(v, b) & 0x01010101u) * 0x01020408u) >> 24 & 0xFu) << (4 * b);
    return bits;
}

__device__ __forceinline__ uint32_t word_of8(const uint4 &A, const uint4 &B, int i) {
    return i < 4 ? word_of(A, i) : word_of(B, i - 4);
}

__device__ __forceinline__ void flip_byte(uint4 &v, int b) {
    const uint32_t m = 1u << (8 * (b & 3));
    const int w = b >> 2;
    if (w == 0) v.x ^= m;
    else if (w == 1) v.y ^= m;
    else if (w == 2) v.z ^= m;
    else v.w ^= m;
}

__device__ __forceinline__ int tile_of_block(int bid, int n_tiles) {
    // Consecutive tiles (neighbouring rails) on the same XCD: the dispatcher
    // deals workgroups round-robin over the 8 XCDs.
    const int full = (n_tiles / 8) * 8;
    return bid < full ? (bid % 8) * (n_tiles / 8) + bid / 8 : bid;
}

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also waits
// for every global load and store the wavefront has in flight; inside the
// persistent loop that would make every barrier wait for the edge-rail
// publications and the neighbour probes.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Arrhenius hop probability with the half-energy barrier shift (paper main
// text Eq. hop_rate and Eq. 2), p = min(nu0 dt exp(-beta (Ea + dE/2)), 1);
// accept when u < p; draws with |u - p| < 1e-6 are appended to the log.
template <typename Real>
__device__ inline bool decide_hop(Real dE, Real ea, uint32_t w, Real beta, Real c0, const HopArgs::LogBuf &log,
                                  int d, int h, int64_t n, int rail, int s) {
    Real p = c0 * exp_r<Real>(-beta * (ea + (Real)0.5 * dE));
    p = p < (Real)1 ? p : (Real)1;
    const Real u = uniform_of<Real>(w);
    const Real gap = u - p;
    if ((gap < 0 ? -gap : gap) < (Real)1e-6) {
        const int64_t k = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(log.count), 1ull);
        if (k < log.cap) {
            unsigned char *e = reinterpret_cast<unsigned char *>(log.entries) + 40 * k;
            *reinterpret_cast<int32_t *>(e + 0) = d;
            *reinterpret_cast<int32_t *>(e + 4) = h;
            *reinterpret_cast<int64_t *>(e + 8) = n;
            *reinterpret_cast<int32_t *>(e + 16) = rail;
            *reinterpret_cast<int32_t *>(e + 20) = s;
            *reinterpret_cast<double *>(e + 24) = (double)u;
            *reinterpret_cast<double *>(e + 32) = (double)p;
        }
    }
    return u < p;
}

// Appends an accepted hop to the recording (a no-op when nothing is recorded
// or the step lies outside the recorded run); dir 0 when the ion at s moves up.
__device__ inline void record_hop(const HopRecord &rec, int d, int h, int64_t n, int rail, int s, int dir) {
    if (!rec.buf) return;
    const int64_t hs = 2 * (n - rec.n0) + h;
    if (hs < 0 || hs >= rec.n_hs) return;
    const int64_t k = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(rec.count + hs), 1ull);
    if (k < rec.cap) rec.buf[hs * rec.cap + k] = make_uint4((uint32_t)d, (uint32_t)rail, (uint32_t)s, (uint32_t)dir);
}

// Inclusive Philox-word threshold of barrier class q: every configuration has
// dE >= -(|alpha V|/L + coul_bound) and every class-q site a barrier >=
// ea_min + q ea_step, so p <= pb.  pb is widened by 1e-3 relative and by twice
// the 1e-6 logging window, so a word above the threshold can neither be
// accepted nor logged.
__device__ inline uint32_t class_threshold(double c0, double beta, double alpha, double V, int L, double ea_min,
                                           double ea_step, double coul_bound, int q) {
    const double field = fabs(alpha * V) / (double)L;
    const double ea_lb = ea_min + (double)q * ea_step;
    const double pb = c0 * exp(-beta * (ea_lb - 0.5 * (field + coul_bound))) * (1.0 + 1e-3) + 2e-6;
    return pb >= 1.0 ? 0xFFFFFFFFu : (uint32_t)(ceil(pb * 4294967296.0) - 1.0);
}

// Inclusive threshold of a Philox word for a class with static factor
// A = exp(-beta ea_lb), widened like class_threshold; g = exp(beta (|alpha V|/L
// + coul_bound) / 2) carries the step's field and the Coulomb bound.
__device__ __forceinline__ uint32_t threshold_of(double c0, double A, double g) {
    const double pb = c0 * A * g * (1.0 + 1e-3) + 2e-6;
    return pb >= 1.0 ? 0xFFFFFFFFu : (uint32_t)(ceil(pb * 4294967296.0) - 1.0);
}


// The end of a tally chunk done by one wavefront (the tail of the wave
// kernel): for the series (device d in [f.d0, f.d1), decile q or net hops) of
// f.steps steps, the per-step deltas become the caller's rows (absolute decile
// counts, net hops per step), the running totals advance and the chunk
// buffers are cleared.  Lane l takes segment l and l + 64 of the series cut
// into pieces of g steps; needs at most 128 segments (`sums` holds 128
// values in LDS).  The chunk buffers are read and cleared with device-scope
// atomics (the launch's tiles added to them with device-scope atomics).
__device__ inline void finish_tallies_wave(const FinishArgs &f, int lane, int64_t *sums) {
    const int S = (f.d1 - f.d0) * (kDeciles + 1);
    const int steps = f.steps, D = f.n_devices;
    int g = (int)(((int64_t)S * steps + 63) / 64);
    g = g < 1 ? 1 : (g > steps ? steps : g);
    const int per = (steps + g - 1) / g;
    const int n_seg = S * per;
    const int64_t row0 = f.ctl.tally_base - f.ctl.call_base;
    auto slot = [&](int q, int d, int k) -> int32_t * {
        return q < kDeciles ? &f.tally_dec[((int64_t)k * D + d) * kDeciles + q] : &f.tally_net[(int64_t)k * D + d];
    };
    // a segment's values are read eight at a time (their loads in flight
    // together); segments of at most eight steps keep them for the second pass
    constexpr int kHeld = 8;
    int64_t sum_r[2] = {0, 0}, carry_r[2] = {0, 0};
    int32_t held[2][kHeld];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int seg = lane + 64 * r;
        if (seg < n_seg) {
            const int s = seg / per, part = seg - s * per;
            const int d = f.d0 + s / (kDeciles + 1), q = s % (kDeciles + 1);
            const int k0 = part * g, k1 = k0 + g < steps ? k0 + g : steps;
            int64_t sum = 0;
            for (int kb = k0; kb < k1; kb += kHeld) {
                int32_t x[kHeld];
#pragma unroll
                for (int u = 0; u < kHeld; ++u)
                    x[u] = kb + u < k1 ? __hip_atomic_load(slot(q, d, kb + u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
#pragma unroll
                for (int u = 0; u < kHeld; ++u) {
                    sum += x[u];
                    held[r][u] = x[u];
                }
            }
            sum_r[r] = sum;
            carry_r[r] = q < kDeciles ? f.dec_run[d * kDeciles + q] : 0;
            sums[seg] = sum;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int seg = lane + 64 * r;
        if (seg < n_seg) {
            const int s = seg / per, part = seg - s * per;
            const int d = f.d0 + s / (kDeciles + 1), q = s % (kDeciles + 1);
            const int k0 = part * g, k1 = k0 + g < steps ? k0 + g : steps;
            int64_t before = 0;
            for (int j = s * per; j < seg; ++j) before += sums[j];
            int64_t run = carry_r[r] + before;
            for (int k = k0; k < k1; ++k) {
                int32_t *p = slot(q, d, k);
                int32_t x = 0;
                if (k1 - k0 <= kHeld) {
#pragma unroll
                    for (int u = 0; u < kHeld; ++u)
                        if (u == k - k0) x = held[r][u];
                } else {
                    x = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                __hip_atomic_store(p, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (q == kDeciles) {
                    if (f.ctl.net_out) f.ctl.net_out[(row0 + k) * D + d] = x;
                } else {
                    run += x;
                    if (f.ctl.dec_out) f.ctl.dec_out[((row0 + k) * D + d) * kDeciles + q] = (int32_t)run;
                }
            }
            if (part == per - 1) {
                if (q < kDeciles) f.dec_run[d * kDeciles + q] = run;
                else f.net_total[d] += before + sum_r[r];
            }
        }
    }
}

}  // namespace kmc
