// Boundary bonds of open electrodes (kmc_set_electrodes in include/kmc.h).
//
// With open electrodes each rail end is one more bond of the checkerboard:
// bond (-1, 0) to the grounded reservoir (odd, half-step 1) and bond (L-1, L)
// to the biased reservoir (half-step (L-1) mod 2).  A reservoir ion has the
// energy mu plus its bias energy at the virtual site and no Coulomb
// interaction.  With o, t the transfer's origin and target (virtual sites
// included) and x the boundary site,
//     dE = (alpha V (t - o) / L + s phi(x)) - s mu,   s = +1 injection, -1 extraction,
// phi(x) the Coulomb potential of the other ions of the snapshot at x (the
// hop's window and kernel), and the rate law of any hop with the electrode's
// barrier: p = min(nu0 dt exp(-(ea + dE/2)/kT), 1), accepted when u < p.
// The word is Philox4x32-10 at counter (0, r, n, 16 d + 2*3 + h), word 0 for
// the grounded side and 1 for the biased side.  This is an extension of the
// paper's model (blocking electrodes, a fixed ion count per rail) in the
// direction its conclusion invites: a new mechanism through altered
// probabilities at a few positions.
//
// One thread per rail end; the interior kernel of the half-step has already
// written the new state, in which the boundary site still holds its
// snapshot value (its interior bond belongs to the other parity).
#include "kmc_electrode.h"

#include "kmc_device.h"

namespace kmc {

namespace {

template <typename Real, int H>
__global__ __launch_bounds__(256) void electrode_bonds(ElectrodeArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 2 * a.rails_total) return;
    const int64_t grow = gid >> 1;
    const int side = (int)(gid & 1);
    const int d = a.rail_dev[grow], r = a.rail_idx[grow];
    const Electrode el = a.el[d];
    if (!el.open) return;
    const DevInfo &dv = a.devs[d];
    const int L = dv.sites, R = dv.rails, pitch = dv.pitch;
    if (side == 0 ? H != 1 : ((L - 1) & 1) != H) return;
    const int x = side == 0 ? 0 : L - 1;
    const int res = side == 0 ? -1 : L;
    const int8_t *snap = a.occ_in + dv.off_pad;
    const uint32_t byte = (uint32_t)(uint8_t)snap[(int64_t)r * pitch + x];
    const bool inject = (byte & 1u) == 0u;
    const int o = inject ? res : x, t = inject ? x : res;
    const double V = protocol_voltage(a.knot_t + d * kMaxKnots, a.knot_v + d * kMaxKnots, dv.n_knots,
                                      (double)(a.n - dv.n_set) * a.dt);
    // phi(x): the window terms rail by rail in the neighbour order, sites in
    // increasing order
    const Real *kt = std::is_same<Real, double>::value ? reinterpret_cast<const Real *>(a.ktab64)
                                                       : reinterpret_cast<const Real *>(a.ktab32);
    const int cs = a.cutoff + 1;
    int lo = x - a.cutoff, hi = x + a.cutoff;
    lo = lo < 0 ? 0 : lo;
    hi = hi > L - 1 ? L - 1 : hi;
    Real phi = (Real)0;
    for (int k = 0; k < dv.n_nbr; ++k) {
        const int off = dv.nbr_off[k];
        const int rr = ((r + off) % R + R) % R;
        const int8_t *row = snap + (int64_t)rr * pitch;
        const Real *ktr = kt + dv.nbr_dist[k] * cs;
        for (int j = lo; j <= hi; ++j) {
            if (off == 0 && j == x) continue;
            if (row[j] & 1) phi += ktr[j < x ? x - j : j - x];
        }
    }
    const Real alpha_r = (Real)a.alpha, V_r = (Real)V;
    const Real e_app = ((alpha_r * V_r) * (Real)(t - o)) / (Real)L;
    const Real sgn = inject ? (Real)1 : (Real)-1;
    const Real mu = (Real)(side == 0 ? el.mu_ground : el.mu_bias);
    const Real dE = (e_app + sgn * phi) - sgn * mu;
    const Real ea = (Real)(side == 0 ? el.ea_ground : el.ea_bias);
    const uint4 blk = philox4x32_10(0u, (uint32_t)r, (uint32_t)a.n, ((uint32_t)d << 4) | (3u << 1) | (uint32_t)H,
                                    a.key0, a.key1);
    const uint32_t w = side == 0 ? blk.x : blk.y;
    if (!decide_hop<Real>(dE, ea, w, (Real)a.beta, (Real)a.c0, a.log, d, H, a.n, r, side == 0 ? -1 : L - 1))
        return;
    a.occ_out[dv.off_pad + (int64_t)r * pitch + x] = (int8_t)(byte ^ 1u);
    const int64_t base = a.tally_row * a.n_devices + d;
    // toward site 0's side: extraction at the grounded end, injection at the biased end
    atomicAdd(&a.tally_net[base], (side == 0) != inject ? 1 : -1);
    atomicAdd(&a.tally_dec[base * kDeciles + (10 * x) / L], inject ? 1 : -1);
}

}  // namespace

hipError_t launch_electrodes(const ElectrodeArgs &a, bool fp64, hipStream_t st) {
    const int64_t threads = 2 * a.rails_total;
    const dim3 grid((unsigned)((threads + 255) / 256)), block(256);
    if (fp64) {
        if (a.h == 0) hipLaunchKernelGGL((electrode_bonds<double, 0>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((electrode_bonds<double, 1>), grid, block, 0, st, a);
    } else {
        if (a.h == 0) hipLaunchKernelGGL((electrode_bonds<float, 0>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((electrode_bonds<float, 1>), grid, block, 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace kmc
