// C ABI of the rail-KMC hop-step library (declared in include/kmc.h).
//
// Host side: parameter validation, workspace layout, the binary64 interaction
// table, the prefilter bound, the tile decomposition and the launch sequence.
// Every step of the hop path itself runs in the HIP kernels of kmc_kernels.hip.
#include "../../include/kmc.h"
#include "../../include/kmc_calib.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kmc_internal.h"
#include "kmc_electrode.h"
#include "kmc_phifix.h"

namespace kmc {
hipError_t launch_hop(const HopArgs &a, size_t lds_bytes, bool fp64, hipStream_t st);
hipError_t launch_score(const HopArgs &a, size_t lds_bytes, bool fp64, hipStream_t st);
hipError_t launch_replay_stream(const HopArgs &a, bool fp64, hipStream_t st);
hipError_t launch_replay_logged(const HopArgs &a, bool fp64, hipStream_t st);
hipError_t launch_compare_bytes(const int8_t *x, const int8_t *y, int64_t n, int64_t *flag, hipStream_t st);
hipError_t launch_pack_occ_bits(const int8_t *src, uint8_t *dst, int64_t n_pad, hipStream_t st);
hipError_t launch_unpack_occ_bits(const uint8_t *src, int8_t *dst, int64_t n_pad, hipStream_t st);
int replay_run_rails(int pitch);
hipError_t set_hop_lds_limit(size_t lds_bytes, size_t score_lds_bytes);
hipError_t launch_import(const int8_t *src, int8_t *dst, const DevInfo *devs, int n_dev, int64_t total_pad,
                         const void *ea, bool fp64, hipStream_t st);
hipError_t launch_export(const int8_t *src, int8_t *dst, const DevInfo *devs, int n_dev, int64_t total,
                         hipStream_t st);
hipError_t launch_place(int8_t *occ_pad, const DevInfo *devs, const int32_t *rail_dev, const int32_t *rail_idx,
                        const int32_t *n_ions, int n_rails_total, uint32_t key0, uint32_t key1, hipStream_t st);
hipError_t launch_barrier_range(const void *ea, bool fp64, DevInfo *devs, int n_dev,
                                unsigned long long *scratch, hipStream_t st);
hipError_t launch_count_deciles(const int8_t *occ_pad, const DevInfo *devs, int n_dev, int64_t *dec_run,
                                hipStream_t st);
hipError_t launch_set_protocol(double *knot_t, double *knot_v, DevInfo *devs, int d0, int d1, int nk,
                               int64_t n_set, const double *t, const double *v, hipStream_t st);
hipError_t launch_finish_chunk(const FinishArgs &f, hipStream_t st);
hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t st);
hipError_t launch_persistent(const PArgs &a, int block, size_t lds, bool fp64, hipStream_t st);
hipError_t persistent_capacity(int block, size_t lds, bool fp64, int *blocks_per_cu);
hipError_t launch_zero_i64(int64_t *p, int64_t n, hipStream_t st);
hipError_t launch_wave(const PArgs &a, int spl, size_t lds, bool fp64, hipStream_t st);
hipError_t wave_capacity(int spl, size_t lds, bool fp64, int *blocks_per_cu);
size_t wave_lds_bytes(int spl, int n_kt, bool fp64);
int wave_band_words(int spl);
hipError_t launch_copy_bytes(const void *src, void *dst, size_t bytes, hipStream_t st);
hipError_t launch_replay_ec_full(const PhiArgs &a, bool fp64, hipStream_t st);
hipError_t launch_replay_ec_update(const PhiArgs &a, bool fp64, hipStream_t st, int64_t hops_known = -1);
hipError_t launch_dense_phi(const DenseArgs &a, hipStream_t st);
hipError_t launch_dense_decide(const HopArgs &a, int pitch, hipStream_t st);
hipError_t set_dense_lds_limit(size_t lds_bytes);
}  // namespace kmc

using namespace kmc;

namespace {

thread_local std::string g_last_error;

kmc_status fail(kmc_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

constexpr int64_t kLogCap = 65536;
constexpr int64_t kMaxPTiles = 2048;
constexpr int kPTileSites = 4096;  // default padded sites per persistent tile
constexpr int kStepWin = 128;      // per-step table window of the persistent kernel
constexpr int64_t kMaxWaveTiles = 8192;  // wave kernel: tiles per launch (publication memory)
constexpr double kElementaryCharge = 1.602176634e-19;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Layout {
    size_t occ_a, occ_b, devs, tiles, knot_t, knot_v, ktab64, ktab32, ctl, tally_net, tally_dec, dec_run,
        net_total, log_count, log_entries, scratch, rail_dev, rail_idx, n_ions, ptiles, pub, status,
        rp_a, rp_b, score_log, rec, hops, hop_ctl, phi, ktiles, dtiles, ctiles, ticket, phifix, kfix, electrodes, rtiles, total;
    int64_t max_ptiles, pub_stride;  // persistent kernel: tiles per launch (ring slots), words per ring
    int64_t max_wtiles, wpub_stride;  // wave kernel: tiles per launch, publication words per tile
    size_t wtiles;                    // wave tiling (PTile array)
    int max_pitch;
    int64_t total_sites, total_pad, rails_total;
    int cut;     // interaction table cutoff actually stored
    int64_t hop_cap;  // score replay: entries of the accepted-hop list
    int dense_nb;  // dense potential: 32-site blocks per rail (0 when not used)
};

// 64-bit words of the publication region (shared by the two persistent kernels)
int64_t pub_words(const Layout &L) { return std::max(L.pub_stride * L.max_ptiles, L.wpub_stride * L.max_wtiles); }

bool is_finite(double x) { return std::isfinite(x); }

kmc_status validate(const kmc_params *p) {
    if (!p) return fail(KMC_EINVAL, "params is NULL");
    if (p->n_devices < 1 || p->n_devices > (1 << 24)) return fail(KMC_EINVAL, "n_devices must be in [1, 2^24]");
    if (!p->rails || !p->sites) return fail(KMC_EINVAL, "rails/sites arrays are NULL");
    int64_t rails_total = 0;
    for (int d = 0; d < p->n_devices; ++d) {
        if (p->rails[d] < 1) return fail(KMC_EINVAL, "device " + std::to_string(d) + ": rails < 1");
        if (p->sites[d] < 2) return fail(KMC_EINVAL, "device " + std::to_string(d) + ": sites < 2");
        if (p->sites[d] > kMaxSites)
            return fail(KMC_EUNSUPPORTED, "device " + std::to_string(d) + ": sites > 4096 per rail");
        rails_total += p->rails[d];
    }
    if (rails_total > (int64_t)1 << 30) return fail(KMC_EUNSUPPORTED, "more than 2^30 rails in total");
    if (!is_finite(p->nu0_hz) || p->nu0_hz < 0) return fail(KMC_EINVAL, "nu0_hz must be finite and >= 0");
    if (!is_finite(p->ea_ev)) return fail(KMC_EINVAL, "ea_ev must be finite");
    if (!is_finite(p->kT_ev) || p->kT_ev <= 0) return fail(KMC_EINVAL, "kT_ev must be > 0");
    if (!is_finite(p->dt_s) || p->dt_s <= 0) return fail(KMC_EINVAL, "dt_s must be > 0");
    if (!is_finite(p->field_coupling)) return fail(KMC_EINVAL, "field_coupling must be finite");
    if (!is_finite(p->coulomb_kappa_v)) return fail(KMC_EINVAL, "coulomb_kappa_v must be finite");
    if (!is_finite(p->screening_sites) || p->screening_sites < 0)
        return fail(KMC_EINVAL, "screening_sites must be >= 0");
    if (p->cutoff_sites < 0) return fail(KMC_EINVAL, "cutoff_sites must be >= 0");
    if (p->rail_range < 0 || p->rail_range > kMaxRailRange)
        return fail(KMC_EUNSUPPORTED, "rail_range must be in [0, 4]");
    if (p->precision != KMC_FP64 && p->precision != KMC_FP32 && p->precision != KMC_BF16X2 &&
        p->precision != KMC_PHI_FIXED)
        return fail(KMC_EINVAL, "unknown precision");
    if (p->precision == KMC_PHI_FIXED)
        for (int d = 0; d < p->n_devices; ++d)
            if (p->sites[d] > kPhiMaxSites) return fail(KMC_EUNSUPPORTED, "KMC_PHI_FIXED supports up to 2048 sites");
    if (p->precision == KMC_BF16X2) {
        for (int d = 1; d < p->n_devices; ++d)
            if (p->sites[d] != p->sites[0])
                return fail(KMC_EUNSUPPORTED, "KMC_BF16X2 needs the same number of sites on every device");
        if (p->sites[0] > kDenseMaxSites) return fail(KMC_EUNSUPPORTED, "KMC_BF16X2 supports up to 1024 sites");
    }
    return KMC_OK;
}

// Wave-kernel geometry of a device: lanes per rail and the most rails one
// wavefront holds (0: the rails do not fit).
struct WaveGeom {
    int lpr, nr_max;
};
WaveGeom wave_geom(int pitch, int spl) {
    const int lpr = (pitch + spl - 1) / spl;
    return WaveGeom{lpr, 64 / lpr};
}

Layout layout_for(const kmc_params *p) {
    Layout L{};
    int64_t sites = 0, pad = 0, rails = 0;
    int max_l = 0;
    for (int d = 0; d < p->n_devices; ++d) {
        const int pitch = (p->sites[d] + kChunkSites - 1) / kChunkSites * kChunkSites;
        sites += (int64_t)p->rails[d] * p->sites[d];
        pad += (int64_t)p->rails[d] * pitch;
        rails += p->rails[d];
        max_l = std::max(max_l, p->sites[d]);
    }
    L.total_sites = sites;
    L.total_pad = pad;
    L.rails_total = rails;
    L.cut = std::min(p->cutoff_sites, max_l);
    const int D = p->n_devices;
    const int m = p->rail_range;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    L.occ_a = take((size_t)pad);
    L.occ_b = take((size_t)pad);
    L.devs = take(sizeof(DevInfo) * D);
    L.tiles = take(sizeof(Tile) * (size_t)rails);
    L.knot_t = take(sizeof(double) * kMaxKnots * D);
    L.knot_v = take(sizeof(double) * kMaxKnots * D);
    L.ktab64 = take(sizeof(double) * (m + 1) * (L.cut + 1));
    L.ktab32 = take(sizeof(float) * (m + 1) * (L.cut + 1));
    L.tally_net = take(sizeof(int32_t) * kTallySteps * D);
    L.tally_dec = take(sizeof(int32_t) * kTallySteps * D * kDeciles);
    L.dec_run = take(sizeof(int64_t) * D * kDeciles);
    L.net_total = take(sizeof(int64_t) * D);
    L.log_count = take(sizeof(int64_t));
    L.log_entries = take(sizeof(kmc_log_entry) * kLogCap);
    L.scratch = take(sizeof(unsigned long long) * 2 * D);
    L.rail_dev = take(sizeof(int32_t) * (size_t)rails);
    L.rail_idx = take(sizeof(int32_t) * (size_t)rails);
    L.n_ions = take(sizeof(int32_t) * D);
    // persistent kernels: tiles and the edge-rail publications
    int max_pitch = 0;
    for (int d = 0; d < D; ++d) max_pitch = std::max(max_pitch, (p->sites[d] + kChunkSites - 1) / kChunkSites * kChunkSites);
    L.max_pitch = max_pitch;
    L.pub_stride = (int64_t)kPubSlots * 2 * std::max(m, 1) * ((max_pitch + 31) / 32);
    // tiles of one launch: at most twice the default tiling's tile count (room
    // for the autotuner's smaller tiles) or 64, and at most 1.25 GiB of publications
    int64_t default_tiles = 0;
    for (int d = 0; d < D; ++d) {
        const int pitch = (p->sites[d] + kChunkSites - 1) / kChunkSites * kChunkSites;
        default_tiles += std::max(1, p->rails[d] / std::max(std::max(m, 1), kPTileSites / pitch));
    }
    const int64_t pub_cap = std::max<int64_t>(1, ((int64_t)5 << 28) / (8 * L.pub_stride));
    L.max_ptiles = std::min<int64_t>(std::min<int64_t>(std::min<int64_t>(kMaxPTiles, rails), pub_cap),
                                     std::max<int64_t>(2 * default_tiles, 64));
    L.ptiles = take(sizeof(PTile) * (size_t)rails);  // every tile is at least one rail
    // wave kernel: per tile one word per state of a launch plus a ring of
    // edge-rail snapshots; tiles of one launch bounded by kMaxWaveTiles
    {
        int64_t tiles = 0, slot = 1;
        for (int spl : {16, 32}) {
            int64_t t = 0;
            for (int d = 0; d < D; ++d) {
                const int pitch = (p->sites[d] + kChunkSites - 1) / kChunkSites * kChunkSites;
                const WaveGeom g = wave_geom(pitch, spl);
                if (g.nr_max < 1) {
                    t = 0;
                    break;
                }
                t += (p->rails[d] + g.nr_max - 1) / g.nr_max;
                slot = std::max<int64_t>(slot, (int64_t)std::min(g.nr_max, 2 * std::max(m, 1)) * ((pitch + 31) / 32));
            }
            tiles = std::max(tiles, t);
        }
        L.max_wtiles = std::min<int64_t>(std::max<int64_t>(tiles, 1), kMaxWaveTiles);
        L.wpub_stride = kPubSlots + (int64_t)kSnapSlots * slot;
    }
    L.pub = take(sizeof(uint64_t) *
                 (size_t)std::max(L.pub_stride * L.max_ptiles, L.wpub_stride * L.max_wtiles));
    L.wtiles = take(sizeof(PTile) * (size_t)rails);  // every wave tile is at least one rail
    L.status = take(sizeof(int32_t) * 4);
    L.ticket = take(sizeof(uint32_t) * kTicketWords);  // wave kernel: tiles that ended the launch
    L.electrodes = take(sizeof(Electrode) * D);       // open-electrode reservoirs per device
    // score replay: its own pair of state planes, a discarded event count, the
    // Coulomb part of every bond's energy change (path precision) and the list
    // of a half-step's accepted hops (a longer list falls back to recomputing
    // every bond)
    L.rp_a = take((size_t)pad);
    L.rp_b = take((size_t)pad);
    L.score_log = take(sizeof(int64_t));
    L.hop_cap = std::min<int64_t>(std::max<int64_t>(L.total_sites / 64, 4096), (int64_t)1 << 24);
    if (p->precision != KMC_BF16X2) {
        const bool f64 = p->precision == KMC_FP64 || p->precision == KMC_PHI_FIXED;
        // (16 values of padding: the streaming replay reads four parts per block
        // and ignores those beyond a rail's end)
        L.rec = take((f64 ? sizeof(double) : sizeof(float)) * ((size_t)L.total_sites + 16));
        L.hops = take(sizeof(uint4) * (size_t)L.hop_cap);
        L.hop_ctl = take(sizeof(int64_t) * 2);
        L.rtiles = take(sizeof(Tile) * (size_t)rails);  // runs of the streaming replay
    }
    if (p->precision == KMC_BF16X2) {
        // potential of every site (rows padded to a multiple of 128 sites), the
        // distinct 32 x 32 Toeplitz blocks of the kernel as MFMA fragments, tiles
        const int lp = (p->sites[0] + 127) / 128 * 128;
        L.dense_nb = lp / 32;
        L.phi = take(sizeof(float) * (size_t)rails * lp);
        L.ktiles = take((size_t)16 * 256 * (m + 1) * (2 * L.dense_nb - 1));
        L.dtiles = take(sizeof(Tile) * (size_t)rails);
        L.ctiles = take(sizeof(Tile) * (size_t)rails);
    }
    if (p->precision == KMC_PHI_FIXED) {
        // the fixed-point potential of every padded site, the kernel table in
        // fixed point and the decision tiles
        L.phifix = take(sizeof(int64_t) * (size_t)pad);
        L.kfix = take(sizeof(int64_t) * (m + 1) * (L.cut + 1));
        L.ctiles = take(sizeof(Tile) * (size_t)rails);
    }
    L.total = off;
    return L;
}

// Interaction kernel in binary64: kappa*exp(-d/lambda)/d (kappa/d unscreened).
double kernel64(const kmc_params *p, int ds, int dr) {
    if (ds == 0 && dr == 0) return 0.0;
    if (std::abs(ds) > p->cutoff_sites || dr > p->rail_range) return 0.0;
    const double d = std::sqrt((double)ds * ds + (double)dr * dr);
    if (p->screening_sites > 0) return p->coulomb_kappa_v * std::exp(-d / p->screening_sites) / d;
    return p->coulomb_kappa_v / d;
}

}  // namespace

struct kmc_ctx {
    kmc_params p{};
    std::vector<int32_t> rails, sites;
    std::vector<DevInfo> devs;
    std::vector<Tile> tiles;
    Layout lay{};
    unsigned char *ws = nullptr;
    int8_t *occ_user = nullptr;
    const void *ea = nullptr;
    hipStream_t stream = nullptr;
    bool poisoned = false;
    bool fp64 = false;
    bool dense = false;                // KMC_BF16X2: Coulomb term from the MFMA potential
    std::vector<Tile> dtiles;          // dense-potential tiles (<= kDenseRails rails)
    std::vector<Tile> ctiles;          // dense decision tiles (whole rails, one 256-thread workgroup)
    int64_t n = 0;            // host mirror of the step counter
    int64_t steps_run = 0;    // steps since init (for the mean current)
    size_t hop_lds = 0;
    size_t score_lds = 0;              // hop_lds plus the occupancy bit rows
    int8_t *cur = nullptr, *nxt = nullptr;
    int tile_sites = 0;                // target padded sites per tile (0 = default)
    int group_limit = 0;               // max tiles per persistent launch (0 = what fits)
    int spin_limit = 1 << 20;          // polls before a neighbour wait is declared hung
    std::vector<PTile> ptiles;         // persistent tiling (prev/next relative to the tile's group)
    std::vector<std::pair<int, int>> pgroups;  // (first tile, tiles): devices run together in one launch
    int p_block = 0;
    size_t p_lds = 0;
    bool p_ok = false;                 // persistent tiling fits co-resident on this GPU
    std::vector<PTile> wtiles;         // wave tiling (prev/next relative to the tile's group)
    std::vector<std::pair<int, int>> wgroups;
    int w_spl = 0;                     // sites per lane of the wave tiling
    size_t w_lds = 0;
    bool w_ok = false;                 // wave tiling fits co-resident on this GPU
    int mode = 0;                      // KMC_LAUNCH_AUTO / _HALF_STEP / _PERSISTENT
    uint64_t epoch = 0;
    float k10 = 0.0f;                  // K(1, 0) rounded to binary32
    double k01 = 0.0;                  // K(1, 0) in binary64 (score replay, fixed-point decisions)
    bool phifix = false;               // KMC_PHI_FIXED: Coulomb term from the fixed-point potential
    int frac_bits = 0;                 // its units: 2^-frac_bits V
    int64_t k10fix = 0;                // K(1, 0) in those units
    std::vector<Electrode> el;         // reservoirs per device (host copy of the workspace's)
    std::vector<Tile> rtiles;          // runs of rails of the streaming replay (empty: the tile replay)
    bool any_open = false;             // some device has open electrodes: half-step launches only
    // recording of accepted hops for the score replay (kmc_record_hops), in
    // the caller's buffer: per half-step counts, then a flag for the replay's
    // check of its start state; the state at the recording's first step; the
    // lists
    bool rec_on = false;
    int64_t *rec_count = nullptr;      // [rec_n_hs + 1]
    int8_t *rec_occ = nullptr;         // [total sites], caller layout
    uint4 *rec_buf = nullptr;          // [rec_n_hs][rec_cap]
    int64_t rec_cap = 0, rec_n0 = 0, rec_n_hs = 0;

    template <typename T>
    T *at(size_t off) { return reinterpret_cast<T *>(ws + off); }
};

namespace {

kmc_status hip_check(kmc_ctx *c, hipError_t e, const char *what) {
    if (e == hipSuccess) return KMC_OK;
    if (c) c->poisoned = true;
    return fail(KMC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define KMC_HIP(c, expr)                                           \
    do {                                                           \
        kmc_status s_ = hip_check((c), (expr), #expr);             \
        if (s_ != KMC_OK) return s_;                               \
    } while (0)

kmc_status usable(kmc_ctx *c) {
    if (!c) return fail(KMC_EINVAL, "context is NULL");
    if (c->poisoned) return fail(KMC_ESTATE, "context poisoned by an earlier HIP error");
    return KMC_OK;
}

// Distinct rails within rail_range of a rail on a ring of R rails, visited in
// the order 0, +1, -1, +2, -2, ...; each listed once with its minimal-image
// distance.
void neighbour_offsets(int R, int m, DevInfo &dv) {
    int cnt = 0;
    std::vector<int> seen;
    for (int k = 0; k <= 2 * m; ++k) {
        const int delta = (k == 0) ? 0 : ((k & 1) ? (k + 1) / 2 : -(k / 2));
        const int rp = ((delta % R) + R) % R;
        if (std::find(seen.begin(), seen.end(), rp) != seen.end()) continue;
        seen.push_back(rp);
        const int a = rp, dist = std::min(a, R - a);
        dv.nbr_off[cnt] = (int8_t)delta;
        dv.nbr_dist[cnt] = (int8_t)dist;
        ++cnt;
    }
    dv.n_nbr = cnt;
}

// Tiles of whole rails, about kTileSites padded sites each.
void make_tiles(kmc_ctx *c) {
    c->tiles.clear();
    const int target = c->tile_sites > 0 ? std::min(c->tile_sites, kTileSites) : kTileSites;
    for (int d = 0; d < c->p.n_devices; ++d) {
        const DevInfo &dv = c->devs[d];
        int nr = std::max(1, target / dv.pitch);
        nr = std::min(nr, dv.rails);
        for (int r0 = 0; r0 < dv.rails; r0 += nr) c->tiles.push_back(Tile{d, r0, std::min(nr, dv.rails - r0), 0});
    }
    size_t lds = 0, score_lds = 0;
    for (const Tile &t : c->tiles) {
        const DevInfo &dv = c->devs[t.d];
        const size_t rows = (size_t)(t.nr + 2 * c->p.rail_range) * dv.pitch;
        const size_t cap = (size_t)t.nr * dv.pitch / 2;
        const size_t n_kt = (size_t)(c->p.rail_range + 1) * (c->lay.cut + 1);
        const size_t kt = n_kt <= (size_t)kLdsTableMax ? n_kt * (c->fp64 ? sizeof(double) : sizeof(float)) : 0;
        const size_t base = rows + (cap + (cap & 1)) * sizeof(uint32_t) + kt;
        lds = std::max(lds, base);
        score_lds = std::max(score_lds, base);
    }
    c->hop_lds = lds;
    c->score_lds = score_lds;
}

// Persistent tiling: every device cut into n_t >= 1 tiles of consecutive rails,
// sizes within one rail of each other and at least max(rail_range, 1) rails
// unless the device is a single tile; prev/next are the cyclic neighbours.
void make_ptiles(kmc_ctx *c) {
    c->ptiles.clear();
    const int m = std::max(c->p.rail_range, 1);
    const int target = c->tile_sites > 0 ? c->tile_sites : kPTileSites;
    int max_chunks = 0;
    size_t lds = 0;
    const size_t real = c->fp64 ? sizeof(double) : sizeof(float);
    const size_t n_kt = (size_t)(c->p.rail_range + 1) * (c->lay.cut + 1);
    const size_t kt = n_kt <= (size_t)kLdsTableMax ? n_kt * real : 0;
    for (int d = 0; d < c->p.n_devices; ++d) {
        const DevInfo &dv = c->devs[d];
        const int want = std::max(m, target / dv.pitch);
        int n_t = std::max(1, dv.rails / want);
        if (n_t > 1 && dv.rails / n_t < m) n_t = 1;
        const int first = (int)c->ptiles.size();
        const int base = dv.rails / n_t, extra = dv.rails % n_t;
        int r0 = 0;
        for (int i = 0; i < n_t; ++i) {
            const int nr = base + (i < extra ? 1 : 0);
            const int prev = first + (i + n_t - 1) % n_t, next = first + (i + 1) % n_t;
            c->ptiles.push_back(PTile{d, r0, nr, prev, next, 0});
            r0 += nr;
            max_chunks = std::max(max_chunks, nr * dv.pitch / kChunkSites);
            // occupancy bits (two buffers), barrier classes, survivor positions, kernel
            // table, a window of per-step tables
            const size_t words = (size_t)nr * ((dv.pitch + 63) / 64);
            const size_t cap = (size_t)nr * dv.pitch / 2;
            lds = std::max(lds, 2 * words * sizeof(uint64_t) + (size_t)nr * dv.pitch +
                                    (cap + (cap & 1)) * sizeof(uint32_t) + ((kt + 7) & ~(size_t)7) +
                                    (size_t)kStepWin * (2 * sizeof(double) + sizeof(uint32_t)));
        }
    }
    c->p_block = std::min(kPMaxBlock, (max_chunks + 63) / 64 * 64);
    c->p_lds = lds;
    c->p_ok = false;
    c->pgroups.clear();
    // one lane per 16-site chunk: a tile holds at most kPMaxBlock chunks
    if (max_chunks > kPMaxBlock || lds > 160 * 1024) return;
    int per_cu = 0, dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return;
    if (persistent_capacity(c->p_block, lds, c->fp64, &per_cu) != hipSuccess) return;
    // Devices are independent: a lattice larger than what is co-resident runs
    // as a sequence of launches over groups of whole devices, each group small
    // enough to be co-resident (and within the ring slots).
    int64_t cap = std::min<int64_t>((int64_t)per_cu * prop.multiProcessorCount, c->lay.max_ptiles);
    if (c->group_limit > 0) cap = std::min<int64_t>(cap, c->group_limit);
    if (cap < 1) return;
    int first = 0, count = 0;
    for (int i = 0; i < (int)c->ptiles.size();) {
        const int d = c->ptiles[i].d;
        int n_d = 0;
        while (i + n_d < (int)c->ptiles.size() && c->ptiles[i + n_d].d == d) ++n_d;
        if (n_d > cap) return;
        if (count + n_d > cap) {
            c->pgroups.emplace_back(first, count);
            first = i;
            count = 0;
        }
        count += n_d;
        i += n_d;
    }
    if (count > 0) c->pgroups.emplace_back(first, count);
    for (const auto &g : c->pgroups)
        for (int i = g.first; i < g.first + g.second; ++i) {
            c->ptiles[i].prev -= g.first;
            c->ptiles[i].next -= g.first;
        }
    c->p_ok = true;
}

// Wave tiling: every device cut into n_t >= 1 tiles of consecutive rails that
// fit one wavefront (rails x lanes per rail <= 64), sizes within one rail of
// each other and at least max(rail_range, 1) rails unless the device is a
// single tile.  Sites per lane: 16 when that tiling exists, else 32;
// tile_sites 1024 or 2048 asks for 16 or 32.  False if the tiling with spl
// sites per lane does not exist.
bool wave_tiles_for(kmc_ctx *c, int spl) {
    c->wtiles.clear();
    const int m = c->p.rail_range, mm = std::max(m, 1);
    for (int d = 0; d < c->p.n_devices; ++d) {
        const DevInfo &dv = c->devs[d];
        const WaveGeom g = wave_geom(dv.pitch, spl);
        if (g.nr_max < 1) return false;
        const int n_t = (dv.rails + g.nr_max - 1) / g.nr_max;
        if (n_t > 1 && dv.rails / n_t < mm) return false;
        const int w32 = (dv.pitch + 31) / 32;
        if (n_t > 1 && 2 * m * w32 > wave_band_words(spl)) return false;
        const int first = (int)c->wtiles.size();
        const int base = dv.rails / n_t, extra = dv.rails % n_t;
        int r0 = 0;
        for (int i = 0; i < n_t; ++i) {
            const int nr = base + (i < extra ? 1 : 0);
            if (kPubSlots + (int64_t)kSnapSlots * std::min(nr, 2 * m) * w32 > c->lay.wpub_stride) return false;
            const int prev = first + (i + n_t - 1) % n_t, next = first + (i + 1) % n_t;
            c->wtiles.push_back(PTile{d, r0, nr, prev, next, 0});
            r0 += nr;
        }
    }
    return true;
}

void make_wtiles(kmc_ctx *c) {
    c->wtiles.clear();
    c->wgroups.clear();
    c->w_ok = false;
    if (c->dense) return;
    int spl = 0;
    if (c->tile_sites == 1024 || c->tile_sites == 2048) {
        spl = c->tile_sites / 64;
        if (!wave_tiles_for(c, spl)) return;
    } else if (wave_tiles_for(c, 16)) {
        spl = 16;
    } else if (wave_tiles_for(c, 32)) {
        spl = 32;
    } else {
        return;
    }
    c->w_spl = spl;
    const size_t n_kt = (size_t)(c->p.rail_range + 1) * (c->lay.cut + 1);
    int per_cu = 0, dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return;
    // Every workgroup asks for a quarter of the CU's LDS, so that a CU holds
    // at most four (one wavefront per SIMD each).  A launch of exactly four
    // workgroups per CU then gives every SIMD the same four tiles; with the
    // occupancy the registers allow (five), the dispatcher stacks five
    // workgroups on some CUs and three on others, and the tiles of the fuller
    // SIMDs set the launch's time.
    c->w_lds = std::max(wave_lds_bytes(spl, (int)n_kt, c->fp64), (size_t)prop.maxSharedMemoryPerMultiProcessor / 4);
    if (wave_capacity(spl, c->w_lds, c->fp64, &per_cu) != hipSuccess) return;
    // groups of whole devices, each co-resident (and within the publication memory)
    int64_t cap = std::min<int64_t>((int64_t)per_cu * prop.multiProcessorCount * kWaveTilesPerWG, c->lay.max_wtiles);
    if (c->group_limit > 0) cap = std::min<int64_t>(cap, c->group_limit);
    if (cap < 1) return;
    int first = 0, count = 0;
    for (int i = 0; i < (int)c->wtiles.size();) {
        const int d = c->wtiles[i].d;
        int n_d = 0;
        while (i + n_d < (int)c->wtiles.size() && c->wtiles[i + n_d].d == d) ++n_d;
        if (n_d > cap) return;
        if (count + n_d > cap) {
            c->wgroups.emplace_back(first, count);
            first = i;
            count = 0;
        }
        count += n_d;
        i += n_d;
    }
    if (count > 0) c->wgroups.emplace_back(first, count);
    for (const auto &g : c->wgroups)
        for (int i = g.first; i < g.first + g.second; ++i) {
            c->wtiles[i].prev -= g.first;
            c->wtiles[i].next -= g.first;
        }
    c->w_ok = true;
}

// The strategy a run uses: KMC_LAUNCH_WAVE, _PERSISTENT or _HALF_STEP.
int launch_kind(const kmc_ctx *c) {
    if (c->dense || c->phifix || c->any_open || c->mode == KMC_LAUNCH_HALF_STEP) return KMC_LAUNCH_HALF_STEP;
    if (c->mode == KMC_LAUNCH_WAVE) return c->w_ok ? KMC_LAUNCH_WAVE : KMC_LAUNCH_HALF_STEP;
    if (c->mode == KMC_LAUNCH_PERSISTENT) return c->p_ok ? KMC_LAUNCH_PERSISTENT : KMC_LAUNCH_HALF_STEP;
    // automatic: a persistent kernel whenever one fits co-resident
    if (c->w_ok) return KMC_LAUNCH_WAVE;
    return c->p_ok ? KMC_LAUNCH_PERSISTENT : KMC_LAUNCH_HALF_STEP;
}


HopArgs hop_args(kmc_ctx *c) {
    const int D = c->p.n_devices;
    HopArgs a{};
    a.devs = c->at<DevInfo>(c->lay.devs);
    a.tiles = c->at<Tile>(c->lay.tiles);
    a.n_tiles = (int32_t)c->tiles.size();
    a.knot_t = c->at<double>(c->lay.knot_t);
    a.knot_v = c->at<double>(c->lay.knot_v);
    a.ea = c->ea;
    a.ktab64 = c->at<double>(c->lay.ktab64);
    a.ktab32 = c->at<float>(c->lay.ktab32);
    a.cutoff = c->lay.cut;
    a.rail_range = c->p.rail_range;
    a.ea_scalar = c->p.ea_ev;
    a.beta = 1.0 / c->p.kT_ev;
    a.c0 = c->p.nu0_hz * c->p.dt_s;
    a.alpha = c->p.field_coupling;
    a.dt = c->p.dt_s;
    a.key0 = (uint32_t)(c->p.seed & 0xffffffffu);
    a.key1 = (uint32_t)(c->p.seed >> 32);
    a.tally_net = c->at<int32_t>(c->lay.tally_net);
    a.tally_dec = c->at<int32_t>(c->lay.tally_dec);
    a.n_devices = D;
    a.log.count = c->at<int64_t>(c->lay.log_count);
    a.log.entries = c->ws + c->lay.log_entries;
    a.log.cap = kLogCap;
    a.nu0 = c->p.nu0_hz;
    a.kappa = c->p.coulomb_kappa_v;
    if (!c->dense) {
        a.rec = c->ws + c->lay.rec;
        a.hops = c->at<uint4>(c->lay.hops);
        a.hop_ctl = c->at<int64_t>(c->lay.hop_ctl);
        a.hop_cap = c->lay.hop_cap;
    }
    if (c->dense) {
        a.phi = c->at<float>(c->lay.phi);
        a.phi_row = (int64_t)c->lay.dense_nb * 32;
        a.k10 = c->k10;
    }
    if (c->dense || c->phifix) {
        a.dtiles = c->at<Tile>(c->lay.ctiles);
        a.n_dtiles = (int32_t)c->ctiles.size();
    }
    return a;
}

// Arguments of the boundary-bond kernel for the half-step described by a.
ElectrodeArgs electrode_args(kmc_ctx *c, const HopArgs &a) {
    ElectrodeArgs e{};
    e.occ_in = a.occ_in;
    e.occ_out = a.occ_out;
    e.devs = a.devs;
    e.rail_dev = c->at<int32_t>(c->lay.rail_dev);
    e.rail_idx = c->at<int32_t>(c->lay.rail_idx);
    e.rails_total = c->lay.rails_total;
    e.el = c->at<Electrode>(c->lay.electrodes);
    e.knot_t = a.knot_t;
    e.knot_v = a.knot_v;
    e.ktab64 = a.ktab64;
    e.ktab32 = a.ktab32;
    e.cutoff = a.cutoff;
    e.beta = a.beta;
    e.c0 = a.c0;
    e.alpha = a.alpha;
    e.dt = a.dt;
    e.key0 = a.key0;
    e.key1 = a.key1;
    e.n = a.ctl.n_base + a.step_in_chunk;
    e.h = a.h;
    e.tally_row = e.n - a.ctl.tally_base;
    e.tally_net = a.tally_net;
    e.tally_dec = a.tally_dec;
    e.n_devices = a.n_devices;
    e.log = a.log;
    return e;
}

// Arguments of the fixed-point potential kernels (every rail from the state
// `occ` when full, else the hop list of parity h).
PhiFixArgs phifix_args(kmc_ctx *c, const int8_t *occ, bool full, int h) {
    PhiFixArgs f{};
    f.occ = occ;
    f.devs = c->at<DevInfo>(c->lay.devs);
    f.rail_dev = c->at<int32_t>(c->lay.rail_dev);
    f.rail_idx = c->at<int32_t>(c->lay.rail_idx);
    f.rails_total = c->lay.rails_total;
    f.kfix = c->at<int64_t>(c->lay.kfix);
    f.cutoff = c->lay.cut;
    f.rail_range = c->p.rail_range;
    f.phi = c->at<int64_t>(c->lay.phifix);
    f.out_unpadded = 0;
    f.hops = c->at<uint4>(c->lay.hops);
    f.hop_count = c->at<int64_t>(c->lay.hop_ctl) + h;
    f.hop_cap = c->lay.hop_cap;
    f.full = full ? 1 : 0;
    return f;
}

DenseArgs dense_args(kmc_ctx *c, const int8_t *occ, float *phi, int64_t phi_row) {
    DenseArgs d{};
    d.occ = occ;
    d.devs = c->at<DevInfo>(c->lay.devs);
    d.tiles = c->at<Tile>(c->lay.dtiles);
    d.n_tiles = (int32_t)c->dtiles.size();
    d.ktiles = c->ws + c->lay.ktiles;
    d.nb = c->lay.dense_nb;
    d.rail_range = c->p.rail_range;
    d.phi = phi;
    d.phi_row = phi_row;
    d.sites = c->sites[0];
    return d;
}

// Tally rows of a chunk that the wave kernel ends itself: at most five
// devices (the finishing wavefront's 128 segments) and short chunks (about 64
// steps per lane); longer chunks get the finish kernel, whose launch costs
// little against them.
bool wave_finishes(int d0, int d1, int steps) {
    const int series = (d1 - d0) * (kDeciles + 1);
    return series <= 64 && (int64_t)series * steps <= 4096;
}

// Enqueue n_steps steps.  Returns in *exported whether the launches already
// wrote the caller's occupancy (the wave kernel does).
kmc_status enqueue_steps(kmc_ctx *c, int64_t n_steps, int32_t *net_out, int32_t *dec_out, bool *exported) {
    const int D = c->p.n_devices;
    HopArgs a = hop_args(c);
    const int kind = launch_kind(c);
    const bool wave = kind == KMC_LAUNCH_WAVE;
    const bool persistent = wave || kind == KMC_LAUNCH_PERSISTENT;
    Ctl ctl{};
    ctl.call_base = c->n;
    ctl.net_out = net_out;
    ctl.dec_out = dec_out;
    FinishArgs fa{};
    fa.tally_net = a.tally_net;
    fa.tally_dec = a.tally_dec;
    fa.dec_run = c->at<int64_t>(c->lay.dec_run);
    fa.net_total = c->at<int64_t>(c->lay.net_total);
    fa.n_devices = D;
    fa.d0 = 0;
    fa.d1 = D;
    PArgs pa{};
    if (persistent) {
        pa.occ = c->cur;
        pa.devs = a.devs;
        pa.tiles = c->at<PTile>(c->lay.ptiles);
        pa.n_tiles = 0;
        pa.knot_t = a.knot_t;
        pa.knot_v = a.knot_v;
        pa.ea = a.ea;
        pa.ktab64 = a.ktab64;
        pa.ktab32 = a.ktab32;
        pa.cutoff = a.cutoff;
        pa.rail_range = a.rail_range;
        pa.ea_scalar = a.ea_scalar;
        pa.beta = a.beta;
        pa.c0 = a.c0;
        pa.alpha = a.alpha;
        pa.dt = a.dt;
        pa.key0 = a.key0;
        pa.key1 = a.key1;
        pa.tally_net = a.tally_net;
        pa.tally_dec = a.tally_dec;
        pa.n_devices = D;
        pa.log = a.log;
        pa.pub = c->at<uint64_t>(c->lay.pub);
        pa.pub_stride = wave ? c->lay.wpub_stride : c->lay.pub_stride;
        pa.status = c->at<int32_t>(c->lay.status);
        pa.spin_limit = c->spin_limit;
        pa.occ_user = c->occ_user;
    }
    if (c->rec_on) {
        HopRecord r{c->rec_buf, c->rec_count, c->rec_cap, c->rec_n0, c->rec_n_hs};
        a.record = r;
        pa.record = r;
    }
    // the fixed-point path's hop counts start at zero (a score replay in
    // between leaves its own there)
    if (c->phifix) KMC_HIP(c, launch_zero_i64(c->at<int64_t>(c->lay.hop_ctl), 2, c->stream));
    int64_t done = 0;
    while (done < n_steps) {
        const int chunk = (int)std::min<int64_t>(kTallySteps, n_steps - done);
        ctl.n_base = c->n + done;
        ctl.tally_base = ctl.n_base;
        a.ctl = ctl;
        pa.ctl = ctl;
        fa.ctl = ctl;
        fa.steps = chunk;
        bool all_finished = false;  // every device's rows ended by the launches themselves
        if (persistent) {
            all_finished = wave;
            for (const auto &g : wave ? c->wgroups : c->pgroups) {
                // publication tags carry the low 20 bits of the epoch: at every
                // wrap the ring is cleared so that no stale word can match a new tag
                if ((++c->epoch & 0xFFFFFu) == 0) {
                    KMC_HIP(c, launch_zero_i64(c->at<int64_t>(c->lay.pub), pub_words(c->lay),
                                               c->stream));
                    ++c->epoch;
                }
                const std::vector<PTile> &tl = wave ? c->wtiles : c->ptiles;
                pa.tiles = c->at<PTile>(wave ? c->lay.wtiles : c->lay.ptiles) + g.first;
                pa.n_tiles = g.second;
                pa.epoch = c->epoch;
                pa.n_steps = chunk;
                pa.fin = fa;
                pa.fin.d0 = tl[g.first].d;
                pa.fin.d1 = tl[g.first + g.second - 1].d + 1;
                pa.ticket = nullptr;
                if (wave && wave_finishes(pa.fin.d0, pa.fin.d1, chunk)) pa.ticket = c->at<uint32_t>(c->lay.ticket);
                else all_finished = false;
                if (wave) KMC_HIP(c, launch_wave(pa, c->w_spl, c->w_lds, c->fp64, c->stream));
                else KMC_HIP(c, launch_persistent(pa, c->p_block, c->p_lds, c->fp64, c->stream));
            }
            if (wave && !all_finished) {
                // the groups whose launches did not end their rows
                for (const auto &g : c->wgroups) {
                    FinishArgs f = fa;
                    f.d0 = c->wtiles[g.first].d;
                    f.d1 = c->wtiles[g.first + g.second - 1].d + 1;
                    if (!wave_finishes(f.d0, f.d1, chunk)) KMC_HIP(c, launch_finish_chunk(f, c->stream));
                }
            }
        }
        for (int k = 0; k < chunk && !persistent; ++k) {
            for (int h = 0; h < 2; ++h) {
                a.occ_in = c->cur;
                a.occ_out = c->nxt;
                a.step_in_chunk = k;
                a.h = h;
                if (c->phifix) {
                    // decisions update the state in place; then the potential
                    // follows the half-step's hops
                    a.occ_in = a.occ_out = c->cur;
                    PhiFixDecide x{c->at<int64_t>(c->lay.phifix), c->frac_bits, c->k10fix};
                    KMC_HIP(c, launch_phifix_decide(a, x, c->stream));
                    KMC_HIP(c, launch_phifix_update(phifix_args(c, c->cur, false, h), c->stream));
                    continue;
                }
                if (c->dense) {
                    // the decisions update the state in place
                    KMC_HIP(c, launch_dense_phi(dense_args(c, c->cur, c->at<float>(c->lay.phi), a.phi_row),
                                                c->stream));
                    a.occ_in = a.occ_out = c->cur;
                    KMC_HIP(c, launch_dense_decide(a, c->devs[0].pitch, c->stream));
                    continue;
                } else {
                    KMC_HIP(c, launch_hop(a, c->hop_lds, c->fp64, c->stream));
                    if (c->any_open) {
                        // boundary bonds of the same half-step, after the interior ones
                        ElectrodeArgs e = electrode_args(c, a);
                        KMC_HIP(c, launch_electrodes(e, c->fp64, c->stream));
                    }
                }
                std::swap(c->cur, c->nxt);
            }
        }
        if (!wave) KMC_HIP(c, launch_finish_chunk(fa, c->stream));
        done += chunk;
    }
    *exported = wave;
    return KMC_OK;
}

// Raised by the persistent kernel when a neighbour wait timed out.
kmc_status check_status(kmc_ctx *c) {
    int32_t st = 0;
    KMC_HIP(c, hipMemcpyAsync(&st, c->ws + c->lay.status, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    KMC_HIP(c, hipStreamSynchronize(c->stream));
    if (st != 0) {
        c->poisoned = true;
        return fail(KMC_EHIP, "persistent hop kernel: a neighbour wait timed out; state is invalid");
    }
    return KMC_OK;
}

kmc_status after_state_change(kmc_ctx *c) {
    c->rec_on = false;  // a recording describes the trajectory from its own start state
    if (c->phifix) KMC_HIP(c, launch_phifix_update(phifix_args(c, c->cur, true, 0), c->stream));
    KMC_HIP(c, launch_count_deciles(c->cur, c->at<DevInfo>(c->lay.devs), c->p.n_devices,
                                    c->at<int64_t>(c->lay.dec_run), c->stream));
    KMC_HIP(c, launch_export(c->cur, c->occ_user, c->at<DevInfo>(c->lay.devs), c->p.n_devices,
                             c->lay.total_sites, c->stream));
    return KMC_OK;
}

}  // namespace

extern "C" {

kmc_status kmc_workspace_bytes(const kmc_params *params, size_t *bytes) {
    kmc_status s = validate(params);
    if (s != KMC_OK) return s;
    if (!bytes) return fail(KMC_EINVAL, "bytes is NULL");
    *bytes = layout_for(params).total;
    return KMC_OK;
}

kmc_status kmc_init_device(const kmc_params *params, int8_t *occ_dev, const void *ea_dev, void *workspace_dev,
                           size_t ws_bytes, void *stream, kmc_ctx **out) {
    kmc_status s = validate(params);
    if (s != KMC_OK) return s;
    if (!out) return fail(KMC_EINVAL, "out is NULL");
    if (!occ_dev) return fail(KMC_EINVAL, "occ_dev is NULL");
    if (!workspace_dev) return fail(KMC_EINVAL, "workspace_dev is NULL");
    const Layout lay = layout_for(params);
    if (ws_bytes < lay.total)
        return fail(KMC_ETOOSMALL, "workspace too small: need " + std::to_string(lay.total) + " bytes");
    if (reinterpret_cast<uintptr_t>(workspace_dev) % 256 != 0)
        return fail(KMC_EINVAL, "workspace_dev must be 256-byte aligned");

    kmc_ctx *c = new kmc_ctx();
    c->p = *params;
    c->rails.assign(params->rails, params->rails + params->n_devices);
    c->sites.assign(params->sites, params->sites + params->n_devices);
    c->p.rails = c->rails.data();
    c->p.sites = c->sites.data();
    c->lay = lay;
    c->ws = static_cast<unsigned char *>(workspace_dev);
    c->occ_user = occ_dev;
    c->ea = ea_dev;
    c->stream = static_cast<hipStream_t>(stream);
    c->fp64 = params->precision == KMC_FP64 || params->precision == KMC_PHI_FIXED;
    c->cur = c->at<int8_t>(lay.occ_a);
    c->nxt = c->at<int8_t>(lay.occ_b);

    // Prefilter bound on the Coulomb term, from the telescoping sums of the
    // kernel differences: |dE_coul| <= |K(1,0)| + sum over distinct other
    // rails of |K(0,dist)|, whatever the configuration.
    const int D = params->n_devices;
    c->devs.resize(D);
    int64_t off = 0, off_pad = 0, rows_before = 0;
    for (int d = 0; d < D; ++d) {
        DevInfo &dv = c->devs[d];
        std::memset(&dv, 0, sizeof(dv));
        dv.rails = c->rails[d];
        dv.sites = c->sites[d];
        dv.pitch = (dv.sites + kChunkSites - 1) / kChunkSites * kChunkSites;
        dv.n_knots = 1;
        dv.off = off;
        dv.off_pad = off_pad;
        dv.row0 = rows_before;
        rows_before += dv.rails;
        dv.n_set = 0;
        dv.ea_min = params->ea_ev;
        neighbour_offsets(dv.rails, params->rail_range, dv);
        double bound = std::fabs(kernel64(params, 1, 0));
        for (int k = 0; k < dv.n_nbr; ++k)
            if (dv.nbr_dist[k] > 0) bound += std::fabs(kernel64(params, 0, dv.nbr_dist[k]));
        dv.coul_bound = bound;
        off += (int64_t)dv.rails * dv.sites;
        off_pad += (int64_t)dv.rails * dv.pitch;
    }
    make_tiles(c);
    make_ptiles(c);

    // binary64 kernel table and its one-time binary32 rounding
    const int m = params->rail_range, cut = lay.cut;
    std::vector<double> k64((size_t)(m + 1) * (cut + 1));
    std::vector<float> k32(k64.size());
    for (int dr = 0; dr <= m; ++dr)
        for (int ds = 0; ds <= cut; ++ds) {
            k64[(size_t)dr * (cut + 1) + ds] = kernel64(params, ds, dr);
            k32[(size_t)dr * (cut + 1) + ds] = (float)k64[(size_t)dr * (cut + 1) + ds];
        }

    // Dense potential (KMC_BF16X2): the distinct 32 x 32 blocks of
    // T[(dist, j)][s] = K(s - j, dist), as MFMA B fragments, each value split
    // into BF16 hi = RN(K) and lo = RN(K - hi).  Block (dist, delta) holds
    // rows j = 32 (sb + delta) + kk and columns s = 32 sb + ss; lane l of
    // k-step q carries kk = 16 q + 8 (l / 32) + e (e = 0..7), ss = l % 32.
    c->dense = params->precision == KMC_BF16X2;
    make_wtiles(c);
    c->k10 = cut >= 1 ? k32[1] : 0.0f;
    c->k01 = cut >= 1 ? k64[1] : 0.0;
    // Fixed-point potential (KMC_PHI_FIXED): F fractional bits such that the
    // largest |phi| any state allows (every site of every window occupied)
    // stays below 2^61, each kernel value rounded once to a multiple of 2^-F.
    c->phifix = params->precision == KMC_PHI_FIXED;
    std::vector<int64_t> kfix_host;
    if (c->phifix) {
        double peak = 0.0;
        for (int d = 0; d < D; ++d) {
            double sum = 0.0;
            const int reach = std::min(cut, c->sites[d] - 1);
            for (int k = 0; k < c->devs[d].n_nbr; ++k)
                for (int ds = -reach; ds <= reach; ++ds) sum += std::fabs(k64[(size_t)c->devs[d].nbr_dist[k] * (cut + 1) + std::abs(ds)]);
            peak = std::max(peak, sum);
        }
        int F = 52;
        if (peak > 0.0) F = std::min(52, 61 - (int)std::ceil(std::log2(peak)));
        if (F < 16) {
            delete c;
            return fail(KMC_EUNSUPPORTED, "KMC_PHI_FIXED: the Coulomb kernel sums too large for a 63-bit potential");
        }
        c->frac_bits = F;
        c->k10fix = cut >= 1 ? (int64_t)std::llrint(std::ldexp(k64[1], F)) : 0;
        kfix_host.resize(k64.size());
        for (size_t i = 0; i < k64.size(); ++i) kfix_host[i] = (int64_t)std::llrint(std::ldexp(k64[i], F));
        // decision runs: consecutive rails of one device, eight passes of a
        // 256-thread workgroup (pitch / 8 threads per rail)
        for (int d = 0; d < D; ++d) {
            const int run = 8 * (256 / (c->devs[d].pitch / 8));
            for (int r0 = 0; r0 < c->rails[d]; r0 += run)
                c->ctiles.push_back(Tile{d, r0, std::min(run, c->rails[d] - r0), 0});
        }
    }
    // runs of the streaming replay, when every rail fits one workgroup
    if (!c->dense) {
        bool fits = true;
        for (int d = 0; d < D; ++d) fits = fits && replay_run_rails(c->devs[d].pitch) > 0;
        for (int d = 0; fits && d < D; ++d) {
            const int run = replay_run_rails(c->devs[d].pitch);
            for (int r0 = 0; r0 < c->rails[d]; r0 += run)
                c->rtiles.push_back(Tile{d, r0, std::min(run, c->rails[d] - r0), 0});
        }
    }
    std::vector<uint16_t> kt_host;
    if (c->dense) {
        auto bf16_rne = [](float f) {
            uint32_t u;
            std::memcpy(&u, &f, 4);
            u += 0x7FFFu + ((u >> 16) & 1u);
            return (uint16_t)(u >> 16);
        };
        auto bf16_val = [](uint16_t h) {
            const uint32_t u = (uint32_t)h << 16;
            float f;
            std::memcpy(&f, &u, 4);
            return (double)f;
        };
        const int nb = lay.dense_nb, nd = 2 * nb - 1;
        kt_host.assign((size_t)(m + 1) * nd * 256 * 8, 0);
        for (int dd = 0; dd <= m; ++dd)
            for (int di = 0; di < nd; ++di)
                for (int q = 0; q < 2; ++q)
                    for (int l = 0; l < 64; ++l)
                        for (int e = 0; e < 8; ++e) {
                            const int delta = di - (nb - 1);
                            const int ds = -32 * delta + (l % 32) - 16 * q - 8 * (l / 32) - e;
                            const double k = kernel64(params, ds, dd);
                            const uint16_t hi = bf16_rne((float)k);
                            const uint16_t lo = bf16_rne((float)(k - bf16_val(hi)));
                            const size_t base = ((size_t)(dd * nd + di) * 2) * 2;
                            kt_host[(((base + 0 * 2 + q) * 64) + l) * 8 + e] = hi;
                            kt_host[(((base + 1 * 2 + q) * 64) + l) * 8 + e] = lo;
                        }
        const int per_wg = 256 / (c->devs[0].pitch / 8);  // rails of one decision workgroup
        for (int d = 0; d < D; ++d) {
            for (int r0 = 0; r0 < c->rails[d]; r0 += kDenseRails)
                c->dtiles.push_back(Tile{d, r0, std::min(kDenseRails, c->rails[d] - r0), 0});
            for (int r0 = 0; r0 < c->rails[d]; r0 += per_wg)
                c->ctiles.push_back(Tile{d, r0, std::min(per_wg, c->rails[d] - r0), 0});
        }
    }

    std::vector<int32_t> rail_dev, rail_idx, n_ions(D, 0);
    rail_dev.reserve(lay.rails_total);
    rail_idx.reserve(lay.rails_total);
    for (int d = 0; d < D; ++d)
        for (int r = 0; r < c->rails[d]; ++r) {
            rail_dev.push_back(d);
            rail_idx.push_back(r);
        }
    hipStream_t st = c->stream;
    auto h2d = [&](size_t at, const void *src, size_t bytes) {
        return hipMemcpyAsync(c->ws + at, src, bytes, hipMemcpyHostToDevice, st);
    };
    kmc_status ok = KMC_OK;
    auto chk = [&](hipError_t e, const char *what) {
        if (ok == KMC_OK) ok = hip_check(c, e, what);
    };
    chk(h2d(lay.devs, c->devs.data(), sizeof(DevInfo) * D), "copy device table");
    chk(h2d(lay.tiles, c->tiles.data(), sizeof(Tile) * c->tiles.size()), "copy tiles");
    chk(h2d(lay.ptiles, c->ptiles.data(), sizeof(PTile) * c->ptiles.size()), "copy persistent tiles");
    if (!c->wtiles.empty())
        chk(h2d(lay.wtiles, c->wtiles.data(), sizeof(PTile) * c->wtiles.size()), "copy wave tiles");
    chk(h2d(lay.ktab64, k64.data(), sizeof(double) * k64.size()), "copy kernel table");
    chk(h2d(lay.ktab32, k32.data(), sizeof(float) * k32.size()), "copy kernel table");
    if (c->dense) {
        chk(h2d(lay.ktiles, kt_host.data(), sizeof(uint16_t) * kt_host.size()), "copy kernel blocks");
        chk(h2d(lay.dtiles, c->dtiles.data(), sizeof(Tile) * c->dtiles.size()), "copy dense tiles");
        chk(h2d(lay.ctiles, c->ctiles.data(), sizeof(Tile) * c->ctiles.size()), "copy decision tiles");
        chk(set_dense_lds_limit((size_t)(kDenseRails + 2 * m) * (lay.dense_nb * 32 + 8)), "LDS limit of the dense kernel");
    }
    if (!c->rtiles.empty()) chk(h2d(lay.rtiles, c->rtiles.data(), sizeof(Tile) * c->rtiles.size()), "copy replay runs");
    if (c->phifix) {
        chk(h2d(lay.kfix, kfix_host.data(), sizeof(int64_t) * kfix_host.size()), "copy fixed-point kernel table");
        chk(h2d(lay.ctiles, c->ctiles.data(), sizeof(Tile) * c->ctiles.size()), "copy decision tiles");
    }
    chk(h2d(lay.rail_dev, rail_dev.data(), sizeof(int32_t) * rail_dev.size()), "copy rail table");
    chk(h2d(lay.rail_idx, rail_idx.data(), sizeof(int32_t) * rail_idx.size()), "copy rail table");
    // the host vectors above go out of scope at return: wait for the copies
    chk(hipStreamSynchronize(st), "synchronise init copies");
    chk(launch_zero_i32(c->at<int32_t>(lay.tally_net), (int64_t)kTallySteps * D, st), "zero tallies");
    chk(launch_zero_i32(c->at<int32_t>(lay.tally_dec), (int64_t)kTallySteps * D * kDeciles, st), "zero tallies");
    chk(launch_zero_i64(c->at<int64_t>(lay.net_total), D, st), "zero totals");
    chk(launch_zero_i64(c->at<int64_t>(lay.log_count), 1, st), "zero log");
    chk(launch_zero_i64(c->at<int64_t>(lay.pub), pub_words(lay), st), "zero publication ring");
    chk(launch_zero_i32(c->at<int32_t>(lay.status), 4, st), "zero status");
    chk(launch_zero_i32(c->at<int32_t>(lay.ticket), kTicketWords, st), "zero ticket");
    c->el.assign(D, Electrode{});
    chk(hipMemcpyAsync(c->ws + lay.electrodes, c->el.data(), sizeof(Electrode) * D, hipMemcpyHostToDevice, st),
        "closed electrodes");
    chk(set_hop_lds_limit(c->hop_lds, c->score_lds), "LDS limit of the hop kernel");
    {
        const double zero_t = 0.0, zero_v = 0.0;
        chk(launch_set_protocol(c->at<double>(lay.knot_t), c->at<double>(lay.knot_v), c->at<DevInfo>(lay.devs), 0, D,
                                1, 0, &zero_t, &zero_v, st),
            "install 0 V protocol");
    }
    if (ea_dev)
        chk(launch_barrier_range(ea_dev, c->fp64, c->at<DevInfo>(lay.devs), D,
                                 c->at<unsigned long long>(lay.scratch), st),
            "barrier range");
    chk(launch_import(occ_dev, c->cur, c->at<DevInfo>(lay.devs), D, lay.total_pad, ea_dev, c->fp64, st),
        "import occupancy");
    if (ok == KMC_OK) ok = after_state_change(c);
    if (ok != KMC_OK) {
        delete c;
        return ok;
    }
    *out = c;
    return KMC_OK;
}

kmc_status kmc_fill_random(kmc_ctx *c, const double *filling) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    if (!filling) return fail(KMC_EINVAL, "filling is NULL");
    const int D = c->p.n_devices;
    std::vector<int32_t> n_ions(D);
    for (int d = 0; d < D; ++d) {
        if (!(filling[d] >= 0.0 && filling[d] <= 1.0))
            return fail(KMC_EINVAL, "filling of device " + std::to_string(d) + " not in [0, 1]");
        n_ions[d] = (int32_t)std::floor(filling[d] * (double)c->sites[d] + 0.5);
    }
    KMC_HIP(c, hipMemcpyAsync(c->ws + c->lay.n_ions, n_ions.data(), sizeof(int32_t) * D, hipMemcpyHostToDevice,
                              c->stream));
    KMC_HIP(c, launch_place(c->cur, c->at<DevInfo>(c->lay.devs), c->at<int32_t>(c->lay.rail_dev),
                            c->at<int32_t>(c->lay.rail_idx), c->at<int32_t>(c->lay.n_ions),
                            (int)c->lay.rails_total, (uint32_t)(c->p.seed & 0xffffffffu),
                            (uint32_t)(c->p.seed >> 32), c->stream));
    KMC_HIP(c, hipStreamSynchronize(c->stream));  // n_ions staging buffer is local
    return after_state_change(c);
}

kmc_status kmc_load_occupancy(kmc_ctx *c) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    KMC_HIP(c, launch_import(c->occ_user, c->cur, c->at<DevInfo>(c->lay.devs), c->p.n_devices, c->lay.total_pad,
                             c->ea, c->fp64, c->stream));
    return after_state_change(c);
}

kmc_status kmc_set_bias_protocol(kmc_ctx *c, int32_t device, const double *t_s, const double *v_volt,
                                 int32_t n_knots) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    if (device < -1 || device >= c->p.n_devices) return fail(KMC_EINVAL, "device index out of range");
    if (n_knots < 1 || n_knots > kMaxKnots) return fail(KMC_EINVAL, "n_knots must be in [1, 64]");
    if (!t_s || !v_volt) return fail(KMC_EINVAL, "knot arrays are NULL");
    for (int i = 0; i < n_knots; ++i) {
        if (!is_finite(t_s[i]) || !is_finite(v_volt[i])) return fail(KMC_EINVAL, "knots must be finite");
        if (i > 0 && t_s[i] < t_s[i - 1]) return fail(KMC_EINVAL, "knot times must be nondecreasing");
    }
    const int d0 = device < 0 ? 0 : device, d1 = device < 0 ? c->p.n_devices : device + 1;
    c->rec_on = false;  // the replay evaluates every step under the installed protocols
    KMC_HIP(c, launch_set_protocol(c->at<double>(c->lay.knot_t), c->at<double>(c->lay.knot_v),
                                   c->at<DevInfo>(c->lay.devs), d0, d1, n_knots, c->n, t_s, v_volt, c->stream));
    return KMC_OK;
}

kmc_status kmc_run_steps(kmc_ctx *c, int64_t n_steps, int32_t *net_hops_dev, int32_t *decile_dev) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    if (n_steps < 0) return fail(KMC_EINVAL, "n_steps < 0");
    if (c->n + n_steps > (int64_t)0xffffffffLL) return fail(KMC_EUNSUPPORTED, "step counter would reach 2^32");
    if (n_steps == 0) return KMC_OK;
    bool exported = false;
    s = enqueue_steps(c, n_steps, net_hops_dev, decile_dev, &exported);
    if (s != KMC_OK) return s;
    if (!exported)
        KMC_HIP(c, launch_export(c->cur, c->occ_user, c->at<DevInfo>(c->lay.devs), c->p.n_devices,
                                 c->lay.total_sites, c->stream));
    c->n += n_steps;
    c->steps_run += n_steps;
    return KMC_OK;
}

kmc_status kmc_read_occupancy(kmc_ctx *c, int8_t *dst, size_t bytes) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    s = check_status(c);
    if (s != KMC_OK) return s;
    if (!dst) return fail(KMC_EINVAL, "dst is NULL");
    if (bytes < (size_t)c->lay.total_sites) return fail(KMC_ETOOSMALL, "dst smaller than the lattice");
    KMC_HIP(c, hipMemcpyAsync(dst, c->occ_user, (size_t)c->lay.total_sites, hipMemcpyDeviceToHost, c->stream));
    KMC_HIP(c, hipStreamSynchronize(c->stream));
    return KMC_OK;
}

kmc_status kmc_read_current(kmc_ctx *c, double *mean_current_A, int64_t *net_hops_total, double *sim_time_s) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    s = check_status(c);
    if (s != KMC_OK) return s;
    const int D = c->p.n_devices;
    std::vector<int64_t> tot(D);
    KMC_HIP(c, hipMemcpyAsync(tot.data(), c->ws + c->lay.net_total, sizeof(int64_t) * D, hipMemcpyDeviceToHost,
                              c->stream));
    KMC_HIP(c, hipStreamSynchronize(c->stream));
    for (int d = 0; d < D; ++d) {
        if (net_hops_total) net_hops_total[d] = tot[d];
        if (mean_current_A) {
            const double steps = (double)c->steps_run;
            mean_current_A[d] = steps > 0 ? kElementaryCharge * (double)tot[d] /
                                                ((double)c->sites[d] * c->p.dt_s * steps)
                                          : 0.0;
        }
    }
    if (sim_time_s) *sim_time_s = (double)c->n * c->p.dt_s;
    return KMC_OK;
}

kmc_status kmc_read_threshold_log(kmc_ctx *c, kmc_log_entry *dst, int64_t cap, int64_t *n_events) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    s = check_status(c);
    if (s != KMC_OK) return s;
    if (cap < 0) return fail(KMC_EINVAL, "cap < 0");
    if (cap > 0 && !dst) return fail(KMC_EINVAL, "dst is NULL");
    int64_t cnt = 0;
    KMC_HIP(c, hipMemcpyAsync(&cnt, c->ws + c->lay.log_count, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    KMC_HIP(c, hipStreamSynchronize(c->stream));
    const int64_t stored = std::min<int64_t>(std::min<int64_t>(cnt, kLogCap), cap);
    if (stored > 0) {
        KMC_HIP(c, hipMemcpyAsync(dst, c->ws + c->lay.log_entries, sizeof(kmc_log_entry) * stored,
                                  hipMemcpyDeviceToHost, c->stream));
        KMC_HIP(c, hipStreamSynchronize(c->stream));
    }
    if (n_events) *n_events = cnt;
    return KMC_OK;
}

kmc_status kmc_get_step(kmc_ctx *c, int64_t *step) {
    if (!c) return fail(KMC_EINVAL, "context is NULL");
    if (!step) return fail(KMC_EINVAL, "step is NULL");
    *step = c->n;
    return KMC_OK;
}

kmc_status kmc_set_launch_mode(kmc_ctx *c, int32_t mode) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    if (mode < KMC_LAUNCH_AUTO || mode > KMC_LAUNCH_WAVE) return fail(KMC_EINVAL, "unknown launch mode");
    if (mode == KMC_LAUNCH_PERSISTENT && !c->p_ok)
        return fail(KMC_EUNSUPPORTED, "the persistent tiling does not fit co-resident on this GPU");
    if (mode == KMC_LAUNCH_WAVE && !c->w_ok)
        return fail(KMC_EUNSUPPORTED, "the wave tiling does not fit co-resident on this GPU");
    c->mode = mode;
    return KMC_OK;
}

kmc_status kmc_get_launch_mode(kmc_ctx *c, int32_t *mode) {
    if (!c) return fail(KMC_EINVAL, "context is NULL");
    if (!mode) return fail(KMC_EINVAL, "mode is NULL");
    *mode = launch_kind(c);
    return KMC_OK;
}

kmc_status kmc_get_persistent_groups(kmc_ctx *c, int32_t *groups) {
    if (!c) return fail(KMC_EINVAL, "context is NULL");
    if (!groups) return fail(KMC_EINVAL, "groups is NULL");
    const int kind = launch_kind(c);
    *groups = kind == KMC_LAUNCH_WAVE ? (int32_t)c->wgroups.size()
                                      : (kind == KMC_LAUNCH_PERSISTENT ? (int32_t)c->pgroups.size() : 0);
    return KMC_OK;
}

}  // extern "C"

namespace {
// Rebuild both tilings after a tuning change and upload them.
kmc_status retile(kmc_ctx *c) {
    KMC_HIP(c, hipStreamSynchronize(c->stream));  // launches in flight use the old tiles
    make_tiles(c);
    make_ptiles(c);
    make_wtiles(c);
    KMC_HIP(c, hipMemcpy(c->ws + c->lay.tiles, c->tiles.data(), sizeof(Tile) * c->tiles.size(),
                         hipMemcpyHostToDevice));
    KMC_HIP(c, hipMemcpy(c->ws + c->lay.ptiles, c->ptiles.data(), sizeof(PTile) * c->ptiles.size(),
                         hipMemcpyHostToDevice));
    if (!c->wtiles.empty())
        KMC_HIP(c, hipMemcpy(c->ws + c->lay.wtiles, c->wtiles.data(), sizeof(PTile) * c->wtiles.size(),
                             hipMemcpyHostToDevice));
    KMC_HIP(c, set_hop_lds_limit(c->hop_lds, c->score_lds));
    if (c->mode == KMC_LAUNCH_PERSISTENT && !c->p_ok) c->mode = KMC_LAUNCH_AUTO;
    if (c->mode == KMC_LAUNCH_WAVE && !c->w_ok) c->mode = KMC_LAUNCH_AUTO;
    return KMC_OK;
}
}  // namespace

extern "C" {

kmc_status kmc_set_tile_sites(kmc_ctx *c, int32_t sites) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    if (sites != 0 && (sites < kChunkSites || sites > (1 << 16)))
        return fail(KMC_EINVAL, "tile sites must be 0 (default) or in [16, 65536]");
    c->tile_sites = sites;
    return retile(c);
}

namespace {
// Everything a trial run changes, saved so that tuning leaves no trace.
struct Saved {
    std::vector<int64_t> net_total, dec_run;
    int64_t log_count = 0;
    int64_t n = 0, steps_run = 0;
};

kmc_status save_state(kmc_ctx *c, Saved &sv) {
    const int D = c->p.n_devices;
    sv.net_total.resize(D);
    sv.dec_run.resize((size_t)D * kDeciles);
    KMC_HIP(c, hipMemcpyAsync(c->ws + c->lay.rp_a, c->cur, (size_t)c->lay.total_pad, hipMemcpyDeviceToDevice,
                              c->stream));
    KMC_HIP(c, hipMemcpyAsync(sv.net_total.data(), c->ws + c->lay.net_total, sizeof(int64_t) * D,
                              hipMemcpyDeviceToHost, c->stream));
    KMC_HIP(c, hipMemcpyAsync(sv.dec_run.data(), c->ws + c->lay.dec_run, sizeof(int64_t) * D * kDeciles,
                              hipMemcpyDeviceToHost, c->stream));
    KMC_HIP(c, hipMemcpyAsync(&sv.log_count, c->ws + c->lay.log_count, sizeof(int64_t), hipMemcpyDeviceToHost,
                              c->stream));
    KMC_HIP(c, hipStreamSynchronize(c->stream));
    sv.n = c->n;
    sv.steps_run = c->steps_run;
    return KMC_OK;
}

kmc_status restore_state(kmc_ctx *c, const Saved &sv) {
    const int D = c->p.n_devices;
    c->rec_on = false;  // the trial steps were recorded too
    KMC_HIP(c, hipMemcpyAsync(c->cur, c->ws + c->lay.rp_a, (size_t)c->lay.total_pad, hipMemcpyDeviceToDevice,
                              c->stream));
    KMC_HIP(c, hipMemcpyAsync(c->ws + c->lay.net_total, sv.net_total.data(), sizeof(int64_t) * D,
                              hipMemcpyHostToDevice, c->stream));
    KMC_HIP(c, hipMemcpyAsync(c->ws + c->lay.dec_run, sv.dec_run.data(), sizeof(int64_t) * D * kDeciles,
                              hipMemcpyHostToDevice, c->stream));
    KMC_HIP(c, hipMemcpyAsync(c->ws + c->lay.log_count, &sv.log_count, sizeof(int64_t), hipMemcpyHostToDevice,
                              c->stream));
    KMC_HIP(c, launch_zero_i32(c->at<int32_t>(c->lay.status), 4, c->stream));
    if (c->phifix) KMC_HIP(c, launch_phifix_update(phifix_args(c, c->cur, true, 0), c->stream));
    // a trial in the wave strategy also wrote the caller's occupancy
    KMC_HIP(c, launch_export(c->cur, c->occ_user, c->at<DevInfo>(c->lay.devs), c->p.n_devices,
                             c->lay.total_sites, c->stream));
    KMC_HIP(c, hipStreamSynchronize(c->stream));  // the host copies above are locals of the caller
    c->n = sv.n;
    c->steps_run = sv.steps_run;
    return KMC_OK;
}
}  // namespace

kmc_status kmc_autotune(kmc_ctx *c, int32_t trial_steps, int32_t *tile_sites, int32_t *mode, double *us_per_step) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    if (trial_steps < 1 || trial_steps > 65536) return fail(KMC_EINVAL, "trial_steps must be in [1, 65536]");
    if (c->n + 2 * (int64_t)trial_steps > (int64_t)0xffffffffLL)
        return fail(KMC_EUNSUPPORTED, "step counter too close to 2^32 for the trials");
    c->rec_on = false;  // the trials would be recorded
    Saved sv;
    s = save_state(c, sv);
    if (s != KMC_OK) return s;
    const int old_tile = c->tile_sites, old_mode = c->mode;
    struct Cand { int mode, tile; };
    std::vector<Cand> cands;
    if (!c->dense && !c->phifix) {
        for (int t : {1024, 2048}) cands.push_back({KMC_LAUNCH_WAVE, t});
        for (int t : {0, 4096, 8192, 12288, 16384}) cands.push_back({KMC_LAUNCH_PERSISTENT, t});
    }
    for (int t : {0, 1024, 2048, 8192}) cands.push_back({KMC_LAUNCH_HALF_STEP, t});
    hipEvent_t e0 = nullptr, e1 = nullptr;
    KMC_HIP(c, hipEventCreate(&e0));
    KMC_HIP(c, hipEventCreate(&e1));
    double best = 1e300;
    Cand pick{old_mode, old_tile};
    for (const Cand &cd : cands) {
        c->tile_sites = cd.tile;
        s = retile(c);
        if (s != KMC_OK) break;
        if (cd.mode == KMC_LAUNCH_PERSISTENT && !c->p_ok) continue;
        if (cd.mode == KMC_LAUNCH_WAVE && !c->w_ok) continue;
        c->mode = cd.mode;
        float ms = 0.0f;
        bool ok = true;
        for (int rep = 0; rep < 2 && ok; ++rep) {  // the first run pays one-time costs
            s = restore_state(c, sv);
            if (s != KMC_OK) break;
            KMC_HIP(c, hipEventRecord(e0, c->stream));
            bool exported = false;
            s = enqueue_steps(c, trial_steps, nullptr, nullptr, &exported);
            if (s != KMC_OK) break;
            KMC_HIP(c, hipEventRecord(e1, c->stream));
            KMC_HIP(c, hipEventSynchronize(e1));
            KMC_HIP(c, hipEventElapsedTime(&ms, e0, e1));
            int32_t st = 0;
            KMC_HIP(c, hipMemcpy(&st, c->ws + c->lay.status, sizeof(int32_t), hipMemcpyDeviceToHost));
            ok = st == 0;  // a configuration whose neighbour waits timed out is not a candidate
        }
        if (s != KMC_OK) break;
        const double us = 1e3 * ms / trial_steps;
        if (ok && us < best) {
            best = us;
            pick = cd;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != KMC_OK) return s;
    c->tile_sites = pick.tile;
    s = retile(c);
    if (s != KMC_OK) return s;
    c->mode = pick.mode;
    if ((c->mode == KMC_LAUNCH_PERSISTENT && !c->p_ok) || (c->mode == KMC_LAUNCH_WAVE && !c->w_ok))
        c->mode = KMC_LAUNCH_AUTO;
    s = restore_state(c, sv);
    if (s != KMC_OK) return s;
    if (tile_sites) *tile_sites = pick.tile;
    if (mode) *mode = pick.mode;
    if (us_per_step) *us_per_step = best;
    return KMC_OK;
}

kmc_status kmc_set_wait_limit(kmc_ctx *c, int32_t polls) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    if (polls < 0) return fail(KMC_EINVAL, "polls must be >= 0");
    c->spin_limit = polls;
    return KMC_OK;
}

kmc_status kmc_set_persistent_group_limit(kmc_ctx *c, int32_t max_tiles) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    if (max_tiles < 0) return fail(KMC_EINVAL, "max_tiles must be >= 0");
    c->group_limit = max_tiles;
    return retile(c);
}

}  // extern "C"

namespace {
// The replay's own buffers: its two state planes, the Coulomb part of every
// bond (path precision), the accepted-hop list with its two counters and the
// discarded near-threshold event count.
struct ReplayBufs {
    int8_t *occ_a, *occ_b;
    void *rec;
    uint4 *hops;
    int64_t *hop_ctl;
    int64_t *score_log;
};

kmc_status check_replay_args(kmc_ctx *c, const int8_t *occ0_dev, int64_t step0, int64_t n_steps,
                             const double *weight_dev, double *grad_dev) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    if (!occ0_dev || !grad_dev) return fail(KMC_EINVAL, "occ0_dev/grad_dev is NULL");
    if (n_steps < 0 || step0 < 0) return fail(KMC_EINVAL, "step0 and n_steps must be >= 0");
    if (n_steps > 0 && !weight_dev) return fail(KMC_EINVAL, "weight_dev is NULL");
    if (step0 + n_steps > (int64_t)0xffffffffLL) return fail(KMC_EUNSUPPORTED, "step index would reach 2^32");
    if (c->p.coulomb_kappa_v == 0.0)
        return fail(KMC_EINVAL, "score replay needs coulomb_kappa_v != 0 (the kappa score is dE_coul/kappa)");
    if (!(c->p.nu0_hz > 0.0)) return fail(KMC_EINVAL, "score replay needs nu0_hz > 0");
    if (c->dense) return fail(KMC_EUNSUPPORTED, "score replay runs the binary64/binary32 window paths only");
    if (c->any_open) return fail(KMC_EUNSUPPORTED, "score replay has no terms for open-electrode transfers");
    return KMC_OK;
}

kmc_status enqueue_replay(kmc_ctx *c, const int8_t *occ0_dev, int64_t step0, int64_t n_steps,
                          const double *weight_dev, double *grad_dev, const ReplayBufs &b, bool use_record) {
    const int D = c->p.n_devices;
    KMC_HIP(c, launch_zero_i64(reinterpret_cast<int64_t *>(grad_dev), 4 * (int64_t)D, c->stream));
    if (n_steps == 0) return KMC_OK;
    // A recording serves the replay when it began at step0, its steps up to
    // step0 + n_steps have been run, and occ0 is the state it began from
    // (checked here); then every half-step whose list did not overflow takes
    // the forward's decisions from it.
    std::vector<int64_t> counts;
    bool recorded = false;
    if (use_record && c->rec_on && !c->rtiles.empty() && step0 == c->rec_n0 && 2 * n_steps <= c->rec_n_hs &&
        step0 + n_steps <= c->n) {
        int64_t *flag = c->rec_count + c->rec_n_hs;
        KMC_HIP(c, launch_zero_i64(flag, 1, c->stream));
        KMC_HIP(c, launch_compare_bytes(occ0_dev, c->rec_occ, c->lay.total_sites, flag, c->stream));
        counts.resize((size_t)(2 * n_steps + 1));
        KMC_HIP(c, hipMemcpyAsync(counts.data(), c->rec_count, sizeof(int64_t) * (size_t)(2 * n_steps),
                                  hipMemcpyDeviceToHost, c->stream));
        KMC_HIP(c, hipMemcpyAsync(&counts.back(), flag, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
        KMC_HIP(c, hipStreamSynchronize(c->stream));
        recorded = counts.back() == 0;
    }
    int8_t *cur = b.occ_a, *nxt = b.occ_b;
    KMC_HIP(c, launch_import(occ0_dev, cur, c->at<DevInfo>(c->lay.devs), D, c->lay.total_pad, c->ea, c->fp64,
                             c->stream));
    HopArgs a = hop_args(c);
    a.log.count = b.score_log;
    a.log.cap = 0;
    a.score_grad = grad_dev;
    a.dtiles = c->at<Tile>(c->lay.rtiles);
    a.n_dtiles = (int32_t)c->rtiles.size();
    a.rec = b.rec;
    a.hops = b.hops;
    a.hop_ctl = b.hop_ctl;
    // the Coulomb parts of the starting state, then per half-step the replay
    // (which lists its accepted hops) and the recomputation of the bonds they
    // changed
    PhiArgs pa{};
    pa.occ = cur;
    pa.devs = c->at<DevInfo>(c->lay.devs);
    pa.n_devices = D;
    pa.ktab64 = c->at<double>(c->lay.ktab64);
    pa.cutoff = c->lay.cut;
    pa.rail_range = c->p.rail_range;
    pa.ec = b.rec;
    pa.k01 = c->k01;
    pa.hops = b.hops;
    pa.hop_cap = c->lay.hop_cap;
    KMC_HIP(c, launch_zero_i64(b.hop_ctl, 2, c->stream));
    KMC_HIP(c, launch_replay_ec_full(pa, c->fp64, c->stream));
    // The recorded half-steps keep the state as one bit per site in the plane
    // not holding it (packed when they begin, unpacked into the byte plane,
    // whose barrier classes are unchanged, before a half-step drawn again).
    bool as_bits = false;
    for (int64_t k = 0; k < n_steps; ++k) {
        a.n_abs = step0 + k;
        a.score_w = weight_dev + k * D;
        for (int h = 0; h < 2; ++h) {
            a.h = h;
            const int64_t hs = 2 * k + h;
            if (recorded && counts[(size_t)hs] <= c->rec_cap) {
                // the recorded decisions; the state is updated in place
                if (!as_bits) {
                    KMC_HIP(c, launch_pack_occ_bits(cur, reinterpret_cast<uint8_t *>(nxt), c->lay.total_pad, c->stream));
                    as_bits = true;
                }
                a.occ_in = nxt;
                a.occ_out = nxt;
                a.rec_hops = c->rec_buf + hs * c->rec_cap;
                a.rec_count = c->rec_count + hs;
                KMC_HIP(c, launch_replay_logged(a, c->fp64, c->stream));
                pa.occ = nxt;
                pa.occ_bits = 1;
                pa.hops = a.rec_hops;
                pa.hop_count = a.rec_count;
                pa.hop_cap = c->rec_cap;
                KMC_HIP(c, launch_replay_ec_update(pa, c->fp64, c->stream, counts[(size_t)hs]));
                continue;
            }
            if (as_bits) {
                KMC_HIP(c, launch_unpack_occ_bits(reinterpret_cast<const uint8_t *>(nxt), cur, c->lay.total_pad,
                                                  c->stream));
                as_bits = false;
            }
            a.occ_in = cur;
            a.occ_out = nxt;
            if (!c->rtiles.empty()) KMC_HIP(c, launch_replay_stream(a, c->fp64, c->stream));
            else KMC_HIP(c, launch_score(a, c->score_lds, c->fp64, c->stream));
            pa.occ = nxt;  // the new state, for a full recomputation after an overflow
            pa.occ_bits = 0;
            pa.hops = b.hops;
            pa.hop_count = b.hop_ctl + h;
            pa.hop_cap = c->lay.hop_cap;
            KMC_HIP(c, launch_replay_ec_update(pa, c->fp64, c->stream));
            std::swap(cur, nxt);
        }
    }
    return KMC_OK;
}
}  // namespace

namespace kmc {
// Bytes a region needs to hold the replay's buffers for this context.
size_t replay_region_bytes(const kmc_ctx *c) {
    const size_t real = c->fp64 ? sizeof(double) : sizeof(float);
    return align_up((size_t)c->lay.total_pad, 256) * 2 + align_up(real * ((size_t)c->lay.total_sites + 16), 256) +
           align_up(sizeof(uint4) * (size_t)c->lay.hop_cap, 256) + 256;
}

// kmc_score_replay with the replay's buffers carved from `region` (device
// memory of region_bytes, 256-byte aligned) instead of the workspace.
kmc_status score_replay_in_region(kmc_ctx *c, const int8_t *occ0_dev, int64_t step0, int64_t n_steps,
                                  const double *weight_dev, double *grad_dev, unsigned char *region,
                                  size_t region_bytes) {
    kmc_status s = check_replay_args(c, occ0_dev, step0, n_steps, weight_dev, grad_dev);
    if (s != KMC_OK) return s;
    const size_t need = replay_region_bytes(c);
    if (need > region_bytes)
        return fail(KMC_EUNSUPPORTED, "the lattice needs " + std::to_string(need) +
                                          " bytes of replay buffers; the static scratch holds " +
                                          std::to_string(region_bytes));
    const size_t real = c->fp64 ? sizeof(double) : sizeof(float);
    ReplayBufs b{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *p = region + off;
        off += align_up(bytes, 256);
        return p;
    };
    b.occ_a = reinterpret_cast<int8_t *>(take((size_t)c->lay.total_pad));
    b.occ_b = reinterpret_cast<int8_t *>(take((size_t)c->lay.total_pad));
    b.rec = take(real * ((size_t)c->lay.total_sites + 16));
    b.hops = reinterpret_cast<uint4 *>(take(sizeof(uint4) * (size_t)c->lay.hop_cap));
    int64_t *ctl = reinterpret_cast<int64_t *>(take(4 * sizeof(int64_t)));
    b.hop_ctl = ctl;
    b.score_log = ctl + 2;
    // (no recorded decisions: their use synchronises the stream)
    return enqueue_replay(c, occ0_dev, step0, n_steps, weight_dev, grad_dev, b, false);
}
}  // namespace kmc

extern "C" {

kmc_status kmc_score_replay(kmc_ctx *c, const int8_t *occ0_dev, int64_t step0, int64_t n_steps,
                            const double *weight_dev, double *grad_dev) {
    kmc_status s = check_replay_args(c, occ0_dev, step0, n_steps, weight_dev, grad_dev);
    if (s != KMC_OK) return s;
    ReplayBufs b{};
    b.occ_a = c->at<int8_t>(c->lay.rp_a);
    b.occ_b = c->at<int8_t>(c->lay.rp_b);
    b.rec = c->ws + c->lay.rec;
    b.hops = c->at<uint4>(c->lay.hops);
    b.hop_ctl = c->at<int64_t>(c->lay.hop_ctl);
    b.score_log = c->at<int64_t>(c->lay.score_log);
    return enqueue_replay(c, occ0_dev, step0, n_steps, weight_dev, grad_dev, b, true);
}

static size_t record_layout(const kmc_ctx *c, int64_t max_steps, int64_t cap, size_t *occ_at, size_t *buf_at) {
    const size_t n_hs = (size_t)(2 * max_steps);
    *occ_at = align_up(sizeof(int64_t) * (n_hs + 1), 256);
    *buf_at = *occ_at + align_up((size_t)c->lay.total_sites, 256);
    return *buf_at + sizeof(uint4) * n_hs * (size_t)cap;
}

static kmc_status check_record_args(kmc_ctx *c, int64_t max_steps, int64_t cap) {
    if (max_steps < 0 || cap < 0) return fail(KMC_EINVAL, "max_steps and cap must be >= 0");
    if (max_steps > 0 && cap < 1) return fail(KMC_EINVAL, "cap must be >= 1");
    if (max_steps > ((int64_t)1 << 31) || cap > ((int64_t)1 << 31) ||
        (double)max_steps * 2.0 * (double)cap > 9.0e15 / sizeof(uint4))
        return fail(KMC_EINVAL, "max_steps * cap is too large");
    if (c->dense || c->phifix) return fail(KMC_EUNSUPPORTED, "the score replay runs the binary64/binary32 window paths only");
    if (c->any_open) return fail(KMC_EUNSUPPORTED, "the score replay has no terms for open-electrode transfers");
    return KMC_OK;
}

kmc_status kmc_record_bytes(kmc_ctx *c, int64_t max_steps, int64_t cap, size_t *bytes) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    if (!bytes) return fail(KMC_EINVAL, "bytes is NULL");
    s = check_record_args(c, max_steps, cap);
    if (s != KMC_OK) return s;
    size_t occ_at, buf_at;
    *bytes = max_steps == 0 ? 0 : record_layout(c, max_steps, cap, &occ_at, &buf_at);
    return KMC_OK;
}

kmc_status kmc_record_hops(kmc_ctx *c, void *buf_dev, size_t bytes, int64_t max_steps, int64_t cap) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    if (max_steps == 0 || !buf_dev) {  // stop
        c->rec_on = false;
        return KMC_OK;
    }
    s = check_record_args(c, max_steps, cap);
    if (s != KMC_OK) return s;
    if (reinterpret_cast<uintptr_t>(buf_dev) & 255) return fail(KMC_EINVAL, "buf_dev must be 256-byte aligned");
    size_t occ_at, buf_at;
    const size_t need = record_layout(c, max_steps, cap, &occ_at, &buf_at);
    if (bytes < need) return fail(KMC_EINVAL, "the buffer needs " + std::to_string(need) + " bytes");
    if (c->n + max_steps > (int64_t)0xffffffffLL) return fail(KMC_EUNSUPPORTED, "step index would reach 2^32");
    unsigned char *base = static_cast<unsigned char *>(buf_dev);
    c->rec_count = reinterpret_cast<int64_t *>(base);
    c->rec_occ = reinterpret_cast<int8_t *>(base + occ_at);
    c->rec_buf = reinterpret_cast<uint4 *>(base + buf_at);
    c->rec_cap = cap;
    c->rec_n0 = c->n;
    c->rec_n_hs = 2 * max_steps;
    KMC_HIP(c, launch_zero_i64(c->rec_count, c->rec_n_hs + 1, c->stream));
    KMC_HIP(c, launch_export(c->cur, c->rec_occ, c->at<DevInfo>(c->lay.devs), c->p.n_devices, c->lay.total_sites,
                             c->stream));
    c->rec_on = true;
    return KMC_OK;
}

kmc_status kmc_dense_potential(kmc_ctx *c, float *phi_dev) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    if (!phi_dev) return fail(KMC_EINVAL, "phi_dev is NULL");
    if (!c->dense) return fail(KMC_EUNSUPPORTED, "the dense potential needs a KMC_BF16X2 context");
    KMC_HIP(c, launch_dense_phi(dense_args(c, c->cur, phi_dev, c->sites[0]), c->stream));
    return KMC_OK;
}

kmc_status kmc_set_electrodes(kmc_ctx *c, int32_t device, int32_t open, double ea_ground, double mu_ground,
                              double ea_bias, double mu_bias) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    if (device < -1 || device >= c->p.n_devices) return fail(KMC_EINVAL, "device index out of range");
    if (open != 0 && open != 1) return fail(KMC_EINVAL, "open must be 0 or 1");
    if (!is_finite(ea_ground) || !is_finite(mu_ground) || !is_finite(ea_bias) || !is_finite(mu_bias))
        return fail(KMC_EINVAL, "electrode barriers and energies must be finite");
    if (open && (c->dense || c->phifix))
        return fail(KMC_EUNSUPPORTED, "open electrodes run the binary64/binary32 window paths only");
    const int d0 = device < 0 ? 0 : device, d1 = device < 0 ? c->p.n_devices : device + 1;
    c->rec_on = false;
    KMC_HIP(c, hipStreamSynchronize(c->stream));  // an earlier copy of the host table may be pending
    for (int d = d0; d < d1; ++d) {
        Electrode &e = c->el[d];
        e.open = open;
        e.ea_ground = ea_ground;
        e.mu_ground = mu_ground;
        e.ea_bias = ea_bias;
        e.mu_bias = mu_bias;
    }
    c->any_open = false;
    for (const Electrode &e : c->el) c->any_open = c->any_open || e.open;
    KMC_HIP(c, hipMemcpyAsync(c->ws + c->lay.electrodes, c->el.data(), sizeof(Electrode) * c->el.size(),
                              hipMemcpyHostToDevice, c->stream));
    KMC_HIP(c, hipStreamSynchronize(c->stream));  // the host copy may change at the next call
    return KMC_OK;
}

kmc_status kmc_fixed_potential(kmc_ctx *c, int64_t *phi_dev, int32_t recompute, int32_t *frac_bits) {
    kmc_status s = usable(c);
    if (s != KMC_OK) return s;
    if (!c->phifix) return fail(KMC_EUNSUPPORTED, "the fixed-point potential needs a KMC_PHI_FIXED context");
    if (!phi_dev) return fail(KMC_EINVAL, "phi_dev is NULL");
    if (recompute != 0 && recompute != 1) return fail(KMC_EINVAL, "recompute must be 0 or 1");
    if (recompute) {
        PhiFixArgs f = phifix_args(c, c->cur, true, 0);
        f.phi = phi_dev;
        f.out_unpadded = 1;
        KMC_HIP(c, launch_phifix_update(f, c->stream));
    } else {
        KMC_HIP(c, launch_phifix_export(c->at<int64_t>(c->lay.phifix), phi_dev, c->at<DevInfo>(c->lay.devs),
                                        c->at<int32_t>(c->lay.rail_dev), c->at<int32_t>(c->lay.rail_idx),
                                        c->lay.rails_total, c->stream));
    }
    if (frac_bits) *frac_bits = c->frac_bits;
    return KMC_OK;
}

kmc_status kmc_calib_copy(const void *src, void *dst, size_t bytes, void *stream) {
    if (!src || !dst) return fail(KMC_EINVAL, "NULL pointer");
    if (bytes % 16 != 0 || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
        return fail(KMC_EINVAL, "copy needs 16-byte aligned pointers and a multiple of 16 bytes");
    const hipError_t e = launch_copy_bytes(src, dst, bytes, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(KMC_EHIP, std::string("copy launch: ") + hipGetErrorString(e));
    return KMC_OK;
}

#ifndef KMC_SOURCE_HASH
#define KMC_SOURCE_HASH "unknown"
#endif
const char *kmc_build_hash(void) { return KMC_SOURCE_HASH; }

const char *kmc_last_error(void) { return g_last_error.c_str(); }

void kmc_destroy(kmc_ctx *c) {
    if (!c) return;
    if (!c->poisoned) (void)hipStreamSynchronize(c->stream);
    delete c;
}

}  // extern "C"

namespace kmc {
// The error text of the calling thread, for the other sources of the library.
kmc_status record_error(kmc_status s, const std::string &msg) { return fail(s, msg); }
}  // namespace kmc
