/*
 * Plain CPU oracle for the rail kinetic Monte Carlo (KMC) hop step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  The product path (the
 * HIP library under paper_2511_09413_amd/) never calls it, and this file shares
 * no code, header, table or constant generator with it.
 *
 * What is computed (paper: Supplementary Information S1-S2; main text
 * section 3 "Mapping to the code"):
 *   - rails of sites, each site empty or holding one cation; ions hop only
 *     along their rail, never between rails (SI S2.1, "Step-by-step"; the
 *     number of ions per rail is fixed);
 *   - hard-core exclusion: a hop goes only into an empty neighbour site
 *     (SI S2.1, "Random sampling and exclusion rules");
 *   - thermally activated hop rate nu0*exp(-Em/kT) (main text, Eq. hop_rate)
 *     whose barrier is shifted by half the energy change of the hop, so that
 *     forward/backward rates keep detailed balance (main text, Eq. 2 and the
 *     paragraph after it);
 *   - the energy change is the applied-bias drop (SI Eq. S1, grounded bottom
 *     electrode and biased top electrode, SI S1.3) plus the Coulomb energy of
 *     nearby ions (main text section 3), here a screened Coulomb kernel with an
 *     inclusive cutoff along the rail and a neighbourhood of rails, periodic
 *     in the rail index (SI S1.4 "periodic lateral edges");
 *   - accept when the uniform draw is below the hop probability (SI S2.1,
 *     movement masks), the update being a pair (bond) checkerboard: even bonds
 *     then odd bonds, each half-step deciding every bond from the state at the
 *     start of the half-step; this is the conflict-free reading of the paper's
 *     "all ions at once" update.
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), written here from that publication.
 *   hop draw of bond (s, s+1) of rail r, device d, step n, half-step h = s&1:
 *     counter = (s>>3, r, n, d<<4 | 0<<1 | h), key = (seed lo, seed hi),
 *     word (s>>1)&3 of the output block;
 *   placement draw of site s: counter = (s>>2, r, 0, d<<4 | 1<<1), word s&3;
 *   transfer draw of a boundary bond (open electrodes): counter =
 *     (0, r, n, d<<4 | 3<<1 | h), word 0 (grounded side) or 1 (biased side).
 *
 * Open electrodes (optional, orc_electrodes): an extension in the direction
 * the paper's conclusion invites (new mechanisms by altering probabilities),
 * not the paper's model, whose electrodes block and whose rails keep their
 * ion count.  Each rail end is one more bond to a reservoir whose ion has a
 * set energy and no Coulomb interaction; see orc_electrode_delta_energy.
 *
 * Two precision paths: binary64 everywhere, or binary32 for the energy, the
 * exponent and the probability (tables rounded once from binary64).  Build
 * with -O2 -ffp-contract=off and no fast-math.
 */
#include "kmc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11): multipliers, Weyl key increments, 10 rounds. */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)prod1;
        uint32_t y2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)prod0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static uint32_t philox_word(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                            uint32_t c3, int word)
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[word];
}

uint32_t orc_hop_word(uint64_t seed, int d, int64_t n, int r, int s)
{
    int h = s & 1;
    return philox_word(seed, (uint32_t)(s >> 3), (uint32_t)r, (uint32_t)n,
                       ((uint32_t)d << 4) | (0u << 1) | (uint32_t)h, (s >> 1) & 3);
}

uint32_t orc_place_word(uint64_t seed, int d, int r, int s)
{
    return philox_word(seed, (uint32_t)(s >> 2), (uint32_t)r, 0u,
                       ((uint32_t)d << 4) | (1u << 1), s & 3);
}

/* The word of a boundary (electrode) bond: stream 3, the block at counter
 * (0, r, n, 16 d + 2*3 + h), word 0 for the grounded side, 1 for the biased
 * side (h is the half-step the bond belongs to). */
uint32_t orc_electrode_word(uint64_t seed, int d, int64_t n, int r, int h, int side)
{
    return philox_word(seed, 0u, (uint32_t)r, (uint32_t)n, ((uint32_t)d << 4) | (3u << 1) | (uint32_t)h,
                       side);
}

/* ------------------------------------------------------------------ */
/* Geometry helpers                                                    */
/* ------------------------------------------------------------------ */
static int64_t dev_offset(const orc_params *P, int d)
{
    int64_t off = 0;
    for (int i = 0; i < d; ++i) off += (int64_t)P->rails[i] * P->sites[i];
    return off;
}

/* minimal-image rail distance on a ring of R rails */
static int rail_dist(int r, int rp, int R)
{
    int a = ((rp - r) % R + R) % R;
    return a < R - a ? a : R - a;
}

/* Distinct rails within rail_range of rail r (each counted once), with their
 * minimal-image distance.  Returns the count. */
static int neighbour_rails(const orc_params *P, int R, int r, int *rail_out, int *dist_out)
{
    int cnt = 0;
    for (int k = 0; k <= 2 * P->rail_range; ++k) {
        /* visit offsets in the order 0, +1, -1, +2, -2, ... */
        int delta = (k == 0) ? 0 : ((k & 1) ? (k + 1) / 2 : -(k / 2));
        int rp = ((r + delta) % R + R) % R;
        int seen = 0;
        for (int i = 0; i < cnt; ++i)
            if (rail_out[i] == rp) seen = 1;
        if (seen) continue;
        rail_out[cnt] = rp;
        dist_out[cnt] = rail_dist(r, rp, R);
        ++cnt;
    }
    return cnt;
}

/* Interaction kernel K(ds, dr) in volts (eV per elementary charge), binary64.
 * Screened Coulomb kappa*exp(-d/lambda)/d, or kappa/d when lambda == 0, with
 * d = sqrt(ds^2 + dr^2); zero at (0,0), beyond |ds| > cutoff or dr > rail_range. */
double orc_kernel(const orc_params *P, int ds, int dr)
{
    if (ds == 0 && dr == 0) return 0.0;
    if (abs(ds) > P->cutoff) return 0.0;
    if (dr > P->rail_range) return 0.0;
    double dist = sqrt((double)ds * (double)ds + (double)dr * (double)dr);
    if (P->lambda > 0.0) return P->kappa * exp(-dist / P->lambda) / dist;
    return P->kappa / dist;
}

/* ------------------------------------------------------------------ */
/* Protocol: piecewise-linear V(t), right-continuous, constant outside. */
/* ------------------------------------------------------------------ */
double orc_protocol_voltage(const double *t_k, const double *v_k, int n_knots, double t_rel)
{
    if (n_knots <= 0) return 0.0;
    if (t_rel < t_k[0]) return v_k[0];
    int k = 0;
    for (int i = 0; i < n_knots; ++i)
        if (t_k[i] <= t_rel) k = i;
    if (k == n_knots - 1) return v_k[n_knots - 1];
    double slope_num = (v_k[k + 1] - v_k[k]) * (t_rel - t_k[k]);
    return v_k[k] + slope_num / (t_k[k + 1] - t_k[k]);
}

static double device_voltage(const orc_protocol *pr, int d, int64_t n, double dt)
{
    const orc_protocol *p = &pr[d];
    double t_rel = (double)(n - p->n_set) * dt;
    return orc_protocol_voltage(p->t, p->v, p->n_knots, t_rel);
}

/* ------------------------------------------------------------------ */
/* Energy change of the hop o -> t on rail r (occupancy snapshot S of   */
/* one device, R x L).  Binary64 and binary32 paths.                    */
/* ------------------------------------------------------------------ */
/* The two parts of the energy change: the applied-bias drop e_app and the
 * Coulomb sum e_coul over the snapshot (window terms visited rail by rail in
 * the neighbour order, sites in increasing order). */
static void delta_energy_parts_f64(const orc_params *P, int R, int L, const int8_t *S,
                                   int r, int o, int t, double V, double *e_app_out,
                                   double *e_coul_out, double *a_abs_out)
{
    double e_app = ((P->alpha * V) * (double)(t - o)) / (double)L;
    int rails[64], dists[64];
    int nr = neighbour_rails(P, R, r, rails, dists);
    int lo = (o < t ? o : t) - P->cutoff;
    int hi = (o > t ? o : t) + P->cutoff;
    if (lo < 0) lo = 0;
    if (hi > L - 1) hi = L - 1;
    double e_coul = 0.0, a_abs = 0.0;
    for (int i = 0; i < nr; ++i) {
        const int8_t *row = S + (int64_t)rails[i] * L;
        for (int j = lo; j <= hi; ++j) {
            if (rails[i] == r && (j == o || j == t)) continue;
            if (!row[j]) continue;
            e_coul += orc_kernel(P, t - j, dists[i]) - orc_kernel(P, o - j, dists[i]);
            a_abs += fabs(orc_kernel(P, t - j, dists[i])) + fabs(orc_kernel(P, o - j, dists[i]));
        }
    }
    *e_app_out = e_app;
    *e_coul_out = e_coul;
    if (a_abs_out) *a_abs_out = a_abs;
}

static void delta_energy_parts_f32(const orc_params *P, int R, int L, const int8_t *S,
                                   int r, int o, int t, double V, float *e_app_out,
                                   float *e_coul_out, double *a_abs_out)
{
    float a = (float)P->alpha, v = (float)V;
    float e_app = ((a * v) * (float)(t - o)) / (float)L;
    int rails[64], dists[64];
    int nr = neighbour_rails(P, R, r, rails, dists);
    int lo = (o < t ? o : t) - P->cutoff;
    int hi = (o > t ? o : t) + P->cutoff;
    if (lo < 0) lo = 0;
    if (hi > L - 1) hi = L - 1;
    float e_coul = 0.0f;
    double a_abs = 0.0;
    for (int i = 0; i < nr; ++i) {
        const int8_t *row = S + (int64_t)rails[i] * L;
        for (int j = lo; j <= hi; ++j) {
            if (rails[i] == r && (j == o || j == t)) continue;
            if (!row[j]) continue;
            float kt = (float)orc_kernel(P, t - j, dists[i]);
            float ko = (float)orc_kernel(P, o - j, dists[i]);
            e_coul += kt - ko;
            a_abs += fabs(orc_kernel(P, t - j, dists[i])) + fabs(orc_kernel(P, o - j, dists[i]));
        }
    }
    *e_app_out = e_app;
    *e_coul_out = e_coul;
    if (a_abs_out) *a_abs_out = a_abs;
}

/* Coulomb potential at site x of rail r from the other ions of the snapshot
 * (window terms in the same order as the hop's sum), binary64 or, with f32,
 * summed in binary32 from once-rounded kernel values. */
static double site_potential_f64(const orc_params *P, int R, int L, const int8_t *S, int r, int x)
{
    int rails[64], dists[64];
    int nr = neighbour_rails(P, R, r, rails, dists);
    int lo = x - P->cutoff, hi = x + P->cutoff;
    if (lo < 0) lo = 0;
    if (hi > L - 1) hi = L - 1;
    double phi = 0.0;
    for (int i = 0; i < nr; ++i) {
        const int8_t *row = S + (int64_t)rails[i] * L;
        for (int j = lo; j <= hi; ++j) {
            if (rails[i] == r && j == x) continue;
            if (row[j]) phi += orc_kernel(P, x - j, dists[i]);
        }
    }
    return phi;
}

static float site_potential_f32(const orc_params *P, int R, int L, const int8_t *S, int r, int x)
{
    int rails[64], dists[64];
    int nr = neighbour_rails(P, R, r, rails, dists);
    int lo = x - P->cutoff, hi = x + P->cutoff;
    if (lo < 0) lo = 0;
    if (hi > L - 1) hi = L - 1;
    float phi = 0.0f;
    for (int i = 0; i < nr; ++i) {
        const int8_t *row = S + (int64_t)rails[i] * L;
        for (int j = lo; j <= hi; ++j) {
            if (rails[i] == r && j == x) continue;
            if (row[j]) phi += (float)orc_kernel(P, x - j, dists[i]);
        }
    }
    return phi;
}

/* Energy change of a transfer across the boundary bond of rail r, side 0
 * (grounded: reservoir at virtual site -1, lattice site 0) or side 1
 * (biased: lattice site L-1, reservoir at virtual site L).  inject = 1: an
 * ion leaves the reservoir for the empty boundary site; 0: the ion on the
 * boundary site leaves for the reservoir.  With o, t the origin and target
 * (virtual sites included) the bias part is alpha V (t - o) / L, as for any
 * hop; the Coulomb part is +phi(x) on injection and -phi(x) on extraction
 * (reservoir ions do not interact); the reservoir's own energy mu leaves on
 * injection (-mu) and arrives on extraction (+mu):
 *     dE = (e_app + sgn phi(x)) - sgn mu,   sgn = +1 injection, -1 extraction,
 * in the path precision (binary32: e_app, phi and mu rounded as the hop's). */
double orc_electrode_delta_energy(const orc_params *P, int R, int L, const int8_t *S, int r, int side,
                                  int inject, double V, double mu)
{
    int x = side == 0 ? 0 : L - 1;
    int res = side == 0 ? -1 : L;
    int o = inject ? res : x, t = inject ? x : res;
    if (P->fp32) {
        float a = (float)P->alpha, v = (float)V;
        float e_app = ((a * v) * (float)(t - o)) / (float)L;
        float phi = site_potential_f32(P, R, L, S, r, x);
        float sgn = inject ? 1.0f : -1.0f;
        return (double)((e_app + sgn * phi) - sgn * (float)mu);
    }
    double e_app = ((P->alpha * V) * (double)(t - o)) / (double)L;
    double phi = site_potential_f64(P, R, L, S, r, x);
    double sgn = inject ? 1.0 : -1.0;
    return (e_app + sgn * phi) - sgn * mu;
}

double orc_delta_energy_f64(const orc_params *P, int R, int L, const int8_t *S,
                            int r, int o, int t, double V)
{
    double e_app, e_coul;
    delta_energy_parts_f64(P, R, L, S, r, o, t, V, &e_app, &e_coul, NULL);
    return e_app + e_coul;
}

float orc_delta_energy_f32(const orc_params *P, int R, int L, const int8_t *S,
                           int r, int o, int t, double V)
{
    float e_app, e_coul;
    delta_energy_parts_f32(P, R, L, S, r, o, t, V, &e_app, &e_coul, NULL);
    return e_app + e_coul;
}

/* Coulomb potential at every site, binary64: phi(r, s) = sum over the distinct
 * rails r' within rail_range of r (r itself included) and sites j of
 * occ(r', j) K(s - j, dist(r, r')), the site itself excluded (K(0,0) = 0).
 * This is the field of the ions that the main text (section 3) adds to the
 * bias; for a hop o -> t on rail r the Coulomb part of the energy change is
 * phi(t) - K(1, 0) - phi(o), the K(1, 0) removing the moving ion's own
 * contribution at its target.  occ and phi are [rails][sites] per device,
 * devices concatenated. */
void orc_dense_potential(const orc_params *P, const int8_t *occ, double *phi)
{
    for (int d = 0; d < P->n_devices; ++d) {
        int R = P->rails[d], L = P->sites[d];
        int64_t off = dev_offset(P, d);
        const int8_t *od = occ + off;
        double *pd = phi + off;
        for (int r = 0; r < R; ++r) {
            int rails[64], dists[64];
            int nr = neighbour_rails(P, R, r, rails, dists);
            for (int s = 0; s < L; ++s) {
                double acc = 0.0;
                for (int i = 0; i < nr; ++i) {
                    const int8_t *row = od + (int64_t)rails[i] * L;
                    for (int j = 0; j < L; ++j)
                        if (row[j]) acc += orc_kernel(P, s - j, dists[i]);
                }
                pd[(int64_t)r * L + s] = acc;
            }
        }
    }
}

/* hop probability p = min(nu0*dt*exp(-beta*(Ea + dE/2)), 1) */
double orc_hop_prob_f64(const orc_params *P, double ea, double dE)
{
    double beta = 1.0 / P->kT;
    double c0 = P->nu0 * P->dt;
    double p = c0 * exp(-beta * (ea + 0.5 * dE));
    return p < 1.0 ? p : 1.0;
}

float orc_hop_prob_f32(const orc_params *P, double ea, float dE)
{
    float beta = (float)(1.0 / P->kT);
    float c0 = (float)(P->nu0 * P->dt);
    float p = c0 * expf(-beta * ((float)ea + 0.5f * dE));
    return p < 1.0f ? p : 1.0f;
}

/* ------------------------------------------------------------------ */
/* Initial placement: floor(f*L + 1/2) ions per rail on the sites with  */
/* the smallest (placement word, site index) keys.                      */
/* ------------------------------------------------------------------ */
typedef struct { uint32_t w; int s; } place_key;

static int cmp_place(const void *a, const void *b)
{
    const place_key *x = (const place_key *)a, *y = (const place_key *)b;
    if (x->w != y->w) return x->w < y->w ? -1 : 1;
    return x->s < y->s ? -1 : (x->s > y->s ? 1 : 0);
}

int orc_ions_per_rail(double filling, int L)
{
    return (int)floor(filling * (double)L + 0.5);
}

void orc_fill(const orc_params *P, const double *filling, int8_t *occ)
{
    for (int d = 0; d < P->n_devices; ++d) {
        int R = P->rails[d], L = P->sites[d];
        int8_t *dev = occ + dev_offset(P, d);
        int nion = orc_ions_per_rail(filling[d], L);
        place_key *keys = (place_key *)malloc(sizeof(place_key) * (size_t)L);
        for (int r = 0; r < R; ++r) {
            for (int s = 0; s < L; ++s) {
                keys[s].w = orc_place_word(P->seed, d, r, s);
                keys[s].s = s;
            }
            qsort(keys, (size_t)L, sizeof(place_key), cmp_place);
            int8_t *row = dev + (int64_t)r * L;
            memset(row, 0, (size_t)L);
            for (int i = 0; i < nion; ++i) row[keys[i].s] = 1;
        }
        free(keys);
    }
}

/* ------------------------------------------------------------------ */
/* The step loop                                                         */
/* ------------------------------------------------------------------ */
static void log_event(orc_log_entry *log, int64_t cap, int64_t *n_log, int d, int h,
                      int64_t n, int r, int s, double u, double p)
{
    if (log && *n_log < cap) {
        orc_log_entry *e = &log[*n_log];
        e->d = d; e->h = h; e->n = n; e->r = r; e->s = s; e->u = u; e->p = p;
    }
    ++*n_log;
}

/* A permutation of 0..m-1 drawn from a 64-bit LCG (only used to prove that the
 * order in which bonds are visited inside a half-step does not matter). */
static void permutation(int64_t m, uint64_t seed, int64_t *perm)
{
    for (int64_t i = 0; i < m; ++i) perm[i] = i;
    uint64_t x = seed * 6364136223846793005ull + 1442695040888963407ull;
    for (int64_t i = m - 1; i > 0; --i) {
        x = x * 6364136223846793005ull + 1442695040888963407ull;
        int64_t j = (int64_t)((x >> 33) % (uint64_t)(i + 1));
        int64_t tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
    }
}

/* Score-function (likelihood-ratio) term of one Bernoulli hop decision.
 * The decision y ~ Bernoulli(p) with p = nu0 dt exp(-beta (Ea + dE/2)) (main
 * text Eq. hop_rate with the half-energy shift of Eq. 2) has
 *     d log P(y) / d theta = (d log p / d theta) (y - p) / (1 - p)
 * while p < 1, and 0 once p is clamped at 1.  The log-derivatives of p for
 * theta = (Ea shift of every barrier, nu0, kappa, alpha) are
 *     -beta,  1/nu0,  -(beta/2) e_coul/kappa,  -(beta/2) V (t - o)/L ,
 * since e_coul is linear in kappa and e_app = alpha V (t - o)/L.  The term is
 * weighted by W[k][d] (the caller's weight of the decision's step) and summed
 * per device.  Also summed: |term| (magnitude) and |W g| p/(1-p)^2, the
 * sensitivity of the term to a relative change of p (its derivative in p
 * times p). */
static void add_score(const orc_params *P, const orc_run_opts *opts, int64_t k, int d,
                      int accept, double p, double e_coul, double V, int o, int t, int L,
                      double ea, double dE, double a_abs)
{
    if (!(p < 1.0)) return;
    const int D = P->n_devices;
    const double beta = 1.0 / P->kT;
    const double W = opts->score_w[k * D + d];
    const double g[4] = {-beta, 1.0 / P->nu0, -0.5 * beta * e_coul / P->kappa,
                         -0.5 * beta * V * (double)(t - o) / (double)L};
    const double ratio = ((double)accept - p) / (1.0 - p);
    const double b = a_abs + fabs(dE) + fabs(e_coul) + 2.0 * fabs(orc_kernel(P, 1, 0));
    for (int q = 0; q < 4; ++q) {
        const double term = W * g[q] * ratio;
        const double base = fabs(W * g[q]) * p / ((1.0 - p) * (1.0 - p));
        opts->score_grad[d * 4 + q] += term;
        if (opts->score_mag) opts->score_mag[d * 4 + q] += fabs(term);
        if (opts->score_sens) opts->score_sens[d * 4 + q] += base;
        if (opts->score_sens_arg) opts->score_sens_arg[d * 4 + q] += base * fabs(beta * (ea + 0.5 * dE));
        if (opts->score_sens_b) {
            double scale = base * 0.5 * beta;
            if (q == 2) scale += fabs(W * 0.5 * beta / P->kappa) * fabs(ratio);
            opts->score_sens_b[d * 4 + q] += scale * b;
        }
    }
}

/* Threads of orc_run's plain path (no shuffle, no score accumulation): the
 * rails of a device are split over OpenMP threads inside each half-step.
 * Every decision reads only the half-step's snapshot and writes only its own
 * rail, so the result does not depend on the thread count (the threshold
 * log's entry order may). */
static int orc_threads = 1;

void orc_set_threads(int n)
{
    orc_threads = n < 1 ? 1 : n;
}

/* One bond (s, s+1) of rail r of device d in half-step h of step n (its k-th
 * step in this run): candidate test, energy change on the snapshot Sd,
 * probability, accept, the log, the score terms, and the update of Od.
 * Returns 1 for a hop toward site 0, 2 toward site L-1, 0 otherwise. */
static int visit_bond(const orc_params *P, int d, int R, int L, int64_t off, const int8_t *Sd,
                      int8_t *Od, int h, int64_t n, int64_t k, double V, int r, int s,
                      orc_log_entry *log, int64_t log_cap, int64_t *n_log, const orc_run_opts *opts,
                      int threaded)
{
    int8_t a0 = Sd[(int64_t)r * L + s], a1 = Sd[(int64_t)r * L + s + 1];
    if (a0 == a1) return 0;
    int o = a0 ? s : s + 1;
    int t = a0 ? s + 1 : s;
    double ea = P->ea_site ? P->ea_site[off + (int64_t)r * L + o] : P->ea;
    uint32_t w = orc_hop_word(P->seed, d, n, r, s);
    int accept, near;
    double u_log, p_log;
    double p_score, e_coul_score, de_score, a_abs = 0.0;
    if (P->fp32) {
        float e_app, e_coul;
        delta_energy_parts_f32(P, R, L, Sd, r, o, t, V, &e_app, &e_coul, &a_abs);
        float dE = e_app + e_coul;
        float p = orc_hop_prob_f32(P, ea, dE);
        float u = ldexpf((float)w, -32);
        accept = u < p;
        u_log = u; p_log = p;
        p_score = p; e_coul_score = e_coul; de_score = dE;
        near = fabsf(u - p) < 1e-6f;
        if (opts && opts->score_grad && opts->score_coul64) {
            double e_app64, e_coul64;
            delta_energy_parts_f64(P, R, L, Sd, r, o, t, V, &e_app64, &e_coul64, &a_abs);
            float dE_s = e_app + (float)e_coul64;
            p_score = orc_hop_prob_f32(P, ea, dE_s);
            e_coul_score = e_coul64;
            de_score = dE_s;
        }
    } else {
        double e_app, e_coul;
        delta_energy_parts_f64(P, R, L, Sd, r, o, t, V, &e_app, &e_coul, &a_abs);
        double dE = e_app + e_coul;
        double p = orc_hop_prob_f64(P, ea, dE);
        double u = ldexp((double)w, -32);
        accept = u < p;
        u_log = u; p_log = p;
        p_score = p; e_coul_score = e_coul; de_score = dE;
        near = fabs(u - p) < 1e-6;
    }
    if (near) {
        if (threaded) {
#pragma omp critical(orc_log)
            log_event(log, log_cap, n_log, d, h, n, r, s, u_log, p_log);
        } else {
            log_event(log, log_cap, n_log, d, h, n, r, s, u_log, p_log);
        }
    }
    if (opts && opts->score_grad)
        add_score(P, opts, k, d, accept, p_score, e_coul_score, V, o, t, L, ea, de_score, a_abs);
    if (accept && opts && opts->score_hops) ++opts->score_hops[d];
    if (!accept) return 0;
    Od[(int64_t)r * L + o] = 0;
    Od[(int64_t)r * L + t] = 1;
    return t < o ? 1 : 2;
}

/* The boundary bond of side `side` of rail r in half-step h, when the
 * device's electrodes are open: a transfer with the rate law of any hop
 * (barrier ea of that electrode), accepted when u < p; logged like a hop
 * (bond index -1 for the grounded side, L-1 for the biased side).  Returns 1
 * for a transfer toward site 0's side (extraction at the grounded electrode,
 * injection at the biased one), 2 for the opposite direction, 0 for none. */
static int visit_electrode(const orc_params *P, const orc_electrodes *el, int d, int R, int L, const int8_t *Sd,
                           int8_t *Od, int h, int64_t n, double V, int r, int side, orc_log_entry *log,
                           int64_t log_cap, int64_t *n_log, int threaded)
{
    int x = side == 0 ? 0 : L - 1;
    int inject = Sd[(int64_t)r * L + x] == 0;
    double mu = side == 0 ? el->mu_ground : el->mu_bias;
    double ea = side == 0 ? el->ea_ground : el->ea_bias;
    double dE = orc_electrode_delta_energy(P, R, L, Sd, r, side, inject, V, mu);
    uint32_t w = orc_electrode_word(P->seed, d, n, r, h, side);
    int accept, near;
    double u_log, p_log;
    if (P->fp32) {
        float p = orc_hop_prob_f32(P, ea, (float)dE);
        float u = ldexpf((float)w, -32);
        accept = u < p;
        near = fabsf(u - p) < 1e-6f;
        u_log = u; p_log = p;
    } else {
        double p = orc_hop_prob_f64(P, ea, dE);
        double u = ldexp((double)w, -32);
        accept = u < p;
        near = fabs(u - p) < 1e-6;
        u_log = u; p_log = p;
    }
    if (near) {
        int sb = side == 0 ? -1 : L - 1;
        if (threaded) {
#pragma omp critical(orc_log)
            log_event(log, log_cap, n_log, d, h, n, r, sb, u_log, p_log);
        } else {
            log_event(log, log_cap, n_log, d, h, n, r, sb, u_log, p_log);
        }
    }
    if (!accept) return 0;
    Od[(int64_t)r * L + x] = inject ? 1 : 0;
    /* toward site 0's side: extraction at the grounded end, injection at the biased end */
    return (side == 0) != inject ? 1 : 2;
}

/* Whether the boundary bond of `side` belongs to half-step h: bond s = -1
 * (grounded) is odd, bond s = L - 1 (biased) has the parity of L - 1. */
static int electrode_in_half_step(int side, int L, int h)
{
    return side == 0 ? h == 1 : ((L - 1) & 1) == h;
}

int orc_run(const orc_params *P, const orc_protocol *protocols, int8_t *occ,
            int64_t n0, int64_t n_steps, int32_t *net_out, int32_t *dec_out,
            int64_t *net_total, orc_log_entry *log, int64_t log_cap, int64_t *n_log,
            const orc_run_opts *opts)
{
    int D = P->n_devices;
    if (n0 < 0 || n0 + n_steps > (int64_t)0xffffffffLL) return -1;
    if (opts && opts->score_grad && (P->kappa == 0.0 || !(P->nu0 > 0.0))) return -2;
    if (opts && opts->score_grad && opts->electrodes) return -3;
    int64_t total = dev_offset(P, D);
    int8_t *S = (int8_t *)malloc((size_t)total);
    int64_t dummy_log = 0;
    if (!n_log) n_log = &dummy_log;
    double *V = (double *)malloc(sizeof(double) * (size_t)D);
    int32_t *n_down = (int32_t *)calloc((size_t)D, sizeof(int32_t));
    int32_t *n_up = (int32_t *)calloc((size_t)D, sizeof(int32_t));
    const int threaded = orc_threads > 1 && !(opts && (opts->shuffle_seed || opts->score_grad || opts->score_hops));

    for (int64_t k = 0; k < n_steps; ++k) {
        int64_t n = n0 + k;
        for (int d = 0; d < D; ++d) {
            V[d] = device_voltage(protocols, d, n, P->dt);
            n_down[d] = 0;
            n_up[d] = 0;
        }
        for (int h = 0; h < 2; ++h) {
            memcpy(S, occ, (size_t)total); /* Jacobi snapshot */
            for (int d = 0; d < D; ++d) {
                int R = P->rails[d], L = P->sites[d];
                int64_t off = dev_offset(P, d);
                const int8_t *Sd = S + off;
                int8_t *Od = occ + off;
                int r_lo = 0, r_hi = R;
                if (opts && opts->rail_hi > opts->rail_lo) {
                    r_lo = opts->rail_lo;
                    r_hi = opts->rail_hi;
                }
                int n_bonds = (L - 1 - h + 1) / 2; /* s = h, h+2, ..., <= L-2 */
                if (n_bonds < 0) n_bonds = 0;
                const orc_electrodes *el =
                    (opts && opts->electrodes && opts->electrodes[d].open) ? &opts->electrodes[d] : NULL;
                if (threaded) {
                    int32_t down = 0, up = 0;
#pragma omp parallel for num_threads(orc_threads) schedule(static) reduction(+ : down, up)
                    for (int r = r_lo; r < r_hi; ++r) {
                        for (int b = 0; b < n_bonds; ++b) {
                            int dir = visit_bond(P, d, R, L, off, Sd, Od, h, n, k, V[d], r, h + 2 * b, log,
                                                 log_cap, n_log, opts, 1);
                            down += dir == 1;
                            up += dir == 2;
                        }
                        for (int side = 0; el && side < 2; ++side) {
                            if (!electrode_in_half_step(side, L, h)) continue;
                            int dir = visit_electrode(P, el, d, R, L, Sd, Od, h, n, V[d], r, side, log, log_cap,
                                                      n_log, 1);
                            down += dir == 1;
                            up += dir == 2;
                        }
                    }
                    n_down[d] += down;
                    n_up[d] += up;
                    continue;
                }
                int64_t m = (int64_t)(r_hi - r_lo) * n_bonds;
                int64_t *perm = NULL;
                if (opts && opts->shuffle_seed) {
                    perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
                    permutation(m, opts->shuffle_seed ^ (uint64_t)(n * 2 + h) ^ ((uint64_t)d << 40), perm);
                }
                for (int64_t idx = 0; idx < m; ++idx) {
                    int64_t b = perm ? perm[idx] : idx;
                    int r = r_lo + (int)(b / n_bonds);
                    int s = h + 2 * (int)(b % n_bonds);
                    int dir = visit_bond(P, d, R, L, off, Sd, Od, h, n, k, V[d], r, s, log, log_cap, n_log,
                                         opts, 0);
                    if (dir == 1) ++n_down[d];
                    else if (dir == 2) ++n_up[d];
                }
                free(perm);
                for (int r = r_lo; el && r < r_hi; ++r)
                    for (int side = 0; side < 2; ++side) {
                        if (!electrode_in_half_step(side, L, h)) continue;
                        int dir = visit_electrode(P, el, d, R, L, Sd, Od, h, n, V[d], r, side, log, log_cap,
                                                  n_log, 0);
                        if (dir == 1) ++n_down[d];
                        else if (dir == 2) ++n_up[d];
                    }
            }
        }
        for (int d = 0; d < D; ++d) {
            int32_t net = n_down[d] - n_up[d];
            if (net_out) net_out[k * D + d] = net;
            if (net_total) net_total[d] += net;
            if (dec_out) {
                int R = P->rails[d], L = P->sites[d];
                const int8_t *Od = occ + dev_offset(P, d);
                int32_t *dk = dec_out + (k * D + d) * 10;
                for (int q = 0; q < 10; ++q) dk[q] = 0;
                for (int r = 0; r < R; ++r)
                    for (int s2 = 0; s2 < L; ++s2)
                        if (Od[(int64_t)r * L + s2]) dk[(10 * s2) / L] += 1;
            }
        }
    }
    free(S);
    free(V);
    free(n_down);
    free(n_up);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Paper-literal zone model (SI S2.1, "Step-by-Step Explanation of the   */
/* Markov Chain Monte Carlo Framework").                                 */
/* ------------------------------------------------------------------ */
/* Zone of column x (1-based) in a rail of `sites` columns cut into `zones`
 * zones of equal width: z = ceil(x / (sites / zones)) = ceil(x zones / sites)
 * (SI S2.1, "Spatial Zones and Local Probabilities"), in 1..zones. */
int orc_zone_index(int x, int sites, int zones)
{
    return (int)(((int64_t)x * zones + sites - 1) / sites);
}

/* The directional probabilities of every zone for bias V and zone
 * populations counts[z-1] (ions of all rails in zone z):
 *   net drop (the implicit space charge: the applied bias less the drop
 *   across the zone due to the ion imbalance of the zones on either side,
 *   scaled by the effective voltage difference factor; a reading, SI S2.1
 *   "Implicit space-charge effects"):
 *     rho_z   = counts_z - N/Z,
 *     dV_net  = V - v_factor (sum_{z' < z} rho_z' - sum_{z' > z} rho_z'),
 *   energy gap (SI Eq. S1):    dE = q dV_net d_hop / t_dev   (q = 1 e),
 *   Boltzmann factor (Eq. S2): B = exp(-dE / kT),
 *   probabilities (Eqs. S3, S4):  P_left = P0 / (1 + B),  P_right = B P_left.
 * "Left" is toward column 1 (the grounded electrode), the direction in
 * which a positive bias drives the cations. */
void orc_zone_table(const orc_zone_params *P, double V, const int64_t *counts, double *p_left,
                    double *p_right, double *dv_net)
{
    int Z = P->zones;
    double total = 0.0;
    for (int z = 0; z < Z; ++z) total += (double)counts[z];
    double mean = total / (double)Z;
    for (int z = 0; z < Z; ++z) {
        double below = 0.0, above = 0.0;
        for (int y = 0; y < z; ++y) below += (double)counts[y] - mean;
        for (int y = z + 1; y < Z; ++y) above += (double)counts[y] - mean;
        double dv = V - P->v_factor * (below - above);
        double dE = dv * P->hop_over_thickness;
        double B = exp(-dE / P->kT);
        p_left[z] = P->p0 / (1.0 + B);
        p_right[z] = B * p_left[z];
        if (dv_net) dv_net[z] = dv;
    }
}

/* The two uniforms of ion j of a rail in step n (SI S2.1, "two independent
 * random matrices"): Philox4x32-10 block at counter (j >> 1, rail, n,
 * 2 << 1) (stream 2, device 0), words 2 (j & 1) and 2 (j & 1) + 1 for the
 * right and the left trial. */
void orc_zone_words(uint64_t seed, int rail, int ion, int64_t n, uint32_t *w_right, uint32_t *w_left)
{
    uint32_t ctr[4] = {(uint32_t)(ion >> 1), (uint32_t)rail, (uint32_t)n, 2u << 1};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    *w_right = out[2 * (ion & 1)];
    *w_left = out[2 * (ion & 1) + 1];
}

/* n_steps steps of the zone model from step n0.  X [rails][ions] holds
 * 1-based columns, strictly increasing along each rail; it is updated in
 * place.  Per step (SI S2.1, in the paper's order):
 *   1. zone populations from X, the bias V(t_n), the table of Eqs. S1-S4;
 *   2. for every ion: its zone, the two uniforms, the gaps to its
 *      neighbours (a virtual ion at column 0 before the first ion and at
 *      sites + 1 after the last: moves stay inside the rail), the masks
 *        M_right = [u_right <= P_right(z) and gap_right > 1],
 *        M_left  = [u_left <= P_left(z) and gap_left > 1],
 *      and the move M_right - M_left;
 *   3. all ions at once: X += move, except that two ions that would land
 *      on the same column (gap 2, the left one moving right and the right
 *      one moving left) both stay (the conflict rule of this reading; the
 *      paper's simultaneous update leaves it open);
 *   4. tallies: net_out[k] = moves toward column 1 minus moves away,
 *      zone_out[k][z] = ions in zone z after the step.
 * Returns 0, or -1 for a step counter beyond 2^32 - 1. */
int orc_zone_run(const orc_zone_params *P, const orc_protocol *protocol, int32_t *X, int64_t n0,
                 int64_t n_steps, int32_t *net_out, int32_t *zone_out, int64_t *net_total)
{
    if (n0 < 0 || n0 + n_steps > (int64_t)0xffffffffLL) return -1;
    int Ny = P->rails, Nr = P->ions, Lx = P->sites, Z = P->zones;
    int64_t *counts = (int64_t *)calloc((size_t)Z, sizeof(int64_t));
    double *pl = (double *)malloc(sizeof(double) * (size_t)Z);
    double *pr = (double *)malloc(sizeof(double) * (size_t)Z);
    int *move = (int *)malloc(sizeof(int) * (size_t)(Nr > 0 ? Nr : 1));
    for (int64_t k = 0; k < n_steps; ++k) {
        int64_t n = n0 + k;
        for (int z = 0; z < Z; ++z) counts[z] = 0;
        for (int i = 0; i < Ny; ++i)
            for (int j = 0; j < Nr; ++j) counts[orc_zone_index(X[(int64_t)i * Nr + j], Lx, Z) - 1] += 1;
        double V = device_voltage(protocol, 0, n, P->dt);
        orc_zone_table(P, V, counts, pl, pr, NULL);
        int32_t net = 0;
        for (int i = 0; i < Ny; ++i) {
            int32_t *row = X + (int64_t)i * Nr;
            for (int j = 0; j < Nr; ++j) {
                int x = row[j];
                int z = orc_zone_index(x, Lx, Z) - 1;
                uint32_t wr, wl;
                orc_zone_words(P->seed, i, j, n, &wr, &wl);
                double ur = ldexp((double)wr, -32), ul = ldexp((double)wl, -32);
                int right_nb = j + 1 < Nr ? row[j + 1] : Lx + 1;
                int left_nb = j > 0 ? row[j - 1] : 0;
                int m_right = ur <= pr[z] && right_nb - x > 1;
                int m_left = ul <= pl[z] && x - left_nb > 1;
                move[j] = m_right - m_left;
            }
            for (int j = 0; j + 1 < Nr; ++j)
                if (move[j] == 1 && move[j + 1] == -1 && row[j + 1] - row[j] == 2) {
                    move[j] = 0;
                    move[j + 1] = 0;
                }
            for (int j = 0; j < Nr; ++j) {
                row[j] += move[j];
                net -= move[j];
            }
        }
        if (net_out) net_out[k] = net;
        if (net_total) *net_total += net;
        if (zone_out) {
            int32_t *zk = zone_out + k * Z;
            for (int z = 0; z < Z; ++z) zk[z] = 0;
            for (int i = 0; i < Ny; ++i)
                for (int j = 0; j < Nr; ++j) zk[orc_zone_index(X[(int64_t)i * Nr + j], Lx, Z) - 1] += 1;
        }
    }
    free(counts);
    free(pl);
    free(pr);
    free(move);
    return 0;
}
