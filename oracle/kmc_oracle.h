/*
 * Plain CPU oracle for the rail-KMC hop step: declarations.
 * TEST INFRASTRUCTURE ONLY (see kmc_oracle.c).  Private to oracle/.
 */
#ifndef KMC_ORACLE_H
#define KMC_ORACLE_H
#include <stdint.h>

typedef struct {
    int n_devices;
    const int *rails;      /* [n_devices] */
    const int *sites;      /* [n_devices] */
    double nu0;            /* attempt frequency, Hz */
    double ea;             /* barrier, eV (used when ea_site == NULL) */
    double kT;             /* eV */
    double dt;             /* s */
    double alpha;          /* field coupling (dimensionless) */
    double kappa;          /* Coulomb amplitude, V */
    double lambda;         /* screening length in sites; 0 = unscreened */
    int cutoff;            /* inclusive cutoff along the rail, sites */
    int rail_range;        /* rails within this minimal-image distance interact */
    int fp32;              /* 0 = binary64 path, 1 = binary32 path */
    uint64_t seed;
    const double *ea_site; /* NULL or per-site barrier, devices concatenated */
} orc_params;

typedef struct {
    const double *t;   /* knot times, s, nondecreasing */
    const double *v;   /* knot voltages, V */
    int n_knots;
    int64_t n_set;     /* step at which the protocol was installed */
} orc_protocol;

typedef struct {
    int32_t d, h;
    int64_t n;
    int32_t r, s;
    double u, p;
} orc_log_entry;

/* Open electrodes of one device (NULL electrodes or open == 0: the paper's
 * blocking electrodes, a fixed ion count per rail).  Each end of a rail is
 * coupled to a reservoir of ions: the grounded one behind site 0 (a virtual
 * site -1) and the biased one behind site L-1 (a virtual site L).  An ion
 * in a reservoir has the energy mu (plus its bias energy at the virtual
 * site) and no Coulomb interaction; a transfer across the boundary bond
 * crosses the barrier ea of that electrode. */
typedef struct {
    int open;
    double ea_ground, mu_ground;   /* eV, the grounded electrode (site 0 side) */
    double ea_bias, mu_bias;       /* eV, the biased electrode (site L-1 side) */
} orc_electrodes;

typedef struct {
    uint64_t shuffle_seed; /* nonzero: visit bonds in a random order */
    int rail_lo, rail_hi;  /* rail_hi > rail_lo: update only these rails */
    /* score-function accumulation (all NULL: none).  score_w [n_steps][D]
     * weights of the decisions of each step; score_grad, score_mag and
     * score_sens [D][4] are accumulated into (theta = Ea shift, nu0, kappa,
     * alpha).  Needs kappa != 0 and nu0 > 0. */
    const double *score_w;
    double *score_grad;
    double *score_mag;
    double *score_sens;
    /* Tolerance diagnostics for a replay whose Coulomb part is summed in
     * another order (all optional, NULL: not accumulated).  Per decision with
     * p < 1 and base_q = |W g_q| p/(1-p)^2:
     *   score_sens_arg [D][4]: base_q |beta (Ea + dE/2)|, the scale of a
     *     rounding difference in the exponent's argument;
     *   score_sens_b [D][4]: (base_q beta/2 + [q = kappa] |W beta/(2 kappa)|
     *     |(y - p)/(1 - p)|) B with B = A + |dE| + |e_coul| + 2 |K(1, 0)| and A
     *     the sum over the occupied window sites of |K(t - j)| + |K(o - j)|
     *     (binary64), the scale of a difference in the summed Coulomb part;
     *   score_hops [D]: accepted hops. */
    double *score_sens_arg;
    double *score_sens_b;
    int64_t *score_hops;
    /* nonzero: in the binary32 path the score terms use the Coulomb part
     * summed in binary64 and rounded once to binary32 (the decisions still
     * use the binary32 sum) */
    int score_coul64;
    /* NULL, or [n_devices] electrodes (see orc_electrodes); not with the
     * score accumulation */
    const orc_electrodes *electrodes;
} orc_run_opts;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint32_t orc_hop_word(uint64_t seed, int d, int64_t n, int r, int s);
uint32_t orc_place_word(uint64_t seed, int d, int r, int s);
uint32_t orc_electrode_word(uint64_t seed, int d, int64_t n, int r, int h, int side);
double orc_electrode_delta_energy(const orc_params *P, int R, int L, const int8_t *S, int r, int side,
                                  int inject, double V, double mu);
double orc_kernel(const orc_params *P, int ds, int dr);
double orc_protocol_voltage(const double *t_k, const double *v_k, int n_knots, double t_rel);
double orc_delta_energy_f64(const orc_params *P, int R, int L, const int8_t *S,
                            int r, int o, int t, double V);
float orc_delta_energy_f32(const orc_params *P, int R, int L, const int8_t *S,
                           int r, int o, int t, double V);
void orc_dense_potential(const orc_params *P, const int8_t *occ, double *phi);
double orc_hop_prob_f64(const orc_params *P, double ea, double dE);
float orc_hop_prob_f32(const orc_params *P, double ea, float dE);
int orc_ions_per_rail(double filling, int L);
void orc_fill(const orc_params *P, const double *filling, int8_t *occ);
void orc_set_threads(int n);
int orc_run(const orc_params *P, const orc_protocol *protocols, int8_t *occ,
            int64_t n0, int64_t n_steps, int32_t *net_out, int32_t *dec_out,
            int64_t *net_total, orc_log_entry *log, int64_t log_cap, int64_t *n_log,
            const orc_run_opts *opts);

/* Paper-literal zone model (SI S2.1): every rail holds `ions` ions at
 * 1-based columns 1..sites (the ion-position matrix X), the lattice is cut
 * into `zones` zones of equal width, and each zone has its own pair of
 * directional hop probabilities per step. */
typedef struct {
    int rails;                  /* N_y */
    int ions;                   /* N_r, ions per rail */
    int sites;                  /* L_x, columns per rail */
    int zones;                  /* Z */
    double p0;                  /* baseline hop probability P0 per ion and step */
    double kT;                  /* k_B T, eV */
    double hop_over_thickness;  /* d_hop / t_dev */
    double v_factor;            /* effective voltage difference factor, V per ion of zone imbalance */
    double dt;                  /* time per step, s (protocol time t_n = n dt) */
    uint64_t seed;
} orc_zone_params;

int orc_zone_index(int x, int sites, int zones);
void orc_zone_table(const orc_zone_params *P, double V, const int64_t *counts, double *p_left,
                    double *p_right, double *dv_net);
void orc_zone_words(uint64_t seed, int rail, int ion, int64_t n, uint32_t *w_right, uint32_t *w_left);
int orc_zone_run(const orc_zone_params *P, const orc_protocol *protocol, int32_t *X, int64_t n0,
                 int64_t n_steps, int32_t *net_out, int32_t *zone_out, int64_t *net_total);

#endif
