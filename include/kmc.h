/*
 * kmc.h — C ABI of the MI355X rail kinetic Monte Carlo (KMC) hop-step library.
 *
 * The library advances lattices of "rails" (one-dimensional chains of sites,
 * each empty or holding one mobile cation) by the vectorised hop step of the
 * paper's simulator: per-bond barrier and bias energies from the applied field
 * plus the screened Coulomb potential of nearby ions, Arrhenius hop
 * probabilities, a stochastic accept/reject under site exclusion, the occupancy
 * update, and electrode-current / decile tallies (paper: main text section 3,
 * Eq. hop_rate and Eq. 2; Supplementary Information S1-S3, Eqs. S1-S4).
 *
 * Conventions shared by every call:
 *   - Return value: kmc_status, 0 on success, < 0 on error.  Nothing throws or
 *     exits.  kmc_last_error() returns a text for the last error of the calling
 *     thread.  Parameters are validated before any work is enqueued, so a
 *     rejected call leaves the state untouched.  After a HIP runtime error the
 *     context answers KMC_ESTATE until kmc_destroy.
 *   - Device pointers are HIP device memory on the current device, owned by the
 *     caller (for example allocated by PyTorch).  The context borrows them
 *     until kmc_destroy and owns only a small amount of host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     work is enqueued on it; only kmc_read_* synchronise it.
 *   - Lattice layout: devices concatenated, each device [rails][sites]
 *     row-major with the site index fastest; int8 occupancy 0/1.
 *   - Units: SI plus eV (potentials in V, energies in eV, charge q = +1 e).
 */
#ifndef KMC_H
#define KMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kmc_ctx kmc_ctx;

typedef enum {
    KMC_OK = 0,
    KMC_EINVAL = -1,        /* a parameter is out of range or inconsistent    */
    KMC_EUNSUPPORTED = -2,  /* valid, but beyond what this build implements   */
    KMC_EHIP = -3,          /* the HIP runtime reported an error              */
    KMC_ESTATE = -4,        /* the context is poisoned by an earlier HIP error */
    KMC_ETOOSMALL = -5      /* a buffer or workspace is too small             */
} kmc_status;

typedef enum {
    KMC_FP64 = 0,   /* binary64 energies, exponent and probabilities          */
    KMC_FP32 = 1,   /* binary32 energies/probabilities, tables from binary64  */
    KMC_BF16X2 = 2, /* Coulomb term from the potential of every site computed
                       as a matrix product on the MFMA units: kernel values
                       split as BF16 hi + lo, FP32 accumulation; energies and
                       probabilities binary32 (needs the same number of sites,
                       at most 1024, on every device)                          */
    KMC_PHI_FIXED = 3 /* Coulomb term from the potential of every site kept in
                       fixed point (kernel values rounded once to multiples of
                       2^-F V, F <= 52 chosen so that no sum can overflow 63
                       bits; kmc_fixed_potential), updated by every accepted
                       hop; dE_coul = phi(t) - K(1, 0) - phi(o) exact in those
                       units, then energies and probabilities in binary64
                       (per-site barriers are double; at most 2048 sites per
                       rail)                                                   */
} kmc_precision;

/* Physical and numerical parameters (paper SI Table S1 for geometry and
 * filling; the rate law of main text Eq. hop_rate with the field split of
 * Eq. 2 for detailed balance).  Hop probability of a candidate bond whose ion
 * moves from origin site o to the empty target t:
 *     dE = alpha*V*(t-o)/L + sum_{j != o,t} occ_j [K(t-j) - K(o-j)],
 *     p  = min(nu0*dt*exp(-(Ea(o) + dE/2)/kT), 1),
 * with K(ds, dr) = kappa*exp(-d/lambda)/d (kappa/d when lambda == 0),
 * d = sqrt(ds^2 + dr^2), for |ds| <= cutoff_sites and minimal-image rail
 * distance dr <= rail_range (periodic lateral edges, SI S1.4), zero at the
 * origin.  V is the device's bias at the step's time; site 0 faces the
 * grounded electrode, site L-1 the biased one (SI S1.3). */
typedef struct {
    int32_t n_devices;       /* independent devices or replicas, >= 1          */
    const int32_t *rails;    /* host [n_devices], each >= 1                     */
    const int32_t *sites;    /* host [n_devices], each in [2, 4096]             */
    double nu0_hz;           /* attempt frequency                               */
    double ea_ev;            /* barrier when no per-site field is given         */
    double kT_ev;            /* thermal energy, > 0                              */
    double dt_s;             /* time step, > 0                                   */
    double field_coupling;   /* alpha                                           */
    double coulomb_kappa_v;  /* kappa; 0 disables ion-ion coupling              */
    double screening_sites;  /* lambda; 0 = unscreened                          */
    int32_t cutoff_sites;    /* inclusive cutoff along the rail, >= 0           */
    int32_t rail_range;      /* interacting rail distance, 0..4                 */
    int32_t precision;       /* kmc_precision                                    */
    uint64_t seed;           /* Philox4x32-10 key                                */
} kmc_params;

/* One logged near-threshold draw (|u - p| < 1e-6) of device d, step n,
 * half-step h, bond (s, s+1) of rail r. */
typedef struct {
    int32_t d, h;
    int64_t n;
    int32_t r, s;
    double u, p;
} kmc_log_entry;

/* Bytes of device workspace kmc_init_device needs for these parameters
 * (apart from the dense precision, this includes one value of the path's
 * precision per site for the score replay's per-bond Coulomb parts). */
kmc_status kmc_workspace_bytes(const kmc_params *params, size_t *bytes);

/* Create a context (paper SI S2.2 "initialization": geometry, filling and
 * constants fixed before a protocol runs).
 *   occ_dev:  device int8 occupancy of all devices (caller-owned, >= the total
 *             number of sites bytes).  Its content becomes the initial state
 *             (values other than 0 count as occupied); after every
 *             kmc_run_steps it holds the current state again.
 *   ea_dev:   NULL (every barrier = ea_ev) or a device array of per-site
 *             barriers in eV in the occupancy layout, float for KMC_FP32 and
 *             KMC_BF16X2, double for KMC_FP64.  The barrier of a hop is that of
 *             its origin site.
 *   workspace_dev, ws_bytes: device memory of at least kmc_workspace_bytes.
 * The step counter starts at 0 and every device's bias is 0 V until
 * kmc_set_bias_protocol. */
kmc_status kmc_init_device(const kmc_params *params, int8_t *occ_dev, const void *ea_dev,
                           void *workspace_dev, size_t ws_bytes, void *stream, kmc_ctx **out);

/* Random initial placement (paper SI S2.1 "Initialization": the ion count
 * follows the filling fraction and is spread evenly over rails): every rail of
 * device d gets exactly floor(filling[d]*L + 1/2) ions on the sites with the
 * smallest Philox placement words.  filling: host [n_devices], in [0, 1]. */
kmc_status kmc_fill_random(kmc_ctx *ctx, const double *filling);

/* Re-read the state from occ_dev (after the caller wrote a new occupancy). */
kmc_status kmc_load_occupancy(kmc_ctx *ctx);

/* Install the voltage-vs-time profile of one device (device >= 0) or of all
 * devices (device == -1) (paper SI S2.2: the protocol is a complete voltage
 * profile).  Piecewise linear through the knots (t_s[i], v_volt[i]), times
 * relative to the current step, nondecreasing; equal times make a jump
 * (right-continuous); constant before the first and after the last knot.
 * n_knots in [1, 64].  Host arrays, copied before return. */
kmc_status kmc_set_bias_protocol(kmc_ctx *ctx, int32_t device, const double *t_s,
                                 const double *v_volt, int32_t n_knots);

/* Advance every device by n_steps steps (paper SI S2.1, the Monte Carlo loop;
 * each step is two half-steps over even then odd bonds).
 *   net_hops_dev: NULL or device int32 [n_steps][n_devices]: hops toward site
 *                 0 minus hops toward site L-1 in each step.
 *   decile_dev:   NULL or device int32 [n_steps][n_devices][10]: ions in each
 *                 tenth of the rail after each step (SI S3).
 * The step counter advances by n_steps; it must stay below 2^32. */
kmc_status kmc_run_steps(kmc_ctx *ctx, int64_t n_steps, int32_t *net_hops_dev,
                         int32_t *decile_dev);

/* Copy the occupancy to host memory (paper SI S2.1, "movement acceptance and
 * position update": the state after the accepted moves of every step; an ion
 * on each occupied site, the caller's layout above).  dst_host: host memory
 * of at least `bytes` >= total sites bytes, not owned by the library.
 * Synchronises the stream.  Errors: KMC_EINVAL for NULL dst_host,
 * KMC_ETOOSMALL when bytes < total sites (nothing copied), KMC_EHIP when a
 * persistent launch reported a failed neighbour wait (the context is then
 * poisoned), KMC_ESTATE on a poisoned context. */
kmc_status kmc_read_occupancy(kmc_ctx *ctx, int8_t *dst_host, size_t bytes);

/* Electrode current and totals since init (paper SI S3, conversion to
 * current: the observable is the charge moved through the device; here the
 * Ramo-Shockley current of blocking electrodes, I = e*net/(L*dt) per step,
 * with net = hops toward site 0 minus hops toward site L-1).  Host outputs,
 * each may be NULL: mean_current_A [n_devices] (the mean over every step run
 * since init), net_hops_total [n_devices], sim_time_s (step counter * dt).
 * Synchronises the stream.  Errors: as kmc_read_occupancy (KMC_EHIP,
 * KMC_ESTATE). */
kmc_status kmc_read_current(kmc_ctx *ctx, double *mean_current_A, int64_t *net_hops_total,
                            double *sim_time_s);

/* Copy up to `cap` logged near-threshold draws to host memory and report how
 * many were logged since init (entries past the device log capacity are
 * counted but not stored).  Synchronises. */
kmc_status kmc_read_threshold_log(kmc_ctx *ctx, kmc_log_entry *dst_host, int64_t cap,
                                  int64_t *n_events);

/* Score-function (likelihood-ratio) gradient of a weighted observable, by
 * replaying the steps [step0, step0 + n_steps) from the state occ0.  Every hop
 * decision y ~ Bernoulli(p) of the replay, with p of the rate law above (main
 * text Eq. hop_rate with the half-energy shift of Eq. 2), contributes
 *     W[k][d] * g_theta * (y - p)/(1 - p)     (0 when p is clamped at 1)
 * to grad[d][theta], k = step - step0, where g_theta = d log p / d theta for
 *     theta = 0: a common shift of every barrier Ea   g = -1/kT
 *             1: nu0                                 g = 1/nu0
 *             2: kappa                               g = -(dE_coul/kappa)/(2 kT)
 *             3: alpha (field_coupling)              g = -V (t - o)/(2 L kT).
 * With W[k][d] = sum_{k' >= k} w[k'] (f_d(k') - b(k')) for an observable f
 * measured after each step, a weight w and a baseline b independent of the
 * replica, the sum is an unbiased estimate of d E[sum_k w[k] f(k)] / d theta.
 *   occ0_dev:   device int8 [total sites], caller layout: the state before
 *               step step0 (for example a copy taken before kmc_run_steps).
 *   weight_dev: device binary64 [n_steps][n_devices].
 *   grad_dev:   device binary64 [n_devices][4], overwritten.
 * The replay uses the protocol installed now (its knots and install step)
 * and the context's parameters; it takes the same decisions as kmc_run_steps
 * from the same state and steps (the Philox stream is a function of the step
 * index).  The context's own state, step counter and tallies are not touched.
 * The hop probability of every candidate is evaluated in full: the Coulomb
 * part of dE is phi(t) - K(1, 0) - phi(o), phi being the window sum of the
 * interaction kernel over the occupied sites, summed in binary64 and rounded
 * once to the path's precision.  It is kept for every bond (computed from
 * occ0, and recomputed after each half-step for the bonds whose window an
 * accepted hop changed); the rest of dE and p are evaluated in the path's
 * precision, and the terms are summed in binary64 (sum order not fixed).  The
 * per-bond values and the hop list live in the workspace.
 * With a recording (kmc_record_hops) that began at step0, whose steps up to
 * step0 + n_steps have been run, and whose start state equals occ0 (checked
 * on the device), each half-step whose list did not overflow takes the
 * forward's decisions from the recording instead of drawing them again: the
 * same decisions and the same terms, summed in another order.  The call then
 * synchronises the stream once (to read the lists' counts).
 * Errors: KMC_EINVAL for NULL pointers, negative indices, coulomb_kappa_v == 0
 * or nu0_hz <= 0; KMC_EUNSUPPORTED if step0 + n_steps exceeds 2^32 - 1. */
kmc_status kmc_score_replay(kmc_ctx *ctx, const int8_t *occ0_dev, int64_t step0, int64_t n_steps,
                            const double *weight_dev, double *grad_dev);

/* Bytes of the caller's buffer for kmc_record_hops(max_steps, cap) (0 when
 * max_steps is 0).  Errors as kmc_record_hops's argument checks. */
kmc_status kmc_record_bytes(kmc_ctx *ctx, int64_t max_steps, int64_t cap, size_t *bytes);

/* Records the accepted hops of the next steps for the score replay (the
 * decisions of SI S2.1, movement acceptance, of the steps that
 * kmc_run_steps takes), so that kmc_score_replay of those steps need not
 * draw them again.  From the context's current step n0 and state, every
 * accepted hop of the steps [n0, n0 + max_steps) that later kmc_run_steps
 * calls take (in any launch strategy) is appended to the list of its
 * half-step, cap entries each; a list that overflows is kept as overflowed,
 * and the replay then draws that half-step's decisions again.
 *   buf_dev:  device memory of kmc_record_bytes(max_steps, cap) bytes,
 *             256-byte aligned, owned by the caller, which keeps it until the
 *             recording ends.  It holds the per-half-step counts, a copy of
 *             the state at n0 (caller layout) and the lists.
 *   bytes:    its size.
 *   max_steps, cap: steps covered and entries per half-step list (>= 1).
 *   max_steps == 0 or buf_dev == NULL ends the recording.
 * Installing a protocol, loading, filling or restoring the occupancy,
 * opening or closing electrodes, autotuning and a new kmc_record_hops end
 * the recording.  Enqueued on the context's stream.
 * Errors: KMC_EINVAL for negative sizes, cap < 1, a small or misaligned
 * buffer or a product max_steps * cap too large; KMC_EUNSUPPORTED for
 * KMC_BF16X2 and KMC_PHI_FIXED contexts, while any device has open
 * electrodes, or when n0 + max_steps would reach 2^32. */
kmc_status kmc_record_hops(kmc_ctx *ctx, void *buf_dev, size_t bytes, int64_t max_steps, int64_t cap);

/* kmc_score_replay for callers that cannot allocate device memory where they
 * call (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same replay, the same arguments and results, but
 * the replay's own buffers (two state planes, the per-bond Coulomb parts, the
 * accepted-hop list and its counters) live in a static device array of
 * 64 MiB per GPU that the library holds until the process ends, instead of
 * in the context's workspace.  The call allocates nothing.  Call it with the
 * context's device current.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (on other streams or threads) race.
 * Errors: as kmc_score_replay, plus KMC_EUNSUPPORTED when the lattice needs
 * more than the array holds (about 10 million sites in binary32, 6 million
 * in binary64; the message gives both sizes) and KMC_EHIP when the array's
 * device address cannot be looked up. */
kmc_status kmc_score_replay_noalloc(kmc_ctx *ctx, const int8_t *occ0_dev, int64_t step0, int64_t n_steps,
                                    const double *weight_dev, double *grad_dev);

/* Coulomb potential of the current state at every site, as used by the
 * KMC_BF16X2 step: phi(r, s) = sum over the distinct rails r' within
 * rail_range (r included) and sites j of occ(r', j) K(s - j, dist(r, r')),
 * K(0, 0) = 0 (the ion field of main text section 3; the hop o -> t then has
 * dE_coul = phi(t) - K(1, 0) - phi(o)).  K is split as BF16 hi + lo with
 * |K - hi - lo| <= 2^-16 |K|, products accumulated in FP32.
 *   phi_dev: device float [total sites], occupancy layout (written).
 * KMC_EUNSUPPORTED unless the context was created with KMC_BF16X2. */
kmc_status kmc_dense_potential(kmc_ctx *ctx, float *phi_dev);

/* Open electrodes of one device (device >= 0) or of all devices (-1); an
 * extension of the paper's model, whose electrodes block ions (SI S1.3) and
 * whose rails keep their ion count (SI S2.1), in the direction its
 * conclusion invites (new mechanisms by altering the probabilities at a few
 * positions).  With open = 1 each rail end is one more bond of the
 * checkerboard, to a reservoir of ions: the grounded reservoir behind site 0
 * (bond (-1, 0), half-step 1) and the biased one behind site L-1 (bond
 * (L-1, L), half-step (L-1) mod 2).  A reservoir ion has the energy mu plus
 * its bias energy at the virtual site (-1 or L) and no Coulomb interaction.
 * A transfer between the boundary site x and its reservoir has
 *     dE = (alpha V (t - o)/L + s phi(x)) - s mu,  s = +1 injection, -1 extraction,
 * with o, t the origin and target (virtual site included) and phi(x) the
 * Coulomb potential of the other ions at x (the hop's kernel and window), and
 * the rate law of a hop with the electrode's barrier ea in place of Ea(o).
 * Transfers count in the net tallies and the current like hops (toward site
 * 0's side positive), and in the deciles; the ion count is then free.  Draws:
 * Philox4x32-10 at counter (0, r, n, 16 d + 6 + h), word 0 (grounded side) or
 * 1 (biased side).  While any device has open electrodes every run uses the
 * half-step strategy, and kmc_score_replay returns KMC_EUNSUPPORTED.
 *   ea_*, mu_*: eV, finite.  open: 0 (blocking, the default) or 1.
 * KMC_EUNSUPPORTED for KMC_BF16X2 and KMC_PHI_FIXED contexts.  Synchronises. */
kmc_status kmc_set_electrodes(kmc_ctx *ctx, int32_t device, int32_t open, double ea_ground, double mu_ground,
                              double ea_bias, double mu_bias);

/* The potential of the current state at every site, as used by the
 * KMC_PHI_FIXED step (the ion field of main text section 3, defined as for
 * kmc_dense_potential), in units of 2^-frac_bits V: phi(r, s) = sum of
 * round(K(s - j, dist) 2^frac_bits) over the ions j of the distinct rails
 * within rail_range.  The sum is an exact integer sum, so the potential kept
 * up to date hop by hop and the one computed from scratch are equal.
 *   phi_dev:    device int64 [total sites], occupancy layout (written).
 *   recompute:  0 returns the potential the step uses (kept up to date hop by
 *               hop); 1 computes it from scratch from the current state
 *               (the context's own copy is left as it is).
 *   frac_bits:  host, receives F (may be NULL).
 * Enqueued on the context's stream (no synchronisation).  KMC_EUNSUPPORTED
 * unless the context was created with KMC_PHI_FIXED. */
kmc_status kmc_fixed_potential(kmc_ctx *ctx, int64_t *phi_dev, int32_t recompute, int32_t *frac_bits);

/* Relaxation time of a decay curve (main text section 4, relaxation decay:
 * once the bias is removed the fraction of ions in the first decile decays as
 * a single exponential towards an asymptote every run shares; SI S5, current
 * relaxation).  Least-squares fit, in binary64 on the host, of
 *     m(t) = C + A exp(-(t - t0)/tau)
 * to the n samples (t[i], m[i]) (for example the replica mean of the decile
 * fraction over the relaxation window, t0 the end of the bias pulse), by
 * Gauss-Newton iteration.
 *   t, m:    host [n], n >= 4, finite, not every t equal to t0.
 *   params:  host [3].  In: a starting point (C, A, tau) when all three are
 *            finite and tau > 0, else ignored.  Out: the fitted (C, A, tau).
 *   weights: NULL or host [n]: d tau / d m[i] at the fit, from the
 *            implicit-function theorem on the fit's stationarity condition
 *            (the weights that turn a gradient of the samples into a gradient
 *            of tau).
 * Touches no context and no device memory.  Errors: KMC_EINVAL for bad
 * arguments, KMC_EUNSUPPORTED when the iteration finds no minimum with
 * tau > 0 (params and weights are then left unspecified). */
kmc_status kmc_fit_decay(const double *t, const double *m, int64_t n, double t0, double *params,
                         double *weights);

/* Launch strategy of kmc_run_steps.
 *   KMC_LAUNCH_HALF_STEP: one kernel launch per half-step; the state makes a
 *     round trip through device memory every half-step.  Always available.
 *   KMC_LAUNCH_PERSISTENT: one launch per chunk of up to 1024 steps and group
 *     of devices; every workgroup keeps its tile of rails in LDS and exchanges
 *     only its edge rails with its two neighbouring tiles.  Needs every single
 *     device's tiling co-resident on the GPU; larger batches of devices run as
 *     several launches per chunk, one per group of whole devices.
 *   KMC_LAUNCH_WAVE: persistent like KMC_LAUNCH_PERSISTENT, but every tile is
 *     one wavefront that keeps its rails' occupancy in registers (16 or 32
 *     sites per lane, so rails of up to 2048 padded sites), so a half-step has
 *     no workgroup barrier; neighbouring tiles exchange edge rails only after
 *     half-steps that changed them.  Needs every device's rails to fit 64
 *     lanes (at least max(rail_range, 1) rails per tile unless the device is
 *     one tile) and every single device's tiling co-resident.
 *   KMC_LAUNCH_AUTO (default): WAVE when it fits, else PERSISTENT when it
 *     fits, else HALF_STEP.
 * All give bit-identical trajectories. */
typedef enum {
    KMC_LAUNCH_AUTO = 0,
    KMC_LAUNCH_HALF_STEP = 1,
    KMC_LAUNCH_PERSISTENT = 2,
    KMC_LAUNCH_WAVE = 3
} kmc_launch_mode;

/* Select the launch strategy; KMC_EUNSUPPORTED if PERSISTENT or WAVE does not
 * fit. */
kmc_status kmc_set_launch_mode(kmc_ctx *ctx, int32_t mode);

/* The strategy kmc_run_steps will use now (HALF_STEP, PERSISTENT or WAVE). */
kmc_status kmc_get_launch_mode(kmc_ctx *ctx, int32_t *mode);

/* Number of launches per 1024-step chunk of the strategy in use (PERSISTENT
 * or WAVE): the devices are split into groups of whole devices whose tiles
 * are co-resident on the GPU (0 for HALF_STEP). */
kmc_status kmc_get_persistent_groups(kmc_ctx *ctx, int32_t *groups);

/* Cap the number of tiles of one persistent launch (0 = as many as are
 * co-resident): workgroups of KMC_LAUNCH_PERSISTENT, wavefronts of
 * KMC_LAUNCH_WAVE.  For example to leave room for other work on the GPU.  A
 * strategy under which one device no longer fits a launch becomes
 * unavailable, and a mode that selected it falls back to KMC_LAUNCH_AUTO.
 * Waits for the work already enqueued.  Trajectories do not depend on it. */
kmc_status kmc_set_persistent_group_limit(kmc_ctx *ctx, int32_t max_tiles);

/* Polls before a neighbour wait of a persistent strategy is declared hung
 * (default 2^20, about a second); 0 makes every wait fail at once.  A wait
 * declared hung stops the launch cleanly: every tile leaves its loop, the
 * kernel ends, and the next read_* call returns KMC_EHIP and poisons the
 * context (the state is invalid).  For tests of that path and for callers
 * that prefer a shorter bound.  Takes effect for launches enqueued after it. */
kmc_status kmc_set_wait_limit(kmc_ctx *ctx, int32_t polls);

/* Target number of (padded) sites per workgroup tile, 0 = built-in default,
 * else in [16, 65536]; tiles are whole rails.  For KMC_LAUNCH_WAVE, 1024 and
 * 2048 select 16 and 32 sites per lane (other values: 16 when that tiling
 * exists, else 32).  Used by the autotuner.  Waits for the
 * work already enqueued.  Trajectories do not depend on it. */
kmc_status kmc_set_tile_sites(kmc_ctx *ctx, int32_t sites);

/* Pick the launch strategy and tile size by timing trial runs of
 * trial_steps steps (1..65536) for each candidate (wave tiles of 16 and 32
 * sites per lane and persistent with several tile sizes when they fit,
 * half-step launches with several tile sizes).  The
 * state, step counter, tallies and log are restored after every trial and at
 * the end, so tuning changes no trajectory; the fastest configuration stays
 * selected.  Outputs (each may be NULL): the chosen tile size (0 = default),
 * strategy (kmc_launch_mode) and its time per step in microseconds.
 * Synchronises; KMC_EUNSUPPORTED if the trials would take the step counter
 * past 2^32. */
kmc_status kmc_autotune(kmc_ctx *ctx, int32_t trial_steps, int32_t *tile_sites, int32_t *mode,
                        double *us_per_step);

/* Current step counter. */
kmc_status kmc_get_step(kmc_ctx *ctx, int64_t *step);

/* ------------------------------------------------------------------------
 * The paper's own zone model (SI S2.1, "Step-by-Step Explanation of the
 * Markov Chain Monte Carlo Framework"), beside the per-site hop step above.
 * The state is the ion-position matrix X [rails][ions_per_rail]: the 1-based
 * column of every ion, strictly increasing along its rail.  The rail of
 * `sites` columns is cut into `zones` zones of equal width, zone
 * z = ceil(X / (sites / zones)).  Per step (in this order):
 *   - the bias V(t_n) of the installed protocol, t_n = (n - n_install) dt_s;
 *   - per zone the net drop with the implicit space charge (a reading of the
 *     paper's "effective voltage difference factor"):
 *       dV_net(z) = V - v_factor (sum_{z'<z} rho_z' - sum_{z'>z} rho_z'),
 *       rho_z = (ions in zone z, all rails) - (all ions) / zones;
 *   - the energy gap dE = dV_net hop_over_thickness (Eq. S1 with q = 1 e and
 *     hop_over_thickness = d_hop / t_dev), B = exp(-dE / kT) (Eq. S2),
 *     P_left = p0 / (1 + B), P_right = B P_left (Eqs. S3, S4); "left" is
 *     toward column 1, the grounded electrode;
 *   - for every ion two uniforms (Philox4x32-10 block at counter
 *     (j >> 1, rail, n, 4), words 2 (j & 1) and 2 (j & 1) + 1 for the right
 *     and the left trial), the masks [u <= P] and [gap to the neighbour > 1]
 *     (a virtual neighbour at column 0 and at sites + 1), the move
 *     M_right - M_left, all ions at once; two ions that would land on one
 *     column (gap 2, moving toward each other) both stay.
 * All arithmetic of the table in binary64.  kmc_zone_ctx is opaque. */
typedef struct kmc_zone_ctx kmc_zone_ctx;

typedef struct {
    int32_t rails;               /* N_y >= 1                                  */
    int32_t sites;               /* L_x in [2, 65534]                         */
    int32_t ions_per_rail;       /* N_r in [0, min(64, sites)], every rail    */
    int32_t zones;               /* Z in [1, 64] (the paper: 10)              */
    double p0;                   /* baseline hop probability, [0, 1]          */
    double kT_ev;                /* k_B T, eV, > 0                            */
    double hop_over_thickness;   /* d_hop / t_dev (1 / sites when the rail
                                    spans the device)                         */
    double v_factor;             /* effective voltage difference factor, V per
                                    ion of zone imbalance (the paper: 5e-5)   */
    double dt_s;                 /* time per step, s (the protocol's clock)   */
    uint64_t seed;               /* Philox4x32-10 key                         */
} kmc_zone_params;

/* Device workspace bytes for kmc_zone_init. */
kmc_status kmc_zone_workspace_bytes(const kmc_zone_params *params, size_t *bytes);

/* Create a zone-model context (paper SI S2.1 "Initialization", SI S2.2).
 *   occ_dev: device int8 [rails][sites] occupancy, caller-owned; every rail
 *            must hold exactly ions_per_rail ions (else KMC_EINVAL).  It
 *            becomes the initial state, and after every kmc_zone_run_steps
 *            it holds the current state again.
 *   workspace_dev: device memory of kmc_zone_workspace_bytes, 256-byte
 *            aligned, caller-owned.
 * The step counter starts at 0 and the bias is 0 V.  Synchronises. */
kmc_status kmc_zone_init(const kmc_zone_params *params, int8_t *occ_dev, void *workspace_dev, size_t ws_bytes,
                         void *stream, kmc_zone_ctx **out);

/* Re-read the state from occ_dev (same rules as at init).  The ion counts
 * are checked before anything is written: on KMC_EINVAL the context's state
 * (positions, populations, step) is unchanged.  Synchronises. */
kmc_status kmc_zone_load_occupancy(kmc_zone_ctx *ctx);

/* Install the voltage-vs-time profile (SI S2.2), piecewise linear through the
 * knots as kmc_set_bias_protocol, times relative to the current step. */
kmc_status kmc_zone_set_bias_protocol(kmc_zone_ctx *ctx, const double *t_s, const double *v_volt,
                                      int32_t n_knots);

/* Advance n_steps steps (SI S2.1, the loop; one kernel launch per step).
 *   net_dev:  NULL or device int32 [n_steps]: moves toward column 1 minus
 *             moves toward column `sites` in each step.
 *   zone_dev: NULL or device int32 [n_steps][zones]: ions in each zone after
 *             each step (with 10 zones, the deciles of SI S3). */
kmc_status kmc_zone_run_steps(kmc_zone_ctx *ctx, int64_t n_steps, int32_t *net_dev, int32_t *zone_dev);

/* Copy X to host int32 [rails][ions_per_rail] (count >= rails * ions).
 * Synchronises. */
kmc_status kmc_zone_read_positions(kmc_zone_ctx *ctx, int32_t *X_host, size_t count);

/* Current step counter of a zone-model context. */
kmc_status kmc_zone_get_step(kmc_zone_ctx *ctx, int64_t *step);

/* Release a zone-model context (enqueued work is completed first). */
void kmc_zone_destroy(kmc_zone_ctx *ctx);

/* SHA-1 (hex) of the sources and build flags this library was built from,
 * so that a loader can refuse a library older than its sources. */
const char *kmc_build_hash(void);

/* Text of the last error of the calling thread ("" if none). */
const char *kmc_last_error(void);

/* Release the context (enqueued work is completed first). */
void kmc_destroy(kmc_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* KMC_H */
