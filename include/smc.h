/*
 * libsmc -- swap Monte Carlo on periodic BCC alloys with a local MLP energy, for AMD
 * Instinct MI355X (gfx950).  C ABI.
 *
 * The method is SMC-X/SMC-AI canonical Monte Carlo (arXiv 2604.08250):
 *   - Algorithm 1 (Sec. III-A): the lattice is cut into link cells; in each sequential
 *     mini-step every link cell tries one nearest-neighbour species swap at the same
 *     offset, the local energies of the affected zone Omega are evaluated before and
 *     after, reduced, and the swap is kept by the Metropolis criterion.
 *   - Sec. II-A: link cells large enough that concurrent trials are independent, which
 *     keeps detailed balance; energies are local and their features computed on the fly.
 *   - Sec. V-A: one MC step (sweep) attempts one swap per site; throughput is counted in
 *     attempts (atom-steps) per second.
 *   - Eqs. (4)-(6), Sec. IV-B: the MLP local energy (here SiLU, two hidden layers).
 *   - Sec. III-A, last paragraphs: the ML model is decoupled from the MC core; here the
 *     model is a caller-owned parameter blob.
 *
 * Conventions shared by every entry point
 *   - Return value: SMC_OK (0) or a negative smc_status.  Nothing aborts or throws across
 *     the ABI.  smc_last_error() gives a message for the last failing call on a context.
 *   - Memory: every large buffer (occupancy, parameters, energy cache, traces) is device
 *     memory owned by the caller, who keeps it alive until smc_destroy.  The library owns
 *     only small tables, packed weight copies, counters and scratch, freed by smc_destroy.
 *   - Streams: all device work is enqueued on the stream given to smc_init.  Calls that
 *     return host values (smc_energy, smc_sweep with stats) synchronise that stream.
 *     Asynchronous device faults are reported as SMC_E_DEVICE by the next synchronising call.
 *   - A context is not thread safe; calls on one context must not overlap.
 *
 * Lattice layout (both ways of the ABI): BCC with Lx x Ly x Lz cubic cells and 2 sites
 * per cell; site index s = ((z*Ly + y)*Lx + x)*2 + b, b = 0 at the cell corner and
 * b = 1 at the body centre; one uint8 species id per site.  Replicas are concatenated
 * in replica order.
 *
 * Features: species ids 0..3 own one one-hot channel each; a species id of 4 (fifth
 * species) has none and contributes zeros.  Neighbour slots follow the coordination
 * shells in ascending distance (8 at a*sqrt(3)/2, 6 at a, 12 at a*sqrt(2)), each shell
 * in lexicographic order of its doubled-coordinate offset (dx, dy, dz).
 *   SMC_FEAT_COUNTS_S12: [one-hot(centre), counts per species in shell 1, in shell 2].
 *   SMC_FEAT_ONEHOT_S123: [one-hot(centre), one-hot(neighbour k) for k = 0..25].
 *
 * Parameter blob (FP32, row-major [out][in]): W0[H][F], b0[H], W1[H][H], b1[H], W2[H],
 * b2[1]; E_j = W2 . silu(W1 . silu(W0 x_j + b0) + b1) + b2 (eV).
 * qSRO blob (FP32, 92 values): V[3][5][5], W[3][5], lambda, C; with n_m^{pp'} the number of
 * pairs of site j with its shell-m neighbours whose species are {p, p'} and pi = n / (pairs in
 * the shell), E_j = sum_{m, p' < p} V[m][p][p'] pi_m^{pp'} + sum_{m, p} W[m][p] (pi_m^{pp})^2
 * + lambda sum_{m, p} W[m][p]^2 + C over species 0..4 (entries of absent species should be 0,
 * they still enter the lambda term).
 *
 * Trial of site i at global sweep t of replica r: Philox4x64-10 with counter
 * (i, t, r, 0) and key (seed, 0) gives (r0, r1, r2, r3); the partner is the shell-1
 * neighbour in slot r0 >> 61; u = ((r1 >> 11) + 1) * 2^-53; theta = -kB T ln u with
 * kB = 8.617333262e-5 eV/K; the swap is accepted iff dE <= theta.  Equal species: no
 * energy evaluation, not accepted, still an attempt.
 *
 * FCC lattice (the paper's physical system, Sec. IV-C; smc_config.lattice = SMC_LATTICE_FCC):
 * cell (x,y,z) holds four sites at doubled coordinates (2x,2y,2z) + (0,0,0), (0,1,1),
 * (1,0,1), (1,1,0) for b = 0..3; s = ((z*Ly + y)*Lx + x)*4 + b.  Shells: 12 at a/sqrt(2),
 * 6 at a, 24 at a*sqrt(3/2), lexicographic within a shell.  Link cells as on BCC with the
 * basis index in the colour: 4 e_x e_y e_z colours (256 for 4x4x4 link cells).  The partner
 * is nearest-neighbour slot floor((r0 >> 32) * 12 / 2^32).
 *   SMC_FEAT_MLPNET_S12: [one-hot(centre), one-hot(neighbour k) for k = 0..17] (76 inputs)
 *   into the MLPNet of Eqs. (4)-(6): h1 = relu(W0 x + b0), h2 = relu(W1 h1 + b1),
 *   h3 = relu(W2 h2 + b2), E = W3 . h3 + b3, hidden = 96; blob W0[96][76], b0[96],
 *   W1[96][96], b1[96], W2[96][96], b2[96], W3[96], b3 (26,113 floats).
 *   SMC_FEAT_QSRO_S123: the qSRO blob above over the FCC shells 1..3.
 */
#ifndef SMC_H
#define SMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smc_ctx smc_ctx;

enum smc_status {
  SMC_OK = 0,
  SMC_E_INVALID = -1,      /* bad argument or configuration */
  SMC_E_UNSUPPORTED = -2,  /* valid request this build does not implement */
  SMC_E_DEVICE = -3,       /* HIP error or device fault */
  SMC_E_STATE = -4,        /* call not allowed in the context's current state */
  SMC_E_NOMEM = -5         /* allocation failed */
};

/* Arithmetic of the energy MLP inside a sweep (pattern: precision). */
enum smc_prec {
  SMC_FP32 = 0,      /* FP32 matrix cores, FP32 accumulation */
  SMC_BF16 = 1,      /* BF16 weights and activations, FP32 accumulation */
  SMC_BF16X3 = 2,    /* split BF16: hi+lo weights and activations, three products */
  SMC_FP8_E4M3 = 3,  /* OCP E4M3 with static per-layer scales, FP32 accumulation */
  SMC_FP64 = 4       /* FP64 throughout (reference mode) */
};

/* Energy model and its inputs.  SMC_FEAT_COUNTS_S12 and SMC_FEAT_ONEHOT_S123 select the MLP
 * (Eqs. (4)-(6)) with those features; SMC_FEAT_QSRO_S123 selects the qSRO model (Eq. 2) over
 * coordination shells 1..3 (hidden is ignored; FP32 or FP64 only). */
enum smc_feat {
  SMC_FEAT_COUNTS_S12 = 0,
  SMC_FEAT_ONEHOT_S123 = 1,
  SMC_FEAT_QSRO_S123 = 2,
  SMC_FEAT_MLPNET_S12 = 3  /* FCC only: the MLPNet of Eqs. (4)-(6), 96 hidden, FP32/BF16/BF16X3/FP64 */
};

/* Lattice of every replica of a context. */
enum smc_lattice { SMC_LATTICE_BCC = 0, SMC_LATTICE_FCC = 1 };

typedef struct {
  int32_t n_replicas;            /* >= 1 */
  const int32_t *cells;          /* host, [n_replicas][3] cubic cells per axis, each >= 4 */
  const double *temperature_K;   /* host, [n_replicas]; +inf accepts every swap */
  int32_t n_species;             /* 2..5 */
  int32_t feature;               /* smc_feat */
  int32_t hidden;                /* H: 64 or 128 (BCC MLP), 96 (FCC MLPNet) */
  int32_t precision;             /* smc_prec */
  uint64_t seed;                 /* Philox key word 0 */
  double guard_eV;               /* FP64 re-decision band |dE - theta| < guard; < 0: default */
  int32_t lattice;               /* smc_lattice; 0 (BCC) for a zero-initialised config */
} smc_config;

/* Optional outputs of smc_sweep.  Host counters accumulate over the sweeps of one call.
 * Device traces hold the last sweep of the call, indexed by trial site. */
typedef struct {
  uint64_t *attempts;      /* host [n_replicas] or NULL */
  uint64_t *diff_species;  /* host [n_replicas] or NULL */
  uint64_t *accepts;       /* host [n_replicas] or NULL */
  uint64_t *rechecks;      /* host [n_replicas] or NULL: trials re-decided in FP64 */
  double *trace_dE;        /* device [N_total] or NULL: dE that decided the trial */
  double *trace_dE_fast;   /* device [N_total] or NULL: dE of the sweep precision */
  uint8_t *trace_flags;    /* device [N_total] or NULL: 1 accept, 2 same species, 4 FP64 */
} smc_stats;

/* Create a context (Algorithm 1 inputs: the lattice sigma0, the link-cell partition it
 * implies, and the model).  occ_dev: uint8 [N_total] occupancy, read and updated in place.
 * params_dev: FP32 blob, read once here (and by smc_set_params).  ecache_dev: float
 * [N_total] per-site local energies, filled here and kept equal to the sweep precision's
 * evaluation of the current occupancy.  hip_stream: hipStream_t or NULL for the null
 * stream.  Sets the global sweep counter to 0 and the running energies to the FP64 total. */
int smc_init(const smc_config *cfg, uint8_t *occ_dev, const float *params_dev,
             float *ecache_dev, void *hip_stream, smc_ctx **out);

/* Run n_sweeps sweeps (Algorithm 1's loop over mini-steps, once per sweep; Sec. V-A).
 * Asynchronous unless stats is non-NULL. */
int smc_sweep(smc_ctx *ctx, int32_t n_sweeps, smc_stats *stats);

/* FP64 energies per replica (host arrays [n_replicas], either may be NULL).  The energy of a
 * configuration is the sum of its local energies (Algorithm 1 reduces local energies over the
 * affected zone; Sec. III-A), so:
 * e_scratch = sum of FP64 local energies of the current occupancy;
 * e_running = initial FP64 total plus every accepted dE.  Synchronises. */
int smc_energy(smc_ctx *ctx, double *e_scratch_host, double *e_running_host);

/* Local energy of every site in the given precision's evaluator: float [N_total] for
 * SMC_FP32/BF16/BF16X3/FP8_E4M3, double [N_total] for SMC_FP64.  Asynchronous. */
int smc_site_energies(smc_ctx *ctx, int32_t precision, void *out_dev);

/* Verification probe: the FP64 energy change of the swap that each listed trial site of
 * `replica` proposes at global sweep `sweep` (its Philox partner), on the current occupancy,
 * by the same FP64 evaluator that re-decides near-threshold trials (affected-zone energies
 * after minus before, Algorithm 1's two reductions over Omega).  Nothing is changed.
 * sites_host: n replica-local site indices; partner_host (nullable) and dE_host: host
 * outputs [n].  Equal species give 0.  On BCC it needs one-hot features and 128 hidden
 * units (else SMC_E_UNSUPPORTED); on FCC both models are supported.  Synchronises. */
int smc_delta_e64(smc_ctx *ctx, int32_t replica, uint64_t sweep, const int64_t *sites_host, int32_t n,
                  int64_t *partner_host, double *dE_host);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): smc_delta_e64 without any allocation, on device
 * arrays.  sites_dev: int64 device [n], replica-local trial sites; partner_dev (nullable): int64
 * device [n]; dE_dev: double device [n].  Same proposals and the same FP64 evaluator as
 * smc_delta_e64 (bit-identical results); a site outside the replica gets partner -1 and dE NaN.
 * Asynchronous on the context's stream: no host synchronisation, no hipMalloc or hipFree.  The
 * work space is a fixed library array of SMC_NOALLOC_MAX_TRIALS queue entries and their FP64
 * row energies (about 8.5 MB) that every GPU the library runs on holds until the process ends;
 * n above the limit gives
 * SMC_E_INVALID, larger batches are split by the caller.  All calls on one GPU share that array
 * and it keeps the last call's contents: calls whose work can overlap on one GPU (other
 * streams, contexts or threads) race, and the caller must order them.  BCC with one-hot
 * features and 128 hidden only (else SMC_E_UNSUPPORTED). */
#define SMC_NOALLOC_MAX_TRIALS 8192
int smc_delta_e64_noalloc(smc_ctx *ctx, int32_t replica, uint64_t sweep, const int64_t *sites_dev, int32_t n,
                          int64_t *partner_dev, double *dE_dev);

/* Replace the model (Sec. III-A: the ML energy model is decoupled from the MC core, so it can
 * be swapped without touching the sweep): re-read params_dev (FP32 blob), re-pack the
 * low-precision copies, refresh the energy cache and reset the running energies to the FP64
 * total.  Asynchronous. */
int smc_set_params(smc_ctx *ctx, const float *params_dev);

/* Re-derive the energy cache and running energies after the caller rewrote occ_dev
 * (e.g. a checkpoint restore).  Asynchronous. */
int smc_refresh(smc_ctx *ctx);

/* Global sweep counter (the Philox counter word 1).  Setting it lets a resumed run
 * continue the same random stream. */
int smc_get_sweep(const smc_ctx *ctx, uint64_t *sweep);
int smc_set_sweep(smc_ctx *ctx, uint64_t sweep);

/* Cumulative counters since smc_init, host array [4][n_replicas]: attempts,
 * different-species attempts, accepted swaps, FP64 re-decisions.  reset != 0 zeroes them
 * after reading.  Synchronises. */
int smc_counters(smc_ctx *ctx, uint64_t *out_host, int32_t reset);

/* Per-kernel timing with HIP events recorded around each launch on the context's stream.
 * enable != 0 starts recording and clears the totals; enable == 0 stops.  smc_kernel_times
 * returns the totals since the last enable: milliseconds inside colour (sweep) kernels and
 * inside FP64 re-decision kernels, and the number of colour-kernel launches.  Synchronises. */
int smc_profile(smc_ctx *ctx, int32_t enable);
int smc_kernel_times(smc_ctx *ctx, double *colour_ms, double *recheck_ms, int64_t *colour_launches);

/* New temperatures (host [n_replicas], >= 0 or +inf) for the following sweeps, e.g. an
 * annealing schedule (the paper anneals its alloy from 2000 K to 1000 K in 250 K steps,
 * Sec. V-F).  The
 * replica table is read by the kernels at run time, so captured sweeps follow the change.
 * Synchronises. */
int smc_set_temperatures(smc_ctx *ctx, const double *temperature_K_host);

/* Warren-Cowley short-range order of one replica's current occupancy: alpha_host [3][S][S]
 * (S = n_species) with alpha_m^{pq} = 1 - P(neighbour in shell m has species q | site has
 * species p) / c_q, c_q the concentration of q; 0 where p or q is absent.  The pair fractions
 * of the qSRO model (Eq. 3) averaged over the lattice.  Pair counts are integers summed on
 * the device; synchronises. */
int smc_warren_cowley(smc_ctx *ctx, int32_t replica, double *alpha_host);

/* Neighbour shells of a lattice (smc_lattice): writes up to max_slots offsets (doubled
 * coordinates, [k][3]) and shell numbers (1-based) in slot order to the host arrays and
 * returns the slot count (26 for BCC, 42 for FCC), or a negative status.  Host only. */
int smc_lattice_shells(int32_t lattice, int32_t *offsets_host, int32_t *shells_host, int32_t max_slots);

/* Sweep strategy (Algorithm 1, Sec. III-A).
 * SMC_STRATEGY_ZONE (default): each trial evaluates the post-swap local energies of its
 *   affected zone Omega (40 sites) and takes the pre-swap ones from the energy cache.
 * SMC_STRATEGY_DOUBLE_LATTICE: the algorithm as the paper writes it: per mini-step the
 *   whole lattice is evaluated before (E0, from sigma0) and after (E1, from the auxiliary
 *   lattice sigma1 in which every trial of the colour has swapped its pair), E1 - E0 is
 *   reduced over each trial's Omega, and accepted pairs are copied from sigma1 to sigma0.
 *   The zone sums keep the zone strategy's order, so both strategies give the same
 *   occupancies and energy cache bit for bit; the double lattice evaluates every site twice
 *   per mini-step.  Needs one-hot features, 128 hidden units and a matrix-core precision (not
 *   SMC_FP64), else SMC_E_UNSUPPORTED; allocates the auxiliary lattice and two energy arrays.
 *   Sweeps with it are submitted per launch (no graph). */
enum smc_strategy { SMC_STRATEGY_ZONE = 0, SMC_STRATEGY_DOUBLE_LATTICE = 1 };
int smc_set_strategy(smc_ctx *ctx, int32_t strategy);
int smc_get_strategy(const smc_ctx *ctx, int32_t *strategy);

/* Batched sweeps.  One launch per colour index covers that colour of every replica whose
 * schedule has it (replicas are independent chains; a replica's colours still run in
 * order).  Without stats, traces or profiling a sweep is replayed from a hipGraph captured
 * once (one host submission per sweep); the sweep counter then advances on the device.
 * smc_use_graph(ctx, 0) forces per-launch submission (results are identical).
 * Kernel variants (link cells per group: 32 or 16; XCD-contiguous or strided group order)
 * give bit-identical results; smc_autotune times all of them on one sweep of the context's
 * current state (restored afterwards), fails with SMC_E_STATE if any variant differs bit for
 * bit, keeps the fastest, and appends it to the JSON-lines cache at cache_path (nullable),
 * where a later call with the same device, precision and replica shapes finds it without
 * timing.  chosen (nullable) receives the variant, ms_per_variant (nullable, [4]) the
 * timings.  Synchronises. */
int smc_use_graph(smc_ctx *ctx, int32_t enable);
int smc_set_variant(smc_ctx *ctx, int32_t variant);
int smc_get_variant(const smc_ctx *ctx, int32_t *variant);
int smc_autotune(smc_ctx *ctx, const char *cache_path, int32_t *chosen, float *ms_per_variant);

/* ---- Differentiation (Sec. IV-B: the energy model is trained by gradient descent with
 * backpropagation; here it is fitted to a synthetic reference Hamiltonian).
 * Snapshots: uint8 device [batch][2 L^3], each a periodic BCC lattice of L cells per axis
 * (4 <= L <= 1024) in the sweep lattice's layout.  Model: the FP32 blob params_dev (same
 * layout as smc_init's), one-hot features, 128 hidden units (else SMC_E_UNSUPPORTED).
 * Arithmetic follows the context's precision: SMC_BF16 runs the matrix cores (BF16 operands,
 * FP32 accumulation); SMC_FP32 and SMC_FP64 run plain per-row evaluators in that precision
 * (reference mode); other precisions give SMC_E_UNSUPPORTED.  Sums over rows are taken in a
 * fixed order, so repeated calls give identical results.  All asynchronous on the context's
 * stream unless stated; work buffers are allocated on first use and kept until smc_destroy. */

/* e_out_dev: double device [batch], S_b = sum over the sites of snapshot b of the local
 * energy (Eqs. (4)-(6)). */
int smc_energy_fwd(smc_ctx *ctx, const uint8_t *snap_dev, int32_t batch, int32_t cells_per_axis,
                   const float *params_dev, double *e_out_dev);

/* Backward of smc_energy_fwd: grad_params_dev (float device [n_params], overwritten) =
 * sum_b grad_e_dev[b] * dS_b/dparams, grad_e_dev double device [batch].  The hand-written
 * reverse pass of the MLP (no autodiff). */
int smc_energy_bwd(smc_ctx *ctx, const uint8_t *snap_dev, int32_t batch, int32_t cells_per_axis,
                   const float *params_dev, const double *grad_e_dev, float *grad_params_dev);

/* One training step on a batch: S = the snapshot energies; loss = mean_b ((S_b - E_b)/N)^2
 * with labels E (label_dev, double device [batch]) and N = 2 L^3; gradient by the backward
 * pass (on the BF16 path one pass gives both S and the per-snapshot gradients, which the loss
 * gradient then weights; S can differ from smc_energy_fwd's in the last bits); Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with step >= 1, learning rate
 * lr > 0) updating params_dev (FP32 masters) and the moments adam_m_dev, adam_v_dev (float
 * device [n_params], zero before step 1) in place.  loss_host (nullable): the loss before
 * the update; giving it synchronises.  Low-precision copies used by sweeps are not touched:
 * call smc_set_params after fitting to sweep with the new model. */
int smc_fit_step(smc_ctx *ctx, const uint8_t *snap_dev, int32_t batch, int32_t cells_per_axis,
                 const double *label_dev, float *params_dev, float *adam_m_dev, float *adam_v_dev,
                 float lr, int32_t step, double *loss_host);

/* Cluster-expansion reference Hamiltonian (the labels of the fit):
 * E = sum over shells m = 1..3 and unordered site pairs at that distance of pair[m-1][p][q]
 *   + sum over items k of J[k] * #{translations of triangle shape triangle[k] whose vertices
 *     0, 1, 2 carry species species[k][0..2]}.
 * Triangle shapes: every point set {0, a, b} with a, b and a - b among the 26 shell-1..3
 * vectors, translated so that its lexicographically smallest point is the origin, written
 * (a, b) with a < b in doubled coordinates, numbered in lexicographic order of (a, b);
 * smc_ce_triangles lists them (44). */
typedef struct {
  int32_t n_species;        /* 2..5 */
  const double *pair;       /* host [3][S][S], symmetric, eV */
  int32_t n_items;
  const int32_t *triangle;  /* host [n_items], index into the shape list */
  const uint8_t *species;   /* host [n_items][3] */
  const double *J;          /* host [n_items], eV */
} smc_ce;

/* e_out_dev: double device [batch], CE energy of each snapshot.  Synchronises. */
int smc_ce_energy(smc_ctx *ctx, const smc_ce *ce, const uint8_t *snap_dev, int32_t batch,
                  int32_t cells_per_axis, double *e_out_dev);

/* Triangle shapes: out_host [max][6] (nullable), count (nullable) = number of shapes. */
int smc_ce_triangles(int32_t *out_host, int32_t max, int32_t *count);

/* Total sites over all replicas, and number of colours (mini-steps) of a replica. */
int smc_n_sites(const smc_ctx *ctx, int64_t *n);
int smc_n_colours(const smc_ctx *ctx, int32_t replica, int32_t *n);

void smc_destroy(smc_ctx *ctx);
const char *smc_last_error(const smc_ctx *ctx);
const char *smc_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif
