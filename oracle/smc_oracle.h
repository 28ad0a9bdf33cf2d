/*
 * Plain CPU oracle of the swap Monte Carlo hot path (test infrastructure only).
 *
 * This library is the slow, obviously correct reference that the HIP path is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product library never links or calls it, and the two
 * share no source.  All floating point is double precision.
 *
 * What it follows (citations are to arXiv 2604.08250):
 *   - Algorithm 1 (Sec. III-A): link-cell partition per mini-step, random swap of the
 *     trial site with a nearest neighbour, local energies before/after, reduction over
 *     the affected zone Omega, Metropolis decision, copy-back of accepted pairs.
 *   - Sec. II-A: link cells chosen so that concurrent trials satisfy detailed balance;
 *     local interaction zones; on-the-fly features.
 *   - Sec. V-A: one MC step (sweep) attempts exactly one trial per site.
 *   - Eqs. (4)-(6), Sec. IV-B: the MLP energy model (here with SiLU and two hidden
 *     layers of equal width; identity/ReLU/square activations exist for pins only).
 * Readings where the paper is silent are listed in the design notes of the repository
 * (lattice indexing, shell order, feature encoding, Philox stream layout, acceptance
 * rule, colour schedule).
 */
#ifndef SMC_ORACLE_H
#define SMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_FEAT_COUNTS_S12 = 0, OR_FEAT_ONEHOT_S123 = 1, OR_FEAT_QSRO_S123 = 2 };
enum { OR_ACT_SILU = 0, OR_ACT_IDENTITY = 1, OR_ACT_RELU = 2, OR_ACT_SQUARE = 3 };
enum { OR_ORDER_SNAPSHOT = 0, OR_ORDER_FORWARD = 1, OR_ORDER_REVERSE = 2, OR_ORDER_GIVEN = 3 };

typedef struct {
  int32_t feature;        /* OR_FEAT_* */
  int32_t hidden;         /* H */
  int32_t act0, act1;     /* activation after layer 0 and layer 1 (OR_ACT_*) */
  const double *params;   /* MLP: W0[H][F], b0[H], W1[H][H], b1[H], W2[H], b2.
                             qSRO: V[3][5][5] (symmetric), W[3][5], lambda, C (92 values). */
} or_model;

typedef struct {
  int64_t site, partner;
  double dE, theta, u;
  int32_t dir, same, accept, colour;
} or_trial_rec;

typedef struct {
  uint64_t attempts, diff_species, accepts;
  double e_run;           /* running FP64 total, advanced by accepted dE */
} or_stats;

/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Geometry: BCC, L[0..2] cubic cells per axis, 2 sites per cell, periodic. */
int64_t or_n_sites(const int32_t L[3]);
void or_site_pos(const int32_t L[3], int64_t s, int32_t P[3]);
int64_t or_site_at(const int32_t L[3], const int32_t P[3]);
void or_shell_table(int32_t off[26 * 3], int32_t shell[26]);
int64_t or_neighbor(const int32_t L[3], int64_t s, int32_t k);
int32_t or_n_inputs(int32_t feature);
int32_t or_n_neighbors_used(int32_t feature);

/* Energy model. */
void or_features(const int32_t L[3], int32_t feature, const uint8_t *occ, int64_t j,
                 int64_t swap_i, int64_t swap_n, double *x);
double or_mlp(const or_model *m, const double *x);
double or_qsro(const int32_t L[3], const double *params, const uint8_t *occ, int64_t j, int64_t swap_i,
               int64_t swap_n);
double or_site_energy(const int32_t L[3], const or_model *m, const uint8_t *occ, int64_t j,
                      int64_t swap_i, int64_t swap_n);
double or_total_energy(const int32_t L[3], const or_model *m, const uint8_t *occ);
void or_all_site_energies(const int32_t L[3], const or_model *m, const uint8_t *occ, double *e);
int32_t or_omega(const int32_t L[3], int32_t feature, int64_t i, int64_t n, int64_t *omega);
double or_delta_e(const int32_t L[3], const or_model *m, const uint8_t *occ, int64_t i, int64_t n);

/* Schedule. */
int32_t or_n_colours(const int32_t L[3]);
int32_t or_colour_of(const int32_t L[3], int64_t s);

/* Trial proposal and Metropolis rule. */
void or_propose(uint64_t seed, int64_t site, int64_t sweep, int64_t replica,
                int32_t *dir, double *u);
double or_theta(double temperature_K, double u);
int32_t or_accept(double dE, double theta);
void or_trial(const int32_t L[3], const or_model *m, const uint8_t *occ, double temperature_K,
              uint64_t seed, int64_t replica, int64_t sweep, int64_t site, or_trial_rec *rec);

/* Sweeps.  trace (optional) is indexed by trial site.  colours_limit < 0 runs every colour. */
int or_sweep(const int32_t L[3], const or_model *m, uint8_t *occ, double temperature_K,
             uint64_t seed, int64_t replica, int64_t sweep, or_stats *st, or_trial_rec *trace,
             int32_t order, const int64_t *given_order, int32_t nthreads, int32_t colours_limit,
             const int8_t *force);
/* force (nullable, [N]): force[s] in {0, 1} replaces the decision of a different-species trial
 * at site s; negative entries leave the Metropolis decision. */
void or_proposals(const int32_t L[3], uint64_t seed, int64_t replica, int64_t sweep, double temperature_K,
                  const int64_t *sites, int64_t n, int32_t *dir, int64_t *partner, double *theta);

/* Observables. alpha is [3][S][S]. */
void or_warren_cowley(const int32_t L[3], const uint8_t *occ, int32_t n_species, double *alpha);

/* FCC lattice with the MLPNet and qSRO models (fcc_oracle.c).  Sites s = ((z*Ly + y)*Lx + x)*4 + b,
 * shells 1-3 = 12 / 6 / 24 neighbours; the MLPNet reads shells 1-2 (76 inputs), qSRO shells 1-3. */
enum { OR_FCC_MLPNET_S12 = 0, OR_FCC_QSRO_S123 = 1 };
typedef struct {
  int32_t model;          /* OR_FCC_* */
  int32_t hidden;         /* H of every hidden layer (MLPNet) */
  const double *params;   /* MLPNet: W0[H][76], b0[H], W1[H][H], b1[H], W2[H][H], b2[H], W3[H], b3.
                             qSRO: V[3][5][5], W[3][5], lambda, C (92 values). */
} or_fcc_model;

int64_t or_fcc_n_sites(const int32_t L[3]);
void or_fcc_site_pos(const int32_t L[3], int64_t s, int32_t P[3]);
int64_t or_fcc_site_at(const int32_t L[3], const int32_t P[3]);
void or_fcc_shell_table(int32_t off[42 * 3], int32_t shell[42]);
int64_t or_fcc_neighbor(const int32_t L[3], int64_t s, int32_t k);
int32_t or_fcc_n_neighbors_used(int32_t model);
int32_t or_fcc_n_inputs(void);
int64_t or_fcc_n_params(const or_fcc_model *m);
void or_fcc_features(const int32_t L[3], const uint8_t *occ, int64_t j, int64_t swap_i, int64_t swap_n,
                     double *x);
double or_fcc_mlpnet(const or_fcc_model *m, const double *x);
double or_fcc_qsro(const int32_t L[3], const double *params, const uint8_t *occ, int64_t j, int64_t swap_i,
                   int64_t swap_n);
double or_fcc_site_energy(const int32_t L[3], const or_fcc_model *m, const uint8_t *occ, int64_t j,
                          int64_t swap_i, int64_t swap_n);
void or_fcc_all_site_energies(const int32_t L[3], const or_fcc_model *m, const uint8_t *occ, double *e);
double or_fcc_total_energy(const int32_t L[3], const or_fcc_model *m, const uint8_t *occ);
int32_t or_fcc_omega(const int32_t L[3], int32_t model, int64_t i, int64_t n, int64_t *omega);
double or_fcc_delta_e(const int32_t L[3], const or_fcc_model *m, const uint8_t *occ, int64_t i, int64_t n);
int32_t or_fcc_n_colours(const int32_t L[3]);
int32_t or_fcc_colour_of(const int32_t L[3], int64_t s);
void or_fcc_propose(uint64_t seed, int64_t site, int64_t sweep, int64_t replica, int32_t *dir, double *u);
int or_fcc_sweep(const int32_t L[3], const or_fcc_model *m, uint8_t *occ, double temperature_K, uint64_t seed,
                 int64_t replica, int64_t sweep, or_stats *st, or_trial_rec *trace, int32_t order,
                 const int64_t *given_order, int32_t nthreads, int32_t colours_limit, const int8_t *force);
void or_fcc_warren_cowley(const int32_t L[3], const uint8_t *occ, int32_t n_species, double *alpha);

/* Differentiation pattern (fit_oracle.c). */
typedef struct {
  int32_t n_species;
  const double *pair;      /* [3][S][S], symmetric; shell m = 1..3 at index m - 1 */
  int32_t n_items;
  const int32_t *offsets;  /* [n_items][6]: canonical triangle, vertices 1 and 2 relative to vertex 0 */
  const uint8_t *species;  /* [n_items][3]: species at vertices 0, 1, 2 */
  const double *J;         /* [n_items] eV */
} or_ce;

int32_t or_ce_triangles(int32_t *out, int32_t max);
double or_ce_site_energy(const int32_t L[3], const or_ce *ce, const uint8_t *occ, int64_t s);
double or_ce_total_local(const int32_t L[3], const or_ce *ce, const uint8_t *occ);
double or_ce_total_brute(const int32_t L[3], const or_ce *ce, const uint8_t *occ);
int64_t or_n_params(const or_model *m);
void or_energy_grad(const int32_t L[3], const or_model *m, const uint8_t *snaps, int32_t batch, double *S,
                    const double *gE, double *grad, int32_t nthreads);
double or_fit_loss_grad(const int32_t L[3], const or_model *m, const uint8_t *snaps, int32_t batch,
                        const double *labels, double *S_out, double *grad, int32_t nthreads);
void or_fit_fd(const int32_t L[3], const or_model *m, const uint8_t *snaps, int32_t batch, const double *labels,
               const int64_t *idx, int32_t n, double h, double *out, int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
