/*
 * Plain CPU oracle of the swap Monte Carlo hot path on the FCC lattice -- TEST
 * INFRASTRUCTURE ONLY.  The paper's physical system is FCC (Sec. IV-C) and its neural
 * energy model is MLPNet (Eqs. (4)-(6)); this file applies Algorithm 1 to that lattice
 * and model the same slow, direct way as the BCC oracle: every local energy recomputed
 * from its definition before and after a swap, in double precision, no caches.
 * Citations are to arXiv 2604.08250.  The product library shares no code with this file.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "smc_oracle.h"

/* ------------------------------------------------------------------------------------
 * FCC geometry in doubled integer coordinates: cell (x,y,z) holds four basis sites at
 * (2x,2y,2z) + {(0,0,0), (0,1,1), (1,0,1), (1,1,0)} for b = 0..3; a doubled position is
 * a lattice site iff its coordinate sum is even.  Periodic modulo 2L per axis.
 * Canonical site index s = ((z*Ly + y)*Lx + x)*4 + b.
 * ---------------------------------------------------------------------------------- */
static const int32_t kFccBasis[4][3] = {{0, 0, 0}, {0, 1, 1}, {1, 0, 1}, {1, 1, 0}};

int64_t or_fcc_n_sites(const int32_t L[3]) { return 4LL * L[0] * L[1] * L[2]; }

void or_fcc_site_pos(const int32_t L[3], int64_t s, int32_t P[3]) {
  int32_t b = (int32_t)(s % 4);
  int64_t c = s / 4;
  int32_t x = (int32_t)(c % L[0]);
  int32_t y = (int32_t)((c / L[0]) % L[1]);
  int32_t z = (int32_t)(c / ((int64_t)L[0] * L[1]));
  P[0] = 2 * x + kFccBasis[b][0];
  P[1] = 2 * y + kFccBasis[b][1];
  P[2] = 2 * z + kFccBasis[b][2];
}

static int32_t fcc_wrap(int32_t v, int32_t m) {
  int32_t r = v % m;
  return r < 0 ? r + m : r;
}

int64_t or_fcc_site_at(const int32_t L[3], const int32_t P[3]) {
  int32_t q[3];
  for (int a = 0; a < 3; ++a) q[a] = fcc_wrap(P[a], 2 * L[a]);
  if ((q[0] + q[1] + q[2]) % 2 != 0) return -1;
  int32_t b = -1;
  for (int k = 0; k < 4; ++k)
    if ((q[0] & 1) == kFccBasis[k][0] && (q[1] & 1) == kFccBasis[k][1] && (q[2] & 1) == kFccBasis[k][2]) b = k;
  int64_t x = q[0] >> 1, y = q[1] >> 1, z = q[2] >> 1;
  return ((z * L[1] + y) * L[0] + x) * 4 + b;
}

/* Coordination shells by enumeration: every non-zero doubled-coordinate vector with even
 * coordinate sum and components in [-2,2], sorted by squared length and then
 * lexicographically on (dx,dy,dz).  The first 42 are shells 1 (12 at a/sqrt(2)),
 * 2 (6 at a) and 3 (24 at a*sqrt(3/2)). */
#define FCC_NBR 42
void or_fcc_shell_table(int32_t off[FCC_NBR * 3], int32_t shell[FCC_NBR]) {
  int32_t cand[125][4];
  int n = 0;
  for (int dx = -2; dx <= 2; ++dx)
    for (int dy = -2; dy <= 2; ++dy)
      for (int dz = -2; dz <= 2; ++dz) {
        if (dx == 0 && dy == 0 && dz == 0) continue;
        if (((dx + dy + dz) % 2 + 2) % 2 != 0) continue;
        cand[n][0] = dx * dx + dy * dy + dz * dz;
        cand[n][1] = dx; cand[n][2] = dy; cand[n][3] = dz;
        ++n;
      }
  for (int i = 1; i < n; ++i) {
    int32_t t[4];
    memcpy(t, cand[i], sizeof t);
    int j = i - 1;
    while (j >= 0 && (cand[j][0] > t[0] ||
                      (cand[j][0] == t[0] && (cand[j][1] > t[1] ||
                      (cand[j][1] == t[1] && (cand[j][2] > t[2] ||
                      (cand[j][2] == t[2] && cand[j][3] > t[3]))))))) {
      memcpy(cand[j + 1], cand[j], sizeof t);
      --j;
    }
    memcpy(cand[j + 1], t, sizeof t);
  }
  int32_t sh = 0, last = -1;
  for (int k = 0; k < FCC_NBR; ++k) {
    if (cand[k][0] != last) { ++sh; last = cand[k][0]; }
    off[3 * k + 0] = cand[k][1];
    off[3 * k + 1] = cand[k][2];
    off[3 * k + 2] = cand[k][3];
    shell[k] = sh;
  }
}

static int32_t f_off[FCC_NBR * 3], f_shell[FCC_NBR];
static int f_ready = 0;

static void fcc_tables(void) {
  if (!f_ready) {
    or_fcc_shell_table(f_off, f_shell);
    f_ready = 1;
  }
}

int64_t or_fcc_neighbor(const int32_t L[3], int64_t s, int32_t k) {
  fcc_tables();
  int32_t P[3];
  or_fcc_site_pos(L, s, P);
  for (int a = 0; a < 3; ++a) P[a] += f_off[3 * k + a];
  return or_fcc_site_at(L, P);
}

/* The MLPNet reads shells 1-2 (18 neighbours), qSRO shells 1-3 (42). */
int32_t or_fcc_n_neighbors_used(int32_t model) { return model == OR_FCC_MLPNET_S12 ? 18 : 42; }
int32_t or_fcc_n_inputs(void) { return 4 * (1 + 18); }

int64_t or_fcc_n_params(const or_fcc_model *m) {
  if (m->model == OR_FCC_QSRO_S123) return 92;
  const int64_t F = or_fcc_n_inputs(), H = m->hidden;
  return H * F + H + 2 * (H * H + H) + H + 1;
}

static uint8_t fcc_species(const uint8_t *occ, int64_t s, int64_t i, int64_t n) {
  if (i >= 0) {
    if (s == i) return occ[n];
    if (s == n) return occ[i];
  }
  return occ[s];
}

/* MLPNet input: one-hot (four channels; species >= 4 contribute zeros) of the site and of
 * its 18 shell-1 and shell-2 neighbours in slot order; images count with multiplicity. */
void or_fcc_features(const int32_t L[3], const uint8_t *occ, int64_t j, int64_t swap_i, int64_t swap_n,
                     double *x) {
  fcc_tables();
  for (int f = 0; f < 76; ++f) x[f] = 0.0;
  uint8_t c = fcc_species(occ, j, swap_i, swap_n);
  if (c < 4) x[c] = 1.0;
  for (int k = 0; k < 18; ++k) {
    uint8_t p = fcc_species(occ, or_fcc_neighbor(L, j, k), swap_i, swap_n);
    if (p < 4) x[4 * (k + 1) + p] = 1.0;
  }
}

/* MLPNet (Eqs. (4)-(6)): h1 = relu(W0 x + b0), h2 = relu(W1 h1 + b1), h3 = relu(W2 h2 + b2),
 * E = W3 . h3 + b3; every hidden layer has H units. */
double or_fcc_mlpnet(const or_fcc_model *m, const double *x) {
  const int32_t F = or_fcc_n_inputs(), H = m->hidden;
  const double *W0 = m->params, *b0 = W0 + (int64_t)H * F;
  const double *W1 = b0 + H, *b1 = W1 + (int64_t)H * H;
  const double *W2 = b1 + H, *b2 = W2 + (int64_t)H * H;
  const double *W3 = b2 + H, *b3 = W3 + H;
  double h1[512], h2[512], h3[512];
  for (int o = 0; o < H; ++o) {
    double acc = b0[o];
    for (int k = 0; k < F; ++k) acc += W0[(int64_t)o * F + k] * x[k];
    h1[o] = acc > 0.0 ? acc : 0.0;
  }
  for (int o = 0; o < H; ++o) {
    double acc = b1[o];
    for (int k = 0; k < H; ++k) acc += W1[(int64_t)o * H + k] * h1[k];
    h2[o] = acc > 0.0 ? acc : 0.0;
  }
  for (int o = 0; o < H; ++o) {
    double acc = b2[o];
    for (int k = 0; k < H; ++k) acc += W2[(int64_t)o * H + k] * h2[k];
    h3[o] = acc > 0.0 ? acc : 0.0;
  }
  double e = b3[0];
  for (int k = 0; k < H; ++k) e += W3[k] * h3[k];
  return e;
}

/* qSRO local energy (Eq. 2) over the first three FCC shells, exactly as on BCC: pair
 * fractions pi_m^{pp'} = n_m^{pp'} / (pairs in shell m), linear in unlike and quadratic in
 * like fractions, plus the regulariser and the constant. */
double or_fcc_qsro(const int32_t L[3], const double *P, const uint8_t *occ, int64_t j, int64_t swap_i,
                   int64_t swap_n) {
  fcc_tables();
  const double *V = P, *W = P + 75, lambda = P[90], C = P[91];
  double e = C;
  const uint8_t c = fcc_species(occ, j, swap_i, swap_n);
  for (int m = 1; m <= 3; ++m) {
    double n[5][5] = {{0}};
    double pairs = 0.0;
    for (int k = 0; k < FCC_NBR; ++k) {
      if (f_shell[k] != m) continue;
      const uint8_t q = fcc_species(occ, or_fcc_neighbor(L, j, k), swap_i, swap_n);
      const int hi = c > q ? c : q, lo = c > q ? q : c;
      n[hi][lo] += 1.0;
      pairs += 1.0;
    }
    for (int p = 0; p < 5; ++p)
      for (int pp = 0; pp < p; ++pp) e += V[((m - 1) * 5 + p) * 5 + pp] * (n[p][pp] / pairs);
    for (int p = 0; p < 5; ++p) {
      const double pi = n[p][p] / pairs;
      e += W[(m - 1) * 5 + p] * pi * pi;
    }
  }
  for (int q = 0; q < 15; ++q) e += lambda * W[q] * W[q];
  return e;
}

double or_fcc_site_energy(const int32_t L[3], const or_fcc_model *m, const uint8_t *occ, int64_t j,
                          int64_t swap_i, int64_t swap_n) {
  if (m->model == OR_FCC_QSRO_S123) return or_fcc_qsro(L, m->params, occ, j, swap_i, swap_n);
  double x[76];
  or_fcc_features(L, occ, j, swap_i, swap_n, x);
  return or_fcc_mlpnet(m, x);
}

void or_fcc_all_site_energies(const int32_t L[3], const or_fcc_model *m, const uint8_t *occ, double *e) {
  const int64_t N = or_fcc_n_sites(L);
  for (int64_t j = 0; j < N; ++j) e[j] = or_fcc_site_energy(L, m, occ, j, -1, -1);
}

double or_fcc_total_energy(const int32_t L[3], const or_fcc_model *m, const uint8_t *occ) {
  const int64_t N = or_fcc_n_sites(L);
  double e = 0.0;
  for (int64_t j = 0; j < N; ++j) e += or_fcc_site_energy(L, m, occ, j, -1, -1);
  return e;
}

static int fcc_cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

/* Omega(i, n): i, n and every site that reads i or n among its neighbours (the shell set
 * is symmetric), sorted ascending without duplicates. */
int32_t or_fcc_omega(const int32_t L[3], int32_t model, int64_t i, int64_t n, int64_t *omega) {
  const int32_t K = or_fcc_n_neighbors_used(model);
  int64_t tmp[2 + 2 * FCC_NBR];
  int32_t c = 0;
  tmp[c++] = i;
  tmp[c++] = n;
  for (int k = 0; k < K; ++k) {
    tmp[c++] = or_fcc_neighbor(L, i, k);
    tmp[c++] = or_fcc_neighbor(L, n, k);
  }
  qsort(tmp, (size_t)c, sizeof(int64_t), fcc_cmp_i64);
  int32_t u = 0;
  for (int32_t a = 0; a < c; ++a)
    if (u == 0 || omega[u - 1] != tmp[a]) omega[u++] = tmp[a];
  return u;
}

/* dE of exchanging i and n: local energies after minus before, reduced over Omega
 * (Algorithm 1's two zone reductions). */
double or_fcc_delta_e(const int32_t L[3], const or_fcc_model *m, const uint8_t *occ, int64_t i, int64_t n) {
  int64_t omega[2 + 2 * FCC_NBR];
  int32_t cnt = or_fcc_omega(L, m->model, i, n, omega);
  double e1 = 0.0, e0 = 0.0;
  for (int32_t a = 0; a < cnt; ++a) {
    e1 += or_fcc_site_energy(L, m, occ, omega[a], i, n);
    e0 += or_fcc_site_energy(L, m, occ, omega[a], -1, -1);
  }
  return e1 - e0;
}

/* Link-cell colouring (Algorithm 1's partition; the 4x4x4 link cell of the FCC runs gives
 * 4 x 4 x 4 x 4 = 256 mini-steps, Sec. V-C): axes are cut as on BCC; the colour is the
 * offset inside the link cell with the basis index, so 4 e_x e_y e_z colours. */
static int32_t fcc_axis_offset(int32_t E, int32_t x, int32_t *emax) {
  int32_t q = E / 4;
  if (q < 1) q = 1;
  int32_t small = E / q, big = small + (E % q ? 1 : 0), nbig = E % q;
  *emax = big;
  int32_t start = 0;
  for (int32_t a = 0; a < q; ++a) {
    int32_t e = a < nbig ? big : small;
    if (x < start + e) return x - start;
    start += e;
  }
  return -1;
}

int32_t or_fcc_n_colours(const int32_t L[3]) {
  int32_t e[3];
  for (int a = 0; a < 3; ++a) (void)fcc_axis_offset(L[a], 0, &e[a]);
  return 4 * e[0] * e[1] * e[2];
}

int32_t or_fcc_colour_of(const int32_t L[3], int64_t s) {
  int32_t b = (int32_t)(s % 4);
  int64_t c = s / 4;
  int32_t x = (int32_t)(c % L[0]);
  int32_t y = (int32_t)((c / L[0]) % L[1]);
  int32_t z = (int32_t)(c / ((int64_t)L[0] * L[1]));
  int32_t ex, ey, ez;
  int32_t ox = fcc_axis_offset(L[0], x, &ex);
  int32_t oy = fcc_axis_offset(L[1], y, &ey);
  int32_t oz = fcc_axis_offset(L[2], z, &ez);
  return ((oz * ey + oy) * ex + ox) * 4 + b;
}

/* Proposal: the Philox block of (site, sweep, replica, 0) with key (seed, 0) as on BCC;
 * the partner is shell-1 slot floor((r0 >> 32) * 12 / 2^32) of the 12 nearest neighbours,
 * and u = ((r1 >> 11) + 1) * 2^-53. */
void or_fcc_propose(uint64_t seed, int64_t site, int64_t sweep, int64_t replica, int32_t *dir, double *u) {
  uint64_t ctr[4] = {(uint64_t)site, (uint64_t)sweep, (uint64_t)replica, 0};
  uint64_t key[2] = {seed, 0};
  uint64_t r[4];
  or_philox4x64_10(ctr, key, r);
  *dir = (int32_t)(((r[0] >> 32) * 12ULL) >> 32);
  *u = (double)((r[1] >> 11) + 1) * 0x1.0p-53;
}

static void fcc_trial(const int32_t L[3], const or_fcc_model *m, const uint8_t *occ, double temperature_K,
                      uint64_t seed, int64_t replica, int64_t sweep, int64_t site, or_trial_rec *rec) {
  int32_t dir;
  double u;
  or_fcc_propose(seed, site, sweep, replica, &dir, &u);
  int64_t n = or_fcc_neighbor(L, site, dir);
  rec->site = site;
  rec->partner = n;
  rec->dir = dir;
  rec->u = u;
  rec->theta = or_theta(temperature_K, u);
  rec->colour = or_fcc_colour_of(L, site);
  rec->same = occ[site] == occ[n];
  if (rec->same) {
    rec->dE = 0.0;
    rec->accept = 0;
  } else {
    rec->dE = or_fcc_delta_e(L, m, occ, site, n);
    rec->accept = or_accept(rec->dE, rec->theta);
  }
}

/* An outside decision replaces the Metropolis decision of a different-species trial
 * (force[site] = 0 or 1; negative: none), so that tests can follow a chain decided the other
 * way within rounding of the threshold. */
static void fcc_force(or_trial_rec *r, const int8_t *force) {
  if (force && force[r->site] >= 0 && !r->same) r->accept = force[r->site] ? 1 : 0;
}

/* One sweep: colours in order, every site of a colour a trial site once.  Snapshot order
 * decides all trials of a mini-step on the same lattice and then copies accepted pairs
 * back (Algorithm 1); the sequential orders test independence from the trial order. */
int or_fcc_sweep(const int32_t L[3], const or_fcc_model *m, uint8_t *occ, double temperature_K, uint64_t seed,
                 int64_t replica, int64_t sweep, or_stats *st, or_trial_rec *trace, int32_t order,
                 const int64_t *given_order, int32_t nthreads, int32_t colours_limit, const int8_t *force) {
  const int64_t N = or_fcc_n_sites(L);
  const int32_t C = or_fcc_n_colours(L);
  fcc_tables();
  int64_t *bucket_start = (int64_t *)calloc((size_t)C + 1, sizeof(int64_t));
  int64_t *sites = (int64_t *)malloc((size_t)N * sizeof(int64_t));
  int32_t *col = (int32_t *)malloc((size_t)N * sizeof(int32_t));
  or_trial_rec *rec = (or_trial_rec *)malloc((size_t)N * sizeof(or_trial_rec));
  int64_t *fill = (int64_t *)malloc((size_t)C * sizeof(int64_t));
  if (!bucket_start || !sites || !col || !rec || !fill) {
    free(bucket_start); free(sites); free(col); free(rec); free(fill);
    return -1;
  }
  for (int64_t s = 0; s < N; ++s) {
    col[s] = or_fcc_colour_of(L, s);
    bucket_start[col[s] + 1]++;
  }
  for (int32_t c = 0; c < C; ++c) bucket_start[c + 1] += bucket_start[c];
  memcpy(fill, bucket_start, (size_t)C * sizeof(int64_t));
  for (int64_t a = 0; a < N; ++a) {
    int64_t s = a;
    if (order == OR_ORDER_REVERSE) s = N - 1 - a;
    if (order == OR_ORDER_GIVEN) s = given_order[a];
    sites[fill[col[s]]++] = s;
  }
  free(fill);
  const int32_t ncol = colours_limit < 0 || colours_limit > C ? C : colours_limit;
  for (int32_t c = 0; c < ncol; ++c) {
    const int64_t b0 = bucket_start[c], b1 = bucket_start[c + 1];
    if (order == OR_ORDER_SNAPSHOT) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
#endif
      for (int64_t a = b0; a < b1; ++a) {
        fcc_trial(L, m, occ, temperature_K, seed, replica, sweep, sites[a], &rec[a - b0]);
        fcc_force(&rec[a - b0], force);
      }
      for (int64_t a = b0; a < b1; ++a) {
        const or_trial_rec *r = &rec[a - b0];
        if (r->accept) {
          uint8_t t = occ[r->site];
          occ[r->site] = occ[r->partner];
          occ[r->partner] = t;
        }
      }
    } else {
      for (int64_t a = b0; a < b1; ++a) {
        fcc_trial(L, m, occ, temperature_K, seed, replica, sweep, sites[a], &rec[a - b0]);
        fcc_force(&rec[a - b0], force);
        const or_trial_rec *r = &rec[a - b0];
        if (r->accept) {
          uint8_t t = occ[r->site];
          occ[r->site] = occ[r->partner];
          occ[r->partner] = t;
        }
      }
    }
    for (int64_t a = b0; a < b1; ++a) {
      const or_trial_rec *r = &rec[a - b0];
      if (st) {
        st->attempts++;
        if (!r->same) st->diff_species++;
        if (r->accept) { st->accepts++; st->e_run += r->dE; }
      }
      if (trace) trace[r->site] = *r;
    }
  }
  free(bucket_start); free(sites); free(col); free(rec);
  return 0;
}

/* Warren-Cowley alpha_m^{pq} = 1 - P(q in shell m | p) / c_q over FCC shells 1-3. */
void or_fcc_warren_cowley(const int32_t L[3], const uint8_t *occ, int32_t n_species, double *alpha) {
  fcc_tables();
  const int64_t N = or_fcc_n_sites(L);
  const int32_t S = n_species;
  double *cnt = (double *)calloc((size_t)3 * S * S, sizeof(double));
  double *nsp = (double *)calloc((size_t)S, sizeof(double));
  double zc[3] = {0, 0, 0};
  for (int k = 0; k < FCC_NBR; ++k) zc[f_shell[k] - 1] += 1.0;
  for (int64_t j = 0; j < N; ++j) {
    nsp[occ[j]] += 1.0;
    for (int k = 0; k < FCC_NBR; ++k)
      cnt[((f_shell[k] - 1) * S + occ[j]) * S + occ[or_fcc_neighbor(L, j, k)]] += 1.0;
  }
  for (int m = 0; m < 3; ++m)
    for (int p = 0; p < S; ++p)
      for (int q = 0; q < S; ++q) {
        double cq = nsp[q] / (double)N;
        double pq = nsp[p] > 0 ? cnt[(m * S + p) * S + q] / (nsp[p] * zc[m]) : 0.0;
        alpha[(m * S + p) * S + q] = (cq > 0 && nsp[p] > 0) ? 1.0 - pq / cq : 0.0;
      }
  free(cnt);
  free(nsp);
}
