/*
 * Plain CPU oracle of the swap Monte Carlo hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Slow and direct on purpose: every energy is recomputed from the definition, both
 * before and after a swap, in double precision, with no caches, no blocking and no
 * reordering beyond what the method states.  Citations are to arXiv 2604.08250.
 * The product library shares no code with this file.
 */
#include "smc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_KB_EV_PER_K 8.617333262e-5 /* Boltzmann constant, eV/K (CODATA 2018, exact) */

/* ------------------------------------------------------------------------------------
 * Philox4x64-10, written from the description in Salmon et al., "Parallel random
 * numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two 64x64->128 multiplications
 * whose high halves are xored with the other counter words and the round key; the key
 * is advanced by the two Weyl constants between rounds.
 * ---------------------------------------------------------------------------------- */
static void or_mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += W0; k1 += W1; }
    uint64_t hi0, lo0, hi1, lo1;
    or_mulhilo64(M0, x0, &hi0, &lo0);
    or_mulhilo64(M1, x2, &hi1, &lo1);
    uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------------------
 * BCC geometry in doubled integer coordinates: cell (x,y,z) holds basis site b = 0 at
 * (2x,2y,2z) and b = 1 at (2x+1,2y+1,2z+1); positions are periodic modulo 2L per axis.
 * Canonical site index s = ((z*Ly + y)*Lx + x)*2 + b.
 * ---------------------------------------------------------------------------------- */
int64_t or_n_sites(const int32_t L[3]) { return 2LL * L[0] * L[1] * L[2]; }

void or_site_pos(const int32_t L[3], int64_t s, int32_t P[3]) {
  int32_t b = (int32_t)(s & 1);
  int64_t c = s >> 1;
  int32_t x = (int32_t)(c % L[0]);
  int32_t y = (int32_t)((c / L[0]) % L[1]);
  int32_t z = (int32_t)(c / ((int64_t)L[0] * L[1]));
  P[0] = 2 * x + b; P[1] = 2 * y + b; P[2] = 2 * z + b;
}

static int32_t or_wrap(int32_t v, int32_t m) {
  int32_t r = v % m;
  return r < 0 ? r + m : r;
}

int64_t or_site_at(const int32_t L[3], const int32_t P[3]) {
  int32_t q[3];
  for (int a = 0; a < 3; ++a) q[a] = or_wrap(P[a], 2 * L[a]);
  int32_t b = q[0] & 1;
  /* a BCC position has all three doubled coordinates of the same parity */
  if ((q[1] & 1) != b || (q[2] & 1) != b) return -1;
  int64_t x = q[0] >> 1, y = q[1] >> 1, z = q[2] >> 1;
  return ((z * L[1] + y) * L[0] + x) * 2 + b;
}

/* Coordination shells by enumeration: every non-zero doubled-coordinate vector of one
 * parity with components in [-2,2], sorted by squared length and then lexicographically
 * on (dx,dy,dz).  The first 26 are shells 1 (8 at a*sqrt(3)/2), 2 (6 at a) and
 * 3 (12 at a*sqrt(2)). */
void or_shell_table(int32_t off[26 * 3], int32_t shell[26]) {
  int32_t cand[125][4];
  int n = 0;
  for (int dx = -2; dx <= 2; ++dx)
    for (int dy = -2; dy <= 2; ++dy)
      for (int dz = -2; dz <= 2; ++dz) {
        if (dx == 0 && dy == 0 && dz == 0) continue;
        int px = dx & 1, py = dy & 1, pz = dz & 1;
        if (px != py || py != pz) continue;
        cand[n][0] = dx * dx + dy * dy + dz * dz;
        cand[n][1] = dx; cand[n][2] = dy; cand[n][3] = dz;
        ++n;
      }
  /* insertion sort on (d2, dx, dy, dz) */
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
  for (int k = 0; k < 26; ++k) {
    if (cand[k][0] != last) { ++sh; last = cand[k][0]; }
    off[3 * k + 0] = cand[k][1];
    off[3 * k + 1] = cand[k][2];
    off[3 * k + 2] = cand[k][3];
    shell[k] = sh;
  }
}

static int32_t g_off[26 * 3], g_shell[26];
static int g_tables_ready = 0;

static void or_tables(void) {
  if (!g_tables_ready) {
    or_shell_table(g_off, g_shell);
    g_tables_ready = 1;
  }
}

int64_t or_neighbor(const int32_t L[3], int64_t s, int32_t k) {
  or_tables();
  int32_t P[3];
  or_site_pos(L, s, P);
  for (int a = 0; a < 3; ++a) P[a] += g_off[3 * k + a];
  return or_site_at(L, P);
}

int32_t or_n_inputs(int32_t feature) { return feature == OR_FEAT_COUNTS_S12 ? 12 : 108; }
/* counts features use shells 1-2 (14 neighbours), one-hot features shells 1-3 (26) */
int32_t or_n_neighbors_used(int32_t feature) { return feature == OR_FEAT_COUNTS_S12 ? 14 : 26; }

/* Species seen at site s when sites i and n are exchanged (i < 0: no exchange). */
static uint8_t or_species(const uint8_t *occ, int64_t s, int64_t i, int64_t n) {
  if (i >= 0) {
    if (s == i) return occ[n];
    if (s == n) return occ[i];
  }
  return occ[s];
}

/* Feature vector of site j (Sec. III-B3: computed on the fly from the species of the
 * site and of its neighbours).  Four species channels; a species id >= 4 has no channel
 * and contributes zeros.  Images on small periodic lattices count with multiplicity. */
void or_features(const int32_t L[3], int32_t feature, const uint8_t *occ, int64_t j,
                 int64_t swap_i, int64_t swap_n, double *x) {
  or_tables();
  int32_t F = or_n_inputs(feature);
  for (int f = 0; f < F; ++f) x[f] = 0.0;
  uint8_t c = or_species(occ, j, swap_i, swap_n);
  if (c < 4) x[c] = 1.0;
  if (feature == OR_FEAT_COUNTS_S12) {
    for (int k = 0; k < 14; ++k) {
      uint8_t p = or_species(occ, or_neighbor(L, j, k), swap_i, swap_n);
      if (p >= 4) continue;
      if (g_shell[k] == 1) x[4 + p] += 1.0;
      else x[8 + p] += 1.0;
    }
  } else {
    for (int k = 0; k < 26; ++k) {
      uint8_t p = or_species(occ, or_neighbor(L, j, k), swap_i, swap_n);
      if (p < 4) x[4 * (k + 1) + p] = 1.0;
    }
  }
}

static double or_act(int32_t a, double z) {
  switch (a) {
    case OR_ACT_SILU: return z / (1.0 + exp(-z));
    case OR_ACT_IDENTITY: return z;
    case OR_ACT_RELU: return z > 0.0 ? z : 0.0;
    case OR_ACT_SQUARE: return z * z;
  }
  return NAN;
}

/* E = W2 . act1(W1 . act0(W0 x + b0) + b1) + b2  (Eqs. (4)-(6) with two hidden layers). */
double or_mlp(const or_model *m, const double *x) {
  const int32_t F = or_n_inputs(m->feature), H = m->hidden;
  const double *W0 = m->params, *b0 = W0 + (int64_t)H * F, *W1 = b0 + H, *b1 = W1 + (int64_t)H * H,
               *W2 = b1 + H, *b2 = W2 + H;
  double h0[512], h1[512];
  for (int o = 0; o < H; ++o) {
    double acc = b0[o];
    for (int k = 0; k < F; ++k) acc += W0[(int64_t)o * F + k] * x[k];
    h0[o] = or_act(m->act0, acc);
  }
  for (int o = 0; o < H; ++o) {
    double acc = b1[o];
    for (int k = 0; k < H; ++k) acc += W1[(int64_t)o * H + k] * h0[k];
    h1[o] = or_act(m->act1, acc);
  }
  double e = b2[0];
  for (int k = 0; k < H; ++k) e += W2[k] * h1[k];
  return e;
}

/* qSRO local energy (Eq. 2).  Pairs of site j with its neighbours in coordination shell m
 * (m = 1..3) are counted per unordered species pair: n_m^{pp'}; pi_m^{pp'} = n_m^{pp'} divided
 * by the number of pairs in the shell.  E_j = sum_{m, p' < p} V_m^{pp'} pi_m^{pp'}
 * + sum_{m, p} W_m^p (pi_m^{pp})^2 + lambda sum_{m, p} (W_m^p)^2 + C, over species 0..4. */
double or_qsro(const int32_t L[3], const double *P, const uint8_t *occ, int64_t j, int64_t swap_i,
               int64_t swap_n) {
  or_tables();
  const double *V = P, *W = P + 75, lambda = P[90], C = P[91];
  double e = C;
  const uint8_t c = or_species(occ, j, swap_i, swap_n);
  for (int m = 1; m <= 3; ++m) {
    double n[5][5] = {{0}};
    double pairs = 0.0;
    for (int k = 0; k < 26; ++k) {
      if (g_shell[k] != m) continue;
      const uint8_t q = or_species(occ, or_neighbor(L, j, k), swap_i, swap_n);
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

double or_site_energy(const int32_t L[3], const or_model *m, const uint8_t *occ, int64_t j,
                      int64_t swap_i, int64_t swap_n) {
  if (m->feature == OR_FEAT_QSRO_S123) return or_qsro(L, m->params, occ, j, swap_i, swap_n);
  double x[108];
  or_features(L, m->feature, occ, j, swap_i, swap_n, x);
  return or_mlp(m, x);
}

void or_all_site_energies(const int32_t L[3], const or_model *m, const uint8_t *occ, double *e) {
  const int64_t N = or_n_sites(L);
  for (int64_t j = 0; j < N; ++j) e[j] = or_site_energy(L, m, occ, j, -1, -1);
}

/* Total energy: plain sequential sum of local energies in canonical order. */
double or_total_energy(const int32_t L[3], const or_model *m, const uint8_t *occ) {
  const int64_t N = or_n_sites(L);
  double e = 0.0;
  for (int64_t j = 0; j < N; ++j) e += or_site_energy(L, m, occ, j, -1, -1);
  return e;
}

static int or_cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

/* Omega(i, n): the sites whose local energy can change when i and n exchange species,
 * i.e. i, n and every site that has i or n among the neighbours its features read.
 * The shell set is symmetric, so "j sees i" <=> "j is a neighbour of i".  Returned
 * sorted ascending without duplicates. */
int32_t or_omega(const int32_t L[3], int32_t feature, int64_t i, int64_t n, int64_t *omega) {
  const int32_t K = or_n_neighbors_used(feature);
  int64_t tmp[2 + 2 * 26];
  int32_t c = 0;
  tmp[c++] = i;
  tmp[c++] = n;
  for (int k = 0; k < K; ++k) {
    tmp[c++] = or_neighbor(L, i, k);
    tmp[c++] = or_neighbor(L, n, k);
  }
  qsort(tmp, (size_t)c, sizeof(int64_t), or_cmp_i64);
  int32_t u = 0;
  for (int32_t a = 0; a < c; ++a)
    if (u == 0 || omega[u - 1] != tmp[a]) omega[u++] = tmp[a];
  return u;
}

/* dE of exchanging the species at i and n: local energies after minus before, reduced
 * over Omega (Algorithm 1, reductions of E1 and E0 within Omega). */
double or_delta_e(const int32_t L[3], const or_model *m, const uint8_t *occ, int64_t i, int64_t n) {
  int64_t omega[2 + 2 * 26];
  int32_t cnt = or_omega(L, m->feature, i, n, omega);
  double e1 = 0.0, e0 = 0.0;
  for (int32_t a = 0; a < cnt; ++a) {
    e1 += or_site_energy(L, m, occ, omega[a], i, n);
    e0 += or_site_energy(L, m, occ, omega[a], -1, -1);
  }
  return e1 - e0;
}

/* ------------------------------------------------------------------------------------
 * Link-cell colouring (Algorithm 1 partition step; Sec. II-A).  Each axis of E cells is
 * cut into q = max(1, floor(E/4)) link cells whose edges differ by at most one, the
 * first (E mod q) cells taking the longer edge.  The colour of a site is its offset
 * inside its link cell together with its basis index; all sites of one colour are
 * updated concurrently, one colour (mini-step) after another.
 * ---------------------------------------------------------------------------------- */
static int32_t or_axis_offset(int32_t E, int32_t x, int32_t *emax) {
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

int32_t or_n_colours(const int32_t L[3]) {
  int32_t e[3];
  for (int a = 0; a < 3; ++a) (void)or_axis_offset(L[a], 0, &e[a]);
  return 2 * e[0] * e[1] * e[2];
}

int32_t or_colour_of(const int32_t L[3], int64_t s) {
  int32_t b = (int32_t)(s & 1);
  int64_t c = s >> 1;
  int32_t x = (int32_t)(c % L[0]);
  int32_t y = (int32_t)((c / L[0]) % L[1]);
  int32_t z = (int32_t)(c / ((int64_t)L[0] * L[1]));
  int32_t ex, ey, ez;
  int32_t ox = or_axis_offset(L[0], x, &ex);
  int32_t oy = or_axis_offset(L[1], y, &ey);
  int32_t oz = or_axis_offset(L[2], z, &ez);
  return ((oz * ey + oy) * ex + ox) * 2 + b;
}

/* ------------------------------------------------------------------------------------
 * Trial proposal (Algorithm 1: swap the trial site with a random nearest neighbour) and
 * Metropolis acceptance.  One Philox4x64-10 block per (site, sweep, replica):
 *   counter = (site, sweep, replica, 0), key = (seed, 0) -> (r0, r1, r2, r3);
 *   partner direction = r0 >> 61 (shell-1 neighbour slot 0..7);
 *   u = ((r1 >> 11) + 1) * 2^-53 in (0, 1];
 *   theta = -kB T ln u; accept iff dE <= theta, so P(accept) = min(1, exp(-dE/kB T)).
 * ---------------------------------------------------------------------------------- */
void or_propose(uint64_t seed, int64_t site, int64_t sweep, int64_t replica, int32_t *dir,
                double *u) {
  uint64_t ctr[4] = {(uint64_t)site, (uint64_t)sweep, (uint64_t)replica, 0};
  uint64_t key[2] = {seed, 0};
  uint64_t r[4];
  or_philox4x64_10(ctr, key, r);
  *dir = (int32_t)(r[0] >> 61);
  *u = (double)((r[1] >> 11) + 1) * 0x1.0p-53;
}

double or_theta(double temperature_K, double u) {
  if (isinf(temperature_K)) return INFINITY;
  return -OR_KB_EV_PER_K * temperature_K * log(u);
}

int32_t or_accept(double dE, double theta) { return dE <= theta; }

void or_trial(const int32_t L[3], const or_model *m, const uint8_t *occ, double temperature_K,
              uint64_t seed, int64_t replica, int64_t sweep, int64_t site, or_trial_rec *rec) {
  int32_t dir;
  double u;
  or_propose(seed, site, sweep, replica, &dir, &u);
  int64_t n = or_neighbor(L, site, dir);
  rec->site = site;
  rec->partner = n;
  rec->dir = dir;
  rec->u = u;
  rec->theta = or_theta(temperature_K, u);
  rec->colour = or_colour_of(L, site);
  rec->same = occ[site] == occ[n];
  if (rec->same) {
    rec->dE = 0.0;
    rec->accept = 0;
  } else {
    rec->dE = or_delta_e(L, m, occ, site, n);
    rec->accept = or_accept(rec->dE, rec->theta);
  }
}

/* Proposals of many trial sites at once (partner slot, partner site, threshold), the same
 * steps as the start of or_trial. */
void or_proposals(const int32_t L[3], uint64_t seed, int64_t replica, int64_t sweep, double temperature_K,
                  const int64_t *sites, int64_t n, int32_t *dir, int64_t *partner, double *theta) {
  for (int64_t a = 0; a < n; ++a) {
    int32_t d;
    double u;
    or_propose(seed, sites[a], sweep, replica, &d, &u);
    if (dir) dir[a] = d;
    if (partner) partner[a] = or_neighbor(L, sites[a], d);
    if (theta) theta[a] = or_theta(temperature_K, u);
  }
}

/* A decision given from outside replaces the Metropolis decision of a different-species
 * trial (force[site] = 0 or 1; negative: no override).  The tests use it to keep following a
 * chain whose decision another implementation took the other way within rounding of the
 * threshold; the trial's dE and theta stay the oracle's own. */
static void or_force(or_trial_rec *r, const int8_t *force) {
  if (force && force[r->site] >= 0 && !r->same) r->accept = force[r->site] ? 1 : 0;
}

/* One sweep: colours 0..C-1 in order; inside a colour every site of that colour is a
 * trial site once.  OR_ORDER_SNAPSHOT follows Algorithm 1 literally (all trials of the
 * mini-step decided on the same lattice, then accepted pairs copied back); the
 * sequential orders exist to test that the result does not depend on the order. */
int or_sweep(const int32_t L[3], const or_model *m, uint8_t *occ, double temperature_K,
             uint64_t seed, int64_t replica, int64_t sweep, or_stats *st, or_trial_rec *trace,
             int32_t order, const int64_t *given_order, int32_t nthreads, int32_t colours_limit,
             const int8_t *force) {
  const int64_t N = or_n_sites(L);
  const int32_t C = or_n_colours(L);
  or_tables(); /* initialise the shell table before any parallel region reads it */
  int64_t *bucket_start = (int64_t *)calloc((size_t)C + 1, sizeof(int64_t));
  int64_t *sites = (int64_t *)malloc((size_t)N * sizeof(int64_t));
  int32_t *col = (int32_t *)malloc((size_t)N * sizeof(int32_t));
  or_trial_rec *rec = (or_trial_rec *)malloc((size_t)N * sizeof(or_trial_rec));
  if (!bucket_start || !sites || !col || !rec) {
    free(bucket_start); free(sites); free(col); free(rec);
    return -1;
  }
  /* bucket the trial sites by colour, in canonical order or in the given order */
  for (int64_t s = 0; s < N; ++s) {
    col[s] = or_colour_of(L, s);
    bucket_start[col[s] + 1]++;
  }
  for (int32_t c = 0; c < C; ++c) bucket_start[c + 1] += bucket_start[c];
  {
    int64_t *fill = (int64_t *)malloc((size_t)C * sizeof(int64_t));
    memcpy(fill, bucket_start, (size_t)C * sizeof(int64_t));
    for (int64_t a = 0; a < N; ++a) {
      int64_t s = a;
      if (order == OR_ORDER_REVERSE) s = N - 1 - a;
      if (order == OR_ORDER_GIVEN) s = given_order[a];
      sites[fill[col[s]]++] = s;
    }
    free(fill);
  }
  (void)nthreads;
  const int32_t ncol = colours_limit < 0 || colours_limit > C ? C : colours_limit;
  for (int32_t c = 0; c < ncol; ++c) {
    const int64_t b0 = bucket_start[c], b1 = bucket_start[c + 1];
    if (order == OR_ORDER_SNAPSHOT) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
#endif
      for (int64_t a = b0; a < b1; ++a) {
        or_trial(L, m, occ, temperature_K, seed, replica, sweep, sites[a], &rec[a - b0]);
        or_force(&rec[a - b0], force);
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
        or_trial(L, m, occ, temperature_K, seed, replica, sweep, sites[a], &rec[a - b0]);
        or_force(&rec[a - b0], force);
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

/* Warren-Cowley short-range order alpha_m^{pq} = 1 - P(q in shell m | p) / c_q. */
void or_warren_cowley(const int32_t L[3], const uint8_t *occ, int32_t n_species, double *alpha) {
  or_tables();
  const int64_t N = or_n_sites(L);
  const int32_t S = n_species;
  double *cnt = (double *)calloc((size_t)3 * S * S, sizeof(double));
  double *nsp = (double *)calloc((size_t)S, sizeof(double));
  double zc[3] = {0, 0, 0};
  for (int k = 0; k < 26; ++k) zc[g_shell[k] - 1] += 1.0;
  for (int64_t j = 0; j < N; ++j) {
    nsp[occ[j]] += 1.0;
    for (int k = 0; k < 26; ++k) {
      int m = g_shell[k] - 1;
      cnt[(m * S + occ[j]) * S + occ[or_neighbor(L, j, k)]] += 1.0;
    }
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
