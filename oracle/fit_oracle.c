/*
 * Oracle of the differentiation pattern (test infrastructure only; see smc_oracle.h).
 *
 * 1. A cluster-expansion (CE) reference Hamiltonian on the BCC lattice: pair terms on the
 *    first three coordination shells plus a set of three-site cluster terms, each a
 *    (triangle shape, species triple) item with its own interaction.  The paper fits its
 *    models to DFT energies (Sec. IV-B); no DFT data exists here, so a seeded CE stands in
 *    for it as the source of labels.  Two independent evaluations are given: a sum of
 *    site-local terms (each pair split half-half between its sites, each triangle assigned
 *    to its lexicographically smallest vertex) and a brute-force sum over all site pairs
 *    and site triples found by distance.
 * 2. The fit objective and its gradient (Sec. IV-B: training by gradient descent with
 *    backpropagation): per-snapshot model energy S_b = sum of local energies of
 *    Eqs. (4)-(6), loss = mean over snapshots of ((S_b - E_b) / N)^2 with N sites per
 *    snapshot, and the gradient by the chain rule written out layer by layer.
 * 3. Central finite differences of that loss, to pin the analytic gradient.
 * Everything is FP64.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "smc_oracle.h"

/* ------------------------------------------------------------------ geometry helpers */

static int fo_lex_less(const int32_t *a, const int32_t *b) {
  for (int c = 0; c < 3; ++c) {
    if (a[c] != b[c]) return a[c] < b[c];
  }
  return 0;
}

static int fo_is_nbr(const int32_t *d, const int32_t off[26 * 3]) {
  for (int k = 0; k < 26; ++k)
    if (off[3 * k] == d[0] && off[3 * k + 1] == d[1] && off[3 * k + 2] == d[2]) return 1;
  return 0;
}

/* Shell (1..3) of a doubled-coordinate difference, 0 if beyond the third shell. */
static int fo_shell_of(const int32_t *d) {
  const int32_t r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  if (r2 == 3) return 1;  /* (1,1,1): a sqrt(3)/2 */
  if (r2 == 4) return 2;  /* (2,0,0): a */
  if (r2 == 8) return 3;  /* (2,2,0): a sqrt(2) */
  return 0;
}

/* Canonical form of the point set {p0, p1, p2}: translate by the lexicographically smallest
 * point and return the other two, in lexicographic order, as out[0..2] and out[3..5]. */
static void fo_canonical(const int32_t *p0, const int32_t *p1, const int32_t *p2, int32_t out[6]) {
  const int32_t *P[3] = {p0, p1, p2};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (fo_lex_less(P[j], P[i])) {
        const int32_t *t = P[i];
        P[i] = P[j];
        P[j] = t;
      }
  for (int c = 0; c < 3; ++c) {
    out[c] = P[1][c] - P[0][c];
    out[3 + c] = P[2][c] - P[0][c];
  }
}

/* Every distinct triangle (up to translation) whose three pairwise distances lie within the
 * third shell, as canonical offset pairs (a, b), a < b lexicographically, in lexicographic
 * order of (a, b).  Returns the count (the list is written up to max entries). */
int32_t or_ce_triangles(int32_t *out, int32_t max) {
  int32_t off[26 * 3], shell[26];
  or_shell_table(off, shell);
  int32_t list[26 * 26][6];
  int32_t n = 0;
  const int32_t zero[3] = {0, 0, 0};
  for (int i = 0; i < 26; ++i)
    for (int j = 0; j < 26; ++j) {
      if (i == j) continue;
      const int32_t d[3] = {off[3 * j] - off[3 * i], off[3 * j + 1] - off[3 * i + 1], off[3 * j + 2] - off[3 * i + 2]};
      if (!fo_is_nbr(d, off)) continue;
      int32_t c[6];
      fo_canonical(zero, &off[3 * i], &off[3 * j], c);
      int dup = 0;
      for (int t = 0; t < n && !dup; ++t) dup = memcmp(list[t], c, sizeof c) == 0;
      if (!dup) memcpy(list[n++], c, sizeof c);
    }
  /* lexicographic order of (a, b) */
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0; --j) {
      int less = 0;
      for (int c = 0; c < 6; ++c)
        if (list[j][c] != list[j - 1][c]) {
          less = list[j][c] < list[j - 1][c];
          break;
        }
      if (!less) break;
      int32_t t[6];
      memcpy(t, list[j], sizeof t);
      memcpy(list[j], list[j - 1], sizeof t);
      memcpy(list[j - 1], t, sizeof t);
    }
  for (int t = 0; t < n && t < max; ++t) memcpy(out + 6 * t, list[t], sizeof list[t]);
  return n;
}

/* ------------------------------------------------------------------ CE energies */

static double fo_pair(const or_ce *ce, int m, int p, int q) {
  const int S = ce->n_species;
  return ce->pair[((m - 1) * S + p) * S + q];
}

/* Site-local CE energy of site s: half of each pair term with its shell-1..3 neighbours and
 * every cluster item whose triangle has s as its canonical origin. */
double or_ce_site_energy(const int32_t L[3], const or_ce *ce, const uint8_t *occ, int64_t s) {
  int32_t off[26 * 3], shell[26];
  or_shell_table(off, shell);
  double e = 0.0;
  for (int k = 0; k < 26; ++k) e += 0.5 * fo_pair(ce, shell[k], occ[s], occ[or_neighbor(L, s, k)]);
  int32_t P[3];
  or_site_pos(L, s, P);
  for (int it = 0; it < ce->n_items; ++it) {
    const int32_t *o = ce->offsets + 6 * it;
    const int32_t Pa[3] = {P[0] + o[0], P[1] + o[1], P[2] + o[2]};
    const int32_t Pb[3] = {P[0] + o[3], P[1] + o[4], P[2] + o[5]};
    const uint8_t *sp = ce->species + 3 * it;
    if (occ[s] == sp[0] && occ[or_site_at(L, Pa)] == sp[1] && occ[or_site_at(L, Pb)] == sp[2]) e += ce->J[it];
  }
  return e;
}

double or_ce_total_local(const int32_t L[3], const or_ce *ce, const uint8_t *occ) {
  const int64_t N = or_n_sites(L);
  double e = 0.0;
  for (int64_t s = 0; s < N; ++s) e += or_ce_site_energy(L, ce, occ, s);
  return e;
}

/* Minimum-image doubled-coordinate difference q - p on the periodic lattice. */
static void fo_min_image(const int32_t L[3], const int32_t *p, const int32_t *q, int32_t *d) {
  for (int c = 0; c < 3; ++c) {
    const int32_t P = 2 * L[c];
    int32_t v = (q[c] - p[c]) % P;
    if (v < 0) v += P;
    if (v > L[c]) v -= P;
    d[c] = v;
  }
}

/* Brute force: every unordered site pair within the third shell, and every unordered site
 * triple whose three pairwise distances lie within it, matched against the items by shape
 * and species.  Needs lattices where minimum images are unique at these distances (>= 4
 * cells per axis). */
double or_ce_total_brute(const int32_t L[3], const or_ce *ce, const uint8_t *occ) {
  const int64_t N = or_n_sites(L);
  int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)N);
  for (int64_t s = 0; s < N; ++s) or_site_pos(L, s, pos + 3 * s);
  double e = 0.0;
  for (int64_t i = 0; i < N; ++i)
    for (int64_t j = i + 1; j < N; ++j) {
      int32_t d[3];
      fo_min_image(L, pos + 3 * i, pos + 3 * j, d);
      const int m = fo_shell_of(d);
      if (m) e += fo_pair(ce, m, occ[i], occ[j]);
    }
  const int32_t zero[3] = {0, 0, 0};
  for (int64_t i = 0; i < N; ++i)
    for (int64_t j = i + 1; j < N; ++j) {
      int32_t dij[3];
      fo_min_image(L, pos + 3 * i, pos + 3 * j, dij);
      if (!fo_shell_of(dij)) continue;
      for (int64_t k = j + 1; k < N; ++k) {
        int32_t dik[3], djk[3];
        fo_min_image(L, pos + 3 * i, pos + 3 * k, dik);
        if (!fo_shell_of(dik)) continue;
        fo_min_image(L, pos + 3 * j, pos + 3 * k, djk);
        if (!fo_shell_of(djk)) continue;
        /* positions relative to i; the canonical order tells which site is which vertex */
        const int32_t *V[3] = {zero, dij, dik};
        const int64_t site[3] = {i, j, k};
        int order[3] = {0, 1, 2};
        for (int a = 0; a < 3; ++a)
          for (int b = a + 1; b < 3; ++b)
            if (fo_lex_less(V[order[b]], V[order[a]])) {
              const int t = order[a];
              order[a] = order[b];
              order[b] = t;
            }
        int32_t c[6];
        fo_canonical(V[0], V[1], V[2], c);
        for (int it = 0; it < ce->n_items; ++it) {
          if (memcmp(ce->offsets + 6 * it, c, sizeof c) != 0) continue;
          const uint8_t *sp = ce->species + 3 * it;
          if (occ[site[order[0]]] == sp[0] && occ[site[order[1]]] == sp[1] && occ[site[order[2]]] == sp[2])
            e += ce->J[it];
        }
      }
    }
  free(pos);
  return e;
}

/* ------------------------------------------------------------------ MLP gradient */

static double fo_act(int32_t a, double z) {
  switch (a) {
    case OR_ACT_SILU: return z / (1.0 + exp(-z));
    case OR_ACT_IDENTITY: return z;
    case OR_ACT_RELU: return z > 0.0 ? z : 0.0;
    case OR_ACT_SQUARE: return z * z;
  }
  return NAN;
}

/* d act / dz.  SiLU: sigma(z) (1 + z (1 - sigma(z))). */
static double fo_act_deriv(int32_t a, double z) {
  switch (a) {
    case OR_ACT_SILU: {
      const double sg = 1.0 / (1.0 + exp(-z));
      return sg * (1.0 + z * (1.0 - sg));
    }
    case OR_ACT_IDENTITY: return 1.0;
    case OR_ACT_RELU: return z > 0.0 ? 1.0 : 0.0;
    case OR_ACT_SQUARE: return 2.0 * z;
  }
  return NAN;
}

int64_t or_n_params(const or_model *m) {
  const int64_t F = or_n_inputs(m->feature), H = m->hidden;
  return H * F + H + H * H + H + H + 1;
}

/* One site: energy, and if grad != NULL, grad += g * dE/dparams (reverse mode through
 * E = W2 h2 + b2, h2 = act1(z2), z2 = W1 h1 + b1, h1 = act0(z1), z1 = W0 x + b0). */
static double fo_site_backprop(const or_model *m, const double *x, double g, double *grad) {
  const int32_t F = or_n_inputs(m->feature), H = m->hidden;
  const double *W0 = m->params, *b0 = W0 + (int64_t)H * F, *W1 = b0 + H, *b1 = W1 + (int64_t)H * H,
               *W2 = b1 + H, *b2 = W2 + H;
  double z1[512], h1[512], z2[512], h2[512], gz2[512], gz1[512];
  for (int o = 0; o < H; ++o) {
    double acc = b0[o];
    for (int k = 0; k < F; ++k) acc += W0[(int64_t)o * F + k] * x[k];
    z1[o] = acc;
    h1[o] = fo_act(m->act0, acc);
  }
  for (int o = 0; o < H; ++o) {
    double acc = b1[o];
    for (int k = 0; k < H; ++k) acc += W1[(int64_t)o * H + k] * h1[k];
    z2[o] = acc;
    h2[o] = fo_act(m->act1, acc);
  }
  double e = b2[0];
  for (int k = 0; k < H; ++k) e += W2[k] * h2[k];
  if (!grad) return e;
  double *dW0 = grad, *db0 = dW0 + (int64_t)H * F, *dW1 = db0 + H, *db1 = dW1 + (int64_t)H * H, *dW2 = db1 + H,
         *db2 = dW2 + H;
  db2[0] += g;
  for (int o = 0; o < H; ++o) {
    dW2[o] += g * h2[o];
    gz2[o] = g * W2[o] * fo_act_deriv(m->act1, z2[o]);
    db1[o] += gz2[o];
    for (int k = 0; k < H; ++k) dW1[(int64_t)o * H + k] += gz2[o] * h1[k];
  }
  for (int k = 0; k < H; ++k) {
    double gh = 0.0;
    for (int o = 0; o < H; ++o) gh += W1[(int64_t)o * H + k] * gz2[o];
    gz1[k] = gh * fo_act_deriv(m->act0, z1[k]);
  }
  for (int o = 0; o < H; ++o) {
    db0[o] += gz1[o];
    for (int k = 0; k < F; ++k) dW0[(int64_t)o * F + k] += gz1[o] * x[k];
  }
  return e;
}

/* Energy of one snapshot; with grad != NULL also grad += g * dS/dparams. */
static double fo_snapshot(const int32_t L[3], const or_model *m, const uint8_t *occ, double g, double *grad) {
  const int64_t N = or_n_sites(L);
  double x[108], S = 0.0;
  for (int64_t j = 0; j < N; ++j) {
    or_features(L, m->feature, occ, j, -1, -1, x);
    S += fo_site_backprop(m, x, g, grad);
  }
  return S;
}

/* Model energies of `batch` snapshots (occupancies back to back) into S[batch]; if gE and
 * grad are given, grad = sum_b gE[b] dS_b/dparams (overwritten). */
void or_energy_grad(const int32_t L[3], const or_model *m, const uint8_t *snaps, int32_t batch, double *S,
                    const double *gE, double *grad, int32_t nthreads) {
  const int64_t N = or_n_sites(L), P = or_n_params(m);
  double *per = grad ? (double *)calloc((size_t)batch * (size_t)P, sizeof(double)) : NULL;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
  for (int32_t b = 0; b < batch; ++b) {
    const double s = fo_snapshot(L, m, snaps + (int64_t)b * N, grad ? gE[b] : 0.0, grad ? per + (int64_t)b * P : NULL);
    if (S) S[b] = s;
  }
  if (grad) {
    for (int64_t p = 0; p < P; ++p) grad[p] = 0.0;
    for (int32_t b = 0; b < batch; ++b)
      for (int64_t p = 0; p < P; ++p) grad[p] += per[(int64_t)b * P + p];
    free(per);
  }
}

/* Fit objective: loss = (1/B) sum_b ((S_b - E_b)/N)^2.  Writes S (nullable) and, if grad is
 * given, dloss/dparams (via dloss/dS_b = 2 (S_b - E_b) / (N^2 B)).  Returns the loss. */
double or_fit_loss_grad(const int32_t L[3], const or_model *m, const uint8_t *snaps, int32_t batch,
                        const double *labels, double *S_out, double *grad, int32_t nthreads) {
  const double N = (double)or_n_sites(L);
  double *S = (double *)malloc(sizeof(double) * (size_t)batch);
  or_energy_grad(L, m, snaps, batch, S, NULL, NULL, nthreads);
  double loss = 0.0;
  for (int32_t b = 0; b < batch; ++b) {
    const double r = (S[b] - labels[b]) / N;
    loss += r * r;
  }
  loss /= batch;
  if (grad) {
    double *gE = (double *)malloc(sizeof(double) * (size_t)batch);
    for (int32_t b = 0; b < batch; ++b) gE[b] = 2.0 * (S[b] - labels[b]) / (N * N * batch);
    or_energy_grad(L, m, snaps, batch, NULL, gE, grad, nthreads);
    free(gE);
  }
  if (S_out) memcpy(S_out, S, sizeof(double) * (size_t)batch);
  free(S);
  return loss;
}

/* Central differences (loss(p + h) - loss(p - h)) / 2h for the listed parameters. */
void or_fit_fd(const int32_t L[3], const or_model *m, const uint8_t *snaps, int32_t batch, const double *labels,
               const int64_t *idx, int32_t n, double h, double *out, int32_t nthreads) {
  const int64_t P = or_n_params(m);
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    double *w = (double *)malloc(sizeof(double) * (size_t)P);
    memcpy(w, m->params, sizeof(double) * (size_t)P);
    or_model mm = *m;
    mm.params = w;
#pragma omp for schedule(dynamic, 1)
    for (int32_t t = 0; t < n; ++t) {
      const int64_t p = idx[t];
      const double v = w[p];
      w[p] = v + h;
      const double lp = or_fit_loss_grad(L, &mm, snaps, batch, labels, NULL, NULL, 1);
      w[p] = v - h;
      const double lm = or_fit_loss_grad(L, &mm, snaps, batch, labels, NULL, NULL, 1);
      w[p] = v;
      out[t] = (lp - lm) / (2.0 * h);
    }
    free(w);
  }
}
