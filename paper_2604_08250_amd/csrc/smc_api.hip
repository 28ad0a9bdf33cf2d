// C ABI of libsmc (declared in include/smc.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>

#include <string>
#include <vector>

#include "../../include/smc.h"
#include "sweep_scalar.hpp"
#include "tables.hpp"

using namespace smc;

struct smc_ctx {
  smc_config cfg{};
  std::vector<int32_t> cells;
  std::vector<double> temps;
  std::vector<Replica> reps;
  int64_t n_total = 0;
  int32_t n_in = 0, hidden = 0, n_params = 0;
  hipStream_t stream = nullptr;
  uint8_t *occ = nullptr;
  float *ecache = nullptr;
  // library-owned device memory
  Replica *d_reps = nullptr;
  float *d_w32 = nullptr;
  double *d_w64 = nullptr;
  int8_t *d_omega = nullptr;
  int32_t omega_n = 0;
  double *d_erun = nullptr;       // [R] running FP64 totals
  double *d_escratch = nullptr;   // [R]
  double *d_partial = nullptr;    // per-block partial sums of accepted dE
  int64_t partial_cap = 0;
  uint64_t *d_counters = nullptr; // [4][R]
  double *d_site64 = nullptr;     // [N] FP64 site energies (lazy)
  uint64_t sweep = 0;
  double guard = 0.0;
  std::string err;
};

namespace {

int fail(smc_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPC(c, expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail((c), SMC_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

double default_guard(int prec) {
  switch (prec) {
    case SMC_FP32: return 1e-5;
    case SMC_BF16X3: return 5e-4;
    case SMC_BF16: return 1e-5;
    case SMC_FP8_E4M3: return 1e-5;
    default: return 0.0;
  }
}

unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

template <int FEAT, int H>
int launch_site_energies32(smc_ctx *c, float *out) {
  for (size_t r = 0; r < c->reps.size(); ++r) {
    hipLaunchKernelGGL((k_site_energies<FEAT, H, float>), dim3(grid_for(c->reps[r].n_sites, 128)),
                       dim3(128), 0, c->stream, c->d_reps, (int32_t)r, c->occ, c->d_w32, out);
  }
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

template <int FEAT, int H>
int launch_site_energies64(smc_ctx *c, double *out) {
  for (size_t r = 0; r < c->reps.size(); ++r) {
    hipLaunchKernelGGL((k_site_energies<FEAT, H, double>), dim3(grid_for(c->reps[r].n_sites, 128)),
                       dim3(128), 0, c->stream, c->d_reps, (int32_t)r, c->occ, c->d_w64, out);
  }
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

int site_energies32(smc_ctx *c, float *out) {
  if (c->cfg.feature == SMC_FEAT_COUNTS_S12) {
    if (c->hidden == 64) return launch_site_energies32<0, 64>(c, out);
    return launch_site_energies32<0, 128>(c, out);
  }
  if (c->hidden == 64) return launch_site_energies32<1, 64>(c, out);
  return launch_site_energies32<1, 128>(c, out);
}

int site_energies64(smc_ctx *c, double *out) {
  if (c->cfg.feature == SMC_FEAT_COUNTS_S12) {
    if (c->hidden == 64) return launch_site_energies64<0, 64>(c, out);
    return launch_site_energies64<0, 128>(c, out);
  }
  if (c->hidden == 64) return launch_site_energies64<1, 64>(c, out);
  return launch_site_energies64<1, 128>(c, out);
}

int ensure_site64(smc_ctx *c) {
  if (!c->d_site64) HIPC(c, hipMalloc(&c->d_site64, sizeof(double) * c->n_total));
  return SMC_OK;
}

// FP64 from-scratch totals per replica into d_escratch.
int scratch_totals(smc_ctx *c) {
  int rc = ensure_site64(c);
  if (rc) return rc;
  rc = site_energies64(c, c->d_site64);
  if (rc) return rc;
  for (size_t r = 0; r < c->reps.size(); ++r)
    hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(256), 0, c->stream, c->d_site64 + c->reps[r].site0,
                       c->reps[r].n_sites, c->d_escratch + r, 0);
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

int refresh(smc_ctx *c) {
  int rc;
  if (c->cfg.precision == SMC_FP64) {
    rc = scratch_totals(c);
    if (rc) return rc;
    hipLaunchKernelGGL(k_narrow, dim3(grid_for(c->n_total, 256)), dim3(256), 0, c->stream, c->d_site64,
                       c->ecache, c->n_total);
  } else {
    rc = site_energies32(c, c->ecache);
    if (rc) return rc;
    rc = scratch_totals(c);
    if (rc) return rc;
  }
  HIPC(c, hipMemcpyAsync(c->d_erun, c->d_escratch, sizeof(double) * c->reps.size(),
                         hipMemcpyDeviceToDevice, c->stream));
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

int load_params(smc_ctx *c, const float *params_dev) {
  const int64_t P = c->n_params;
  hipLaunchKernelGGL(k_copy_f32, dim3(grid_for(P, 256)), dim3(256), 0, c->stream, params_dev, c->d_w32, P);
  hipLaunchKernelGGL(k_widen, dim3(grid_for(P, 256)), dim3(256), 0, c->stream, params_dev, c->d_w64, P);
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

template <int FEAT, int H>
void launch_colour_scalar(smc_ctx *c, SweepArgs a, int64_t n_trials) {
  hipLaunchKernelGGL((k_sweep_colour_scalar<FEAT, H>), dim3(grid_for(n_trials, kScalarBlock)),
                     dim3(kScalarBlock), 0, c->stream, a);
}

int run_sweep(smc_ctx *c, const smc_stats *st, bool last) {
  const int R = (int)c->reps.size();
  int64_t poff = 0;
  std::vector<int64_t> pstart(R + 1, 0);
  for (int r = 0; r < R; ++r) {
    const Replica &rep = c->reps[r];
    const int64_t blocks = grid_for(rep.n_trials, kScalarBlock);
    for (int col = 0; col < rep.n_colours; ++col) {
      SweepArgs a{};
      a.reps = c->d_reps;
      a.occ = c->occ;
      a.ecache = c->ecache;
      a.w32 = c->d_w32;
      a.w64 = c->d_w64;
      a.omega = c->d_omega;
      a.omega_n = c->omega_n;
      a.replica = r;
      a.colour = col;
      a.fp64_mode = c->cfg.precision == SMC_FP64;
      a.seed = c->cfg.seed;
      a.sweep = c->sweep;
      a.guard = c->guard;
      a.partial = c->d_partial + poff;
      a.counters = c->d_counters;
      a.n_replicas = R;
      if (last && st) {
        a.trace_dE = st->trace_dE;
        a.trace_dE_fast = st->trace_dE_fast;
        a.trace_flags = st->trace_flags;
      }
      const bool onehot = c->cfg.feature == SMC_FEAT_ONEHOT_S123;
      if (!onehot && c->hidden == 64) launch_colour_scalar<0, 64>(c, a, rep.n_trials);
      else if (!onehot) launch_colour_scalar<0, 128>(c, a, rep.n_trials);
      else if (c->hidden == 64) launch_colour_scalar<1, 64>(c, a, rep.n_trials);
      else launch_colour_scalar<1, 128>(c, a, rep.n_trials);
      poff += blocks;
    }
    pstart[r + 1] = poff;
  }
  for (int r = 0; r < R; ++r)
    hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(256), 0, c->stream, c->d_partial + pstart[r],
                       pstart[r + 1] - pstart[r], c->d_erun + r, 1);
  HIPC(c, hipGetLastError());
  c->sweep++;
  return SMC_OK;
}

}  // namespace

extern "C" {

const char *smc_status_string(int s) {
  switch (s) {
    case SMC_OK: return "ok";
    case SMC_E_INVALID: return "invalid argument";
    case SMC_E_UNSUPPORTED: return "unsupported";
    case SMC_E_DEVICE: return "device error";
    case SMC_E_STATE: return "bad state";
    case SMC_E_NOMEM: return "out of memory";
  }
  return "unknown status";
}

const char *smc_last_error(const smc_ctx *c) { return c ? c->err.c_str() : "null context"; }

int smc_init(const smc_config *cfg, uint8_t *occ_dev, const float *params_dev, float *ecache_dev,
             void *hip_stream, smc_ctx **out) {
  if (!out) return SMC_E_INVALID;
  *out = nullptr;
  if (!cfg || !occ_dev || !params_dev || !ecache_dev || !cfg->cells || !cfg->temperature_K)
    return SMC_E_INVALID;
  if (cfg->n_replicas < 1 || cfg->n_species < 2 || cfg->n_species > 5) return SMC_E_INVALID;
  if (cfg->feature != SMC_FEAT_COUNTS_S12 && cfg->feature != SMC_FEAT_ONEHOT_S123) return SMC_E_INVALID;
  if (cfg->hidden != 64 && cfg->hidden != 128) return SMC_E_UNSUPPORTED;
  if (cfg->precision < SMC_FP32 || cfg->precision > SMC_FP64) return SMC_E_INVALID;
  if (cfg->precision != SMC_FP32 && cfg->precision != SMC_FP64) return SMC_E_UNSUPPORTED;
  for (int r = 0; r < cfg->n_replicas; ++r) {
    for (int a = 0; a < 3; ++a)
      if (cfg->cells[3 * r + a] < 4 || cfg->cells[3 * r + a] > (1 << 20)) return SMC_E_INVALID;
    const double T = cfg->temperature_K[r];
    if (!(T >= 0.0)) return SMC_E_INVALID;
  }
  smc_ctx *c = new (std::nothrow) smc_ctx();
  if (!c) return SMC_E_NOMEM;
  c->cfg = *cfg;
  c->cells.assign(cfg->cells, cfg->cells + 3 * cfg->n_replicas);
  c->temps.assign(cfg->temperature_K, cfg->temperature_K + cfg->n_replicas);
  c->cfg.cells = c->cells.data();
  c->cfg.temperature_K = c->temps.data();
  c->stream = (hipStream_t)hip_stream;
  c->occ = occ_dev;
  c->ecache = ecache_dev;
  c->n_in = cfg->feature == SMC_FEAT_COUNTS_S12 ? 12 : 108;
  c->hidden = cfg->hidden;
  c->n_params = c->hidden * c->n_in + c->hidden + c->hidden * c->hidden + c->hidden + c->hidden + 1;
  c->guard = cfg->guard_eV < 0 ? default_guard(cfg->precision) : cfg->guard_eV;
  int64_t site0 = 0, partials = 0;
  for (int r = 0; r < cfg->n_replicas; ++r) {
    c->reps.push_back(make_replica(&c->cells[3 * r], site0, c->temps[r]));
    site0 += c->reps.back().n_sites;
    partials += (int64_t)c->reps.back().n_colours * grid_for(c->reps.back().n_trials, kScalarBlock);
  }
  c->n_total = site0;
  const OmegaTable om = build_omega(cfg->feature == SMC_FEAT_COUNTS_S12 ? kNbrS12 : kNbr);
  c->omega_n = om.count;
  const int R = cfg->n_replicas;
  auto cleanup = [&](int code) {
    smc_destroy(c);
    return code;
  };
#define INIT_HIP(expr)                                  \
  do {                                                  \
    if ((expr) != hipSuccess) return cleanup(SMC_E_NOMEM); \
  } while (0)
  INIT_HIP(hipMalloc(&c->d_reps, sizeof(Replica) * R));
  INIT_HIP(hipMalloc(&c->d_w32, sizeof(float) * c->n_params));
  INIT_HIP(hipMalloc(&c->d_w64, sizeof(double) * c->n_params));
  INIT_HIP(hipMalloc(&c->d_omega, sizeof(om.off)));
  INIT_HIP(hipMalloc(&c->d_erun, sizeof(double) * R));
  INIT_HIP(hipMalloc(&c->d_escratch, sizeof(double) * R));
  INIT_HIP(hipMalloc(&c->d_partial, sizeof(double) * partials));
  INIT_HIP(hipMalloc(&c->d_counters, sizeof(uint64_t) * 4 * R));
#undef INIT_HIP
  c->partial_cap = partials;
  if (hipMemcpyAsync(c->d_reps, c->reps.data(), sizeof(Replica) * R, hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->d_omega, om.off.data(), sizeof(om.off), hipMemcpyHostToDevice, c->stream))
    return cleanup(SMC_E_DEVICE);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, c->stream, c->d_counters, (int64_t)4 * R, (uint64_t)0);
  int rc = load_params(c, params_dev);
  if (!rc) rc = refresh(c);
  if (!rc && hipStreamSynchronize(c->stream) != hipSuccess) rc = SMC_E_DEVICE;
  if (rc) return cleanup(rc);
  *out = c;
  return SMC_OK;
}

int smc_counters(smc_ctx *c, uint64_t *out, int32_t reset) {
  if (!c || !out) return SMC_E_INVALID;
  const int R = (int)c->reps.size();
  HIPC(c, hipMemcpyAsync(out, c->d_counters, sizeof(uint64_t) * 4 * R, hipMemcpyDeviceToHost, c->stream));
  if (reset) hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, c->stream, c->d_counters, (int64_t)4 * R, (uint64_t)0);
  HIPC(c, hipStreamSynchronize(c->stream));
  return SMC_OK;
}

int smc_sweep(smc_ctx *c, int32_t n_sweeps, smc_stats *st) {
  if (!c) return SMC_E_INVALID;
  if (n_sweeps < 0) return fail(c, SMC_E_INVALID, "n_sweeps < 0");
  const int R = (int)c->reps.size();
  std::vector<uint64_t> before(4 * R, 0), after(4 * R, 0);
  if (st) {
    int rc = smc_counters(c, before.data(), 0);
    if (rc) return rc;
  }
  for (int s = 0; s < n_sweeps; ++s) {
    int rc = run_sweep(c, st, s == n_sweeps - 1);
    if (rc) return rc;
  }
  if (st) {
    int rc = smc_counters(c, after.data(), 0);
    if (rc) return rc;
    for (int r = 0; r < R; ++r) {
      if (st->attempts) st->attempts[r] = after[0 * R + r] - before[0 * R + r];
      if (st->diff_species) st->diff_species[r] = after[1 * R + r] - before[1 * R + r];
      if (st->accepts) st->accepts[r] = after[2 * R + r] - before[2 * R + r];
      if (st->rechecks) st->rechecks[r] = after[3 * R + r] - before[3 * R + r];
    }
  }
  return SMC_OK;
}

int smc_energy(smc_ctx *c, double *e_scratch, double *e_running) {
  if (!c) return SMC_E_INVALID;
  int rc = scratch_totals(c);
  if (rc) return rc;
  const size_t R = c->reps.size();
  if (e_scratch)
    HIPC(c, hipMemcpyAsync(e_scratch, c->d_escratch, sizeof(double) * R, hipMemcpyDeviceToHost, c->stream));
  if (e_running)
    HIPC(c, hipMemcpyAsync(e_running, c->d_erun, sizeof(double) * R, hipMemcpyDeviceToHost, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  return SMC_OK;
}

int smc_site_energies(smc_ctx *c, int32_t precision, void *out_dev) {
  if (!c || !out_dev) return SMC_E_INVALID;
  if (precision == SMC_FP64) return site_energies64(c, (double *)out_dev);
  if (precision == SMC_FP32) return site_energies32(c, (float *)out_dev);
  return fail(c, SMC_E_UNSUPPORTED, "precision not built");
}

int smc_set_params(smc_ctx *c, const float *params_dev) {
  if (!c || !params_dev) return SMC_E_INVALID;
  int rc = load_params(c, params_dev);
  return rc ? rc : refresh(c);
}

int smc_refresh(smc_ctx *c) {
  if (!c) return SMC_E_INVALID;
  return refresh(c);
}

int smc_get_sweep(const smc_ctx *c, uint64_t *s) {
  if (!c || !s) return SMC_E_INVALID;
  *s = c->sweep;
  return SMC_OK;
}

int smc_set_sweep(smc_ctx *c, uint64_t s) {
  if (!c) return SMC_E_INVALID;
  c->sweep = s;
  return SMC_OK;
}

int smc_n_sites(const smc_ctx *c, int64_t *n) {
  if (!c || !n) return SMC_E_INVALID;
  *n = c->n_total;
  return SMC_OK;
}

int smc_n_colours(const smc_ctx *c, int32_t r, int32_t *n) {
  if (!c || !n || r < 0 || r >= (int32_t)c->reps.size()) return SMC_E_INVALID;
  *n = c->reps[r].n_colours;
  return SMC_OK;
}

void smc_destroy(smc_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  (void)hipFree(c->d_reps);
  (void)hipFree(c->d_w32);
  (void)hipFree(c->d_w64);
  (void)hipFree(c->d_omega);
  (void)hipFree(c->d_erun);
  (void)hipFree(c->d_escratch);
  (void)hipFree(c->d_partial);
  (void)hipFree(c->d_counters);
  (void)hipFree(c->d_site64);
  delete c;
}

}  // extern "C"
