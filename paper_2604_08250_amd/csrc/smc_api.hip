// C ABI of libsmc (declared in include/smc.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "context.hpp"
#include "smc.h"
#include "pack.hpp"
#include "double_lattice.hpp"
#include "fcc_host.hpp"
#include "recheck.hpp"
#include "reduce.hpp"
#include "site64.hpp"
#include "sweep_mfma.hpp"
#include "sweep_scalar.hpp"
#include "tables.hpp"

using namespace smc;

namespace {

void drop_graph(smc_ctx *c);

// Default FP64 re-decision band per precision: several times the largest |dE| error of the
// precision measured against FP64 over every trial of whole sweeps of the 256^3 lattice
// (3.0e7 trials; split BF16: largest 2.19e-5 eV, RMS 3.8e-6 eV; FP32: 1.6e-6, 2.8e-7).
double default_guard(int prec) {
  switch (prec) {
    case SMC_FP32: return 1e-5;
    case SMC_BF16X3: return 1e-4;
    case SMC_BF16: return 1e-5;
    case SMC_FP8_E4M3: return 1e-5;
    default: return 0.0;
  }
}

template <int FEAT, int H, typename T>
void launch_site_energies(smc_ctx *c, const T *W, T *out) {
  for (size_t r = 0; r < c->reps.size(); ++r)
    hipLaunchKernelGGL((k_site_energies<FEAT, H, T>), dim3(grid_for(c->reps[r].n_sites, 128)), dim3(128), 0,
                       c->stream, c->d_reps, (int32_t)r, c->occ, W, out);
}

template <typename T>
int site_energies_scalar(smc_ctx *c, const T *W, T *out) {
  const bool counts = c->cfg.feature == SMC_FEAT_COUNTS_S12;
  if (c->cfg.feature == SMC_FEAT_QSRO_S123) launch_site_energies<2, 0, T>(c, W, out);
  else if (counts && c->hidden == 64) launch_site_energies<0, 64, T>(c, W, out);
  else if (counts) launch_site_energies<0, 128, T>(c, W, out);
  else if (c->hidden == 64) launch_site_energies<1, 64, T>(c, W, out);
  else launch_site_energies<1, 128, T>(c, W, out);
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

// FP64 local energies of every site: the matrix-core kernel for the one-hot 128-hidden model
// (the re-decision's row arithmetic), the per-lane kernel otherwise.
int site_energies64(smc_ctx *c, double *out) {
  if (!c->mfma) return site_energies_scalar<double>(c, c->d_w64, out);
  for (size_t r = 0; r < c->reps.size(); ++r) {
    const int64_t items = (c->reps[r].n_sites + kS64Rows - 1) / kS64Rows;
    const unsigned grid = (unsigned)std::min<int64_t>(items, c->n_cu);  // one block per CU (LDS)
    hipLaunchKernelGGL(k_site_energies64_onehot, dim3(grid), dim3(kS64Threads), 0, c->stream, c->d_reps,
                       (int32_t)r, c->occ, c->d_w32t, c->d_w64t, out);
  }
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

int ensure_pack(smc_ctx *c, int P) {
  DevPack &dp = c->packs[P];
  if (dp.ready) return SMC_OK;
  dp.host = pack_model(P, c->host_params.data());
  if (!dp.dev) HIPC(c, hipMalloc(&dp.dev, dp.host.bytes.size()));
  HIPC(c, hipMemcpyAsync(dp.dev, dp.host.bytes.data(), dp.host.bytes.size(), hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));  // the host image may be replaced by a later pack
  dp.ready = true;
  return SMC_OK;
}

template <int P>
void launch_site_energies_mfma(smc_ctx *c, float *out, const uint8_t *occ = nullptr, int only = -1) {
  const DevPack &dp = c->packs[P];
  for (size_t r = 0; r < c->reps.size(); ++r) {
    if (only >= 0 && (int)r != only) continue;
    const int64_t tiles = (c->reps[r].n_sites + 31) / 32;
    const unsigned grid = (unsigned)std::min<int64_t>((tiles + 7) / 8, (int64_t)c->n_cu);
    hipLaunchKernelGGL((k_site_energies_mfma<P>), dim3(grid), dim3(kSeThreads), 0, c->stream, c->d_reps, (int32_t)r,
                       occ ? occ : c->occ, dp.dev, dp.host.b2, dp.host.k_scale_a0, dp.host.k_scale_a1,
                       dp.host.k_scale_h, dp.host.sh, out);
  }
}

// Local energies with the evaluator of precision P (float out).
int site_energies_fast(smc_ctx *c, int P, float *out) {
  if (c->fcc.on) return fcc::site_energies_fast(c, P, out);
  if (!c->mfma) {
    if (P != SMC_FP32) return fail(c, SMC_E_UNSUPPORTED, "low precisions need one-hot features and 128 hidden");
    return site_energies_scalar<float>(c, c->d_w32, out);
  }
  int rc = ensure_pack(c, P);
  if (rc) return rc;
  switch (P) {
    case SMC_FP32: launch_site_energies_mfma<kP32>(c, out); break;
    case SMC_BF16: launch_site_energies_mfma<kPBF16>(c, out); break;
    case SMC_BF16X3: launch_site_energies_mfma<kPBF16X3>(c, out); break;
    case SMC_FP8_E4M3: launch_site_energies_mfma<kPFP8>(c, out); break;
    default: return fail(c, SMC_E_INVALID, "precision");
  }
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

int ensure_site64(smc_ctx *c) {
  if (!c->d_site64) HIPC(c, hipMalloc(&c->d_site64, sizeof(double) * c->n_total));
  if (!c->d_psum) HIPC(c, hipMalloc(&c->d_psum, sizeof(double) * kSumChunks));
  return SMC_OK;
}

// FP64 from-scratch totals per replica into d_escratch.
int scratch_totals(smc_ctx *c) {
  if (c->fcc.on) return fcc::scratch_totals(c);
  int rc = ensure_site64(c);
  if (!rc) rc = site_energies64(c, c->d_site64);
  if (rc) return rc;
  for (size_t r = 0; r < c->reps.size(); ++r)
    sum_doubles(c->stream, c->d_site64 + c->reps[r].site0, c->reps[r].n_sites, c->d_psum, c->d_escratch + r);
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

int refresh(smc_ctx *c) {
  if (c->fcc.on) return fcc::refresh(c);
  int rc = scratch_totals(c);
  if (rc) return rc;
  if (c->cfg.precision == SMC_FP64)
    hipLaunchKernelGGL(k_narrow, dim3(grid_for(c->n_total, 256)), dim3(256), 0, c->stream, c->d_site64,
                       c->ecache, c->n_total);
  else if ((rc = site_energies_fast(c, c->cfg.precision, c->ecache)))
    return rc;
  const int R = (int)c->reps.size();
  HIPC(c, hipMemcpyAsync(c->d_ebase, c->d_escratch, sizeof(double) * R, hipMemcpyDeviceToDevice, c->stream));
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(R, 256)), dim3(256), 0, c->stream, (uint64_t *)c->d_efixed, (int64_t)R,
                     (uint64_t)0);
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

int load_params(smc_ctx *c, const float *params_dev) {
  if (c->fcc.on) {
    drop_graph(c);  // the captured sweep holds the output bias by value
    return fcc::load_params(c, params_dev);
  }
  const int64_t P = c->n_params;
  c->host_params.resize(P);
  HIPC(c, hipMemcpyAsync(c->host_params.data(), params_dev, sizeof(float) * P, hipMemcpyDeviceToHost, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < 4; ++k) c->packs[k].ready = false;
  drop_graph(c);  // the captured sweep holds the packed scales and output bias by value
  if (c->mfma) {
    // [input][unit] FP64 copy: consecutive threads of the re-decision kernel own consecutive
    // hidden units, so their weight loads are contiguous
    const int H = c->hidden, F = c->n_in;
    const float *p = c->host_params.data();
    std::vector<double> t(P);
    for (int o = 0; o < H; ++o)
      for (int f = 0; f < F; ++f) t[(size_t)f * H + o] = p[(size_t)o * F + f];
    const size_t b0 = (size_t)H * F, w1 = b0 + H;
    for (int o = 0; o < H; ++o) t[b0 + o] = p[b0 + o];
    for (int o = 0; o < H; ++o)
      for (int k = 0; k < H; ++k) t[w1 + (size_t)k * H + o] = p[w1 + (size_t)o * H + k];
    for (size_t q = w1 + (size_t)H * H; q < (size_t)P; ++q) t[q] = p[q];
    std::vector<float> tf(t.begin(), t.end());  // exact: every entry is an FP32 parameter
    HIPC(c, hipMemcpyAsync(c->d_w64t, t.data(), sizeof(double) * P, hipMemcpyHostToDevice, c->stream));
    HIPC(c, hipMemcpyAsync(c->d_w32t, tf.data(), sizeof(float) * P, hipMemcpyHostToDevice, c->stream));
    HIPC(c, hipStreamSynchronize(c->stream));
  }
  if (c->cfg.feature == SMC_FEAT_QSRO_S123) {
    // folded coefficients of the per-lane qSRO evaluator (FP64 and its FP32 rounding)
    const float *p = c->host_params.data();
    const double z[3] = {8.0, 6.0, 12.0};
    std::vector<double> f(kQsroPacked, 0.0);
    std::vector<float> f32(kQsroPacked);
    for (int m = 0; m < 3; ++m)
      for (int cc = 0; cc < 5; ++cc) {
        for (int q = 0; q < 5; ++q)
          if (q != cc) f[(m * 5 + cc) * 5 + q] = (double)p[(m * 5 + std::max(cc, q)) * 5 + std::min(cc, q)] / z[m];
        f[75 + m * 5 + cc] = (double)p[75 + m * 5 + cc] / (z[m] * z[m]);
      }
    double K = (double)p[91];
    for (int q = 0; q < 15; ++q) K += (double)p[90] * (double)p[75 + q] * (double)p[75 + q];
    f[90] = K;
    for (int q = 0; q < kQsroPacked; ++q) f32[q] = (float)f[q];
    HIPC(c, hipMemcpyAsync(c->d_w64, f.data(), sizeof(double) * kQsroPacked, hipMemcpyHostToDevice, c->stream));
    HIPC(c, hipMemcpyAsync(c->d_w32, f32.data(), sizeof(float) * kQsroPacked, hipMemcpyHostToDevice, c->stream));
    HIPC(c, hipStreamSynchronize(c->stream));
    return SMC_OK;
  }
  hipLaunchKernelGGL(k_copy_f32, dim3(grid_for(P, 256)), dim3(256), 0, c->stream, params_dev, c->d_w32, P);
  hipLaunchKernelGGL(k_widen, dim3(grid_for(P, 256)), dim3(256), 0, c->stream, params_dev, c->d_w64, P);
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

template <int FEAT, int H>
void launch_colour_scalar(smc_ctx *c, SweepArgs a, int64_t n_blocks) {
  hipLaunchKernelGGL((k_sweep_colour_scalar<FEAT, H>), dim3((unsigned)std::max<int64_t>(1, n_blocks)),
                     dim3(kScalarBlock), 0, c->stream, a);
}

// Kernel variants picked by the autotuner: link cells per group and XCD-contiguous order.
constexpr int kNumVariants = 4;
constexpr int kVariantGroup[kNumVariants] = {32, 32, 16, 16};
constexpr int kVariantXcd[kNumVariants] = {1, 0, 1, 0};

template <int P, int GROUP>
void launch_colour_mfma_g(smc_ctx *c, const MfmaArgs &a, int n_groups) {
  // the qSRO evaluation holds no weights in LDS (34 KB per block) and 125 VGPRs: two blocks
  // per CU (measured 1.31e9 against 0.95e9 attempts/s with one, 1.27e9 with four)
  int G = std::min(n_groups, (P == kPQsro ? 2 : 1) * c->n_cu);
  if (G >= 8) G -= G % 8;
  hipLaunchKernelGGL((k_sweep_colour_mfma<P, GROUP>), dim3(std::max(G, 1)), dim3(kMfmaThreads), 0, c->stream, a);
}

template <int P>
void launch_colour_mfma(smc_ctx *c, const MfmaArgs &a, int n_groups, int group) {
  if (group == 16) launch_colour_mfma_g<P, 16>(c, a, n_groups);
  else launch_colour_mfma_g<P, 32>(c, a, n_groups);
}

// Enqueue one sweep of the matrix-core path on c->stream (also used under graph capture):
// clear the per-colour queue counters, then per colour index one batched colour kernel over
// every replica that has that colour and one FP64 re-decision kernel; finally advance the
// device sweep counter.
int enqueue_sweep_mfma(smc_ctx *c, const smc_stats *st, bool trace) {
  const int R = (int)c->reps.size();
  const bool fp64 = c->cfg.precision == SMC_FP64;
  const bool qsro = c->qsro_tiled;
  const int P = qsro ? kPQsro : (fp64 ? SMC_FP32 : c->cfg.precision);
  const DevPack &dp = c->packs[qsro ? 0 : P];  // unused for qSRO
  const int group = kVariantGroup[c->variant];
  const int gi = group == 16 ? 1 : 0;
  const int64_t qwords = (c->max_colours + 1) / 2;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(qwords, 256)), dim3(256), 0, c->stream, (uint64_t *)c->d_qcount,
                     qwords, (uint64_t)0);
  for (int col = 0; col < c->max_colours; ++col) {
    const int so = c->seg_off[col], ns = c->seg_off[col + 1] - so;
    MfmaArgs a{};
    a.reps = c->d_reps;
    a.occ = c->occ;
    a.ecache = c->ecache;
    a.wpack = qsro ? (const uint8_t *)c->d_w32 : dp.dev;  // qSRO: the folded FP32 coefficients
    a.reg_off = c->d_reg_off;
    a.om_off = c->d_om_off;
    a.idx = c->d_idx;
    a.reg_pos = c->d_reg_pos;
    a.b2 = dp.host.b2;
    a.k_a0 = dp.host.k_scale_a0;
    a.k_a1 = dp.host.k_scale_a1;
    a.k_h = dp.host.k_scale_h;
    a.sh = dp.host.sh;
    a.colour = col;
    a.seg_rep = c->d_seg_rep + so;
    a.seg_start = c->d_seg_start[gi] + so + col;  // ns + 1 entries per colour
    a.nseg = ns;
    a.xcd_order = kVariantXcd[c->variant];
    a.seed = c->cfg.seed;
    a.sweep = c->d_sweep;
    a.guard = fp64 ? (double)INFINITY : c->guard;
    a.q_count = c->d_qcount + col;
    a.queue = c->d_queue;
    a.e_fixed = c->d_efixed;
    a.counters = c->d_counters;
    a.n_replicas = R;
    if (trace) {
      a.trace_dE = st->trace_dE;
      a.trace_dE_fast = st->trace_dE_fast;
      a.trace_flags = st->trace_flags;
    }
    const int n_groups = c->seg_groups[gi][col];
    const int ev = prof_begin(c);
    switch (P) {
      case SMC_FP32: launch_colour_mfma<kP32>(c, a, n_groups, group); break;
      case SMC_BF16: launch_colour_mfma<kPBF16>(c, a, n_groups, group); break;
      case SMC_BF16X3: launch_colour_mfma<kPBF16X3>(c, a, n_groups, group); break;
      case kPQsro: launch_colour_mfma<kPQsro>(c, a, n_groups, group); break;
      default: launch_colour_mfma<kPFP8>(c, a, n_groups, group); break;
    }
    prof_end(c, ev, 0);
    RecheckArgs ra{};
    ra.reps = c->d_reps;
    ra.occ = c->occ;
    ra.ecache = c->ecache;
    ra.w64 = c->d_w64t;
    ra.w32t = c->d_w32t;
    ra.reg_off = c->d_reg_off;
    ra.om_off = c->d_om_off;
    ra.idx = c->d_idx;
    ra.reg_pos = c->d_reg_pos;
    ra.q_count = c->d_qcount + col;
    ra.queue = c->d_queue;
    ra.e_fixed = c->d_efixed;
    ra.counters = c->d_counters;
    ra.n_replicas = R;
    ra.row_e = c->d_rowe;
    if (trace) {
      ra.trace_dE = st->trace_dE;
      ra.trace_flags = st->trace_flags;
    }
    const int ev2 = prof_begin(c);
    if (qsro)
      launch_recheck_qsro(ra, c->d_w64, c->col_trials[col], c->n_cu, c->stream);
    else
      launch_recheck(ra, c->col_trials[col], c->n_cu, c->stream);
    prof_end(c, ev2, 1);
  }
  hipLaunchKernelGGL(k_next_sweep, dim3(1), dim3(64), 0, c->stream, c->d_sweep);
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

void drop_graph(smc_ctx *c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
}

// Capture one sweep into a graph on the internal capture stream (the caller's stream may be
// the null stream, which cannot be captured); replays run on the caller's stream.
int build_graph(smc_ctx *c) {
  if (!c->cap_stream) HIPC(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipStream_t user = c->stream;
  c->stream = c->cap_stream;
  const bool prof = c->profiling;
  c->profiling = false;
  hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  int rc = e != hipSuccess ? SMC_E_DEVICE
                           : (c->fcc.on ? fcc::enqueue_sweep(c, nullptr, false) : enqueue_sweep_mfma(c, nullptr, false));
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
  c->stream = user;
  c->profiling = prof;
  if (rc || e2 != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return fail(c, SMC_E_DEVICE, std::string("graph capture failed: ") + hipGetErrorString(e2));
  }
  c->graph = g;
  if (hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
    drop_graph(c);
    return fail(c, SMC_E_DEVICE, "graph instantiation failed");
  }
  return SMC_OK;
}

// One sweep with the double-lattice strategy: per replica and colour, proposals into sigma1,
// all-site energies of sigma0 and sigma1, zone reductions and decisions, FP64 re-decisions,
// and sigma1 brought back to sigma0 at the trial pairs.
int enqueue_sweep_dl(smc_ctx *c, const smc_stats *st, bool trace) {
  const int R = (int)c->reps.size();
  const int P = c->cfg.precision;
  HIPC(c, hipMemcpyAsync(c->d_sigma1, c->occ, (size_t)c->n_total, hipMemcpyDeviceToDevice, c->stream));
  const int qslot = (c->max_colours + 1) & ~1;  // a 64-bit word of the counter array no colour uses
  for (int r = 0; r < R; ++r) {
    const Replica &rep = c->reps[r];
    for (int col = 0; col < rep.n_colours; ++col) {
      DlArgs a{};
      a.reps = c->d_reps;
      a.r = r;
      a.colour = col;
      a.sweep = c->d_sweep;
      a.seed = c->cfg.seed;
      a.occ = c->occ;
      a.sigma1 = c->d_sigma1;
      a.trials = c->d_dltrials;
      a.E0 = c->d_E0;
      a.E1 = c->d_E1;
      a.ecache = c->ecache;
      a.om_off = c->d_om_off;
      a.guard = c->guard;
      a.q_count = c->d_qcount + qslot;
      a.queue = c->d_queue;
      a.e_fixed = c->d_efixed;
      a.counters = c->d_counters;
      a.n_replicas = R;
      if (trace) {
        a.trace_dE = st->trace_dE;
        a.trace_dE_fast = st->trace_dE_fast;
        a.trace_flags = st->trace_flags;
      }
      const unsigned tg = grid_for(std::max<int64_t>(1, rep.n_trials), 256);
      hipLaunchKernelGGL(k_dl_propose, dim3(tg), dim3(256), 0, c->stream, a);
      switch (P) {
        case SMC_FP32:
          launch_site_energies_mfma<kP32>(c, c->d_E0, c->occ, r);
          launch_site_energies_mfma<kP32>(c, c->d_E1, c->d_sigma1, r);
          break;
        case SMC_BF16:
          launch_site_energies_mfma<kPBF16>(c, c->d_E0, c->occ, r);
          launch_site_energies_mfma<kPBF16>(c, c->d_E1, c->d_sigma1, r);
          break;
        case SMC_BF16X3:
          launch_site_energies_mfma<kPBF16X3>(c, c->d_E0, c->occ, r);
          launch_site_energies_mfma<kPBF16X3>(c, c->d_E1, c->d_sigma1, r);
          break;
        default:
          launch_site_energies_mfma<kPFP8>(c, c->d_E0, c->occ, r);
          launch_site_energies_mfma<kPFP8>(c, c->d_E1, c->d_sigma1, r);
          break;
      }
      hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, c->stream, (uint64_t *)(c->d_qcount + qslot), (int64_t)1,
                         (uint64_t)0);
      const int ev = prof_begin(c);
      hipLaunchKernelGGL(k_dl_decide, dim3(tg), dim3(256), 0, c->stream, a);
      prof_end(c, ev, 0);
      RecheckArgs ra{};
      ra.reps = c->d_reps;
      ra.occ = c->occ;
      ra.ecache = c->ecache;
      ra.w64 = c->d_w64t;
    ra.w32t = c->d_w32t;
      ra.reg_off = c->d_reg_off;
      ra.om_off = c->d_om_off;
      ra.idx = c->d_idx;
      ra.reg_pos = c->d_reg_pos;
      ra.q_count = c->d_qcount + qslot;
      ra.queue = c->d_queue;
      ra.e_fixed = c->d_efixed;
      ra.counters = c->d_counters;
      ra.n_replicas = R;
      ra.row_e = c->d_rowe;
      if (trace) {
        ra.trace_dE = st->trace_dE;
        ra.trace_flags = st->trace_flags;
      }
      const int ev2 = prof_begin(c);
      launch_recheck(ra, rep.n_trials, c->n_cu, c->stream);
      prof_end(c, ev2, 1);
      hipLaunchKernelGGL(k_dl_sync, dim3(tg), dim3(256), 0, c->stream, a);
    }
  }
  hipLaunchKernelGGL(k_next_sweep, dim3(1), dim3(64), 0, c->stream, c->d_sweep);
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

int run_sweep(smc_ctx *c, const smc_stats *st, bool last) {
  const int R = (int)c->reps.size();
  const bool trace = last && st;
  if (c->fcc.on) {
    int rc = SMC_OK;
    const int P = c->cfg.precision == SMC_FP64 ? SMC_FP32 : c->cfg.precision;
    if (c->fcc.model == 0 && (rc = fcc::ensure_pack(c, P))) return rc;
    if (c->use_graph && !trace && !c->profiling) {
      if (!c->graph_exec && (rc = build_graph(c))) return rc;
      HIPC(c, hipGraphLaunch(c->graph_exec, c->stream));
    } else if ((rc = fcc::enqueue_sweep(c, st, trace))) {
      return rc;
    }
  } else if (c->mfma || c->qsro_tiled) {
    int rc = SMC_OK;
    if (c->mfma && (rc = ensure_pack(c, c->cfg.precision == SMC_FP64 ? SMC_FP32 : c->cfg.precision))) return rc;
    if (c->strategy == SMC_STRATEGY_DOUBLE_LATTICE) {
      if ((rc = enqueue_sweep_dl(c, st, trace))) return rc;
    } else if (c->use_graph && !trace && !c->profiling) {
      if (!c->graph_exec && (rc = build_graph(c))) return rc;
      HIPC(c, hipGraphLaunch(c->graph_exec, c->stream));
    } else if ((rc = enqueue_sweep_mfma(c, st, trace))) {
      return rc;
    }
  } else {
    // per colour index, one launch over every replica that has that colour
    for (int col = 0; col < c->max_colours; ++col) {
      const int so = c->seg_off[col], ns = c->seg_off[col + 1] - so;
      const int64_t nb = c->seg_groups[2][col];
      SweepArgs a{};
      a.reps = c->d_reps;
      a.occ = c->occ;
      a.ecache = c->ecache;
      a.w32 = c->d_w32;
      a.w64 = c->d_w64;
      a.omega = c->d_omega;
      a.omega_n = c->omega_n;
      a.seg_rep = c->d_seg_rep + so;
      a.seg_start = c->d_seg_start[2] + so + col;  // ns + 1 entries per colour
      a.nseg = ns;
      a.colour = col;
      a.fp64_mode = c->cfg.precision == SMC_FP64;
      a.seed = c->cfg.seed;
      a.sweep = c->sweep;
      a.guard = c->guard;
      a.e_fixed = c->d_efixed;
      a.counters = c->d_counters;
      a.n_replicas = R;
      if (trace) {
        a.trace_dE = st->trace_dE;
        a.trace_dE_fast = st->trace_dE_fast;
        a.trace_flags = st->trace_flags;
      }
      const bool onehot = c->cfg.feature == SMC_FEAT_ONEHOT_S123;
      const int ev = prof_begin(c);
      if (c->cfg.feature == SMC_FEAT_QSRO_S123) launch_colour_scalar<2, 0>(c, a, nb);
      else if (!onehot && c->hidden == 64) launch_colour_scalar<0, 64>(c, a, nb);
      else if (!onehot) launch_colour_scalar<0, 128>(c, a, nb);
      else if (c->hidden == 64) launch_colour_scalar<1, 64>(c, a, nb);
      else launch_colour_scalar<1, 128>(c, a, nb);
      prof_end(c, ev, 0);
    }
    hipLaunchKernelGGL(k_next_sweep, dim3(1), dim3(64), 0, c->stream, c->d_sweep);
  }
  HIPC(c, hipGetLastError());
  c->sweep++;
  return SMC_OK;
}

}  // namespace

// ---------------------------------------------------------------- probe without allocation
//
// Work space of smc_delta_e64_noalloc: the probe's queue entries, their FP64 row energies and
// the queue length.  Each GPU the library runs on holds its own copy until the process ends.
// On the host this name is only a stand-in symbol, never a device address: host code uses the
// address resolved per device by noalloc_scratch() (at context creation, with the context's
// device current) and passes that to the kernels.
constexpr size_t kNoAllocEntryBytes = (sizeof(RecheckEntry) * SMC_NOALLOC_MAX_TRIALS + 255) / 256 * 256;
constexpr size_t kNoAllocRowBytes = sizeof(double) * kRows64 * SMC_NOALLOC_MAX_TRIALS;
constexpr size_t kNoAllocBytes = kNoAllocEntryBytes + kNoAllocRowBytes + 256;
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

namespace smc {

// Device address of `scratch` on device `dev`, resolved once per device (the device must be
// current).  SMC_E_DEVICE if the runtime cannot resolve it.
int noalloc_scratch(int dev, void **out) {
  static std::mutex mu;
  static std::vector<void *> addr;
  std::lock_guard<std::mutex> lock(mu);
  if (dev < 0) return SMC_E_INVALID;
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SMC_E_DEVICE;
    addr[dev] = p;
  }
  *out = addr[dev];
  return SMC_OK;
}

// Queue entries of the probe from device site indices: the proposal of each trial site (the
// Philox block of (site, sweep, replica, 0), partner slot r0 >> 61).  A site outside the
// replica gets no evaluation: partner -1 and dE NaN.
__global__ void k_probe_entries(const Replica *reps, int32_t replica, uint64_t sweep, uint64_t seed,
                                const int64_t *sites, int32_t n, RecheckEntry *entries, uint32_t *q_count,
                                int64_t *partner_out, double *dE_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) *q_count = (uint32_t)n;
  if (k >= n) return;
  const Replica R = reps[replica];
  const int64_t s = sites[k];
  RecheckEntry &e = entries[k];
  e.replica = replica;
  e.theta = 0.0;
  e.dE_fast = 0.0f;
  e.has_reg = 0;
  if (s < 0 || s >= R.n_sites) {
    e.site = -1;
    e.partner = -1;
    e.dir = 0;
    if (partner_out) partner_out[k] = -1;
    dE_out[k] = (double)NAN;
    return;
  }
  const U64x4 r = philox4x64_10((uint64_t)s, sweep, (uint64_t)replica, 0, seed, 0);
  const int d = (int)(r.v[0] >> 61);
  const Pos p = site_pos(s, R.L[0], R.L[1]);
  e.site = s;
  e.dir = d;
  e.partner = site_at(p, shell_dx(d), shell_dy(d), shell_dz(d), R.L[0], R.L[1], R.L[2]);
  if (partner_out) partner_out[k] = e.partner;
}

}  // namespace smc

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
  if (cfg->precision < SMC_FP32 || cfg->precision > SMC_FP64) return SMC_E_INVALID;
  if (cfg->lattice == SMC_LATTICE_FCC)
    return fcc::create(cfg, occ_dev, params_dev, ecache_dev, hip_stream,
                       cfg->guard_eV < 0 ? default_guard(cfg->precision) : cfg->guard_eV, out);
  if (cfg->lattice != SMC_LATTICE_BCC) return SMC_E_INVALID;
  if (cfg->feature != SMC_FEAT_COUNTS_S12 && cfg->feature != SMC_FEAT_ONEHOT_S123 &&
      cfg->feature != SMC_FEAT_QSRO_S123)
    return SMC_E_INVALID;
  if (cfg->precision < SMC_FP32 || cfg->precision > SMC_FP64) return SMC_E_INVALID;
  const bool qsro = cfg->feature == SMC_FEAT_QSRO_S123;
  if (!qsro && cfg->hidden != 64 && cfg->hidden != 128) return SMC_E_UNSUPPORTED;
  const bool mfma = cfg->feature == SMC_FEAT_ONEHOT_S123 && cfg->hidden == 128;
  if (!mfma && cfg->precision != SMC_FP32 && cfg->precision != SMC_FP64) return SMC_E_UNSUPPORTED;
  int64_t total = 0;
  for (int r = 0; r < cfg->n_replicas; ++r) {
    for (int a = 0; a < 3; ++a)
      if (cfg->cells[3 * r + a] < 4 || cfg->cells[3 * r + a] > 4096) return SMC_E_INVALID;
    const double T = cfg->temperature_K[r];
    if (!(T >= 0.0)) return SMC_E_INVALID;
    total += 2LL * cfg->cells[3 * r] * cfg->cells[3 * r + 1] * cfg->cells[3 * r + 2];
  }
  if (total >= (1LL << 31)) return SMC_E_UNSUPPORTED;  // replica-local indices are 32-bit in the fast path
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
  c->mfma = mfma;
  c->qsro_tiled = qsro && cfg->precision == SMC_FP32;
  c->n_in = cfg->feature == SMC_FEAT_COUNTS_S12 ? 12 : 108;
  c->hidden = cfg->hidden;
  c->n_params = c->hidden * c->n_in + c->hidden + c->hidden * c->hidden + c->hidden + c->hidden + 1;
  if (qsro) {
    c->n_in = 0;
    c->hidden = 0;
    c->n_params = 92;  // V[3][5][5], W[3][5], lambda, C
  }
  c->guard = cfg->guard_eV < 0 ? default_guard(cfg->precision) : cfg->guard_eV;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0) c->n_cu = n;
  }
  c->device = dev;
  int64_t site0 = 0, max_trials = 0;
  for (int r = 0; r < cfg->n_replicas; ++r) {
    c->reps.push_back(make_replica(&c->cells[3 * r], site0, c->temps[r]));
    site0 += c->reps.back().n_sites;
    max_trials = std::max(max_trials, c->reps.back().n_trials);
    c->colours_total += c->reps.back().n_colours;
  }
  c->n_total = site0;
  // batched schedule: colour index -> replicas that have it, with flattened group offsets
  std::vector<int32_t> seg_rep, seg_start[3];
  for (const Replica &rp : c->reps) c->max_colours = std::max(c->max_colours, rp.n_colours);
  c->seg_off.assign(c->max_colours + 1, 0);
  for (int k = 0; k < 3; ++k) c->seg_groups[k].assign(c->max_colours, 0);
  c->col_trials.assign(c->max_colours, 0);
  for (int col = 0; col < c->max_colours; ++col) {
    c->seg_off[col] = (int32_t)seg_rep.size();
    int32_t g32 = 0, g16 = 0, gs = 0;
    for (int k = 0; k < 3; ++k) seg_start[k].push_back(0);
    for (int r = 0; r < cfg->n_replicas; ++r) {
      const Replica &rp = c->reps[r];
      if (rp.n_colours <= col) continue;
      seg_rep.push_back(r);
      const int64_t nt = colour_trials(rp, col);
      g32 += (int32_t)((nt + 31) / 32);
      g16 += (int32_t)((nt + 15) / 16);
      gs += (int32_t)((nt + kScalarBlock - 1) / kScalarBlock);
      seg_start[0].push_back(g32);
      seg_start[1].push_back(g16);
      seg_start[2].push_back(gs);
      c->col_trials[col] += nt;
    }
    c->seg_groups[0][col] = g32;
    c->seg_groups[1][col] = g16;
    c->seg_groups[2][col] = gs;
    max_trials = std::max(max_trials, c->col_trials[col]);
  }
  c->seg_off[c->max_colours] = (int32_t)seg_rep.size();
  const OmegaTable om = build_omega(cfg->feature == SMC_FEAT_COUNTS_S12 ? kNbrS12 : kNbr);
  c->omega_n = om.count;
  const int R = cfg->n_replicas;
  auto cleanup = [&](int code) {
    smc_destroy(c);
    return code;
  };
#define INIT_HIP(expr)                                     \
  do {                                                     \
    if ((expr) != hipSuccess) return cleanup(SMC_E_NOMEM); \
  } while (0)
  INIT_HIP(hipMalloc(&c->d_reps, sizeof(Replica) * R));
  INIT_HIP(hipMalloc(&c->d_w32, sizeof(float) * c->n_params));
  INIT_HIP(hipMalloc(&c->d_w64, sizeof(double) * c->n_params));
  INIT_HIP(hipMalloc(&c->d_w64t, sizeof(double) * c->n_params));
  INIT_HIP(hipMalloc(&c->d_w32t, sizeof(float) * c->n_params));
  INIT_HIP(hipMalloc(&c->d_omega, sizeof(om.off)));
  INIT_HIP(hipMalloc(&c->d_ebase, sizeof(double) * R));
  INIT_HIP(hipMalloc(&c->d_efixed, sizeof(unsigned long long) * R));
  INIT_HIP(hipMalloc(&c->d_escratch, sizeof(double) * R));
  INIT_HIP(hipMalloc(&c->d_counters, sizeof(uint64_t) * 4 * R));
  INIT_HIP(hipMalloc(&c->d_sweep, sizeof(uint64_t)));
  INIT_HIP(hipMemset(c->d_sweep, 0, sizeof(uint64_t)));
  if (hipMemcpyAsync(c->d_reps, c->reps.data(), sizeof(Replica) * R, hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->d_omega, om.off.data(), sizeof(om.off), hipMemcpyHostToDevice, c->stream))
    return cleanup(SMC_E_DEVICE);
  // batched schedule tables (both sweep paths)
  INIT_HIP(hipMalloc(&c->d_seg_rep, sizeof(int32_t) * std::max<size_t>(1, seg_rep.size())));
  for (int k = 0; k < 3; ++k) {
    INIT_HIP(hipMalloc(&c->d_seg_start[k], sizeof(int32_t) * seg_start[k].size()));
    INIT_HIP(hipMemcpy(c->d_seg_start[k], seg_start[k].data(), sizeof(int32_t) * seg_start[k].size(),
                       hipMemcpyHostToDevice));
  }
  if (!seg_rep.empty())
    INIT_HIP(hipMemcpy(c->d_seg_rep, seg_rep.data(), sizeof(int32_t) * seg_rep.size(), hipMemcpyHostToDevice));
  if (mfma) {
    // work space of the probe without allocation, resolved once per device
    if (noalloc_scratch(dev, &c->scratch) != SMC_OK) {
      smc_destroy(c);
      return SMC_E_DEVICE;
    }
  }
  if (mfma || c->qsro_tiled) {
    const RegionTables t = build_region_tables();
    if (t.reg_off.empty()) return cleanup(SMC_E_DEVICE);
    c->queue_cap = max_trials;
    INIT_HIP(hipMalloc(&c->d_reg_off, sizeof(uint16_t) * t.reg_off.size()));
    INIT_HIP(hipMalloc(&c->d_om_off, sizeof(uint16_t) * t.om_off.size()));
    INIT_HIP(hipMalloc(&c->d_idx, t.idx.size()));
    INIT_HIP(hipMalloc(&c->d_reg_pos, t.reg_pos.size()));
    INIT_HIP(hipMalloc(&c->d_queue, sizeof(RecheckEntry) * c->queue_cap));
    INIT_HIP(hipMalloc(&c->d_rowe, sizeof(double) * kRows64 * c->queue_cap));
    INIT_HIP(hipMalloc(&c->d_qcount, sizeof(uint32_t) * (c->max_colours + 4)));
    if (hipMemcpy(c->d_reg_off, t.reg_off.data(), sizeof(uint16_t) * t.reg_off.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(c->d_om_off, t.om_off.data(), sizeof(uint16_t) * t.om_off.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(c->d_idx, t.idx.data(), t.idx.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(c->d_reg_pos, t.reg_pos.data(), t.reg_pos.size(), hipMemcpyHostToDevice))
      return cleanup(SMC_E_DEVICE);
  }
#undef INIT_HIP
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(4 * R, 256)), dim3(256), 0, c->stream, c->d_counters, (int64_t)4 * R,
                     (uint64_t)0);
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
  if (reset)
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(4 * R, 256)), dim3(256), 0, c->stream, c->d_counters, (int64_t)4 * R,
                     (uint64_t)0);
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
  std::vector<double> es(R), eb(R);
  std::vector<unsigned long long> ef(R);
  HIPC(c, hipMemcpyAsync(es.data(), c->d_escratch, sizeof(double) * R, hipMemcpyDeviceToHost, c->stream));
  HIPC(c, hipMemcpyAsync(eb.data(), c->d_ebase, sizeof(double) * R, hipMemcpyDeviceToHost, c->stream));
  HIPC(c, hipMemcpyAsync(ef.data(), c->d_efixed, sizeof(unsigned long long) * R, hipMemcpyDeviceToHost, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  for (size_t r = 0; r < R; ++r) {
    if (e_scratch) e_scratch[r] = es[r];
    if (e_running) e_running[r] = eb[r] + (double)(long long)ef[r] * 0x1.0p-32;
  }
  return SMC_OK;
}

int smc_site_energies(smc_ctx *c, int32_t precision, void *out_dev) {
  if (!c || !out_dev) return SMC_E_INVALID;
  if (c->fcc.on && precision == SMC_FP64) return fcc::site_energies64(c, (double *)out_dev);
  if (precision == SMC_FP64) return site_energies64(c, (double *)out_dev);
  if (precision < SMC_FP32 || precision > SMC_FP8_E4M3) return fail(c, SMC_E_INVALID, "precision");
  return site_energies_fast(c, precision, (float *)out_dev);
}

int smc_delta_e64(smc_ctx *c, int32_t replica, uint64_t sweep, const int64_t *sites, int32_t n,
                  int64_t *partner_out, double *dE_out) {
  if (!c || !sites || n < 0 || replica < 0 || replica >= (int32_t)c->reps.size()) return SMC_E_INVALID;
  if (n == 0) return SMC_OK;
  if (c->fcc.on) return fcc::delta_e64(c, replica, sweep, sites, n, partner_out, dE_out);
  if (!c->mfma) return fail(c, SMC_E_UNSUPPORTED, "FP64 probe needs one-hot features and 128 hidden");
  const Replica &R = c->reps[replica];
  std::vector<RecheckEntry> h(n);
  for (int32_t k = 0; k < n; ++k) {
    if (sites[k] < 0 || sites[k] >= R.n_sites) return fail(c, SMC_E_INVALID, "site out of range");
    const U64x4 r = philox4x64_10((uint64_t)sites[k], sweep, (uint64_t)replica, 0, c->cfg.seed, 0);
    const int d = (int)(r.v[0] >> 61);
    const Pos p = site_pos(sites[k], R.L[0], R.L[1]);
    RecheckEntry e{};
    e.site = sites[k];
    e.partner = site_at(p, shell_dx(d), shell_dy(d), shell_dz(d), R.L[0], R.L[1], R.L[2]);
    e.replica = replica;
    e.dir = d;
    h[k] = e;
    if (partner_out) partner_out[k] = e.partner;
  }
  RecheckEntry *d_e = nullptr;
  double *d_out = nullptr, *d_rowe = nullptr;
  uint32_t *d_n = nullptr;
  const uint32_t nn = (uint32_t)n;
  int rc = SMC_OK;
  if (hipMalloc(&d_e, sizeof(RecheckEntry) * n) || hipMalloc(&d_out, sizeof(double) * n) ||
      hipMalloc(&d_n, sizeof(uint32_t)) || hipMalloc(&d_rowe, sizeof(double) * kRows64 * n))
    rc = fail(c, SMC_E_NOMEM, "probe buffers");
  if (!rc && (hipMemcpyAsync(d_e, h.data(), sizeof(RecheckEntry) * n, hipMemcpyHostToDevice, c->stream) ||
              hipMemcpyAsync(d_n, &nn, sizeof(uint32_t), hipMemcpyHostToDevice, c->stream)))
    rc = fail(c, SMC_E_DEVICE, "probe upload");
  if (!rc) {
    RecheckArgs ra{};
    ra.reps = c->d_reps;
    ra.occ = c->occ;
    ra.ecache = c->ecache;
    ra.w64 = c->d_w64t;
    ra.w32t = c->d_w32t;
    ra.reg_off = c->d_reg_off;
    ra.om_off = c->d_om_off;
    ra.idx = c->d_idx;
    ra.reg_pos = c->d_reg_pos;
    ra.q_count = d_n;
    ra.queue = d_e;
    ra.e_fixed = c->d_efixed;
    ra.counters = c->d_counters;
    ra.n_replicas = (int32_t)c->reps.size();
    ra.probe_dE = d_out;
    ra.row_e = d_rowe;
    launch_recheck(ra, n, c->n_cu, c->stream);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(dE_out, d_out, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream) ||
        hipStreamSynchronize(c->stream))
      rc = fail(c, SMC_E_DEVICE, "probe kernel");
  }
  (void)hipFree(d_e);
  (void)hipFree(d_out);
  (void)hipFree(d_rowe);
  (void)hipFree(d_n);
  return rc;
}


int smc_delta_e64_noalloc(smc_ctx *c, int32_t replica, uint64_t sweep, const int64_t *sites_dev, int32_t n,
                          int64_t *partner_dev, double *dE_dev) {
  if (!c) return SMC_E_INVALID;
  if (replica < 0 || replica >= (int32_t)c->reps.size()) return fail(c, SMC_E_INVALID, "replica out of range");
  if (n < 0) return fail(c, SMC_E_INVALID, "n < 0");
  if (n > SMC_NOALLOC_MAX_TRIALS)
    return fail(c, SMC_E_INVALID, "n = " + std::to_string(n) + " exceeds the work space of " +
                                      std::to_string(SMC_NOALLOC_MAX_TRIALS) + " trials (SMC_NOALLOC_MAX_TRIALS)");
  if (c->fcc.on || !c->mfma)
    return fail(c, SMC_E_UNSUPPORTED, "the probe without allocation needs BCC, one-hot features and 128 hidden");
  if (n == 0) return SMC_OK;
  if (!sites_dev || !dE_dev) return fail(c, SMC_E_INVALID, "null device array");
  if (!c->scratch) return fail(c, SMC_E_DEVICE, "work-space address not resolved");
  RecheckEntry *entries = (RecheckEntry *)c->scratch;
  double *rows = (double *)((uint8_t *)c->scratch + kNoAllocEntryBytes);
  uint32_t *qn = (uint32_t *)((uint8_t *)c->scratch + kNoAllocEntryBytes + kNoAllocRowBytes);
  hipLaunchKernelGGL(k_probe_entries, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, c->d_reps, replica, sweep,
                     c->cfg.seed, sites_dev, n, entries, qn, partner_dev, dE_dev);
  RecheckArgs ra{};
  ra.reps = c->d_reps;
  ra.occ = c->occ;
  ra.ecache = c->ecache;
  ra.w64 = c->d_w64t;
    ra.w32t = c->d_w32t;
  ra.reg_off = c->d_reg_off;
  ra.om_off = c->d_om_off;
  ra.idx = c->d_idx;
  ra.reg_pos = c->d_reg_pos;
  ra.q_count = qn;
  ra.queue = entries;
  ra.e_fixed = c->d_efixed;
  ra.counters = c->d_counters;
  ra.n_replicas = (int32_t)c->reps.size();
  ra.probe_dE = dE_dev;  // probe mode: writes dE, changes nothing else
  ra.row_e = rows;
  launch_recheck(ra, n, c->n_cu, c->stream);
  HIPC(c, hipGetLastError());
  return SMC_OK;
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

int smc_profile(smc_ctx *c, int32_t enable) {
  if (!c) return SMC_E_INVALID;
  HIPC(c, hipStreamSynchronize(c->stream));
  c->profiling = enable != 0;
  if (enable) c->ev_used = 0;
  return SMC_OK;
}

int smc_kernel_times(smc_ctx *c, double *colour_ms, double *recheck_ms, int64_t *colour_launches) {
  if (!c) return SMC_E_INVALID;
  HIPC(c, hipStreamSynchronize(c->stream));
  double t[2] = {0.0, 0.0};
  int64_t n0 = 0;
  for (size_t k = 0; k < c->ev_used; ++k) {
    float ms = 0.0f;
    HIPC(c, hipEventElapsedTime(&ms, c->ev_pool[2 * k], c->ev_pool[2 * k + 1]));
    t[c->ev_kind[k]] += ms;
    if (c->ev_kind[k] == 0) ++n0;
  }
  if (colour_ms) *colour_ms = t[0];
  if (recheck_ms) *recheck_ms = t[1];
  if (colour_launches) *colour_launches = n0;
  return SMC_OK;
}

int smc_get_sweep(const smc_ctx *c, uint64_t *s) {
  if (!c || !s) return SMC_E_INVALID;
  *s = c->sweep;
  return SMC_OK;
}

int smc_set_sweep(smc_ctx *c, uint64_t s) {
  if (!c) return SMC_E_INVALID;
  HIPC(c, hipMemcpyAsync(c->d_sweep, &s, sizeof(uint64_t), hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  c->sweep = s;
  return SMC_OK;
}

int smc_set_variant(smc_ctx *c, int32_t variant) {
  if (!c || variant < 0 || variant >= kNumVariants) return SMC_E_INVALID;
  if (variant != c->variant) drop_graph(c);
  c->variant = variant;
  return SMC_OK;
}

int smc_get_variant(const smc_ctx *c, int32_t *variant) {
  if (!c || !variant) return SMC_E_INVALID;
  *variant = c->variant;
  return SMC_OK;
}

int smc_set_temperatures(smc_ctx *c, const double *temperature_K) {
  if (!c || !temperature_K) return SMC_E_INVALID;
  const int R = (int)c->reps.size();
  for (int r = 0; r < R; ++r)
    if (!(temperature_K[r] >= 0.0)) return fail(c, SMC_E_INVALID, "temperatures must be >= 0 or +inf");
  for (int r = 0; r < R; ++r) {
    c->temps[r] = temperature_K[r];
    c->reps[r].temperature = temperature_K[r];
  }
  // kernels (and replays of the captured sweep) read the replica table at run time
  HIPC(c, hipMemcpyAsync(c->d_reps, c->reps.data(), sizeof(Replica) * R, hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  return SMC_OK;
}

int smc_warren_cowley(smc_ctx *c, int32_t replica, double *alpha) {
  if (!c || !alpha || replica < 0 || replica >= (int32_t)c->reps.size()) return SMC_E_INVALID;
  const int S = c->cfg.n_species;
  unsigned long long *d = nullptr;
  if (hipMalloc(&d, sizeof(unsigned long long) * (3 * S * S + S)) != hipSuccess) return fail(c, SMC_E_NOMEM, "counts");
  std::vector<unsigned long long> h(3 * S * S + S);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, c->stream, (uint64_t *)d, (int64_t)(3 * S * S + S), (uint64_t)0);
  const int64_t n = c->reps[replica].n_sites;
  const unsigned grid = (unsigned)std::min<int64_t>(grid_for(n, 256), 4 * (int64_t)c->n_cu);
  if (c->fcc.on)
    hipLaunchKernelGGL(fcc::k_pair_counts, dim3(grid), dim3(256), 0, c->stream, c->d_reps, replica, c->occ, S, d,
                       d + 3 * S * S);
  else
    hipLaunchKernelGGL(k_pair_counts, dim3(grid), dim3(256), 0, c->stream, c->d_reps, replica, c->occ, S, d,
                       d + 3 * S * S);
  const hipError_t e1 = hipMemcpyAsync(h.data(), d, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost,
                                       c->stream);
  const hipError_t e2 = hipStreamSynchronize(c->stream);
  (void)hipFree(d);
  if (e1 != hipSuccess || e2 != hipSuccess) return fail(c, SMC_E_DEVICE, "pair counts");
  const unsigned long long *cnt = h.data(), *nsp = h.data() + 3 * S * S;
  const double zb[3] = {8.0, 6.0, 12.0}, zf[3] = {12.0, 6.0, 24.0};
  const double *z = c->fcc.on ? zf : zb;
  for (int m = 0; m < 3; ++m)
    for (int p = 0; p < S; ++p)
      for (int q = 0; q < S; ++q) {
        const double cq = (double)nsp[q] / (double)n;
        const double pq = nsp[p] > 0 ? (double)cnt[(m * S + p) * S + q] / ((double)nsp[p] * z[m]) : 0.0;
        alpha[(m * S + p) * S + q] = (cq > 0 && nsp[p] > 0) ? 1.0 - pq / cq : 0.0;
      }
  return SMC_OK;
}

int smc_lattice_shells(int32_t lattice, int32_t *off, int32_t *shell, int32_t max_slots) {
  if (max_slots < 0 || (max_slots > 0 && (!off || !shell))) return SMC_E_INVALID;
  if (lattice == SMC_LATTICE_BCC) {
    for (int k = 0; k < kNbr && k < max_slots; ++k) {
      off[3 * k] = shell_dx(k);
      off[3 * k + 1] = shell_dy(k);
      off[3 * k + 2] = shell_dz(k);
      shell[k] = shell_of(k);
    }
    return kNbr;
  }
  if (lattice == SMC_LATTICE_FCC) {
    for (int k = 0; k < fcc::kNbr && k < max_slots; ++k) {
      off[3 * k] = fcc::dx(k);
      off[3 * k + 1] = fcc::dy(k);
      off[3 * k + 2] = fcc::dz(k);
      shell[k] = fcc::shell_of(k);
    }
    return fcc::kNbr;
  }
  return SMC_E_INVALID;
}

int smc_set_strategy(smc_ctx *c, int32_t strategy) {
  if (!c) return SMC_E_INVALID;
  if (strategy != SMC_STRATEGY_ZONE && strategy != SMC_STRATEGY_DOUBLE_LATTICE)
    return fail(c, SMC_E_INVALID, "unknown strategy");
  if (strategy == SMC_STRATEGY_DOUBLE_LATTICE) {
    if (!c->mfma || c->cfg.precision == SMC_FP64)
      return fail(c, SMC_E_UNSUPPORTED, "the double-lattice strategy needs one-hot features, 128 hidden units "
                                        "and a matrix-core precision");
    int64_t most = 1;
    for (const Replica &rp : c->reps) most = std::max(most, rp.n_trials);
    if (!c->d_sigma1 && hipMalloc(&c->d_sigma1, (size_t)c->n_total) != hipSuccess) return fail(c, SMC_E_NOMEM, "sigma1");
    if (!c->d_E0 && hipMalloc(&c->d_E0, sizeof(float) * c->n_total) != hipSuccess) return fail(c, SMC_E_NOMEM, "E0");
    if (!c->d_E1 && hipMalloc(&c->d_E1, sizeof(float) * c->n_total) != hipSuccess) return fail(c, SMC_E_NOMEM, "E1");
    if (!c->d_dltrials && hipMalloc(&c->d_dltrials, sizeof(DlTrial) * most) != hipSuccess)
      return fail(c, SMC_E_NOMEM, "trial records");
  }
  c->strategy = strategy;
  return SMC_OK;
}

int smc_get_strategy(const smc_ctx *c, int32_t *strategy) {
  if (!c || !strategy) return SMC_E_INVALID;
  *strategy = c->strategy;
  return SMC_OK;
}

int smc_use_graph(smc_ctx *c, int32_t enable) {
  if (!c) return SMC_E_INVALID;
  c->use_graph = enable != 0;
  if (!c->use_graph) drop_graph(c);
  return SMC_OK;
}

int smc_autotune(smc_ctx *c, const char *cache_path, int32_t *chosen, float *ms_per_variant) {
  if (!c) return SMC_E_INVALID;
  if (!c->mfma && !c->qsro_tiled) {
    if (chosen) *chosen = c->variant;
    return SMC_OK;  // the per-lane path has a single variant
  }
  if (c->strategy != SMC_STRATEGY_ZONE) return fail(c, SMC_E_STATE, "the autotuner tunes the zone strategy's kernel");
  // cache key: device, precision and the replica shapes
  hipDeviceProp_t prop{};
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipGetDeviceProperties(&prop, dev);
  std::string key = std::string(prop.gcnArchName) + "/p" + std::to_string(c->cfg.precision);
  for (size_t r = 0; r < c->reps.size(); ++r)
    key += "/" + std::to_string(c->cells[3 * r]) + "x" + std::to_string(c->cells[3 * r + 1]) + "x" +
           std::to_string(c->cells[3 * r + 2]);
  if (key.size() > 200) key = key.substr(0, 120) + "/n" + std::to_string(c->reps.size()) + "/s" + std::to_string(c->n_total);
  if (cache_path) {
    FILE *f = fopen(cache_path, "r");
    if (f) {
      char line[512];
      while (fgets(line, sizeof line, f)) {
        int v = -1;
        char k[400];
        if (sscanf(line, "{\"key\": \"%399[^\"]\", \"variant\": %d", k, &v) == 2 && key == k && v >= 0 &&
            v < kNumVariants) {
          fclose(f);
          if (chosen) *chosen = v;
          return smc_set_variant(c, v);
        }
      }
      fclose(f);
    }
  }
  // time every variant on the same sweep from the same state; all must agree bit for bit
  const size_t R = c->reps.size(), N = (size_t)c->n_total;
  uint8_t *occ0 = nullptr, *occ1 = nullptr;
  float *ec0 = nullptr;
  unsigned long long *ef0 = nullptr;
  uint64_t *cnt0 = nullptr;
  int rc = SMC_OK;
  if (hipMalloc(&occ0, N) || hipMalloc(&occ1, N) || hipMalloc(&ec0, 4 * N) || hipMalloc(&ef0, 8 * R) ||
      hipMalloc(&cnt0, 32 * R))
    rc = fail(c, SMC_E_NOMEM, "autotune buffers");
  const uint64_t sweep0 = c->sweep;
  const int v0 = c->variant;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!rc && (hipEventCreate(&e0) || hipEventCreate(&e1))) rc = fail(c, SMC_E_DEVICE, "autotune events");
  if (!rc && (hipMemcpyAsync(occ0, c->occ, N, hipMemcpyDeviceToDevice, c->stream) ||
              hipMemcpyAsync(ec0, c->ecache, 4 * N, hipMemcpyDeviceToDevice, c->stream) ||
              hipMemcpyAsync(ef0, c->d_efixed, 8 * R, hipMemcpyDeviceToDevice, c->stream) ||
              hipMemcpyAsync(cnt0, c->d_counters, 32 * R, hipMemcpyDeviceToDevice, c->stream)))
    rc = fail(c, SMC_E_DEVICE, "autotune save");
  int best = v0;
  float best_ms = 1e30f;
  std::vector<uint8_t> ref, got;
  for (int v = 0; v < kNumVariants && !rc; ++v) {
    if ((rc = smc_set_variant(c, v)) || (rc = smc_set_sweep(c, sweep0))) break;
    if (hipMemcpyAsync(c->occ, occ0, N, hipMemcpyDeviceToDevice, c->stream) ||
        hipMemcpyAsync(c->ecache, ec0, 4 * N, hipMemcpyDeviceToDevice, c->stream)) {
      rc = fail(c, SMC_E_DEVICE, "autotune restore");
      break;
    }
    if ((rc = run_sweep(c, nullptr, false))) break;  // warm (graph build); same sweep replayed below
    if ((rc = smc_set_sweep(c, sweep0))) break;
    if (hipMemcpyAsync(c->occ, occ0, N, hipMemcpyDeviceToDevice, c->stream) ||
        hipMemcpyAsync(c->ecache, ec0, 4 * N, hipMemcpyDeviceToDevice, c->stream) ||
        hipEventRecord(e0, c->stream)) {
      rc = fail(c, SMC_E_DEVICE, "autotune restore");
      break;
    }
    if ((rc = run_sweep(c, nullptr, false))) break;
    float ms = 0.0f;
    if (hipEventRecord(e1, c->stream) || hipEventSynchronize(e1) || hipEventElapsedTime(&ms, e0, e1)) {
      rc = fail(c, SMC_E_DEVICE, "autotune timing");
      break;
    }
    if (ms_per_variant) ms_per_variant[v] = ms;
    // bit-exactness gate against the first variant
    got.resize(N);
    if (hipMemcpy(got.data(), c->occ, N, hipMemcpyDeviceToHost)) {
      rc = fail(c, SMC_E_DEVICE, "autotune compare");
      break;
    }
    if (v == 0) ref = got;
    else if (got != ref) {
      rc = fail(c, SMC_E_STATE, "kernel variant " + std::to_string(v) + " is not bit-identical to variant 0");
      break;
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  // restore the caller's state and the chosen variant
  if (occ0 && ec0) {
    (void)hipMemcpyAsync(c->occ, occ0, N, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(c->ecache, ec0, 4 * N, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(c->d_efixed, ef0, 8 * R, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(c->d_counters, cnt0, 32 * R, hipMemcpyDeviceToDevice, c->stream);
  }
  const int rc2 = smc_set_sweep(c, sweep0);
  (void)smc_set_variant(c, rc ? v0 : best);
  (void)hipStreamSynchronize(c->stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (void *p : {(void *)occ0, (void *)occ1, (void *)ec0, (void *)ef0, (void *)cnt0})
    if (p) (void)hipFree(p);
  if (rc) return rc;
  if (rc2) return rc2;
  if (chosen) *chosen = best;
  if (cache_path) {
    FILE *f = fopen(cache_path, "a");
    if (f) {
      fprintf(f, "{\"key\": \"%s\", \"variant\": %d, \"ms\": %.4f}\n", key.c_str(), best, best_ms);
      fclose(f);
    }
  }
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
  drop_graph(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  void *bufs[] = {c->d_reps, c->d_w32, c->d_w64, c->d_w64t, c->d_w32t, c->d_omega, c->d_reg_off, c->d_om_off, c->d_idx,
                  c->d_reg_pos, c->d_queue, c->d_rowe, c->d_qcount, c->d_ebase, c->d_efixed, c->d_escratch,
                  c->d_counters, c->d_site64, c->d_psum, c->packs[0].dev, c->packs[1].dev, c->packs[2].dev,
                  c->packs[3].dev, c->d_seg_rep, c->d_seg_start[0], c->d_seg_start[1], c->d_seg_start[2], c->d_sweep,
                  c->d_sigma1, c->d_E0, c->d_E1, c->d_dltrials};
  for (void *p : bufs)
    if (p) (void)hipFree(p);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  fit_release(c);
  fcc::release(c);
  delete c;
}

}  // extern "C"
