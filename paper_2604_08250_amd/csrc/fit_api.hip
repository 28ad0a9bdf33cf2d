// C ABI of the differentiation pattern (declared in include/smc.h): snapshot energies,
// their parameter gradient, one fused fit step with Adam, and cluster-expansion labels.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <array>
#include <set>
#include <string>
#include <vector>

#include "context.hpp"
#include "fit.hpp"
#include "smc.h"

using namespace smc;

namespace {

constexpr int32_t kRefChunk = 16384;  // rows per chunk of the reference-precision path

template <typename P>
int grow(smc_ctx *c, P *&p, size_t &cap_bytes, size_t need_bytes) {
  if (need_bytes <= cap_bytes && p) return SMC_OK;
  if (p) {
    HIPC(c, hipStreamSynchronize(c->stream));
    (void)hipFree(p);
    p = nullptr;
    cap_bytes = 0;
  }
  if (hipMalloc(&p, need_bytes) != hipSuccess) {
    p = nullptr;
    return fail(c, SMC_E_NOMEM, "fit buffer of " + std::to_string(need_bytes) + " bytes");
  }
  cap_bytes = need_bytes;
  return SMC_OK;
}

int fit_check(smc_ctx *c, const void *snap, int32_t batch, int32_t L, const void *params) {
  if (!c) return SMC_E_INVALID;
  if (!snap || !params) return fail(c, SMC_E_INVALID, "null snapshot or parameter pointer");
  if (batch < 1 || L < 4 || L > 1024) return fail(c, SMC_E_INVALID, "batch >= 1 and 4 <= cells_per_axis <= 1024");
  if (c->cfg.feature != SMC_FEAT_ONEHOT_S123 || c->hidden != 128)
    return fail(c, SMC_E_UNSUPPORTED, "fit path needs one-hot features and 128 hidden units");
  const int p = c->cfg.precision;
  if (p != SMC_FP32 && p != SMC_FP64 && p != SMC_BF16)
    return fail(c, SMC_E_UNSUPPORTED, "fit path runs in FP32, FP64 (reference) or BF16 (matrix cores)");
  return SMC_OK;
}

// Small per-call buffers: S, gs, loss [batch], row energies [rows], gradient [params].
int fit_buffers(smc_ctx *c, int32_t batch, int64_t rows) {
  FitState &f = c->fit;
  if (batch > f.batch_cap) {
    for (double **p : {&f.S, &f.gs}) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
    if (hipMalloc(&f.S, sizeof(double) * batch) != hipSuccess || hipMalloc(&f.gs, sizeof(double) * batch) != hipSuccess)
      return fail(c, SMC_E_NOMEM, "fit batch buffers");
    f.batch_cap = batch;
  }
  if (!f.loss && hipMalloc(&f.loss, sizeof(double)) != hipSuccess) return fail(c, SMC_E_NOMEM, "fit loss");
  if (!f.grad && hipMalloc(&f.grad, sizeof(float) * kFitParams) != hipSuccess) return fail(c, SMC_E_NOMEM, "fit grad");
  if (rows > f.row_cap) {
    if (f.row_e) {
      HIPC(c, hipStreamSynchronize(c->stream));
      (void)hipFree(f.row_e);
    }
    f.row_e = nullptr;
    f.row_cap = 0;
    if (hipMalloc(&f.row_e, sizeof(double) * rows) != hipSuccess) return fail(c, SMC_E_NOMEM, "fit row energies");
    f.row_cap = rows;
  }
  return SMC_OK;
}

int fit_pack(smc_ctx *c, const float *params) {
  FitState &f = c->fit;
  if (!f.pack && hipMalloc(&f.pack, kFitPack) != hipSuccess) return fail(c, SMC_E_NOMEM, "fit pack");
  if (!f.bwd && hipMalloc(&f.bwd, kBwdPack) != hipSuccess) return fail(c, SMC_E_NOMEM, "fit backward pack");
  hipLaunchKernelGGL(k_fit_pack_bf16, dim3(grid_for(kFitPackThreads, 256)), dim3(256), 0, c->stream, params, f.pack,
                     f.bwd);
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

// Reference path: scratch [sp | W(T) | Z1 | Z2 | G1 | G2 | acc(double)] for one chunk.
template <typename T>
struct RefLayout {
  uint8_t *sp;
  T *W, *Z1, *Z2, *G1, *G2;
  double *acc;
  static size_t bytes() {
    const size_t rc = kRefChunk;
    return 256 * ((rc * 27 + 255) / 256) + sizeof(T) * (kFitParams + 64) + 4 * sizeof(T) * rc * kHid +
           sizeof(double) * kFitParams + 1024;
  }
  explicit RefLayout(void *base) {
    uint8_t *p = (uint8_t *)base;
    sp = p;
    p += 256 * (((size_t)kRefChunk * 27 + 255) / 256);
    W = (T *)p;
    p += sizeof(T) * (kFitParams + 64);
    Z1 = (T *)p;
    Z2 = Z1 + (size_t)kRefChunk * kHid;
    G1 = Z2 + (size_t)kRefChunk * kHid;
    G2 = G1 + (size_t)kRefChunk * kHid;
    acc = (double *)(G2 + (size_t)kRefChunk * kHid);
  }
};

template <typename T>
int ref_forward_backward(smc_ctx *c, const uint8_t *snap, int32_t batch, int32_t L, const float *params,
                         const double *gE, float *grad_out) {
  int rc_ = grow(c, c->fit.ref, c->fit.ref_bytes, RefLayout<T>::bytes());
  if (rc_) return rc_;
  RefLayout<T> R(c->fit.ref);
  const int64_t N = 2LL * L * L * L, rows = N * batch;
  hipLaunchKernelGGL((k_fit_convert<T>), dim3(grid_for(kFitParams, 256)), dim3(256), 0, c->stream, params, R.W,
                     kFitParams);
  if (gE) hipLaunchKernelGGL(k_fit_zero_f64, dim3(grid_for(kFitParams, 256)), dim3(256), 0, c->stream, R.acc, kFitParams);
  for (int64_t r0 = 0; r0 < rows; r0 += kRefChunk) {
    FitRefArgs a{};
    a.snap = snap;
    a.L = L;
    a.n_sites = N;
    a.r0 = r0;
    a.rc = (int32_t)std::min<int64_t>(kRefChunk, rows - r0);
    a.gE = gE;
    a.sp = R.sp;
    const int64_t nu = (int64_t)a.rc * kHid;
    hipLaunchKernelGGL(k_ref_species, dim3(grid_for((int64_t)a.rc * 27, 256)), dim3(256), 0, c->stream, a);
    hipLaunchKernelGGL((k_ref_l0<T>), dim3(grid_for(nu, 256)), dim3(256), 0, c->stream, a, (const T *)R.W, R.Z1);
    hipLaunchKernelGGL((k_ref_l1<T>), dim3(grid_for(nu, 256)), dim3(256), 0, c->stream, a, (const T *)R.W,
                       (const T *)R.Z1, R.Z2);
    if (!gE) {
      hipLaunchKernelGGL((k_ref_out<T>), dim3(grid_for(a.rc, 256)), dim3(256), 0, c->stream, a, (const T *)R.W,
                         (const T *)R.Z2, c->fit.row_e);
    } else {
      hipLaunchKernelGGL((k_ref_g2<T>), dim3(grid_for(nu, 256)), dim3(256), 0, c->stream, a, (const T *)R.W,
                         (const T *)R.Z2, R.G2);
      hipLaunchKernelGGL((k_ref_g1<T>), dim3(grid_for(nu, 256)), dim3(256), 0, c->stream, a, (const T *)R.W,
                         (const T *)R.Z1, (const T *)R.G2, R.G1);
      hipLaunchKernelGGL((k_ref_wgrad<T>), dim3(grid_for(kFitParams, 128)), dim3(128), 0, c->stream, a,
                         (const T *)R.Z1, (const T *)R.Z2, (const T *)R.G1, (const T *)R.G2, R.acc);
    }
    HIPC(c, hipGetLastError());
  }
  if (gE) hipLaunchKernelGGL(k_fit_to_f32, dim3(grid_for(kFitParams, 256)), dim3(256), 0, c->stream, R.acc, grad_out,
                             kFitParams);
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

// S_out[b] = model energy of snapshot b (packs the BF16 images first on the BF16 path).
int fit_forward(smc_ctx *c, const uint8_t *snap, int32_t batch, int32_t L, const float *params, double *S_out) {
  const int64_t N = 2LL * L * L * L, rows = N * batch;
  int rc = fit_buffers(c, batch, rows);
  if (rc) return rc;
  if (c->cfg.precision == SMC_BF16) {
    if ((rc = fit_pack(c, params))) return rc;
    FitArgs a{};
    a.snap = snap;
    a.L = L;
    a.n_sites = N;
    a.n_rows = rows;
    a.pack = c->fit.pack;
    a.bwd = c->fit.bwd;
    a.b2 = params + kOffB2;
    a.row_e = c->fit.row_e;
    const int64_t tiles = (rows + 31) / 32;
    const int grid = (int)std::min<int64_t>(2 * c->n_cu, (tiles + 7) / 8);
    hipLaunchKernelGGL(k_fit_fwd_bf16, dim3(grid), dim3(kFitFwdThreads), 0, c->stream, a);
  } else if (c->cfg.precision == SMC_FP32) {
    if ((rc = ref_forward_backward<float>(c, snap, batch, L, params, nullptr, nullptr))) return rc;
  } else {
    if ((rc = ref_forward_backward<double>(c, snap, batch, L, params, nullptr, nullptr))) return rc;
  }
  hipLaunchKernelGGL(k_fit_snap_sum, dim3(batch), dim3(256), 0, c->stream, (const double *)c->fit.row_e, N, S_out);
  HIPC(c, hipGetLastError());
  return SMC_OK;
}

// BF16 backward pass: the gradient and energy sum of every segment of every snapshot with a
// unit upstream gradient (f.partial, f.row_e).  Segments split a snapshot's chunks only when
// there are fewer snapshots than CUs.  The images must be packed from params already.
int fit_segments(smc_ctx *c, const uint8_t *snap, int32_t batch, int32_t L, const float *params, int32_t *nps_out,
                 int32_t *n_seg_out) {
  FitState &f = c->fit;
  const int64_t N = 2LL * L * L * L;
  const int chunks = (int)((N + kFitRows - 1) / kFitRows);
  int want = std::min(chunks, std::max(1, (c->n_cu + batch - 1) / batch));
  const int cps = (chunks + want - 1) / want, nps = (chunks + cps - 1) / cps;
  const int64_t n_seg = (int64_t)batch * nps;
  if (n_seg > INT32_MAX) return fail(c, SMC_E_INVALID, "too many snapshot segments");
  const int grid = (int)std::min<int64_t>(c->n_cu, n_seg);
  size_t cap = (size_t)f.partial_blocks * kFitParams * sizeof(float);
  int rc = grow(c, f.partial, cap, (size_t)n_seg * kFitParams * sizeof(float));
  if (rc) return rc;
  f.partial_blocks = (int)(cap / (kFitParams * sizeof(float)));
  FitArgs a{};
  a.snap = snap;
  a.L = L;
  a.n_sites = N;
  a.n_rows = N * batch;
  a.pack = f.pack;
  a.bwd = f.bwd;
  a.b2 = params + kOffB2;
  a.partial = f.partial;
  a.row_e = f.row_e;  // rows >= segments
  a.n_seg = (int32_t)n_seg;
  a.nps = nps;
  a.cps = cps;
  a.chunks_snap = chunks;
  hipLaunchKernelGGL(k_fit_bwd_bf16, dim3(grid), dim3(kFitThreads), 0, c->stream, a);
  HIPC(c, hipGetLastError());
  *nps_out = nps;
  *n_seg_out = (int32_t)n_seg;
  return SMC_OK;
}

// grad_out = sum over segments of ge[snapshot] * segment gradient, in segment order.
void fit_combine(smc_ctx *c, int32_t nps, int32_t n_seg, const double *ge, float *grad_out) {
  hipLaunchKernelGGL(k_fit_combine, dim3((kFitParams + 63) / 64), dim3(512), 0, c->stream, (const float *)c->fit.partial,
                     n_seg, nps, ge, grad_out);
}

// grad_out = sum_b gE[b] dS_b/dparams.  On the BF16 path the images must be packed from
// params already (fit_forward or fit_pack).
int fit_backward(smc_ctx *c, const uint8_t *snap, int32_t batch, int32_t L, const float *params, const double *gE,
                 float *grad_out) {
  if (c->cfg.precision == SMC_BF16) {
    int32_t nps = 0, n_seg = 0;
    int rc = fit_segments(c, snap, batch, L, params, &nps, &n_seg);
    if (rc) return rc;
    fit_combine(c, nps, n_seg, gE, grad_out);
    HIPC(c, hipGetLastError());
    return SMC_OK;
  }
  if (c->cfg.precision == SMC_FP32) return ref_forward_backward<float>(c, snap, batch, L, params, gE, grad_out);
  return ref_forward_backward<double>(c, snap, batch, L, params, gE, grad_out);
}

// The library's own list of triangle shapes: point sets {0, a, b} with a, b and a - b
// among the 26 shell-1..3 vectors, translated so that the lexicographically smallest point
// is the origin; stored as (a, b) with a < b, sorted lexicographically.
std::vector<std::array<int, 6>> ce_triangles() {
  std::vector<std::array<int, 3>> nb;
  for (int k = 0; k < kNbr; ++k) nb.push_back({shell_dx(k), shell_dy(k), shell_dz(k)});
  auto is_nb = [&](const std::array<int, 3> &v) { return std::find(nb.begin(), nb.end(), v) != nb.end(); };
  std::set<std::array<int, 6>> shapes;
  for (const auto &a : nb)
    for (const auto &b : nb) {
      if (a == b || !is_nb({a[0] - b[0], a[1] - b[1], a[2] - b[2]})) continue;
      std::array<std::array<int, 3>, 3> pts = {std::array<int, 3>{0, 0, 0}, a, b};
      std::sort(pts.begin(), pts.end());
      shapes.insert({pts[1][0] - pts[0][0], pts[1][1] - pts[0][1], pts[1][2] - pts[0][2], pts[2][0] - pts[0][0],
                     pts[2][1] - pts[0][1], pts[2][2] - pts[0][2]});
    }
  return std::vector<std::array<int, 6>>(shapes.begin(), shapes.end());
}

}  // namespace

namespace smc {

void fit_release(smc_ctx *c) {
  FitState &f = c->fit;
  void *bufs[] = {f.pack, f.bwd, f.partial, f.row_e, f.S, f.gs, f.loss, f.grad, f.ref, f.ce_table};
  for (void *p : bufs)
    if (p) (void)hipFree(p);
  f = FitState{};
}

}  // namespace smc

extern "C" {

int smc_energy_fwd(smc_ctx *c, const uint8_t *snap, int32_t batch, int32_t L, const float *params, double *e_out) {
  int rc = fit_check(c, snap, batch, L, params);
  if (rc) return rc;
  if (!e_out) return fail(c, SMC_E_INVALID, "null output");
  return fit_forward(c, snap, batch, L, params, e_out);
}

int smc_energy_bwd(smc_ctx *c, const uint8_t *snap, int32_t batch, int32_t L, const float *params,
                   const double *grad_e, float *grad_params) {
  int rc = fit_check(c, snap, batch, L, params);
  if (rc) return rc;
  if (!grad_e || !grad_params) return fail(c, SMC_E_INVALID, "null gradient pointer");
  if ((rc = fit_buffers(c, batch, 2LL * L * L * L * batch))) return rc;
  if (c->cfg.precision == SMC_BF16 && (rc = fit_pack(c, params))) return rc;
  return fit_backward(c, snap, batch, L, params, grad_e, grad_params);
}

int smc_fit_step(smc_ctx *c, const uint8_t *snap, int32_t batch, int32_t L, const double *labels, float *params,
                 float *adam_m, float *adam_v, float lr, int32_t step, double *loss_host) {
  int rc = fit_check(c, snap, batch, L, params);
  if (rc) return rc;
  if (!labels || !adam_m || !adam_v) return fail(c, SMC_E_INVALID, "null label or Adam state pointer");
  if (step < 1 || !(lr > 0.0f)) return fail(c, SMC_E_INVALID, "step >= 1 and lr > 0");
  FitState &f = c->fit;
  if ((rc = fit_buffers(c, batch, 2LL * L * L * L * batch))) return rc;
  const double N = 2.0 * L * L * L;
  if (c->cfg.precision == SMC_BF16) {
    // one pass: segment energy sums and unit-gradient segment gradients, then the loss
    // gradient per snapshot weights the segments
    int32_t nps = 0, n_seg = 0;
    if ((rc = fit_pack(c, params)) || (rc = fit_segments(c, snap, batch, L, params, &nps, &n_seg))) return rc;
    hipLaunchKernelGGL(k_fit_loss, dim3(1), dim3(256), 0, c->stream, (const double *)f.row_e, nps, labels, batch, N,
                       f.gs, f.loss);
    fit_combine(c, nps, n_seg, f.gs, f.grad);
  } else {
    if ((rc = fit_forward(c, snap, batch, L, params, f.S))) return rc;
    hipLaunchKernelGGL(k_fit_loss, dim3(1), dim3(256), 0, c->stream, (const double *)f.S, 1, labels, batch, N, f.gs,
                       f.loss);
    if ((rc = fit_backward(c, snap, batch, L, params, f.gs, f.grad))) return rc;
  }
  const double beta1 = 0.9, beta2 = 0.999;
  const float bc1 = (float)(1.0 - pow(beta1, step)), bc2s = (float)sqrt(1.0 - pow(beta2, step));
  hipLaunchKernelGGL(k_adam, dim3(grid_for(kFitParams, 256)), dim3(256), 0, c->stream, params, adam_m, adam_v,
                     (const float *)f.grad, kFitParams, lr, (float)beta1, (float)beta2, 1e-8f, bc1, bc2s);
  HIPC(c, hipGetLastError());
  if (loss_host) {
    HIPC(c, hipMemcpyAsync(loss_host, f.loss, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPC(c, hipStreamSynchronize(c->stream));
  }
  return SMC_OK;
}

int smc_ce_triangles(int32_t *out_host, int32_t max, int32_t *count) {
  const auto t = ce_triangles();
  if (count) *count = (int32_t)t.size();
  if (out_host)
    for (int32_t i = 0; i < max && i < (int32_t)t.size(); ++i)
      for (int q = 0; q < 6; ++q) out_host[6 * i + q] = t[i][q];
  return SMC_OK;
}

int smc_ce_energy(smc_ctx *c, const smc_ce *ce, const uint8_t *snap, int32_t batch, int32_t L, double *e_out) {
  if (!c) return SMC_E_INVALID;
  if (!ce || !snap || !e_out || !ce->pair || (ce->n_items > 0 && (!ce->triangle || !ce->species || !ce->J)))
    return fail(c, SMC_E_INVALID, "null CE or buffer pointer");
  if (batch < 1 || L < 4 || L > 1024) return fail(c, SMC_E_INVALID, "batch >= 1 and 4 <= cells_per_axis <= 1024");
  const int S = ce->n_species;
  if (S < 2 || S > 5) return fail(c, SMC_E_INVALID, "CE species count must be 2..5");
  const auto tri = ce_triangles();
  const int nt = (int)tri.size();
  std::vector<double> tab(3 * S * S + (size_t)nt * S * S * S, 0.0);
  for (int q = 0; q < 3 * S * S; ++q) tab[q] = ce->pair[q];
  for (int32_t it = 0; it < ce->n_items; ++it) {
    const int t = ce->triangle[it];
    const uint8_t *sp = ce->species + 3 * it;
    if (t < 0 || t >= nt || sp[0] >= S || sp[1] >= S || sp[2] >= S)
      return fail(c, SMC_E_INVALID, "CE item " + std::to_string(it) + " out of range");
    tab[3 * S * S + ((t * S + sp[0]) * S + sp[1]) * S + sp[2]] += ce->J[it];
  }
  std::vector<int8_t> off(6 * nt);
  for (int t = 0; t < nt; ++t)
    for (int q = 0; q < 6; ++q) off[6 * t + q] = (int8_t)tri[t][q];
  const size_t tab_bytes = sizeof(double) * tab.size();
  int rc = grow(c, c->fit.ce_table, c->fit.ce_bytes, tab_bytes + off.size() + 64);
  if (rc) return rc;
  int8_t *d_off = (int8_t *)((uint8_t *)c->fit.ce_table + tab_bytes);
  HIPC(c, hipMemcpyAsync(c->fit.ce_table, tab.data(), tab_bytes, hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(d_off, off.data(), off.size(), hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_ce_energy, dim3(batch), dim3(256), tab_bytes, c->stream, snap, L, 2LL * L * L * L, S, nt,
                     (const double *)c->fit.ce_table, (const int8_t *)d_off, e_out);
  HIPC(c, hipGetLastError());
  // the host tables above must outlive the asynchronous copies
  HIPC(c, hipStreamSynchronize(c->stream));
  return SMC_OK;
}

}  // extern "C"
