// Library state behind the opaque smc_ctx handle, shared by the sweep and the fit entry
// points.  Host-only declarations: no kernels live here.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "pack.hpp"
#include "smc.h"
#include "tables.hpp"

namespace smc {

struct RecheckEntry;
struct DlTrial;
namespace fcc {
struct Trial;
struct QEntry;
}

// Buffers of the FCC lattice path.
struct FccState {
  bool on = false;
  int model = 0;                     // 0: MLPNet (shells 1-2), 1: qSRO (shells 1-3)
  int om_n = 0;                      // zone size: 28 or 60
  int8_t *d_om = nullptr;            // [12][60][3] zone offsets per partner slot
  fcc::Trial *d_trials = nullptr;    // [cap]
  int32_t *d_active = nullptr;       // [cap]
  float *d_e1 = nullptr;             // [cap][om_n]
  fcc::QEntry *d_queue = nullptr;    // [cap]
  double *d_rowe = nullptr;          // [cap][56] FP64 zone energies of queued MLPNet trials
  uint64_t *d_dpart = nullptr;       // [2][k_decide blocks] per-block accepted dE and accepts
  uint32_t *d_counts = nullptr;      // [replica colours] active trials, queued trials (one 64-bit word each)
  uint16_t *d_rq_off = nullptr;      // qSRO: [12][304] read-region offsets per partner slot
  uint16_t *d_rq_idx = nullptr;      // qSRO: [12][60][43] region position of each zone row's slots
  uint16_t *d_rq_pos = nullptr;      // qSRO: [12][2] region positions of the trial site and partner
  int64_t cap = 0;                   // largest trial count of a colour
  uint8_t *d_pack[4] = {nullptr, nullptr, nullptr, nullptr};  // FP32, BF16, split BF16, FP8 weight images
  bool pack_ready[4] = {false, false, false, false};
  float b3 = 0.0f;
};

struct DevPack {  // one precision's packed weights on the device
  bool ready = false;
  PackedModel host;
  uint8_t *dev = nullptr;
};

// Buffers of the differentiation entry points (allocated on first use, grown on demand).
struct FitState {
  uint8_t *pack = nullptr;     // BF16 forward images (layer 0, layer 1) + c1 + w2
  uint8_t *bwd = nullptr;      // BF16 images of the backward (layer 0, W1, W1^T in 16x16 tiles)
  float *partial = nullptr;    // [blocks][params] per-block gradient partials
  int partial_blocks = 0;
  double *row_e = nullptr;     // [rows] local energies of the last forward
  int64_t row_cap = 0;
  double *S = nullptr, *gs = nullptr, *loss = nullptr;  // [batch], [batch], [1]
  int32_t batch_cap = 0;
  float *grad = nullptr;       // [params]
  void *ref = nullptr;         // reference-precision scratch (per-row layer values)
  size_t ref_bytes = 0;
  double *ce_table = nullptr;  // CE lookup tables
  size_t ce_bytes = 0;
};

void fit_release(smc_ctx *c);

}  // namespace smc

struct smc_ctx {
  smc_config cfg{};
  std::vector<int32_t> cells;
  std::vector<double> temps;
  std::vector<smc::Replica> reps;
  int64_t n_total = 0;
  int32_t n_in = 0, hidden = 0, n_params = 0;
  bool mfma = false;              // one-hot features with 128 hidden: matrix-core path
  bool qsro_tiled = false;        // BCC qSRO in FP32: the same colour kernel, qSRO evaluation
  int n_cu = 256;
  int device = 0;                 // device current at smc_init
  void *scratch = nullptr;        // device address of the probe's static work space on that device
  hipStream_t stream = nullptr;
  uint8_t *occ = nullptr;
  float *ecache = nullptr;
  std::vector<float> host_params;
  // library-owned device memory
  smc::Replica *d_reps = nullptr;
  float *d_w32 = nullptr;
  double *d_w64 = nullptr;
  double *d_w64t = nullptr;       // FP64 blob with W0, W1 stored [input][unit] (re-decision kernel)
  float *d_w32t = nullptr;        // the same layout in FP32 (staged in LDS by the re-decision kernel)
  int8_t *d_omega = nullptr;      // per-lane path Omega offsets
  int32_t omega_n = 0;
  uint16_t *d_reg_off = nullptr, *d_om_off = nullptr;
  uint8_t *d_idx = nullptr, *d_reg_pos = nullptr;
  smc::DevPack packs[4];
  smc::RecheckEntry *d_queue = nullptr;
  double *d_rowe = nullptr;       // [queue_cap][80] FP64 local energies of queued trials
  uint32_t *d_qcount = nullptr;   // one counter per colour index of a sweep
  int64_t queue_cap = 0;
  int32_t colours_total = 0;
  int32_t max_colours = 0;        // colour indices per sweep (largest replica schedule)
  // per colour index: the replicas that have it and their flattened group offsets, for
  // groups of 32 [0] and 16 [1] link cells
  std::vector<int32_t> seg_off;               // [max_colours + 1] into the segment lists
  std::vector<int32_t> seg_groups[3];         // [max_colours] total groups of 32, 16 and kScalarBlock trials
  std::vector<int64_t> col_trials;            // [max_colours] link cells over all replicas
  int32_t *d_seg_rep = nullptr;               // [segments]
  int32_t *d_seg_start[3] = {nullptr, nullptr, nullptr};  // [segments + max_colours] per group size
  uint64_t *d_sweep = nullptr;                // device sweep counter
  int variant = 0;                            // kernel variant (autotuner)
  bool use_graph = true;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  double *d_ebase = nullptr;      // [R] FP64 total at the last refresh
  unsigned long long *d_efixed = nullptr;  // [R] accepted dE since then, 2^-32 eV units
  double *d_escratch = nullptr;   // [R]
  uint64_t *d_counters = nullptr; // [4][R]
  double *d_site64 = nullptr;     // [N] FP64 site energies (lazy)
  double *d_psum = nullptr;       // [kSumChunks] partial sums of the FP64 totals (lazy)
  uint64_t sweep = 0;
  double guard = 0.0;
  // per-kernel timing: event pairs recorded around launches while profiling is on
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;         // 2 per recorded launch
  std::vector<int> ev_kind;                // 0 colour kernel, 1 re-decision kernel
  size_t ev_used = 0;
  // double-lattice strategy (Algorithm 1 as written)
  int strategy = 0;                  // smc_strategy
  uint8_t *d_sigma1 = nullptr;       // [N] auxiliary lattice
  float *d_E0 = nullptr, *d_E1 = nullptr;  // [N] all-site energies before / after
  smc::DlTrial *d_dltrials = nullptr;      // [largest colour of a replica]
  smc::FitState fit;
  smc::FccState fcc;
  std::string err;
};

namespace smc {

inline int fail(smc_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// Start event of a timed launch (index of the pair), or -1 when not profiling.
inline int prof_begin(smc_ctx *c) {
  if (!c->profiling) return -1;
  const size_t k = c->ev_used;
  if (2 * k + 2 > c->ev_pool.size()) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1;
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return -1;
    }
    c->ev_pool.push_back(e0);
    c->ev_pool.push_back(e1);
    c->ev_kind.push_back(0);
  }
  if (hipEventRecord(c->ev_pool[2 * k], c->stream) != hipSuccess) return -1;
  c->ev_used++;
  return (int)k;
}

inline void prof_end(smc_ctx *c, int k, int kind) {
  if (k < 0) return;
  c->ev_kind[k] = kind;
  (void)hipEventRecord(c->ev_pool[2 * k + 1], c->stream);
}


// Return SMC_E_DEVICE with the failing call and HIP's message.
#define HIPC(c, expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail((c), SMC_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)


}  // namespace smc
