// Host-side packing of the FP32 parameter blob into the LDS images used by the matrix-core
// evaluator, and the read-region tables of the swap kernel.
#pragma once
#include <stdint.h>

#include <vector>

namespace smc {

struct PackedModel {
  std::vector<uint8_t> bytes;  // pack_bytes<P>() bytes: layer 0, layer 1, c0, c1, w2, pad
  float b2 = 0.0f;
  int k_scale_a0 = 127, k_scale_a1 = 127, k_scale_h = 127;  // biased E8M0 exponents (FP8)
  float sh = 1.0f;                                          // FP8 activation scale 2^kh
};

// params: FP32 blob W0[128][108], b0[128], W1[128][128], b1[128], W2[128], b2[1].
PackedModel pack_model(int precision, const float *params);

uint16_t f32_to_bf16_rne(float x);
float bf16_to_f32(uint16_t h);
uint8_t f32_to_e4m3_rne(float x);  // OCP E4M3 (bias 7, max 448, saturating)
float e4m3_to_f32(uint8_t v);

// Sites read by one trial (one-hot features, shells 1-3): the affected zone Omega of the
// swap with partner slot d plus every neighbour of Omega.  Offsets are doubled coordinates
// in [-5, 5] packed as (dx+8) | (dy+8) << 4 | (dz+8) << 8.
constexpr int kRegion = 192;
constexpr int kOmegaOneHot = 40;
constexpr int kSlotsOneHot = 27;
struct RegionTables {
  std::vector<uint16_t> reg_off;  // [8][192]
  std::vector<uint16_t> om_off;   // [8][40]
  std::vector<uint8_t> idx;      // [8][40][28]: region position of slot m of Omega site k
  std::vector<uint8_t> reg_pos;  // [8][2]: region position of the trial site and of the partner
};
RegionTables build_region_tables();

}  // namespace smc
