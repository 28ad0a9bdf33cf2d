// BCC lattice geometry, neighbour shells, link-cell schedule and the Philox4x64-10
// counter-based generator, usable from host and device code.
//
// Geometry: cell (x,y,z) holds basis site b = 0 at doubled coordinates (2x,2y,2z) and
// b = 1 at (2x+1,2y+1,2z+1); positions are periodic modulo 2L per axis; the canonical
// site index is s = ((z*Ly + y)*Lx + x)*2 + b.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc {

// Neighbour slots in doubled coordinates: shell 1 (8 vectors (+-1,+-1,+-1), distance
// a*sqrt(3)/2), shell 2 (6 vectors (+-2,0,0) and permutations, distance a), shell 3
// (12 vectors (+-2,+-2,0) and permutations, distance a*sqrt(2)); each shell in
// lexicographic order of (dx,dy,dz).
constexpr int kNbr = 26;
constexpr int kNbrS12 = 14;
__host__ __device__ constexpr int8_t shell_dx(int k) {
  constexpr int8_t t[kNbr] = {-1, -1, -1, -1, 1, 1, 1, 1, -2, 0, 0, 0, 0, 2,
                              -2, -2, -2, -2, 0, 0, 0, 0, 2, 2, 2, 2};
  return t[k];
}
__host__ __device__ constexpr int8_t shell_dy(int k) {
  constexpr int8_t t[kNbr] = {-1, -1, 1, 1, -1, -1, 1, 1, 0, -2, 0, 0, 2, 0,
                              -2, 0, 0, 2, -2, -2, 2, 2, -2, 0, 0, 2};
  return t[k];
}
__host__ __device__ constexpr int8_t shell_dz(int k) {
  constexpr int8_t t[kNbr] = {-1, 1, -1, 1, -1, 1, -1, 1, 0, 0, -2, 2, 0, 0,
                              0, -2, 2, 0, -2, 2, -2, 2, 0, -2, 2, 0};
  return t[k];
}
__host__ __device__ constexpr int shell_of(int k) { return k < 8 ? 1 : (k < 14 ? 2 : 3); }

// Doubled-coordinate position of a site index (relative to its replica).
struct Pos {
  int32_t x, y, z;
};

__host__ __device__ inline Pos site_pos(int64_t s, int32_t lx, int32_t ly) {
  int32_t b = (int32_t)(s & 1);
  int64_t c = s >> 1;
  int32_t x = (int32_t)(c % lx);
  int64_t r = c / lx;
  int32_t y = (int32_t)(r % ly);
  int32_t z = (int32_t)(r / ly);
  return Pos{2 * x + b, 2 * y + b, 2 * z + b};
}

// Wrap v into [0, m) for |v| < 2m (every offset used here is at most 5 doubled units and
// every axis at least 8).
__host__ __device__ inline int32_t wrap1(int32_t v, int32_t m) {
  v = v < 0 ? v + m : v;
  return v >= m ? v - m : v;
}

__host__ __device__ inline int64_t site_index(Pos p, int32_t lx, int32_t ly) {
  return (((int64_t)(p.z >> 1) * ly + (p.y >> 1)) * lx + (p.x >> 1)) * 2 + (p.x & 1);
}

// 32-bit forms for replica-local indices, which stay below 2^31 (checked when a context is
// made).
__host__ __device__ inline Pos site_pos32(int32_t s, int32_t lx, int32_t ly) {
  const uint32_t u = (uint32_t)s;
  const int32_t b = (int32_t)(u & 1u);
  const uint32_t c = u >> 1;
  const int32_t x = (int32_t)(c % (uint32_t)lx);
  const uint32_t r = c / (uint32_t)lx;
  const int32_t y = (int32_t)(r % (uint32_t)ly);
  const int32_t z = (int32_t)(r / (uint32_t)ly);
  return Pos{2 * x + b, 2 * y + b, 2 * z + b};
}

__host__ __device__ inline int32_t site_at32(Pos p, int dx, int dy, int dz, int32_t lx, int32_t ly, int32_t lz) {
  const int32_t x = wrap1(p.x + dx, 2 * lx), y = wrap1(p.y + dy, 2 * ly), z = wrap1(p.z + dz, 2 * lz);
  return (((z >> 1) * ly + (y >> 1)) * lx + (x >> 1)) * 2 + (x & 1);
}

__host__ __device__ inline int64_t site_at(Pos p, int dx, int dy, int dz, int32_t lx, int32_t ly,
                                           int32_t lz) {
  Pos q{wrap1(p.x + dx, 2 * lx), wrap1(p.y + dy, 2 * ly), wrap1(p.z + dz, 2 * lz)};
  return site_index(q, lx, ly);
}

// Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64x64->128-bit products; the
// high halves are mixed with the other two counter words and the round key, which
// advances by two Weyl increments between rounds.
struct U64x4 {
  uint64_t v[4];
};

__host__ __device__ inline void mulhilo64(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo) {
#if defined(__HIP_DEVICE_COMPILE__)
  hi = __umul64hi(a, b);
  lo = a * b;
#else
  unsigned __int128 p = (unsigned __int128)a * b;
  hi = (uint64_t)(p >> 64);
  lo = (uint64_t)p;
#endif
}

__host__ __device__ inline U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ULL, kMul1 = 0xCA5A826395121157ULL;
  constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ULL, kWeyl1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t h0, l0, h1, l1;
    mulhilo64(kMul0, c0, h0, l0);
    mulhilo64(kMul1, c2, h1, l1);
    uint64_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
    c0 = n0;
    c1 = l1;
    c2 = n2;
    c3 = l0;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
  return U64x4{{c0, c1, c2, c3}};
}

// Boltzmann constant in eV/K.
constexpr double kBoltzmannEvPerK = 8.617333262e-5;

// Link cells along one axis of E cells: q = max(1, E/4) cells whose lengths differ by at
// most one, the first (E mod q) taking the longer length.
struct AxisCells {
  int32_t q, small, big, nbig;
};

__host__ __device__ inline AxisCells axis_cells(int32_t E) {
  AxisCells a;
  a.q = E / 4 < 1 ? 1 : E / 4;
  a.small = E / a.q;
  a.nbig = E % a.q;
  a.big = a.small + (a.nbig ? 1 : 0);
  return a;
}

// Start of link cell i along the axis.
__host__ __device__ inline int32_t axis_start(const AxisCells &a, int32_t i) {
  return i < a.nbig ? i * a.big : a.nbig * a.big + (i - a.nbig) * a.small;
}

__host__ __device__ inline int32_t axis_len(const AxisCells &a, int32_t i) {
  return i < a.nbig ? a.big : a.small;
}

// Link cells along an axis long enough to hold offset o: all of them when o fits a short
// cell, else only the long cells, which come first.
__host__ __device__ inline int32_t axis_cells_holding(const AxisCells &a, int32_t o) {
  return o < a.small ? a.q : a.nbig;
}

}  // namespace smc
