// Host-side tables: the affected zone of a swap and the per-replica schedule.
#pragma once
#include <stdint.h>

#include <array>
#include <vector>

#include "lattice.hpp"

namespace smc {

constexpr int kOmegaMax = 40;  // |Omega| with shells 1-3; 22 with shells 1-2

// Affected zone of swapping the site at the origin with its shell-1 neighbour in slot d:
// the origin, the partner, and every site that has either among the neighbours its
// features read (the shell set is symmetric, so these are the neighbours of either).
// Offsets are doubled coordinates, sorted lexicographically, duplicates removed.
struct OmegaTable {
  int count = 0;                                  // 22 or 40
  std::array<std::array<int8_t, 3>, 8 * kOmegaMax> off{};  // [d][k]
};

OmegaTable build_omega(int n_nbr_used);

// Device-side description of one replica.
struct Replica {
  int32_t L[3];         // cubic cells per axis
  AxisCells ax[3];      // link cells per axis
  int32_t n_colours;    // basis * big0 * big1 * big2
  int32_t basis;        // sites per cubic cell: 2 (BCC) or 4 (FCC)
  int64_t site0;        // first site of this replica in the concatenated arrays
  int64_t n_sites;
  int64_t n_trials;     // link cells: the most trials a colour has (colour_trials gives each)
  double temperature;   // kelvin
};

Replica make_replica(const int32_t cells[3], int64_t site0, double temperature, int32_t basis = 2);

// Offsets (ox, oy, oz) of a colour inside its link cell; the basis site is colour % basis.
__host__ __device__ inline void colour_offsets(const Replica &R, int32_t colour, int32_t o[3]) {
  int32_t rest = colour / R.basis;
  o[0] = rest % R.ax[0].big;
  rest /= R.ax[0].big;
  o[1] = rest % R.ax[1].big;
  o[2] = rest / R.ax[1].big;
}

// Trials of a colour: the link cells that hold its offset on every axis.
__host__ __device__ inline int64_t colour_trials(const Replica &R, int32_t colour) {
  int32_t o[3];
  colour_offsets(R, colour, o);
  return (int64_t)axis_cells_holding(R.ax[0], o[0]) * axis_cells_holding(R.ax[1], o[1]) *
         axis_cells_holding(R.ax[2], o[2]);
}

}  // namespace smc
