// Host-side tables: affected zone templates and replica schedule descriptors.
#include "tables.hpp"

#include <algorithm>

namespace smc {

OmegaTable build_omega(int n_nbr_used) {
  OmegaTable t;
  for (int d = 0; d < 8; ++d) {
    std::vector<std::array<int8_t, 3>> v;
    const int8_t px = shell_dx(d), py = shell_dy(d), pz = shell_dz(d);
    v.push_back({0, 0, 0});
    v.push_back({px, py, pz});
    for (int k = 0; k < n_nbr_used; ++k) {
      v.push_back({shell_dx(k), shell_dy(k), shell_dz(k)});
      v.push_back({(int8_t)(px + shell_dx(k)), (int8_t)(py + shell_dy(k)), (int8_t)(pz + shell_dz(k))});
    }
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    t.count = (int)v.size();
    for (int k = 0; k < t.count && k < kOmegaMax; ++k) t.off[d * kOmegaMax + k] = v[k];
  }
  return t;
}

Replica make_replica(const int32_t cells[3], int64_t site0, double temperature, int32_t basis) {
  Replica r{};
  int32_t colours = basis;
  int64_t trials = 1;
  for (int a = 0; a < 3; ++a) {
    r.L[a] = cells[a];
    r.ax[a] = axis_cells(cells[a]);
    colours *= r.ax[a].big;
    trials *= r.ax[a].q;
  }
  r.n_colours = colours;
  r.site0 = site0;
  r.basis = basis;
  r.n_sites = (int64_t)basis * cells[0] * cells[1] * cells[2];
  r.n_trials = trials;
  r.temperature = temperature;
  return r;
}

}  // namespace smc
