// Test driver: runs the solvers' host-side flat-direction and gauge-projection
// routines on problems read from stdin, for comparison with the oracle.
//   F L n_mod  ranks[L]  traces[L]  (K axes[K]) x n_mod   -> d, then d rows of L
//   Q q L  flats[q][L]  eps[L]  mins[L]  t_star[q]        -> q values
#include <cstdio>
#include <vector>

#include "solve_host.h"

using gmgm_sv::Axis;

int main() {
  char op;
  while (std::scanf(" %c", &op) == 1) {
    if (op == 'F') {
      int L, nm;
      if (std::scanf("%d %d", &L, &nm) != 2) return 1;
      std::vector<Axis> ax(L);
      for (auto& a : ax)
        if (std::scanf("%d", &a.r) != 1) return 1;
      for (auto& a : ax)
        if (std::scanf("%lf", &a.trace) != 1) return 1;
      std::vector<std::vector<int>> mods(nm);
      for (auto& m : mods) {
        int K;
        if (std::scanf("%d", &K) != 1) return 1;
        m.resize(K);
        for (auto& x : m)
          if (std::scanf("%d", &x) != 1) return 1;
      }
      const auto F = gmgm_sv::flat_directions(ax, mods);
      std::printf("%d\n", (int)F.size());
      for (auto& v : F) {
        for (double x : v) std::printf("%.17g ", x);
        std::printf("\n");
      }
    } else if (op == 'Q') {
      int q, L;
      if (std::scanf("%d %d", &q, &L) != 2) return 1;
      std::vector<std::vector<double>> flats(q, std::vector<double>(L));
      for (auto& f : flats)
        for (auto& x : f)
          if (std::scanf("%lf", &x) != 1) return 1;
      std::vector<Axis> ax(L);
      std::vector<double> mins(L), ts(q);
      for (auto& a : ax)
        if (std::scanf("%lf", &a.eps) != 1) return 1;
      for (auto& x : mins)
        if (std::scanf("%lf", &x) != 1) return 1;
      for (auto& x : ts)
        if (std::scanf("%lf", &x) != 1) return 1;
      const auto t = gmgm_sv::nearest_feasible_shift(ts, flats, ax, mins.data());
      for (double x : t) std::printf("%.17g ", x);
      std::printf("\n");
    } else {
      return 1;
    }
    std::fflush(stdout);
  }
  return 0;
}
