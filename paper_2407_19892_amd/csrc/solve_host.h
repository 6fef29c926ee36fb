// Host-side pieces of the eigenvalue solvers that involve no device work: the
// per-axis record, the flat shift directions of the NLL and the gauge
// projection inside the box.  Plain C++ (no HIP), so that they can be built and
// checked on a CPU alone.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <vector>

namespace gmgm_sv {

struct Axis {
  int r = 0;
  size_t off = 0;   // offset in the concatenated coordinate vectors
  double eps = 0;
  double trace = 0;
};

// Axis shifts c along which the NLL is constant: every modality's tuple sums
// unchanged (the sum of c over the modality's axes is zero: the null space of
// the modality-axis incidence matrix, Identifiability appendix) and the linear
// term unchanged (slope 1/2 sum_l c_l tr_l = 0).  A null-space basis comes from
// the reduced row echelon form; if some basis vector has a slope (beyond 1e-12
// of sum_l |c_l| tr_l), the one with the largest relative slope cancels the
// slopes of the others and is dropped.  Returned orthonormal in the metric
// sum_l r_l c_l c'_l.
inline std::vector<std::vector<double>> flat_directions(const std::vector<Axis>& ax,
                                                        const std::vector<std::vector<int>>& mods) {
  const int L = (int)ax.size();
  std::vector<std::vector<double>> M(mods.size(), std::vector<double>(L, 0.0));
  for (size_t t = 0; t < mods.size(); ++t)
    for (int a : mods[t]) M[t][a] = 1.0;
  std::vector<int> pivcol;
  int row = 0;
  for (int c = 0; c < L && row < (int)M.size(); ++c) {
    int p = -1;
    for (int r2 = row; r2 < (int)M.size(); ++r2)
      if (std::fabs(M[r2][c]) > 1e-12) {
        p = r2;
        break;
      }
    if (p < 0) continue;
    std::swap(M[row], M[p]);
    const double dv = M[row][c];
    for (auto& v : M[row]) v /= dv;
    for (int r2 = 0; r2 < (int)M.size(); ++r2)
      if (r2 != row && M[r2][c] != 0.0) {
        const double f = M[r2][c];
        for (int c2 = 0; c2 < L; ++c2) M[r2][c2] -= f * M[row][c2];
      }
    pivcol.push_back(c);
    row++;
  }
  std::vector<std::vector<double>> basis;
  std::vector<double> slope, scale;
  for (int c = 0; c < L; ++c) {
    if (std::find(pivcol.begin(), pivcol.end(), c) != pivcol.end()) continue;
    std::vector<double> v(L, 0.0);
    v[c] = 1.0;
    for (size_t r2 = 0; r2 < pivcol.size(); ++r2) v[pivcol[r2]] = -M[r2][c];
    double sl = 0, sc = 0;
    for (int l = 0; l < L; ++l) {
      sl += v[l] * ax[l].trace;
      sc += std::fabs(v[l]) * ax[l].trace;
    }
    basis.push_back(v);
    slope.push_back(sl);
    scale.push_back(sc);
  }
  int pick = -1;
  double best = 0;
  for (size_t q = 0; q < basis.size(); ++q)
    if (std::fabs(slope[q]) > 1e-12 * scale[q] && std::fabs(slope[q]) / scale[q] > best) {
      best = std::fabs(slope[q]) / scale[q];
      pick = (int)q;
    }
  std::vector<std::vector<double>> zero_slope;
  for (size_t q = 0; q < basis.size(); ++q) {
    if ((int)q == pick) continue;
    std::vector<double> v = basis[q];
    if (pick >= 0) {
      const double f = slope[q] / slope[pick];
      for (int l = 0; l < L; ++l) v[l] -= f * basis[pick][l];
    }
    zero_slope.push_back(v);
  }
  std::vector<std::vector<double>> flats;
  for (auto v : zero_slope) {
    for (auto& q : flats) {
      double pr = 0;
      for (int l = 0; l < L; ++l) pr += ax[l].r * v[l] * q[l];
      for (int l = 0; l < L; ++l) v[l] -= pr * q[l];
    }
    double nrm = 0;
    for (int l = 0; l < L; ++l) nrm += ax[l].r * v[l] * v[l];
    nrm = std::sqrt(nrm);
    if (nrm > 1e-12) {
      for (auto& e : v) e /= nrm;
      flats.push_back(v);
    }
  }
  return flats;
}

// The gauge rule inside the box.  A move by sum_q t_q c_q along the flat
// directions (orthonormal in the gauge metric) changes the q-th gauge value by
// t_q and leaves every tuple sum, hence the NLL and its gradient, unchanged; it
// keeps axis l in the box while mins[l] + u_l >= eps_l, u_l = sum_q t_q c_q,l.
// Returns the t nearest to t_star under these constraints by the primal
// active-set method for strictly convex quadratic programs (Nocedal and Wright,
// Numerical Optimization, Algorithm 16.3), started at the feasible t = 0 with
// no working constraints.  Every iterate is feasible.
inline std::vector<double> nearest_feasible_shift(const std::vector<double>& t_star,
                                           const std::vector<std::vector<double>>& flats,
                                           const std::vector<Axis>& ax, const double* mins) {
  const int q = (int)flats.size(), L = (int)ax.size();
  std::vector<double> b(L), t(q, 0.0);
  for (int l = 0; l < L; ++l) b[l] = ax[l].eps - mins[l];
  double tnorm = 0;
  for (double x : t_star) tnorm += x * x;
  tnorm = std::sqrt(tnorm);
  auto normal_dot = [&](int l, const std::vector<double>& v) {
    double s = 0;
    for (int p = 0; p < q; ++p) s += flats[p][l] * v[p];
    return s;
  };
  std::vector<int> W;
  std::vector<char> in_w(L, 0);
  for (int it = 0; it < 10000; ++it) {
    std::vector<double> step(q);
    double gn = 0;
    for (int p = 0; p < q; ++p) {
      step[p] = t_star[p] - t[p];
      gn += step[p] * step[p];
    }
    const double tol = 1e-12 * (std::sqrt(gn) + tnorm + 1e-300);
    const int k = (int)W.size();
    std::vector<double> mu(k);
    if (k > 0) {
      // least-squares fit of the step by the working normals: (N^T N) mu = N^T step
      std::vector<double> G(k * k);
      for (int i = 0; i < k; ++i) {
        for (int j = 0; j <= i; ++j) {
          double v = 0;
          for (int p = 0; p < q; ++p) v += flats[p][W[i]] * flats[p][W[j]];
          G[i * k + j] = v;
        }
        mu[i] = normal_dot(W[i], step);
      }
      for (int j = 0; j < k; ++j) {   // Cholesky, lower triangle
        double d = G[j * k + j];
        for (int p = 0; p < j; ++p) d -= G[j * k + p] * G[j * k + p];
        if (!(d > 0)) return t;        // dependent normals: cannot happen (a blocking normal is independent)
        G[j * k + j] = std::sqrt(d);
        for (int i = j + 1; i < k; ++i) {
          double v = G[i * k + j];
          for (int p = 0; p < j; ++p) v -= G[i * k + p] * G[j * k + p];
          G[i * k + j] = v / G[j * k + j];
        }
      }
      for (int i = 0; i < k; ++i) {
        for (int p = 0; p < i; ++p) mu[i] -= G[i * k + p] * mu[p];
        mu[i] /= G[i * k + i];
      }
      for (int i = k - 1; i >= 0; --i) {
        for (int p = i + 1; p < k; ++p) mu[i] -= G[p * k + i] * mu[p];
        mu[i] /= G[i * k + i];
      }
      if (k == q)   // q independent normals span the space: the step is zero
        std::fill(step.begin(), step.end(), 0.0);
      else
        for (int p = 0; p < q; ++p)
          for (int i = 0; i < k; ++i) step[p] -= flats[p][W[i]] * mu[i];
    }
    double pn = 0;
    for (double x : step) pn += x * x;
    if (std::sqrt(pn) <= tol) {
      // at the minimiser of the working set: the objective's gradient is -N mu, so
      // a constraint with mu > 0 has a negative multiplier and leaves (compared
      // by mu times the normal's length)
      int drop = -1;
      double worst = tol;
      for (int i = 0; i < k; ++i) {
        double len = 0;
        for (int p = 0; p < q; ++p) len += flats[p][W[i]] * flats[p][W[i]];
        const double size = mu[i] * std::sqrt(len);
        if (size > worst) {
          worst = size;
          drop = i;
        }
      }
      if (drop < 0) return t;
      in_w[W[drop]] = 0;
      W.erase(W.begin() + drop);
      continue;
    }
    double alpha = 1.0;
    int block = -1;
    for (int l = 0; l < L; ++l) {
      if (in_w[l]) continue;
      const double rate = normal_dot(l, step);
      if (rate < 0.0) {
        const double a_l = std::max(0.0, normal_dot(l, t) - b[l]) / -rate;
        if (a_l < alpha) {
          alpha = a_l;
          block = l;
        }
      }
    }
    for (int p = 0; p < q; ++p) t[p] += alpha * step[p];
    if (block >= 0) {
      W.push_back(block);
      in_w[block] = 1;
    }
  }
  return t;
}

}  // namespace gmgm_sv
