// Barycentric gradients and volume of a simplex (device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mg {

// barycentric gradients g[a][x] and volume of a simplex
__device__ inline double simplex_grads(const double *X, const int32_t *v, int dim, double g[4][3]) {
  if (dim == 2) {
    double x0 = X[2 * v[0]], y0 = X[2 * v[0] + 1];
    double a = X[2 * v[1]] - x0, b = X[2 * v[2]] - x0;
    double c = X[2 * v[1] + 1] - y0, d = X[2 * v[2] + 1] - y0;
    double det = a * d - b * c;  // J = [[a, b], [c, d]] (columns x1-x0, x2-x0)
    double id = 1.0 / det;
    g[1][0] = d * id;
    g[1][1] = -b * id;
    g[2][0] = -c * id;
    g[2][1] = a * id;
    g[0][0] = -g[1][0] - g[2][0];
    g[0][1] = -g[1][1] - g[2][1];
    return fabs(det) * 0.5;
  }
  double J[3][3];
  for (int x = 0; x < 3; ++x)
    for (int k = 0; k < 3; ++k) J[x][k] = X[3 * (int64_t)v[k + 1] + x] - X[3 * (int64_t)v[0] + x];
  double C00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  double C01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  double C02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  double det = J[0][0] * C00 + J[0][1] * C01 + J[0][2] * C02;
  double id = 1.0 / det;
  // rows of J^-1 = grad lam_1..3 ; (J^-1)[k][x] = cof[x][k] / det
  double inv[3][3];
  inv[0][0] = C00 * id;
  inv[1][0] = C01 * id;
  inv[2][0] = C02 * id;
  inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  for (int x = 0; x < 3; ++x) {
    g[1][x] = inv[0][x];
    g[2][x] = inv[1][x];
    g[3][x] = inv[2][x];
    g[0][x] = -inv[0][x] - inv[1][x] - inv[2][x];
  }
  return fabs(det) / 6.0;
}

}  // namespace mg
