// Lagrange bases of degree 1-3 on simplices, written in barycentric coordinates
// lam[0..d].  Local DOF order: vertices 0..d; then the local edges
// (0,1),(0,2),(1,2) [2D] or (0,1),(0,2),(0,3),(1,2),(1,3),(2,3) [3D] with one
// DOF each (P2) or two (P3: the node nearer the first vertex, then the node
// nearer the second); then the interior node of a P3 triangle.
#pragma once

#include <hip/hip_runtime.h>

namespace mg {

__host__ __device__ inline void local_edge(int dim, int k, int &a, int &b) {
  if (dim == 2) {
    const int E[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    a = E[k][0];
    b = E[k][1];
  } else {
    const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    a = E[k][0];
    b = E[k][1];
  }
}

__host__ __device__ inline int n_local(int dim, int degree) {
  if (degree == 1) return dim + 1;
  if (degree == 2) return dim == 2 ? 6 : 10;
  return 10;
}

// value of local basis function i at barycentric point lam
__host__ __device__ inline double basis_value(int dim, int degree, int i, const double *lam) {
  int nv = dim + 1;
  if (degree == 1) return lam[i];
  if (degree == 2) {
    if (i < nv) return lam[i] * (2.0 * lam[i] - 1.0);
    int a, b;
    local_edge(dim, i - nv, a, b);
    return 4.0 * lam[a] * lam[b];
  }
  // degree 3, triangles
  if (i < 3) return 0.5 * lam[i] * (3.0 * lam[i] - 1.0) * (3.0 * lam[i] - 2.0);
  if (i < 9) {
    int k = (i - 3) / 2, a, b;
    local_edge(2, k, a, b);
    int near = ((i - 3) % 2 == 0) ? a : b;
    return 4.5 * lam[a] * lam[b] * (3.0 * lam[near] - 1.0);
  }
  return 27.0 * lam[0] * lam[1] * lam[2];
}

// derivative of local basis function i with respect to lam[c]
__host__ __device__ inline double basis_dlam(int dim, int degree, int i, int c, const double *lam) {
  int nv = dim + 1;
  if (degree == 1) return i == c ? 1.0 : 0.0;
  if (degree == 2) {
    if (i < nv) return i == c ? 4.0 * lam[i] - 1.0 : 0.0;
    int a, b;
    local_edge(dim, i - nv, a, b);
    return (c == a ? 4.0 * lam[b] : 0.0) + (c == b ? 4.0 * lam[a] : 0.0);
  }
  if (i < 3) return i == c ? 0.5 * (27.0 * lam[i] * lam[i] - 18.0 * lam[i] + 2.0) : 0.0;
  if (i < 9) {
    int k = (i - 3) / 2, a, b;
    local_edge(2, k, a, b);
    int near = ((i - 3) % 2 == 0) ? a : b;
    int far = near == a ? b : a;
    // f = 4.5 (3 lam_n^2 lam_f - lam_n lam_f)
    if (c == near) return 4.5 * (6.0 * lam[near] * lam[far] - lam[far]);
    if (c == far) return 4.5 * (3.0 * lam[near] * lam[near] - lam[near]);
    return 0.0;
  }
  double p = 27.0;
  for (int q = 0; q < 3; ++q)
    if (q != c) p *= lam[q];
  return p;
}

}  // namespace mg
