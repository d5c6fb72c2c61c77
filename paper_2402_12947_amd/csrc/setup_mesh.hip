// Degree-of-freedom map and cell quality on the GPU.
//
// DOF numbering (the paper does not fix one): vertices first, then edges in the
// order of their sorted (low, high) vertex pairs -- one DOF each for P2, two for
// P3 (the node nearer the low vertex first) -- then one interior DOF per P3
// triangle.  Edges are found by a device radix sort of the (low, high) keys of
// every cell edge.  A non-vertex DOF is Dirichlet iff it lies on a boundary
// facet (a facet of exactly one cell) whose vertices are all Dirichlet.
//
// Cell quality: the normalised radius ratio gamma = d R_I / R_C (paper Sec. 3,
// eq. radius_ratio; ideal simplex = 1).  Triangles use 2 R_I / R_C =
// 16 A^2 / ((a+b+c) a b c); tetrahedra use R_I = 3V / (sum of face areas) and the
// circumradius formula 24 V R_C = sqrt((aA+bB+cC)(aA+bB-cC)(aA-bB+cC)(-aA+bB+cC))
// over the three pairs (a, A), (b, B), (c, C) of opposite edge lengths.
#include "devutil.h"

namespace mg {

__constant__ int c_edge2[3][2] = {{0, 1}, {0, 2}, {1, 2}};
__constant__ int c_edge3[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

__global__ void k_edge_keys(const int32_t *cells, int64_t nc, int dim, int64_t nv, uint64_t *keys) {
  int nle = dim == 2 ? 3 : 6;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * nle) return;
  int64_t c = t / nle;
  int k = (int)(t - c * nle);
  int a = dim == 2 ? c_edge2[k][0] : c_edge3[k][0];
  int b = dim == 2 ? c_edge2[k][1] : c_edge3[k][1];
  uint64_t va = (uint64_t)cells[c * (dim + 1) + a], vb = (uint64_t)cells[c * (dim + 1) + b];
  uint64_t lo = va < vb ? va : vb, hi = va < vb ? vb : va;
  keys[t] = lo * (uint64_t)nv + hi;
}

__global__ void k_cell_edges(const uint64_t *keys, int64_t nkeys, const uint64_t *edges, int64_t ne,
                             int32_t *cell_edge) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nkeys) return;
  cell_edge[t] = (int32_t)lower_bound_dev(edges, ne, keys[t]);
}

// 2D: an edge occurring once in the sorted key list is a boundary facet.
__global__ void k_boundary_edges_2d(const uint64_t *sorted, int64_t n, const uint64_t *edges, int64_t ne,
                                    const uint8_t *dirv, int64_t nv, uint8_t *dir_edge) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t k = sorted[i];
  bool single = (i == 0 || sorted[i - 1] != k) && (i == n - 1 || sorted[i + 1] != k);
  if (!single) return;
  uint64_t lo = k / (uint64_t)nv, hi = k % (uint64_t)nv;
  if (dirv[lo] && dirv[hi]) dir_edge[lower_bound_dev(edges, ne, k)] = 1;
}

// 3D: faces whose three vertices are all Dirichlet, keyed by compact ids.
__global__ void k_dirichlet_face_keys(const int32_t *cells, int64_t nc, const uint8_t *dirv,
                                      const int32_t *did, uint64_t nd, uint64_t *keys) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * 4) return;
  int64_t c = t / 4;
  int skip = (int)(t - c * 4);
  uint64_t v[3];
  int m = 0;
  bool all = true;
  for (int a = 0; a < 4; ++a) {
    if (a == skip) continue;
    int32_t g = cells[c * 4 + a];
    all = all && dirv[g];
    v[m++] = all ? (uint64_t)did[g] : 0;
  }
  if (!all) { keys[t] = ~0ULL; return; }
  // sort three values
  if (v[0] > v[1]) { uint64_t x = v[0]; v[0] = v[1]; v[1] = x; }
  if (v[1] > v[2]) { uint64_t x = v[1]; v[1] = v[2]; v[2] = x; }
  if (v[0] > v[1]) { uint64_t x = v[0]; v[0] = v[1]; v[1] = x; }
  keys[t] = (v[0] * nd + v[1]) * nd + v[2];
}

__global__ void k_boundary_faces_3d(const uint64_t *sorted, int64_t n, uint64_t nd, const int32_t *dvert,
                                    const uint64_t *edges, int64_t ne, int64_t nv, uint8_t *dir_edge) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t k = sorted[i];
  if (k == ~0ULL) return;
  bool single = (i == 0 || sorted[i - 1] != k) && (i == n - 1 || sorted[i + 1] != k);
  if (!single) return;
  uint64_t c = k % nd, b = (k / nd) % nd, a = k / (nd * nd);
  uint64_t g[3] = {(uint64_t)dvert[a], (uint64_t)dvert[b], (uint64_t)dvert[c]};
  for (int p = 0; p < 3; ++p)
    for (int q = p + 1; q < 3; ++q) {
      uint64_t lo = g[p] < g[q] ? g[p] : g[q], hi = g[p] < g[q] ? g[q] : g[p];
      int64_t e = lower_bound_dev(edges, ne, lo * (uint64_t)nv + hi);
      if (e < ne && edges[e] == lo * (uint64_t)nv + hi) dir_edge[e] = 1;
    }
}

__global__ void k_cell_dofs(const int32_t *cells, const int32_t *cell_edge, int64_t nc, int dim, int degree,
                            int64_t nv, int64_t ne, int nloc, int32_t *cd) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  int nvert = dim + 1, nle = dim == 2 ? 3 : 6;
  int32_t *o = cd + c * nloc;
  for (int a = 0; a < nvert; ++a) o[a] = cells[c * nvert + a];
  if (degree == 2) {
    for (int k = 0; k < nle; ++k) o[nvert + k] = (int32_t)(nv + cell_edge[c * nle + k]);
  } else if (degree == 3) {
    for (int k = 0; k < 3; ++k) {
      int32_t ga = cells[c * 3 + c_edge2[k][0]], gb = cells[c * 3 + c_edge2[k][1]];
      int64_t base = nv + 2 * (int64_t)cell_edge[c * 3 + k];
      o[3 + 2 * k] = (int32_t)(base + (ga > gb ? 1 : 0));      // node nearer local vertex a
      o[3 + 2 * k + 1] = (int32_t)(base + (ga < gb ? 1 : 0));  // node nearer local vertex b
    }
    o[9] = (int32_t)(nv + 2 * ne + c);
  }
}

__global__ void k_dof_flags(const uint8_t *dirv, int64_t nv, const uint8_t *dir_edge, int64_t ne, int degree,
                            int64_t ndofs, int32_t *isfree) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndofs) return;
  uint8_t d;
  if (i < nv) d = dirv[i];
  else if (degree == 2 && i < nv + ne) d = dir_edge[i - nv];
  else if (degree == 3 && i < nv + 2 * ne) d = dir_edge[(i - nv) / 2];
  else d = 0;
  isfree[i] = d ? 0 : 1;
}

__global__ void k_free_maps(const int32_t *isfree, const int32_t *scan, int64_t ndofs, int32_t *free_index,
                            int32_t *free_dofs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndofs) return;
  if (isfree[i]) {
    free_index[i] = scan[i];
    free_dofs[scan[i]] = (int32_t)i;
  } else {
    free_index[i] = -1;
  }
}

__global__ void k_vertex_nodes(const double *coords, int64_t n, double *nodes) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) nodes[i] = coords[i];
}

__global__ void k_edge_nodes(const uint64_t *edges, int64_t ne, int64_t nv, int dim, int degree,
                             const double *coords, double *nodes) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int64_t lo = (int64_t)(edges[e] / (uint64_t)nv), hi = (int64_t)(edges[e] % (uint64_t)nv);
  for (int x = 0; x < dim; ++x) {
    double a = coords[lo * dim + x], b = coords[hi * dim + x];
    if (degree == 2) {
      nodes[(nv + e) * dim + x] = 0.5 * (a + b);
    } else {
      nodes[(nv + 2 * e) * dim + x] = (2.0 * a + b) / 3.0;
      nodes[(nv + 2 * e + 1) * dim + x] = (a + 2.0 * b) / 3.0;
    }
  }
}

__global__ void k_cell_centroids(const int32_t *cells, int64_t nc, int64_t off, const double *coords,
                                 double *nodes) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  for (int x = 0; x < 2; ++x) {
    double s = coords[(int64_t)cells[c * 3] * 2 + x] + coords[(int64_t)cells[c * 3 + 1] * 2 + x] +
               coords[(int64_t)cells[c * 3 + 2] * 2 + x];
    nodes[(off + c) * 2 + x] = s / 3.0;
  }
}

void build_dofmap(Ctx &c, Level &L, const mg_mesh &m) {
  hipStream_t s = c.stream;
  L.dim = m.dim;
  L.nv = m.n_vertices;
  L.nc = m.n_cells;
  const int dim = L.dim, deg = L.degree, nvert = dim + 1;
  const int nle = dim == 2 ? 3 : 6;
  upload(L.coords, m.coords, (size_t)(L.nv * dim), s);
  upload(L.cells, m.cells, (size_t)(L.nc * nvert), s);
  upload(L.dirv, m.dirichlet_vertex, (size_t)L.nv, s);
  L.nloc = deg == 1 ? nvert : deg == 2 ? (dim == 2 ? 6 : 10) : 10;

  DBuf<uint64_t> edges;
  DBuf<int32_t> cell_edge;
  DBuf<uint8_t> dir_edge;
  L.ne = 0;
  if (deg >= 2) {
    int64_t nkeys = L.nc * nle;
    DBuf<uint64_t> keys, sorted;
    keys.alloc(nkeys);
    sorted.alloc(nkeys);
    k_edge_keys<<<grid_for(nkeys, 256), 256, 0, s>>>(L.cells, L.nc, dim, L.nv, keys);
    MG_LAUNCH_CHECK();
    int endbit = bits_for((uint64_t)L.nv * (uint64_t)L.nv);
    sort_keys(s, keys.p, sorted.p, nkeys, endbit);
    edges.alloc(nkeys);
    DBuf<int32_t> runlen;
    runlen.alloc(nkeys);
    L.ne = run_length(s, sorted.p, edges.p, runlen.p, nkeys);
    cell_edge.alloc(nkeys);
    k_cell_edges<<<grid_for(nkeys, 256), 256, 0, s>>>(keys, nkeys, edges, L.ne, cell_edge);
    MG_LAUNCH_CHECK();
    dir_edge.alloc(L.ne);
    MG_HIP(hipMemsetAsync(dir_edge.p, 0, L.ne, s));
    if (dim == 2) {
      k_boundary_edges_2d<<<grid_for(nkeys, 256), 256, 0, s>>>(sorted, nkeys, edges, L.ne, L.dirv, L.nv,
                                                              dir_edge);
      MG_LAUNCH_CHECK();
    } else {
      // compact ids of Dirichlet vertices
      std::vector<int32_t> hdid(L.nv), hdvert;
      for (int64_t v = 0; v < L.nv; ++v) {
        hdid[v] = (int32_t)hdvert.size();
        if (m.dirichlet_vertex[v]) hdvert.push_back((int32_t)v);
      }
      uint64_t nd = hdvert.size();
      if (nd > 0) {
        if (nd > 2000000ULL) fail(MG_ERR_LIMIT, "more than 2e6 Dirichlet vertices in 3D");
        DBuf<int32_t> did, dvert;
        upload(did, hdid.data(), hdid.size(), s);
        upload(dvert, hdvert.data(), hdvert.size(), s);
        int64_t nf = L.nc * 4;
        DBuf<uint64_t> fk, fs;
        fk.alloc(nf);
        fs.alloc(nf);
        k_dirichlet_face_keys<<<grid_for(nf, 256), 256, 0, s>>>(L.cells, L.nc, L.dirv, did, nd, fk);
        MG_LAUNCH_CHECK();
        sort_keys(s, fk.p, fs.p, nf, 64);
        k_boundary_faces_3d<<<grid_for(nf, 256), 256, 0, s>>>(fs, nf, nd, dvert, edges, L.ne, L.nv, dir_edge);
        MG_LAUNCH_CHECK();
      }
    }
  }
  L.ndofs = L.nv + (deg == 2 ? L.ne : deg == 3 ? 2 * L.ne + L.nc : 0);
  if (L.ndofs >= 2147483647LL) fail(MG_ERR_LIMIT, "more than 2^31 DOFs");
  L.cell_dofs.alloc(L.nc * L.nloc);
  k_cell_dofs<<<grid_for(L.nc, 256), 256, 0, s>>>(L.cells, cell_edge.p, L.nc, dim, deg, L.nv, L.ne, L.nloc,
                                                  L.cell_dofs);
  MG_LAUNCH_CHECK();
  DBuf<int32_t> isfree, scan;
  isfree.alloc(L.ndofs);
  scan.alloc(L.ndofs);
  k_dof_flags<<<grid_for(L.ndofs, 256), 256, 0, s>>>(L.dirv, L.nv, dir_edge.p, L.ne, deg, L.ndofs, isfree);
  MG_LAUNCH_CHECK();
  L.nfree = exclusive_scan(s, isfree.p, scan.p, L.ndofs);
  if (L.nfree == 0) fail(MG_ERR_ARG, "level has no free DOFs");
  L.nfree_s = L.nfree;
  L.ncomp = 1;
  L.free_index.alloc(L.ndofs);
  L.free_dofs.alloc(L.nfree);
  k_free_maps<<<grid_for(L.ndofs, 256), 256, 0, s>>>(isfree, scan, L.ndofs, L.free_index, L.free_dofs);
  MG_LAUNCH_CHECK();
  L.nodes.alloc(L.ndofs * dim);
  k_vertex_nodes<<<grid_for(L.nv * dim, 256), 256, 0, s>>>(L.coords, L.nv * dim, L.nodes);
  MG_LAUNCH_CHECK();
  if (deg >= 2) {
    k_edge_nodes<<<grid_for(L.ne, 256), 256, 0, s>>>(edges, L.ne, L.nv, dim, deg, L.coords, L.nodes);
    MG_LAUNCH_CHECK();
  }
  if (deg == 3) {
    k_cell_centroids<<<grid_for(L.nc, 256), 256, 0, s>>>(L.cells, L.nc, L.nv + 2 * L.ne, L.coords, L.nodes);
    MG_LAUNCH_CHECK();
  }
  MG_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// quality
// ---------------------------------------------------------------------------
__device__ inline double len3(double x, double y, double z) { return sqrt(x * x + y * y + z * z); }

__global__ void k_quality(const double *X, const int32_t *cells, int64_t nc, int dim, double tau, double *gamma,
                          uint8_t *flags, unsigned long long *gmin, int *bad) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  double g;
  if (dim == 2) {
    const int32_t *v = cells + c * 3;
    double x0 = X[2 * v[0]], y0 = X[2 * v[0] + 1], x1 = X[2 * v[1]], y1 = X[2 * v[1] + 1];
    double x2 = X[2 * v[2]], y2 = X[2 * v[2] + 1];
    double cr = (x1 - x0) * (y2 - y0) - (y1 - y0) * (x2 - x0);  // 2 * signed area
    if (!(cr > 0)) atomicMax(bad, 1);
    double a = hypot(x1 - x2, y1 - y2), b = hypot(x0 - x2, y0 - y2), e = hypot(x0 - x1, y0 - y1);
    g = 4.0 * cr * cr / ((a + b + e) * a * b * e);
  } else {
    const int32_t *v = cells + c * 4;
    double p[4][3];
    for (int k = 0; k < 4; ++k)
      for (int x = 0; x < 3; ++x) p[k][x] = X[3 * (int64_t)v[k] + x];
    double u[3], w[3], t[3];
    for (int x = 0; x < 3; ++x) { u[x] = p[1][x] - p[0][x]; w[x] = p[2][x] - p[0][x]; t[x] = p[3][x] - p[0][x]; }
    double det = u[0] * (w[1] * t[2] - w[2] * t[1]) - u[1] * (w[0] * t[2] - w[2] * t[0]) +
                 u[2] * (w[0] * t[1] - w[1] * t[0]);
    if (!(det > 0)) atomicMax(bad, 1);
    double V = det / 6.0;
    // face areas: face opposite vertex k
    double S = 0;
    const int fv[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    for (int k = 0; k < 4; ++k) {
      const double *A = p[fv[k][0]], *B = p[fv[k][1]], *C = p[fv[k][2]];
      double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
      double e2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
      S += 0.5 * len3(e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]);
    }
    double rin = 3.0 * V / S;
    auto L = [&](int i, int j) { return len3(p[i][0] - p[j][0], p[i][1] - p[j][1], p[i][2] - p[j][2]); };
    double aA = L(0, 1) * L(2, 3), bB = L(0, 2) * L(1, 3), cC = L(0, 3) * L(1, 2);
    double prod = (aA + bB + cC) * (aA + bB - cC) * (aA - bB + cC) * (-aA + bB + cC);
    double rc = sqrt(fmax(prod, 0.0)) / (24.0 * V);
    g = 3.0 * rin / rc;
  }
  gamma[c] = g;
  flags[c] = g < tau ? 1 : 0;
  if (g > 0) atomicMin(gmin, (unsigned long long)__double_as_longlong(g));
}

void compute_quality(Ctx &c, Level &L) {
  hipStream_t s = c.stream;
  L.gamma.alloc(L.nc);
  L.flags.alloc(L.nc);
  DBuf<unsigned long long> gmin;
  DBuf<int> bad;
  gmin.alloc(1);
  bad.alloc(1);
  unsigned long long init = (unsigned long long)__builtin_bit_cast(long long, 1e300);
  MG_HIP(hipMemcpyAsync(gmin.p, &init, sizeof(init), hipMemcpyHostToDevice, s));
  MG_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
  k_quality<<<grid_for(L.nc, 256), 256, 0, s>>>(L.coords, L.cells, L.nc, L.dim, c.tau, L.gamma, L.flags, gmin, bad);
  MG_LAUNCH_CHECK();
  unsigned long long hg = 0;
  int hb = 0;
  MG_HIP(hipMemcpyAsync(&hg, gmin.p, sizeof(hg), hipMemcpyDeviceToHost, s));
  MG_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  if (hb) fail(MG_ERR_MESH, "a cell has non-positive volume (cells must be positively oriented)");
  L.gamma_min = __builtin_bit_cast(double, (long long)hg);
}

}  // namespace mg
