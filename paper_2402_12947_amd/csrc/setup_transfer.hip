// Non-nested interpolation prolongation (paper Sec. 2: [P_l]_ij = phi_j^(l+1)(x_i))
// by point location of the fine DOF nodes in the coarse mesh, and R = P^T.
//
// Location rule (the paper is silent on ties): the coarse cell of a node is the
// lowest-id cell whose smallest barycentric coordinate at the node is >= -1e-12;
// if there is none, the cell with the largest smallest barycentric coordinate
// (lowest id on ties) provided it is >= -1e-8; otherwise location fails.
// Candidates come from a uniform bucket grid over the coarse mesh: every cell
// is listed in each bucket its (slightly enlarged) bounding box overlaps, so
// every cell that can satisfy either test at a point is a candidate of the
// point's bucket.
#include <algorithm>
#include <cmath>

#include "basis.h"
#include "devutil.h"
#include "geom.h"

namespace mg {

struct Grid {
  double lo[3], inv_h[3], pad;
  int n[3];
};

__device__ inline int bucket_coord(double x, const Grid &g, int a) {
  int i = (int)floor((x - g.lo[a]) * g.inv_h[a]);
  return i < 0 ? 0 : (i >= g.n[a] ? g.n[a] - 1 : i);
}

__device__ inline void cell_box(const double *X, const int32_t *v, int dim, const Grid &g, int b0[3], int b1[3]) {
  for (int a = 0; a < dim; ++a) {
    double mn = 1e300, mx = -1e300;
    for (int k = 0; k <= dim; ++k) {
      double x = X[(int64_t)v[k] * dim + a];
      mn = fmin(mn, x);
      mx = fmax(mx, x);
    }
    double ext = (mx - mn) * 1e-6 + g.pad;
    b0[a] = bucket_coord(mn - ext, g, a);
    b1[a] = bucket_coord(mx + ext, g, a);
  }
  for (int a = dim; a < 3; ++a) b0[a] = b1[a] = 0;
}

__global__ void k_bucket_count(const double *X, const int32_t *cells, int64_t nc, int dim, Grid g, int32_t *cnt) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  int b0[3], b1[3];
  cell_box(X, cells + c * (dim + 1), dim, g, b0, b1);
  for (int k = b0[2]; k <= b1[2]; ++k)
    for (int j = b0[1]; j <= b1[1]; ++j)
      for (int i = b0[0]; i <= b1[0]; ++i) atomicAdd(&cnt[(k * g.n[1] + j) * g.n[0] + i], 1);
}

__global__ void k_bucket_fill(const double *X, const int32_t *cells, int64_t nc, int dim, Grid g,
                              const int64_t *off, int32_t *cursor, int32_t *list) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  int b0[3], b1[3];
  cell_box(X, cells + c * (dim + 1), dim, g, b0, b1);
  for (int k = b0[2]; k <= b1[2]; ++k)
    for (int j = b0[1]; j <= b1[1]; ++j)
      for (int i = b0[0]; i <= b1[0]; ++i) {
        int b = (k * g.n[1] + j) * g.n[0] + i;
        int pos = atomicAdd(&cursor[b], 1);
        list[off[b] + pos] = (int32_t)c;
      }
}

__device__ inline void barycentric(const double *X, const int32_t *v, int dim, const double *x, double lam[4]) {
  double g[4][3];
  simplex_grads(X, v, dim, g);
  double s = 0;
  for (int k = 1; k <= dim; ++k) {
    double l = 0;
    for (int a = 0; a < dim; ++a) l += g[k][a] * (x[a] - X[(int64_t)v[0] * dim + a]);
    lam[k] = l;
    s += l;
  }
  lam[0] = 1.0 - s;
}

__global__ void k_locate(const double *fnodes, const int32_t *ffree, int64_t nf, const double *X,
                         const int32_t *cells, const int32_t *ccd, const int32_t *cfree_index, int dim, int cdeg,
                         int cnloc, Grid g, const int64_t *off, const int32_t *list, int32_t *locate, int32_t *pcol,
                         double *pval, int *bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  double x[3] = {0, 0, 0};
  int64_t node = ffree[i];
  for (int a = 0; a < dim; ++a) x[a] = fnodes[node * dim + a];
  int bc[3] = {0, 0, 0};
  for (int a = 0; a < dim; ++a) bc[a] = bucket_coord(x[a], g, a);
  int b = (bc[2] * g.n[1] + bc[1]) * g.n[0] + bc[0];
  int32_t inside = 2147483647, best = -1;
  double bestmin = -1e300;
  for (int64_t k = off[b]; k < off[b + 1]; ++k) {
    int32_t c = list[k];
    double lam[4];
    barycentric(X, cells + (int64_t)c * (dim + 1), dim, x, lam);
    double mn = lam[0];
    for (int a = 1; a <= dim; ++a) mn = fmin(mn, lam[a]);
    if (mn >= -1e-12 && c < inside) inside = c;
    if (mn > bestmin || (mn == bestmin && c < best)) {
      bestmin = mn;
      best = c;
    }
  }
  int32_t cell;
  if (inside != 2147483647) {
    cell = inside;
  } else if (best >= 0 && bestmin >= -1e-8) {
    cell = best;
  } else {
    atomicMin(bad, (int)i);
    cell = best >= 0 ? best : 0;
  }
  locate[i] = cell;
  double lam[4];
  barycentric(X, cells + (int64_t)cell * (dim + 1), dim, x, lam);
  for (int j = 0; j < cnloc; ++j) {
    int32_t cf = cfree_index[ccd[(int64_t)cell * cnloc + j]];
    pcol[i * cnloc + j] = cf;
    pval[i * cnloc + j] = cf >= 0 ? basis_value(dim, cdeg, j, lam) : 0.0;
  }
}

// vector ELL row (i, c) = scalar row i with columns j -> j * ncomp + c
__global__ void k_expand_ell(const int32_t *col, const double *val, int64_t nrows, int pw, int ncomp,
                             int32_t *vcol, double *vval) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * ncomp * pw) return;
  int64_t vr = t / pw;
  int k = (int)(t - vr * pw);
  int64_t r = vr / ncomp;
  int cmp = (int)(vr - r * ncomp);
  int32_t j = col[r * pw + k];
  vcol[t] = j >= 0 ? j * ncomp + cmp : -1;
  vval[t] = val[r * pw + k];
}

void build_prolongation(Ctx &c, Level &F, const Level &C, const mg_mesh &cm) {
  hipStream_t s = c.stream;
  const int dim = C.dim;
  // bucket grid over the coarse mesh
  Grid g{};
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < cm.n_vertices; ++v)
    for (int a = 0; a < dim; ++a) {
      lo[a] = std::min(lo[a], cm.coords[v * dim + a]);
      hi[a] = std::max(hi[a], cm.coords[v * dim + a]);
    }
  double per = std::pow((double)C.nc / 2.0, 1.0 / dim);
  int64_t nb = 1;
  double diam = 0;
  for (int a = 0; a < dim; ++a) {
    double ext = std::max(hi[a] - lo[a], 1e-300);
    g.n[a] = std::max(1, std::min(4096, (int)std::ceil(per)));
    g.lo[a] = lo[a];
    g.inv_h[a] = g.n[a] / ext;
    nb *= g.n[a];
    diam = std::max(diam, ext);
  }
  for (int a = dim; a < 3; ++a) {
    g.n[a] = 1;
    g.lo[a] = 0;
    g.inv_h[a] = 0;
  }
  g.pad = 1e-9 * diam;
  DBuf<int32_t> cnt, cursor;
  DBuf<int64_t> off;
  cnt.alloc(nb);
  cursor.alloc(nb);
  off.alloc(nb + 1);
  MG_HIP(hipMemsetAsync(cnt.p, 0, nb * sizeof(int32_t), s));
  MG_HIP(hipMemsetAsync(cursor.p, 0, nb * sizeof(int32_t), s));
  k_bucket_count<<<grid_for(C.nc, 256), 256, 0, s>>>(C.coords, C.cells, C.nc, dim, g, cnt);
  MG_LAUNCH_CHECK();
  int64_t total = exclusive_scan(s, cnt.p, off.p, nb);
  MG_HIP(hipMemcpyAsync(off.p + nb, &total, sizeof(int64_t), hipMemcpyHostToDevice, s));
  DBuf<int32_t> list;
  list.alloc(total);
  k_bucket_fill<<<grid_for(C.nc, 256), 256, 0, s>>>(C.coords, C.cells, C.nc, dim, g, off, cursor, list);
  MG_LAUNCH_CHECK();
  // locate and evaluate the coarse basis (per free DOF node)
  F.pw = C.nloc;
  F.locate.alloc(F.nfree_s);
  F.pcol.alloc(F.nfree_s * F.pw);
  F.pval.alloc(F.nfree_s * F.pw);
  DBuf<int> bad;
  bad.alloc(1);
  int init = 2147483647;
  MG_HIP(hipMemcpyAsync(bad.p, &init, sizeof(int), hipMemcpyHostToDevice, s));
  k_locate<<<grid_for(F.nfree_s, 128), 128, 0, s>>>(F.nodes, F.free_dofs, F.nfree_s, C.coords, C.cells, C.cell_dofs,
                                                 C.free_index, dim, C.degree, C.nloc, g, off, list, F.locate,
                                                 F.pcol, F.pval, bad);
  MG_LAUNCH_CHECK();
  int hb = 0;
  MG_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  if (hb != 2147483647)
    fail(MG_ERR_LOCATE, "free DOF %d of a fine level lies outside the next coarser mesh", hb);
  if (F.ncomp > 1) {  // P (x) I: every component interpolated on its own
    DBuf<int32_t> vc;
    DBuf<double> vv;
    vc.alloc(F.nfree * F.pw);
    vv.alloc(F.nfree * F.pw);
    k_expand_ell<<<grid_for(F.nfree * F.pw, 256), 256, 0, s>>>(F.pcol, F.pval, F.nfree_s, F.pw, F.ncomp, vc, vv);
    MG_LAUNCH_CHECK();
    F.pcol = std::move(vc);
    F.pval = std::move(vv);
  }
  ell_to_csr(c, F.nfree, C.nfree, F.pw, F.pcol, F.pval, false, F.Pc);
  ell_to_csr(c, F.nfree, C.nfree, F.pw, F.pcol, F.pval, true, F.Rc);
}

}  // namespace mg
