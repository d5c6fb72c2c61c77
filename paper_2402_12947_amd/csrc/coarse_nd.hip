// Coarsest-level direct solve by nested dissection (paper Sec. 2: a direct
// solver on the coarsest grid).
//
// The dense explicit inverse reads n^2 / 2 entries per solve, which grows to
// 5.4 GB on a 36,863-unknown coarsest level.  Here the unknowns are ordered by
// nested dissection (recursive coordinate bisection of the DOF nodes; the
// separator of a split is the boundary of the smaller side in the matrix
// graph; leaves of at most `leaf` unknowns; subtrees first, separator last),
// the permuted matrix is factored A = L L^T (dense Cholesky on the matrix
// cores, setup only), and the solve reads only what the ordering leaves
// nonzero:
//   * per supernode s (a leaf or a separator, a contiguous range of the
//     order) the inverse of its diagonal block, (L_ss)^-1 = (L^-1)_ss, stored
//     as lower 32 x 32 tiles;
//   * per supernode the rows of L below it, which lie in its ancestors, as
//     32-row tile rows; tile rows that are zero (ancestor rows the subtree does
//     not touch) are not stored.
// Forward (L y = b) from the leaves up, one height of the tree per step:
// gather b_s minus the contributions of the descendants (fixed order), y_s =
// (L_ss)^-1 b_s, contributions of s to its ancestors' rows.  Backward
// (L^T x = y) from the root down: t_s = sum over the stored tile rows of their
// transpose times x, x_s = (L_ss)^-T (y_s - t_s).  Five launches per tree
// height, one workgroup per output tile, every sum in a fixed order
// (deterministic, no atomics).  All in FP64 (the coarsest solve stays FP64 in
// the mixed cycle).
#include <algorithm>
#include <cmath>
#include <numeric>

#include "devutil.h"
#include "sell_row.h"

namespace mg {

void dense_cholesky(hipStream_t s, double *M, int64_t n, int *bad);
void dense_lower_inverse(hipStream_t s, const double *M, int64_t n, double *W);

namespace {

constexpr int T = 32;  // tile edge

// A in the nested-dissection order, dense: M[q[r] n + q[c]] = a_rc
__global__ void k_dense_nd(const int64_t *rp, const int32_t *col, const double *val, const int32_t *q, int64_t n,
                           double *M) {
  const int64_t r = blockIdx.x;
  if (r >= n) return;
  const int64_t qr = q[r];
  for (int64_t k = rp[r] + threadIdx.x; k < rp[r + 1]; k += blockDim.x) M[qr * n + q[col[k]]] = val[k];
}

// 1 if the block rows [r0, r0 + nr) x cols [c0, c0 + nc) of the n x n matrix
// hold a nonzero (one workgroup per candidate)
__global__ void k_block_nonzero(const double *M, int64_t n, const int32_t *r0, const int32_t *nr,
                                const int32_t *c0, const int32_t *nc, int *flag) {
  const int k = blockIdx.x;
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  const int64_t rows = nr[k], cols = nc[k];
  int mine = 0;
  for (int64_t t = threadIdx.x; t < rows * cols && !mine; t += blockDim.x)
    mine = M[(r0[k] + t / cols) * n + c0[k] + t % cols] != 0.0;
  if (mine) any = 1;
  __syncthreads();
  if (threadIdx.x == 0) flag[k] = any;
}

// copy a (rows x cols) block at (r0, c0) of the n x n matrix into one 32 x 32
// tile (zero beyond the block); one workgroup per tile
__global__ void k_copy_tiles(const double *M, int64_t n, const int32_t *r0, const int32_t *nr, const int32_t *c0,
                             const int32_t *nc, const int64_t *off, double *out) {
  const int k = blockIdx.x;
  double *o = out + off[k];
  for (int e = threadIdx.x; e < T * T; e += blockDim.x) {
    const int i = e / T, j = e % T;
    o[e] = (i < nr[k] && j < nc[k]) ? M[(int64_t)(r0[k] + i) * n + c0[k] + j] : 0.0;
  }
}

// ---- solve kernels: one workgroup (four wavefronts) per output tile -------
// The loop over the tiles that contribute to an output tile is dealt to the
// four wavefronts (tile k to wavefront k mod 4), each keeping the next tile of
// its share in flight; the four partial sums are added in wavefront order.
// In a wavefront, lane (h, j) = (lane >> 5, lane & 31) reads rows 2 s + h,
// s = 0..15, column j of a tile, so each tile is read once in 512-byte lines:
//   row products  T v: the tile goes through the wavefront's LDS area and lane
//                      (h, i) sums half of row i;
//   column products T^T w: lane-private, the two halves added by a shuffle.

struct NdArgs {
  const int32_t *t_sup, *t_loc;     // per global tile: supernode, local tile index
  const int32_t *s_a, *s_n, *s_t0;  // per supernode: first index, size, first global tile
  const int64_t *s_doff;            // per supernode: offset of its diagonal-inverse tiles
  const double *dinv;
  const int32_t *q_sup, *q_tgt;     // per stored tile row: supernode, target global tile
  const int64_t *q_off;
  const double *bval;
  const int32_t *s_qptr, *s_q;      // per supernode: its stored tile rows
  const int32_t *g_qptr, *g_q;      // per global tile: tile rows that target it
  const int32_t *pos;               // ND index -> unknown
  double *bp, *y, *t, *x, *contrib;
};

// entry r (< 32) of global tile g in the ND order, or -1 past its supernode
__device__ inline int64_t tile_row(const NdArgs &A, int g, int r) {
  const int s = A.t_sup[g], l = A.t_loc[g];
  const int i = l * T + r;
  return i < A.s_n[s] ? (int64_t)A.s_a[s] + i : -1;
}

struct NdSmem {
  double tl[4][T][T + 1];  // tile transposes, per wavefront
  double vl[4][T];         // vector segments, per wavefront
  double part[4][T];       // partial sums, per wavefront
};

__device__ inline void load_tile(const double *__restrict__ tile, int lane, double v[16]) {
  const int h = lane >> 5, j = lane & 31;
#pragma unroll
  for (int s = 0; s < 16; ++s) v[s] = __builtin_nontemporal_load(tile + (2 * s + h) * T + j);
}

// row products of a tile held in registers with the segment vs (LDS); returns
// row (lane & 31)'s dot product in both halves of the wavefront
__device__ inline double rows_of(const double v[16], const double *vs, double (*Ts)[T + 1], int lane) {
  const int h = lane >> 5, j = lane & 31;
#pragma unroll
  for (int s = 0; s < 16; ++s) Ts[2 * s + h][j] = v[s];
  wave_sync();
  double a = 0;
#pragma unroll
  for (int t = 0; t < 16; ++t) a += Ts[j][16 * h + t] * vs[16 * h + t];
  wave_sync();
  return a + __shfl_xor(a, 32);
}

// column products: column (lane & 31)'s dot product in both halves
__device__ inline double cols_of(const double v[16], const double *ws, int lane) {
  const int h = lane >> 5;
  double c = 0;
#pragma unroll
  for (int s = 0; s < 16; ++s) c += v[s] * ws[2 * s + h];
  return c + __shfl_xor(c, 32);
}

// the four wavefronts' partial sums, added in wavefront order (lanes < 32 of
// wavefront 0 hold the result)
__device__ inline double combine(NdSmem &sm, int wave, int lane, double acc) {
  if (lane < T) sm.part[wave][lane] = acc;
  __syncthreads();
  double r = 0;
  if (wave == 0 && lane < T) r = ((sm.part[0][lane] + sm.part[1][lane]) + sm.part[2][lane]) + sm.part[3][lane];
  return r;
}

// Generic loop: output = sum over k < count of op(tile(k), seg(k)); wavefront
// w takes k = w, w + 4, ...; ROWS selects row products (else columns).
template <bool ROWS, class TileF, class SegF>
__device__ inline double wg_sum(NdSmem &sm, int count, TileF tile, SegF seg) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double acc = 0;
  double v[16], nxt[16];
  if (wave < count) load_tile(tile(wave), lane, nxt);
  for (int k = wave; k < count; k += 4) {
#pragma unroll
    for (int s = 0; s < 16; ++s) v[s] = nxt[s];
    if (k + 4 < count) load_tile(tile(k + 4), lane, nxt);
    if (lane < T) sm.vl[wave][lane] = seg(k, lane);
    wave_sync();
    acc += ROWS ? rows_of(v, sm.vl[wave], sm.tl[wave], lane) : cols_of(v, sm.vl[wave], lane);
    wave_sync();
  }
  return combine(sm, wave, lane, acc);
}

// K1: bp = b (in the ND order) minus the descendants' contributions; eight
// streams (four wavefronts, two halves) take the incoming tile rows k = 8 m +
// stream, added in stream order
template <class TV>
__global__ __launch_bounds__(256) void k_nd_gather(NdArgs A, const int32_t *tiles, const TV *b, int vs) {
  __shared__ double part[8][T];
  const int g = tiles[blockIdx.x];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, h = lane >> 5, j = lane & 31;
  const int st = wave * 2 + h;
  const int k0 = A.g_qptr[g], k1 = A.g_qptr[g + 1];
  double acc = 0;
  for (int k = k0 + st; k < k1; k += 8) acc += A.contrib[(int64_t)A.g_q[k] * T + j];
  part[st][j] = acc;
  __syncthreads();
  if (threadIdx.x < T) {
    const int64_t i = tile_row(A, g, j);
    if (i >= 0) {
      double c = 0;
      for (int q = 0; q < 8; ++q) c += part[q][j];
      A.bp[i] = (double)b[(int64_t)A.pos[i] * vs] - c;
    }
  }
}

// K2: y_I = sum_{J <= I} Dinv_s(I, J) bp_J
__global__ __launch_bounds__(256) void k_nd_diag(NdArgs A, const int32_t *tiles) {
  __shared__ NdSmem sm;
  const int g = tiles[blockIdx.x], s = A.t_sup[g], I = A.t_loc[g];
  const int a = A.s_a[s], n = A.s_n[s];
  const double *t0 = A.dinv + A.s_doff[s] + (int64_t)I * (I + 1) / 2 * T * T;
  const double r = wg_sum<true>(
      sm, I + 1, [&](int J) { return t0 + (int64_t)J * T * T; },
      [&](int J, int l) { return J * T + l < n ? A.bp[a + J * T + l] : 0.0; });
  const int lane = threadIdx.x;
  if (lane < T && I * T + lane < n) A.y[a + I * T + lane] = r;
}

// K3: contrib_q = B_q y_s (one workgroup per stored tile row)
__global__ __launch_bounds__(256) void k_nd_off(NdArgs A, const int32_t *items) {
  __shared__ NdSmem sm;
  const int q = items[blockIdx.x], s = A.q_sup[q];
  const int a = A.s_a[s], n = A.s_n[s], nt = (n + T - 1) / T;
  const double *t0 = A.bval + A.q_off[q];
  const double r = wg_sum<true>(
      sm, nt, [&](int J) { return t0 + (int64_t)J * T * T; },
      [&](int J, int l) { return J * T + l < n ? A.y[a + J * T + l] : 0.0; });
  if (threadIdx.x < T) A.contrib[(int64_t)q * T + threadIdx.x] = r;
}

// K4: t_J = sum over the stored tile rows q of s of B_q(J)^T x_(target q)
__global__ __launch_bounds__(256) void k_nd_off_t(NdArgs A, const int32_t *tiles) {
  __shared__ NdSmem sm;
  const int g = tiles[blockIdx.x], s = A.t_sup[g], J = A.t_loc[g];
  const int k0 = A.s_qptr[s], cnt = A.s_qptr[s + 1] - k0;
  const double r = wg_sum<false>(
      sm, cnt, [&](int k) { return A.bval + A.q_off[A.s_q[k0 + k]] + (int64_t)J * T * T; },
      [&](int k, int l) {
        const int64_t i = tile_row(A, A.q_tgt[A.s_q[k0 + k]], l);
        return i >= 0 ? A.x[i] : 0.0;
      });
  const int i = J * T + threadIdx.x;
  if (threadIdx.x < T && i < A.s_n[s]) A.t[A.s_a[s] + i] = r;
}

// K5: x_J = sum_{I >= J} Dinv_s(I, J)^T (y - t)_I, scattered to the caller's order
template <class TV>
__global__ __launch_bounds__(256) void k_nd_diag_t(NdArgs A, const int32_t *tiles, TV *u, int vs) {
  __shared__ NdSmem sm;
  const int g = tiles[blockIdx.x], s = A.t_sup[g], J = A.t_loc[g];
  const int a = A.s_a[s], n = A.s_n[s], nt = (n + T - 1) / T;
  const double *base = A.dinv + A.s_doff[s];
  const double r = wg_sum<false>(
      sm, nt - J, [&](int k) { const int I = J + k; return base + ((int64_t)I * (I + 1) / 2 + J) * T * T; },
      [&](int k, int l) {
        const int i = (J + k) * T + l;
        return i < n ? A.y[a + i] - A.t[a + i] : 0.0;
      });
  const int i = J * T + threadIdx.x;
  if (threadIdx.x < T && i < n) {
    A.x[a + i] = r;
    u[(int64_t)A.pos[a + i] * vs] = (TV)r;
  }
}

struct Sup {
  std::vector<int32_t> idx;  // unknowns
  int parent = -1, height = 0;
};

// nested dissection of the unknowns `V` (coordinates xyz, graph rp/col); the
// supernodes are appended in postorder; returns the index of the subtree's root
int dissect(std::vector<int32_t> V, const std::vector<double> &xyz, int dim, const std::vector<int64_t> &rp,
            const std::vector<int32_t> &col, std::vector<int> &side, int leaf, std::vector<Sup> &out) {
  if ((int)V.size() > leaf) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int32_t i : V)
      for (int d = 0; d < dim; ++d) {
        lo[d] = std::min(lo[d], xyz[(size_t)i * dim + d]);
        hi[d] = std::max(hi[d], xyz[(size_t)i * dim + d]);
      }
    int ax = 0;
    for (int d = 1; d < dim; ++d)
      if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
    std::stable_sort(V.begin(), V.end(), [&](int32_t p, int32_t q) {
      const double a = xyz[(size_t)p * dim + ax], b = xyz[(size_t)q * dim + ax];
      return a < b || (a == b && p < q);
    });
    const size_t half = V.size() / 2;
    for (size_t k = 0; k < V.size(); ++k) side[V[k]] = k < half ? 0 : 1;
    // boundary of each side in the matrix graph; the smaller one separates
    std::vector<int32_t> part[2], bnd[2];
    for (int32_t i : V) {
      bool b = false;
      for (int64_t e = rp[i]; e < rp[i + 1] && !b; ++e) {
        const int32_t j = col[e];
        b = side[j] >= 0 && side[j] != side[i];
      }
      (b ? bnd : part)[side[i]].push_back(i);
    }
    const int sep = bnd[0].size() <= bnd[1].size() ? 0 : 1;
    std::vector<int32_t> L = part[0], R = part[1];
    if (sep == 0) R.insert(R.end(), bnd[1].begin(), bnd[1].end());
    else L.insert(L.end(), bnd[0].begin(), bnd[0].end());
    std::vector<int32_t> S = bnd[sep];
    for (int32_t i : V) side[i] = -1;
    if (!L.empty() && !R.empty() && !S.empty()) {
      std::sort(L.begin(), L.end());
      std::sort(R.begin(), R.end());
      std::sort(S.begin(), S.end());
      for (int32_t i : L) side[i] = -1;
      const int l = dissect(L, xyz, dim, rp, col, side, leaf, out);
      const int r = dissect(R, xyz, dim, rp, col, side, leaf, out);
      Sup sp;
      sp.idx = std::move(S);
      sp.height = 1 + std::max(out[l].height, out[r].height);
      out.push_back(std::move(sp));
      const int me = (int)out.size() - 1;
      out[l].parent = me;
      out[r].parent = me;
      return me;
    }
  }
  Sup lf;
  lf.idx = std::move(V);
  std::sort(lf.idx.begin(), lf.idx.end());
  out.push_back(std::move(lf));
  return (int)out.size() - 1;
}

}  // namespace

void factor_coarsest_nd(Ctx &c, Level &L, int leaf) {
  hipStream_t s = c.stream;
  CoarseNd &N = L.cnd;
  const int64_t n = L.nfree;
  // graph and coordinates of the unknowns (the coarsest level's solve order is
  // its canonical order)
  std::vector<int64_t> rp;
  std::vector<int32_t> col, fdofs;
  std::vector<double> nodes;
  download(rp, L.A.rowptr.p, (size_t)n + 1, s);
  download(col, L.A.col.p, (size_t)L.A.nnz, s);
  download(fdofs, L.free_dofs.p, (size_t)L.nfree_s, s);
  download(nodes, L.nodes.p, (size_t)(L.ndofs * L.dim), s);
  std::vector<double> xyz((size_t)n * L.dim);
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < L.dim; ++d) xyz[(size_t)i * L.dim + d] = nodes[(size_t)fdofs[i / L.ncomp] * L.dim + d];
  std::vector<int32_t> all(n);
  std::iota(all.begin(), all.end(), 0);
  std::vector<int> side(n, -1);
  std::vector<Sup> sups;
  dissect(all, xyz, L.dim, rp, col, side, leaf, sups);
  const int ns = (int)sups.size();
  // the order: supernodes in postorder, each ascending
  std::vector<int32_t> pos, a(ns), sz(ns), t0(ns), q(n);
  for (int k = 0; k < ns; ++k) {
    a[k] = (int32_t)pos.size();
    sz[k] = (int32_t)sups[k].idx.size();
    pos.insert(pos.end(), sups[k].idx.begin(), sups[k].idx.end());
  }
  for (int64_t i = 0; i < n; ++i) q[pos[i]] = (int32_t)i;
  // global tiles
  std::vector<int32_t> t_sup, t_loc;
  for (int k = 0; k < ns; ++k) {
    t0[k] = (int32_t)t_sup.size();
    for (int l = 0; l < (sz[k] + T - 1) / T; ++l) {
      t_sup.push_back(k);
      t_loc.push_back(l);
    }
  }
  // dense factor of the permuted matrix and its inverse
  DBuf<double> M, W;
  M.alloc(n * n);
  fill<double>(s, M.p, n * n, 0.0);
  DBuf<int32_t> dq;
  upload(dq, q.data(), q.size(), s);
  k_dense_nd<<<(unsigned)n, 256, 0, s>>>(L.A.rowptr, L.A.col, L.A.val, dq, n, M);
  MG_LAUNCH_CHECK();
  DBuf<int> bad;
  bad.alloc(1);
  int init = 2147483647, hb = 0;
  MG_HIP(hipMemcpyAsync(bad.p, &init, sizeof(int), hipMemcpyHostToDevice, s));
  dense_cholesky(s, M, n, bad);
  MG_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  if (hb != 2147483647) fail(MG_ERR_NOT_SPD, "coarsest operator: non-positive pivot at row %d", hb);
  W.alloc(n * n);
  dense_lower_inverse(s, M, n, W);
  // diagonal-block inverses: lower tiles of W inside each supernode
  std::vector<int32_t> r0, nr, c0, nc;
  std::vector<int64_t> off, doff(ns);
  int64_t acc = 0;
  for (int k = 0; k < ns; ++k) {
    doff[k] = acc;
    const int nt = (sz[k] + T - 1) / T;
    for (int I = 0; I < nt; ++I)
      for (int J = 0; J <= I; ++J) {
        r0.push_back(a[k] + I * T);
        nr.push_back(std::min(T, sz[k] - I * T));
        c0.push_back(a[k] + J * T);
        nc.push_back(std::min(T, sz[k] - J * T));
        off.push_back(acc);
        acc += T * T;
      }
  }
  auto copy = [&](const double *src, DBuf<double> &dst, int64_t total) {
    dst.alloc(std::max<int64_t>(total, 1));
    if (r0.empty()) return;
    DBuf<int32_t> d0, d1, d2, d3;
    DBuf<int64_t> d4;
    upload(d0, r0.data(), r0.size(), s);
    upload(d1, nr.data(), nr.size(), s);
    upload(d2, c0.data(), c0.size(), s);
    upload(d3, nc.data(), nc.size(), s);
    upload(d4, off.data(), off.size(), s);
    k_copy_tiles<<<(unsigned)r0.size(), 256, 0, s>>>(src, n, d0, d1, d2, d3, d4, dst);
    MG_LAUNCH_CHECK();
    MG_HIP(hipStreamSynchronize(s));
  };
  copy(W.p, N.dinv, acc);
  W.release();
  N.dinv_bytes = acc * 8;
  // candidate tile rows below each supernode: every tile of every ancestor
  std::vector<int32_t> cs, cg;
  for (int k = 0; k < ns; ++k)
    for (int p = sups[k].parent; p >= 0; p = sups[p].parent)
      for (int l = 0; l < (sz[p] + T - 1) / T; ++l) {
        cs.push_back(k);
        cg.push_back(t0[p] + l);
      }
  std::vector<int> keep(cs.size(), 0);
  if (!cs.empty()) {
    r0.clear(); nr.clear(); c0.clear(); nc.clear();
    for (size_t k = 0; k < cs.size(); ++k) {
      const int g = cg[k], p = t_sup[g];
      r0.push_back(a[p] + t_loc[g] * T);
      nr.push_back(std::min(T, sz[p] - t_loc[g] * T));
      c0.push_back(a[cs[k]]);
      nc.push_back(sz[cs[k]]);
    }
    DBuf<int32_t> d0, d1, d2, d3;
    DBuf<int> flag;
    upload(d0, r0.data(), r0.size(), s);
    upload(d1, nr.data(), nr.size(), s);
    upload(d2, c0.data(), c0.size(), s);
    upload(d3, nc.data(), nc.size(), s);
    flag.alloc(cs.size());
    k_block_nonzero<<<(unsigned)cs.size(), 256, 0, s>>>(M, n, d0, d1, d2, d3, flag);
    MG_LAUNCH_CHECK();
    download(keep, flag.p, cs.size(), s);
  }
  // stored tile rows: item q = (supernode, target tile), its tiles J = 0..nt-1
  std::vector<int32_t> q_sup, q_tgt;
  std::vector<int64_t> q_off;
  r0.clear(); nr.clear(); c0.clear(); nc.clear(); off.clear();
  acc = 0;
  for (size_t k = 0; k < cs.size(); ++k) {
    if (!keep[k]) continue;
    const int sk = cs[k], g = cg[k], p = t_sup[g];
    q_sup.push_back(sk);
    q_tgt.push_back(g);
    q_off.push_back(acc);
    const int nt = (sz[sk] + T - 1) / T;
    for (int J = 0; J < nt; ++J) {
      r0.push_back(a[p] + t_loc[g] * T);
      nr.push_back(std::min(T, sz[p] - t_loc[g] * T));
      c0.push_back(a[sk] + J * T);
      nc.push_back(std::min(T, sz[sk] - J * T));
      off.push_back(acc);
      acc += T * T;
    }
  }
  copy(M.p, N.bval, acc);
  N.b_bytes = acc * 8;
  M.release();
  const int nq = (int)q_sup.size(), ng = (int)t_sup.size();
  // per supernode: its items; per target tile: items in ascending order
  std::vector<int32_t> s_qptr(ns + 1, 0), s_q, g_qptr(ng + 1, 0), g_q(nq);
  for (int k = 0; k < nq; ++k) s_qptr[q_sup[k] + 1]++;
  for (int k = 0; k < ns; ++k) s_qptr[k + 1] += s_qptr[k];
  s_q.resize(nq);
  {
    std::vector<int32_t> cur(s_qptr.begin(), s_qptr.end() - 1);
    for (int k = 0; k < nq; ++k) s_q[cur[q_sup[k]]++] = k;
  }
  for (int k = 0; k < nq; ++k) g_qptr[q_tgt[k] + 1]++;
  for (int g = 0; g < ng; ++g) g_qptr[g + 1] += g_qptr[g];
  {
    std::vector<int32_t> cur(g_qptr.begin(), g_qptr.end() - 1);
    for (int k = 0; k < nq; ++k) g_q[cur[q_tgt[k]]++] = k;
  }
  // schedule: tiles and items grouped by their supernode's height
  int H = 0;
  for (auto &sp : sups) H = std::max(H, sp.height);
  N.height = H;
  N.lvl_tiles_first.assign(H + 2, 0);
  N.lvl_items_first.assign(H + 2, 0);
  std::vector<int32_t> lt, li;
  for (int h = 0; h <= H; ++h) {
    N.lvl_tiles_first[h] = (int)lt.size();
    N.lvl_items_first[h] = (int)li.size();
    for (int g = 0; g < ng; ++g)
      if (sups[t_sup[g]].height == h) lt.push_back(g);
    for (int k = 0; k < nq; ++k)
      if (sups[q_sup[k]].height == h) li.push_back(k);
  }
  N.lvl_tiles_first[H + 1] = (int)lt.size();
  N.lvl_items_first[H + 1] = (int)li.size();
  upload(N.pos, pos.data(), pos.size(), s);
  upload(N.t_sup, t_sup.data(), t_sup.size(), s);
  upload(N.t_loc, t_loc.data(), t_loc.size(), s);
  upload(N.s_a, a.data(), a.size(), s);
  upload(N.s_n, sz.data(), sz.size(), s);
  upload(N.s_t0, t0.data(), t0.size(), s);
  upload(N.s_doff, doff.data(), doff.size(), s);
  std::vector<int32_t> one = {0};
  upload(N.q_sup, nq ? q_sup.data() : one.data(), std::max(nq, 1), s);
  upload(N.q_tgt, nq ? q_tgt.data() : one.data(), std::max(nq, 1), s);
  std::vector<int64_t> one64 = {0};
  upload(N.q_off, nq ? q_off.data() : one64.data(), std::max(nq, 1), s);
  upload(N.s_qptr, s_qptr.data(), s_qptr.size(), s);
  upload(N.s_q, nq ? s_q.data() : one.data(), std::max(nq, 1), s);
  upload(N.g_qptr, g_qptr.data(), g_qptr.size(), s);
  upload(N.g_q, nq ? g_q.data() : one.data(), std::max(nq, 1), s);
  upload(N.lvl_tiles, lt.data(), lt.size(), s);
  upload(N.lvl_items, li.empty() ? one.data() : li.data(), std::max<size_t>(li.size(), 1), s);
  N.bp.alloc(n);
  N.y.alloc(n);
  N.t.alloc(n);
  N.x.alloc(n);
  N.contrib.alloc((int64_t)std::max(nq, 1) * T);
  N.nsup = ns;
  N.leaf = leaf;
  N.on = true;
  MG_HIP(hipStreamSynchronize(s));
}

template <class TV>
void coarse_apply_nd(hipStream_t s, const Level &L, const TV *b, TV *u, int vs) {
  const CoarseNd &N = L.cnd;
  NdArgs A{N.t_sup, N.t_loc, N.s_a, N.s_n, N.s_t0, N.s_doff, N.dinv, N.q_sup, N.q_tgt, N.q_off, N.bval,
           N.s_qptr, N.s_q, N.g_qptr, N.g_q, N.pos, N.bp, N.y, N.t, N.x, N.contrib};
  for (int h = 0; h <= N.height; ++h) {
    const int t0 = N.lvl_tiles_first[h], tc = N.lvl_tiles_first[h + 1] - t0;
    const int i0 = N.lvl_items_first[h], ic = N.lvl_items_first[h + 1] - i0;
    if (tc > 0) {
      k_nd_gather<TV><<<(unsigned)tc, 256, 0, s>>>(A, N.lvl_tiles.p + t0, b, vs);
      MG_LAUNCH_CHECK();
      k_nd_diag<<<(unsigned)tc, 256, 0, s>>>(A, N.lvl_tiles.p + t0);
      MG_LAUNCH_CHECK();
    }
    if (ic > 0) {
      k_nd_off<<<(unsigned)ic, 256, 0, s>>>(A, N.lvl_items.p + i0);
      MG_LAUNCH_CHECK();
    }
  }
  for (int h = N.height; h >= 0; --h) {
    const int t0 = N.lvl_tiles_first[h], tc = N.lvl_tiles_first[h + 1] - t0;
    if (tc == 0) continue;
    k_nd_off_t<<<(unsigned)tc, 256, 0, s>>>(A, N.lvl_tiles.p + t0);
    MG_LAUNCH_CHECK();
    k_nd_diag_t<TV><<<(unsigned)tc, 256, 0, s>>>(A, N.lvl_tiles.p + t0, u, vs);
    MG_LAUNCH_CHECK();
  }
}
template void coarse_apply_nd<double>(hipStream_t, const Level &, const double *, double *, int);
template void coarse_apply_nd<float>(hipStream_t, const Level &, const float *, float *, int);

}  // namespace mg
