// Galerkin coarse operators A_(l+1) = P_l^T A_l P_l (paper Sec. 2) as two
// row-wise sparse products C = A B on the GPU: AP = A P, then A_c = R (AP) with
// R = P^T.
//
// One wavefront per output row keeps a hash table of the row's columns in LDS.
// The row of A is walked in CSR order; for each entry a_ik the lanes add
// a_ik * b_kj for the distinct columns j of row k of B.  Every sum c_ij is thus
// accumulated in increasing k, so the result is deterministic.  A symbolic
// pass counts the columns of every row, a numeric pass writes the sorted row.
#include "devutil.h"

namespace mg {

// Hash tables of HT slots accept rows of up to 3 HT / 4 distinct columns.  Rows
// are first tried with a 1024-slot table; rows that overflow it are redone with
// a 4096-slot table (3D P2 Galerkin rows reach several hundred columns).
template <int HT>
__device__ inline int hash_slot(int key) {
  return (int)(((uint32_t)key * 2654435761u) >> 16) & (HT - 1);
}

template <int HT>
__device__ inline int ht_insert(int *keys, int key, bool &fresh) {
  int h = hash_slot<HT>(key);
  fresh = false;
  for (int probe = 0; probe < HT; ++probe) {
    int old = atomicCAS(&keys[h], -1, key);
    if (old == -1) { fresh = true; return h; }
    if (old == key) return h;
    h = (h + 1) & (HT - 1);
  }
  return -1;
}

// cnt[row] = distinct columns of row, or -1 if the row does not fit
template <int HT>
__global__ __launch_bounds__(64) void k_spgemm_count(const int64_t *arp, const int32_t *acol, const int64_t *brp,
                                                     const int32_t *bcol, int64_t nrows, const int32_t *rows,
                                                     int64_t *cnt) {
  constexpr int MAXF = 3 * HT / 4;
  __shared__ int keys[HT];
  __shared__ int n_new;
  int64_t row = rows ? rows[blockIdx.x] : (int64_t)blockIdx.x;
  if (row >= nrows) return;
  int lane = threadIdx.x;
  for (int h = lane; h < HT; h += 64) keys[h] = -1;
  if (lane == 0) n_new = 0;
  __syncthreads();
  bool full = false;
  for (int64_t ka = arp[row]; ka < arp[row + 1]; ++ka) {
    int k = acol[ka];
    for (int64_t kb = brp[k] + lane; kb < brp[k + 1]; kb += 64) {
      bool fresh;
      int slot = ht_insert<HT>(keys, bcol[kb], fresh);
      if (slot < 0) full = true;
      if (fresh) atomicAdd(&n_new, 1);
    }
    __syncthreads();
    if (n_new > MAXF) full = true;
    if (__syncthreads_or(full)) break;
  }
  if (lane == 0) cnt[row] = (full || n_new > MAXF) ? -1 : n_new;
}

template <int HT>
__global__ __launch_bounds__(64) void k_spgemm_fill(const int64_t *arp, const int32_t *acol, const double *aval,
                                                    const int64_t *brp, const int32_t *bcol, const double *bval,
                                                    int64_t nrows, const int32_t *rows, const int64_t *crp,
                                                    int32_t *ccol, double *cval) {
  constexpr int MAXF = 3 * HT / 4;
  __shared__ int keys[HT];
  __shared__ double vals[HT];
  __shared__ int ckey[MAXF];
  __shared__ double cv[MAXF];
  __shared__ int ncomp;
  int64_t row = rows ? rows[blockIdx.x] : (int64_t)blockIdx.x;
  if (row >= nrows) return;
  int64_t base = crp[row];
  if (!rows && crp[row + 1] - base > MAXF) return;  // redone with the larger table
  int lane = threadIdx.x;
  for (int h = lane; h < HT; h += 64) {
    keys[h] = -1;
    vals[h] = 0.0;
  }
  if (lane == 0) ncomp = 0;
  __syncthreads();
  for (int64_t ka = arp[row]; ka < arp[row + 1]; ++ka) {
    int k = acol[ka];
    double a = aval[ka];
    for (int64_t kb = brp[k] + lane; kb < brp[k + 1]; kb += 64) {
      bool fresh;
      int slot = ht_insert<HT>(keys, bcol[kb], fresh);
      if (slot >= 0) vals[slot] += a * bval[kb];
    }
    __syncthreads();
  }
  for (int h = lane; h < HT; h += 64) {
    if (keys[h] >= 0) {
      int p = atomicAdd(&ncomp, 1);
      if (p < MAXF) {
        ckey[p] = keys[h];
        cv[p] = vals[h];
      }
    }
  }
  __syncthreads();
  int n = ncomp < MAXF ? ncomp : MAXF;
  for (int e = lane; e < n; e += 64) {
    int key = ckey[e], rank = 0;
    for (int f = 0; f < n; ++f) rank += ckey[f] < key ? 1 : 0;
    ccol[base + rank] = key;
    cval[base + rank] = cv[e];
  }
}

void spgemm(Ctx &c, const Csr &A, const Csr &B, Csr &C) {
  hipStream_t s = c.stream;
  constexpr int SMALL = 1024, LARGE = 4096;
  if (A.ncols != B.nrows) fail(MG_ERR_ARG, "spgemm shape mismatch");
  if (A.nrows > 2147483647LL) fail(MG_ERR_LIMIT, "spgemm: too many rows");
  C.nrows = A.nrows;
  C.ncols = B.ncols;
  DBuf<int64_t> cnt;
  cnt.alloc(A.nrows);
  k_spgemm_count<SMALL><<<(unsigned)A.nrows, 64, 0, s>>>(A.rowptr, A.col, B.rowptr, B.col, A.nrows, nullptr, cnt);
  MG_LAUNCH_CHECK();
  std::vector<int64_t> hc;
  download(hc, cnt.p, (size_t)A.nrows, s);
  std::vector<int32_t> big;
  for (int64_t r = 0; r < A.nrows; ++r)
    if (hc[r] < 0) big.push_back((int32_t)r);
  DBuf<int32_t> dbig;
  if (!big.empty()) {
    upload(dbig, big.data(), big.size(), s);
    k_spgemm_count<LARGE><<<(unsigned)big.size(), 64, 0, s>>>(A.rowptr, A.col, B.rowptr, B.col, A.nrows, dbig, cnt);
    MG_LAUNCH_CHECK();
    std::vector<int64_t> hb;
    download(hb, cnt.p, (size_t)A.nrows, s);
    for (int32_t r : big)
      if (hb[r] < 0) fail(MG_ERR_LIMIT, "Galerkin product: coarse row %d has more than %d nonzeros", r, 3 * LARGE / 4);
  }
  C.rowptr.alloc(A.nrows + 1);
  C.nnz = exclusive_scan(s, cnt.p, C.rowptr.p, A.nrows);
  MG_HIP(hipMemcpyAsync(C.rowptr.p + A.nrows, &C.nnz, sizeof(int64_t), hipMemcpyHostToDevice, s));
  C.col.alloc(C.nnz);
  C.val.alloc(C.nnz);
  k_spgemm_fill<SMALL><<<(unsigned)A.nrows, 64, 0, s>>>(A.rowptr, A.col, A.val, B.rowptr, B.col, B.val, A.nrows,
                                                        nullptr, C.rowptr, C.col, C.val);
  MG_LAUNCH_CHECK();
  if (!big.empty()) {
    k_spgemm_fill<LARGE><<<(unsigned)big.size(), 64, 0, s>>>(A.rowptr, A.col, A.val, B.rowptr, B.col, B.val,
                                                             A.nrows, dbig, C.rowptr, C.col, C.val);
    MG_LAUNCH_CHECK();
  }
  MG_HIP(hipStreamSynchronize(s));
}

void galerkin_product(Ctx &c, Level &F, Level &C) {
  Csr AP;
  spgemm(c, F.A, F.Pc, AP);
  spgemm(c, F.Rc, AP, C.A);
  drop_cancelled(c, C.A);
}

}  // namespace mg
