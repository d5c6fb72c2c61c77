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

constexpr int HT = 1024;          // hash slots per row
constexpr int HT_MAX_FILL = 768;  // rows with more distinct columns are rejected

__device__ inline int hash_slot(int key) { return (int)(((uint32_t)key * 2654435761u) >> 22) & (HT - 1); }

// insert key; returns slot or -1 when the table is full
__device__ inline int ht_insert(int *keys, int key, bool &fresh) {
  int h = hash_slot(key);
  fresh = false;
  for (int probe = 0; probe < HT; ++probe) {
    int old = atomicCAS(&keys[h], -1, key);
    if (old == -1) { fresh = true; return h; }
    if (old == key) return h;
    h = (h + 1) & (HT - 1);
  }
  return -1;
}

__global__ __launch_bounds__(64) void k_spgemm_count(const int64_t *arp, const int32_t *acol, const int64_t *brp,
                                                     const int32_t *bcol, int64_t nrows, int64_t *cnt, int *overflow) {
  __shared__ int keys[HT];
  __shared__ int n_new;
  int64_t row = blockIdx.x;
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
      int slot = ht_insert(keys, bcol[kb], fresh);
      if (slot < 0) full = true;
      if (fresh) atomicAdd(&n_new, 1);
    }
    __syncthreads();
    if (n_new > HT_MAX_FILL) full = true;
    if (__syncthreads_or(full)) break;
  }
  if (lane == 0) {
    cnt[row] = n_new;
    if (n_new > HT_MAX_FILL || full) atomicMax(overflow, 1);
  }
}

__global__ __launch_bounds__(64) void k_spgemm_fill(const int64_t *arp, const int32_t *acol, const double *aval,
                                                    const int64_t *brp, const int32_t *bcol, const double *bval,
                                                    int64_t nrows, const int64_t *crp, int32_t *ccol, double *cval) {
  __shared__ int keys[HT];
  __shared__ double vals[HT];
  __shared__ int ckey[HT_MAX_FILL];
  __shared__ double cv[HT_MAX_FILL];
  __shared__ int ncomp;
  int64_t row = blockIdx.x;
  if (row >= nrows) return;
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
      int slot = ht_insert(keys, bcol[kb], fresh);
      if (slot >= 0) vals[slot] += a * bval[kb];
    }
    __syncthreads();
  }
  for (int h = lane; h < HT; h += 64) {
    if (keys[h] >= 0) {
      int p = atomicAdd(&ncomp, 1);
      if (p < HT_MAX_FILL) {
        ckey[p] = keys[h];
        cv[p] = vals[h];
      }
    }
  }
  __syncthreads();
  int n = ncomp < HT_MAX_FILL ? ncomp : HT_MAX_FILL;
  int64_t base = crp[row];
  for (int e = lane; e < n; e += 64) {
    int key = ckey[e], rank = 0;
    for (int f = 0; f < n; ++f) rank += ckey[f] < key ? 1 : 0;
    ccol[base + rank] = key;
    cval[base + rank] = cv[e];
  }
}

void spgemm(Ctx &c, const Csr &A, const Csr &B, Csr &C) {
  hipStream_t s = c.stream;
  if (A.ncols != B.nrows) fail(MG_ERR_ARG, "spgemm shape mismatch");
  if (A.nrows > 2147483647LL) fail(MG_ERR_LIMIT, "spgemm: too many rows");
  C.nrows = A.nrows;
  C.ncols = B.ncols;
  DBuf<int64_t> cnt;
  DBuf<int> ovf;
  cnt.alloc(A.nrows);
  ovf.alloc(1);
  MG_HIP(hipMemsetAsync(ovf.p, 0, sizeof(int), s));
  k_spgemm_count<<<(unsigned)A.nrows, 64, 0, s>>>(A.rowptr, A.col, B.rowptr, B.col, A.nrows, cnt, ovf);
  MG_LAUNCH_CHECK();
  int hovf = 0;
  MG_HIP(hipMemcpyAsync(&hovf, ovf.p, sizeof(int), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  if (hovf) fail(MG_ERR_LIMIT, "Galerkin product: a coarse row has more than %d nonzeros", HT_MAX_FILL);
  C.rowptr.alloc(A.nrows + 1);
  C.nnz = exclusive_scan(s, cnt.p, C.rowptr.p, A.nrows);
  MG_HIP(hipMemcpyAsync(C.rowptr.p + A.nrows, &C.nnz, sizeof(int64_t), hipMemcpyHostToDevice, s));
  C.col.alloc(C.nnz);
  C.val.alloc(C.nnz);
  k_spgemm_fill<<<(unsigned)A.nrows, 64, 0, s>>>(A.rowptr, A.col, A.val, B.rowptr, B.col, B.val, A.nrows,
                                                 C.rowptr, C.col, C.val);
  MG_LAUNCH_CHECK();
  MG_HIP(hipStreamSynchronize(s));
}

void galerkin_product(Ctx &c, Level &F, Level &C) {
  Csr AP;
  spgemm(c, F.A, F.Pc, AP);
  spgemm(c, F.Rc, AP, C.A);
}

}  // namespace mg
