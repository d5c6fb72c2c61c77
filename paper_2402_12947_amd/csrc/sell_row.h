// Device helpers shared by the single-vector and the block (several
// right-hand sides) solve kernels: SELL-C row products, the wavefront LDS
// ordering and the deterministic block reduction.
#pragma once

#include "mg_internal.h"

namespace mg {

// Column arrays of a SELL matrix as the solve kernels read them.
struct SellCols {
  const int64_t *sptr;
  const int32_t *col;
  const uint16_t *col16;
  const int32_t *cbase;
  const int32_t *ctab;
  const uint16_t *rlen;
  const int32_t *smin;
  int rpl;
};
static inline SellCols cols_of(const Sell &S) {
  return {S.slice_ptr.p, S.col.p, S.col16.p, S.cbase.p, S.ctab.p, S.rlen.p, S.smin.p, S.rpl};
}

// Row of SELL position pos (64 positions per slice, rpl lanes per row) and
// whether this lane stores the row's result (the first of its lanes).
struct SellRow {
  int64_t row;
  bool lead;
};
__device__ inline SellRow sell_row_of(const SellCols &S, int64_t pos) {
  const int rpl = S.rpl;
  if (rpl == 1) return {pos, true};
  const int lane = (int)(pos & 63);
  return {(pos >> 6) * (64 / rpl) + lane / rpl, (lane & (rpl - 1)) == 0};
}

// Row `lane` of slice `sl` (sl is the same for the whole wavefront): the matrix
// entries are streamed once per product, so they are loaded non-temporally and
// leave the cache to the gathered vector; slices whose columns fit two windows
// of 32768 read 16-bit columns.  The slice is walked in rounds of U entries
// (U gathers in flight per lane): rounds inside every row of the slice (below
// the slice's shortest row, wmin) load all entries; the later rounds load
// values and gather only up to each lane's own row length `len`, so the
// padding at the end of the shorter rows costs no value traffic wherever a
// whole cache line of it is padding (the sorted layouts order the rows of a
// slice by length).  With len = wmin = w every stored entry is used (padding
// values are zero).  Entry j of the lane's share of its row goes to
// accumulator j mod U and the accumulators are summed pairwise, an order that
// depends only on the row and the lanes per row, so both variants round
// identically.
template <int U, class T, class C, class F>
__device__ inline T sell_dot(const C *__restrict__ cp, const T *__restrict__ vp, const T *__restrict__ x, int w,
                             int wmin, int len, F decode) {
  T a[U];
#pragma unroll
  for (int u = 0; u < U; ++u) a[u] = 0;
  int j = 0;
  for (; j + U <= wmin; j += U) {
    C cr[U];
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cr[u] = __builtin_nontemporal_load(cp + (j + u) * 64);
      v[u] = __builtin_nontemporal_load(vp + (j + u) * 64);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] += v[u] * x[decode(cr[u])];
  }
  for (; j < w; j += U) {
    // all loads of the round are issued before the first use: the columns
    // (past the slice width the last one again, which keeps every lane in
    // the decode, as it may read across lanes), then the values and the
    // gathers of the lane's own entries (zero beyond them)
    C cr[U];
    T v[U], g[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cr[u] = __builtin_nontemporal_load(cp + (j + u < w ? j + u : w - 1) * 64);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = 0;
      if (j + u < len) v[u] = __builtin_nontemporal_load(vp + (j + u) * 64);
    }
    int c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) c[u] = decode(cr[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      g[u] = 0;
      if (j + u < len) g[u] = x[c[u]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] += v[u] * g[u];
  }
  T s = (a[0] + a[1]) + (a[2] + a[3]);
  if constexpr (U >= 8) s += (a[4] + a[5]) + (a[6] + a[7]);
  if constexpr (U == 16) s += ((a[8] + a[9]) + (a[10] + a[11])) + ((a[12] + a[13]) + (a[14] + a[15]));
  return s;
}

// MASK: the rounds past the slice's shortest row skip each lane's padding
// (row lengths read per lane); otherwise every stored entry is used.  Both
// give bitwise the same result; which one is faster depends on the padding.
// With rpl lanes per row the lanes' partial sums are added by a butterfly,
// which leaves the same row product in every lane of the row.
template <class T, int U, bool MASK>
__device__ inline T sell_lane(const SellCols &S, const T *__restrict__ val, const T *__restrict__ x, int s32,
                              int lane) {
  const int64_t base = S.sptr[s32];
  const int w = (int)((S.sptr[s32 + 1] - base) >> 6);
  const T *vp = val + base + lane;
  const int wmin = MASK ? S.smin[s32] : w;
  const int len = MASK ? (int)S.rlen[64 * (int64_t)s32 + lane] : w;
  const int b0 = S.cbase[2 * s32];
  if (b0 >= 0) {
    const int bh = S.cbase[2 * s32 + 1] - 0x8000;
    return sell_dot<U>(S.col16 + base + lane, vp, x, w, wmin, len,
                       [=](uint16_t c) { return ((c & 0x8000) ? bh : b0) + (int)c; });
  }
  if (b0 < -1) {
    // window bases in lanes 0..15, picked per entry by a cross-lane read
    const int tb = S.ctab[16 * (int64_t)s32 + (lane & 15)];
    const int shift = b0 == -2 ? 13 : 12;
    const int mask = (1 << shift) - 1;
    return sell_dot<U>(S.col16 + base + lane, vp, x, w, wmin, len,
                       [=](uint16_t c) { return __shfl(tb, (int)c >> shift) + ((int)c & mask); });
  }
  return sell_dot<U>(S.col + base + lane, vp, x, w, wmin, len, [](int32_t c) { return (int)c; });
}

template <class T, int U = 8, bool MASK = false>
__device__ inline T sell_row(const SellCols &S, const T *__restrict__ val, const T *__restrict__ x, int64_t sl,
                             int lane) {
  static_assert(U == 4 || U == 8 || U == 16, "4, 8 or 16 gathers in flight");
  const int s32 = __builtin_amdgcn_readfirstlane((int)sl);
  T r = sell_lane<T, U, MASK>(S, val, x, s32, lane);
  for (int m = 1; m < S.rpl; m <<= 1) r += __shfl_xor(r, m);
  return r;
}

// the value array of the cycle's precision
template <class T>
static inline const T *sell_vals(const Sell &S) {
  if constexpr (std::is_same<T, double>::value) return S.v64.p;
  else return S.v32.p;
}

static inline unsigned sell_grid(const Sell &S) { return (unsigned)((S.nslices * 64 + 255) / 256); }

// K values of one unknown in a block vector: the K right-hand sides of a
// block solve are interleaved, unknown i holding entries i K .. i K + K - 1,
// so one gather fetches all K columns (8 to 32 bytes).
template <class T, int K>
struct alignas(sizeof(T) * K) BlockRow {
  T v[K];
};

// Row `lane` of a slice times K interleaved vectors: every matrix entry is
// read once and used K times.  U gathers in flight per lane (4 when a gather
// is 32 bytes, to bound the registers of the K U accumulators); rounds, value
// loads up to the row length and the order of the sums as in sell_dot.
template <int U, int K, class T, class C, class F>
__device__ inline void sell_dot_k(const C *__restrict__ cp, const T *__restrict__ vp, const T *__restrict__ x, int w,
                                  int wmin, int len, F decode, T (&out)[K]) {
  using R = BlockRow<T, K>;
  const R *__restrict__ xr = reinterpret_cast<const R *>(x);
  T a[U][K];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int q = 0; q < K; ++q) a[u][q] = 0;
  int j = 0;
  for (; j + U <= wmin; j += U) {
    C cr[U];
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cr[u] = __builtin_nontemporal_load(cp + (j + u) * 64);
      v[u] = __builtin_nontemporal_load(vp + (j + u) * 64);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const R xv = xr[decode(cr[u])];
#pragma unroll
      for (int q = 0; q < K; ++q) a[u][q] += v[u] * xv.v[q];
    }
  }
  for (; j < w; j += U) {
    C cr[U];
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cr[u] = __builtin_nontemporal_load(cp + (j + u < w ? j + u : w - 1) * 64);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = 0;
      if (j + u < len) v[u] = __builtin_nontemporal_load(vp + (j + u) * 64);
    }
    int c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) c[u] = decode(cr[u]);
    R g[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int q = 0; q < K; ++q) g[u].v[q] = 0;
      if (j + u < len) g[u] = xr[c[u]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < K; ++q) a[u][q] += v[u] * g[u].v[q];
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
    T s = (a[0][q] + a[1][q]) + (a[2][q] + a[3][q]);
    if constexpr (U == 8) s += (a[4][q] + a[5][q]) + (a[6][q] + a[7][q]);
    out[q] = s;
  }
}

template <class T, int K>
__device__ inline void sell_lane_k(const SellCols &S, const T *__restrict__ val, const T *__restrict__ x, int s32,
                                   int lane, T (&out)[K]) {
  constexpr int U = sizeof(T) * K > 16 ? 4 : 8;
  const int64_t base = S.sptr[s32];
  const int w = (int)((S.sptr[s32 + 1] - base) >> 6);
  const T *vp = val + base + lane;
  const int wmin = S.smin[s32];
  const int len = S.rlen[64 * (int64_t)s32 + lane];
  const int b0 = S.cbase[2 * s32];
  if (b0 >= 0) {
    const int bh = S.cbase[2 * s32 + 1] - 0x8000;
    sell_dot_k<U, K>(S.col16 + base + lane, vp, x, w, wmin, len,
                     [=](uint16_t c) { return ((c & 0x8000) ? bh : b0) + (int)c; }, out);
  } else if (b0 < -1) {
    const int tb = S.ctab[16 * (int64_t)s32 + (lane & 15)];
    const int shift = b0 == -2 ? 13 : 12;
    const int mask = (1 << shift) - 1;
    sell_dot_k<U, K>(S.col16 + base + lane, vp, x, w, wmin, len,
                     [=](uint16_t c) { return __shfl(tb, (int)c >> shift) + ((int)c & mask); }, out);
  } else {
    sell_dot_k<U, K>(S.col + base + lane, vp, x, w, wmin, len, [](int32_t c) { return (int)c; }, out);
  }
}

template <class T, int K>
__device__ inline void sell_row_k(const SellCols &S, const T *__restrict__ val, const T *__restrict__ x, int64_t sl,
                                  int lane, T (&out)[K]) {
  const int s32 = __builtin_amdgcn_readfirstlane((int)sl);
  sell_lane_k<T, K>(S, val, x, s32, lane, out);
  for (int m = 1; m < S.rpl; m <<= 1)
#pragma unroll
    for (int q = 0; q < K; ++q) out[q] += __shfl_xor(out[q], m);
}

// Orders this wavefront's LDS accesses (writes before reads of other lanes).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double block_sum(double v) {
  __shared__ double red[256];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

}  // namespace mg
