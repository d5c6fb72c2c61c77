// Matrix-core tile products shared by the dense factorisations: a wavefront
// computes one 32 x 32 output tile as 2 x 2 blocks of 16 x 16 x 4 MFMA steps
// (v_mfma_f64_16x16x4 in FP64, v_mfma_f32_16x16x4 in FP32, FP32 accumulate),
// with its operands read straight from memory into the register layout the
// instruction expects.  Both instructions take operand A as lane l holding
// (row l % 16, k l / 16) and operand B as (k l / 16, column l % 16); their
// result layouts differ (checked on the device): in FP64 lane l holds rows
// l / 16 + 4 e, e = 0..3, of column l % 16, in FP32 rows 4 (l / 16) + e.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace mg {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// MFMA operand registers of one 32 x 32 tile, read straight from the n x n
// row-major matrix M: element (x, y) of the operand is M[r0 + x][c0 + y], or
// M[r0 + y][c0 + x] when swap is set (zero outside the matrix).  For the A
// operand lane l holds (x, y) = (16 blk + l % 16, 4 s + l / 16), for the B
// operand (4 s + l / 16, 16 blk + l % 16); o[blk * 8 + s].  I: the type of
// the element offsets (int32_t where n^2 < 2^31: half the address registers).
template <bool ROLE_A, class I = int64_t, class T>
__device__ inline void fetch_ops(const T *M, int n, int r0, int c0, bool swap, T o[16], int lane) {
  const int p = lane & 15, q = lane >> 4;
#pragma unroll
  for (int blk = 0; blk < 2; ++blk)
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int x = ROLE_A ? 16 * blk + p : 4 * s + q;
      const int y = ROLE_A ? 4 * s + q : 16 * blk + p;
      const int r = swap ? r0 + y : r0 + x, c = swap ? c0 + x : c0 + y;
      o[blk * 8 + s] = (r < n && c < n) ? M[(I)r * n + c] : (T)0;
    }
}

// acc (a 32 x 32 tile as 2 x 2 MFMA blocks) += A B
__device__ inline void mma_ops(v4d acc[2][2], const double a[16], const double b[16]) {
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[8 + s], acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[8 + s], b[s], acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[8 + s], b[8 + s], acc[1][1], 0, 0, 0);
  }
}
__device__ inline void mma_ops(v4f acc[2][2], const float a[16], const float b[16]) {
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[8 + s], acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[8 + s], b[s], acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[8 + s], b[8 + s], acc[1][1], 0, 0, 0);
  }
}

__device__ inline void zero_acc(v4d acc[2][2]) {
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
}
__device__ inline void zero_acc(v4f acc[2][2]) {
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
}

// f(i, j, v) for the elements (i, j) of the tile held by this lane
template <class F>
__device__ inline void for_acc(v4d acc[2][2], int lane, F f) {
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 4; ++e) f(16 * a + (lane >> 4) + 4 * e, 16 * b + (lane & 15), acc[a][b][e]);
}
template <class F>
__device__ inline void for_acc(v4f acc[2][2], int lane, F f) {
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 4; ++e) f(16 * a + 4 * (lane >> 4) + e, 16 * b + (lane & 15), acc[a][b][e]);
}

// acc = the 32 x 32 tile M[r0 + i][c0 + j] of the n x n row-major matrix M
// (zero outside it), in the accumulator layout of for_acc, so that a product
// can accumulate onto it (C - A B as C + (-A) B: one round trip to memory
// for the tile instead of a read after the products)
__device__ inline int acc_row(const v4d *, int a, int lane, int e) { return 16 * a + (lane >> 4) + 4 * e; }
__device__ inline int acc_row(const v4f *, int a, int lane, int e) { return 16 * a + 4 * (lane >> 4) + e; }
template <class I = int64_t, class V, class T>
__device__ inline void load_acc(V acc[2][2], const T *M, int n, int r0, int c0, int lane) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = r0 + acc_row(&acc[0][0], a, lane, e), c = c0 + 16 * b + (lane & 15);
        acc[a][b][e] = (r < n && c < n) ? M[(I)r * n + c] : (T)0;
      }
}

template <class T>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
  using type = v4d;
};
template <>
struct MfmaAcc<float> {
  using type = v4f;
};

}  // namespace mg
