// Device-wide primitives (hipCUB radix sort, run-length encoding, scans) and
// small helpers shared by the setup kernels.
#pragma once

#include <hipcub/hipcub.hpp>

#include "mg_internal.h"

namespace mg {

inline int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 2147483647LL) fail(MG_ERR_LIMIT, "grid of %lld blocks too large", (long long)g);
  return (int)g;
}

inline void check_items(int64_t n, const char *what) {
  if (n > 2147483647LL) fail(MG_ERR_LIMIT, "%s: %lld items exceed the 2^31 limit", what, (long long)n);
}

template <class K>
void sort_keys(hipStream_t s, const K *in, K *out, int64_t n, int end_bit) {
  check_items(n, "sort_keys");
  if (n == 0) return;
  size_t tmp = 0;
  MG_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, tmp, in, out, (int)n, 0, end_bit, s));
  DBuf<char> t;
  t.alloc(tmp);
  MG_HIP(hipcub::DeviceRadixSort::SortKeys(t.p, tmp, in, out, (int)n, 0, end_bit, s));
  MG_HIP(hipStreamSynchronize(s));
}

template <class K, class V>
void sort_pairs(hipStream_t s, const K *kin, K *kout, const V *vin, V *vout, int64_t n, int end_bit) {
  check_items(n, "sort_pairs");
  if (n == 0) return;
  size_t tmp = 0;
  MG_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, kin, kout, vin, vout, (int)n, 0, end_bit, s));
  DBuf<char> t;
  t.alloc(tmp);
  MG_HIP(hipcub::DeviceRadixSort::SortPairs(t.p, tmp, kin, kout, vin, vout, (int)n, 0, end_bit, s));
  MG_HIP(hipStreamSynchronize(s));
}

// Unique keys of a sorted array with their run lengths; returns the number of runs.
template <class K>
int64_t run_length(hipStream_t s, const K *in, K *uniq, int32_t *len, int64_t n) {
  check_items(n, "run_length");
  if (n == 0) return 0;
  DBuf<int32_t> nr;
  nr.alloc(1);
  size_t tmp = 0;
  MG_HIP(hipcub::DeviceRunLengthEncode::Encode(nullptr, tmp, in, uniq, len, nr.p, (int)n, s));
  DBuf<char> t;
  t.alloc(tmp);
  MG_HIP(hipcub::DeviceRunLengthEncode::Encode(t.p, tmp, in, uniq, len, nr.p, (int)n, s));
  int32_t h = 0;
  MG_HIP(hipMemcpyAsync(&h, nr.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  return h;
}

// out[i] = sum_{k<i} in[k]; returns the total (in[n-1] + out[n-1]).
template <class T, class U>
U exclusive_scan(hipStream_t s, const T *in, U *out, int64_t n) {
  check_items(n, "exclusive_scan");
  if (n == 0) return U(0);
  size_t tmp = 0;
  MG_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, in, out, (int)n, s));
  DBuf<char> t;
  t.alloc(tmp);
  MG_HIP(hipcub::DeviceScan::ExclusiveSum(t.p, tmp, in, out, (int)n, s));
  T last_in;
  U last_out;
  MG_HIP(hipMemcpyAsync(&last_in, in + n - 1, sizeof(T), hipMemcpyDeviceToHost, s));
  MG_HIP(hipMemcpyAsync(&last_out, out + n - 1, sizeof(U), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  return last_out + (U)last_in;
}

inline int bits_for(uint64_t maxval) {
  int b = 1;
  while (b < 64 && (maxval >> b) != 0) ++b;
  return b;
}

template <class K>
__device__ inline int64_t lower_bound_dev(const K *a, int64_t n, K key) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

}  // namespace mg
