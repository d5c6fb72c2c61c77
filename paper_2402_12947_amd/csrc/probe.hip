// Streaming-bandwidth probes: what plain streams reach on this GPU, as the
// practical ceilings next to the datasheet peak for the solve kernels (pure
// read; copy; seven read streams and one write stream, the read/write mix of
// the Chebyshev step).  One pass per element, 16-byte accesses, non-temporal.
#include <chrono>

#include "mg_internal.h"

namespace mg {

typedef double f64x2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void k_probe_read(const f64x2 *__restrict__ a, int64_t n, double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const f64x2 v = __builtin_nontemporal_load(a + i);
  if (v.x + v.y == 1.0) out[0] = v.x;  // the buffers hold zeros: never taken, keeps the load
}

// streams = number of read streams (1: copy, 7: the smoother's mix), one write
__global__ __launch_bounds__(256) void k_probe_mix(const f64x2 *__restrict__ a, f64x2 *__restrict__ b, int64_t n,
                                                   int streams) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  f64x2 s = __builtin_nontemporal_load(a + i);
  for (int k = 1; k < streams; ++k) s += __builtin_nontemporal_load(a + k * n + i);
  __builtin_nontemporal_store(s, b + i);
}

}  // namespace mg

using namespace mg;

extern "C" mg_status mg_stream_probe(int32_t kind, int64_t bytes, int32_t reps, double *gbs) {
  if (!gbs || kind < 0 || kind > 2 || reps < 1 || bytes < (1 << 20)) return MG_ERR_ARG;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  try {
    MG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    MG_HIP(hipEventCreate(&e0));
    MG_HIP(hipEventCreate(&e1));
    const int streams = kind == 2 ? 7 : 1;
    // kind 0 reads `bytes`; kinds 1 and 2 read (streams / (streams + 1)) of
    // `bytes` and write the rest
    const int64_t n = kind == 0 ? bytes / 16 : bytes / 16 / (streams + 1);
    DBuf<f64x2> a, b;
    DBuf<double> o;
    a.alloc(kind == 0 ? n : n * streams);
    b.alloc(kind == 0 ? 1 : n);
    o.alloc(1);
    MG_HIP(hipMemsetAsync(a.p, 0, a.bytes(), s));
    const unsigned g = (unsigned)((n + 255) / 256);
    auto launch = [&]() {
      if (kind == 0) k_probe_read<<<g, 256, 0, s>>>(a, n, o);
      else k_probe_mix<<<g, 256, 0, s>>>(a, b, n, streams);
      MG_LAUNCH_CHECK();
    };
    launch();  // warm-up
    MG_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) launch();
    MG_HIP(hipEventRecord(e1, s));
    MG_HIP(hipEventSynchronize(e1));
    float ms = 0;
    MG_HIP(hipEventElapsedTime(&ms, e0, e1));
    const double moved = 16.0 * (double)n * (kind == 0 ? 1 : streams + 1);
    *gbs = moved * reps / (ms * 1e-3) / 1e9;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    return MG_OK;
  } catch (const Error &e) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    return e.code;
  }
}
