// Roofline ceilings measured on the device the library runs on: the rates
// the hot path's memory operations can reach at best.
//   stream copy          bytes/s of a coalesced 16-byte-per-lane copy
//   random 16-byte load  slot-sized gathers/s from a table-sized buffer
//   random u32 atomics   returning and non-returning atomic adds/s on a
//                        count-array-sized buffer (device scope)
// Each kernel is timed with HIP events on the caller's stream.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nd_roofline.h"

namespace {

__device__ __forceinline__ uint64_t mixr(uint64_t x) {
  // splitmix64 output mixer (Steele, Lea, Flood 2014)
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

__global__ __launch_bounds__(256) void k_copy(const uint4 *__restrict__ a, uint4 *__restrict__ b,
                                              uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

__global__ __launch_bounds__(256) void k_gather(const uint4 *__restrict__ a, uint64_t n_slots,
                                                uint64_t n_ops, uint32_t *sink) {
  uint32_t acc = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_ops;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint4 v = a[((mixr(i) >> 32) * n_slots) >> 32];
    acc += v.x ^ v.w;
  }
  if (acc == 0x9e3779b9u) sink[0] = acc;  // keeps the loads alive
}

__global__ __launch_bounds__(256) void k_atomic(uint32_t *__restrict__ a, uint64_t n_words,
                                                uint64_t n_ops, int with_return, uint32_t *sink) {
  uint32_t acc = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_ops;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t *p = a + (((mixr(i) >> 32) * n_words) >> 32);
    if (with_return) acc += __hip_atomic_fetch_add(p, 0xFFFFFFFFu, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
    else __hip_atomic_fetch_add(p, 0xFFFFFFFFu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (with_return && acc == 0x9e3779b9u) sink[0] = acc;
}

float time_it(hipStream_t st, void (*launch)(hipStream_t, void *), void *ctx, int reps) {
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  launch(st, ctx);  // warm-up
  hipEventRecord(a, st);
  for (int r = 0; r < reps; r++) launch(st, ctx);
  hipEventRecord(b, st);
  hipEventSynchronize(b);
  float ms = 0;
  hipEventElapsedTime(&ms, a, b);
  hipEventDestroy(a);
  hipEventDestroy(b);
  return ms / (float)reps;
}

struct Ctx {
  void *a, *b;
  uint64_t n, ops;
  int with_return;
  uint32_t *sink;
};

const unsigned kGrid = 256 * 64;

void launch_copy(hipStream_t st, void *c) {
  Ctx *x = (Ctx *)c;
  hipLaunchKernelGGL(k_copy, dim3(kGrid), dim3(256), 0, st, (const uint4 *)x->a, (uint4 *)x->b,
                     x->n);
}
void launch_gather(hipStream_t st, void *c) {
  Ctx *x = (Ctx *)c;
  hipLaunchKernelGGL(k_gather, dim3(kGrid), dim3(256), 0, st, (const uint4 *)x->a, x->n, x->ops,
                     x->sink);
}
void launch_atomic(hipStream_t st, void *c) {
  Ctx *x = (Ctx *)c;
  hipLaunchKernelGGL(k_atomic, dim3(kGrid), dim3(256), 0, st, (uint32_t *)x->a, x->n, x->ops,
                     x->with_return, x->sink);
}

}  // namespace

extern "C" int nd_roofline_measure(uint64_t table_bytes, uint64_t count_bytes, void *hip_stream,
                                   nd_roofline *out) {
  if (!out) return 1;
  hipStream_t st = (hipStream_t)hip_stream;
  const uint64_t copy_bytes = 1ull << 30;
  uint64_t big = table_bytes > copy_bytes ? table_bytes : copy_bytes;
  if (count_bytes > big) big = count_bytes;
  void *a = nullptr, *b = nullptr;
  uint32_t *sink = nullptr;
  if (hipMalloc(&a, big) != hipSuccess) return 5;
  if (hipMalloc(&b, copy_bytes) != hipSuccess) {
    hipFree(a);
    return 5;
  }
  if (hipMalloc(&sink, 64) != hipSuccess) {
    hipFree(a);
    hipFree(b);
    return 5;
  }
  hipMemsetAsync(a, 0, big, st);
  Ctx c{a, b, copy_bytes / 16, 0, 0, sink};
  float ms = time_it(st, launch_copy, &c, 5);
  out->copy_gbs = 2.0 * (double)copy_bytes / (ms * 1e-3) / 1e9;
  const uint64_t ops = 1ull << 28;
  c.n = table_bytes / 16;
  c.ops = ops;
  ms = time_it(st, launch_gather, &c, 3);
  out->gather16_gops = (double)ops / (ms * 1e-3) / 1e9;
  c.n = count_bytes / 4;
  c.with_return = 1;
  ms = time_it(st, launch_atomic, &c, 3);
  out->atomic_ret_gops = (double)ops / (ms * 1e-3) / 1e9;
  c.with_return = 0;
  ms = time_it(st, launch_atomic, &c, 3);
  out->atomic_noret_gops = (double)ops / (ms * 1e-3) / 1e9;
  hipStreamSynchronize(st);
  hipFree(a);
  hipFree(b);
  hipFree(sink);
  return hipGetLastError() == hipSuccess ? 0 : 6;
}
