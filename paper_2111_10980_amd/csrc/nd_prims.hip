// Parallel primitives used around the hot path (paper Section 2, "Parallel
// Primitives": prefix sum and filter), written for wave64 CDNA4:
//   - tile scan: 256 threads x 8 items per tile, tile sums scanned recursively;
//   - stable LSD radix sort with 8-bit digits: one wave per 1024-key tile,
//     in-wave ranks from 8 ballots (lanes with equal digits), per-tile
//     digit histograms scanned in digit-major order;
//   - fills, reductions.
#include "nd_host.h"

namespace nd {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

int64_t blocks_for(int64_t n, int64_t per, int64_t cap = 1 << 20) {
  int64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  return b < cap ? b : cap;
}

template <class T>
__device__ __forceinline__ T wave_incl_scan_t(T v) {
  int lane = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T o = __shfl_up(v, off);
    if (lane >= off) v += o;
  }
  return v;
}

template <class T>
__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const T *__restrict__ in, int64_t n,
                                                            T *__restrict__ sums) {
  __shared__ T part[kScanThreads / kWave];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  T acc = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    int64_t i = base + j * kScanThreads + threadIdx.x;
    if (i < n) acc += in[i];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane_id() == 0) part[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T t = 0;
    for (int w = 0; w < kScanThreads / kWave; w++) t += part[w];
    sums[blockIdx.x] = t;
  }
}

template <class T>
__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const T *in, T *out, int64_t n,
                                                            const T *__restrict__ offs) {
  __shared__ T tile[kScanTile];
  __shared__ T wsum[kScanThreads / kWave];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    int idx = j * kScanThreads + threadIdx.x;
    int64_t i = base + idx;
    tile[idx] = i < n ? in[i] : (T)0;
  }
  __syncthreads();
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    v[j] = tile[threadIdx.x * kScanItems + j];
    s += v[j];
  }
  T incl = wave_incl_scan_t<T>(s);
  int w = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) wsum[w] = incl;
  __syncthreads();
  T woff = 0;
  for (int q = 0; q < w; q++) woff += wsum[q];
  T run = incl - s + woff + (offs ? offs[blockIdx.x] : (T)0);
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    tile[threadIdx.x * kScanItems + j] = run;
    run += v[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    int idx = j * kScanThreads + threadIdx.x;
    int64_t i = base + idx;
    if (i < n) out[i] = tile[idx];
  }
}

template <class T>
void scan_impl(const T *in, T *out, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    hipLaunchKernelGGL(k_tile_scan<T>, dim3(1), dim3(kScanThreads), 0, st, in, out, n,
                       (const T *)nullptr);
    return;
  }
  DevBuf<T> sums((size_t)nb);
  hipLaunchKernelGGL(k_tile_sums<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n,
                     sums.get());
  scan_impl<T>(sums.get(), sums.get(), nb, st);
  hipLaunchKernelGGL(k_tile_scan<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, out, n,
                     (const T *)sums.get());
}

// ------------------------------------------------------------- radix sort

constexpr int kSortItems = 16;
constexpr int kSortTile = kWave * kSortItems;

__global__ __launch_bounds__(kWave) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                   int shift, uint32_t *__restrict__ hist,
                                                   int64_t nb) {
  __shared__ uint32_t h[256];
  for (int d = threadIdx.x; d < 256; d += kWave) h[d] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
  for (int j = 0; j < kSortItems; j++) {
    int64_t i = base + j * kWave + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < 256; d += kWave) hist[(int64_t)d * nb + blockIdx.x] = h[d];
}

__global__ __launch_bounds__(kWave) void k_rs_scatter(const uint64_t *__restrict__ kin,
                                                      const uint32_t *__restrict__ vin,
                                                      uint64_t *__restrict__ kout,
                                                      uint32_t *__restrict__ vout, int64_t n,
                                                      int shift, const uint32_t *__restrict__ offs,
                                                      int64_t nb) {
  __shared__ uint32_t run[256];
  for (int d = threadIdx.x; d < 256; d += kWave) run[d] = offs[(int64_t)d * nb + blockIdx.x];
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int j = 0; j < kSortItems; j++) {
    int64_t i = base + j * kWave + threadIdx.x;
    bool valid = i < n;
    uint64_t key = valid ? kin[i] : 0ull;
    uint32_t digit = (uint32_t)(key >> shift) & 255u;
    uint64_t match = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      bool bit = (digit >> b) & 1u;
      uint64_t m = __ballot(valid && bit);
      match &= bit ? m : ~m;
    }
    uint32_t rank = (uint32_t)__popcll(match & lanes_below());
    uint32_t pos = run[digit] + rank;
    if (valid) {
      kout[pos] = key;
      if (vin) vout[pos] = vin[i];
    }
    __syncthreads();
    if (valid && rank == 0) run[digit] += (uint32_t)__popcll(match);
    __syncthreads();
  }
}

// ------------------------------------------------------------------ fills

template <class T>
__global__ void k_fill(T *p, T v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_slots(Slot *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    Slot s;
    s.key = 0;
    s.cnt = 0;
    s.stamp = kLive;
    p[i] = s;
  }
}

__global__ void k_widen(const uint32_t *__restrict__ a, uint64_t *b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

__global__ void k_iota(uint32_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_sum_u32(const uint32_t *__restrict__ p, int64_t n,
                                                 unsigned long long *out) {
  uint64_t acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += p[i];
  acc = wave_sum_u64(acc);
  if (lane_id() == 0 && acc) atomicAdd(out, (unsigned long long)acc);
}

__global__ __launch_bounds__(256) void k_max_u32(const uint32_t *__restrict__ p, int64_t n,
                                                 uint32_t *out) {
  uint32_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = p[i] > m ? p[i] : m;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    uint32_t o = __shfl_xor(m, off);
    m = o > m ? o : m;
  }
  if (lane_id() == 0 && m) atomicMax(out, m);
}

}  // namespace

void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3((unsigned)blocks_for(n, 256 * 8, 8192)), dim3(256),
                     0, st, p, v, n);
}

void fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<uint64_t>, dim3((unsigned)blocks_for(n, 256 * 8, 8192)), dim3(256),
                     0, st, p, v, n);
}

void fill_slots(Slot *p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_slots, dim3((unsigned)blocks_for(n, 256 * 4, 16384)), dim3(256), 0,
                     st, p, n);
}

void widen_u32_to_u64(const uint32_t *a, uint64_t *b, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_widen, dim3((unsigned)blocks_for(n, 256 * 8, 8192)), dim3(256), 0, st, a,
                     b, n);
}

void iota_u32(uint32_t *p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_iota, dim3((unsigned)blocks_for(n, 256 * 8, 8192)), dim3(256), 0, st, p,
                     n);
}

void scan_exclusive_u64(const uint64_t *in, uint64_t *out, int64_t n, hipStream_t st) {
  scan_impl<uint64_t>(in, out, n, st);
}

void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t st) {
  scan_impl<uint32_t>(in, out, n, st);
}

uint64_t scan_ws_bytes(int64_t n, size_t elem) {
  if (n <= 0) return 0;
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) return 0;
  return ws_block((uint64_t)nb * elem) + scan_ws_bytes(nb, elem);
}

uint64_t radix_sort_ws_bytes(int64_t n, int bits, int lo_bit, bool vals) {
  if (n <= 1 || bits <= lo_bit) return 0;
  const int passes = (bits - lo_bit + 7) / 8;
  const int64_t nb = (n + kSortTile - 1) / kSortTile;
  return ws_buf<uint64_t>((uint64_t)n) + (vals ? ws_buf<uint32_t>((uint64_t)n) : 0) +
         ws_buf<uint32_t>((uint64_t)(256 * nb)) + (uint64_t)passes * scan_ws_bytes(256 * nb, 4);
}

void radix_sort(uint64_t *keys, uint32_t *vals, int64_t n, int bits, hipStream_t st,
                int lo_bit) {
  if (n <= 1 || bits <= lo_bit) return;
  int passes = (bits - lo_bit + 7) / 8;
  int64_t nb = (n + kSortTile - 1) / kSortTile;
  DevBuf<uint64_t> k2((size_t)n);
  DevBuf<uint32_t> v2(vals ? (size_t)n : 0);
  DevBuf<uint32_t> hist((size_t)(256 * nb));
  uint64_t *ks = keys, *kd = k2.get();
  uint32_t *vs = vals, *vd = v2.get();
  for (int p = 0; p < passes; p++) {
    int shift = lo_bit + 8 * p;
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(kWave), 0, st, ks, n, shift,
                       hist.get(), nb);
    scan_exclusive_u32(hist.get(), hist.get(), 256 * nb, st);
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(kWave), 0, st, ks, vs, kd, vd, n,
                       shift, hist.get(), nb);
    uint64_t *tk = ks; ks = kd; kd = tk;
    uint32_t *tv = vs; vs = vd; vd = tv;
  }
  if (ks != keys) {
    hip_ok(hipMemcpyAsync(keys, ks, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToDevice, st),
           "copy sorted keys");
    if (vals)
      hip_ok(hipMemcpyAsync(vals, vs, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, st),
             "copy sorted values");
  }
}

void sum_u32(const uint32_t *p, int64_t n, uint64_t *out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_sum_u32, dim3((unsigned)blocks_for(n, 256 * 16, 4096)), dim3(256), 0, st,
                     p, n, (unsigned long long *)out);
}

uint32_t max_u32_host(const uint32_t *p, int64_t n, hipStream_t st) {
  if (n <= 0) return 0;
  DevBuf<uint32_t> m(1);
  fill_u32(m.get(), 0, 1, st);
  hipLaunchKernelGGL(k_max_u32, dim3((unsigned)blocks_for(n, 256 * 16, 4096)), dim3(256), 0, st,
                     p, n, m.get());
  uint32_t h = 0;
  read_back(&h, m.get(), sizeof(uint32_t), st);
  return h;
}

}  // namespace nd
