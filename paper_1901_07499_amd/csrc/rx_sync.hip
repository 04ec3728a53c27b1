// rx_sync.hip -- PN-preamble frame synchronisation and slot extraction (gfx950).
//
// The receiver correlates every antenna's stream with the maximum-length PN
// sequence that opens a frame and takes the correlation peak as the start of
// the frame (paper Sec. II-B; Table I: PN length 255):
//   c_a[n] = sum_m p[m] y_a[n+m],   M[n] = sum_a |c_a[n]|^2,
//   offset = the first n with the largest M[n].
// With chips p in {-1, 0, +1} and int16 samples the metric is exact in
// integers (|c| < 2^25 per component, M < 2^64), so the peak decision needs no
// floating point at all.
//
// sync_metric_kernel: one thread per candidate n; a workgroup stages the
// samples its candidates need (kCand + L - 1 per antenna) in LDS and loops over
// the antennas in order, so M[n] is a fixed-order integer sum.  Each workgroup
// also reduces its (M, n) pairs to the best one; sync_argmax_kernel reduces
// those in one workgroup.  "Best" = larger M, then smaller n: a total order,
// so the result does not depend on the reduction order.
// sync_extract_kernel: copies the slots that follow the preamble into the
// receive path's layout [S][T][A][CP+N] (one complex sample per dword); the
// start index is read from device memory (the detected offset) plus a
// constant, so detection and extraction chain without a host round trip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rx_launch.h"

namespace rx {
namespace sync {

constexpr int kCand = 128;  // candidates (threads) per workgroup

struct Best {
  uint64_t v;
  int64_t i;
};

__device__ __forceinline__ Best better(Best a, Best b) { return (a.v > b.v || (a.v == b.v && a.i < b.i)) ? a : b; }

__device__ __forceinline__ Best shfl_xor(Best x, int o) {
  Best r;
  r.v = ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(x.v >> 32), o, 64) << 32) |
        (uint32_t)__shfl_xor((int)(uint32_t)x.v, o, 64);
  r.i = (int64_t)(((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)((uint64_t)x.i >> 32), o, 64) << 32) |
                  (uint32_t)__shfl_xor((int)(uint32_t)(uint64_t)x.i, o, 64));
  return r;
}

// Best over the workgroup; valid in thread 0.
__device__ __forceinline__ Best block_best(Best b, Best* sh) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) b = better(b, shfl_xor(b, o));
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[wave] = b;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < nw; w++) b = better(b, sh[w]);
  return b;
}

__global__ __launch_bounds__(kCand) void sync_metric_kernel(const uint32_t* __restrict__ raw, int A,
                                                            int64_t n_samples, int64_t stride, SyncChips ch,
                                                            int64_t n_search, uint64_t* __restrict__ M,
                                                            uint64_t* __restrict__ cand_v,
                                                            int64_t* __restrict__ cand_i) {
  extern __shared__ uint32_t ys[];  // [kCand + L - 1]
  __shared__ int chip[kMaxPn];
  __shared__ Best sh[kCand / 64];
  const int tid = threadIdx.x, L = ch.L;
  const int64_t n0 = (int64_t)blockIdx.x * kCand, n = n0 + tid;
  for (int m = tid; m < L; m += kCand) chip[m] = ch.c[m];
  const int span = kCand + L - 1;
  uint64_t acc = 0;
  for (int a = 0; a < A; a++) {
    __syncthreads();  // the previous antenna's readers are done (and the chips are in place)
    const uint32_t* ya = raw + (int64_t)a * stride;
    for (int j = tid; j < span; j += kCand) {
      const int64_t i = n0 + j;
      ys[j] = i < n_samples ? ya[i] : 0u;
    }
    __syncthreads();
    int re = 0, im = 0;
    for (int m = 0; m < L; m++) {
      const uint32_t s = ys[tid + m];
      const int c = chip[m];
      re += c * (int)(int16_t)(s & 0xFFFFu);
      im += c * (int)(int16_t)(s >> 16);
    }
    acc += (uint64_t)((int64_t)re * re) + (uint64_t)((int64_t)im * im);
  }
  const bool ok = n < n_search;
  if (ok && M) M[n] = acc;
  Best b = {ok ? acc : 0ull, ok ? n : INT64_MAX};
  b = block_best(b, sh);
  if (tid == 0) {
    cand_v[blockIdx.x] = b.v;
    cand_i[blockIdx.x] = b.i;
  }
}

__global__ __launch_bounds__(256) void sync_argmax_kernel(const uint64_t* __restrict__ cand_v,
                                                          const int64_t* __restrict__ cand_i, int n_blocks,
                                                          int64_t* __restrict__ offset, uint64_t* __restrict__ peak) {
  __shared__ Best sh[4];
  Best b = {0ull, INT64_MAX};
  for (int k = threadIdx.x; k < n_blocks; k += blockDim.x) b = better(b, Best{cand_v[k], cand_i[k]});
  b = block_best(b, sh);
  if (threadIdx.x == 0) {
    *offset = b.i;
    if (peak) *peak = b.v;
  }
}

// Row r = (s * T + t) * A + a of the output holds symbol t of slot s on
// antenna a: stream samples start + (s * T + t) * sym_len + j, j < sym_len,
// zero outside [0, n_samples).
__global__ __launch_bounds__(256) void sync_extract_kernel(const uint32_t* __restrict__ raw, int A,
                                                           int64_t n_samples, int64_t stride,
                                                           const int64_t* __restrict__ start_dev,
                                                           int64_t start_add, int sym_len, int T, int64_t rows,
                                                           uint32_t* __restrict__ out) {
  const int64_t start = (start_dev ? *start_dev : 0) + start_add;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const int a = (int)(r % A);
    const int64_t st = r / A;  // s * T + t
    const int64_t base = start + st * sym_len;
    const uint32_t* ya = raw + (int64_t)a * stride;
    uint32_t* o = out + r * sym_len;
    for (int j = threadIdx.x; j < sym_len; j += blockDim.x) {
      const int64_t i = base + j;
      o[j] = (i >= 0 && i < n_samples) ? ya[i] : 0u;
    }
  }
}

}  // namespace sync

int64_t sync_blocks(int64_t n_search) { return (n_search + sync::kCand - 1) / sync::kCand; }

hipError_t sync_find(const uint32_t* raw, int A, int64_t n_samples, int64_t stride, const SyncChips& ch,
                     int64_t n_search, uint64_t* M, int64_t* offset, uint64_t* peak, void* workspace,
                     hipStream_t st) {
  const int64_t nb = sync_blocks(n_search);
  uint64_t* cv = static_cast<uint64_t*>(workspace);
  int64_t* ci = reinterpret_cast<int64_t*>(cv + nb);
  const size_t lds = sizeof(uint32_t) * (size_t)(sync::kCand + ch.L - 1);
  hipLaunchKernelGGL(sync::sync_metric_kernel, dim3((unsigned)nb), dim3(sync::kCand), lds, st, raw, A, n_samples,
                     stride, ch, n_search, M, cv, ci);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sync::sync_argmax_kernel, dim3(1), dim3(256), 0, st, (const uint64_t*)cv, (const int64_t*)ci,
                     (int)nb, offset, peak);
  return hipGetLastError();
}

hipError_t sync_extract(const uint32_t* raw, int A, int64_t n_samples, int64_t stride, const int64_t* start,
                        int64_t start_add, int sym_len, int T, int64_t S, uint32_t* out, hipStream_t st) {
  const int64_t rows = S * T * A;
  const int64_t grid = rows < 65536 ? rows : 65536;
  hipLaunchKernelGGL(sync::sync_extract_kernel, dim3((unsigned)grid), dim3(256), 0, st, raw, A, n_samples, stride,
                     start, start_add, sym_len, T, rows, out);
  return hipGetLastError();
}

}  // namespace rx
