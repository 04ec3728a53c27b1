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
// sync_metric_kernel: workgroup = (1024 candidates, group of antennas); per
// antenna the workgroup stages the samples its candidates need in LDS and
// each thread correlates 4 consecutive candidates through a sliding register
// window.  The staged samples sit in four planes by sample index mod 4, so
// the window's reads (thread t, sample 4t + m) are consecutive across lanes
// with compile-time offsets instead of a 4-dword stride (4-way LDS bank
// conflicts).  The per-group partial metrics are summed by sync_reduce_kernel
// (integer sums: exact in any order, 4 threads per candidate), which also
// reduces each 64 candidates to the best (M, n); sync_argmax_kernel reduces
// those in one workgroup.
// "Best" = larger M, then smaller n: a total order, so the result does not
// depend on the reduction order.
// sync_extract_kernel: copies the slots that follow the preamble into the
// receive path's layout [S][T][A][CP+N] (one complex sample per dword); the
// start index is read from device memory (the detected offset) plus a
// constant, so detection and extraction chain without a host round trip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rx_launch.h"

namespace rx {
namespace sync {

constexpr int kThreads = 256;       // threads per metric workgroup
constexpr int kTile = 4 * kThreads;  // candidates per metric workgroup
constexpr int kMaxGroups = 64;       // antenna groups (grid.y) at most
constexpr int kTargetGroups = 2048;  // metric workgroups aimed for (8 per CU)
constexpr int kRedCand = 64;         // candidates per reduce workgroup (4 threads each)

// Dwords per sample plane of the metric kernel's staging buffer: at least a
// quarter of the staged samples, and 16 more than a multiple of 64 so the
// four planes' rows fall in different LDS banks.
__host__ __device__ constexpr int plane_dwords(int L) {
  return ((kTile + L + 3 + 3) / 4 + 47) / 64 * 64 + 16;
}

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

// Partial metric of one antenna group for kTile candidates: thread t owns
// candidates n0 + 4t .. n0 + 4t + 3 and slides a 4-sample register window
// along the staged samples, so each LDS read feeds 4 (candidate, chip) pairs.
template <int Q>
__device__ __forceinline__ void unpack(uint32_t s, int (&re)[Q], int (&im)[Q], int j) {
  re[j] = (int)(int16_t)(s & 0xFFFFu);
  im[j] = (int)(int16_t)(s >> 16);
}

__global__ __launch_bounds__(kThreads) void sync_metric_kernel(const uint32_t* __restrict__ raw, int A, int ag,
                                                               int64_t n_samples, int64_t stride, SyncChips ch,
                                                               int64_t n_search, uint64_t* __restrict__ part) {
  extern __shared__ uint32_t ys[];  // 4 planes of plane_dwords(L): sample j at (j % 4) * P + j / 4
  const int tid = threadIdx.x, L = ch.L;
  const int P = plane_dwords(L);
  const int64_t n0 = (int64_t)blockIdx.x * kTile;
  const int g = blockIdx.y, a0 = g * ag, a1 = min(A, a0 + ag);
  const int span = kTile + L + 3;
  uint64_t acc[4] = {0, 0, 0, 0};
  // sample 4t + k of this thread's window: plane k % 4, row t + k / 4
  auto Y = [&](int k) { return ys[(k & 3) * P + tid + (k >> 2)]; };
  for (int a = a0; a < a1; a++) {
    __syncthreads();  // the previous antenna's readers are done
    const uint32_t* ya = raw + (int64_t)a * stride;
    for (int j = tid; j < span; j += kThreads) {
      const int64_t i = n0 + j;
      ys[(j & 3) * P + (j >> 2)] = i < n_samples ? ya[i] : 0u;
    }
    __syncthreads();
    int wr[4], wi[4];
#pragma unroll
    for (int j = 0; j < 4; j++) unpack<4>(Y(j), wr, wi, j);
    int re[4] = {0, 0, 0, 0}, im[4] = {0, 0, 0, 0};
    // window slot (m + j) % 4 holds sample 4t + m + j
    // Steps of four chips, software-pipelined: the next step's chips (one
    // dword, little-endian bytes) and window samples are requested once this
    // step has taken its own, so the wait for them (one counter for scalar and
    // LDS loads) falls a whole step after they were issued.
    int m = 0;
    if (L >= 4) {
      int cn;
      uint32_t yn[4];
      __builtin_memcpy(&cn, ch.c, 4);
#pragma unroll
      for (int u = 0; u < 4; u++) yn[u] = Y(u + 4);
      for (; m + 4 <= L; m += 4) {
        const int cw = cn;
        uint32_t yc[4];
#pragma unroll
        for (int u = 0; u < 4; u++) yc[u] = yn[u];
        __builtin_amdgcn_sched_barrier(0);
        if (m + 8 <= L) {
          __builtin_memcpy(&cn, ch.c + m + 4, 4);
#pragma unroll
          for (int u = 0; u < 4; u++) yn[u] = Y(m + u + 8);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const int c = (int)(int8_t)(uint32_t)(cw >> (8 * u));  // chip m + u
#pragma unroll
          for (int j = 0; j < 4; j++) {
            // 24-bit products (samples are 16-bit, chips 8-bit): exact, and a
            // full-rate multiply-add instead of a 32-bit integer multiply
            re[j] += __mul24(c, wr[(u + j) & 3]);
            im[j] += __mul24(c, wi[(u + j) & 3]);
          }
          unpack<4>(yc[u], wr, wi, u);  // slot u now holds sample 4t + m + u + 4
        }
      }
    }
    for (; m < L; m++) {  // tail: rotate by hand
      const int c = ch.c[m];
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int s = (m + j) & 3;
        int vr = wr[0], vi = wi[0];
#pragma unroll
        for (int k = 1; k < 4; k++)
          if (s == k) {
            vr = wr[k];
            vi = wi[k];
          }
        re[j] += __mul24(c, vr);
        im[j] += __mul24(c, vi);
      }
      const int s = m & 3;
      const uint32_t nx = Y(m + 4);
#pragma unroll
      for (int k = 0; k < 4; k++)
        if (s == k) unpack<4>(nx, wr, wi, k);
    }
#pragma unroll
    for (int j = 0; j < 4; j++) acc[j] += (uint64_t)((int64_t)re[j] * re[j]) + (uint64_t)((int64_t)im[j] * im[j]);
  }
  uint64_t* out = part + (int64_t)g * n_search;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const int64_t n = n0 + 4 * tid + j;
    if (n < n_search) out[n] = acc[j];
  }
}

// M[n] = sum over antenna groups (integers: any order is exact), 4 threads
// per candidate (wave w sums groups w, w + 4, ...), plus the best (M, n) of
// each workgroup's kRedCand candidates.
__global__ __launch_bounds__(256) void sync_reduce_kernel(const uint64_t* __restrict__ part, int G, int64_t n_search,
                                                          uint64_t* __restrict__ M, uint64_t* __restrict__ cand_v,
                                                          int64_t* __restrict__ cand_i) {
  __shared__ uint64_t sums[4][kRedCand];
  const int c = threadIdx.x & (kRedCand - 1), w = threadIdx.x / kRedCand;
  const int64_t n = (int64_t)blockIdx.x * kRedCand + c;
  const bool ok = n < n_search;
  uint64_t v = 0;
  if (ok)
    for (int g = w; g < G; g += 4) v += part[(int64_t)g * n_search + n];
  sums[w][c] = v;
  __syncthreads();
  if (w == 0) {
    v += sums[1][c] + sums[2][c] + sums[3][c];
    if (ok && M) M[n] = v;
    Best b = {ok ? v : 0ull, ok ? n : INT64_MAX};
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) b = better(b, shfl_xor(b, o));
    if (c == 0) {
      cand_v[blockIdx.x] = b.v;
      cand_i[blockIdx.x] = b.i;
    }
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

// Antenna groups: enough workgroups to fill the GPU (about kTargetGroups), at
// most one group per antenna.
int sync_groups(int A, int64_t n_search) {
  const int64_t tiles = (n_search + sync::kTile - 1) / sync::kTile;
  int64_t g = (sync::kTargetGroups + tiles - 1) / tiles;
  if (g > A) g = A;
  if (g > sync::kMaxGroups) g = sync::kMaxGroups;
  if (g < 1) g = 1;
  const int ag = (A + (int)g - 1) / (int)g;
  return (A + ag - 1) / ag;
}

size_t sync_workspace(int A, int64_t n_search) {
  const int64_t nb = (n_search + sync::kRedCand - 1) / sync::kRedCand;
  return (size_t)sync_groups(A, n_search) * n_search * 8 + (size_t)nb * 16;
}

hipError_t sync_find(const uint32_t* raw, int A, int64_t n_samples, int64_t stride, const SyncChips& ch,
                     int64_t n_search, uint64_t* M, int64_t* offset, uint64_t* peak, void* workspace,
                     hipStream_t st) {
  const int G = sync_groups(A, n_search);
  const int ag = (A + G - 1) / G;
  const int64_t tiles = (n_search + sync::kTile - 1) / sync::kTile;
  const int64_t nb = (n_search + sync::kRedCand - 1) / sync::kRedCand;
  uint64_t* part = static_cast<uint64_t*>(workspace);
  uint64_t* cv = part + (int64_t)G * n_search;
  int64_t* ci = reinterpret_cast<int64_t*>(cv + nb);
  const size_t lds = sizeof(uint32_t) * 4 * (size_t)sync::plane_dwords(ch.L);
  hipLaunchKernelGGL(sync::sync_metric_kernel, dim3((unsigned)tiles, (unsigned)G), dim3(sync::kThreads), lds, st,
                     raw, A, ag, n_samples, stride, ch, n_search, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sync::sync_reduce_kernel, dim3((unsigned)nb), dim3(256), 0, st, (const uint64_t*)part, G,
                     n_search, M, cv, ci);
  if ((e = hipGetLastError()) != hipSuccess) return e;
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
