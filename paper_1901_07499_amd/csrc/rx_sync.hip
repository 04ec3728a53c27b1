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
// (integer sums: exact in any order, 16 threads per candidate), which also
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

typedef short s16x2 __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;       // threads per metric workgroup
constexpr int kTile = 4 * kThreads;  // candidates per metric workgroup
constexpr int kMaxGroups = 64;       // antenna groups (grid.y) at most
constexpr int kTargetGroups = 2048;  // metric workgroups aimed for (8 per CU)
constexpr int kRedCand = 64;         // candidates per reduce workgroup
constexpr int kRedWaves = 16;        // wavefronts per reduce workgroup (threads per candidate)

// Dwords per sample plane of the metric kernel's staging buffer: at least a
// quarter of the staged samples plus the window words the last step
// requests ahead (thread 255, window index up to L + 7), and 16 more than a
// multiple of 64 so the four planes' rows fall in different LDS banks.
__host__ __device__ constexpr int plane_dwords(int L) {
  return ((kTile + L + 8 + 3) / 4 + 47) / 64 * 64 + 16;
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
    // Raw sample words in a sliding window: sw0 = samples 4t + m .. + 3,
    // sw1 = the next four, at the top of the step of chips m .. m + 3.  A
    // step applies chip pairs (m, m + 1) and (m + 2, m + 3) to the four
    // candidates with one 2-way 16-bit dot product (exact, into int32) per
    // candidate and component: re[j] += c_m yr[m + j] + c_(m+1) yr[m + j + 1].
    // The dot products take the real (imaginary) parts of samples k and k + 1
    // packed into one word, pr[k - m] (pi[k - m]), built once per k with a
    // byte permute and kept for the next step (k = m + 4, m + 5 become its
    // first two).
    uint32_t sw0[4], sw1[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      sw0[u] = Y(u);
      sw1[u] = Y(u + 4);
    }
    auto pre = [](uint32_t lo, uint32_t hi) { return __builtin_amdgcn_perm(hi, lo, 0x05040100u); };
    auto pim = [](uint32_t lo, uint32_t hi) { return __builtin_amdgcn_perm(hi, lo, 0x07060302u); };
    uint32_t pr[6], pi[6];
    pr[0] = pre(sw0[0], sw0[1]);
    pi[0] = pim(sw0[0], sw0[1]);
    pr[1] = pre(sw0[1], sw0[2]);
    pi[1] = pim(sw0[1], sw0[2]);
    int re[4] = {0, 0, 0, 0}, im[4] = {0, 0, 0, 0};
    int m = 0;
    // Steps of four chips (one little-endian dword of them), software-
    // pipelined: the next step's chips and samples are requested once this
    // step has taken its own, so the wait for them falls a whole step after
    // they were issued.  The samples are requested on every step, also ahead
    // of a tail of 1..3 chips or of nothing (window indices up to L + 7,
    // inside the staging planes; those past the staged span are never used).
    int cn = 0;
    if (L >= 4) __builtin_memcpy(&cn, ch.c, 4);
    // One step of chips m .. m + 3 over the window words a (samples m ..),
    // b (m + 4 ..); requests the next four into n.
    auto step = [&](int mm, uint32_t (&a)[4], uint32_t (&b)[4], uint32_t (&n)[4]) {
      const int cw = cn;
      __builtin_amdgcn_sched_barrier(0);
      if (mm + 8 <= L) __builtin_memcpy(&cn, ch.c + mm + 4, 4);
#pragma unroll
      for (int u = 0; u < 4; u++) n[u] = Y(mm + u + 8);  // window index <= L + 7
      pr[2] = pre(a[2], a[3]);
      pi[2] = pim(a[2], a[3]);
      pr[3] = pre(a[3], b[0]);
      pi[3] = pim(a[3], b[0]);
      pr[4] = pre(b[0], b[1]);
      pi[4] = pim(b[0], b[1]);
      pr[5] = pre(b[1], b[2]);
      pi[5] = pim(b[1], b[2]);
      // chips mm .. mm + 3 as two pairs of int16
      const s16x2 c01 = {(short)(int8_t)(uint32_t)cw, (short)(int8_t)((uint32_t)cw >> 8)};
      const s16x2 c23 = {(short)(int8_t)((uint32_t)cw >> 16), (short)(int8_t)((uint32_t)cw >> 24)};
#pragma unroll
      for (int j = 0; j < 4; j++) {
        re[j] = __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, pr[j]), c01, re[j], false);
        im[j] = __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, pi[j]), c01, im[j], false);
      }
#pragma unroll
      for (int j = 0; j < 4; j++) {
        re[j] = __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, pr[j + 2]), c23, re[j], false);
        im[j] = __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, pi[j + 2]), c23, im[j], false);
      }
      pr[0] = pr[4];
      pi[0] = pi[4];
      pr[1] = pr[5];
      pi[1] = pi[5];
    };
    // Three steps per iteration, the three window buffers taking turns (the
    // roles cycle with period three, so no register copies), then at most
    // two more steps; the tail reads the window from sw0, sw1.
    uint32_t sw2[4];
    for (; m + 12 <= L; m += 12) {
      step(m, sw0, sw1, sw2);
      step(m + 4, sw1, sw2, sw0);
      step(m + 8, sw2, sw0, sw1);
    }
    if (m + 4 <= L) {
      step(m, sw0, sw1, sw2);
      m += 4;
      if (m + 4 <= L) {
        step(m, sw1, sw2, sw0);
        m += 4;
#pragma unroll
        for (int u = 0; u < 4; u++) {  // window: sw2, sw0
          sw1[u] = sw0[u];
          sw0[u] = sw2[u];
        }
      } else {
#pragma unroll
        for (int u = 0; u < 4; u++) {  // window: sw1, sw2
          sw0[u] = sw1[u];
          sw1[u] = sw2[u];
        }
      }
    }
    // tail of L mod 4 chips: chip m + e meets sample m + e + j, which is
    // window word e + j (sw0, then sw1)
#pragma unroll
    for (int e = 0; e < 3; e++) {
      if (m + e < L) {
        const int c = ch.c[m + e];
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const uint32_t w = (e + j) < 4 ? sw0[(e + j) & 3] : sw1[(e + j) & 3];
          re[j] += __mul24(c, (int)(int16_t)(w & 0xFFFFu));
          im[j] += __mul24(c, (int)(int16_t)(w >> 16));
        }
      }
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

// M[n] = sum over antenna groups (integers: any order is exact), kRedWaves
// threads per candidate (wave w sums groups w, w + kRedWaves, ...: at most
// four loads each, so the partial metrics stream with many loads in flight),
// plus the best (M, n) of each workgroup's kRedCand candidates.
__global__ __launch_bounds__(64 * kRedWaves) void sync_reduce_kernel(const uint64_t* __restrict__ part, int G,
                                                                     int64_t n_search, uint64_t* __restrict__ M,
                                                                     uint64_t* __restrict__ cand_v,
                                                                     int64_t* __restrict__ cand_i) {
  __shared__ uint64_t sums[kRedWaves][kRedCand];
  const int c = threadIdx.x & (kRedCand - 1), w = threadIdx.x / kRedCand;
  const int64_t n = (int64_t)blockIdx.x * kRedCand + c;
  const bool ok = n < n_search;
  uint64_t v = 0;
  if (ok)
    for (int g = w; g < G; g += kRedWaves) v += part[(int64_t)g * n_search + n];
  sums[w][c] = v;
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int k = 1; k < kRedWaves; k++) v += sums[k][c];
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
  hipLaunchKernelGGL(sync::sync_reduce_kernel, dim3((unsigned)nb), dim3(64 * sync::kRedWaves), 0, st,
                     (const uint64_t*)part, G,
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
