// rx_mfma_fft.hip -- the receive path with the 2048-point FFT recast as
// DFT-stage GEMMs on the fp16 / bf16 matrix cores (gfx950), FP32 accumulate,
// optionally with a hi+lo split of both operands (three products per GEMM).
//
// Transform (one wavefront per antenna symbol), N = 2048 = 8 x 16 x 16:
//   n = n1 + 16 n2 + 256 n3,  k = k3 + 8 k2 + 128 k1
//   A[n1,n2,k3] = W^(16 n2 k3) / 8  * sum_n3 x[n] W8^(n3 k3)        (FP32, vector ALU)
//   B[n1,k2,k3] = W^(n1 (k3+8k2)) / 16 * sum_n2 A W16^(n2 k2)       (GEMM 1)
//   X[k]        = 128 * sum_n1 B W16^(n1 k1)                          (GEMM 2)
// with W = exp(-2 pi i / 2048).  The two radix-16 stages are real GEMMs of
// the 32 x 32 real form of the 16-point DFT, [[C, S], [-S, C]] (C = cos,
// S = sin of 2 pi k n / 16), against 32 x 16 column blocks [Re; Im] of the
// data, on v_mfma_f32_16x16x32_{f16,bf16}: per stage 8 column blocks x 2
// output halves (real, imaginary) = 16 MFMAs, 48 with the split
// (hi*hi + hi*lo + lo*hi, where x = hi + lo, hi = round(x), lo = round(x - hi)).
// The radix-8 stage stays FP32 on the vector units: in the real form its
// 16 x 16 block would leave half of every K = 32 MFMA empty.  The 1/8 and
// 1/16 scalings are exact and keep every GEMM operand inside the fp16 range
// (|value| <= 32768 * sqrt 2) whatever the int16 input.
//
// Data movement: a wavefront owns an LDS region of two planes (real,
// imaginary).  The radix-8 stage writes plane[k3][n2][n1] (rows padded so the
// GEMM operand reads of lanes n1 = 0..15 and both n2 halves are conflict
// free); GEMM 1 reads every operand block into registers, then writes
// plane[n1][k3 + 8 k2]; GEMM 2 reads those blocks, and its outputs (lane
// (r, q) of column block t holds bins 16 t + r + 128 (4 q + i), i = 0..3)
// go to the region as the spectrum at the used subcarriers, spec[d].
//
// mfma_estimate_kernel: LS H = spec * pilot factor (paper Sec. II-B; II-C LS).
// mfma_demod_kernel: per (slot, data symbol), the wavefronts split the
// antennas; lane l accumulates conj(H) Y and |H|^2 of subcarriers l + 64 j
// (paper Sec. II-C, MRC), then a fixed-order cross-wave sum, x = z / g,
// decisions and packed bits.
// mfma_fft_kernel: the whole spectrum of every symbol (FFT validation).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rx_fft.hpp"
#include "rx_launch.h"

namespace rx {
namespace mf {

constexpr int N = 2048;
constexpr int kWaves = 4;
constexpr int RA = 288;                 // plane A row pitch (k3 rows of 16 x 16 + pad)
constexpr int RB = 130;                 // plane B row pitch (n1 rows of 128 columns + pad)
constexpr int kPlane = 8 * RA;          // floats per plane (>= 16 * RB)
constexpr int kIm = kPlane + 8;         // offset of the imaginary plane (bank shift)
constexpr int kWaveFloats = kIm + kPlane;  // 4616 floats = 18.5 KB per wavefront
static_assert(16 * RB <= kPlane, "plane B fits");
static_assert(2 * N <= kWaveFloats, "spectrum fits");
static_assert(3 * 1536 <= kWaveFloats, "demod partial sums fit");

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Vec8;
template <>
struct Vec8<_Float16> {
  typedef _Float16 type __attribute__((ext_vector_type(8)));
};
template <>
struct Vec8<__bf16> {
  typedef __bf16 type __attribute__((ext_vector_type(8)));
};

template <typename T>
__device__ __forceinline__ f32x4 mfma(const typename Vec8<T>::type& a, const typename Vec8<T>::type& b,
                                      const f32x4& c) {
  if constexpr (sizeof(T) == 2 && __is_same(T, _Float16))
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// hi = round(x) in T, lo = round(x - hi) in T
template <typename T, bool SPLIT>
__device__ __forceinline__ void split8(const float (&x)[8], typename Vec8<T>::type& hi, typename Vec8<T>::type& lo) {
#pragma unroll
  for (int j = 0; j < 8; j++) {
    const T h = (T)x[j];
    hi[j] = h;
    if constexpr (SPLIT) lo[j] = (T)(x[j] - (float)h);
  }
}

// Real 32 x 32 form of the 16-point DFT as two 16 x 32 MFMA A operands:
// rows k (real outputs: tile 0, imaginary: tile 1), k-slots s = 8q + j:
// s < 16 multiplies Re x[s], s >= 16 multiplies Im x[s - 16].
template <typename T, bool SPLIT>
struct Dft16 {
  typename Vec8<T>::type hi[2], lo[2];
  __device__ __forceinline__ void init(int lane) {
    const int k = lane & 15, q = lane >> 4;
#pragma unroll
    for (int t = 0; t < 2; t++) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const int s = 8 * q + j, n = s & 15;
        float sn, cs;
        sincospif((float)((2 * k * n) & 31) / 16.0f, &sn, &cs);  // angle 2 pi k n / 16
        // Yr = sum cos Xr + sin Xi;  Yi = sum -sin Xr + cos Xi
        v[j] = (t == 0) ? (s < 16 ? cs : sn) : (s < 16 ? -sn : cs);
      }
      split8<T, SPLIT>(v, hi[t], lo[t]);
    }
  }
};

template <typename T, bool SPLIT>
__device__ __forceinline__ void gemm_block(const Dft16<T, SPLIT>& F, const typename Vec8<T>::type& bh,
                                           const typename Vec8<T>::type& bl, f32x4 (&acc)[2]) {
#pragma unroll
  for (int t = 0; t < 2; t++) {
    acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (SPLIT) {
      acc[t] = mfma<T>(F.lo[t], bh, acc[t]);
      acc[t] = mfma<T>(F.hi[t], bl, acc[t]);
    }
    acc[t] = mfma<T>(F.hi[t], bh, acc[t]);
  }
}

// One 2048-point transform of the symbol at `sym` (one dword per complex
// int16 sample).  On return the wavefront's region holds the spectrum
// (interleaved complex) either at used subcarriers (spec[d], U of them) or,
// with FULL, at every bin k.  Ends with a wave fence.
template <typename T, bool SPLIT, bool FULL>
__device__ __forceinline__ void fft2048(const uint32_t* __restrict__ sym, float* __restrict__ wb,
                                        const float2* __restrict__ tw, const Dft16<T, SPLIT>& F, int U) {
  const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
  float* re = wb;
  float* im = wb + kIm;
  // ---- stage A: radix 8 over n3 for columns c1 = lane + 64 i (n1 = r, n2 = q + 4 i)
  {
    uint32_t raw[4][8];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int n3 = 0; n3 < 8; n3++) raw[i][n3] = __builtin_nontemporal_load(sym + lane + 64 * i + 256 * n3);
#pragma unroll
    for (int i = 0; i < 4; i++) {
      float2 v[8];
#pragma unroll
      for (int n3 = 0; n3 < 8; n3++) v[n3] = iq_to_float(raw[i][n3]);
      dft8(v, 0);
      const int n2 = q + 4 * i;
#pragma unroll
      for (int k3 = 0; k3 < 8; k3++) {
        const float2 w = k3 ? tw[(16 * n2 * k3) & (N - 1)] : make_float2(1.f, 0.f);
        const float2 a = cmul(v[k3], w);
        const int addr = k3 * RA + n2 * 16 + (n2 >> 3) * 16 + r;
        re[addr] = a.x * 0.125f;
        im[addr] = a.y * 0.125f;
      }
    }
  }
  wave_fence();
  // ---- GEMM 1: radix 16 over n2, column block t = k3, column r = n1
  typename Vec8<T>::type bh[8], bl[8];
#pragma unroll
  for (int t = 0; t < 8; t++) {
    const float* p = ((q >> 1) ? im : re) + t * RA + (8 * (q & 1)) * 16 + (q & 1) * 16 + r;
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; j++) x[j] = p[16 * j];
    split8<T, SPLIT>(x, bh[t], bl[t]);
  }
  wave_fence();  // every lane's reads precede any lane's writes
#pragma unroll
  for (int t = 0; t < 8; t++) {
    f32x4 acc[2];
    gemm_block<T, SPLIT>(F, bh[t], bl[t], acc);
    // lane holds B[n1 = r][k2 = 4q + i][k3 = t]
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int k2 = 4 * q + i;
      const int e = (r * (t + 8 * k2)) & (N - 1);
      const float2 w = e ? tw[e] : make_float2(1.f, 0.f);
      const float2 b = cmul(make_float2(acc[0][i], acc[1][i]), w);
      const int addr = r * RB + t + 8 * k2;
      re[addr] = b.x * 0.0625f;
      im[addr] = b.y * 0.0625f;
    }
  }
  wave_fence();
  // ---- GEMM 2: radix 16 over n1, column block t, column j' = 16 t + r = k3 + 8 k2
#pragma unroll
  for (int t = 0; t < 8; t++) {
    const float* p = ((q >> 1) ? im : re) + (8 * (q & 1)) * RB + 16 * t + r;
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; j++) x[j] = p[RB * j];
    split8<T, SPLIT>(x, bh[t], bl[t]);
  }
  wave_fence();
  float2* spec = reinterpret_cast<float2*>(wb);
  const int h = U >> 1;
#pragma unroll
  for (int t = 0; t < 8; t++) {
    f32x4 acc[2];
    gemm_block<T, SPLIT>(F, bh[t], bl[t], acc);
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int k = 16 * t + r + 128 * (4 * q + i);
      const float2 y = make_float2(acc[0][i] * 128.0f, acc[1][i] * 128.0f);
      if constexpr (FULL) {
        spec[k] = y;
      } else {
        // used subcarrier of bin k (fftshift order, DC excluded)
        const int d = (k >= 1 && k <= h) ? k - 1 + h : (k >= N - h ? k - (N - h) : -1);
        if (d >= 0) spec[d] = y;
      }
    }
  }
  wave_fence();
}

// ------------------------------------------------------------------ estimate
// Workgroup = (slot, 4 antennas x J jobs); wavefront w transforms antennas
// a0 + w, a0 + w + 4, ...
template <typename T, bool SPLIT>
__global__ __launch_bounds__(64 * kWaves) void mfma_estimate_kernel(const uint32_t* __restrict__ iq, int A, int T_,
                                                                    int CP, int U, const float2* __restrict__ tw,
                                                                    const float2* __restrict__ pf,
                                                                    float2* __restrict__ H, int blocks_per_slot,
                                                                    int jobs) {
  extern __shared__ __align__(16) float smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float* wb = smem + wave * kWaveFloats;
  Dft16<T, SPLIT> F;
  F.init(lane);
  const int64_t s = blockIdx.x / blocks_per_slot;
  const int blk = blockIdx.x % blocks_per_slot;
  const uint32_t* slot = iq + s * (int64_t)T_ * A * (N + CP);
  for (int j = 0; j < jobs; j++) {
    const int a = (blk * jobs + j) * kWaves + wave;
    if (a >= A) break;
    fft2048<T, SPLIT, false>(slot + (int64_t)a * (N + CP) + CP, wb, tw, F, U);
    const float2* spec = reinterpret_cast<const float2*>(wb);
    float2* hrow = H + (s * A + a) * (int64_t)U;
    for (int d = lane; d < U; d += 64) hrow[d] = cmul(spec[d], pf[d]);
    wave_fence();  // the next transform overwrites the region
  }
}

// ------------------------------------------------------------------ demod
constexpr int kMaxJ = 24;  // subcarriers per lane: U <= 64 * kMaxJ (the plan allows U <= 1536)

template <typename T, bool SPLIT, int J>
__global__ __launch_bounds__(64 * kWaves) void mfma_demod_kernel(const uint32_t* __restrict__ iq, int64_t S, int A,
                                                                 int T_, int CP, int U, int B,
                                                                 const float2* __restrict__ tw,
                                                                 const float2* __restrict__ H,
                                                                 float2* __restrict__ xhat,
                                                                 uint8_t* __restrict__ bits) {
  extern __shared__ __align__(16) float smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float* wb = smem + wave * kWaveFloats;
  Dft16<T, SPLIT> F;
  F.init(lane);
  const int Td = T_ - 1;
  const int64_t s = blockIdx.x / Td;
  const int t = 1 + (int)(blockIdx.x % Td);
  const uint32_t* symrow = iq + ((s * T_ + t) * A) * (int64_t)(N + CP) + CP;
  const float2* Hs = H + s * A * (int64_t)U;
  float2 z[J];
  float g[J];
#pragma unroll
  for (int j = 0; j < J; j++) {
    z[j] = make_float2(0.f, 0.f);
    g[j] = 0.f;
  }
  for (int a = wave; a < A; a += kWaves) {
    fft2048<T, SPLIT, false>(symrow + (int64_t)a * (N + CP), wb, tw, F, U);
    const float2* spec = reinterpret_cast<const float2*>(wb);
    const float2* hrow = Hs + (int64_t)a * U;
#pragma unroll
    for (int j = 0; j < J; j++) {
      const int d = lane + 64 * j;
      if (d < U) {
        const float2 y = spec[d], h = hrow[d];
        z[j].x = fmaf(h.x, y.x, fmaf(h.y, y.y, z[j].x));  // conj(h) * y
        z[j].y = fmaf(h.x, y.y, fmaf(-h.y, y.x, z[j].y));
        g[j] = fmaf(h.x, h.x, fmaf(h.y, h.y, g[j]));
      }
    }
    wave_fence();  // the next transform overwrites the region
  }
  // fixed-order cross-wave reduction: wave w stores its sums in its region
  float* mine = wb;
#pragma unroll
  for (int j = 0; j < J; j++) {
    const int d = lane + 64 * j;
    if (d < U) {
      mine[3 * d] = z[j].x;
      mine[3 * d + 1] = z[j].y;
      mine[3 * d + 2] = g[j];
    }
  }
  __syncthreads();
  const int row_bytes = U * B / 8;
  const int64_t out_row = s * Td + (t - 1);
  const float c16 = 3.16227766016837933f;  // sqrt(10)
  const float c64 = 6.48074069840786023f;  // sqrt(42)
  for (int qd = threadIdx.x; 4 * qd < U; qd += 64 * kWaves) {
    const int nsym = min(4, U - 4 * qd);
    uint32_t accb = 0;
    for (int e = 0; e < nsym; e++) {
      const int d = 4 * qd + e;
      float zx = 0.f, zy = 0.f, gg = 0.f;
      for (int w = 0; w < kWaves; w++) {
        const float* p = smem + w * kWaveFloats + 3 * d;
        zx += p[0];
        zy += p[1];
        gg += p[2];
      }
      const float2 x = gg > 0.f ? make_float2(zx / gg, zy / gg) : make_float2(0.f, 0.f);
      if (xhat) xhat[out_row * U + d] = x;
      uint32_t br[3] = {0, 0, 0}, bi[3] = {0, 0, 0};
      br[0] = x.x < 0.f;
      bi[0] = x.y < 0.f;
      if (B == 4) {
        br[1] = fabsf(x.x) * c16 > 2.f;
        bi[1] = fabsf(x.y) * c16 > 2.f;
      } else if (B == 6) {
        const float ur = fabsf(x.x) * c64, ui = fabsf(x.y) * c64;
        br[1] = ur > 4.f;
        bi[1] = ui > 4.f;
        br[2] = fabsf(ur - 4.f) > 2.f;
        bi[2] = fabsf(ui - 4.f) > 2.f;
      }
      for (int j = 0; j < B / 2; j++) accb = (accb << 2) | (br[j] << 1) | bi[j];
    }
    if (bits) {
      const int nbits = nsym * B;
      uint8_t* o = bits + out_row * row_bytes + (qd * B) / 2;
      for (int byte = 0; byte < nbits / 8; byte++) o[byte] = (uint8_t)(accb >> (nbits - 8 * (byte + 1)));
    }
  }
}

// ------------------------------------------------------------------ FFT only
template <typename T, bool SPLIT>
__global__ __launch_bounds__(64 * kWaves) void mfma_fft_kernel(const uint32_t* __restrict__ iq, int64_t n_sym_total,
                                                               int CP, const float2* __restrict__ tw,
                                                               float2* __restrict__ Y) {
  extern __shared__ __align__(16) float smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float* wb = smem + wave * kWaveFloats;
  Dft16<T, SPLIT> F;
  F.init(lane);
  const int64_t sym = (int64_t)blockIdx.x * kWaves + wave;  // flat (slot, symbol, antenna)
  if (sym >= n_sym_total) return;
  fft2048<T, SPLIT, true>(iq + sym * (N + CP) + CP, wb, tw, F, 0);
  const float2* spec = reinterpret_cast<const float2*>(wb);
  float2* out = Y + sym * N;
  for (int k = lane; k < N; k += 64) out[k] = spec[k];
}

}  // namespace mf

// ------------------------------------------------------------------ launchers
namespace {
constexpr size_t kLds = sizeof(float) * mf::kWaveFloats * mf::kWaves;  // 73.9 KB

template <typename K>
hipError_t allow(K k) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kLds);
}

template <typename T, bool SPLIT>
hipError_t est(const LaunchArgs& la, float2* H) {
  const int jobs = 2;
  const int per_blk = mf::kWaves * jobs;
  const int bps = (la.A + per_blk - 1) / per_blk;
  auto k = mf::mfma_estimate_kernel<T, SPLIT>;
  hipError_t e = allow(k);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3((unsigned)(la.S * bps)), dim3(64 * mf::kWaves), kLds, la.stream, la.iq, la.A, la.T,
                     la.CP, la.U, la.tw, la.pf, H, bps, jobs);
  return hipGetLastError();
}

template <typename T, bool SPLIT, int J>
hipError_t dem_j(const LaunchArgs& la, const float2* H, float2* xhat, uint8_t* bits) {
  auto k = mf::mfma_demod_kernel<T, SPLIT, J>;
  hipError_t e = allow(k);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3((unsigned)(la.S * (la.T - 1))), dim3(64 * mf::kWaves), kLds, la.stream, la.iq, la.S,
                     la.A, la.T, la.CP, la.U, la.B, la.tw, H, xhat, bits);
  return hipGetLastError();
}

template <typename T, bool SPLIT>
hipError_t dem(const LaunchArgs& la, const float2* H, float2* xhat, uint8_t* bits) {
  const int j = (la.U + 63) / 64;
  if (j <= 8) return dem_j<T, SPLIT, 8>(la, H, xhat, bits);
  if (j <= 19) return dem_j<T, SPLIT, 19>(la, H, xhat, bits);
  return dem_j<T, SPLIT, mf::kMaxJ>(la, H, xhat, bits);
}

template <typename T, bool SPLIT>
hipError_t fft(const LaunchArgs& la, float2* Y) {
  const int64_t total = la.S * la.T * la.A;
  auto k = mf::mfma_fft_kernel<T, SPLIT>;
  hipError_t e = allow(k);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3((unsigned)((total + mf::kWaves - 1) / mf::kWaves)), dim3(64 * mf::kWaves), kLds,
                     la.stream, la.iq, total, la.CP, la.tw, Y);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_mfma_estimate(const LaunchArgs& la, float2* H) {
  switch (la.fft_mode) {
    case 1: return est<_Float16, false>(la, H);
    case 2: return est<__bf16, false>(la, H);
    case 3: return est<_Float16, true>(la, H);
    case 4: return est<__bf16, true>(la, H);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_mfma_demod(const LaunchArgs& la, const float2* H, float2* xhat, uint8_t* bits) {
  switch (la.fft_mode) {
    case 1: return dem<_Float16, false>(la, H, xhat, bits);
    case 2: return dem<__bf16, false>(la, H, xhat, bits);
    case 3: return dem<_Float16, true>(la, H, xhat, bits);
    case 4: return dem<__bf16, true>(la, H, xhat, bits);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_mfma_fft(const LaunchArgs& la, float2* Y) {
  switch (la.fft_mode) {
    case 1: return fft<_Float16, false>(la, Y);
    case 2: return fft<__bf16, false>(la, Y);
    case 3: return fft<_Float16, true>(la, Y);
    case 4: return fft<__bf16, true>(la, Y);
  }
  return hipErrorInvalidValue;
}

}  // namespace rx
