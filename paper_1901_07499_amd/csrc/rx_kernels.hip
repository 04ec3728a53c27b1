// rx_kernels.hip -- HIP kernels of the uplink receive path for gfx950.
//
// estimate_kernel  pilot symbol of every (slot, antenna): int16 load with the
//                  CP skipped, FFT, LS divide by the pilot (paper Sec. II-B;
//                  Sec. II-C, LS paragraph), H written in subcarrier order.
// demod_kernel     one workgroup per (slot, data symbol): its wavefronts split
//                  the antennas, FFT each antenna's symbol and accumulate the
//                  MRC sums conj(H) Y and |H|^2 per used subcarrier in VGPRs
//                  (paper Sec. II-C, MRC paragraph); a fixed-order cross-wave
//                  reduction in LDS follows, then x = z / g, hard decisions and
//                  packed bits.  ZF (one user) instead weights every antenna by
//                  conj(H)/g, with g summed first.
// g_kernel         g[s][d] = sum_a |H[s][a][d]|^2 for the estimate call.
// fft_kernel       CP removal + FFT only (validation of the FFT stage).
//
// Subcarrier d (0..U-1) is FFT bin k_d: d + N - U/2 for d < U/2, else
// d - U/2 + 1 (fftshift order without DC).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rx_fft.hpp"
#include "rx_launch.h"

namespace rx {

__device__ __forceinline__ int bin_of(int d, int n, int u) {
  return d < (u >> 1) ? d + n - (u >> 1) : d - (u >> 1) + 1;
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).
// Remap so that each XCD walks a contiguous range of work items: the
// workgroups of one slot then share an XCD and its L2, where the slot's
// channel estimate stays resident.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t n) {
  const int64_t q = n >> 3, r = n & 7;
  const int64_t x = b & 7, j = b >> 3;
  return (x < r) ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

// ------------------------------------------------------------------ estimate
template <int N, int W>
__global__ __launch_bounds__(64 * W) void estimate_kernel(const uint32_t* __restrict__ iq, int A, int T, int CP,
                                                          int U, const float2* __restrict__ tw,
                                                          const float2* __restrict__ pf, float2* __restrict__ H,
                                                          int blocks_per_slot) {
  using Sh = FftShape<N>;
  extern __shared__ float2 lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int f = lane / Sh::L, li = lane % Sh::L;
  const int64_t s = blockIdx.x / blocks_per_slot;
  const int blk = blockIdx.x % blocks_per_slot;
  const int a0 = (blk * W + wave) * Sh::F;
  if (a0 >= A) return;  // no workgroup barrier in this kernel
  const int a = a0 + f;
  const bool valid = a < A;
  const uint32_t* rec = iq + ((s * T) * A + (valid ? a : a0)) * (int64_t)(N + CP) + CP;
  uint32_t raw[Sh::P];
  load_symbol<N>(raw, rec, li, valid);
  float2 v[Sh::P];
  unpack_symbol<N>(v, raw);
  float2* slot = lds + (wave * Sh::F) * Lds<N>::kSlot;
  fft_to_lds<N>(v, slot + f * Lds<N>::kSlot, li, tw);
  for (int ff = 0; ff < Sh::F; ff++) {
    const int aa = a0 + ff;
    if (aa >= A) break;
    const float2* y = slot + ff * Lds<N>::kSlot;
    float2* hrow = H + (s * A + aa) * (int64_t)U;
    for (int d = lane; d < U; d += 64) hrow[d] = cmul(y[pad(bin_of(d, N, U))], pf[d]);
  }
}

// ------------------------------------------------------------------ demod
template <int N, int NI, int W, bool ZF>
__global__ __launch_bounds__(64 * W) void demod_kernel(const uint32_t* __restrict__ iq, int64_t S, int A, int T,
                                                       int CP, int U, int B, const float2* __restrict__ tw,
                                                       const float2* __restrict__ H, float2* __restrict__ xhat,
                                                       uint8_t* __restrict__ bits) {
  using Sh = FftShape<N>;
  extern __shared__ float2 lds[];
  const int Td = T - 1;
  const int64_t item = xcd_remap(blockIdx.x, S * Td);
  const int64_t s = item / Td;
  const int t = 1 + (int)(item % Td);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int f = lane / Sh::L, li = lane % Sh::L;
  const float2* Hs = H + s * A * (int64_t)U;

  int kofs[NI];
#pragma unroll
  for (int i = 0; i < NI; i++) {
    const int d = lane + 64 * i;
    kofs[i] = pad(bin_of(d < U ? d : 0, N, U));
  }
  float2 z[NI];
  float g[NI];
#pragma unroll
  for (int i = 0; i < NI; i++) {
    z[i] = make_float2(0.f, 0.f);
    g[i] = 0.f;
  }
  if constexpr (ZF) {
    // ZF weights need the full normaliser first: g over all antennas, in order.
    for (int a = 0; a < A; a++) {
#pragma unroll
      for (int i = 0; i < NI; i++) {
        const int d = lane + 64 * i;
        if (d < U) {
          const float2 h = Hs[(int64_t)a * U + d];
          g[i] = fmaf(h.x, h.x, fmaf(h.y, h.y, g[i]));
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NI; i++) g[i] = g[i] > 0.f ? 1.0f / g[i] : 0.f;  // now 1/g
  }

  float2* slot = lds + (wave * Sh::F) * Lds<N>::kSlot;
  const int64_t sym_base = ((s * T + t) * A) * (int64_t)(N + CP) + CP;
  for (int a0 = wave * Sh::F; a0 < A; a0 += W * Sh::F) {
    const int a = a0 + f;
    const bool valid = a < A;
    uint32_t raw[Sh::P];
    load_symbol<N>(raw, iq + sym_base + (int64_t)(valid ? a : a0) * (N + CP), li, valid);
    float2 v[Sh::P];
    unpack_symbol<N>(v, raw);
    fft_to_lds<N>(v, slot + f * Lds<N>::kSlot, li, tw);
    for (int ff = 0; ff < Sh::F; ff++) {
      const int aa = a0 + ff;
      if (aa >= A) break;
      const float2* y = slot + ff * Lds<N>::kSlot;
      const float2* hrow = Hs + (int64_t)aa * U;
#pragma unroll
      for (int i = 0; i < NI; i++) {
        const int d = lane + 64 * i;
        if (d < U) {
          const float2 yy = y[kofs[i]];
          const float2 h = hrow[d];
          if constexpr (ZF) {
            const float2 w = make_float2(h.x * g[i], -h.y * g[i]);  // conj(h) / g
            z[i].x = fmaf(w.x, yy.x, fmaf(-w.y, yy.y, z[i].x));
            z[i].y = fmaf(w.x, yy.y, fmaf(w.y, yy.x, z[i].y));
          } else {
            z[i].x = fmaf(h.x, yy.x, fmaf(h.y, yy.y, z[i].x));  // conj(h) * y
            z[i].y = fmaf(h.x, yy.y, fmaf(-h.y, yy.x, z[i].y));
            g[i] = fmaf(h.x, h.x, fmaf(h.y, h.y, g[i]));
          }
        }
      }
    }
    wave_fence();  // this job's LDS reads precede the next job's writes
  }

  // Cross-wave reduction, fixed order over waves.
  __syncthreads();
  float2* rz = lds;                                   // [W][U]
  float* rg = reinterpret_cast<float*>(lds + W * U);  // [W][U]
#pragma unroll
  for (int i = 0; i < NI; i++) {
    const int d = lane + 64 * i;
    if (d < U) {
      rz[wave * U + d] = z[i];
      if constexpr (!ZF) rg[wave * U + d] = g[i];
    }
  }
  __syncthreads();

  const int row_bytes = U * B / 8;
  const int64_t out_row = s * Td + (t - 1);
  const float c16 = 3.16227766016837933f;  // sqrt(10)
  const float c64 = 6.48074069840786023f;  // sqrt(42)
  for (int q = threadIdx.x; 4 * q < U; q += 64 * W) {
    const int nsym = min(4, U - 4 * q);
    uint32_t acc = 0;  // bits of up to 4 symbols, MSB-first
    for (int e = 0; e < nsym; e++) {
      const int d = 4 * q + e;
      float2 zz = make_float2(0.f, 0.f);
      float gg = 0.f;
#pragma unroll
      for (int w = 0; w < W; w++) {
        const float2 p = rz[w * U + d];
        zz.x += p.x;
        zz.y += p.y;
        if constexpr (!ZF) gg += rg[w * U + d];
      }
      float2 x;
      if constexpr (ZF) {
        x = zz;
      } else {
        x = gg > 0.f ? make_float2(zz.x / gg, zz.y / gg) : make_float2(0.f, 0.f);
      }
      if (xhat) xhat[out_row * U + d] = x;
      // hard decisions: strict comparisons, so ties and -0.0 give 0
      uint32_t br[3], bi[3];
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
      for (int j = 0; j < B / 2; j++) acc = (acc << 2) | (br[j] << 1) | bi[j];
    }
    if (bits) {
      const int nbits = nsym * B;  // a multiple of 8
      uint8_t* o = bits + out_row * row_bytes + (q * B) / 2;  // 4 symbols = B/2 bytes
      for (int byte = 0; byte < nbits / 8; byte++) o[byte] = (uint8_t)(acc >> (nbits - 8 * (byte + 1)));
    }
  }
}

// ------------------------------------------------------------------ g
__global__ void g_kernel(const float2* __restrict__ H, float* __restrict__ g, int64_t S, int A, int U,
                         int blocks_per_slot) {
  const int64_t s = blockIdx.x / blocks_per_slot;
  const int d = (blockIdx.x % blocks_per_slot) * blockDim.x + threadIdx.x;
  if (s >= S || d >= U) return;
  const float2* h = H + s * A * (int64_t)U + d;
  float acc = 0.f;
  for (int a = 0; a < A; a++) {
    const float2 v = h[(int64_t)a * U];
    acc = fmaf(v.x, v.x, fmaf(v.y, v.y, acc));
  }
  g[s * U + d] = acc;
}

// ------------------------------------------------------------------ FFT only
template <int N, int W>
__global__ __launch_bounds__(64 * W) void fft_kernel(const uint32_t* __restrict__ iq, int A, int T, int CP,
                                                     const float2* __restrict__ tw, float2* __restrict__ Y,
                                                     int blocks_per_sym) {
  using Sh = FftShape<N>;
  extern __shared__ float2 lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int f = lane / Sh::L, li = lane % Sh::L;
  const int64_t st = blockIdx.x / blocks_per_sym;  // s * T + t
  const int blk = blockIdx.x % blocks_per_sym;
  const int a0 = (blk * W + wave) * Sh::F;
  if (a0 >= A) return;
  const int a = a0 + f;
  const bool valid = a < A;
  const uint32_t* rec = iq + (st * A + (valid ? a : a0)) * (int64_t)(N + CP) + CP;
  uint32_t raw[Sh::P];
  load_symbol<N>(raw, rec, li, valid);
  float2 v[Sh::P];
  unpack_symbol<N>(v, raw);
  float2* slot = lds + (wave * Sh::F) * Lds<N>::kSlot;
  fft_to_lds<N>(v, slot + f * Lds<N>::kSlot, li, tw);
  for (int ff = 0; ff < Sh::F; ff++) {
    const int aa = a0 + ff;
    if (aa >= A) break;
    const float2* y = slot + ff * Lds<N>::kSlot;
    float2* out = Y + (st * A + aa) * (int64_t)N;
    for (int k = lane; k < N; k += 64) out[k] = y[pad(k)];
  }
}

// ------------------------------------------------------------------ launchers
namespace {
constexpr int kWavesEst = 4;
constexpr int kWavesDemod = 4;
constexpr int kWavesFft = 4;

template <int N>
size_t fft_lds_bytes(int waves) {
  return (size_t)waves * FftShape<N>::F * Lds<N>::kSlot * sizeof(float2);
}

// Dynamic LDS above 64 KB must be allowed per kernel before launching it.
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <int N>
hipError_t estimate_n(const LaunchArgs& la, float2* H) {
  using Sh = FftShape<N>;
  const int jobs = (la.A + Sh::F - 1) / Sh::F;
  const int bps = (jobs + kWavesEst - 1) / kWavesEst;
  const int64_t grid = la.S * bps;
  const size_t lds = fft_lds_bytes<N>(kWavesEst);
  hipError_t e = allow_lds(estimate_kernel<N, kWavesEst>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((estimate_kernel<N, kWavesEst>), dim3((unsigned)grid), dim3(64 * kWavesEst), lds, la.stream, la.iq, la.A, la.T, la.CP, la.U, la.tw, la.pf, H, bps);
  return hipGetLastError();
}

template <int N>
hipError_t fft_n(const LaunchArgs& la, float2* Y) {
  using Sh = FftShape<N>;
  const int jobs = (la.A + Sh::F - 1) / Sh::F;
  const int bps = (jobs + kWavesFft - 1) / kWavesFft;
  const int64_t grid = la.S * la.T * bps;
  const size_t lds = fft_lds_bytes<N>(kWavesFft);
  hipError_t e = allow_lds(fft_kernel<N, kWavesFft>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((fft_kernel<N, kWavesFft>), dim3((unsigned)grid), dim3(64 * kWavesFft), lds, la.stream, la.iq, la.A, la.T, la.CP, la.tw, Y, bps);
  return hipGetLastError();
}

template <int N, int NI, bool ZF>
hipError_t demod_ni(const LaunchArgs& la, const float2* H, float2* xhat, uint8_t* bits) {
  const int64_t grid = la.S * (la.T - 1);
  size_t lds = fft_lds_bytes<N>(kWavesDemod);
  const size_t red = (size_t)kWavesDemod * la.U * (sizeof(float2) + sizeof(float));
  if (red > lds) lds = red;
  hipError_t e = allow_lds(demod_kernel<N, NI, kWavesDemod, ZF>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((demod_kernel<N, NI, kWavesDemod, ZF>), dim3((unsigned)grid), dim3(64 * kWavesDemod), lds,
                     la.stream, la.iq, la.S, la.A, la.T, la.CP, la.U, la.B, la.tw, H, xhat, bits);
  return hipGetLastError();
}

// Accumulator tiers: the smallest tier holding ceil(U/64) subcarriers per lane.
template <int N, bool ZF>
hipError_t demod_n(const LaunchArgs& la, const float2* H, float2* xhat, uint8_t* bits) {
  const int need = (la.U + 63) / 64;
  constexpr int cap = (N - 2 + 63) / 64;
  if (need <= 1) return demod_ni<N, 1, ZF>(la, H, xhat, bits);
  if (need <= 2) return demod_ni<N, (cap < 2 ? cap : 2), ZF>(la, H, xhat, bits);
  if constexpr (cap >= 4) {
    if (need <= 4) return demod_ni<N, 4, ZF>(la, H, xhat, bits);
  }
  if constexpr (cap >= 8) {
    if (need <= 8) return demod_ni<N, 8, ZF>(la, H, xhat, bits);
  }
  if constexpr (cap >= 16) {
    if (need <= 10) return demod_ni<N, 10, ZF>(la, H, xhat, bits);
    if (need <= 16) return demod_ni<N, 16, ZF>(la, H, xhat, bits);
  }
  if constexpr (cap >= 32) {
    if (need <= 19) return demod_ni<N, 19, ZF>(la, H, xhat, bits);
    if (need <= 24) return demod_ni<N, 24, ZF>(la, H, xhat, bits);
    if (need <= 32) return demod_ni<N, 32, ZF>(la, H, xhat, bits);
  }
  return hipErrorInvalidValue;
}

template <bool ZF>
hipError_t demod_dispatch(const LaunchArgs& la, const float2* H, float2* xhat, uint8_t* bits) {
  switch (la.N) {
    case 64: return demod_n<64, ZF>(la, H, xhat, bits);
    case 128: return demod_n<128, ZF>(la, H, xhat, bits);
    case 256: return demod_n<256, ZF>(la, H, xhat, bits);
    case 512: return demod_n<512, ZF>(la, H, xhat, bits);
    case 1024: return demod_n<1024, ZF>(la, H, xhat, bits);
    case 2048: return demod_n<2048, ZF>(la, H, xhat, bits);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

hipError_t launch_estimate(const LaunchArgs& la, float2* H) {
  switch (la.N) {
    case 64: return estimate_n<64>(la, H);
    case 128: return estimate_n<128>(la, H);
    case 256: return estimate_n<256>(la, H);
    case 512: return estimate_n<512>(la, H);
    case 1024: return estimate_n<1024>(la, H);
    case 2048: return estimate_n<2048>(la, H);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_g(const LaunchArgs& la, const float2* H, float* g) {
  const int bs = 256;
  const int bps = (la.U + bs - 1) / bs;
  hipLaunchKernelGGL(g_kernel, dim3((unsigned)(la.S * bps)), dim3(bs), 0, la.stream, H, g, la.S, la.A, la.U, bps);
  return hipGetLastError();
}

hipError_t launch_demod(const LaunchArgs& la, bool zf, const float2* H, float2* xhat, uint8_t* bits) {
  return zf ? demod_dispatch<true>(la, H, xhat, bits) : demod_dispatch<false>(la, H, xhat, bits);
}

hipError_t launch_fft(const LaunchArgs& la, float2* Y) {
  switch (la.N) {
    case 64: return fft_n<64>(la, Y);
    case 128: return fft_n<128>(la, Y);
    case 256: return fft_n<256>(la, Y);
    case 512: return fft_n<512>(la, Y);
    case 1024: return fft_n<1024>(la, Y);
    case 2048: return fft_n<2048>(la, Y);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rx
