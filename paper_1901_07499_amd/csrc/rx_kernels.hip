// rx_kernels.hip -- HIP kernels of the uplink receive path for gfx950.
//
// estimate_kernel  pilot symbol of every (slot, antenna): int16 load with the
//                  CP skipped, FFT, LS divide by the pilot (paper Sec. II-B;
//                  Sec. II-C, LS paragraph), H written in subcarrier order
//                  straight from the FFT's output registers.
// demod_kernel     one workgroup per (slot, data symbol): its wavefronts split
//                  the antennas, FFT each antenna's symbol and accumulate the
//                  MRC sums conj(H) Y and |H|^2 of the used subcarriers from
//                  the FFT's output registers (paper Sec. II-C, MRC
//                  paragraph); a fixed-order cross-wave reduction in LDS
//                  follows, then x = z / g, hard decisions and packed bits.
//                  ZF (one user) instead weights every antenna by conj(H)/g,
//                  with g summed first.
//
// After the FFT a lane holds bins li + L*q, q = 0..P-1 (see rx_fft.hpp).  The
// used subcarriers are the bins within U/2 of DC, so only the registers
// q < QH and q >= P - QH (QH = ceil((U/2 + 1) / L)) can hold one: the demod
// kernel is instantiated for a window of 2*QH registers and the other FFT
// outputs are never computed.
// g_kernel         g[s][d] = sum_a |H[s][a][d]|^2 for the estimate call.
// fft_kernel       CP removal + FFT only (validation of the FFT stage).
//
// Subcarrier d (0..U-1) is FFT bin k_d: d + N - U/2 for d < U/2, else
// d - U/2 + 1 (fftshift order without DC).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rx_fft.hpp"
#include "rx_launch.h"

// Tuning constants (compile time): wavefronts per demod workgroup and the
// minimum wavefronts per SIMD the demod kernel's register budget must allow.
#ifndef RX_DEMOD_WAVES
#define RX_DEMOD_WAVES 4
#endif
#ifndef RX_DEMOD_MIN_WAVES_PER_EU
#define RX_DEMOD_MIN_WAVES_PER_EU 1
#endif
// Symbols a demod wavefront transforms side by side per loop iteration when
// one transform fills the wavefront (N >= 1024): independent work that hides
// the LDS round trips between FFT passes.
#ifndef RX_DEMOD_ILP
#define RX_DEMOD_ILP 1
#endif
// How many jobs ahead a demod wavefront requests its input samples (1 or 2).
#ifndef RX_DEMOD_PREFETCH
#define RX_DEMOD_PREFETCH 1
#endif

namespace rx {

// Used-subcarrier index of FFT bin k (0 <= k < n), or -1 when the bin is not
// used: bins 1..U/2 are subcarriers U/2..U-1, bins n-U/2..n-1 are 0..U/2-1.
__device__ __forceinline__ int sub_of_bin(int k, int n, int u) {
  const int h = u >> 1;
  if (k >= 1 && k <= h) return k - 1 + h;
  if (k >= n - h) return k - (n - h);
  return -1;
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
  __shared__ float2 twtab[FftTwiddles<N>::kLdsFloat2 > 0 ? FftTwiddles<N>::kLdsFloat2 : 1];
  if constexpr (FftTwiddles<N>::kLdsLast) {
    FftTwiddles<N>::P3Lds::fill(twtab, tw, threadIdx.x, blockDim.x);
    __syncthreads();
  }
  if (a0 >= A) return;  // no workgroup barrier below
  const int a = a0 + f;
  const bool valid = a < A;
  const uint32_t* rec = iq + ((s * T) * A + (valid ? a : a0)) * (int64_t)(N + CP) + CP;
  uint32_t raw[Sh::P];
  load_symbol<N>(raw, rec, li, valid);
  FftTwiddles<N> twr;
  twr.load(tw, li, twtab);
  float2 v[Sh::P];
  unpack_symbol<N>(v, raw);
  fft_in_regs<N>(v, lds + (wave * Sh::F + f) * Lds<N>::kSlot, li, twr);
  if (valid) {
    float2* hrow = H + (s * A + a) * (int64_t)U;
#pragma unroll
    for (int q = 0; q < Sh::P; q++) {
      const int d = sub_of_bin(li + Sh::L * q, N, U);
      if (d >= 0) hrow[d] = cmul(v[Spectrum<N>::reg(q)], pf[d]);
    }
  }
}

// ------------------------------------------------------------------ demod
template <int N, int QH, int W, bool ZF>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(RX_DEMOD_MIN_WAVES_PER_EU)))
void demod_kernel(const uint32_t* __restrict__ iq, int64_t S, int A, int T, int CP, int U, int B,
                  const float2* __restrict__ tw, const float2* __restrict__ H, float2* __restrict__ xhat,
                  uint8_t* __restrict__ bits) {
  using Sh = FftShape<N>;
  constexpr int NI = 2 * QH;  // spectrum registers that can hold a used subcarrier
  static_assert(NI <= Sh::P, "window wider than the lane's spectrum");
  extern __shared__ float2 lds[];
  const int Td = T - 1;
  const int64_t item = xcd_remap(blockIdx.x, S * Td);
  const int64_t s = item / Td;
  const int t = 1 + (int)(item % Td);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int f = lane / Sh::L, li = lane % Sh::L;
  const float2* Hs = H + s * A * (int64_t)U;

  // Window register i holds spectrum register q(i) = i (i < QH, bins
  // li + L*i above DC) or P - NI + i (bins below N, i.e. negative
  // frequencies).  Its subcarrier is li + doff(i) when wok(i).  Channel
  // loads use that index clamped into [0, U): a lane whose bin is unused
  // reads some in-bounds value and its (meaningless) sum is never stored, so
  // the loop needs no per-lane branches.
  const int hU = U >> 1;
  auto qof = [](int i) { return i < QH ? i : Sh::P - NI + i; };
  auto doff = [&](int i) { return Sh::L * qof(i) + (i < QH ? hU - 1 : hU - N); };
  auto wok = [&](int i) {
    const int k = li + Sh::L * qof(i);
    return i < QH ? (k >= 1 && k <= hU) : (k >= N - hU);
  };
  auto dcl = [&](int i) { return min(max(li + doff(i), 0), U - 1); };
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
        const float2 h = Hs[(int64_t)a * U + dcl(i)];
        g[i] = fmaf(h.x, h.x, fmaf(h.y, h.y, g[i]));
      }
    }
#pragma unroll
    for (int i = 0; i < NI; i++) g[i] = g[i] > 0.f ? 1.0f / g[i] : 0.f;  // now 1/g
  }

  // C symbols (antennas) per lane per iteration; antenna of lane group f and
  // slot c in job J: J*F*C + c*F + f.  Job J = iteration * W + wave.
  constexpr int C = Sh::F == 1 ? RX_DEMOD_ILP : 1;
  float2* bufs[C];
#pragma unroll
  for (int c = 0; c < C; c++) bufs[c] = lds + ((wave * C + c) * Sh::F + f) * Lds<N>::kSlot;
  float2* const(&buf)[C] = bufs;
  const int64_t sym_base = ((s * T + t) * A) * (int64_t)(N + CP) + CP;
  __shared__ float2 twtab[FftTwiddles<N>::kLdsFloat2 > 0 ? FftTwiddles<N>::kLdsFloat2 : 1];
  if constexpr (FftTwiddles<N>::kLdsLast) {
    FftTwiddles<N>::P3Lds::fill(twtab, tw, threadIdx.x, blockDim.x);
    __syncthreads();
  }
  FftTwiddles<N> twr;
  twr.load(tw, li, twtab);
  // Software pipeline over this wavefront's antennas: each job's samples are
  // requested D jobs ahead.
  constexpr int JA = Sh::F * C;  // antennas per job
  const int a_step = W * JA;
  int a0 = wave * JA;
  constexpr int D = RX_DEMOD_PREFETCH;
  static_assert(D == 1 || D == 2, "prefetch depth 1 or 2");
  auto request = [&](uint32_t (&dst)[C][Sh::P], int aj) {
#pragma unroll
    for (int c = 0; c < C; c++) {
      const int a = aj + c * Sh::F + f;
      load_symbol<N>(dst[c], iq + sym_base + (int64_t)(a < A ? a : aj) * (N + CP), li, a < A);
    }
  };
  // One job: its samples are in `cur`; once unpacked, `cur` is refilled with
  // the samples of the job D steps ahead (after this job's channel rows were
  // requested: vector loads complete in issue order, so waiting for the rows
  // does not wait for those later sample loads).
  auto job = [&](uint32_t (&cur)[C][Sh::P], int aj) {
    float2 v[C][Sh::P];
#pragma unroll
    for (int c = 0; c < C; c++) unpack_symbol<N>(v[c], cur[c]);
    fft_first_pass<N, C>(v, buf, li);
    float2 h[C][NI];
#pragma unroll
    for (int c = 0; c < C; c++) {
      const int a = aj + c * Sh::F + f;
      const bool ok = a < A;
      const float2* hrow = Hs + (int64_t)(ok ? a : aj) * U;
#pragma unroll
      for (int i = 0; i < NI; i++) {
        const float2 hv = hrow[dcl(i)];
        // a lane group whose antenna is past A must add nothing to its row
        h[c][i] = (Sh::F == 1 || ok) ? hv : make_float2(0.f, 0.f);
      }
    }
    if (aj + D * a_step < A) request(cur, aj + D * a_step);
    fft_rest<N, C>(v, buf, li, twr);
#pragma unroll
    for (int c = 0; c < C; c++)
#pragma unroll
      for (int i = 0; i < NI; i++) {
        const int q = i < QH ? i : Sh::P - NI + i;
        const float2 y = v[c][Spectrum<N>::reg(q)];
        const float2 hh = h[c][i];  // zero for antennas past A
        if constexpr (ZF) {
          const float2 w = make_float2(hh.x * g[i], -hh.y * g[i]);  // conj(h) / g
          z[i].x = fmaf(w.x, y.x, fmaf(-w.y, y.y, z[i].x));
          z[i].y = fmaf(w.x, y.y, fmaf(w.y, y.x, z[i].y));
        } else {
          z[i].x = fmaf(hh.x, y.x, fmaf(hh.y, y.y, z[i].x));  // conj(h) * y
          z[i].y = fmaf(hh.x, y.y, fmaf(-hh.y, y.x, z[i].y));
          g[i] = fmaf(hh.x, hh.x, fmaf(hh.y, hh.y, g[i]));
        }
      }
    wave_fence();  // this job's LDS reads precede the next job's writes
  };
  // D sample buffers used round robin by a loop unrolled D times, so no
  // register copies (which would wait for the loads) are needed.
  uint32_t nxt[D][C][Sh::P];
#pragma unroll
  for (int d = 0; d < D; d++)
    if (a0 + d * a_step < A) request(nxt[d], a0 + d * a_step);
  for (; a0 < A; a0 += D * a_step) {
    job(nxt[0], a0);
    if constexpr (D == 2) {
      if (a0 + a_step < A) job(nxt[1], a0 + a_step);
    }
  }

  // Cross-wave reduction in a fixed order: row = wave * F + f holds the
  // partial sums of one group of antennas for every used subcarrier (each
  // subcarrier sits in exactly one lane of a transform's lane group; h = 0
  // made invalid antennas contribute zeros).
  constexpr int ROWS = W * Sh::F;
  __syncthreads();
  float2* rz = lds;                                      // [ROWS][U]
  float* rg = reinterpret_cast<float*>(lds + ROWS * U);  // [ROWS][U]
  const int row = wave * Sh::F + f;
#pragma unroll
  for (int i = 0; i < NI; i++) {
    if (wok(i)) {
      rz[row * U + li + doff(i)] = z[i];
      if constexpr (!ZF) rg[row * U + li + doff(i)] = g[i];
    }
  }
  __syncthreads();

  const int row_bytes = U * B / 8;
  const int64_t out_row = s * Td + (t - 1);
  const float c16 = 3.16227766016837933f;  // sqrt(10)
  const float c64 = 6.48074069840786023f;  // sqrt(42)
  for (int qd = threadIdx.x; 4 * qd < U; qd += 64 * W) {
    const int nsym = min(4, U - 4 * qd);
    uint32_t acc = 0;  // bits of up to 4 symbols, MSB-first
    for (int e = 0; e < nsym; e++) {
      const int d = 4 * qd + e;
      float2 zz = make_float2(0.f, 0.f);
      float gg = 0.f;
      for (int w = 0; w < ROWS; w++) {
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
      const int nbits = nsym * B;                                // a multiple of 8
      uint8_t* o = bits + out_row * row_bytes + (qd * B) / 2;   // 4 symbols = B/2 bytes
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
  __shared__ float2 twtab[FftTwiddles<N>::kLdsFloat2 > 0 ? FftTwiddles<N>::kLdsFloat2 : 1];
  if constexpr (FftTwiddles<N>::kLdsLast) {
    FftTwiddles<N>::P3Lds::fill(twtab, tw, threadIdx.x, blockDim.x);
    __syncthreads();
  }
  if (a0 >= A) return;  // no workgroup barrier below
  const int a = a0 + f;
  const bool valid = a < A;
  const uint32_t* rec = iq + (st * A + (valid ? a : a0)) * (int64_t)(N + CP) + CP;
  uint32_t raw[Sh::P];
  load_symbol<N>(raw, rec, li, valid);
  FftTwiddles<N> twr;
  twr.load(tw, li, twtab);
  float2 v[Sh::P];
  unpack_symbol<N>(v, raw);
  fft_in_regs<N>(v, lds + (wave * Sh::F + f) * Lds<N>::kSlot, li, twr);
  if (valid) {
    float2* out = Y + (st * A + a) * (int64_t)N;
#pragma unroll
    for (int q = 0; q < Sh::P; q++) out[li + Sh::L * q] = v[Spectrum<N>::reg(q)];
  }
}

// ------------------------------------------------------------------ launchers
namespace {
constexpr int kWavesEst = 4;
constexpr int kWavesDemod = RX_DEMOD_WAVES;
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

template <int N, int QH, bool ZF>
hipError_t demod_qh(const LaunchArgs& la, const float2* H, float2* xhat, uint8_t* bits) {
  const int64_t grid = la.S * (la.T - 1);
  constexpr int C = FftShape<N>::F == 1 ? RX_DEMOD_ILP : 1;
  size_t lds = fft_lds_bytes<N>(kWavesDemod) * C;
  const size_t red = (size_t)kWavesDemod * FftShape<N>::F * la.U * (sizeof(float2) + sizeof(float));
  if (red > lds) lds = red;
  hipError_t e = allow_lds(demod_kernel<N, QH, kWavesDemod, ZF>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((demod_kernel<N, QH, kWavesDemod, ZF>), dim3((unsigned)grid), dim3(64 * kWavesDemod), lds,
                     la.stream, la.iq, la.S, la.A, la.T, la.CP, la.U, la.B, la.tw, H, xhat, bits);
  return hipGetLastError();
}

// Register-window tiers: the smallest instantiated QH >= ceil((U/2 + 1) / L).
template <int N, bool ZF>
hipError_t demod_n(const LaunchArgs& la, const float2* H, float2* xhat, uint8_t* bits) {
  constexpr int P = FftShape<N>::P, L = FftShape<N>::L;
  const int need = (la.U / 2 + 1 + L - 1) / L;
  if constexpr (P == 16) {
    if (need <= 2) return demod_qh<N, 2, ZF>(la, H, xhat, bits);
    if (need <= 4) return demod_qh<N, 4, ZF>(la, H, xhat, bits);
    if (need <= 5) return demod_qh<N, 5, ZF>(la, H, xhat, bits);
    if (need <= 8) return demod_qh<N, 8, ZF>(la, H, xhat, bits);
  } else {
    if (need <= 4) return demod_qh<N, 4, ZF>(la, H, xhat, bits);
    if (need <= 8) return demod_qh<N, 8, ZF>(la, H, xhat, bits);
    if (need <= 10) return demod_qh<N, 10, ZF>(la, H, xhat, bits);
    if (need <= 16) return demod_qh<N, 16, ZF>(la, H, xhat, bits);
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
