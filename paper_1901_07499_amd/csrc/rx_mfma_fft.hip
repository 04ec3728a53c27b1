// rx_mfma_fft.hip -- the receive path with the 2048-point FFT recast as
// DFT-stage GEMMs on the fp16 / bf16 matrix cores (gfx950), FP32 accumulate,
// optionally with a hi+lo split of both operands (three products per GEMM).
// The transform is the FFT of every antenna's symbol after CP removal (paper
// Sec. II-B, Sec. II-C); the LS estimate and MRC around it are those of the
// FP32 path (Sec. II-C, LS and MRC paragraphs).
//
// Transform (one wavefront per antenna symbol), N = 2048 = 8 x 16 x 16:
//   n = n1 + 16 n2 + 256 n3,  k = k3 + 8 k2 + 128 k1,  W = exp(-2 pi i / 2048)
//   A[n1,n2,k3] = W^(16 n2 k3) / 8 * sum_n3 x[n] W8^(n3 k3)       FP32, vector ALU
//   B[n1,k2,k3] = W^(n1 (k3+8k2)) / 16 * sum_n2 A W16^(n2 k2)       GEMM 1 + twiddle
//   X[k]        = 128 * sum_n1 B W16^(n1 k1)                         GEMM 2
// The 1/8 and 1/16 scalings are exact and keep every GEMM operand inside the
// fp16 range (|value| <= 32768 sqrt 2) whatever the int16 input; the 128 is
// folded into the second GEMM's matrix.
//
// Lane l = 16 q + r of the wavefront (r = l & 15, q = l >> 4).  The GEMMs run
// on v_mfma_f32_16x16x32_{f16,bf16}, whose operand layouts are
//   A (16 x 32): lane holds row r, K slots 8q .. 8q+7
//   B (32 x 16): lane holds column r, K slots 8q .. 8q+7
//   D (16 x 16): lane holds column r, rows 4q .. 4q+3
// and the stages are laid out so that each stage's output registers are the
// next stage's operand registers -- no data moves between lanes:
//   radix 8:  lane (r, q) transforms the columns (n1, n2) = (r, 4q + i),
//             i = 0..3, and holds A[r, 4q+i, k3] for every k3;
//   GEMM 1:   block t = k3; data as the A operand, row n1 = r, K slot
//             8q + 2i + c = (n2 = 4q + i, component c); the DFT matrix as the
//             B operand, column k2; the output lane (r, q) holds
//             B[n1 = 4q + i, k2 = r, k3 = t] -- rows n1, column k2;
//   GEMM 2:   block t; that data as the B operand (column k2 = r, K slot
//             8q + 2i + c = (n1 = 4q + i, c)); the DFT matrix as the A operand,
//             row rho -> k1 = sigma(rho); the output lane (r, q) holds
//             X[t + 8 r + 128 sigma(4q + i)].
// A 16-point DFT in real form is [Re; Im] out = [[C, S], [-S, C]] [Re; Im] in
// (C = cos, S = sin of 2 pi k n / 16); each GEMM runs two 16-row tiles (real
// and imaginary outputs).  With the split, x = hi + lo (hi = x rounded to the
// format, lo = x - hi rounded) and the products hi*hi + lo*hi + hi*lo are
// accumulated.
//
// sigma orders the 16 k1 of the second GEMM's rows: for the whole spectrum the
// identity; for the receive kernels the k1 whose 128 bins hold used
// subcarriers first, so that rows 4q + i with i < NI (NI = ceil(used k1 / 4))
// hold every used bin: the demod accumulates conj(H) Y and |H|^2 for 8 x NI
// bins per lane straight from the GEMM's output registers.
//
// mfma_estimate_kernel: LS H = Y * pilot factor at the used bins.
// mfma_demod_kernel: one workgroup per (slot, data symbol); its wavefronts
// split the antennas; a fixed-order cross-wave sum in LDS, then x = z / g,
// decisions and packed bits.
// mfma_fft_kernel: the whole spectrum of every symbol (FFT validation).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rx_fft.hpp"
#include "rx_launch.h"

namespace rx {
namespace mf {

#ifndef RX_MF_INTERLEAVE
#define RX_MF_INTERLEAVE 1
#endif

constexpr int N = 2048;
constexpr int kWaves = 4;
constexpr int kTwA = 16 * 8;        // stage-A twiddles, float2: [k3 pair][n2][2]
constexpr int kTwB = 8 * 64 * 4;    // GEMM-1 output twiddles, float2: [t][i pair][lane][2]

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t v2u32 __attribute__((ext_vector_type(2)));

template <typename T>
struct Fmt;
template <>
struct Fmt<_Float16> {
  typedef _Float16 v8 __attribute__((ext_vector_type(8)));
  typedef _Float16 v2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ f32x4 mma(const v8& a, const v8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  // (x, y) -> packed (hi, and lo = x - hi) halves; hi rounds toward zero
  // (one conversion for both values), lo to nearest
  // lo = x - hi by the mixed-precision FMA (v_fma_mix_f32 reads a half of the
  // packed hi as its f16 operand; fma(hi, -1, x) is exact), then one packing
  // conversion: four instructions per pair where conversion back, subtraction
  // and repacking take six.  neg1 is -1 supplied at run time: with a literal
  // -1 the compiler turns the FMA into a subtraction and loses the form.
  static __device__ __forceinline__ void split(float x, float y, uint32_t& hi, uint32_t* lo, float neg1) {
    const v2 h = __builtin_bit_cast(v2, __builtin_amdgcn_cvt_pkrtz(x, y));
    hi = __builtin_bit_cast(uint32_t, h);
    if (lo) {
      v2 l;
      l[0] = (_Float16)__builtin_fmaf((float)h[0], neg1, x);
      l[1] = (_Float16)__builtin_fmaf((float)h[1], neg1, y);
      *lo = __builtin_bit_cast(uint32_t, l);
    }
  }
};
template <>
struct Fmt<__bf16> {
  typedef __bf16 v8 __attribute__((ext_vector_type(8)));
  typedef __bf16 v2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ f32x4 mma(const v8& a, const v8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ void split(float x, float y, uint32_t& hi, uint32_t* lo, float) {
    v2 h;
    h[0] = (__bf16)x;  // nearest even (v_cvt_pk_bf16_f32)
    h[1] = (__bf16)y;
    hi = __builtin_bit_cast(uint32_t, h);
    if (lo) {
      v2 l;
      l[0] = (__bf16)(x - __uint_as_float(hi << 16));
      l[1] = (__bf16)(y - __uint_as_float(hi & 0xffff0000u));
      *lo = __builtin_bit_cast(uint32_t, l);
    }
  }
};

// Four complex values -> a GEMM operand (K slots 2i + c) and, with SPLIT, its
// lo part.
template <typename T, bool SPLIT>
__device__ __forceinline__ void pack_operand(const float2 (&v)[4], typename Fmt<T>::v8& hi, typename Fmt<T>::v8& lo,
                                             float neg1) {
  uint32_t h[4], l[4];
#pragma unroll
  for (int i = 0; i < 4; i++) Fmt<T>::split(v[i].x, v[i].y, h[i], SPLIT ? &l[i] : nullptr, neg1);
  hi = __builtin_bit_cast(typename Fmt<T>::v8, make_uint4(h[0], h[1], h[2], h[3]));
  if constexpr (SPLIT) lo = __builtin_bit_cast(typename Fmt<T>::v8, make_uint4(l[0], l[1], l[2], l[3]));
}

// A 16-point DFT in real form as this lane's share of a GEMM operand: for
// output index kk (the lane's row or column) and K slots 8q + 2i + c (input
// index 4q + i, component c): tile 0 (real outputs) C, S; tile 1 (imaginary)
// -S, C; all times `scale`.  kk < 0: a zero row.
template <typename T, bool SPLIT>
struct Dft16 {
  typename Fmt<T>::v8 hi[2], lo[2];
  __device__ __forceinline__ void init(int kk, int q, float scale, float neg1) {
#pragma unroll
    for (int tile = 0; tile < 2; tile++) {
      uint32_t h[4], l[4];
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int n = 4 * q + i;
        float sn, cs;
        sincospif((float)((2 * n * (kk < 0 ? 0 : kk)) & 31) / 16.0f, &sn, &cs);  // angle 2 pi n kk / 16
        const float z = kk < 0 ? 0.f : scale;
        const float re = tile == 0 ? cs * z : -sn * z;  // multiplies the real input
        const float im = tile == 0 ? sn * z : cs * z;   // multiplies the imaginary input
        Fmt<T>::split(re, im, h[i], SPLIT ? &l[i] : nullptr, neg1);
      }
      hi[tile] = __builtin_bit_cast(typename Fmt<T>::v8, make_uint4(h[0], h[1], h[2], h[3]));
      if constexpr (SPLIT) lo[tile] = __builtin_bit_cast(typename Fmt<T>::v8, make_uint4(l[0], l[1], l[2], l[3]));
    }
  }
};

// GEMM 1 of block t: data (A operand) times the DFT (B operand).
template <typename T, bool SPLIT>
__device__ __forceinline__ void gemm1(const typename Fmt<T>::v8& xh, const typename Fmt<T>::v8& xl,
                                      const Dft16<T, SPLIT>& F, f32x4 (&acc)[2]) {
#pragma unroll
  for (int tile = 0; tile < 2; tile++) {
    acc[tile] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (SPLIT) {
      acc[tile] = Fmt<T>::mma(xl, F.hi[tile], acc[tile]);
      acc[tile] = Fmt<T>::mma(xh, F.lo[tile], acc[tile]);
    }
    acc[tile] = Fmt<T>::mma(xh, F.hi[tile], acc[tile]);
  }
}

// GEMM 2 of block t: the DFT (A operand) times the data (B operand).
template <typename T, bool SPLIT>
__device__ __forceinline__ void gemm2(const typename Fmt<T>::v8& xh, const typename Fmt<T>::v8& xl,
                                      const Dft16<T, SPLIT>& F, f32x4 (&acc)[2]) {
#pragma unroll
  for (int tile = 0; tile < 2; tile++) {
    acc[tile] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (SPLIT) {
      acc[tile] = Fmt<T>::mma(F.hi[tile], xl, acc[tile]);
      acc[tile] = Fmt<T>::mma(F.lo[tile], xh, acc[tile]);
    }
    acc[tile] = Fmt<T>::mma(F.hi[tile], xh, acc[tile]);
  }
}

// Twiddle tables in LDS, filled once per workgroup from tw[k] = W^k, laid
// out so that every 16-byte read of a wavefront is free of bank conflicts:
//   twA: float4 [p][n2] = (W^(16 n2 (2p)), W^(16 n2 (2p + 1))) / 8
//        (lanes of one q read the same entry, the four q distinct banks)
//   twB: float4 [t][p][lane] = (w(2p), w(2p + 1)), w(i) = W^((4q + i)(t + 8r)) / 16
//        (consecutive lanes read consecutive 16 bytes)
__device__ __forceinline__ void fill_twiddles(float2* __restrict__ twA, float2* __restrict__ twB,
                                              const float2* __restrict__ tw) {
  for (int e = threadIdx.x; e < kTwA; e += blockDim.x) {
    const int k3 = 2 * (e >> 5) + (e & 1), n2 = (e >> 1) & 15;
    const float2 w = tw[(16 * n2 * k3) & (N - 1)];
    twA[e] = make_float2(w.x * 0.125f, w.y * 0.125f);
  }
  for (int e = threadIdx.x; e < kTwB; e += blockDim.x) {
    const int i = 2 * ((e >> 7) & 1) + (e & 1), l = (e >> 1) & 63, t = e >> 8;
    const int r = l & 15, q = l >> 4;
    const float2 w = tw[((4 * q + i) * (t + 8 * r)) & (N - 1)];
    twB[e] = make_float2(w.x * 0.0625f, w.y * 0.0625f);
  }
}

// Samples of this lane's radix-8 columns: raw[i][n3] = x[r + 16 (4q + i) + 256 n3].
__device__ __forceinline__ void load_columns(uint32_t (&raw)[4][8], const uint32_t* __restrict__ sym, int lane) {
  const int r = lane & 15, q = lane >> 4;
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int n3 = 0; n3 < 8; n3++)
      raw[i][n3] = __builtin_nontemporal_load(sym + r + 16 * (4 * q + i) + 256 * n3);
}

// Sample staging through LDS (receive kernels): a wavefront's 2048 samples
// go from memory straight into its 8 KB LDS region (global_load_lds, 16
// bytes per lane, no registers held while they are in flight), in 16-byte
// granules placed so that the radix-8 stage's reads are free of bank
// conflicts.  Sample n = r + 16 (4q + i) + 256 n3 (granule (r >> 2) +
// 4 (4q + i) + 64 n3) is stored as if it belonged to column (i + q) & 3:
// the 64 lanes of one read then hit 64 different banks.
constexpr int kStage = 2048;  // dwords per wavefront region
__device__ __forceinline__ void stage_samples(uint32_t* __restrict__ region, const uint32_t* __restrict__ sym,
                                              int lane) {
  // position p = lane within a 64-granule block holds the granule whose
  // column field (bits 2-3) is p's minus its q field (bits 4-5)
  const int g = (lane & ~0xC) | (((((lane >> 2) & 3) - ((lane >> 4) & 3)) & 3) << 2);
#pragma unroll
  for (int k = 0; k < 8; k++)
    __builtin_amdgcn_global_load_lds(sym + 256 * k + 4 * g, region + 256 * k, 16, 0, 0);
}

// Wait for this wavefront's outstanding memory loads (the staged samples
// among them) / for its LDS reads.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0f70); }  // vmcnt(0)
// ... all but the last K (loads complete in the order they were issued)
template <int K>
__device__ __forceinline__ void wait_vmem_but() { __builtin_amdgcn_s_waitcnt(0x0f70 | K); }  // vmcnt(K)
__device__ __forceinline__ void wait_lds() { __builtin_amdgcn_s_waitcnt(0xc07f); }   // lgkmcnt(0)

// Radix-8 of column i: a[k3] = A[r, 4q + i, k3] from its 8 samples.
__device__ __forceinline__ void radix8_column(const uint32_t (&raw)[8], const float2* __restrict__ twA, int q, int i,
                                              float2 (&a)[8]) {
  float2 v[8];
#pragma unroll
  for (int n3 = 0; n3 < 8; n3++) v[n3] = iq_to_float(raw[n3]);
  dft8(v, 0);
  const float4* w4 = reinterpret_cast<const float4*>(twA) + (4 * q + i);
  a[0] = make_float2(v[0].x * 0.125f, v[0].y * 0.125f);
#pragma unroll
  for (int p = 0; p < 4; p++) {
    const float4 w = w4[16 * p];  // W^(16 n2 k3) / 8 for k3 = 2p, 2p + 1
    if (p > 0) a[2 * p] = cmul(v[2 * p], make_float2(w.x, w.y));
    a[2 * p + 1] = cmul(v[2 * p + 1], make_float2(w.z, w.w));
  }
}

// Radix-8 stage from the staged samples, one column at a time: the next
// column's 8 samples are read while this one is transformed.
__device__ __forceinline__ void stage_a_lds(const uint32_t* __restrict__ region, const float2* __restrict__ twA,
                                            int lane, float2 (&a)[4][8]) {
  const int r = lane & 15, q = lane >> 4;
  const uint32_t* base = region + r + 64 * q;
  auto read = [&](int i, uint32_t (&raw)[8]) {
    const uint32_t* col = base + 16 * ((i + q) & 3);  // see stage_samples
#pragma unroll
    for (int n3 = 0; n3 < 8; n3++) raw[n3] = col[256 * n3];
  };
  uint32_t raw[2][8];
  read(0, raw[0]);
#pragma unroll
  for (int i = 0; i < 4; i++) {
    __builtin_amdgcn_sched_barrier(0);
    if (i + 1 < 4) read(i + 1, raw[(i + 1) & 1]);
    radix8_column(raw[i & 1], twA, q, i, a[i]);
  }
  __builtin_amdgcn_sched_barrier(0);
}

// Radix-8 stage: a[i][k3] = A[r, 4q + i, k3].
__device__ __forceinline__ void stage_a(const uint32_t (&raw)[4][8], const float2* __restrict__ twA, int q,
                                        float2 (&a)[4][8]) {
#pragma unroll
  for (int i = 0; i < 4; i++) {
    float2 v[8];
#pragma unroll
    for (int n3 = 0; n3 < 8; n3++) v[n3] = iq_to_float(raw[i][n3]);
    dft8(v, 0);
    const float4* w4 = reinterpret_cast<const float4*>(twA) + (4 * q + i);
    a[i][0] = make_float2(v[0].x * 0.125f, v[0].y * 0.125f);
#pragma unroll
    for (int p = 0; p < 4; p++) {
      const float4 w = w4[16 * p];  // W^(16 n2 k3) / 8 for k3 = 2p, 2p + 1
      if (p > 0) a[i][2 * p] = cmul(v[2 * p], make_float2(w.x, w.y));
      a[i][2 * p + 1] = cmul(v[2 * p + 1], make_float2(w.z, w.w));
    }
  }
}

// The used-subcarrier layout of a plan: sigma (k1 of each GEMM-2 row, -1 for a
// zero row) and NI; passed by value to the kernels.
struct Layout {
  int8_t sigma[16];
  int ni;
  float neg1;  // -1 (see Fmt<_Float16>::split)
};

// GEMM 1, its output twiddle and GEMM 2 for every block, from the radix-8
// results a; cb(t, y_re, y_im) receives GEMM 2's output of block t:
// y[i] = X[t + 8 r + 128 sigma(4q + i)], i < NI.
//
// Software pipeline over the blocks: step t issues GEMM 1 of block t + 1,
// then the twiddle, split and GEMM 2 of block t, then hands block t - 1's
// GEMM 2 output to cb -- so the matrix cores work on one block while the
// vector units finish the one before.  The steps are separated by scheduling
// barriers, which keep the register footprint at one step's.
template <typename T, bool SPLIT, int NI, typename CB>
__device__ __forceinline__ void gemm_blocks(const float2 (&a)[4][8], const float2* __restrict__ twB,
                                            const Dft16<T, SPLIT>& F1, const Dft16<T, SPLIT>& F2, int lane,
                                            float neg1, CB&& cb) {
  const float4* tb = reinterpret_cast<const float4*>(twB) + lane;
  auto gemm1_block = [&](int t, f32x4 (&acc)[2]) {
    typename Fmt<T>::v8 xh, xl;
    const float2 col[4] = {a[0][t], a[1][t], a[2][t], a[3][t]};
    pack_operand<T, SPLIT>(col, xh, xl, neg1);
    gemm1<T, SPLIT>(xh, xl, F1, acc);
  };
  f32x4 g1[2][2], g2[2][2];
  gemm1_block(0, g1[0]);
#pragma unroll
  for (int t = 0; t <= 8; t++) {
    __builtin_amdgcn_sched_barrier(0);
    if (t + 1 < 8) gemm1_block(t + 1, g1[(t + 1) & 1]);
    if (t < 8) {
      // twiddle W^((4q + i)(t + 8r)) / 16 on B[n1 = 4q + i, k2 = r, k3 = t]
      const float4 w01 = tb[t * 128], w23 = tb[t * 128 + 64];
      const float2 w[4] = {make_float2(w01.x, w01.y), make_float2(w01.z, w01.w), make_float2(w23.x, w23.y),
                           make_float2(w23.z, w23.w)};
      float2 b[4];
#pragma unroll
      for (int i = 0; i < 4; i++) b[i] = cmul(make_float2(g1[t & 1][0][i], g1[t & 1][1][i]), w[i]);
      typename Fmt<T>::v8 xh, xl;
      pack_operand<T, SPLIT>(b, xh, xl, neg1);
      gemm2<T, SPLIT>(xh, xl, F2, g2[t & 1]);
    }
    if (t > 0) {
      float yr[NI], yi[NI];
#pragma unroll
      for (int i = 0; i < NI; i++) {
        yr[i] = g2[(t - 1) & 1][0][i];
        yi[i] = g2[(t - 1) & 1][1][i];
      }
      cb(t - 1, yr, yi);
    }
#if RX_MF_INTERLEAVE
    // issue order within the step: the next block's operand packing, then
    // each product followed by a few vector instructions (this block's
    // twiddle and packing, the previous block's combining), so that the
    // matrix core works while the wavefront keeps issuing
    if (t > 0 && t < 7) {
      __builtin_amdgcn_sched_group_barrier(0x0002, 8, 0);
#pragma unroll
      for (int m = 0; m < 2 * (SPLIT ? 6 : 2); m++) {
        __builtin_amdgcn_sched_group_barrier(0x0008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x0002, SPLIT ? 5 : 12, 0);
      }
    }
#endif
  }
}

// Per lane and used register i: the bin of block 0 (k = kb + t for block t)
// and its sigma.
template <int NI>
struct Bins {
  int kb[NI];
  int k1[NI];
  __device__ __forceinline__ void init(const Layout& L, int lane) {
    const int r = lane & 15, q = lane >> 4;
#pragma unroll
    for (int i = 0; i < NI; i++) {
      k1[i] = L.sigma[4 * q + i];
      kb[i] = 8 * r + 128 * k1[i];
    }
  }
  // subcarrier of bin k (fftshift order, DC excluded), -1 if unused
  static __device__ __forceinline__ int sub(int k, int h) {
    return (k >= 1 && k <= h) ? k - 1 + h : (k >= N - h ? k - (N - h) : -1);
  }
};

__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t n) {
  // workgroups are dispatched round robin over the 8 XCDs; give each XCD a
  // contiguous range of (slot, symbol) items so a slot's estimate stays in
  // one L2
  const int64_t qn = n >> 3, rn = n & 7;
  const int64_t x = b & 7, j = b >> 3;
  return (x < rn) ? x * (qn + 1) + j : rn * (qn + 1) + (x - rn) * qn + j;
}

// ------------------------------------------------------------------ estimate
// A resident grid: wavefront g of the G in the grid transforms the pilot
// symbols g, g + G, ... of the S*A list of (slot, antenna), the next one's
// samples staged while the current one is transformed.  The pilot factors
// of the lane's bins are the same for every job and are loaded once.
template <typename T, bool SPLIT, int NI>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(2))) void mfma_estimate_kernel(
    const uint32_t* __restrict__ iq, int64_t S, int A, int T_, int CP, int U, const float2* __restrict__ tw,
    const float2* __restrict__ pf, float2* __restrict__ H, Layout L) {
  __shared__ float2 twA[kTwA];
  __shared__ float2 twB[kTwB];
  __shared__ __align__(16) uint32_t stage[kWaves * kStage];
  fill_twiddles(twA, twB, tw);
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63, q = lane >> 4;
  const int64_t jobs = S * A;
  const int64_t G = (int64_t)gridDim.x * kWaves;
  int64_t j = (int64_t)blockIdx.x * kWaves + wave;
  if (j >= jobs) return;  // no workgroup barrier below
  Dft16<T, SPLIT> F1, F2;
  F1.init(lane & 15, q, 1.0f, L.neg1);
  F2.init(L.sigma[lane & 15], q, 128.0f, L.neg1);
  Bins<NI> bins;
  bins.init(L, lane);
  const int h = U >> 1;
  // per block and used register: byte offset of the subcarrier in a row
  // (past the row for an unused bin, where stores are dropped) and its pilot
  // factor (zero there)
  int off[8][NI];
  float2 pfv[8][NI];
  const __amdgpu_buffer_rsrc_t pr =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(pf), (short)0, U * 8, 0x00020000);
#pragma unroll
  for (int t = 0; t < 8; t++)
#pragma unroll
    for (int i = 0; i < NI; i++) {
      const int d = bins.k1[i] < 0 ? -1 : Bins<NI>::sub(bins.kb[i] + t, h);
      off[t][i] = d >= 0 ? 8 * d : 8 * U;
      pfv[t][i] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(pr, off[t][i], 0, 0));
    }
  auto pilot_sym = [&](int64_t jj) {
    const int64_t ss = jj / A;
    const int aa = (int)(jj - ss * A);
    return iq + (ss * T_ * A + aa) * (int64_t)(N + CP) + CP;
  };
  uint32_t* region = stage + wave * kStage;
  stage_samples(region, pilot_sym(j), lane);
  for (; j < jobs; j += G) {
    float2 av[4][8];
    wait_vmem();
    stage_a_lds(region, twA, lane, av);
    // the region is read: stage the next job's samples, in flight during
    // this one's GEMMs
    wait_lds();
    if (j + G < jobs) stage_samples(region, pilot_sym(j + G), lane);
    const __amdgpu_buffer_rsrc_t hr =
        __builtin_amdgcn_make_buffer_rsrc(H + j * (int64_t)U, (short)0, U * 8, 0x00020000);
    gemm_blocks<T, SPLIT, NI>(av, twB, F1, F2, lane, L.neg1, [&](int t, const float (&yr)[NI], const float (&yi)[NI]) {
#pragma unroll
      for (int i = 0; i < NI; i++)
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(v2u32, cmul(make_float2(yr[i], yi[i]), pfv[t][i])), hr, off[t][i], 0, 0);
    });
  }
}

// ------------------------------------------------------------------ demod
// One workgroup per (slot, data symbol).  Channel rows are read through a
// buffer resource over the slot's estimate at per-lane offsets (bin of block
// 0) plus 8 t bytes: a lane whose bin is unused reads some value of the slot
// (or zero past its end) and its sum is never stored.
template <typename T, bool SPLIT, int NI>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(2))) void mfma_demod_kernel(
    const uint32_t* __restrict__ iq, int64_t S, int A, int T_, int CP, int U, int B, const float2* __restrict__ tw,
    const float2* __restrict__ H, float2* __restrict__ xhat, uint8_t* __restrict__ bits, Layout L) {
  __shared__ float2 twA[kTwA];
  __shared__ float2 twB[kTwB];
  __shared__ __align__(16) uint32_t stage[kWaves * kStage];
  extern __shared__ float red[];  // [U][3]: z.x, z.y, g
  fill_twiddles(twA, twB, tw);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4;
  Dft16<T, SPLIT> F1, F2;
  F1.init(lane & 15, q, 1.0f, L.neg1);
  F2.init(L.sigma[lane & 15], q, 128.0f, L.neg1);
  Bins<NI> bins;
  bins.init(L, lane);
  const int Td = T_ - 1;
  const int64_t item = xcd_remap(blockIdx.x, S * Td);
  const int64_t s = item / Td;
  const int t_sym = 1 + (int)(item % Td);
  const uint32_t* symrow = iq + ((s * T_ + t_sym) * A) * (int64_t)(N + CP) + CP;
  const int h = U >> 1;
  // Channel rows are read through a buffer resource over one row, at the
  // byte offset of each used register's block-0 subcarrier plus 8 t: bins
  // past either end of the used band (and zero GEMM rows) fall outside the
  // row, where the load returns zero without touching memory.
  int hoff[NI];
#pragma unroll
  for (int i = 0; i < NI; i++)
    hoff[i] = bins.k1[i] < 0 ? INT32_MIN / 2 : (bins.kb[i] + (bins.k1[i] < 8 ? h - 1 : h - N)) * 8;
  const float2* Hs = H + s * A * (int64_t)U;
  auto row_rsrc = [&](int a) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(Hs + (int64_t)a * U), (short)0, U * 8,
                                             0x00020000);
  };
  float2 z[8][NI];
  float g[8][NI];
#pragma unroll
  for (int t = 0; t < 8; t++)
#pragma unroll
    for (int i = 0; i < NI; i++) {
      z[t][i] = make_float2(0.f, 0.f);
      g[t][i] = 0.f;
    }
  // channel values of one block, requested one block ahead of their use
  auto load_h = [&](float2 (&dst)[NI], __amdgpu_buffer_rsrc_t rs, int t) {
#pragma unroll
    for (int i = 0; i < NI; i++)
      dst[i] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, hoff[i] + 8 * t, 0, 0));
  };
  float2 hnext[NI];
  uint32_t* region = stage + __builtin_amdgcn_readfirstlane(wave) * kStage;
  if (wave < A) {
    stage_samples(region, symrow + (int64_t)wave * (N + CP), lane);
    load_h(hnext, row_rsrc(wave), 0);
  }
  for (int a = __builtin_amdgcn_readfirstlane(wave); a < A; a += kWaves) {
    const bool more = a + kWaves < A;
    float2 av[4][8];
    // the samples staged during the previous job; the NI channel loads
    // issued after them (this job's first block) may stay in flight
    wait_vmem_but<NI>();
    stage_a_lds(region, twA, lane, av);
    // the region is read: stage the next antenna's samples, in flight during
    // this one's GEMMs
    wait_lds();
    if (more) stage_samples(region, symrow + (int64_t)(a + kWaves) * (N + CP), lane);
    const __amdgpu_buffer_rsrc_t rs = row_rsrc(a), rs_next = row_rsrc(more ? a + kWaves : a);
    gemm_blocks<T, SPLIT, NI>(av, twB, F1, F2, lane, L.neg1, [&](int t, const float (&yr)[NI], const float (&yi)[NI]) {
      float2 hv[NI];
#pragma unroll
      for (int i = 0; i < NI; i++) hv[i] = hnext[i];
      if (t < 7) load_h(hnext, rs, t + 1);
      else if (more) load_h(hnext, rs_next, 0);
#pragma unroll
      for (int i = 0; i < NI; i++) {
        const float2 hh = hv[i];
        z[t][i].x = fmaf(hh.x, yr[i], fmaf(hh.y, yi[i], z[t][i].x));  // conj(h) * y
        z[t][i].y = fmaf(hh.x, yi[i], fmaf(-hh.y, yr[i], z[t][i].y));
        g[t][i] = fmaf(hh.x, hh.x, fmaf(hh.y, hh.y, g[t][i]));
      }
    });
  }
  // fixed-order cross-wave sum into red[d]: wave 0 stores, waves 1.. add in turn
#pragma unroll 1
  for (int w = 0; w < kWaves; w++) {
    if (w == wave) {
#pragma unroll
      for (int t = 0; t < 8; t++)
#pragma unroll
        for (int i = 0; i < NI; i++) {
          const int d = bins.k1[i] < 0 ? -1 : Bins<NI>::sub(bins.kb[i] + t, h);
          if (d >= 0) {
            float* p = red + 3 * d;
            if (w == 0) {
              p[0] = z[t][i].x;
              p[1] = z[t][i].y;
              p[2] = g[t][i];
            } else {
              p[0] += z[t][i].x;
              p[1] += z[t][i].y;
              p[2] += g[t][i];
            }
          }
        }
    }
    __syncthreads();
  }
  const int row_bytes = U * B / 8;
  const int64_t out_row = s * Td + (t_sym - 1);
  const float c16 = 3.16227766016837933f;  // sqrt(10)
  const float c64 = 6.48074069840786023f;  // sqrt(42)
  for (int qd = threadIdx.x; 4 * qd < U; qd += 64 * kWaves) {
    const int nsym = min(4, U - 4 * qd);
    uint32_t accb = 0;  // bits of up to 4 symbols, MSB-first
    for (int e = 0; e < nsym; e++) {
      const int d = 4 * qd + e;
      const float zx = red[3 * d], zy = red[3 * d + 1], gg = red[3 * d + 2];
      const float2 x = gg > 0.f ? make_float2(zx / gg, zy / gg) : make_float2(0.f, 0.f);
      if (xhat) xhat[out_row * U + d] = x;
      // hard decisions: strict comparisons, so ties and -0.0 give 0
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
      const int nbits = nsym * B;                              // a multiple of 8
      uint8_t* o = bits + out_row * row_bytes + (qd * B) / 2;  // 4 symbols = B/2 bytes
      for (int byte = 0; byte < nbits / 8; byte++) o[byte] = (uint8_t)(accb >> (nbits - 8 * (byte + 1)));
    }
  }
}

// ------------------------------------------------------------------ FFT only
template <typename T, bool SPLIT>
__global__ __launch_bounds__(64 * kWaves) void mfma_fft_kernel(const uint32_t* __restrict__ iq, int64_t n_sym_total,
                                                               int CP, const float2* __restrict__ tw,
                                                               float2* __restrict__ Y, float neg1) {
  __shared__ float2 twA[kTwA];
  __shared__ float2 twB[kTwB];
  fill_twiddles(twA, twB, tw);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
  const int64_t sym = (int64_t)blockIdx.x * kWaves + wave;  // flat (slot, symbol, antenna)
  if (sym >= n_sym_total) return;                           // no barrier below
  Dft16<T, SPLIT> F1, F2;
  F1.init(r, q, 1.0f, neg1);
  F2.init(r, q, 128.0f, neg1);
  uint32_t raw[4][8];
  load_columns(raw, iq + sym * (N + CP) + CP, lane);
  float2* out = Y + sym * N;
  float2 av[4][8];
  stage_a(raw, twA, q, av);
  gemm_blocks<T, SPLIT, 4>(av, twB, F1, F2, lane, neg1, [&](int t, const float (&yr)[4], const float (&yi)[4]) {
#pragma unroll
    for (int i = 0; i < 4; i++) out[t + 8 * r + 128 * (4 * q + i)] = make_float2(yr[i], yi[i]);
  });
}

}  // namespace mf

// ------------------------------------------------------------------ launchers
namespace {

// Row order of GEMM 2 for U used subcarriers: the k1 whose bins
// [128 k1, 128 k1 + 128) hold a used subcarrier, ascending, go to rows
// 4q + i with list index 4i + q; the other rows are zero.
mf::Layout layout_for(int U) {
  mf::Layout L{};
  int used[16], n = 0;
  const int h = U / 2;
  for (int k1 = 0; k1 < 16; k1++) {
    const int lo = 128 * k1, hi = lo + 127;
    const bool any = (hi >= 1 && lo <= h) || hi >= mf::N - h;
    if (any) used[n++] = k1;
  }
  for (int rho = 0; rho < 16; rho++) {
    const int q = rho >> 2, i = rho & 3, idx = 4 * i + q;
    L.sigma[rho] = (int8_t)(idx < n ? used[idx] : -1);
  }
  L.ni = (n + 3) / 4;
  L.neg1 = -1.0f;
  return L;
}

// Workgroups of the estimate kernel resident at once on the current device
// (0 on error), cached per device and instantiation.
template <typename T, bool SPLIT, int NI>
int est_capacity() {
  static int cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
  if (dev < 64 && cached[dev] > 0) return cached[dev];
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(mf::mfma_estimate_kernel<T, SPLIT, NI>), 64 * mf::kWaves, 0) !=
          hipSuccess)
    return 0;
  const int n = cus * (per_cu > 0 ? per_cu : 1);
  if (dev < 64) cached[dev] = n;
  return n;
}

template <typename T, bool SPLIT, int NI>
hipError_t est_ni(const LaunchArgs& la, float2* H, const mf::Layout& L) {
  const int cap = est_capacity<T, SPLIT, NI>();
  if (cap <= 0) return hipErrorInvalidValue;
  const int64_t needed = (la.S * la.A + mf::kWaves - 1) / mf::kWaves;
  const int64_t grid = needed < cap ? needed : cap;
  hipLaunchKernelGGL((mf::mfma_estimate_kernel<T, SPLIT, NI>), dim3((unsigned)grid), dim3(64 * mf::kWaves), 0,
                     la.stream, la.iq, la.S, la.A, la.T, la.CP, la.U, la.tw, la.pf, H, L);
  return hipGetLastError();
}

template <typename T, bool SPLIT>
hipError_t est(const LaunchArgs& la, float2* H) {
  const mf::Layout L = layout_for(la.U);
  switch (L.ni) {
    case 1: return est_ni<T, SPLIT, 1>(la, H, L);
    case 2: return est_ni<T, SPLIT, 2>(la, H, L);
    case 3: return est_ni<T, SPLIT, 3>(la, H, L);
    // NI = 4 would need more than 12 k1 with used bins: U > 1536, which
    // the plan rejects for these modes
  }
  return hipErrorInvalidValue;
}

template <typename T, bool SPLIT, int NI>
hipError_t dem_ni(const LaunchArgs& la, const float2* H, float2* xhat, uint8_t* bits, const mf::Layout& L) {
  const size_t lds = sizeof(float) * 3 * (size_t)la.U;
  hipLaunchKernelGGL((mf::mfma_demod_kernel<T, SPLIT, NI>), dim3((unsigned)(la.S * (la.T - 1))),
                     dim3(64 * mf::kWaves), lds, la.stream, la.iq, la.S, la.A, la.T, la.CP, la.U, la.B, la.tw, H,
                     xhat, bits, L);
  return hipGetLastError();
}

template <typename T, bool SPLIT>
hipError_t dem(const LaunchArgs& la, const float2* H, float2* xhat, uint8_t* bits) {
  const mf::Layout L = layout_for(la.U);
  switch (L.ni) {
    case 1: return dem_ni<T, SPLIT, 1>(la, H, xhat, bits, L);
    case 2: return dem_ni<T, SPLIT, 2>(la, H, xhat, bits, L);
    case 3: return dem_ni<T, SPLIT, 3>(la, H, xhat, bits, L);
    // (NI = 4 needs U > 1536, which the plan rejects for these modes)
  }
  return hipErrorInvalidValue;
}

template <typename T, bool SPLIT>
hipError_t fft(const LaunchArgs& la, float2* Y) {
  const int64_t total = la.S * la.T * la.A;
  hipLaunchKernelGGL((mf::mfma_fft_kernel<T, SPLIT>), dim3((unsigned)((total + mf::kWaves - 1) / mf::kWaves)),
                     dim3(64 * mf::kWaves), 0, la.stream, la.iq, total, la.CP, la.tw, Y, -1.0f);
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
