// rx_denoise.hip -- learned refinement of a comb-pilot LS channel estimate,
// its training kernels and the generator of its training channels (gfx950).
//
// The network, per row h[0..U) (one antenna of one slot):
//   s = sqrt(mean |h|^2);  x0 = (Re h, Im h) / s                (2 channels)
//   a_l = b_l + sum_{ci,k} W_l[co][ci][k] x_{l-1}[ci][d+k-3]    (7 taps, zero outside 0..U-1)
//   x_l = max(a_l, 0) (l = 1, 2, 3);  channels 2 -> 32 -> 32 -> 32 -> 2
//   out = h + s (a_4[0] + i a_4[1])
// LS stays the fallback: at inference a row keeps h when the correction
// out - h has non-finite energy or more than max_corr^2 times sum |h|^2.
// Training loss: mean over rows and d of |x0 + a_4 - h_true / s|^2.
// The paper computes the LS estimate only (Sec. II-C, LS paragraph); this
// refinement and its comb-pilot input extend it.
//
// Every product runs on the bf16 MFMA v_mfma_f32_16x16x32_bf16 (16 x 16
// output, K = 32) with FP32 accumulation; weights, activations and backward
// deltas enter the products as bf16 (round to nearest even), sums stay FP32.
// Operand layout of that MFMA (lane l = 16 q + r, q = 0..3):
//   A (16 x 32): lane holds row r, k-slots 8q .. 8q+7
//   B (32 x 16): lane holds column r, k-slots 8q .. 8q+7
//   C (16 x 16): lane holds column r, rows 4q .. 4q+3 (one per register)
//
// Forward (dn_forward_kernel): a persistent workgroup of 4 wavefronts takes
// whole rows; a row is cut into tiles of TO = 240 output positions.  Each
// tile recomputes a halo (3 positions per layer and side), so the layers of
// a tile run back to back out of LDS: x0 [pos][2], then x1, x2, x3 in two
// [pos][40] bf16 ping-pong buffers (32 channels + 8 pad; the row pitch is
// discussed at RS below).  A
// GEMM unit is 16 positions x 32 output channels (two MFMA rows of 16); the
// K dimension is (tap, input channel): one 16-byte LDS read per tap.  The
// last layer (2 output channels) puts its 7 taps into the MFMA rows instead
// (14 of 16 rows used, one MFMA per 16 positions) and sums the taps over
// positions from LDS.  The weights of all four layers stay in registers for
// the workgroup's life.
// Training stores x0..x3 and the output delta d4 = 2 (x0 + a_4 - t) / (R U)
// channel-major in global memory, plus a per-workgroup loss partial.
//
// Backward (dn_backward_kernel): same tiling, transposed convolutions
// g_{l-1}[ci][p] = sum_{co,k} W_l[co][ci][k] d_l[co][p+3-k], masked by
// x_{l-1} > 0, give d3, d2, d1.  The masks come as one 32-bit word per
// position and layer, written by the training forward from LDS.
//
// Weight gradients (dn_wgrad_kernel): dW_l[co][ci][k] = sum_{r,p} d_l[co][p]
// x_{l-1}[ci][p+k-3], a GEMM with K = positions; workgroup (x, y) reduces
// rows range x of layer y into partial vector x, and dn_reduce_kernel sums
// the partials in a fixed order (deterministic) and applies Adam (Kingma and
// Ba, 2015).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rx_comb.hpp"
#include "rx_launch.h"

namespace rx {
namespace dn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t bfbits;  // raw bf16

constexpr int kBlock = 256;
constexpr int TO = 240;    // output positions per tile
constexpr int NPOS = 288;  // LDS positions per activation buffer
// Row pitch of the activation buffers.  gfx950's LDS has 64 banks of 4
// bytes; probes of the bank-conflict counter show that a 16-byte read is
// served 16 lanes at a time, each group of 16 taking lanes from two
// quarter-waves (for example lanes 0-7 with 24-31), while 8-byte accesses are
// served 32 lanes at a time.  For the operand reads (lane (r, q): 16 bytes at
// row r, slot q) a pitch of 20 dwords (80 bytes) then gives two-way conflicts
// and a pitch of 24 dwords none; but at 24 the unit stores (8 bytes, rows r,
// slots q) conflict two-way instead, and the 96-byte pitch measured 3 %
// slower over 4096 rows, so the buffers keep 80-byte rows.
constexpr int RS = 40;     // bf16 per LDS position row (32 channels + 8 pad)
constexpr int BASE_F = 12; // forward: LDS index of position t0
constexpr int BASE_B = 18; // backward: LDS index of position t0
// GEMM units (16 positions) per layer and tile; see the halo layout below.
constexpr int U1 = 17, U2 = 16, U3 = 16, U4P = 16;
constexpr int PS = 260;  // LDS row pitch (floats) of the folded last layer's per-tap outputs
static_assert(14 * PS * 4 <= NPOS * RS * 2, "per-tap outputs fit in one activation buffer");
constexpr int BU3 = 16, BU2 = 16, BU1 = 15;

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// float -> bf16 bits, round to nearest even: the conversion gfx950 does in
// hardware (v_cvt_pk_bf16_f32, two values per instruction)
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float bf16_float(uint32_t b) { return __uint_as_float(b << 16); }
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
  bf16x2 v;
  v[0] = (__bf16)lo;
  v[1] = (__bf16)hi;
  return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) {
  bf16x8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order sum over the workgroup's 4 wavefronts; every thread gets it.
__device__ __forceinline__ float block_sum(float v, float* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// One GEMM unit of a 32-input-channel layer: 16 positions, 32 output channels
// (acc[h] holds output channels 16 h .. 16 h + 15).  `row0` is the LDS index
// of the unit's first position minus the tap offset (tap k reads row0 + k + r).
// SIGN = +1: forward taps; -1: transposed (tap k reads row0 - k + r).
template <int SIGN>
__device__ __forceinline__ void unit32(const bfbits* __restrict__ X, int row0, const bf16x8 (&w)[2][7],
                                       f32x4 (&acc)[2]) {
  const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
  bf16x8 b[7];
#pragma unroll
  for (int k = 0; k < 7; k++)
    b[k] = as_bf16x8(*reinterpret_cast<const uint4*>(X + (row0 + SIGN * k + r) * RS + 8 * q));
#pragma unroll
  for (int k = 0; k < 7; k++) {
    acc[0] = mfma(w[0][k], b[k], acc[0]);
    acc[1] = mfma(w[1][k], b[k], acc[1]);
  }
}

// The 7 tap operands of a unit (the loads of unit32, apart from its products).
__device__ __forceinline__ void unit32_load(const bfbits* __restrict__ X, int row0, bf16x8 (&b)[7]) {
  const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
#pragma unroll
  for (int k = 0; k < 7; k++) b[k] = as_bf16x8(*reinterpret_cast<const uint4*>(X + (row0 + k + r) * RS + 8 * q));
}

// Four dwords at dword index i of an LDS buffer of 2-channel positions
// (4-byte aligned reads).
__device__ __forceinline__ bf16x8 read4(const uint32_t* __restrict__ X, int i) {
  return as_bf16x8(make_uint4(X[i], X[i + 1], X[i + 2], X[i + 3]));
}

// Store an output unit (ReLU or delta masks applied by the caller) into an
// LDS [pos][RS] buffer: lane (r, q) holds position row `idx`, channels
// 16 h + 4 q + 0..3 in acc[h].
__device__ __forceinline__ void store_unit(bfbits* __restrict__ Y, int idx, const f32x4 (&v)[2]) {
  const int q = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const uint2 pk = make_uint2(pack2(v[h][0], v[h][1]), pack2(v[h][2], v[h][3]));
    *reinterpret_cast<uint2*>(Y + idx * RS + 16 * h + 4 * q) = pk;
  }
}

// Channel-major global store of a unit: G[(ch)*UP + p].
__device__ __forceinline__ void store_global(bfbits* __restrict__ G, int64_t UP, int p, const f32x4 (&v)[2]) {
  const int q = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int h = 0; h < 2; h++)
#pragma unroll
    for (int i = 0; i < 4; i++) G[(int64_t)(16 * h + 4 * q + i) * UP + p] = (bfbits)bf16_bits(v[h][i]);
}

// ReLU mask words of the tile's own positions [t0, t0 + TO) of a layer just
// written to X (LDS index of position p is p - t0 + 12): bit c of
// Mg[p] = (x[c][p] > 0).  One thread per position.
__device__ __forceinline__ void store_masks(const bfbits* __restrict__ X, int t0, int U, uint32_t* __restrict__ Mg) {
  const int i = threadIdx.x;
  const int p = t0 + i;
  if (i < TO && p < U) {
    const uint4* row = reinterpret_cast<const uint4*>(X + (i + BASE_F) * RS);
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint4 v = row[k];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const uint32_t lo = w[j] & 0xFFFFu, hi = w[j] >> 16;
        m |= (uint32_t)((lo & 0x8000u) == 0 && lo != 0) << (8 * k + 2 * j);
        m |= (uint32_t)((hi & 0x8000u) == 0 && hi != 0) << (8 * k + 2 * j + 1);
      }
    }
    Mg[p] = m;
  }
}

// ReLU of a unit's outputs (lane r holds position p0 + r), zero for positions
// outside the row [0, U).  The ReLU is a signed-integer max of the float's
// bits: positive floats order as positive integers, negative ones and -0 as
// negative, so max(bits, 0) is max(x, +0) for every non-NaN x -- one
// instruction per value, where a float max first canonicalises its operand.
// Only units that reach past an end of the row (a wavefront-uniform test)
// pay for the position mask.
__device__ __forceinline__ float relu_bits(float x) { return __int_as_float(max(__float_as_int(x), 0)); }
__device__ __forceinline__ void relu_unit(f32x4 (&acc)[2], int p0, int U) {
  if (p0 >= 0 && p0 + 15 < U) {
#pragma unroll
    for (int h = 0; h < 2; h++)
#pragma unroll
      for (int i = 0; i < 4; i++) acc[h][i] = relu_bits(acc[h][i]);
  } else {
    const int p = p0 + (threadIdx.x & 15);
    const bool in = p >= 0 && p < U;
#pragma unroll
    for (int h = 0; h < 2; h++)
#pragma unroll
      for (int i = 0; i < 4; i++) acc[h][i] = in ? relu_bits(acc[h][i]) : 0.f;
  }
}

__device__ __forceinline__ void bias_init(f32x4 (&acc)[2], const float* __restrict__ b) {
  const int q = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int h = 0; h < 2; h++)
#pragma unroll
    for (int i = 0; i < 4; i++) acc[h][i] = b[16 * h + 4 * q + i];
}

// A 32-input-channel layer of an inference tile, two units at a time: the
// wavefront's units u = wave + 4 j (NU in all per layer, a multiple of 8)
// are taken in pairs (j, j + 1), whose 14 tap operands are requested
// together and whose products run as four interleaved accumulation chains
// (each product waits on the one four places back instead of two).  Unit u
// covers LDS rows first + 16 u + r of the output, reading rows from
// first + 16 u - 3; positions p0 + 16 u + r.  One unit at a time with the
// next unit's operands requested ahead (the same registers) ran 2 % slower.
template <int NU>
__device__ __forceinline__ void layer32_paired(const bfbits* __restrict__ X, bfbits* __restrict__ Y, int first,
                                               int p0, int U, const bf16x8 (&w)[2][7],
                                               const float* __restrict__ bias) {
  static_assert(NU % 8 == 0, "pairs of whole rounds of the 4 wavefronts");
  const int wave = threadIdx.x >> 6, r = threadIdx.x & 15;
#pragma unroll
  for (int j = 0; j < NU / 4; j += 2) {
    const int u0 = wave + 4 * j, u1 = u0 + 4;
    bf16x8 b0[7], b1[7];
    unit32_load(X, first + 16 * u0 - 3, b0);
    unit32_load(X, first + 16 * u1 - 3, b1);
    f32x4 a0[2], a1[2];
    bias_init(a0, bias);
    bias_init(a1, bias);
#pragma unroll
    for (int k = 0; k < 7; k++) {
      a0[0] = mfma(w[0][k], b0[k], a0[0]);
      a1[0] = mfma(w[0][k], b1[k], a1[0]);
      a0[1] = mfma(w[1][k], b0[k], a0[1]);
      a1[1] = mfma(w[1][k], b1[k], a1[1]);
    }
    relu_unit(a0, p0 + 16 * u0, U);
    store_unit(Y, first + 16 * u0 + r, a0);
    relu_unit(a1, p0 + 16 * u1, U);
    store_unit(Y, first + 16 * u1 + r, a1);
  }
}

// ------------------------------------------------------------------ forward
// Halo layout of a forward tile starting at output position t0 (LDS index
// of position p is p - t0 + 12):
//   x0  positions t0-12 .. t0+275  (indices 0..287)
//   x1  computed for t0-9  + [0, 272)  (17 units)   -> buffer A
//   x2  computed for t0-6  + [0, 256)  (16 units)   -> buffer B
//   x3  computed for t0-3  + [0, 256)  (16 units)   -> buffer A
//   P   layer 4 per tap, for t0-3 + [0, 256) (16 units) -> buffer B (float)
//   out summed for t0 + [0, 240) from P at p-3..p+3
// Layer l's output at p needs x_{l-1} at p-3..p+3; each range above covers
// what the next layer needs for the final 240 outputs (layer 3 also reads up
// to 6 stale positions past x2's range; they reach only discarded outputs).
// Layer 1's K = 32 slots are (tap 0..15, channel 0..1) with taps 7..15 zero.
// The register budget of two wavefronts per SIMD is stated: left to itself
// the compiler took 225 VGPRs + 32 AGPRs for the inference instance (one
// wavefront per SIMD), which ran 0.34 ms for 4096 rows against 0.19 ms with
// the budget (256 VGPRs, a 12-byte spill).
template <bool TRAIN>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void dn_forward_kernel(const float2* __restrict__ Hin, int64_t rows, int U,
                                                            const bf16x8* __restrict__ frag,
                                                            const float* __restrict__ theta,
                                                            float2* __restrict__ Hout, DnTrainIo io) {
  extern __shared__ __align__(16) unsigned char smem[];
  bfbits* XA = reinterpret_cast<bfbits*>(smem);
  bfbits* XB = XA + NPOS * RS;
  uint32_t* X0 = reinterpret_cast<uint32_t*>(XB + NPOS * RS);
  float2* hrow = reinterpret_cast<float2*>(X0 + NPOS);
  __shared__ float red[4];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, q = lane >> 4;

  bf16x8 w1[2], w2[2][7], w3[2][7], w4;
#pragma unroll
  for (int h = 0; h < 2; h++) {
    w1[h] = frag[kF1 + h * 64 + lane];
#pragma unroll
    for (int k = 0; k < 7; k++) {
      w2[h][k] = frag[kF2 + (h * 7 + k) * 64 + lane];
      w3[h][k] = frag[kF3 + (h * 7 + k) * 64 + lane];
    }
  }
  w4 = frag[kF4 + lane];
  const float* b1 = theta + kPB1;
  const float* b2 = theta + kPB2;
  const float* b3 = theta + kPB3;
  const float* b4 = theta + kPB4;

  // stale LDS is read only into discarded outputs; start it finite
  for (int i = tid; i < 2 * NPOS * RS / 2; i += kBlock) reinterpret_cast<uint32_t*>(XA)[i] = 0u;
  const int64_t UP = io.UP;
  float loss = 0.f;

  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const float2* hr = Hin + row * U;
    float ss = 0.f;
    __syncthreads();  // the previous row's readers of hrow are done
    for (int d = tid; d < U; d += kBlock) {
      const float2 v = hr[d];
      hrow[d] = v;
      ss = fmaf(v.x, v.x, fmaf(v.y, v.y, ss));
    }
    const float hs = block_sum(ss, red);  // sum_d |h[d]|^2
    const float s = sqrtf(hs / (float)U);
    const float inv = s > 0.f ? 1.0f / s : 0.f;  // a zero row passes through (out = h)
    float ce = 0.f;                               // inference: energy of the correction s * a_4

    // the tile start is kept in a scalar register (readfirstlane): the loop
    // holds barriers, and its exit must stay uniform even where the compiler
    // computes the increment on divergent paths
    for (int t0 = 0; t0 < U; t0 = __builtin_amdgcn_readfirstlane(t0 + TO)) {
      __syncthreads();  // the previous tile's readers are done
      for (int i = tid; i < NPOS; i += kBlock) {
        const int p = t0 - BASE_F + i;
        const float2 v = (p >= 0 && p < U) ? hrow[p] : make_float2(0.f, 0.f);
        const uint32_t pk = pack2(v.x * inv, v.y * inv);
        X0[i] = pk;
        if (TRAIN && p >= t0 && p < t0 + TO && p < U) {
          io.X0[(row * 2 + 0) * UP + p] = (bfbits)(pk & 0xFFFFu);
          io.X0[(row * 2 + 1) * UP + p] = (bfbits)(pk >> 16);
        }
      }
      __syncthreads();
      // layer 1: x0 -> A
      for (int u = wave; u < U1; u += 4) {
        const int idx = 3 + 16 * u + r;  // LDS index of this lane's output position
        const int p = t0 - 9 + 16 * u + r;
        const bf16x8 bv = read4(X0, idx - 3 + 4 * q);
        f32x4 acc[2];
        bias_init(acc, b1);
        acc[0] = mfma(w1[0], bv, acc[0]);
        acc[1] = mfma(w1[1], bv, acc[1]);
        const bool in = p >= 0 && p < U;
        relu_unit(acc, t0 - 9 + 16 * u, U);
        store_unit(XA, idx, acc);
        if (TRAIN && in && p >= t0 && p < t0 + TO) store_global(io.X1 + row * 32 * UP, UP, p, acc);
      }
      __syncthreads();
      if (TRAIN) store_masks(XA, t0, U, io.M1 + row * UP);
      // layer 2: A -> B
      if constexpr (!TRAIN) layer32_paired<U2>(XA, XB, 6, t0 - 6, U, w2, b2);
      else for (int u = wave; u < U2; u += 4) {
        const int idx = 6 + 16 * u + r;
        const int p = t0 - 6 + 16 * u + r;
        f32x4 acc[2];
        bias_init(acc, b2);
        unit32<1>(XA, 6 + 16 * u - 3, w2, acc);
        const bool in = p >= 0 && p < U;
        relu_unit(acc, t0 - 6 + 16 * u, U);
        store_unit(XB, idx, acc);
        if (TRAIN && in && p >= t0 && p < t0 + TO) store_global(io.X2 + row * 32 * UP, UP, p, acc);
      }
      __syncthreads();
      if (TRAIN) store_masks(XB, t0, U, io.M2 + row * UP);
      // layer 3: B -> A
      if constexpr (!TRAIN) layer32_paired<U3>(XB, XA, 9, t0 - 3, U, w3, b3);
      else for (int u = wave; u < U3; u += 4) {
        const int idx = 9 + 16 * u + r;
        const int p = t0 - 3 + 16 * u + r;
        f32x4 acc[2];
        bias_init(acc, b3);
        unit32<1>(XB, 9 + 16 * u - 3, w3, acc);
        const bool in = p >= 0 && p < U;
        relu_unit(acc, t0 - 3 + 16 * u, U);
        store_unit(XA, idx, acc);
        if (TRAIN && in && p >= t0 && p < t0 + TO) store_global(io.X3 + row * 32 * UP, UP, p, acc);
      }
      __syncthreads();
      if (TRAIN) store_masks(XA, t0, U, io.M3 + row * UP);
      // layer 4, taps folded into the MFMA rows: P[(co, k)][p] = sum_ci
      // W4[co][ci][k] x3[ci][p] (rows co * 7 + k, 14 of 16 used) for positions
      // t0 - 3 .. t0 + 252, kept in LDS as float [row][position] in buffer B
      // (so the tap sums below read consecutive words)
      float* Pb = reinterpret_cast<float*>(XB);
      for (int u = wave; u < U4P; u += 4) {
        const bf16x8 bv = as_bf16x8(*reinterpret_cast<const uint4*>(XA + (9 + 16 * u + r) * RS + 8 * q));
        const f32x4 acc = mfma(w4, bv, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int i = 0; i < 4; i++)
          if (4 * q + i < 14) Pb[(4 * q + i) * PS + 16 * u + r] = acc[i];
      }
      __syncthreads();
      // out[co][p] = b4[co] + sum_k P[(co, k)][p + k - 3]
      const int nt = min(TO, U - t0);  // positions of this tile (a uniform bound: no early exit before
                                       // the next tile's barrier)
      for (int i = tid; i < nt; i += kBlock) {
        const int p = t0 + i;
        float o0 = b4[0], o1 = b4[1];
#pragma unroll
        for (int k = 0; k < 7; k++) {
          o0 += Pb[k * PS + i + k];
          o1 += Pb[(7 + k) * PS + i + k];
        }
        const float2 h = hrow[p];
        if (!TRAIN) {
          Hout[row * U + p] = make_float2(fmaf(s, o0, h.x), fmaf(s, o1, h.y));
          const float cx = s * o0, cy = s * o1;
          ce = fmaf(cx, cx, fmaf(cy, cy, ce));
        } else {
          const float2 t = io.Htrue[row * U + p];
          const float ex = h.x * inv + o0 - t.x * inv;
          const float ey = h.y * inv + o1 - t.y * inv;
          const bool live = s > 0.f;
          if (live) loss = fmaf(ex, ex, fmaf(ey, ey, loss));
          const float c = live ? 2.0f * io.inv_count : 0.f;
          io.D4[(row * 2 + 0) * UP + p] = (bfbits)bf16_bits(c * ex);
          io.D4[(row * 2 + 1) * UP + p] = (bfbits)bf16_bits(c * ey);
        }
      }
    }
    if (!TRAIN) {
      // LS fallback: the row keeps its LS estimate when the correction's
      // energy is not finite or exceeds max_corr^2 times the row's own (NaN
      // compares false, so it falls back too).  The rewrite uses the thread
      // that wrote each position above, so it lands after that store.
      const float E = block_sum(ce, red);
      const bool fell = !__builtin_isfinite(E) || !(E <= io.fb_max2 * hs);
      if (fell) {
        for (int t0 = 0; t0 < U; t0 += TO)
          for (int i = tid; i < min(TO, U - t0); i += kBlock) Hout[row * U + t0 + i] = hrow[t0 + i];
      }
      if (tid == 0 && io.fell) io.fell[row] = fell ? 1 : 0;
    }
  }
  if (TRAIN) {
    const float tot = block_sum(loss, red);
    if (tid == 0) io.loss_part[blockIdx.x] = tot * io.inv_count;
  }
}

// ------------------------------------------------------------------ backward (data)
// Tile layout (LDS index of position p is p - t0 + 18):
//   d4   positions t0-18 .. t0+269  (2 channels)
//   g3   computed for t0-6 + [0, 256) (16 units) -> d3 = g3 [x3 > 0] -> buffer A
//   g2   computed for t0-3 + [0, 256) (16 units) -> d2 = g2 [x2 > 0] -> buffer B
//   g1   computed for t0   + [0, 240) (15 units) -> d1 = g1 [x1 > 0]
// The transposed layer 4 has K = 32 slots (tap 3+4q-j/2, channel j%2) of which
// taps 0..6 are real: lane quarter q reads d4 at p-4q .. p-4q+3.
__device__ __forceinline__ void mask_unit(f32x4 (&acc)[2], const uint32_t* __restrict__ Mg, int p, bool in) {
  const int q = (threadIdx.x & 63) >> 4;
  const uint32_t m = in ? Mg[p] : 0u;
#pragma unroll
  for (int h = 0; h < 2; h++)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const bool on = (m >> (16 * h + 4 * q + i)) & 1u;
      // round to bf16 here: the delta enters the next products and the
      // weight gradient as bf16
      acc[h][i] = on ? bf16_float(bf16_bits(acc[h][i])) : 0.f;
    }
}

__global__ __launch_bounds__(kBlock) void dn_backward_kernel(int64_t rows, int U, const bf16x8* __restrict__ frag,
                                                             DnTrainIo io) {
  extern __shared__ __align__(16) unsigned char smem[];
  bfbits* DA = reinterpret_cast<bfbits*>(smem);
  bfbits* DB = DA + NPOS * RS;
  uint32_t* D4s = reinterpret_cast<uint32_t*>(DB + NPOS * RS);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, q = lane >> 4;
  bf16x8 g4[2], g3[2][7], g2[2][7];
#pragma unroll
  for (int h = 0; h < 2; h++) {
    g4[h] = frag[kG4 + h * 64 + lane];
#pragma unroll
    for (int k = 0; k < 7; k++) {
      g3[h][k] = frag[kG3 + (h * 7 + k) * 64 + lane];
      g2[h][k] = frag[kG2 + (h * 7 + k) * 64 + lane];
    }
  }
  for (int i = tid; i < 2 * NPOS * RS / 2; i += kBlock) reinterpret_cast<uint32_t*>(DA)[i] = 0u;
  const int64_t UP = io.UP;

  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const bfbits* d4r = io.D4 + row * 2 * UP;
    for (int t0 = 0; t0 < U; t0 += TO) {
      __syncthreads();
      for (int i = tid; i < NPOS; i += kBlock) {
        const int p = t0 - BASE_B + i;
        D4s[i] = (p >= 0 && p < U) ? (uint32_t)d4r[p] | ((uint32_t)d4r[UP + p] << 16) : 0u;
      }
      __syncthreads();
      // transposed layer 4: d4 -> d3 (buffer A)
      for (int u = wave; u < BU3; u += 4) {
        const int idx = 12 + 16 * u + r;
        const int p = t0 - 6 + 16 * u + r;
        f32x4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
        const bf16x8 bv = read4(D4s, idx - 4 * q);
        acc[0] = mfma(g4[0], bv, acc[0]);
        acc[1] = mfma(g4[1], bv, acc[1]);
        const bool in = p >= 0 && p < U;
        mask_unit(acc, io.M3 + row * UP, p, in);
        store_unit(DA, idx, acc);
        if (in && p >= t0 && p < t0 + TO) store_global(io.D3 + row * 32 * UP, UP, p, acc);
      }
      __syncthreads();
      // transposed layer 3: d3 -> d2 (buffer B)
      for (int u = wave; u < BU2; u += 4) {
        const int idx = 15 + 16 * u + r;
        const int p = t0 - 3 + 16 * u + r;
        f32x4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
        unit32<-1>(DA, 15 + 16 * u + 3, g3, acc);
        const bool in = p >= 0 && p < U;
        mask_unit(acc, io.M2 + row * UP, p, in);
        store_unit(DB, idx, acc);
        if (in && p >= t0 && p < t0 + TO) store_global(io.D2 + row * 32 * UP, UP, p, acc);
      }
      __syncthreads();
      // transposed layer 2: d2 -> d1 (global only)
      for (int u = wave; u < BU1; u += 4) {
        const int p = t0 + 16 * u + r;
        f32x4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
        unit32<-1>(DB, 18 + 16 * u + 3, g2, acc);
        const bool in = p < U;
        mask_unit(acc, io.M1 + row * UP, p, in);
        if (in) store_global(io.D1 + row * 32 * UP, UP, p, acc);
      }
    }
  }
}

// ------------------------------------------------------------------ weight gradients
// Chunks of 64 positions of one row are staged channel-major in LDS:
// deltas dT[co][0..63] (row stride 72) and inputs xT[ci][0..79] holding
// positions q0-8 .. q0+71 (row stride 88; both strides make the 16-byte
// fragment reads conflict-free).  Per 32-position K step, lane (r, q) of the
// A operand reads delta row co = r at positions 8q..8q+7; the B operand for
// tap k needs input row ci = r at positions 8q+k-3 .. 8q+k+4, cut out of
// three aligned 16-byte reads with a compile-time shift.
constexpr int CHUNK = 64, DT_RS = 72, XT_RS = 88;

template <int O>
__device__ __forceinline__ bf16x8 shifted(const uint4& cm, const uint4& c0, const uint4& cp) {
  const uint32_t D[12] = {cm.x, cm.y, cm.z, cm.w, c0.x, c0.y, c0.z, c0.w, cp.x, cp.y, cp.z, cp.w};
  uint32_t o[4];
#pragma unroll
  for (int t = 0; t < 4; t++) {
    constexpr int base = 8 + O;
    const int e = base + 2 * t;  // element index of the dword's low half
    if constexpr ((base & 1) == 0)
      o[t] = D[e >> 1];
    else
      o[t] = (D[e >> 1] >> 16) | (D[(e >> 1) + 1] << 16);
  }
  return as_bf16x8(make_uint4(o[0], o[1], o[2], o[3]));
}

template <int K>
__device__ __forceinline__ void tap_mfma(const uint4& cm, const uint4& c0, const uint4& cp, const bf16x8& a,
                                         f32x4& acc) {
  acc = mfma(a, shifted<K - 3>(cm, c0, cp), acc);
}

// Stage channels [0, nch) of G (channel-major, pitch UP) for positions
// q0+off .. q0+off+8*n8-1 into T (row stride rs), zero outside [0, U).
__device__ __forceinline__ void stage(bfbits* __restrict__ T, int rs, const bfbits* __restrict__ G, int64_t UP,
                                      int nch, int q0, int off, int n8, int U) {
  for (int i = threadIdx.x; i < nch * n8; i += kBlock) {
    const int ch = i / n8, c = i % n8;
    const int p = q0 + off + 8 * c;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (p >= 0 && p < U) {
      v = *reinterpret_cast<const uint4*>(G + ch * UP + p);
      if (p + 8 > U) {  // zero the positions past U
        uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 8; j++)
          if (p + j >= U) w[j >> 1] &= (j & 1) ? 0x0000FFFFu : 0xFFFF0000u;
        v = make_uint4(w[0], w[1], w[2], w[3]);
      }
    }
    *reinterpret_cast<uint4*>(T + ch * rs + 8 * c) = v;
  }
}

// Accumulate the weight gradient of one layer over rows [r0, r1).
// CIN, COUT in {2, 32}.  Wave roles: for 32 x 32 layers wave w owns output
// channel half w&1 and input channel half w>>1, all 7 taps; for layers with
// 2 channels on one side, wave w owns half w&1 of the 32-channel side and
// the taps of parity w>>1.
template <int CIN, int COUT>
__device__ void wgrad_layer(const bfbits* __restrict__ D, const bfbits* __restrict__ X, int64_t UP, int U,
                            int64_t r0, int64_t r1, bfbits* dT, bfbits* xT, float* __restrict__ out_w,
                            float* __restrict__ out_b) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, q = lane >> 4;
  constexpr bool FULL = CIN == 32 && COUT == 32;
  const int ch_half = wave & 1;       // output-channel half (FULL, or CIN == 2) / input half (COUT == 2)
  const int other_half = wave >> 1;   // input-channel half (FULL) / tap parity (otherwise)
  f32x4 acc[7];
#pragma unroll
  for (int k = 0; k < 7; k++) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;
  // rows of the A (delta) and B (input) operands this lane reads
  const int co_row = COUT == 32 ? 16 * ch_half + r : r;                      // valid if < COUT
  const int ci_row = CIN == 32 ? 16 * (FULL ? other_half : ch_half) + r : r;  // valid if < CIN
  const bool a_ok = co_row < COUT, b_ok = ci_row < CIN;

  for (int64_t row = r0; row < r1; row++) {
    for (int q0 = 0; q0 < U; q0 += CHUNK) {
      __syncthreads();
      stage(dT, DT_RS, D + row * COUT * UP, UP, COUT, q0, 0, CHUNK / 8, U);
      stage(xT, XT_RS, X + row * CIN * UP, UP, CIN, q0, -8, CHUNK / 8 + 2, U);
      __syncthreads();
      if (tid < COUT) {
        float sacc = 0.f;
        for (int j = 0; j < CHUNK; j++) sacc += bf16_float(dT[tid * DT_RS + j]);
        bacc += sacc;
      }
#pragma unroll
      for (int ks = 0; ks < CHUNK / 32; ks++) {
        const int pos = 32 * ks + 8 * q;
        const uint4 z = make_uint4(0u, 0u, 0u, 0u);
        const uint4 av = a_ok ? *reinterpret_cast<const uint4*>(dT + co_row * DT_RS + pos) : z;
        const bf16x8 a = as_bf16x8(av);
        const bfbits* xr = xT + ci_row * XT_RS + 8 + pos;
        const uint4 cm = b_ok ? *reinterpret_cast<const uint4*>(xr - 8) : z;
        const uint4 c0 = b_ok ? *reinterpret_cast<const uint4*>(xr) : z;
        const uint4 cp = b_ok ? *reinterpret_cast<const uint4*>(xr + 8) : z;
        if constexpr (FULL) {
          tap_mfma<0>(cm, c0, cp, a, acc[0]);
          tap_mfma<1>(cm, c0, cp, a, acc[1]);
          tap_mfma<2>(cm, c0, cp, a, acc[2]);
          tap_mfma<3>(cm, c0, cp, a, acc[3]);
          tap_mfma<4>(cm, c0, cp, a, acc[4]);
          tap_mfma<5>(cm, c0, cp, a, acc[5]);
          tap_mfma<6>(cm, c0, cp, a, acc[6]);
        } else if (other_half == 0) {
          tap_mfma<0>(cm, c0, cp, a, acc[0]);
          tap_mfma<2>(cm, c0, cp, a, acc[2]);
          tap_mfma<4>(cm, c0, cp, a, acc[4]);
          tap_mfma<6>(cm, c0, cp, a, acc[6]);
        } else {
          tap_mfma<1>(cm, c0, cp, a, acc[1]);
          tap_mfma<3>(cm, c0, cp, a, acc[3]);
          tap_mfma<5>(cm, c0, cp, a, acc[5]);
        }
      }
    }
  }
  // C: lane (r, q), register i -> output channel row 4q+i of the A half, input column r of the B half
#pragma unroll
  for (int k = 0; k < 7; k++) {
    const bool mine = FULL || ((k & 1) == other_half);
    if (!mine) continue;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int co = (COUT == 32 ? 16 * ch_half : 0) + 4 * q + i;
      const int ci = (CIN == 32 ? 16 * (FULL ? other_half : ch_half) : 0) + r;
      if (co < COUT && ci < CIN) out_w[(co * CIN + ci) * 7 + k] = acc[k][i];
    }
  }
  if (tid < COUT) out_b[tid] = bacc;
}

__global__ __launch_bounds__(kBlock) void dn_wgrad_kernel(int64_t rows, int U, DnTrainIo io) {
  __shared__ __align__(16) bfbits dT[32 * DT_RS];
  __shared__ __align__(16) bfbits xT[32 * XT_RS];
  const int64_t G = gridDim.x;
  const int64_t r0 = rows * blockIdx.x / G, r1 = rows * (blockIdx.x + 1) / G;
  float* part = io.part + (int64_t)blockIdx.x * kParams;
  const int64_t UP = io.UP;
  // one layer per workgroup (grid y): each parameter of partial vector
  // blockIdx.x is written by exactly one workgroup
  switch (blockIdx.y) {
    case 0: wgrad_layer<2, 32>(io.D1, io.X0, UP, U, r0, r1, dT, xT, part + kPW1, part + kPB1); break;
    case 1: wgrad_layer<32, 32>(io.D2, io.X1, UP, U, r0, r1, dT, xT, part + kPW2, part + kPB2); break;
    case 2: wgrad_layer<32, 32>(io.D3, io.X2, UP, U, r0, r1, dT, xT, part + kPW3, part + kPB3); break;
    default: wgrad_layer<32, 2>(io.D4, io.X3, UP, U, r0, r1, dT, xT, part + kPW4, part + kPB4); break;
  }
}

// ------------------------------------------------------------------ reduce + Adam
// grad[i] = sum over workgroup partials g of part[g][i]: a block owns 64
// parameters; its 4 wavefronts sum the partials g = w, w + 4, ... (in order,
// coalesced over the 64 parameters), then wavefront 0 adds the 4 sums in
// order, so the result is deterministic.  Optionally the Adam update of theta,
// m, v (bias corrections c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t) from the
// host).  Block 0 also sums the loss partials.
constexpr int kRedParams = 64;

__global__ __launch_bounds__(kBlock) void dn_reduce_kernel(const float* __restrict__ part, int n_part,
                                                           const float* __restrict__ loss_part, int n_loss,
                                                           float* __restrict__ grad, float* __restrict__ loss,
                                                           AdamArgs adam) {
  __shared__ float sums[4][kRedParams];
  const int j = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * kRedParams + j;
  float acc = 0.f;
  if (i < kParams) {
    int b = w;
    for (; b + 12 < n_part; b += 16) {  // four independent loads in flight
      const float v0 = part[(int64_t)b * kParams + i], v1 = part[(int64_t)(b + 4) * kParams + i];
      const float v2 = part[(int64_t)(b + 8) * kParams + i], v3 = part[(int64_t)(b + 12) * kParams + i];
      acc = (((acc + v0) + v1) + v2) + v3;
    }
    for (; b < n_part; b += 4) acc += part[(int64_t)b * kParams + i];
  }
  sums[w][j] = acc;
  __syncthreads();
  if (w == 0 && i < kParams) {
    const float g = ((sums[0][j] + sums[1][j]) + sums[2][j]) + sums[3][j];
    if (grad) grad[i] = g;
    if (adam.theta) {
      const float m = adam.beta1 * adam.m[i] + (1.0f - adam.beta1) * g;
      const float v = adam.beta2 * adam.v[i] + (1.0f - adam.beta2) * g * g;
      adam.m[i] = m;
      adam.v[i] = v;
      adam.theta[i] -= adam.lr * (m * adam.c1) / (sqrtf(v * adam.c2) + adam.eps);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
    float s = 0.f;
    for (int b = 0; b < n_loss; b++) s += loss_part[b];
    *loss = s;
  }
}

// ------------------------------------------------------------------ weight fragments
// frag element e = unit * 8 + j (unit = fragment block, 16 bytes per lane):
// which parameter (or zero) sits in each MFMA operand slot.
__device__ __forceinline__ int frag_param(int e) {
  const int j = e & 7, unit = e >> 3;
  const int lane = unit & 63, blk = unit >> 6;  // 64 lanes per block
  const int r = lane & 15, q = lane >> 4;
  int b = blk;
  if (b < 2) {  // F1[h]: row co = 16h + r, slot (tap 4q + j/2, channel j%2)
    const int co = 16 * b + r, tap = 4 * q + (j >> 1), ci = j & 1;
    return tap < 7 ? kPW1 + (co * 2 + ci) * 7 + tap : -1;
  }
  b -= 2;
  if (b < 28) {  // F2/F3[h][k]: row co = 16h + r, slot ci = 8q + j
    const int layer = b / 14, hk = b % 14, h = hk / 7, k = hk % 7;
    const int co = 16 * h + r, ci = 8 * q + j;
    return (layer == 0 ? kPW2 : kPW3) + (co * 32 + ci) * 7 + k;
  }
  b -= 28;
  if (b < 1) {  // F4 (taps folded into rows): row r = co * 7 + k (< 14), slot ci = 8q + j
    const int co = r / 7, k = r % 7, ci = 8 * q + j;
    return r < 14 ? kPW4 + (co * 32 + ci) * 7 + k : -1;
  }
  b -= 1;
  if (b < 2) {  // G4[h]: row ci = 16h + r, slot (tap 3 + 4q - j/2, channel j%2)
    const int ci = 16 * b + r, tap = 3 + 4 * q - (j >> 1), co = j & 1;
    return tap <= 6 ? kPW4 + (co * 32 + ci) * 7 + tap : -1;
  }
  b -= 2;
  {  // G3/G2[h][k]: row ci = 16h + r, slot co = 8q + j
    const int layer = b / 14, hk = b % 14, h = hk / 7, k = hk % 7;
    const int ci = 16 * h + r, co = 8 * q + j;
    return (layer == 0 ? kPW3 : kPW2) + (co * 32 + ci) * 7 + k;
  }
}

__global__ __launch_bounds__(kBlock) void dn_relayout_kernel(const float* __restrict__ theta,
                                                             bfbits* __restrict__ frag) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e < kFragUnits * 8) {
    const int pi = frag_param(e);
    frag[e] = pi >= 0 ? (bfbits)bf16_bits(theta[pi]) : (bfbits)0;
  }
}

// ------------------------------------------------------------------ training channels
// Philox4x64-10 (Salmon et al., SC 2011): counter {j, row, 0, 0}, key {seed, 0}.
__device__ __forceinline__ void philox(uint64_t c0, uint64_t c1, uint64_t key, uint64_t (&o)[4]) {
  uint64_t c2 = 0, c3 = 0, k0 = key, k1 = 0;
#pragma unroll
  for (int round = 0; round < 10; round++) {
    if (round > 0) {
      k0 += 0x9E3779B97F4A7C15ull;
      k1 += 0xBB67AE8584CAA73Bull;
    }
    const uint64_t hi0 = __umul64hi(0xD2E7470EE14C6C93ull, c0), lo0 = 0xD2E7470EE14C6C93ull * c0;
    const uint64_t hi1 = __umul64hi(0xCA5A826395121157ull, c2), lo1 = 0xCA5A826395121157ull * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  o[0] = c0;
  o[1] = c1;
  o[2] = c2;
  o[3] = c3;
}

__device__ __forceinline__ float unit_u(uint64_t w) { return (float)(2 * (w >> 41) + 1) * 0x1p-24f; }
__device__ __forceinline__ int int_draw(uint64_t w, int n) { return (int)(((w >> 32) * (uint64_t)n) >> 32); }
__device__ __forceinline__ float2 normal_pair(uint64_t wa, uint64_t wb) {
  const float rr = sqrtf(-2.0f * logf(unit_u(wa)));
  float sn, cs;
  sincospif(2.0f * unit_u(wb), &sn, &cs);
  return make_float2(rr * cs, rr * sn);
}

__global__ __launch_bounds__(kBlock) void dn_gen_kernel(GenArgs g, uint64_t seed, int64_t first_row, int64_t rows,
                                                        float2* __restrict__ Htrue, float2* __restrict__ Hls) {
  extern __shared__ __align__(16) unsigned char smem[];
  float2* tw = reinterpret_cast<float2*>(smem);  // [N]: exp(-2 pi i m / N)
  float2* ht = tw + g.N;                         // [U]
  float2* pil = ht + g.U;                        // [U / ps + 1]
  __shared__ float2 taps[64];
  __shared__ int delays[64];
  const int tid = threadIdx.x, N = g.N, U = g.U, ps = g.ps;
  for (int m = tid; m < N; m += kBlock) {
    float sn, cs;
    sincospif(2.0f * (float)m / (float)N, &sn, &cs);
    tw[m] = make_float2(cs, -sn);
  }
  const int n_pil = (U - 1) / ps + 1;
  const int noise_block = 1 + (g.taps_max + 1) / 2;
  for (int64_t rr = blockIdx.x; rr < rows; rr += gridDim.x) {
    const uint64_t row = (uint64_t)(first_row + rr);
    uint64_t w[4];
    philox(0, row, seed, w);
    const int L = g.taps_min + int_draw(w[0], g.taps_max - g.taps_min + 1);
    const int span = g.tau_min + int_draw(w[1], g.tau_max - g.tau_min + 1);
    const float snr_db = g.snr_min + (g.snr_max - g.snr_min) * unit_u(w[2]);
    __syncthreads();  // previous row's readers of taps / ht / pil are done
    if (tid < L) {
      const int l = tid;
      float psum = 0.f;
      for (int i = 0; i < L; i++) psum += exp10f(-g.decay_db * (float)i / 10.0f);
      const int dl = L > 1 ? (l * span + (L - 1) / 2) / (L - 1) : 0;
      delays[l] = dl < g.CP ? dl : g.CP;
      uint64_t b[4];
      philox((uint64_t)(1 + l / 2), row, seed, b);
      const float2 z = (l % 2 == 0) ? normal_pair(b[0], b[1]) : normal_pair(b[2], b[3]);
      const float a = sqrtf(exp10f(-g.decay_db * (float)l / 10.0f) / psum * 0.5f);
      taps[l] = make_float2(a * z.x, a * z.y);
    }
    __syncthreads();
    for (int d = tid; d < U; d += kBlock) {
      const int f = d < U / 2 ? d - U / 2 : d - U / 2 + 1;
      float2 acc = make_float2(0.f, 0.f);
      for (int l = 0; l < L; l++) {
        const int m = (int)((((int64_t)f * delays[l]) % N + N) % N);
        const float2 e = tw[m], h = taps[l];
        acc.x += h.x * e.x - h.y * e.y;
        acc.y += h.x * e.y + h.y * e.x;
      }
      ht[d] = acc;
      if (Htrue) Htrue[rr * U + d] = acc;
    }
    __syncthreads();
    if (Hls) {
      const float sd = sqrtf(exp10f(-snr_db / 10.0f) * 0.5f);
      for (int j = tid; j < n_pil; j += kBlock) {
        uint64_t b[4];
        philox((uint64_t)(noise_block + j / 2), row, seed, b);
        const float2 z = (j % 2 == 0) ? normal_pair(b[0], b[1]) : normal_pair(b[2], b[3]);
        const float2 h = ht[j * ps];
        pil[j] = make_float2(h.x + sd * z.x, h.y + sd * z.y);
      }
      __syncthreads();
      for (int d = tid; d < U; d += kBlock) Hls[rr * U + d] = comb_value(pil, d, U, ps);
    }
  }
}

}  // namespace dn

// ------------------------------------------------------------------ launchers
namespace {
constexpr int kMaxGrid = 512;
size_t fwd_lds(int U) { return (size_t)2 * dn::NPOS * dn::RS * 2 + dn::NPOS * 4 + (size_t)U * 8; }
size_t bwd_lds() { return (size_t)2 * dn::NPOS * dn::RS * 2 + dn::NPOS * 4; }
}  // namespace

int dn_grid(int64_t rows) { return (int)(rows < kMaxGrid ? rows : kMaxGrid); }

namespace {
__global__ void fill_u8_kernel(uint8_t* __restrict__ p, uint8_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
}  // namespace

hipError_t fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t dn_relayout(const float* theta, uint16_t* frag, hipStream_t st) {
  const int n = kFragUnits * 8;
  hipLaunchKernelGGL(dn::dn_relayout_kernel, dim3((n + dn::kBlock - 1) / dn::kBlock), dim3(dn::kBlock), 0, st,
                     theta, frag);
  return hipGetLastError();
}

hipError_t dn_apply(const float2* Hin, int64_t rows, int U, const void* frag, const float* theta, float2* Hout,
                    float fb_max2, uint8_t* fell, hipStream_t st) {
  DnTrainIo io{};
  io.fb_max2 = fb_max2;
  io.fell = fell;
  hipLaunchKernelGGL(dn::dn_forward_kernel<false>, dim3(dn_grid(rows)), dim3(dn::kBlock), fwd_lds(U), st, Hin,
                     rows, U, reinterpret_cast<const dn::bf16x8*>(frag), theta, Hout, io);
  return hipGetLastError();
}

hipError_t dn_train(const float2* Hin, const float2* Htrue, int64_t rows, int U, const void* frag,
                    const float* theta, const DnTrainIo& io_in, float* grad, float* loss, const AdamArgs& adam,
                    hipStream_t st) {
  DnTrainIo io = io_in;
  io.Htrue = Htrue;
  const int G = dn_grid(rows);
  const auto* fr = reinterpret_cast<const dn::bf16x8*>(frag);
  hipLaunchKernelGGL(dn::dn_forward_kernel<true>, dim3(G), dim3(dn::kBlock), fwd_lds(U), st, Hin, rows, U, fr,
                     theta, (float2*)nullptr, io);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dn::dn_backward_kernel, dim3(G), dim3(dn::kBlock), bwd_lds(), st, rows, U, fr, io);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(dn::dn_wgrad_kernel, dim3(G, 4), dim3(dn::kBlock), 0, st, rows, U, io);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(dn::dn_reduce_kernel, dim3((kParams + dn::kRedParams - 1) / dn::kRedParams), dim3(dn::kBlock), 0, st,
                     (const float*)io.part, G, (const float*)io.loss_part, G, grad, loss, adam);
  return hipGetLastError();
}

hipError_t dn_generate(const GenArgs& g, uint64_t seed, int64_t first_row, int64_t rows, float2* Htrue,
                       float2* Hls, hipStream_t st) {
  const size_t lds = (size_t)g.N * 8 + (size_t)g.U * 8 + (size_t)((g.U - 1) / g.ps + 1) * 8;
  hipLaunchKernelGGL(dn::dn_gen_kernel, dim3(dn_grid(rows)), dim3(dn::kBlock), lds, st, g, seed, first_row, rows,
                     Htrue, Hls);
  return hipGetLastError();
}

}  // namespace rx
