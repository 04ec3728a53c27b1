// rx_kernels.hip -- HIP kernels of the uplink receive path for gfx950.
//
// estimate_kernel  pilot symbol of every (slot, antenna): int16 load with the
//                  CP skipped, FFT, LS divide by the pilot (paper Sec. II-B;
//                  Sec. II-C, LS paragraph), H written in subcarrier order
//                  straight from the FFT's output registers.  With a comb
//                  pilot (every ps-th used subcarrier) the LS values go to
//                  the transform's LDS slot and every subcarrier is then
//                  interpolated from them (comb_value).
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

#include "rx_comb.hpp"
#include "rx_fft.hpp"
#include "rx_launch.h"

// Tuning constants (compile time): wavefronts per demod workgroup.
#ifndef RX_DEMOD_WAVES
#define RX_DEMOD_WAVES 4
#endif
// Symbols a demod wavefront transforms side by side per loop iteration when
// one transform fills the wavefront (N >= 1024): independent work that hides
// the LDS round trips between FFT passes.
#ifndef RX_DEMOD_ILP
#define RX_DEMOD_ILP 1
#endif
// Jobs (transforms of F antennas) per estimate wavefront.
#ifndef RX_EST_JOBS
#define RX_EST_JOBS 4
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
// Transforms a workgroup of W wavefronts runs side by side.
template <int N, int W>
constexpr int transforms_per_group() {
  static_assert((64 * W) % FftShape<N>::L == 0, "a workgroup must hold whole transforms");
  return 64 * W / FftShape<N>::L;
}

// Per-lane constants of the estimate for the spectrum registers that can hold
// a used subcarrier: window register i holds spectrum register qof(i) (the
// window of the demod kernel: q < QH and q >= P - QH; QH = P / 2 is the whole
// spectrum), its subcarrier (-1 when its bin is unused) and that subcarrier's
// pilot factor.
template <int N, int QH = FftShape<N>::P / 2>
struct EstLane {
  static constexpr int NI = 2 * QH;
  static_assert(NI <= FftShape<N>::P, "window wider than the lane's spectrum");
  static constexpr int qof(int i) { return i < QH ? i : FftShape<N>::P - NI + i; }
  int dq[NI];
  float2 pq[NI];
  __device__ __forceinline__ void init(int li, int U, const float2* __restrict__ pf) {
#pragma unroll
    for (int i = 0; i < NI; i++) {
      dq[i] = sub_of_bin(li + FftShape<N>::L * qof(i), N, U);
      pq[i] = pf[dq[i] >= 0 ? dq[i] : 0];  // clamped load; unused bins are never stored
    }
  }
};

// One pilot symbol (samples unpacked into v): FFT, LS by the pilot factors,
// H row out (hrow null: nothing stored).  COMB: a comb pilot (every ps-th
// used subcarrier): the LS values go to the transform's LDS slot and every
// subcarrier is interpolated from them.  Only the window's spectrum registers
// are used, so the last pass computes nothing else.  Ends with an exchange
// fence.
template <int N, int S, bool LL, int QH, bool COMB>
__device__ __forceinline__ void estimate_job(float2 (&v)[FftShape<N>::P], const EstLane<N, QH>& el, float2* buf,
                                             int li, const FftTwiddles<N, S, LL>& twr, float2* __restrict__ hrow,
                                             int U, int ps) {
  using Sh = FftShape<N>;
  using El = EstLane<N, QH>;
  fft_in_regs<N>(v, buf, li, twr);
  if constexpr (!COMB) {
    if (hrow) {
#pragma unroll
      for (int i = 0; i < El::NI; i++)
        if (el.dq[i] >= 0) hrow[el.dq[i]] = cmul(v[Spectrum<N, S>::reg(El::qof(i))], el.pq[i]);
    }
  } else {
    // comb: LS on the pilot subcarriers into this transform's LDS slot (the
    // FFT's last LDS reads are behind), then every subcarrier
    exchange_fence<N>();
#pragma unroll
    for (int i = 0; i < El::NI; i++)
      if (el.dq[i] >= 0 && el.dq[i] % ps == 0)
        buf[el.dq[i] / ps] = cmul(v[Spectrum<N, S>::reg(El::qof(i))], el.pq[i]);
    exchange_fence<N>();
    if (hrow)
      for (int d = li; d < U; d += Sh::L) hrow[d] = comb_value(buf, d, U, ps);
  }
  exchange_fence<N>();  // this job's LDS reads precede the next job's writes
}

// LS estimate of one slot's antennas a_wg .. a_wg + TPW*J - 1: transform slot
// ts = tid / L of the workgroup takes antennas a_wg + ts + j*TPW, j < J, the
// next job's samples requested before the current transform.  slot_iq: the
// slot's samples [T][A][CP+N]; Hs: its estimate [A][U].  The loop bound is
// uniform over whoever shares an exchange fence (the wavefront, or the
// workgroup for two-wavefront transforms): a transform whose antenna is past
// A transforms a valid antenna's samples and stores nothing.
template <int N, int W, int J, int QH, bool COMB, int S, bool LL>
__device__ __forceinline__ void estimate_tile(const uint32_t* __restrict__ slot_iq, int A, int CP, int U,
                                              const float2* __restrict__ pf, float2* __restrict__ Hs,
                                              int a_wg, float2* lds, const FftTwiddles<N, S, LL>& twr, int ps) {
  using Sh = FftShape<N>;
  constexpr int TPW = transforms_per_group<N, W>();
  const int li = threadIdx.x % Sh::L, ts = threadIdx.x / Sh::L;
  const int f = ts % Sh::F;
  // antenna whose validity ends the loop: the wavefront's first, or the
  // workgroup's first when a transform spans wavefronts
  const int a_lead = Sh::WPT > 1 ? a_wg : a_wg + ts - f;
  if (a_lead >= A) return;
  EstLane<N, QH> el;
  el.init(li, U, pf);
  const uint32_t* pilot_sym = slot_iq + CP;  // symbol 0
  // record of antenna a, or of the (valid) lead antenna lead when a >= A
  auto rec_of = [&](int a, int lead) { return pilot_sym + (int64_t)(a < A ? a : lead) * (N + CP); };
  float2* buf = lds + ts * Lds<N>::kSlot;
  uint32_t nxt[Sh::P];
  load_symbol<N>(nxt, rec_of(a_wg + ts, a_lead), li, a_wg + ts < A);
#pragma unroll 1
  for (int j = 0; j < J; j++) {
    const int lead = a_lead + j * TPW;
    if (lead >= A) break;
    const int a = a_wg + ts + j * TPW;
    float2 v[Sh::P];
    unpack_symbol<N>(v, nxt);
    if (j + 1 < J && lead + TPW < A) load_symbol<N>(nxt, rec_of(a + TPW, lead + TPW), li, a + TPW < A);
    estimate_job<N, S, LL, QH, COMB>(v, el, buf, li, twr, a < A ? Hs + (int64_t)a * U : nullptr, U, ps);
  }
}

// Fill the last-pass twiddle table (once per workgroup) and load this lane's
// twiddles.  Contains a workgroup barrier when the table is used.
template <int N, int S, bool LL>
__device__ __forceinline__ void tile_setup(FftTwiddles<N, S, LL>& twr, float2* twtab, const float2* __restrict__ tw) {
  if constexpr (FftTwiddles<N, S, LL>::kLdsLast) {
    FftTwiddles<N, S, LL>::P3Lds::fill(twtab, tw, threadIdx.x, blockDim.x);
    __syncthreads();
  }
  twr.load(tw, threadIdx.x % FftShape<N>::L, twtab);
}

// Uniform slots: workgroup = (slot, group of W*F*J antennas).
// Last-pass twiddles of the estimate kernels: in VGPRs where the kernel runs
// 2 wavefronts per SIMD either way (N >= 1024 in the workgroup grid below;
// every batch kernel), in the LDS table where VGPRs would cost a wavefront
// (N = 512, and the resident-grid kernel at 3 per SIMD).
template <int N>
constexpr bool estimate_twiddles_in_lds() { return N < 1024; }

// The N = 2048 estimate with the 5-register window needs a register budget
// of 3 wavefronts per SIMD to stay there (the compiler otherwise takes 170
// VGPRs and drops to 2).
template <int N, int QH, bool COMB>
constexpr int estimate_min_waves() { return N == 2048 && QH <= 5 && !COMB ? 3 : 1; }

template <int N, int W, int J, int QH, bool COMB>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(estimate_min_waves<N, QH, COMB>())))
void estimate_kernel(const uint32_t* __restrict__ iq, int A, int T, int CP,
                                                          int U, const float2* __restrict__ tw,
                                                          const float2* __restrict__ pf, float2* __restrict__ H,
                                                          int blocks_per_slot, int ps) {
  using Tw = FftTwiddles<N, 0, estimate_twiddles_in_lds<N>()>;
  extern __shared__ float2 lds[];
  __shared__ float2 twtab[Tw::kLdsFloat2 > 0 ? Tw::kLdsFloat2 : 1];
  Tw twr;
  tile_setup(twr, twtab, tw);
  const int64_t s = blockIdx.x / blocks_per_slot;
  const int blk = blockIdx.x % blocks_per_slot;
  const int a_wg = blk * (transforms_per_group<N, W>() * J);
  estimate_tile<N, W, J, QH, COMB>(iq + s * T * (int64_t)A * (N + CP), A, CP, U, pf, H + s * A * (int64_t)U, a_wg,
                                   lds, twr, ps);
}

// Staged sample loads for transforms of at most 8 lanes (F >= 8 per
// wavefront), where direct loads would give each load instruction L dwords of
// each of F records: the records of a wavefront's job are read as 16-byte
// pieces that cover them end to end (lane l, load q: dwords 4 (64 q + l) ..
// + 3 of the F records laid end to end), then reordered.  The 16-byte pieces
// of a wavefront's F records go to its LDS area, record f at dword f * kSt,
// and each lane reads back its first-pass inputs x[li + r N / 16].  Ends
// with the LDS area free again (wavefront-order fences around the reads).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int N>
struct Staged {
  using Sh = FftShape<N>;
  static constexpr int kSt = N + Sh::L;             // dwords per record in LDS
  static constexpr int kLoads = Sh::F * N / 256;    // 16-byte loads per lane (F N = 1024: 4)
  static_assert(Sh::F * kSt <= 2 * Sh::F * Lds<N>::kSlot, "staging fits the exchange area");
  static __device__ __forceinline__ void reorder(uint32_t (&raw)[Sh::P], const u32x4 (&w)[kLoads], uint32_t* stg,
                                                 int f, int li) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < kLoads; q++) {
      const int e = 4 * (64 * q + lane), fq = e / N;
      *reinterpret_cast<u32x4*>(stg + fq * kSt + (e - fq * N)) = w[q];
    }
    wave_fence();
#pragma unroll
    for (int r = 0; r < Sh::P; r++) raw[r] = stg[f * kSt + li + r * (N / 16)];
    wave_fence();
  }
};

// Uniform slots, transforms within one wavefront (N <= 1024): a grid of
// resident workgroups only; transform slot g of the grid (G in all) takes jobs
// g, g + G, ... of the S*A list of (slot, antenna) pilot symbols, the next
// job's samples requested before the current transform.  Every wavefront then
// ends within one job of the others, where (slot, group) workgroups leave a
// partial last round of workgroups running alone whenever their count exceeds
// what the GPU holds at once (c2: 3200 wavefronts against 3072 resident), and
// short transforms of small antenna counts would leave most slots idle.  The
// F slots of a wavefront hold consecutive jobs; the loop runs while the
// wavefront's first job exists, and a slot past the end transforms the last
// job's samples and stores nothing.
template <int N, int W, bool STAGED, int QH, bool COMB>
__global__ __launch_bounds__(64 * W) void estimate_grid_kernel(const uint32_t* __restrict__ iq, int64_t S, int A,
                                                               int T, int CP, int U, const float2* __restrict__ tw,
                                                               const float2* __restrict__ pf,
                                                               float2* __restrict__ H, int ps) {
  using Sh = FftShape<N>;
  static_assert(Sh::WPT == 1, "a transform within one wavefront");
  extern __shared__ float2 lds[];
  __shared__ float2 twtab[FftTwiddles<N>::kLdsFloat2 > 0 ? FftTwiddles<N>::kLdsFloat2 : 1];
  FftTwiddles<N> twr;
  tile_setup<N>(twr, twtab, tw);
  const int li = threadIdx.x % Sh::L, ts = threadIdx.x / Sh::L;
  const int f = ts % Sh::F;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t jobs = S * A;
  const int64_t G = (int64_t)gridDim.x * W * Sh::F;
  int64_t j0 = ((int64_t)blockIdx.x * W + wave) * Sh::F;  // the wavefront's first job (uniform)
  if (j0 >= jobs) return;                                 // no workgroup barrier below
  EstLane<N, QH> el;
  el.init(li, U, pf);
  // (slot, antenna) of this slot's job j, advanced by G per step without a
  // division (meaningless once j is past the list: the last job is read)
  int64_t j = j0 + f;
  const int Gs = (int)(G / A), Ga = (int)(G % A);
  int64_t s = j / A;
  int a = (int)(j - s * A);
  auto rec = [&](int64_t jj, int64_t ss, int aa) {
    if (jj >= jobs) {
      ss = S - 1;
      aa = A - 1;
    }
    return iq + (ss * T * A + aa) * (int64_t)(N + CP) + CP;
  };
  float2* buf = lds + ts * Lds<N>::kSlot;
  // STAGED: this lane's 16-byte pieces belong to the jobs j0 + fq of the
  // wavefront's slots fq, whose (slot, antenna) advance like the slot's own
  using Sg = Staged<N>;
  constexpr int NQ = STAGED ? Sg::kLoads : 1;
  int64_t jq[NQ], sq[NQ];
  int aq[NQ], nq[NQ];
  if constexpr (STAGED) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < NQ; q++) {
      const int e = 4 * (64 * q + lane), fq = e / N;
      nq[q] = e - fq * N;
      jq[q] = j0 + fq;
      sq[q] = jq[q] / A;
      aq[q] = (int)(jq[q] - sq[q] * A);
    }
  }
  uint32_t* stg = reinterpret_cast<uint32_t*>(lds + wave * Sh::F * Lds<N>::kSlot);
  uint32_t nxt[STAGED ? 1 : Sh::P];
  u32x4 nx4[NQ];
  auto request = [&]() {
    if constexpr (STAGED) {
#pragma unroll
      for (int q = 0; q < NQ; q++)
        nx4[q] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(rec(jq[q], sq[q], aq[q]) + nq[q]));
    } else {
      load_symbol<N>(nxt, rec(j, s, a), li, true);
    }
  };
  request();
  for (; j0 < jobs; j0 += G) {
    float2 v[Sh::P];
    if constexpr (STAGED) {
      uint32_t raw[Sh::P];
      Sg::reorder(raw, nx4, stg, f, li);
      unpack_symbol<N>(v, raw);
#pragma unroll
      for (int q = 0; q < NQ; q++) {
        jq[q] += G;
        sq[q] += Gs;
        aq[q] += Ga;
        if (aq[q] >= A) {
          aq[q] -= A;
          sq[q]++;
        }
      }
    } else {
      unpack_symbol<N>(v, nxt);
    }
    const int64_t s0 = s, jcur = j;
    const int a0 = a;
    j += G;
    s += Gs;
    a += Ga;
    if (a >= A) {
      a -= A;
      s++;
    }
    if (j0 + G < jobs) request();
    estimate_job<N, 0, true, QH, COMB>(v, el, buf, li, twr, jcur < jobs ? H + (s0 * A + a0) * (int64_t)U : nullptr,
                                       U, ps);
  }
}

// ------------------------------------------------------------------ demod
// Hard decisions of one equalized symbol x (paper Sec. II-C, demodulation):
// per-axis Gray decisions, B bits in the order b0 (Re sign), b1 (Im sign),
// then the amplitude bits of Re and Im alternately, MSB first.  Strict
// comparisons, so ties and -0.0 give 0.
__device__ __forceinline__ uint32_t qam_code(float2 x, int B) {
  const float c16 = 3.16227766016837933f;  // sqrt(10)
  const float c64 = 6.48074069840786023f;  // sqrt(42)
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
  uint32_t acc = 0;
  for (int j = 0; j < B / 2; j++) acc = (acc << 2) | (br[j] << 1) | bi[j];
  return acc;
}

// x = z / g, the MRC output normalised by the channel energy (0 when g = 0),
// as a reciprocal (within 1 ulp) and two products; a subnormal g takes the
// division.
__device__ __forceinline__ float2 mrc_equalize(float2 z, float g) {
  if (g >= 1.17549435e-38f) {
    const float r = __builtin_amdgcn_rcpf(g);
    return make_float2(z.x * r, z.y * r);
  }
  return g > 0.f ? make_float2(z.x / g, z.y / g) : make_float2(0.f, 0.f);
}

// Output of subcarriers 4 qd .. 4 qd + 3 (fewer at the end of the row) of one
// data symbol: sum(d, z, g) adds the partial sums of subcarrier d to z and g
// (ZF: z is already the equalized symbol); x = z / g (0 when g = 0), then the
// decisions, packed MSB-first (4 symbols = B/2 bytes).  xrow, brow: the
// symbol's output rows, or null.
template <bool ZF, typename SumF>
__device__ __forceinline__ void finish_quad(int qd, int U, int B, SumF sum, float2* __restrict__ xrow,
                                            uint8_t* __restrict__ brow) {
  const int nsym = min(4, U - 4 * qd);
  uint32_t acc = 0;  // bits of up to 4 symbols, MSB-first
  for (int e = 0; e < nsym; e++) {
    const int d = 4 * qd + e;
    float2 zz = make_float2(0.f, 0.f);
    float gg = 0.f;
    sum(d, zz, gg);
    float2 x;
    if constexpr (ZF) {
      x = zz;
    } else {
      x = mrc_equalize(zz, gg);
    }
    if (xrow) xrow[d] = x;
    acc = (acc << B) | qam_code(x, B);
  }
  if (brow) {
    const int nbits = nsym * B;  // a multiple of 8
    uint8_t* o = brow + (qd * B) / 2;
    for (int byte = 0; byte < nbits / 8; byte++) o[byte] = (uint8_t)(acc >> (nbits - 8 * (byte + 1)));
  }
}

// One slot as seen by the per-tile routines (pointers already offset to the
// slot; outputs may be null).
struct SlotView {
  const uint32_t* iq;  // samples, [T][A][CP+N] dwords
  const float2* H;     // channel estimate, [A][U]
  float2* xhat;        // [T-1][U]
  uint8_t* bits;       // [T-1][U*B/8]
  int A, T, CP, U, B;
};

// Demodulate data symbol t of one slot with the W wavefronts of the
// workgroup.  Uses the dynamic LDS `lds` (exchange buffers, then the
// reduction rows); every thread of the workgroup must call it.
template <int N, int QH, int W, bool ZF, int S, bool LL>
__device__ __forceinline__ void demod_tile(const SlotView& sv, int t, float2* lds,
                                           const FftTwiddles<N, S, LL>& twr) {
  using Sh = FftShape<N>;
  constexpr int NI = 2 * QH;  // spectrum registers that can hold a used subcarrier
  static_assert(NI <= Sh::P, "window wider than the lane's spectrum");
  const int A = sv.A, CP = sv.CP, U = sv.U, B = sv.B;
  // transform slot ts = tid / L; group tg = ts / F: the wavefront, or the
  // wavefront pair of a two-wavefront transform
  const int li = threadIdx.x % Sh::L, ts = threadIdx.x / Sh::L;
  const int f = ts % Sh::F, tg = ts / Sh::F;
  constexpr int NG = W / Sh::WPT;  // transform groups per workgroup
  const float2* Hs = sv.H;
  const uint32_t* iq = sv.iq;

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
  // One transform per wavefront or pair (F == 1): channel rows are read
  // through a buffer resource over the slot's estimate (A*U*8 < 2^31 bytes;
  // reads past it would return zero) at byte offsets hoff[i] within a row.
  const __amdgpu_buffer_rsrc_t hrs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(Hs), (short)0, A * U * 8, 0x00020000);
  const __amdgpu_buffer_rsrc_t hrs_empty =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(Hs), (short)0, 0, 0x00020000);
  int hoff[Sh::F == 1 ? NI : 1];
  if constexpr (Sh::F == 1) {
#pragma unroll
    for (int i = 0; i < NI; i++) hoff[i] = dcl(i) * 8;
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
        const float2 h = Hs[(int64_t)a * U + dcl(i)];
        g[i] = fmaf(h.x, h.x, fmaf(h.y, h.y, g[i]));
      }
    }
#pragma unroll
    for (int i = 0; i < NI; i++) g[i] = g[i] > 0.f ? 1.0f / g[i] : 0.f;  // now 1/g
  }

  // C symbols (antennas) per lane per iteration; antenna of lane group f and
  // slot c in job J: J*F*C + c*F + f.  Job J = iteration * NG + tg.
  constexpr int C = Sh::F == 1 ? RX_DEMOD_ILP : 1;
  float2* bufs[C];
#pragma unroll
  for (int c = 0; c < C; c++) bufs[c] = lds + ((tg * C + c) * Sh::F + f) * Lds<N>::kSlot;
  float2* const(&buf)[C] = bufs;
  const int64_t sym_base = ((int64_t)t * A) * (N + CP) + CP;
  // Software pipeline over this group's antennas: each job's samples are
  // requested D jobs ahead.
  constexpr int JA = Sh::F * C;  // antennas per job
  const int a_step = NG * JA;
  int a0 = tg * JA;
  constexpr int D = RX_DEMOD_PREFETCH;
  static_assert(D == 1 || D == 2, "prefetch depth 1 or 2");
  // A job's antennas past A read a valid record (the job's first antenna, or
  // antenna A-1 for a two-wavefront transform, whose job may lie wholly past
  // A) and add nothing (their channel rows are taken as zero).
  auto valid_row = [&](int a, int aj) { return a < A ? a : (Sh::WPT > 1 ? A - 1 : aj); };
  auto request = [&](uint32_t (&dst)[C][Sh::P], int aj) {
#pragma unroll
    for (int c = 0; c < C; c++) {
      const int a = aj + c * Sh::F + f;
      load_symbol<N>(dst[c], iq + sym_base + (int64_t)valid_row(a, aj) * (N + CP), li, a < A);
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
      float2 hv[NI];
      if constexpr (Sh::F == 1) {
        // the antenna is uniform over the wavefront: row offset in a scalar
        // register, per-lane offsets loop-invariant, no address arithmetic; a
        // transform past A reads through an empty resource, which returns 0
        // (with one symbol per wavefront job, C == 1, the loop bound already
        // keeps au below A)
        const int au = __builtin_amdgcn_readfirstlane(a);
        const int so = (au < A ? au : A - 1) * (U * 8);
        const __amdgpu_buffer_rsrc_t rs = ((Sh::WPT == 1 && C == 1) || au < A) ? hrs : hrs_empty;
#pragma unroll
        for (int i = 0; i < NI; i++)
          hv[i] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, hoff[i], so, 0));
      } else {
        const float2* hrow = Hs + (int64_t)valid_row(a, aj) * U;
#pragma unroll
        for (int i = 0; i < NI; i++) hv[i] = hrow[dcl(i)];
      }
#pragma unroll
      for (int i = 0; i < NI; i++) {
        // a transform whose antenna is past A must add nothing to its row
        h[c][i] = (Sh::F == 1 || ok) ? hv[i] : make_float2(0.f, 0.f);
      }
    }
    if (aj + D * a_step < A) request(cur, aj + D * a_step);
    fft_rest<N, C>(v, buf, li, twr);
#pragma unroll
    for (int c = 0; c < C; c++)
#pragma unroll
      for (int i = 0; i < NI; i++) {
        const int q = i < QH ? i : Sh::P - NI + i;
        const float2 y = v[c][Spectrum<N, S>::reg(q)];
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
    exchange_fence<N>();  // this job's LDS reads precede the next job's writes
  };
  // D sample buffers used round robin by a loop unrolled D times, so no
  // register copies (which would wait for the loads) are needed.
  uint32_t nxt[D][C][Sh::P];
  if constexpr (Sh::WPT == 1) {
#pragma unroll
    for (int d = 0; d < D; d++)
      if (a0 + d * a_step < A) request(nxt[d], a0 + d * a_step);
    for (; a0 < A; a0 += D * a_step) {
      job(nxt[0], a0);
      if constexpr (D == 2) {
        if (a0 + a_step < A) job(nxt[1], a0 + a_step);
      }
    }
  } else {
    // Exchange fences are workgroup barriers: every group runs the same
    // number of jobs, counted from the workgroup's first antenna.
#pragma unroll
    for (int d = 0; d < D; d++) request(nxt[d], a0 + d * a_step);
    for (int base = 0; base < A; base += D * a_step) {
      job(nxt[0], base + a0);
      if constexpr (D == 2) {
        if (base + a_step < A) job(nxt[1], base + a_step + a0);
      }
    }
  }

  // Cross-group reduction in a fixed order: row ts holds the partial sums of
  // one transform slot's antennas for every used subcarrier (each subcarrier
  // sits in exactly one lane of a transform; h = 0 made invalid antennas
  // contribute zeros).
  constexpr int ROWS = NG * Sh::F;
  __syncthreads();
  float2* rz = lds;                                      // [ROWS][U]
  float* rg = reinterpret_cast<float*>(lds + ROWS * U);  // [ROWS][U]
  const int row = ts;
#pragma unroll
  for (int i = 0; i < NI; i++) {
    if (wok(i)) {
      rz[row * U + li + doff(i)] = z[i];
      if constexpr (!ZF) rg[row * U + li + doff(i)] = g[i];
    }
  }
  __syncthreads();

  const int64_t out_row = t - 1;
  const int nq = (U + 3) / 4;
  for (int qd = threadIdx.x; qd < nq; qd += 64 * W) {
    finish_quad<ZF>(qd, U, B, [&](int d, float2& zz, float& gg) {
      for (int w = 0; w < ROWS; w++) {
        const float2 p = rz[w * U + d];
        zz.x += p.x;
        zz.y += p.y;
        if constexpr (!ZF) gg += rg[w * U + d];
      }
    }, sv.xhat ? sv.xhat + out_row * U : nullptr, sv.bits ? sv.bits + out_row * (U * B / 8) : nullptr);
  }
}

// Where the uniform demod keeps the last pass's twiddles: in VGPRs (no LDS
// reads in the antenna loop) for N = 1024 and 2048 at the widest spectrum
// windows, where the kernel keeps its wavefronts per SIMD (3 at the 5-register
// window, 2 at the 8-register one) and the 5-register kernels were measured
// faster; elsewhere in the LDS table.  The N = 2048 kernel with the 5-register
// window needs a register budget of 3 wavefronts per SIMD to stay there (168
// VGPRs; without the bound the compiler takes 169 and drops to 2).
template <int N, int QH>
constexpr bool demod_twiddles_in_lds() { return !((N == 1024 || N == 2048) && QH >= 5); }
template <int N, int QH>
constexpr int demod_min_waves() { return N == 2048 && QH == 5 ? 3 : 1; }

// Uniform slots: one workgroup per (slot, data symbol).
template <int N, int QH, int W, bool ZF>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(demod_min_waves<N, QH>())))
void demod_kernel(const uint32_t* __restrict__ iq, int64_t S, int A, int T, int CP, int U, int B,
                  const float2* __restrict__ tw, const float2* __restrict__ H, float2* __restrict__ xhat,
                  uint8_t* __restrict__ bits) {
  using Tw = FftTwiddles<N, 0, demod_twiddles_in_lds<N, QH>()>;
  extern __shared__ float2 lds[];
  __shared__ float2 twtab[Tw::kLdsFloat2 > 0 ? Tw::kLdsFloat2 : 1];
  Tw twr;
  tile_setup(twr, twtab, tw);
  const int Td = T - 1;
  const int64_t item = xcd_remap(blockIdx.x, S * Td);
  const int64_t s = item / Td;
  const int t = 1 + (int)(item % Td);
  SlotView sv;
  sv.iq = iq + s * T * (int64_t)A * (N + CP);
  sv.H = H + s * A * (int64_t)U;
  sv.xhat = xhat ? xhat + s * Td * (int64_t)U : nullptr;
  sv.bits = bits ? bits + s * Td * (int64_t)(U * B / 8) : nullptr;
  sv.A = A; sv.T = T; sv.CP = CP; sv.U = U; sv.B = B;
  demod_tile<N, QH, W, ZF>(sv, t, lds, twr);
}

// Several (slot, data symbol) items per workgroup, for transforms shorter than
// a wavefront (F > 1 per wavefront) and for antenna counts too small to share
// among the W wavefronts of one item.  A workgroup takes IPW = F * W / Wa
// consecutive items: Wa wavefronts (1, 2 or 4) share an item's antennas
// (wavefront w takes antennas w % Wa, w % Wa + Wa, ...), and transform slot f
// of wavefront w serves item (w / Wa) * F + f of the workgroup, so one job of
// a wavefront is one antenna of F items.  Each item's Wa partial sums meet in
// LDS rows (row = transform slot, as in demod_tile); x-hat, decisions and
// bits follow per item (paper Sec. II-C, MRC paragraph).
// The N = 1024 items kernel with the 5-register window is held at 3
// wavefronts per SIMD (168 VGPRs; the compiler would otherwise take 169).
template <int N, int QH>
constexpr int demod_items_min_waves() { return N == 1024 && QH == 5 ? 3 : 1; }

template <int N, int QH, int W, bool ZF, bool STAGED>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(demod_items_min_waves<N, QH>())))
void demod_items_kernel(const uint32_t* __restrict__ iq, int64_t S, int A,
                                                             int T, int CP, int U, int B,
                                                             const float2* __restrict__ tw,
                                                             const float2* __restrict__ H,
                                                             float2* __restrict__ xhat, uint8_t* __restrict__ bits,
                                                             int Wa) {
  using Sh = FftShape<N>;
  static_assert(Sh::WPT == 1, "a transform within one wavefront");
  constexpr int NI = 2 * QH;
  static_assert(NI <= Sh::P, "window wider than the lane's spectrum");
  using Tw = FftTwiddles<N, 0, demod_twiddles_in_lds<N, QH>()>;
  extern __shared__ float2 lds[];
  __shared__ float2 twtab[Tw::kLdsFloat2 > 0 ? Tw::kLdsFloat2 : 1];
  Tw twr;
  tile_setup(twr, twtab, tw);

  const int Td = T - 1;
  const int64_t items = S * Td;
  const int IPW = (W / Wa) * Sh::F;
  const int64_t item0 = xcd_remap(blockIdx.x, gridDim.x) * IPW;
  const int li = threadIdx.x % Sh::L, ts = threadIdx.x / Sh::L;
  const int f = ts % Sh::F;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sub = wave % Wa;
  // item of this transform slot (uniform over the wavefront when F == 1); a
  // slot past the last item reads the last item's data and stores nothing
  const int64_t item = item0 + (wave / Wa) * Sh::F + f;
  const int64_t ic = item < items ? item : items - 1;
  const int64_t s = ic / Td;
  const int t = 1 + (int)(ic - s * Td);
  const uint32_t* sym = iq + (s * T + t) * (int64_t)A * (N + CP) + CP;  // antenna 0 of symbol t
  const float2* Hs = H + s * A * (int64_t)U;

  // Spectrum window as in demod_tile: window register i holds spectrum
  // register qof(i), subcarrier li + doff(i) when wok(i); channel loads use
  // that index clamped into [0, U).
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
  // F == 1: the slot's estimate through a buffer resource (uniform base,
  // row offset in a scalar register, loop-invariant lane offsets)
  const __amdgpu_buffer_rsrc_t hrs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(Hs), (short)0, A * U * 8, 0x00020000);
  int hoff[NI];
#pragma unroll
  for (int i = 0; i < NI; i++) hoff[i] = dcl(i) * 8;

  float2* bufs[1] = {lds + ts * Lds<N>::kSlot};
  float2* const(&buf)[1] = bufs;
  // STAGED (transforms of at most 8 lanes): the F records of a job are read
  // as 16-byte pieces that cover them end to end (lane l, load q: dwords
  // 4 (64 q + l) .. + 3 of the F records laid end to end), then reordered
  // through the wavefront's LDS area into the first pass's order (record f at
  // dword f * kSt, kSt = N + L, so the strided reads hit distinct banks).
  // Direct loads would give each instruction L dwords of each of F records.
  using Sg = Staged<N>;
  const uint32_t* srec[STAGED ? Sg::kLoads : 1];
  if constexpr (STAGED) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < Sg::kLoads; q++) {
      const int e = 4 * (64 * q + lane), fq = e / N;
      const int64_t iq_ = item0 + (wave / Wa) * Sh::F + fq;
      const int64_t icq = iq_ < items ? iq_ : items - 1;
      const int64_t sq = icq / Td;
      const int tq = 1 + (int)(icq - sq * Td);
      srec[q] = iq + (sq * T + tq) * (int64_t)A * (N + CP) + CP + (e - fq * N);
    }
  }
  uint32_t* stg = reinterpret_cast<uint32_t*>(lds + wave * Sh::F * Lds<N>::kSlot);
  uint32_t nxt[STAGED ? 1 : Sh::P];
  u32x4 nx4[STAGED ? Sg::kLoads : 1];
  auto request = [&](int aa) {
    if constexpr (STAGED) {
#pragma unroll
      for (int q = 0; q < Sg::kLoads; q++)
        nx4[q] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(srec[q] + (int64_t)aa * (N + CP)));
    } else {
      load_symbol<N>(nxt, sym + (int64_t)aa * (N + CP), li, true);
    }
  };
  if (sub < A) request(sub);
  for (int a = sub; a < A; a += Wa) {  // uniform over the wavefront
    float2 v[1][Sh::P];
    if constexpr (STAGED) {
      uint32_t raw[Sh::P];
      Sg::reorder(raw, nx4, stg, f, li);
      unpack_symbol<N>(v[0], raw);
    } else {
      unpack_symbol<N>(v[0], nxt);
    }
    fft_first_pass<N, 1>(v, buf, li);
    float2 hv[NI];
    if constexpr (Sh::F == 1) {
      const int so = a * (U * 8);
#pragma unroll
      for (int i = 0; i < NI; i++)
        hv[i] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(hrs, hoff[i], so, 0));
    } else {
      const float2* hrow = Hs + (int64_t)a * U;
#pragma unroll
      for (int i = 0; i < NI; i++) hv[i] = hrow[dcl(i)];
    }
    if (a + Wa < A) request(a + Wa);
    fft_rest<N, 1>(v, buf, li, twr);
#pragma unroll
    for (int i = 0; i < NI; i++) {
      const float2 y = v[0][Spectrum<N, 0>::reg(qof(i))];
      const float2 hh = hv[i];
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
    exchange_fence<N>();  // this job's LDS reads precede the next job's writes
  }

  // The workgroup's items are consecutive, so their x-hat rows and bit rows
  // are contiguous.  x-hat and the decision codes (to LDS) come straight from
  // the registers when one wavefront holds an item (Wa == 1); otherwise every
  // transform slot's partial sums go to its LDS row and one thread per
  // subcarrier sums the item's Wa rows in a fixed order.  Then one thread per
  // four codes packs the bits.
  constexpr int ROWS = W * Sh::F;
  const int nitems = (int)min((int64_t)IPW, items - item0);  // the last workgroup may hold fewer
  const int nsub = nitems * U;
  __syncthreads();
  float2* rz = lds;                                      // [ROWS][U]
  float* rg = reinterpret_cast<float*>(lds + ROWS * U);  // [ROWS][U]
  uint8_t* codes = reinterpret_cast<uint8_t*>(rg + ROWS * U);  // [nsub] (+ 4 bytes of slack)
  if (Wa == 1) {
    const int litem = wave * Sh::F + f;
    if (litem < nitems) {
#pragma unroll
      for (int i = 0; i < NI; i++) {
        if (wok(i)) {
          const int d = li + doff(i);
          const float2 x = ZF ? z[i] : mrc_equalize(z[i], g[i]);
          if (xhat) xhat[(item0 + litem) * U + d] = x;
          codes[litem * U + d] = (uint8_t)qam_code(x, B);
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < NI; i++) {
      if (wok(i)) {
        rz[ts * U + li + doff(i)] = z[i];
        if constexpr (!ZF) rg[ts * U + li + doff(i)] = g[i];
      }
    }
    __syncthreads();
    // subcarrier v = litem * U + d, stepped without a division
    constexpr int kStride = 64 * W;
    const int sq = kStride / U, sr = kStride - sq * U;
    int litem = threadIdx.x / U, d = threadIdx.x - litem * U;
    for (int v = threadIdx.x; v < nsub; v += kStride) {
      const int row0 = (litem / Sh::F) * Wa * Sh::F + litem % Sh::F;  // row of wavefront sub 0
      float2 zz = make_float2(0.f, 0.f);
      float gg = 0.f;
      for (int k = 0; k < Wa; k++) {
        const int r = row0 + k * Sh::F;
        const float2 p = rz[r * U + d];
        zz.x += p.x;
        zz.y += p.y;
        if constexpr (!ZF) gg += rg[r * U + d];
      }
      const float2 x = ZF ? zz : mrc_equalize(zz, gg);
      if (xhat) xhat[item0 * U + v] = x;
      codes[v] = (uint8_t)qam_code(x, B);
      d += sr;
      litem += sq;
      if (d >= U) {
        d -= U;
        litem++;
      }
    }
  }
  if (bits) {
    __syncthreads();
    // codes 4k .. 4k+3 (fewer at the end) -> bytes k B / 2 .. of the bit rows
    // (every row is a whole number of bytes, so the rows concatenate)
    uint8_t* out = bits + item0 * (int64_t)(U * B / 8);
    for (int k = threadIdx.x; 4 * k < nsub; k += 64 * W) {
      const int n = min(4, nsub - 4 * k);
      const uint32_t w = *reinterpret_cast<const uint32_t*>(codes + 4 * k);
      uint32_t acc = 0;
      for (int e = 0; e < n; e++) acc = (acc << B) | ((w >> (8 * e)) & 0xffu);
      const int nbytes = n * B / 8;
      for (int byte = 0; byte < nbytes; byte++)
        out[k * (B / 2) + byte] = (uint8_t)(acc >> (n * B - 8 * (byte + 1)));
    }
  }
}

// ------------------------------------------------------------------ batches
// Persistent kernels for a batch of frames sharing one FFT length: each
// workgroup repeatedly takes the next tile from a device work queue (tiles
// are numbered in frame order) and looks its frame up in a tile->frame map.
// Thread 0 first stamps the completion of the workgroup's previous tile when
// it was the last data symbol of its frame (done_index >= 0: the frame's
// completion counter reaches done_last; 100 MHz device clock), then takes the
// next tile.  Doing both here, before the barrier, keeps every path through
// the caller's tile loop uniform (a divergent step at the end of the loop body
// lets the compiler split the loop around its barriers).
__device__ __forceinline__ int next_tile(int* queue, int n_tiles, const int* tile_frame, int* tile_sh,
                                         int* frame_sh, int& frame, int* done_count = nullptr,
                                         unsigned long long* done_time = nullptr, int done_index = -1,
                                         int done_last = 0) {
  if (threadIdx.x == 0) {
    if (done_index >= 0 && atomicAdd(done_count + done_index, 1) == done_last)
      done_time[done_index] = __builtin_amdgcn_s_memrealtime();
    const int tile = atomicAdd(queue, 1);
    *tile_sh = tile;
    *frame_sh = tile < n_tiles ? tile_frame[tile] : -1;
  }
  __syncthreads();
  const int tile = *tile_sh;
  frame = *frame_sh;
  __syncthreads();  // every thread has read both before thread 0 writes the next ones
  return tile;
}

// Batch kernels: S is the radix schedule of the class's transforms.
template <int N, int W, int J, int S>
__global__ __launch_bounds__(64 * W) void batch_estimate_kernel(const FrameDesc* __restrict__ fd,
                                                                const int* __restrict__ tile_frame, int n_tiles,
                                                                BatchIo io, const float2* __restrict__ tw,
                                                                int* queue) {
  extern __shared__ float2 lds[];
  using Tw = FftTwiddles<N, S, false>;  // 2 wavefronts per SIMD either way
  __shared__ float2 twtab[Tw::kLdsFloat2 > 0 ? Tw::kLdsFloat2 : 1];
  __shared__ int tile_sh, frame_sh;
  Tw twr;
  tile_setup<N>(twr, twtab, tw);
  for (;;) {
    int frame;
    const int tile = next_tile(queue, n_tiles, tile_frame, &tile_sh, &frame_sh, frame);
    if (tile >= n_tiles) break;
    const FrameDesc d = fd[frame];
    const int a_wg = (tile - d.est_tile0) * (transforms_per_group<N, W>() * J);
    estimate_tile<N, W, J, FftShape<N>::P / 2, false>(io.iq + d.iq_off, d.A, d.CP, d.U, d.pf, io.H + d.h_off, a_wg,
                                                     lds, twr, 1);
  }
}

template <int N, int QH, int W, int S>
__global__ __launch_bounds__(64 * W) void batch_demod_kernel(const FrameDesc* __restrict__ fd,
                                                             const int* __restrict__ tile_frame, int n_tiles,
                                                             BatchIo io, const float2* __restrict__ tw,
                                                             int* queue, int* done_count,
                                                             unsigned long long* done_time) {
  extern __shared__ float2 lds[];
  // the last-pass twiddle table in LDS keeps the schedule-0 kernels with the
  // narrower window at 3 wavefronts per SIMD; the others run 2 either way and
  // hold the twiddles in VGPRs
  using Tw = FftTwiddles<N, S, (S == 0 && QH <= 5)>;
  __shared__ float2 twtab[Tw::kLdsFloat2 > 0 ? Tw::kLdsFloat2 : 1];
  __shared__ int tile_sh, frame_sh;
  Tw twr;
  tile_setup<N>(twr, twtab, tw);
  int done_index = -1, done_last = 0;  // the previous tile's frame, stamped by next_tile
  for (;;) {
    int frame;
    const int tile = next_tile(queue, n_tiles, tile_frame, &tile_sh, &frame_sh, frame, done_count, done_time,
                               done_index, done_last);
    if (tile >= n_tiles) break;
    const FrameDesc d = fd[frame];
    SlotView sv;
    sv.iq = io.iq + d.iq_off;
    sv.H = io.H + d.h_off;
    sv.xhat = io.xhat ? io.xhat + d.x_off : nullptr;
    sv.bits = io.bits ? io.bits + d.b_off : nullptr;
    sv.A = d.A; sv.T = d.T; sv.CP = d.CP; sv.U = d.U; sv.B = d.B;
    demod_tile<N, QH, W, false>(sv, 1 + tile - d.dem_tile0, lds, twr);
    __syncthreads();  // outputs written and LDS free before the next tile
    done_index = d.index;
    done_last = d.T - 2;  // the frame's last data symbol completes it
  }
}

// Start of a batch: clear the work queues and completion counters, stamp the
// start time (100 MHz device clock).
__global__ void batch_reset_kernel(int* queues, int n_queues, int* done_count, int n_frames,
                                   unsigned long long* start_time) {
  for (int i = threadIdx.x; i < n_queues; i += blockDim.x) queues[i] = 0;
  for (int i = threadIdx.x; i < n_frames; i += blockDim.x) done_count[i] = 0;
  if (threadIdx.x == 0) *start_time = __builtin_amdgcn_s_memrealtime();
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
  const int li = threadIdx.x % Sh::L, ts = threadIdx.x / Sh::L;
  const int f = ts % Sh::F;
  const int64_t st = blockIdx.x / blocks_per_sym;  // s * T + t
  const int blk = blockIdx.x % blocks_per_sym;
  const int a_wg = blk * transforms_per_group<N, W>();
  // first antenna of this thread's wavefront; for a two-wavefront transform
  // the workgroup's first (the exchange fences are workgroup barriers)
  const int a0 = Sh::WPT > 1 ? a_wg : a_wg + ts - f;
  __shared__ float2 twtab[FftTwiddles<N>::kLdsFloat2 > 0 ? FftTwiddles<N>::kLdsFloat2 : 1];
  if constexpr (FftTwiddles<N>::kLdsLast) {
    FftTwiddles<N>::P3Lds::fill(twtab, tw, threadIdx.x, blockDim.x);
    __syncthreads();
  }
  if (a0 >= A) return;  // uniform over whoever shares an exchange fence
  const int a = a_wg + ts;
  const bool valid = a < A;
  const uint32_t* rec = iq + (st * A + (valid ? a : a0)) * (int64_t)(N + CP) + CP;
  uint32_t raw[Sh::P];
  load_symbol<N>(raw, rec, li, valid);
  FftTwiddles<N> twr;
  twr.load(tw, li, twtab);
  float2 v[Sh::P];
  unpack_symbol<N>(v, raw);
  fft_in_regs<N>(v, lds + ts * Lds<N>::kSlot, li, twr);
  if (valid) {
    float2* out = Y + (st * A + a) * (int64_t)N;
#pragma unroll
    for (int q = 0; q < Sh::P; q++) out[li + Sh::L * q] = v[Spectrum<N>::reg(q)];
  }
}

// ------------------------------------------------------------------ launchers
namespace {
constexpr int kWavesEst = 4;
constexpr int kJobsEst = RX_EST_JOBS;  // jobs per estimate wavefront
constexpr int kWavesDemod = RX_DEMOD_WAVES;
constexpr int kWavesFft = 4;

// Exchange buffers of a workgroup of W wavefronts: one per transform.
template <int N, int W>
size_t fft_lds_bytes() {
  return (size_t)transforms_per_group<N, W>() * Lds<N>::kSlot * sizeof(float2);
}

// Dynamic LDS above 64 KB must be allowed per kernel before launching it.
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

// Workgroups of `kernel` (block threads, lds bytes) the current device holds at
// once.  Callers cache the answer per device and kernel instantiation.
template <typename K>
int resident_groups(K kernel, int block, size_t lds, int dev) {
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), block, lds) !=
          hipSuccess)
    return 0;
  return cus * (per_cu > 0 ? per_cu : 1);
}

// Resident workgroups of an estimate_grid_kernel instantiation on the current
// device (0 on error), cached per device for this instantiation; concurrent
// first calls store the same value.
template <int N, int W, bool STAGED, int QH, bool COMB>
int estimate_grid_capacity(size_t lds) {
  static int cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
  if (dev < 64 && cached[dev] > 0) return cached[dev];
  const int n = resident_groups(estimate_grid_kernel<N, W, STAGED, QH, COMB>, 64 * W, lds, dev);
  if (dev < 64 && n > 0) cached[dev] = n;
  return n;
}

// The resident-grid estimate: only as many workgroups as the GPU holds at once.
template <int N, bool STAGED, int QH, bool COMB>
hipError_t estimate_grid_launch(const LaunchArgs& la, float2* H) {
  const size_t lds = fft_lds_bytes<N, kWavesEst>();
  hipError_t e = allow_lds(estimate_grid_kernel<N, kWavesEst, STAGED, QH, COMB>, lds);
  if (e != hipSuccess) return e;
  const int resident = estimate_grid_capacity<N, kWavesEst, STAGED, QH, COMB>(lds);
  if (resident <= 0) return hipErrorInvalidValue;
  constexpr int per_group = transforms_per_group<N, kWavesEst>();
  const int64_t needed = (la.S * la.A + per_group - 1) / per_group;
  const int64_t grid = needed < resident ? needed : resident;
  hipLaunchKernelGGL((estimate_grid_kernel<N, kWavesEst, STAGED, QH, COMB>), dim3((unsigned)grid),
                     dim3(64 * kWavesEst), lds, la.stream, la.iq, la.S, la.A, la.T, la.CP, la.U, la.tw, la.pf, H,
                     la.ps);
  return hipGetLastError();
}

template <int N, int QH, bool COMB>
hipError_t estimate_nq(const LaunchArgs& la, float2* H) {
  if constexpr (FftShape<N>::WPT == 1) {
    if constexpr (FftShape<N>::L <= 8) {
      if (la.CP % 4 == 0 && reinterpret_cast<uintptr_t>(la.iq) % 16 == 0)
        return estimate_grid_launch<N, true, QH, COMB>(la, H);
    }
    return estimate_grid_launch<N, false, QH, COMB>(la, H);
  }
  const int per_block = transforms_per_group<N, kWavesEst>() * kJobsEst;  // antennas per workgroup
  const int bps = (la.A + per_block - 1) / per_block;
  const int64_t grid = la.S * bps;
  const size_t lds = fft_lds_bytes<N, kWavesEst>();
  hipError_t e = allow_lds(estimate_kernel<N, kWavesEst, kJobsEst, QH, COMB>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((estimate_kernel<N, kWavesEst, kJobsEst, QH, COMB>), dim3((unsigned)grid),
                     dim3(64 * kWavesEst), lds, la.stream, la.iq, la.A, la.T, la.CP, la.U, la.tw, la.pf, H, bps,
                     la.ps);
  return hipGetLastError();
}

// The estimate with the demod's register-window tiers for a block pilot (the
// last pass computes only the used window) and the whole spectrum for a comb.
template <int N>
hipError_t estimate_n(const LaunchArgs& la, float2* H) {
  constexpr int L = FftShape<N>::L;
  if (la.ps > 1) return estimate_nq<N, 8, true>(la, H);
  const int need = (la.U / 2 + 1 + L - 1) / L;
  if (need <= 2) return estimate_nq<N, 2, false>(la, H);
  if (need <= 4) return estimate_nq<N, 4, false>(la, H);
  if (need <= 5) return estimate_nq<N, 5, false>(la, H);
  if (need <= 8) return estimate_nq<N, 8, false>(la, H);
  return hipErrorInvalidValue;
}

template <int N>
hipError_t fft_n(const LaunchArgs& la, float2* Y) {
  constexpr int TPW = transforms_per_group<N, kWavesFft>();
  const int bps = (la.A + TPW - 1) / TPW;
  const int64_t grid = la.S * la.T * bps;
  const size_t lds = fft_lds_bytes<N, kWavesFft>();
  hipError_t e = allow_lds(fft_kernel<N, kWavesFft>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((fft_kernel<N, kWavesFft>), dim3((unsigned)grid), dim3(64 * kWavesFft), lds, la.stream, la.iq, la.A, la.T, la.CP, la.tw, Y, bps);
  return hipGetLastError();
}

// Wavefronts per item of demod_items_kernel: every wavefront takes at least
// one antenna, and an item's antennas spread over fewer wavefronts (at least 8
// per wavefront) while the grid still has many wavefronts per resident slot.
int demod_waves_per_item(int A, int64_t items, int F) {
  int wa = kWavesDemod;
  while (wa > 1 && wa > A) wa /= 2;
  while (wa > 1 && A / wa < 8 && items * (wa / 2) / F >= 8192) wa /= 2;
  return wa;
}

template <int N, int QH, bool ZF, bool STAGED>
hipError_t demod_items_launch(const LaunchArgs& la, const float2* H, float2* xhat, uint8_t* bits, int wa,
                              int64_t grid, size_t lds) {
  hipError_t e = allow_lds(demod_items_kernel<N, QH, kWavesDemod, ZF, STAGED>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((demod_items_kernel<N, QH, kWavesDemod, ZF, STAGED>), dim3((unsigned)grid),
                     dim3(64 * kWavesDemod), lds, la.stream, la.iq, la.S, la.A, la.T, la.CP, la.U, la.B, la.tw, H,
                     xhat, bits, wa);
  return hipGetLastError();
}

template <int N, int QH, bool ZF>
hipError_t demod_qh(const LaunchArgs& la, const float2* H, float2* xhat, uint8_t* bits) {
  using Sh = FftShape<N>;
  const int64_t items = la.S * (la.T - 1);
  if constexpr (Sh::WPT == 1) {
    const int wa = demod_waves_per_item(la.A, items, Sh::F);
    if (Sh::F > 1 || wa < kWavesDemod) {
      // several items per workgroup
      const int ipw = (kWavesDemod / wa) * Sh::F;
      const int64_t grid = (items + ipw - 1) / ipw;
      size_t lds = fft_lds_bytes<N, kWavesDemod>();
      // reduction rows (z, g) and one decision code per subcarrier, with 4
      // bytes of slack for the packing's last 4-byte read
      const size_t red =
          (size_t)transforms_per_group<N, kWavesDemod>() * la.U * (sizeof(float2) + sizeof(float) + 1) + 4;
      if (red > lds) lds = red;
      // staged 16-byte sample loads for transforms of at most 8 lanes when
      // every record piece is 16-byte aligned
      if constexpr (Sh::L <= 8) {
        if (la.CP % 4 == 0 && reinterpret_cast<uintptr_t>(la.iq) % 16 == 0)
          return demod_items_launch<N, QH, ZF, true>(la, H, xhat, bits, wa, grid, lds);
      }
      return demod_items_launch<N, QH, ZF, false>(la, H, xhat, bits, wa, grid, lds);
    }
  }
  const int64_t grid = items;
  constexpr int C = Sh::F == 1 ? RX_DEMOD_ILP : 1;
  size_t lds = fft_lds_bytes<N, kWavesDemod>() * C;
  const size_t red = (size_t)transforms_per_group<N, kWavesDemod>() * la.U * (sizeof(float2) + sizeof(float));
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
  constexpr int L = FftShape<N>::L;
  static_assert(FftShape<N>::P == 16, "tiers assume 16 points per lane");
  const int need = (la.U / 2 + 1 + L - 1) / L;
  if (need <= 2) return demod_qh<N, 2, ZF>(la, H, xhat, bits);
  if (need <= 4) return demod_qh<N, 4, ZF>(la, H, xhat, bits);
  if (need <= 5) return demod_qh<N, 5, ZF>(la, H, xhat, bits);
  if (need <= 8) return demod_qh<N, 8, ZF>(la, H, xhat, bits);
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
  if (la.fft_mode != 0) return launch_mfma_estimate(la, H);
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
  if (la.fft_mode != 0) return launch_mfma_demod(la, H, xhat, bits);
  return zf ? demod_dispatch<true>(la, H, xhat, bits) : demod_dispatch<false>(la, H, xhat, bits);
}

hipError_t launch_fft(const LaunchArgs& la, float2* Y) {
  if (la.fft_mode != 0) return launch_mfma_fft(la, Y);
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


// ------------------------------------------------------------------ batch kernel lookup
namespace {
template <int N, int QH, int W, int S>
void demod_entry(BatchKernel& k) {
  k.func = reinterpret_cast<const void*>(batch_demod_kernel<N, QH, W, S>);
  k.block = 64 * W;
}
template <int N, int W, int J, int S>
void est_entry(BatchKernel& k) {
  k.func = reinterpret_cast<const void*>(batch_estimate_kernel<N, W, J, S>);
  k.block = 64 * W;
}
template <int N, int W, int S>
bool demod_qh_pick(int need, BatchKernel& k) {
  static_assert(FftShape<N>::P == 16, "tiers assume 16 points per lane");
  if (need <= 5) { demod_entry<N, 5, W, S>(k); return true; }
  if (need <= 8) { demod_entry<N, 8, W, S>(k); return true; }
  return false;
}
// Transforms per workgroup of w wavefronts (w a multiple of the wavefronts per transform).
template <int N>
int tpw(int w) { return 64 * w / FftShape<N>::L; }
template <int N, int S>
bool dem_pick(int max_u, int demod_waves, BatchKernel& dem) {
  constexpr int L = FftShape<N>::L;
  const int need = (max_u / 2 + 1 + L - 1) / L;
  bool ok = false;
  switch (demod_waves) {
    case 2: ok = demod_qh_pick<N, 2, S>(need, dem); break;
    case 4: ok = demod_qh_pick<N, 4, S>(need, dem); break;
    case 8: ok = demod_qh_pick<N, 8, S>(need, dem); break;
    default: return false;
  }
  if (!ok) return false;
  // LDS of the demod tile: exchange buffers, or the reduction rows if larger
  dem.lds_fft = (size_t)tpw<N>(demod_waves) * Lds<N>::kSlot * sizeof(float2);
  dem.lds_per_u = (size_t)tpw<N>(demod_waves) * (sizeof(float2) + sizeof(float));
  dem.ants_per_tile = 0;
  return true;
}
template <int N, int S>
bool est_pick(int est_jobs, BatchKernel& est) {
  switch (est_jobs) {
    case 2: est_entry<N, 4, 2, S>(est); break;
    case 4: est_entry<N, 4, 4, S>(est); break;
    case 8: est_entry<N, 4, 8, S>(est); break;
    default: return false;
  }
  est.lds_fft = (size_t)tpw<N>(4) * Lds<N>::kSlot * sizeof(float2);
  est.lds_per_u = 0;
  est.ants_per_tile = tpw<N>(4) * est_jobs;
  return true;
}
template <int N>
bool batch_pick_n(int max_u, int demod_waves, int est_jobs, int dem_sched, int est_sched, BatchKernel& dem,
                  BatchKernel& est) {
  bool ok_d = false, ok_e = false;
  if (dem_sched == 0) ok_d = dem_pick<N, 0>(max_u, demod_waves, dem);
  if (est_sched == 0) ok_e = est_pick<N, 0>(est_jobs, est);
  if constexpr (fft_schedules(N) > 1) {
    if (dem_sched == 1) ok_d = dem_pick<N, 1>(max_u, demod_waves, dem);
    if (est_sched == 1) ok_e = est_pick<N, 1>(est_jobs, est);
  }
  return ok_d && ok_e;
}
}  // namespace

int fft_schedule_count(int N) {
  switch (N) {
    case 64: case 128: case 256: case 512: case 1024: case 2048: return fft_schedules(N);
    default: return 0;
  }
}

namespace {
template <int N>
void radices_of(int sched, int radices[3]) {
  if (sched == 0) {
    radices[0] = Radices<N, 0>::R1; radices[1] = Radices<N, 0>::R2; radices[2] = Radices<N, 0>::R3;
  } else if constexpr (fft_schedules(N) > 1) {
    if (sched == 1) {
      radices[0] = Radices<N, 1>::R1; radices[1] = Radices<N, 1>::R2; radices[2] = Radices<N, 1>::R3;
    }
  }
}
}  // namespace

void fft_schedule_radices(int N, int sched, int radices[3]) {
  radices[0] = radices[1] = radices[2] = 0;
  switch (N) {
    case 64: radices_of<64>(sched, radices); break;
    case 128: radices_of<128>(sched, radices); break;
    case 256: radices_of<256>(sched, radices); break;
    case 512: radices_of<512>(sched, radices); break;
    case 1024: radices_of<1024>(sched, radices); break;
    case 2048: radices_of<2048>(sched, radices); break;
    default: break;
  }
}

bool batch_kernels(int N, int max_u, int demod_waves, int est_jobs, int dem_sched, int est_sched, BatchKernel& dem,
                   BatchKernel& est) {
  switch (N) {
    case 64: return batch_pick_n<64>(max_u, demod_waves, est_jobs, dem_sched, est_sched, dem, est);
    case 128: return batch_pick_n<128>(max_u, demod_waves, est_jobs, dem_sched, est_sched, dem, est);
    case 256: return batch_pick_n<256>(max_u, demod_waves, est_jobs, dem_sched, est_sched, dem, est);
    case 512: return batch_pick_n<512>(max_u, demod_waves, est_jobs, dem_sched, est_sched, dem, est);
    case 1024: return batch_pick_n<1024>(max_u, demod_waves, est_jobs, dem_sched, est_sched, dem, est);
    case 2048: return batch_pick_n<2048>(max_u, demod_waves, est_jobs, dem_sched, est_sched, dem, est);
    default: return false;
  }
}

const void* batch_reset_func() { return reinterpret_cast<const void*>(batch_reset_kernel); }

}  // namespace rx
