// rx_fft.hpp -- wavefront-level FFT building blocks for gfx950.
//
// An N-point FFT (N = 64 .. 2048) is computed by L = N / 16 lanes, each lane
// holding P = 16 complex points in VGPRs.  For N < 1024 one 64-wide wavefront
// runs F = 64 / L transforms side by side; N = 1024 fills one wavefront; N =
// 2048 spans a pair of wavefronts of the workgroup (L = 128), which keeps the
// per-lane state (and so the occupancy) of the N = 1024 transform.  Lane li of
// a transform is thread li of its L-thread group: li = tid % L, transform slot
// tid / L.  The transform is a self-sorting (Stockham) sequence of radix-R
// passes: each lane applies R-point DFTs to R of its points held in registers,
// and consecutive passes exchange data through a padded LDS region private to
// the transform.  Within one wavefront no barrier is needed: its LDS
// operations execute in program order, so a wavefront-scope fence (a pure
// compiler ordering point) separates the reads and writes of each pass.  A
// two-wavefront transform separates them with a workgroup barrier taken once
// the wavefront's own LDS operations are complete; its outstanding global
// loads (the next symbol's samples) stay in flight across it.
//
// Pass with radix R after stride NS (product of the earlier radices):
// butterfly j in [0, N/R) takes x[j + r*N/R], r = 0..R-1, multiplies element r
// by W^(r*(j mod NS)) with W = exp(-2 pi i / (NS*R)), takes the R-point DFT and
// stores output r at (j / NS)*NS*R + (j mod NS) + r*NS.  The last pass keeps
// its outputs in registers: lane li ends with bins li + L*q, q = 0..P-1.
//
// The transform computed is Y[k] = sum_n y[n] exp(-2 pi i k n / N) (forward,
// unscaled) -- the FFT taken after CP removal on every antenna (paper
// Sec. II-B, Sec. II-C).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rx {

// ------------------------------------------------------------ complex helpers
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// a * w
__device__ __forceinline__ float2 cmul(float2 a, float2 w) {
  return make_float2(fmaf(a.x, w.x, -a.y * w.y), fmaf(a.x, w.y, a.y * w.x));
}
// a * (-i)
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }
// a * exp(-i pi/4) = a * (1 - i)/sqrt(2)
__device__ __forceinline__ float2 mul_w8_1(float2 a) {
  const float c = 0.70710678118654752f;
  return make_float2((a.x + a.y) * c, (a.y - a.x) * c);
}
// a * exp(-3 i pi/4) = a * (-1 - i)/sqrt(2)
__device__ __forceinline__ float2 mul_w8_3(float2 a) {
  const float c = 0.70710678118654752f;
  return make_float2((a.y - a.x) * c, -(a.x + a.y) * c);
}

// ------------------------------------------------------------ R-point DFTs in registers
// All take v[o .. o+R) in natural order and leave the DFT there in natural
// order.  `o` is a compile-time constant after unrolling.
template <int P>
__device__ __forceinline__ void dft2(float2 (&v)[P], int o) {
  float2 a = v[o], b = v[o + 1];
  v[o] = cadd(a, b);
  v[o + 1] = csub(a, b);
}

// 4-point DFT of (a0, a1, a2, a3) in place.
__device__ __forceinline__ void dft4_raw(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  float2 t2 = cadd(a1, a3), t3 = mul_mi(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <int P>
__device__ __forceinline__ void dft4(float2 (&v)[P], int o) {
  dft4_raw(v[o], v[o + 1], v[o + 2], v[o + 3]);
}

// 8 = 2 x 4: even/odd 4-point DFTs, then one radix-2 layer with W8^k.
template <int P>
__device__ __forceinline__ void dft8(float2 (&v)[P], int o) {
  float2 e0 = v[o], e1 = v[o + 2], e2 = v[o + 4], e3 = v[o + 6];
  float2 d0 = v[o + 1], d1 = v[o + 3], d2 = v[o + 5], d3 = v[o + 7];
  dft4_raw(e0, e1, e2, e3);
  dft4_raw(d0, d1, d2, d3);
  d1 = mul_w8_1(d1);
  d2 = mul_mi(d2);
  d3 = mul_w8_3(d3);
  v[o + 0] = cadd(e0, d0);
  v[o + 4] = csub(e0, d0);
  v[o + 1] = cadd(e1, d1);
  v[o + 5] = csub(e1, d1);
  v[o + 2] = cadd(e2, d2);
  v[o + 6] = csub(e2, d2);
  v[o + 3] = cadd(e3, d3);
  v[o + 7] = csub(e3, d3);
}

// 16 = 4 x 4: n = n1 + 4 n2, k = k2 + 4 k1;
// X[k2 + 4 k1] = sum_n1 W4^(n1 k1) W16^(n1 k2) sum_n2 x[n1 + 4 n2] W4^(n2 k2).
template <int P>
__device__ __forceinline__ void dft16(float2 (&v)[P], int o) {
  const float2 w1 = make_float2(0.92387953251128674f, -0.38268343236508977f);  // W16^1
  const float2 w3 = make_float2(0.38268343236508977f, -0.92387953251128674f);  // W16^3
  // inner 4-point DFTs over n2 for each n1; results a[n1][k2] stay at v[o + n1 + 4 k2]
#pragma unroll
  for (int n1 = 0; n1 < 4; n1++) dft4_raw(v[o + n1], v[o + n1 + 4], v[o + n1 + 8], v[o + n1 + 12]);
  // twiddles W16^(n1 k2)
  v[o + 1 + 4] = cmul(v[o + 1 + 4], w1);          // n1=1,k2=1
  v[o + 1 + 8] = mul_w8_1(v[o + 1 + 8]);          // n1=1,k2=2 : W16^2
  v[o + 1 + 12] = cmul(v[o + 1 + 12], w3);        // n1=1,k2=3
  v[o + 2 + 4] = mul_w8_1(v[o + 2 + 4]);          // n1=2,k2=1 : W16^2
  v[o + 2 + 8] = mul_mi(v[o + 2 + 8]);            // n1=2,k2=2 : W16^4
  v[o + 2 + 12] = mul_w8_3(v[o + 2 + 12]);        // n1=2,k2=3 : W16^6
  v[o + 3 + 4] = cmul(v[o + 3 + 4], w3);          // n1=3,k2=1
  v[o + 3 + 8] = mul_w8_3(v[o + 3 + 8]);          // n1=3,k2=2 : W16^6
  {                                               // n1=3,k2=3 : W16^9 = -W16^1
    float2 t = cmul(v[o + 3 + 12], w1);
    v[o + 3 + 12] = make_float2(-t.x, -t.y);
  }
  // outer 4-point DFTs over n1 for each k2; output k = k2 + 4 k1
  float2 r[16];
#pragma unroll
  for (int k2 = 0; k2 < 4; k2++) {
    float2 a0 = v[o + 4 * k2], a1 = v[o + 1 + 4 * k2], a2 = v[o + 2 + 4 * k2], a3 = v[o + 3 + 4 * k2];
    dft4_raw(a0, a1, a2, a3);
    r[k2] = a0;
    r[k2 + 4] = a1;
    r[k2 + 8] = a2;
    r[k2 + 12] = a3;
  }
#pragma unroll
  for (int k = 0; k < 16; k++) v[o + k] = r[k];
}

template <int R, int P>
__device__ __forceinline__ void dft(float2 (&v)[P], int o) {
  if constexpr (R == 2) dft2(v, o);
  else if constexpr (R == 4) dft4(v, o);
  else if constexpr (R == 8) dft8(v, o);
  else if constexpr (R == 16) dft16(v, o);
  else static_assert(R == 2 || R == 4 || R == 8 || R == 16, "unsupported radix");
}

// ------------------------------------------------------------ LDS layout
// One complex of padding every 16 keeps the 16-point stride of the first
// pass's writes off a single bank.
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }
template <int N>
struct Lds {
  static constexpr int kSlot = N + N / 16;  // float2 per transform
};

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroup barrier for LDS data only: waits for this wavefront's LDS
// operations (lgkmcnt = 0, the gfx9 s_waitcnt encoding with vmcnt and expcnt
// left at their maxima) and not for its global loads.  Every wavefront of the
// workgroup must reach it the same number of times.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------ pass schedule per N
template <int N>
struct FftShape {
  static constexpr int P = 16;                      // points per lane
  static constexpr int L = N / P;                   // lanes per transform
  static constexpr int F = L < 64 ? 64 / L : 1;     // transforms per wavefront
  static constexpr int WPT = L > 64 ? L / 64 : 1;   // wavefronts per transform
  static_assert(N >= 64 && N <= 2048 && (N & (N - 1)) == 0, "N must be a power of two in [64, 2048]");
};

// Separation of two passes' LDS accesses (see the top of this file).  With
// WPT > 1 it is a workgroup barrier: code that calls it must be reached by
// every wavefront of the workgroup equally often.
template <int N>
__device__ __forceinline__ void exchange_fence() {
  if constexpr (FftShape<N>::WPT == 1) wave_fence();
  else lds_barrier();
}

// Radix schedules per N: the first pass is always radix 16 (16 points of one
// transform per lane, loaded straight from memory).  Schedule 0 puts the
// small radix in the middle (its pass has few distinct twiddles per lane and
// the last pass is a full radix 16); schedule 1, for the three-pass lengths,
// puts it last (16 twiddles of the middle pass per lane instead, a smaller
// last-pass table).  Lengths with two passes have schedule 0 only.
template <int N>
struct Radices0;
template <> struct Radices0<64>   { static constexpr int R1 = 16, R2 = 4, R3 = 0; };
template <> struct Radices0<128>  { static constexpr int R1 = 16, R2 = 8, R3 = 0; };
template <> struct Radices0<256>  { static constexpr int R1 = 16, R2 = 16, R3 = 0; };
template <> struct Radices0<512>  { static constexpr int R1 = 16, R2 = 2, R3 = 16; };
template <> struct Radices0<1024> { static constexpr int R1 = 16, R2 = 4, R3 = 16; };
template <> struct Radices0<2048> { static constexpr int R1 = 16, R2 = 8, R3 = 16; };

template <int N, int S = 0>
struct Radices : Radices0<N> {
  static_assert(S == 0 || Radices0<N>::R3 > 0, "schedule 1 exists for three-pass lengths only");
  static constexpr int R2 = S == 0 ? Radices0<N>::R2 : Radices0<N>::R3;
  static constexpr int R3 = S == 0 ? Radices0<N>::R3 : Radices0<N>::R2;
};

// Number of radix schedules of length N.
__host__ __device__ constexpr int fft_schedules(int N) { return N >= 512 ? 2 : 1; }

// Twiddles of one pass (radix R after stride NS) for this lane's butterflies
// j_m = li + L*m: element r of butterfly m is multiplied by
// exp(-2 pi i r (j_m mod NS) / (NS R)).  When L is a multiple of NS every
// butterfly of the lane shares one set.  Loaded once per kernel into VGPRs.
template <int N, int R, int NS>
struct PassTwiddles {
  static constexpr int P = FftShape<N>::P, L = FftShape<N>::L, NB = R > 0 ? P / R : 1;
  static constexpr bool kShared = (NS == 1) || (L % NS == 0);
  static constexpr int kSets = kShared ? 1 : NB;
  static constexpr int kCount = (NS == 1 || R == 0) ? 1 : kSets * (R - 1);
  float2 w[kCount];
  __device__ __forceinline__ void load(const float2* __restrict__ tw, int li) {
    if constexpr (NS > 1 && R > 0) {
#pragma unroll
      for (int s = 0; s < kSets; s++) {
        const int step = ((li + L * s) & (NS - 1)) * (N / (NS * R));
#pragma unroll
        for (int r = 1; r < R; r++) w[s * (R - 1) + r - 1] = tw[step * r];
      }
    }
  }
  __device__ __forceinline__ float2 get(int m, int r) const { return w[(kShared ? 0 : m) * (R - 1) + r - 1]; }
};

// Twiddles of the last pass kept in LDS instead of VGPRs: entry
// [(s*(R-1) + r-1)*L + li] = exp(-2 pi i r ((li + L s) mod NS) / (NS R)).
// Lanes read consecutive entries (no bank conflicts); every transform of the
// wavefront reads the same values.
template <int N, int R, int NS>
struct LdsTwiddles {
  static constexpr int P = FftShape<N>::P, L = FftShape<N>::L, NB = R > 0 ? P / R : 1;
  static constexpr bool kShared = (NS == 1) || (L % NS == 0);
  static constexpr int kSets = kShared ? 1 : NB;
  static constexpr int kCount = (NS == 1 || R == 0) ? 1 : kSets * (R - 1) * L;  // float2 entries
  const float2* tab;
  int li;
  // Cooperative fill by the whole workgroup (caller synchronises afterwards).
  static __device__ __forceinline__ void fill(float2* tab, const float2* __restrict__ tw, int tid, int nthreads) {
    if constexpr (NS > 1 && R > 0) {
      for (int e = tid; e < kCount; e += nthreads) {
        const int lane = e % L, sr = e / L, s = sr / (R - 1), r = sr % (R - 1) + 1;
        const int step = ((lane + L * s) & (NS - 1)) * (N / (NS * R));
        tab[e] = tw[step * r];
      }
    }
  }
  __device__ __forceinline__ float2 get(int m, int r) const { return tab[((kShared ? 0 : m) * (R - 1) + r - 1) * L + li]; }
};

// Twiddles of the passes after the first.  With LDS_LAST the last pass of a
// three-pass schedule reads its twiddles from a per-workgroup LDS table
// (fewer VGPRs); otherwise they are held in VGPRs (no LDS reads).
template <int N, int S = 0, bool LDS_LAST = true>
struct FftTwiddles {
  static constexpr int kSchedule = S;
  using Rd = Radices<N, S>;
  static constexpr bool kLdsLast = LDS_LAST && Rd::R3 > 0;
  using P3Regs = PassTwiddles<N, Rd::R3, Rd::R1 * Rd::R2>;
  using P3Lds = LdsTwiddles<N, Rd::R3, Rd::R1 * Rd::R2>;
  static constexpr int kLdsFloat2 = kLdsLast ? P3Lds::kCount : 0;  // LDS table size
  PassTwiddles<N, Rd::R2, Rd::R1> p2;
  typename std::conditional<kLdsLast, P3Lds, P3Regs>::type p3;
  // lds_tab: the filled table (only read when kLdsLast)
  __device__ __forceinline__ void load(const float2* __restrict__ tw, int li, const float2* lds_tab = nullptr) {
    p2.load(tw, li);
    if constexpr (kLdsLast) {
      p3.tab = lds_tab;
      p3.li = li;
    } else if constexpr (Rd::R3 > 0) {
      p3.load(tw, li);
    }
  }
};

// One Stockham pass over C independent transforms held by the lane (C > 1
// gives the scheduler independent work to overlap with LDS latency).  With
// FIRST, v[c] already holds this lane's inputs v[c][m*R + r] = x[j_m + r*N/R],
// j_m = li + L*m; otherwise they are gathered from buf[c].  Output goes to
// buf[c] (padded indexing) unless LAST, where it stays in v (fft_in_regs).
template <int N, int R, int NS, bool FIRST, bool LAST, int C, typename TW>
__device__ __forceinline__ void stockham_pass(float2 (&v)[C][FftShape<N>::P], float2* const (&buf)[C], int li,
                                              const TW& tw) {
  constexpr int P = FftShape<N>::P;
  constexpr int L = FftShape<N>::L;
  constexpr int NB = P / R;
  static_assert(P % R == 0, "radix must divide the points per lane");
  if constexpr (!FIRST) {
    const int pli = pad(li);
#pragma unroll
    for (int c = 0; c < C; c++)
#pragma unroll
      for (int m = 0; m < NB; m++)
#pragma unroll
        for (int r = 0; r < R; r++) {
          const int k = L * m + r * (N / R);
          v[c][m * R + r] = buf[c][(k % 16 == 0) ? pli + k + k / 16 : pad(li + k)];
        }
    // every lane's reads happen before any lane's writes; the last pass writes
    // nothing, and a two-wavefront transform skips that (barrier) fence: the
    // caller fences before the buffer is written again
    if constexpr (!LAST || FftShape<N>::WPT == 1) exchange_fence<N>();
  }
#pragma unroll
  for (int c = 0; c < C; c++)
#pragma unroll
    for (int m = 0; m < NB; m++) {
      const int j = li + L * m;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; r++) v[c][m * R + r] = cmul(v[c][m * R + r], tw.get(m, r));
      }
      dft<R>(v[c], m * R);
      if constexpr (!LAST) {
        const int o = (j / NS) * NS * R + (j & (NS - 1));
        const int po = pad(o);
        const bool o16 = (NS == 1) && (R == 16);  // o = 16 j
#pragma unroll
        for (int r = 0; r < R; r++) {
          const int k = r * NS;
          buf[c][(k % 16 == 0) ? po + k + k / 16 : (o16 ? po + k : pad(o + k))] = v[c][m * R + r];
        }
      }
    }
  if constexpr (!LAST) exchange_fence<N>();
}

// Whole transform of C symbols.  Inputs in v (first-pass order).  On return
// the spectra are in v: the last pass has stride NS = N / R and one output
// per butterfly j = li + L*m and r, at bin j + NS*r = li + L*q with
// q = m + NB*r, so the lane holds bins k = li + L*q, q = 0..P-1, in
// v[c][Spectrum<N>::reg(q)].  buf[c] is left holding the previous pass's
// data; the caller fences before writing it again.
template <int N, int S = 0>
struct Spectrum {
  using Rd = Radices<N, S>;
  static constexpr int R = Rd::R3 > 0 ? Rd::R3 : Rd::R2;  // last radix
  static constexpr int NB = FftShape<N>::P / R;
  static constexpr int reg(int q) { return (q % NB) * R + q / NB; }
};

// First pass only (inputs in registers, output to LDS); radix 16 in every
// schedule.
template <int N, int C>
__device__ __forceinline__ void fft_first_pass(float2 (&v)[C][FftShape<N>::P], float2* const (&buf)[C], int li) {
  using Rd = Radices<N>;
  const PassTwiddles<N, Rd::R1, 1> none{};
  stockham_pass<N, Rd::R1, 1, true, false, C>(v, buf, li, none);
}

// The passes after the first; the spectrum ends in v.  The schedule comes
// with the twiddles' type.
template <int N, int C, int S, bool LL>
__device__ __forceinline__ void fft_rest(float2 (&v)[C][FftShape<N>::P], float2* const (&buf)[C], int li,
                                         const FftTwiddles<N, S, LL>& tw) {
  using Rd = Radices<N, S>;
  if constexpr (Rd::R3 > 0) {
    stockham_pass<N, Rd::R2, Rd::R1, false, false, C>(v, buf, li, tw.p2);
    stockham_pass<N, Rd::R3, Rd::R1 * Rd::R2, false, true, C>(v, buf, li, tw.p3);
  } else {
    stockham_pass<N, Rd::R2, Rd::R1, false, true, C>(v, buf, li, tw.p2);
  }
}

template <int N, int C, int S, bool LL>
__device__ __forceinline__ void fft_in_regs(float2 (&v)[C][FftShape<N>::P], float2* const (&buf)[C], int li,
                                            const FftTwiddles<N, S, LL>& tw) {
  fft_first_pass<N, C>(v, buf, li);
  fft_rest<N, C>(v, buf, li, tw);
}

// Single-transform form.
template <int N, int S, bool LL>
__device__ __forceinline__ void fft_in_regs(float2 (&v)[FftShape<N>::P], float2* buf, int li,
                                            const FftTwiddles<N, S, LL>& tw) {
  float2 vv[1][FftShape<N>::P];
#pragma unroll
  for (int i = 0; i < FftShape<N>::P; i++) vv[0][i] = v[i];
  float2* const b[1] = {buf};
  fft_in_regs<N, 1>(vv, b, li, tw);
#pragma unroll
  for (int i = 0; i < FftShape<N>::P; i++) v[i] = vv[0][i];
}

// int16 I/Q packed in one dword (I in the low half) -> complex float, exact.
__device__ __forceinline__ float2 iq_to_float(uint32_t w) {
  return make_float2((float)(int16_t)(w & 0xffffu), (float)((int32_t)w >> 16));
}

// Load this lane's first-pass inputs for one symbol: x[n] = sample CP + n of
// the record starting at `rec` (one dword per complex sample).  The loads
// are unconditional (the caller passes a valid record); lanes whose
// transform slot is unused get zeros afterwards, without branching.
template <int N>
__device__ __forceinline__ void load_symbol(uint32_t (&raw)[FftShape<N>::P], const uint32_t* __restrict__ rec,
                                            int li, bool valid) {
  constexpr int P = FftShape<N>::P;
  constexpr int L = FftShape<N>::L;
  constexpr int R = 16;  // first pass radix for every N
  constexpr int NB = P / R;
#pragma unroll
  for (int m = 0; m < NB; m++)
#pragma unroll
    for (int r = 0; r < R; r++) raw[m * R + r] = __builtin_nontemporal_load(rec + li + L * m + r * (N / R));
  if constexpr (FftShape<N>::F > 1) {
#pragma unroll
    for (int i = 0; i < P; i++) raw[i] = valid ? raw[i] : 0u;
  }
}

template <int N>
__device__ __forceinline__ void unpack_symbol(float2 (&v)[FftShape<N>::P], const uint32_t (&raw)[FftShape<N>::P]) {
#pragma unroll
  for (int i = 0; i < FftShape<N>::P; i++) v[i] = iq_to_float(raw[i]);
}

}  // namespace rx
