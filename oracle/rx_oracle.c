/*
 * rx_oracle.c -- plain, slow FP64 reference of the uplink receive path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the GPU library.
 *
 * What is computed (paper, Section II-B and II-C):
 *   - every OFDM symbol of every antenna has its cyclic prefix dropped and is
 *     taken through an N-point FFT (Section II-B, last paragraph; Section II-C);
 *   - the first symbol of a slot is the channel-estimation symbol: block
 *     least squares divides each received subcarrier by the pilot
 *     (Section II-B; Section II-C, LS paragraph);
 *   - every later symbol is combined over the antennas by maximal ratio
 *     combining, one sum per subcarrier (Section II-C, MRC paragraph);
 *   - subcarriers are taken in fftshift (centred) order (Section II-C, last
 *     sentence).
 * The paper is silent on the FFT sign/scale, the used-subcarrier set, LS for
 * non-unit pilots, MRC normalisation, the QAM map, decision ties and bit
 * packing; the readings taken here are:
 *   FFT      Y[k] = sum_n y[n] exp(-2 pi i k n / N), no scaling;
 *   bins     d = 0..U-1 carries signed frequency f_d = d-U/2 (d < U/2) or
 *            d-U/2+1, at FFT bin k_d = f_d mod N (DC and Nyquist unused);
 *   LS       H[a,d] = Y_0[a,k_d] conj(Xp[d]) / |Xp[d]|^2;
 *   MRC      z = sum_a conj(H[a,d]) Y_t[a,k_d],  g = sum_a |H[a,d]|^2,
 *            xhat = z / g, or 0 when g == 0;
 *   ZF (one user)  w_a = conj(H[a,d]) / g,  xhat = sum_a w_a Y_t[a,k_d];
 *   demap    per-axis Gray decisions with strict comparisons (ties and -0.0
 *            give bit 0); bits packed MSB-first in [slot][data sym][d][bit].
 *   comb     (pilot_spacing s > 1; not in the paper, which uses a block
 *            pilot: the comb-type arrangement with linear interpolation that
 *            the learned denoiser starts from) LS only on d = 0, s, 2s, ...;
 *            every other d takes the straight line in signed frequency f_d
 *            between the pilot at or below it and the next pilot (so the
 *            line spans the DC gap), and beyond the last pilot that pilot's
 *            value is held.
 *
 * Floating point is FP64 throughout; compile without fast-math.
 */
#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_PI 3.14159265358979323846264338327950288

typedef struct {
  int32_t n_ant;        /* A */
  int32_t fft_len;      /* N, a power of two */
  int32_t cp_len;       /* CP */
  int32_t n_used;       /* U, even, 2 <= U <= N-2 */
  int32_t n_sym;        /* T, symbol 0 is the pilot */
  int32_t bits_per_sym; /* 2, 4 or 6 */
  int32_t combiner;     /* 0 = MRC, 1 = ZF */
  const double* pilot;  /* U complex values (re, im interleaved), d order */
  int32_t pilot_spacing; /* 0 or 1: block pilot; s > 1: comb on d % s == 0 */
} oracle_params;

static int spacing_of(const oracle_params* p) { return p->pilot_spacing > 1 ? p->pilot_spacing : 1; }

/* Signed frequency of used subcarrier d (DC excluded). */
static int signed_freq(int d, int U) { return d < U / 2 ? d - U / 2 : d - U / 2 + 1; }

/* Linear interpolation of rows of U complex values (interleaved doubles)
 * whose entries d % s == 0 hold pilot estimates; the others are overwritten. */
void oracle_comb_interp(int U, int s, double* H, int64_t rows) {
  if (s <= 1) return;
  const int last = ((U - 1) / s) * s;
  for (int64_t r = 0; r < rows; r++) {
    double* h = H + (size_t)r * U * 2;
    for (int d = 0; d < U; d++) {
      if (d % s == 0) continue;
      const int d0 = (d / s) * s;
      if (d0 == last) {
        h[2 * d] = h[2 * last];
        h[2 * d + 1] = h[2 * last + 1];
        continue;
      }
      const int d1 = d0 + s;
      const double t = (double)(signed_freq(d, U) - signed_freq(d0, U)) /
                       (double)(signed_freq(d1, U) - signed_freq(d0, U));
      h[2 * d] = h[2 * d0] + t * (h[2 * d1] - h[2 * d0]);
      h[2 * d + 1] = h[2 * d0 + 1] + t * (h[2 * d1 + 1] - h[2 * d0 + 1]);
    }
  }
}

/* ---------------------------------------------------------------------------
 * FFT.  Iterative radix-2 decimation in time: bit-reversal permutation, then
 * log2(N) passes of butterflies of growing length.  Twiddles are evaluated
 * with cos/sin in FP64 where they are used.  Computes exactly the DFT
 * Y[k] = sum_n y[n] e^{-2 pi i k n / N} up to rounding.
 * ------------------------------------------------------------------------- */
static int is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

int oracle_fft(double complex* x, int n) {
  if (!is_pow2(n)) return -1;
  /* bit-reversal permutation */
  for (int i = 1, j = 0; i < n; i++) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      double complex t = x[i];
      x[i] = x[j];
      x[j] = t;
    }
  }
  for (int len = 2; len <= n; len <<= 1) {
    int half = len / 2;
    for (int j = 0; j < half; j++) {
      double ang = -2.0 * ORACLE_PI * (double)j / (double)len;
      double complex w = cos(ang) + I * sin(ang);
      for (int i = 0; i < n; i += len) {
        double complex u = x[i + j];
        double complex v = x[i + j + half] * w;
        x[i + j] = u + v;
        x[i + j + half] = u - v;
      }
    }
  }
  return 0;
}

/* Used-subcarrier index -> FFT bin (fftshift order, DC excluded). */
void oracle_subcarrier_map(int n, int u, int32_t* k_of_d) {
  for (int d = 0; d < u; d++) {
    int f = (d < u / 2) ? d - u / 2 : d - u / 2 + 1;
    k_of_d[d] = (int32_t)(((f % n) + n) % n);
  }
}

/* ---------------------------------------------------------------------------
 * Hard decisions.  Axis coordinate c (real or imaginary part of xhat):
 *   first bit of the axis  = [c < 0]
 *   16-QAM second bit      = [|c| sqrt(10) > 2]
 *   64-QAM second bit      = [|c| sqrt(42) > 4], third = [| |c| sqrt(42) - 4 | > 2]
 * Even bit positions come from the real axis, odd ones from the imaginary.
 * ------------------------------------------------------------------------- */
static void decide_axis(double c, int bits_per_sym, uint8_t* out /* bits_per_sym/2 */) {
  out[0] = (uint8_t)(c < 0.0);
  if (bits_per_sym == 4) {
    out[1] = (uint8_t)(fabs(c) * sqrt(10.0) > 2.0);
  } else if (bits_per_sym == 6) {
    double u = fabs(c) * sqrt(42.0);
    out[1] = (uint8_t)(u > 4.0);
    out[2] = (uint8_t)(fabs(u - 4.0) > 2.0);
  }
}

/* xhat: n complex (re, im); bitvals: n * bits_per_sym values in {0,1}. */
int oracle_demap(const double* xhat, int64_t n, int bits_per_sym, uint8_t* bitvals) {
  if (bits_per_sym != 2 && bits_per_sym != 4 && bits_per_sym != 6) return -1;
  int h = bits_per_sym / 2;
  for (int64_t i = 0; i < n; i++) {
    uint8_t re[3], im[3];
    decide_axis(xhat[2 * i], bits_per_sym, re);
    decide_axis(xhat[2 * i + 1], bits_per_sym, im);
    for (int j = 0; j < h; j++) {
      bitvals[i * bits_per_sym + 2 * j] = re[j];
      bitvals[i * bits_per_sym + 2 * j + 1] = im[j];
    }
  }
  return 0;
}

/* Pack a row of bit values MSB-first; nbits must be a multiple of 8. */
void oracle_pack_bits(const uint8_t* bitvals, int64_t nbits, uint8_t* bytes) {
  for (int64_t i = 0; i < nbits / 8; i++) {
    uint8_t v = 0;
    for (int j = 0; j < 8; j++) v = (uint8_t)((v << 1) | (bitvals[8 * i + j] & 1));
    bytes[i] = v;
  }
}

/* ---------------------------------------------------------------------------
 * One slot.  `sample(t, a, n)` yields payload sample n (after the CP) of
 * symbol t on antenna a.  Outputs (any may be NULL):
 *   H    [A][U] complex, g [U], xhat [T-1][U] complex, bits [T-1][U*b/8].
 * ------------------------------------------------------------------------- */
typedef double complex (*sample_fn)(const void* src, const oracle_params* p, int t, int a, int n);

static double complex sample_i16(const void* src, const oracle_params* p, int t, int a, int n) {
  const int16_t* iq = (const int16_t*)src;
  int64_t len = p->fft_len + p->cp_len;
  int64_t off = (((int64_t)t * p->n_ant + a) * len + p->cp_len + n) * 2;
  return (double)iq[off] + I * (double)iq[off + 1];
}

static double complex sample_f64(const void* src, const oracle_params* p, int t, int a, int n) {
  const double* y = (const double*)src;
  int64_t len = p->fft_len + p->cp_len;
  int64_t off = (((int64_t)t * p->n_ant + a) * len + p->cp_len + n) * 2;
  return y[off] + I * y[off + 1];
}

static int slot_process(const oracle_params* p, const void* src, sample_fn sample, const double* H_in,
                        double* H, double* g, double* xhat, uint8_t* bits) {
  const int A = p->n_ant, N = p->fft_len, U = p->n_used, T = p->n_sym, B = p->bits_per_sym;
  int32_t* kmap = malloc(sizeof(int32_t) * U);
  double complex* Y = malloc(sizeof(double complex) * (size_t)T * A * N);
  double complex* Hs = malloc(sizeof(double complex) * (size_t)A * U);
  double* gs = malloc(sizeof(double) * U);
  double* xs = malloc(sizeof(double) * 2 * (size_t)(T - 1) * U);
  uint8_t* bv = malloc((size_t)U * B);
  if (!kmap || !Y || !Hs || !gs || !xs || !bv) {
    free(kmap); free(Y); free(Hs); free(gs); free(xs); free(bv);
    return -4;
  }
  oracle_subcarrier_map(N, U, kmap);

  /* CP removal + FFT of every symbol of every antenna */
  for (int t = 0; t < T; t++)
    for (int a = 0; a < A; a++) {
      double complex* y = Y + ((size_t)t * A + a) * N;
      for (int n = 0; n < N; n++) y[n] = sample(src, p, t, a, n);
      oracle_fft(y, N);
    }

  if (H_in) {
    /* a channel estimate supplied by the caller replaces LS */
    for (size_t i = 0; i < (size_t)A * U; i++) Hs[i] = H_in[2 * i] + I * H_in[2 * i + 1];
  } else {
    /* LS from symbol 0 on the pilot subcarriers (all of them for a block
     * pilot), then comb interpolation */
    const int sp = spacing_of(p);
    for (int a = 0; a < A; a++)
      for (int d = 0; d < U; d += sp) {
        double complex xp = p->pilot[2 * d] + I * p->pilot[2 * d + 1];
        double mag2 = creal(xp) * creal(xp) + cimag(xp) * cimag(xp);
        Hs[(size_t)a * U + d] = Y[(size_t)a * N + kmap[d]] * conj(xp) / mag2;
      }
    if (sp > 1) oracle_comb_interp(U, sp, (double*)Hs, A);
  }

  /* combining normaliser g = sum_a |H|^2 */
  for (int d = 0; d < U; d++) {
    double s = 0.0;
    for (int a = 0; a < A; a++) {
      double complex h = Hs[(size_t)a * U + d];
      s += creal(h) * creal(h) + cimag(h) * cimag(h);
    }
    gs[d] = s;
  }

  /* combining of the data symbols */
  for (int t = 1; t < T; t++)
    for (int d = 0; d < U; d++) {
      double complex x = 0.0;
      if (gs[d] > 0.0) {
        if (p->combiner == 1) {
          for (int a = 0; a < A; a++) {
            double complex w = conj(Hs[(size_t)a * U + d]) / gs[d];
            x += w * Y[((size_t)t * A + a) * N + kmap[d]];
          }
        } else {
          double complex z = 0.0;
          for (int a = 0; a < A; a++)
            z += conj(Hs[(size_t)a * U + d]) * Y[((size_t)t * A + a) * N + kmap[d]];
          x = z / gs[d];
        }
      }
      xs[2 * ((size_t)(t - 1) * U + d)] = creal(x);
      xs[2 * ((size_t)(t - 1) * U + d) + 1] = cimag(x);
    }

  if (H)
    for (size_t i = 0; i < (size_t)A * U; i++) {
      H[2 * i] = creal(Hs[i]);
      H[2 * i + 1] = cimag(Hs[i]);
    }
  if (g) memcpy(g, gs, sizeof(double) * U);
  if (xhat) memcpy(xhat, xs, sizeof(double) * 2 * (size_t)(T - 1) * U);
  if (bits) {
    int64_t row = (int64_t)U * B / 8;
    for (int t = 1; t < T; t++) {
      oracle_demap(xs + 2 * (size_t)(t - 1) * U, U, B, bv);
      oracle_pack_bits(bv, (int64_t)U * B, bits + (size_t)(t - 1) * row);
    }
  }
  free(kmap); free(Y); free(Hs); free(gs); free(xs); free(bv);
  return 0;
}

static int params_ok(const oracle_params* p) {
  if (!p || !p->pilot) return 0;
  if (p->n_ant < 1 || !is_pow2(p->fft_len) || p->cp_len < 0 || p->cp_len >= p->fft_len) return 0;
  if (p->n_used < 2 || p->n_used > p->fft_len - 2 || (p->n_used & 1)) return 0;
  if (p->n_sym < 2) return 0;
  if (p->bits_per_sym != 2 && p->bits_per_sym != 4 && p->bits_per_sym != 6) return 0;
  if (((int64_t)p->n_used * p->bits_per_sym) % 8) return 0;
  if (p->combiner != 0 && p->combiner != 1) return 0;
  if (p->pilot_spacing < 0 || p->pilot_spacing > p->n_used) return 0;
  for (int d = 0; d < p->n_used; d += spacing_of(p))
    if (p->pilot[2 * d] == 0.0 && p->pilot[2 * d + 1] == 0.0) return 0;
  return 1;
}

/* ---------------------------------------------------------------------------
 * Whole run of S slots, optionally split over n_threads threads (slots are
 * independent).  Layouts:
 *   iq   int16 [S][T][A][CP+N][2]          (oracle_process_frame)
 *   y    double [S][T][A][CP+N][2]          (oracle_process_frame_f64)
 *   H    double [S][A][U][2], g double [S][U],
 *   xhat double [S][T-1][U][2], bits uint8 [S][T-1][U*b/8].
 * Returns 0, -1 on bad parameters, -4 on allocation failure.
 * ------------------------------------------------------------------------- */
typedef struct {
  const oracle_params* p;
  const void* src;
  size_t src_slot_bytes;
  sample_fn sample;
  const double* H_in;
  double *H, *g, *xhat;
  uint8_t* bits;
  int64_t s0, s1;
  int status;
} slot_range;

static void* run_range(void* arg) {
  slot_range* r = (slot_range*)arg;
  const oracle_params* p = r->p;
  size_t A = p->n_ant, U = p->n_used, Td = p->n_sym - 1;
  size_t row = U * p->bits_per_sym / 8;
  for (int64_t s = r->s0; s < r->s1 && r->status == 0; s++) {
    r->status = slot_process(p, (const char*)r->src + (size_t)s * r->src_slot_bytes, r->sample,
                             r->H_in ? r->H_in + (size_t)s * A * U * 2 : NULL,
                             r->H ? r->H + (size_t)s * A * U * 2 : NULL,
                             r->g ? r->g + (size_t)s * U : NULL,
                             r->xhat ? r->xhat + (size_t)s * Td * U * 2 : NULL,
                             r->bits ? r->bits + (size_t)s * Td * row : NULL);
  }
  return NULL;
}

static int run_all(const oracle_params* p, const void* src, size_t elem_bytes, sample_fn sample,
                   int64_t S, const double* H_in, double* H, double* g, double* xhat, uint8_t* bits, int n_threads) {
  if (!params_ok(p) || S < 0 || (S > 0 && !src)) return -1;
  if (n_threads < 1) n_threads = 1;
  if (n_threads > S) n_threads = S > 0 ? (int)S : 1;
  size_t slot_bytes = (size_t)p->n_sym * p->n_ant * (p->fft_len + p->cp_len) * 2 * elem_bytes;
  slot_range* rs = calloc((size_t)n_threads, sizeof(slot_range));
  pthread_t* th = calloc((size_t)n_threads, sizeof(pthread_t));
  if (!rs || !th) { free(rs); free(th); return -4; }
  for (int i = 0; i < n_threads; i++) {
    rs[i] = (slot_range){p, src, slot_bytes, sample, H_in, H, g, xhat, bits,
                         S * i / n_threads, S * (i + 1) / n_threads, 0};
  }
  for (int i = 1; i < n_threads; i++) pthread_create(&th[i], NULL, run_range, &rs[i]);
  run_range(&rs[0]);
  int status = rs[0].status;
  for (int i = 1; i < n_threads; i++) {
    pthread_join(th[i], NULL);
    if (rs[i].status) status = rs[i].status;
  }
  free(rs); free(th);
  return status;
}

int oracle_process_frame(const oracle_params* p, const int16_t* iq, int64_t S, double* H, double* g,
                         double* xhat, uint8_t* bits, int n_threads) {
  return run_all(p, iq, sizeof(int16_t), sample_i16, S, NULL, H, g, xhat, bits, n_threads);
}

/* Combining and demapping with a caller-supplied channel estimate H_in
 * (double [S][A][U][2]) in place of LS; H (if not null) receives a copy. */
int oracle_demod_given_h(const oracle_params* p, const int16_t* iq, int64_t S, const double* H_in, double* g,
                         double* xhat, uint8_t* bits, int n_threads) {
  if (!H_in) return -1;
  return run_all(p, iq, sizeof(int16_t), sample_i16, S, H_in, NULL, g, xhat, bits, n_threads);
}

int oracle_process_frame_f64(const oracle_params* p, const double* y, int64_t S, double* H, double* g,
                             double* xhat, uint8_t* bits, int n_threads) {
  return run_all(p, y, sizeof(double), sample_f64, S, NULL, H, g, xhat, bits, n_threads);
}

/* Y of every symbol: CP removal + FFT only.  out: double [S][T][A][N][2]. */
int oracle_fft_symbols(const oracle_params* p, const int16_t* iq, int64_t S, double* out) {
  if (!params_ok(p) || S < 0) return -1;
  const int A = p->n_ant, N = p->fft_len, T = p->n_sym;
  double complex* y = malloc(sizeof(double complex) * N);
  if (!y) return -4;
  size_t slot_elems = (size_t)T * A * (N + p->cp_len) * 2;
  for (int64_t s = 0; s < S; s++)
    for (int t = 0; t < T; t++)
      for (int a = 0; a < A; a++) {
        for (int n = 0; n < N; n++) y[n] = sample_i16(iq + (size_t)s * slot_elems, p, t, a, n);
        oracle_fft(y, N);
        double* o = out + ((((size_t)s * T + t) * A + a) * N) * 2;
        for (int k = 0; k < N; k++) {
          o[2 * k] = creal(y[k]);
          o[2 * k + 1] = cimag(y[k]);
        }
      }
  free(y);
  return 0;
}

/* In-place FFT of a buffer of interleaved (re, im) doubles: the test hook for the FFT pins. */
int oracle_fft_interleaved(double* x, int n) {
  if (!is_pow2(n)) return -1;
  double complex* c = malloc(sizeof(double complex) * n);
  if (!c) return -4;
  for (int i = 0; i < n; i++) c[i] = x[2 * i] + I * x[2 * i + 1];
  int r = oracle_fft(c, n);
  for (int i = 0; i < n; i++) {
    x[2 * i] = creal(c[i]);
    x[2 * i + 1] = cimag(c[i]);
  }
  free(c);
  return r;
}

/* ---------------------------------------------------------------------------
 * Training channels of the learned denoiser (frequency domain).
 *
 * Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC 2011), counter {j, r, 0, 0} for
 * block j of row r, key {seed, 0}.  A 64-bit word w gives the uniform
 * u = (2 (w >> 41) + 1) 2^-24 in (0, 1) and, for integer draws over n values,
 * ((w >> 32) n) >> 32.  Box-Muller on (u_a, u_b):
 * sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b), one complex normal with unit
 * variance per component.
 *
 * One row is one antenna of one slot, drawn independently:
 *   block 0        L = taps_min + int(w0, taps_max - taps_min + 1),
 *                  span = tau_min + int(w1, tau_max - tau_min + 1) samples,
 *                  snr_db = snr_min + (snr_max - snr_min) u(w2);
 *   delays         delay_l = (l span + (L-1)/2) div (L-1) (0 for L = 1),
 *                  clamped to the CP; powers p_l ~ 10^(-decay l / 10), sum 1;
 *   blocks 1..     tap gains h_l = sqrt(p_l / 2) z, z from block 1 + l/2
 *                  (words 0,1 for even l, 2,3 for odd l);
 *   H_true[d]      sum_l h_l exp(-2 pi i ((f_d delay_l) mod N) / N);
 *   noise          sigma^2 = 10^(-snr_db / 10) per subcarrier (E|H|^2 = 1),
 *                  n_j = sqrt(sigma^2 / 2) z for pilot j, z from block
 *                  1 + ceil(taps_max / 2) + j/2 in the same way;
 *   H_ls           H_true + n on the comb d = j s, then comb interpolation.
 * With a unit-modulus pilot, LS of the received pilot subcarrier is exactly
 * H + n / X_p, and n / X_p has the distribution of n, so the time-domain chain
 * (OFDM, channel within the CP, AWGN, FFT) gives the same statistics.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t fft_len, n_used, cp_len, pilot_spacing;
  int32_t taps_min, taps_max, tau_min, tau_max; /* taps; max excess delay in samples */
  double snr_min_db, snr_max_db, tap_decay_db;
} oracle_gen_params;

static void mul64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 p = (unsigned __int128)a * b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; round++) {
    if (round > 0) {
      k0 += 0x9E3779B97F4A7C15ull;
      k1 += 0xBB67AE8584CAA73Bull;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mul64(0xD2E7470EE14C6C93ull, c0, &hi0, &lo0);
    mul64(0xCA5A826395121157ull, c2, &hi1, &lo1);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double unit_uniform(uint64_t w) { return (double)(2 * (w >> 41) + 1) * 0x1p-24; }
static int64_t int_draw(uint64_t w, int64_t n) { return (int64_t)(((w >> 32) * (uint64_t)n) >> 32); }

static void block_words(uint64_t seed, int64_t row, int64_t j, uint64_t w[4]) {
  const uint64_t ctr[4] = {(uint64_t)j, (uint64_t)row, 0, 0}, key[2] = {seed, 0};
  oracle_philox4x64(ctr, key, w);
}

static double complex normal_pair(uint64_t wa, uint64_t wb) {
  const double r = sqrt(-2.0 * log(unit_uniform(wa))), th = 2.0 * ORACLE_PI * unit_uniform(wb);
  return r * cos(th) + I * r * sin(th);
}

/* H_true, H_ls: double [rows][U][2]; the draws of each row (for tests):
 * n_taps [rows], delays int32 [rows][64], taps double [rows][64][2], snr_db
 * [rows].  Every output may be null.  Returns 0, -1 (bad parameters) or -4. */
int oracle_gen_channels(const oracle_gen_params* g, uint64_t seed, int64_t first_row, int64_t rows,
                        double* H_true, double* H_ls, int32_t* n_taps, int32_t* delays, double* taps,
                        double* snr_out) {
  if (!g || rows < 0 || !is_pow2(g->fft_len) || g->n_used < 2 || (g->n_used & 1) ||
      g->n_used > g->fft_len - 2 || g->pilot_spacing < 1 || g->pilot_spacing > g->n_used ||
      g->taps_min < 1 || g->taps_max < g->taps_min || g->taps_max > 64 || g->tau_min < 0 ||
      g->tau_max < g->tau_min || g->cp_len < 0)
    return -1;
  const int N = g->fft_len, U = g->n_used, s = g->pilot_spacing;
  const int64_t noise_block = 1 + (g->taps_max + 1) / 2;
  double complex h[64];
  int delay[64];
  double* ht = malloc(sizeof(double) * 2 * (size_t)U);
  if (!ht) return -4;
  for (int64_t rr = 0; rr < rows; rr++) {
    const int64_t row = first_row + rr;
    uint64_t w[4];
    block_words(seed, row, 0, w);
    const int L = g->taps_min + (int)int_draw(w[0], g->taps_max - g->taps_min + 1);
    const int span = g->tau_min + (int)int_draw(w[1], g->tau_max - g->tau_min + 1);
    const double snr_db = g->snr_min_db + (g->snr_max_db - g->snr_min_db) * unit_uniform(w[2]);
    double psum = 0.0;
    for (int l = 0; l < L; l++) psum += pow(10.0, -g->tap_decay_db * l / 10.0);
    for (int l = 0; l < L; l++) {
      int dl = L > 1 ? (l * span + (L - 1) / 2) / (L - 1) : 0;
      delay[l] = dl < g->cp_len ? dl : g->cp_len;
      uint64_t b[4];
      block_words(seed, row, 1 + l / 2, b);
      const double complex z = (l % 2 == 0) ? normal_pair(b[0], b[1]) : normal_pair(b[2], b[3]);
      h[l] = sqrt(pow(10.0, -g->tap_decay_db * l / 10.0) / psum / 2.0) * z;
    }
    if (n_taps) n_taps[rr] = L;
    if (snr_out) snr_out[rr] = snr_db;
    for (int l = 0; l < 64; l++) {
      if (delays) delays[rr * 64 + l] = l < L ? delay[l] : 0;
      if (taps) {
        taps[(rr * 64 + l) * 2] = l < L ? creal(h[l]) : 0.0;
        taps[(rr * 64 + l) * 2 + 1] = l < L ? cimag(h[l]) : 0.0;
      }
    }
    for (int d = 0; d < U; d++) {
      double complex acc = 0.0;
      const int f = signed_freq(d, U);
      for (int l = 0; l < L; l++) {
        const int m = (int)((((int64_t)f * delay[l]) % N + N) % N);
        acc += h[l] * (cos(-2.0 * ORACLE_PI * m / N) + I * sin(-2.0 * ORACLE_PI * m / N));
      }
      ht[2 * d] = creal(acc);
      ht[2 * d + 1] = cimag(acc);
    }
    if (H_true) memcpy(H_true + (size_t)rr * U * 2, ht, sizeof(double) * 2 * U);
    if (H_ls) {
      double* o = H_ls + (size_t)rr * U * 2;
      const double sd = sqrt(pow(10.0, -snr_db / 10.0) / 2.0);
      for (int d = 0, j = 0; d < U; d += s, j++) {
        uint64_t b[4];
        block_words(seed, row, noise_block + j / 2, b);
        const double complex z = (j % 2 == 0) ? normal_pair(b[0], b[1]) : normal_pair(b[2], b[3]);
        o[2 * d] = ht[2 * d] + sd * creal(z);
        o[2 * d + 1] = ht[2 * d + 1] + sd * cimag(z);
      }
      oracle_comb_interp(U, s, o, 1);
    }
  }
  free(ht);
  return 0;
}

/* ---------------------------------------------------------------------------
 * Frame synchronisation (paper Sec. II-B, implementation outline: the received
 * baseband stream is correlated with the maximum-length PN sequence that
 * opens every transmitted frame, and the correlation gives the offset of the
 * first OFDM frame; Table I: PN length 255).
 *
 * Reading: chips p[m] in {-1, 0, +1}; for every candidate start n in
 * [0, n_search) and every antenna a,
 *   c_a[n] = sum_{m=0}^{L-1} p[m] y_a[n+m]        (complex, integer)
 *   M[n]   = sum_a |c_a[n]|^2                      (non-coherent over antennas)
 * in exact integer arithmetic; the offset is the first n at which M is
 * largest.  y_a[i] is sample i of antenna a's stream (int16 I, Q), read at
 * raw[(a * stride + i) * 2]; samples at i >= n_samples count as zero.
 * ------------------------------------------------------------------------- */
int oracle_sync_metric(const int16_t* raw, int n_ant, int64_t n_samples, int64_t stride, const int8_t* pn, int L,
                       int64_t n_search, uint64_t* M, int64_t* offset) {
  if (!raw || !pn || n_ant < 1 || L < 1 || n_search < 1 || n_samples < 0 || stride < n_samples) return -1;
  int64_t best = -1;
  uint64_t best_v = 0;
  for (int64_t n = 0; n < n_search; n++) {
    uint64_t acc = 0;
    for (int a = 0; a < n_ant; a++) {
      int64_t re = 0, im = 0;
      for (int m = 0; m < L; m++) {
        const int64_t i = n + m;
        if (i >= n_samples) break;
        const int16_t* s = raw + ((size_t)a * stride + i) * 2;
        re += (int64_t)pn[m] * s[0];
        im += (int64_t)pn[m] * s[1];
      }
      acc += (uint64_t)(re * re) + (uint64_t)(im * im);
    }
    if (M) M[n] = acc;
    if (best < 0 || acc > best_v) {
      best = n;
      best_v = acc;
    }
  }
  if (offset) *offset = best;
  return 0;
}
