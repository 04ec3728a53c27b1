/*
 * rx.h -- C ABI of the MI355X (gfx950) uplink OFDM receive library librx.so.
 *
 * The library runs the receive path of a single-user, many-antenna uplink:
 * int16 IQ samples of every antenna and OFDM symbol -> cyclic-prefix removal
 * -> N-point FFT per antenna and symbol -> block least-squares channel
 * estimate from the first (pilot) symbol -> combining over the antennas
 * (maximal ratio, or zero forcing for one user) -> hard QAM decisions packed
 * into bytes.
 *
 * The operations follow the paper (Gokalgandhi et al., "Accelerating Channel
 * Estimation and Demodulation of Uplink OFDM symbols for Large Scale Antenna
 * Systems using GPU"): the CP is dropped and an FFT taken for every antenna's
 * symbol (Sec. II-B, II-C); the first symbol gives the LS estimate, the
 * received subcarrier divided by the pilot (Sec. II-B; Sec. II-C, LS
 * paragraph); later symbols are combined per subcarrier over all antennas by
 * MRC (Sec. II-C, MRC paragraph); subcarriers are in fftshift order
 * (Sec. II-C, last sentence).  Where the paper is silent this library fixes:
 *   - FFT: Y[k] = sum_n y[n] exp(-2 pi i k n / N), no scaling;
 *   - used subcarrier d (0..U-1) has signed frequency d-U/2 for d < U/2 and
 *     d-U/2+1 otherwise, i.e. FFT bin k_d = f_d mod N (DC, Nyquist unused);
 *   - LS: H[a][d] = Y_0[a][k_d] * conj(X_p[d]) / |X_p[d]|^2;
 *   - MRC: xhat = sum_a conj(H[a][d]) Y_t[a][k_d] / g[d], g[d] = sum_a |H[a][d]|^2,
 *     and xhat = 0 when g[d] == 0;  ZF (one user): xhat = sum_a w_a Y_t[a][k_d],
 *     w_a = conj(H[a][d]) / g[d];
 *   - decisions per axis with strict comparisons (a value exactly on a
 *     threshold, or -0.0, gives bit 0): first bit of an axis = [c < 0];
 *     16-QAM second bit = [|c| sqrt(10) > 2]; 64-QAM second = [|c| sqrt(42) > 4],
 *     third = [| |c| sqrt(42) - 4 | > 2]; bits of the real axis take even
 *     positions b0, b2, b4 and of the imaginary axis odd positions b1, b3, b5;
 *   - bits are packed MSB-first in the order [slot][data symbol][d][b0..].
 *
 * Memory layouts (all row-major, C order; "complex" = two floats re, im):
 *   iq    int16   [S][T][A][CP+N][2]     input, 4-byte aligned
 *   H     float   [S][A][U][2]           LS channel estimate, 8-byte aligned
 *   g     float   [S][U]                 sum over antennas of |H|^2
 *   xhat  float   [S][T-1][U][2]         combined data symbols, 8-byte aligned
 *   bits  uint8   [S][T-1][U*b/8]        hard decisions, packed
 * S = n_slots, T = n_sym (symbol 0 is the pilot), A = n_ant, N = fft_len,
 * CP = cp_len, U = n_used, b = bits_per_sym.
 *
 * Ownership: every data pointer passed to the compute calls is a DEVICE
 * pointer owned by the caller and valid on the plan's device.  The plan owns
 * a copy of the parameters and small device tables (twiddles, pilot factors;
 * a few tens of KB) created in rx_plan_create and freed in rx_plan_destroy.
 * Scratch beyond that is caller-provided (see rx_workspace_bytes).
 *
 * Errors: every argument check runs before anything is launched, so a call
 * that returns an error has written nothing.  n_slots == 0 is a valid no-op
 * (only the plan is checked; data pointers may then be NULL).  Compute calls are asynchronous
 * on the given HIP stream (NULL = the null stream); faults during execution
 * surface at the caller's next synchronisation.  A plan is immutable after
 * creation and may be used from several streams at once provided each call
 * has its own output and workspace buffers.
 */
#ifndef RX_H
#define RX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rx_plan_s* rx_plan_t;

enum rx_status {
  RX_OK = 0,
  RX_E_INVALID_ARG = -1, /* bad shape, null/misaligned pointer, zero pilot, wrong device */
  RX_E_UNSUPPORTED = -2, /* valid but not implemented: N not a power of two in 64..2048,
                            bits_per_sym not in {2,4,6}, more than one user, unknown combiner */
  RX_E_HIP = -3,         /* a HIP runtime call or kernel launch failed */
  RX_E_NOMEM = -4,       /* device or host allocation failed */
  RX_E_SCRATCH = -5      /* the call needs more than the library's fixed scratch
                            (rx_process_frame_noalloc) */
};

enum rx_combiner { RX_COMB_MRC = 0, RX_COMB_ZF = 1 };

/* FFT arithmetic.  RX_FFT_RADIX_F32: Stockham radix FFT in FP32 on the vector
 * units (every N).  The MFMA modes (N = 2048, U <= 1536, MRC, block pilot
 * only) recast the transform as 2048 = 8 x 16 x 16: an FP32 radix-8 stage,
 * then two 16-point DFT stages as GEMMs on the fp16 or bf16 matrix cores
 * with FP32 accumulation; _SPLIT also splits both GEMM operands into
 * hi + lo parts and sums the three significant products. */
enum rx_fft_mode {
  RX_FFT_RADIX_F32 = 0,
  RX_FFT_MFMA_F16 = 1,
  RX_FFT_MFMA_BF16 = 2,
  RX_FFT_MFMA_F16_SPLIT = 3,
  RX_FFT_MFMA_BF16_SPLIT = 4
};

typedef struct {
  int32_t n_ant;        /* A >= 1 receive antennas */
  int32_t fft_len;      /* N, a power of two in [64, 2048] */
  int32_t cp_len;       /* CP, 0 <= CP < N */
  int32_t n_used;       /* U, even, 2 <= U <= N-2, and U*b a multiple of 8 */
  int32_t n_sym;        /* T >= 2: symbol 0 = pilot, 1..T-1 = data */
  int32_t bits_per_sym; /* b: 2 (QPSK), 4 (16-QAM), 6 (64-QAM) */
  int32_t combiner;     /* RX_COMB_MRC or RX_COMB_ZF */
  int32_t n_users;      /* K, must be 1 (single-user uplink) */
  const float* pilot;   /* HOST pointer to U complex pilot values in d order;
                           every pilot value non-zero and finite; copied by rx_plan_create */
  int32_t pilot_spacing; /* 0 or 1: block pilot, every used subcarrier of symbol 0
                            carries one (the paper's arrangement).  s > 1 (s <= U): comb
                            pilot on d = 0, s, 2s, ... only (values elsewhere ignored);
                            LS there, then every subcarrier is interpolated along a
                            straight line in signed frequency between the pilot at or
                            below it and the next pilot (spanning the DC gap), and past
                            the last pilot that pilot's value is held.  The comb form is
                            the standard LS-with-interpolation estimator the learned
                            refinement below starts from.  Batches need 0 or 1. */
  int32_t fft_mode;      /* enum rx_fft_mode; 0 = FP32 radix (batches need 0) */
} rx_params;

/* Validate parameters without touching the GPU.  Returns RX_OK or the status
 * rx_plan_create would return for them. */
int rx_params_check(const rx_params* p);

/* Create a plan on the current HIP device.  *out is set only on RX_OK. */
int rx_plan_create(const rx_params* p, rx_plan_t* out);

/* Release a plan and its device tables.  NULL is accepted (no-op). */
int rx_plan_destroy(rx_plan_t plan);

/* Bytes of device scratch that rx_process_frame needs when H == NULL
 * (it then keeps the channel estimate there): S*A*U*8.  0 for a NULL plan or
 * n_slots <= 0.  rx_estimate and rx_demod need none. */
size_t rx_workspace_bytes(rx_plan_t plan, int64_t n_slots);

/* Channel estimation (paper Sec. II-B, first symbol; Sec. II-C, LS):
 * CP removal + FFT of the pilot symbol of every antenna, then
 * H[s][a][d] = Y_0[s][a][k_d] * conj(X_p[d]) / |X_p[d]|^2 (on the comb and
 * interpolated in between when pilot_spacing > 1).
 * iq required; H required; g optional (NULL = not computed); workspace unused. */
int rx_estimate(rx_plan_t plan, const int16_t* iq, int64_t n_slots, float* H, float* g,
                void* workspace, void* hip_stream);

/* Demodulation of the data symbols (paper Sec. II-B; Sec. II-C, MRC): CP
 * removal + FFT of symbols 1..T-1 of every antenna, combining with the given
 * channel estimate H (layout above, e.g. from rx_estimate), hard decisions.
 * xhat and bits are optional but not both NULL; workspace unused. */
int rx_demod(rx_plan_t plan, const int16_t* iq, const float* H, int64_t n_slots, float* xhat,
             uint8_t* bits, void* workspace, void* hip_stream);

/* The whole path for S slots: rx_estimate followed by rx_demod on one stream.
 * H optional: when NULL the estimate is kept in `workspace`
 * (>= rx_workspace_bytes(plan, n_slots) bytes, 256-byte aligned).
 * xhat and bits optional but not both NULL. */
int rx_process_frame(rx_plan_t plan, const int16_t* iq, int64_t n_slots, float* H, float* xhat,
                     uint8_t* bits, void* workspace, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the whole
 * path of rx_process_frame without H or workspace arguments; nothing is
 * allocated.  The channel estimate is kept in a library-owned device array of
 * RX_NOALLOC_SCRATCH_BYTES on each GPU the library runs on, held until the
 * process ends, and the slots go through in chunks whose estimates fit it
 * (one launch pair per chunk; results equal rx_process_frame's).  One slot's
 * estimate, A*U*8 bytes, must fit, else RX_E_SCRATCH.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (different streams,
 * or host threads) race and must be serialised by the caller.  The array
 * needs no clearing (each chunk's estimate is written before it is read).
 * xhat and bits optional but not both NULL. */
#define RX_NOALLOC_SCRATCH_BYTES (64u << 20)
int rx_process_frame_noalloc(rx_plan_t plan, const int16_t* iq, int64_t n_slots, float* xhat, uint8_t* bits,
                             void* hip_stream);

/* CP removal + FFT only, for every symbol of every antenna:
 * Y float [S][T][A][N][2] in natural bin order.  For validating the FFT stage. */
int rx_debug_fft(rx_plan_t plan, const int16_t* iq, int64_t n_slots, float* Y, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Batches of frames with mixed shapes.  A frame is one slot (n_sym symbols,
 * symbol 0 the pilot) with its own rx_params (antennas, FFT length, CP, used
 * subcarriers, QAM order, pilot; combiner must be RX_COMB_MRC).  Frames are
 * packed back to back in batch order: frame i's int16 samples start at
 * iq_off[i] (int16 elements, layout [T][A][CP+N][2]), its estimate at
 * h_off[i] complex entries of the H buffer ([A][U]), its x-hat at x_off[i]
 * complex entries ([T-1][U]) and its bits at b_off[i] bytes ([T-1][U*b/8]).
 * The path per frame is the one of rx_process_frame (paper Sec. II-B and
 * II-C); the batch runs it for every frame in one graph launch.  Frames with
 * equal FFT length share one persistent estimate kernel and one persistent
 * demod kernel that take tiles from device work queues (frames with more
 * antennas first, ties in batch order); different FFT lengths run on
 * independent graph branches.
 * ------------------------------------------------------------------------- */
typedef struct rx_batch_s* rx_batch_t;

/* Create a batch of n_frames (1..65536) frames on the current HIP device.
 * Every frame is validated as by rx_params_check; pilots are copied. */
int rx_batch_create(const rx_params* frames, int32_t n_frames, rx_batch_t* out);

/* NULL-safe. */
int rx_batch_destroy(rx_batch_t batch);

/* Packed offsets: each non-NULL array receives n_frames + 1 entries, the last
 * one being the total size (units as described above). */
int rx_batch_layout(rx_batch_t batch, int64_t* iq_off, int64_t* h_off, int64_t* x_off, int64_t* b_off);

/* Bytes of scratch rx_batch_process needs for the estimates when H == NULL. */
size_t rx_batch_workspace_bytes(rx_batch_t batch);

/* Run the whole batch on hip_stream (asynchronous; one graph launch).  iq
 * required (4-byte aligned); H optional (then `workspace` holds the
 * estimates, >= rx_batch_workspace_bytes, 256-byte aligned); xhat and bits
 * optional but not both NULL.  The graph is rebuilt when the pointers differ
 * from the previous call's. */
int rx_batch_process(rx_batch_t batch, const int16_t* iq, float* H, float* xhat, uint8_t* bits,
                     void* workspace, void* hip_stream);

/* Time the launch configurations of every FFT-length class on these buffers
 * (reps timed runs each after one warm-up, the minimum counts).  A
 * configuration is the demod workgroup size, the estimate's jobs per
 * wavefront and the radix schedule of each kernel's transforms (see
 * rx_fft_radices).  First each class alone: every shape under every
 * schedule, the estimate's and the demod's choices made separately; then,
 * class by class from the longest, within the whole batch graph with the
 * other classes as chosen so far: every shape with the class's schedules,
 * then every pair of schedules with the best shape, a choice replaced only
 * by one more than 1 % faster.  The whole batch runs 16 times first, untimed.
 * Synchronous; overwrites the outputs. */
int rx_batch_autotune(rx_batch_t batch, const int16_t* iq, float* H, float* xhat, uint8_t* bits,
                      void* workspace, int32_t reps, void* hip_stream);

/* Configuration in use for the class of FFT length fft_len: wavefronts per
 * demod workgroup and jobs per estimate wavefront. */
int rx_batch_config(rx_batch_t batch, int32_t fft_len, int32_t* demod_waves, int32_t* est_jobs);

/* Radix schedules in use for the class of FFT length fft_len: of the demod
 * kernel's transforms and of the estimate kernel's (indices as in
 * rx_fft_radices).  RX_E_INVALID_ARG if the batch has no such class. */
int rx_batch_schedules(rx_batch_t batch, int32_t fft_len, int32_t* dem_sched, int32_t* est_sched);

/* Set the configuration of the class of FFT length fft_len instead of tuning
 * it: demod_waves and est_jobs in {2, 4, 8}, schedules below the count
 * rx_fft_radices accepts for fft_len.  The batch's current device only;
 * RX_E_INVALID_ARG for anything else (the configuration is then unchanged).
 * The next rx_batch_process rebuilds its graph. */
int rx_batch_set_config(rx_batch_t batch, int32_t fft_len, int32_t demod_waves, int32_t est_jobs,
                        int32_t dem_sched, int32_t est_sched);

/* Radix schedule `sched` of the fft_len-point transform of the batch kernels
 * (paper Sec. II-B, the per-symbol FFT of the outline, and Sec. II-C, the
 * batched FFT of all antennas' symbols): radices[0..2] receive the radix of each
 * Stockham pass, first pass first, 0 after the last pass (radix 16 first in
 * every schedule; 512, 1024 and 2048 have two schedules, 16-R-16 and 16-16-R,
 * the other lengths one).  RX_E_UNSUPPORTED when fft_len has no schedule
 * `sched`; host only. */
int rx_fft_radices(int32_t fft_len, int32_t sched, int32_t* radices);

/* Per-frame completion time of the most recent rx_batch_process, in ms after
 * the batch started on the device (device clock); ms has n_frames entries.
 * Waits for hip_stream. */
int rx_batch_frame_latency(rx_batch_t batch, double* ms, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Learned refinement of a comb-pilot LS channel estimate.
 *
 * The paper estimates the channel by LS alone (Sec. II-C, LS paragraph); a
 * comb pilot (rx_params.pilot_spacing) gives LS on every s-th subcarrier plus
 * linear interpolation, and this network refines that estimate per antenna.
 * For a row h[0..U) (one antenna of one slot; complex):
 *   s = sqrt(mean_d |h[d]|^2),  x0 = (Re h / s, Im h / s)        2 channels
 *   a_l[co][d] = b_l[co] + sum_ci sum_k W_l[co][ci][k] x_{l-1}[ci][d+k-3],
 *     k = 0..6, x zero outside 0..U-1;  x_l = max(a_l, 0) for l = 1, 2, 3;
 *     channels 2 -> 32 -> 32 -> 32 -> 2
 *   out[d] = h[d] + s (a_4[0][d] + i a_4[1][d])      (a zero row passes through)
 * Parameters (RX_DN_PARAMS floats): for l = 1..4, W_l[co][ci][k] then b_l[co].
 * Training loss: mean over rows and d of |x0 + a_4 - h_true / s|^2, with the
 * gradient by backpropagation and Adam (Kingma and Ba, 2015).  Products run
 * on bf16 MFMA with FP32 accumulation: weights, activations and backward
 * deltas are rounded to bf16 (nearest even) where they enter a product.
 * Rows are float [rows][U][2]; every pointer is a device pointer.
 * ------------------------------------------------------------------------- */
#define RX_DN_PARAMS 15330

typedef struct rx_dn_s* rx_dn_t;

/* Create a denoiser for rows of n_used (2..2046) subcarriers on the current
 * device.  Holds a copy of the parameters and their bf16 operand layout
 * (about 130 KB).  Parameters must be loaded before use. */
int rx_dn_create(int32_t n_used, rx_dn_t* out);

/* NULL-safe. */
int rx_dn_destroy(rx_dn_t dn);

/* Load parameters (device float [RX_DN_PARAMS]) into the denoiser. */
int rx_dn_load(rx_dn_t dn, const float* params, void* hip_stream);

/* out = refined rows, with plain LS as the fallback: a row keeps its input
 * (LS) estimate when its correction c = out - h has a non-finite entry or
 * carries more energy than the row, sum_d |c[d]|^2 > max_corr^2 sum_d |h[d]|^2
 * (max_corr from rx_dn_set_fallback, default 1: a refinement that removes
 * noise never changes a row by more than the row itself).  Without loaded
 * parameters every row keeps its LS estimate.  H_out may equal H_in (each row
 * is read before it is written); otherwise the two must not overlap.
 * rows == 0 is a no-op. */
int rx_dn_apply(rx_dn_t dn, const float* H_in, int64_t rows, float* H_out, void* hip_stream);

/* rx_dn_apply that also reports, per row, whether it kept LS: fell device
 * uint8 [rows] (1 = LS kept, 0 = refined) or NULL; it must not overlap the
 * row buffers. */
int rx_dn_apply_judged(rx_dn_t dn, const float* H_in, int64_t rows, float* H_out, uint8_t* fell,
                       void* hip_stream);

/* Threshold of the LS fallback: max_corr > 0, +infinity keeps only rows whose
 * correction is not finite.  Host only; applies to later calls. */
int rx_dn_set_fallback(rx_dn_t dn, float max_corr);

/* Device scratch for rx_dn_grad and rx_dn_train_step on `rows` rows
 * (activations and deltas in bf16, per-workgroup partial sums). */
size_t rx_dn_workspace_bytes(rx_dn_t dn, int64_t rows);

/* Loss (device float [1]) and its gradient (device float [RX_DN_PARAMS]) at
 * the loaded parameters for inputs H_in and targets H_true (both
 * [rows][U][2]).  workspace >= rx_dn_workspace_bytes, 256-byte aligned.
 * Deterministic for a given row count.  grad and loss may be NULL. */
int rx_dn_grad(rx_dn_t dn, const float* H_in, const float* H_true, int64_t rows, float* grad, float* loss,
               void* workspace, void* hip_stream);

/* One training step: gradient at the loaded parameters (which must equal
 * params), then Adam step number `step` (>= 1) on params, m and v (device
 * float [RX_DN_PARAMS] each; m, v start at zero) with learning rate lr,
 * then the updated params are loaded.  loss may be NULL. */
int rx_dn_train_step(rx_dn_t dn, float* params, float* adam_m, float* adam_v, int64_t step, float lr, float beta1,
                     float beta2, float eps, const float* H_in, const float* H_true, int64_t rows, float* loss,
                     void* workspace, void* hip_stream);

/* Recipe of the training channels (delays in samples). */
typedef struct {
  int32_t fft_len;       /* N, power of two, 64..2048 */
  int32_t n_used;        /* U, even, 2..N-2 */
  int32_t cp_len;        /* delays are clamped to the CP, 0 <= CP < N */
  int32_t pilot_spacing; /* comb spacing s, 1..U */
  int32_t taps_min, taps_max;  /* 1 <= taps_min <= taps_max <= 64 */
  int32_t tau_min, tau_max;    /* maximum excess delay range, samples, 0 <= min <= max */
  float snr_min_db, snr_max_db;
  float tap_decay_db;    /* power drop per tap */
} rx_chan_gen;

/* Training pairs for rows first_row .. first_row+rows-1 of a seeded stream
 * (each row independent): the true frequency response H_true (unit mean
 * power) and the comb LS estimate H_ls (true response plus complex Gaussian
 * noise of variance 10^(-snr/10) on the pilots, then comb interpolation).
 * Per row, from Philox4x64-10 (counter {block, row, 0, 0}, key {seed, 0};
 * uniform u = (2 (w >> 41) + 1) 2^-24; integer draws ((w >> 32) n) >> 32;
 * complex normals by Box-Muller):
 *   block 0: L = taps_min + int(w0, taps_max-taps_min+1), span = tau_min +
 *     int(w1, tau_max-tau_min+1), snr = snr_min + (snr_max-snr_min) u(w2);
 *   delay_l = (l span + (L-1)/2) / (L-1) clamped to the CP; power of tap l
 *     proportional to 10^(-decay l / 10), summing to 1; gain of tap l from
 *     block 1 + l/2 (words 0,1 for even l, 2,3 for odd);
 *   H_true[d] = sum_l h_l exp(-2 pi i (f_d delay_l mod N) / N);
 *   pilot j's noise from block 1 + ceil(taps_max/2) + j/2.
 * H_true or H_ls may be NULL. */
int rx_dn_generate(const rx_chan_gen* gen, uint64_t seed, int64_t first_row, int64_t rows, float* H_true,
                   float* H_ls, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Frame synchronisation.  The transmitter opens a frame with a maximum-length
 * PN sequence; the receiver correlates every antenna's stream with it and the
 * correlation peak marks the frame start, from which the OFDM slots are cut
 * (paper Sec. II-B, implementation outline; Table I: PN length 255).
 *
 * Streams: raw int16 [A][stride][2], antenna a's sample i at raw[(a*stride +
 * i)*2] (I, Q); samples i >= n_samples (and i < 0) count as zero.
 * Metric, in exact integer arithmetic, for candidate starts n < n_search:
 *   c_a[n] = sum_{m<L} p[m] y_a[n+m],  M[n] = sum_a |c_a[n]|^2  (uint64)
 * offset = the smallest n with the largest M[n].  Chips p[m] in {-1, 0, +1}.
 * ------------------------------------------------------------------------- */
#define RX_SYNC_MAX_PN 1024

/* Device scratch of rx_sync_find for n_ant antennas and n_search candidates
 * (per-antenna-group partial metrics and per-block maxima; at most
 * 64 * 8 * n_search bytes plus 16 per 64 candidates).  0 on bad arguments. */
size_t rx_sync_workspace_bytes(int32_t n_ant, int64_t n_search);

/* Correlation metric and peak.  raw: device, 4-byte aligned; 1 <= n_ant <= 4096;
 * 1 <= n_search <= 2^36;
 * pn: HOST array of pn_len (1..RX_SYNC_MAX_PN) chips, copied into the launch;
 * metric: device uint64 [n_search] or NULL; offset: device int64 [1]; peak:
 * device uint64 [1] or NULL; workspace >= rx_sync_workspace_bytes(n_ant, n_search),
 * 256-byte aligned.  Asynchronous. */
int rx_sync_find(const int16_t* raw, int32_t n_ant, int64_t n_samples, int64_t stride, const int8_t* pn,
                 int32_t pn_len, int64_t n_search, uint64_t* metric, int64_t* offset, uint64_t* peak,
                 void* workspace, void* hip_stream);

/* Cut n_slots slots of n_sym symbols of sym_len (= CP + N) samples, back to
 * back from stream sample (*start + start_add) (start: device int64 [1], e.g.
 * rx_sync_find's offset, or NULL for 0), into iq int16 [n_slots][n_sym][A]
 * [sym_len][2] (device, 4-byte aligned): the input layout of rx_estimate,
 * rx_demod and rx_process_frame.  Out-of-stream samples are written as zero.
 * For a preamble of L chips detected at offset o, start_add = L puts the first
 * slot right after it. */
int rx_sync_extract(const int16_t* raw, int32_t n_ant, int64_t n_samples, int64_t stride, const int64_t* start,
                    int64_t start_add, int32_t sym_len, int32_t n_sym, int64_t n_slots, int16_t* iq,
                    void* hip_stream);

/* Static description of a status code. */
const char* rx_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* RX_H */
