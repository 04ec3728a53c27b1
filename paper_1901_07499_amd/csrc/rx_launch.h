// rx_launch.h -- internal interface between the C ABI (rx_api.cpp) and the
// kernel launchers (rx_kernels.hip).  Not part of the public API.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct rx_plan_s;

namespace rx {

struct LaunchArgs {
  const uint32_t* iq;  // one dword per complex int16 sample, [S][T][A][CP+N]
  int64_t S;
  int A, N, CP, U, T, B;
  const float2* tw;    // tw[k] = exp(-2 pi i k / N), k < N
  const float2* pf;    // pf[d] = conj(Xp[d]) / |Xp[d]|^2 (pilot subcarriers only)
  int ps;              // pilot spacing: 1 = block pilot, > 1 = comb on d % ps == 0
  int fft_mode;        // enum rx_fft_mode
  hipStream_t stream;
};

// MFMA DFT-GEMM path (rx_mfma_fft.hip), N = 2048, fft_mode 1..4.
hipError_t launch_mfma_estimate(const LaunchArgs& la, float2* H);
hipError_t launch_mfma_demod(const LaunchArgs& la, const float2* H, float2* xhat, uint8_t* bits);
hipError_t launch_mfma_fft(const LaunchArgs& la, float2* Y);

hipError_t launch_estimate(const LaunchArgs& la, float2* H);
hipError_t launch_g(const LaunchArgs& la, const float2* H, float* g);
hipError_t launch_demod(const LaunchArgs& la, bool zf, const float2* H, float2* xhat, uint8_t* bits);
hipError_t launch_fft(const LaunchArgs& la, float2* Y);
// rx_process_frame with the estimate in a fixed buffer, slots in chunks that
// fit it (rx_api.cpp); returns an rx_status.
int process_frame_in(::rx_plan_s* plan, const int16_t* iq, int64_t n_slots, float* xhat, uint8_t* bits,
                     float2* hbuf, size_t hbuf_bytes, void* hip_stream);

// ---- batches of frames with mixed shapes (one slot per frame)
// Device descriptor of one frame; offsets index the packed batch buffers.
struct FrameDesc {
  int64_t iq_off;    // dwords (complex int16 samples) into the packed input
  int64_t h_off;     // complex entries into the packed channel estimates
  int64_t x_off;     // complex entries into the packed x-hat
  int64_t b_off;     // bytes into the packed bits
  const float2* pf;  // pilot factors of the frame, [U]
  int A, T, CP, U, B;
  int est_tile0;     // first estimate tile of the frame in its class queue
  int dem_tile0;     // first demod tile of the frame in its class queue
  int index;         // position of the frame in the batch
};

struct BatchIo {
  const uint32_t* iq;
  float2* H;
  float2* xhat;   // may be null
  uint8_t* bits;  // may be null
};

// A kernel chosen for one FFT-length class, with its launch geometry.
struct BatchKernel {
  const void* func = nullptr;
  int block = 0;             // threads per workgroup
  size_t lds_fft = 0;        // dynamic LDS for the FFT exchange buffers
  size_t lds_per_u = 0;      // extra dynamic LDS per used subcarrier (demod reduction rows)
  int ants_per_tile = 0;     // estimate: antennas per tile
};

// Kernels for FFT length N whose frames have at most max_u used subcarriers,
// with demod_waves in {2,4,8} wavefronts per demod workgroup, est_jobs in
// {2,4,8} jobs per estimate wavefront and radix schedules dem_sched and
// est_sched (below fft_schedule_count(N)).  False if unsupported.
bool batch_kernels(int N, int max_u, int demod_waves, int est_jobs, int dem_sched, int est_sched, BatchKernel& dem,
                   BatchKernel& est);
// Radix schedules of the N-point transform (0 if N is unsupported), and the
// radices of schedule sched, first pass first (0 after the last pass; all
// zero if there is no such schedule).
int fft_schedule_count(int N);
void fft_schedule_radices(int N, int sched, int radices[3]);
const void* batch_reset_func();

// ---- learned refinement of the channel estimate (rx_denoise.hip)
// Parameter vector: per layer W[co][ci][7] then b[co]; layers 2->32->32->32->2.
constexpr int kParams = 15330;
constexpr int kPW1 = 0, kPB1 = 448, kPW2 = 480, kPB2 = 7648, kPW3 = 7680, kPB3 = 14848, kPW4 = 14880,
              kPB4 = 15328;
// bf16 MFMA operand fragments of the weights, in 16-byte units (64 per block):
// forward F1[2], F2[2][7], F3[2][7], F4 (taps folded into rows); transposed
// G4[2], G3[2][7], G2[2][7].
constexpr int kF1 = 0, kF2 = 128, kF3 = 1024, kF4 = 1920, kG4 = 1984, kG3 = 2112, kG2 = 3008,
              kFragUnits = 3904;

// Training buffers (bf16 bits, channel-major [row][channel][UP], UP = U
// rounded up to 8) and partial sums.
struct DnTrainIo {
  const float2* Htrue;
  int64_t UP;
  float inv_count;  // 1 / (rows * U)
  uint16_t *X0, *X1, *X2, *X3;  // x0 (2 channels), x1..x3 (32)
  uint16_t *D1, *D2, *D3, *D4;  // deltas: d1..d3 (32 channels), d4 (2)
  uint32_t *M1, *M2, *M3;       // ReLU masks of x1..x3: [row][UP], bit c = (x[c] > 0)
  float* part;       // [grid][kParams] weight-gradient partials
  float* loss_part;  // [grid]
  // inference only: LS fallback threshold (max_corr^2) and per-row flags (or null)
  float fb_max2;
  uint8_t* fell;
};

struct AdamArgs {
  float* theta;  // null: no update
  float* m;
  float* v;
  float lr, beta1, beta2, eps, c1, c2;  // c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t)
};

// Training-channel recipe (delays in samples).
struct GenArgs {
  int N, U, CP, ps, taps_min, taps_max, tau_min, tau_max;
  float snr_min, snr_max, decay_db;
};

int dn_grid(int64_t rows);
hipError_t dn_relayout(const float* theta, uint16_t* frag, hipStream_t st);
// p[0 .. n) = v (a kernel rather than hipMemsetAsync, so callers may capture it).
hipError_t fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t st);
hipError_t dn_apply(const float2* Hin, int64_t rows, int U, const void* frag, const float* theta, float2* Hout,
                    float fb_max2, uint8_t* fell, hipStream_t st);
hipError_t dn_train(const float2* Hin, const float2* Htrue, int64_t rows, int U, const void* frag,
                    const float* theta, const DnTrainIo& io, float* grad, float* loss, const AdamArgs& adam,
                    hipStream_t st);
hipError_t dn_generate(const GenArgs& g, uint64_t seed, int64_t first_row, int64_t rows, float2* Htrue,
                       float2* Hls, hipStream_t st);

// ---- PN frame synchronisation (rx_sync.hip)
constexpr int kMaxPn = 1024;
struct SyncChips {  // passed by value as a kernel argument
  int L;
  int8_t c[kMaxPn];
};
int sync_groups(int A, int64_t n_search);
size_t sync_workspace(int A, int64_t n_search);
hipError_t sync_find(const uint32_t* raw, int A, int64_t n_samples, int64_t stride, const SyncChips& ch,
                     int64_t n_search, uint64_t* M, int64_t* offset, uint64_t* peak, void* workspace,
                     hipStream_t st);
hipError_t sync_extract(const uint32_t* raw, int A, int64_t n_samples, int64_t stride, const int64_t* start,
                        int64_t start_add, int sym_len, int T, int64_t S, uint32_t* out, hipStream_t st);

}  // namespace rx
