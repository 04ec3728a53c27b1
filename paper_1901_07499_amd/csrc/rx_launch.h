// rx_launch.h -- internal interface between the C ABI (rx_api.cpp) and the
// kernel launchers (rx_kernels.hip).  Not part of the public API.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rx {

struct LaunchArgs {
  const uint32_t* iq;  // one dword per complex int16 sample, [S][T][A][CP+N]
  int64_t S;
  int A, N, CP, U, T, B;
  const float2* tw;    // tw[k] = exp(-2 pi i k / N), k < N
  const float2* pf;    // pf[d] = conj(Xp[d]) / |Xp[d]|^2
  hipStream_t stream;
};

hipError_t launch_estimate(const LaunchArgs& la, float2* H);
hipError_t launch_g(const LaunchArgs& la, const float2* H, float* g);
hipError_t launch_demod(const LaunchArgs& la, bool zf, const float2* H, float2* xhat, uint8_t* bits);
hipError_t launch_fft(const LaunchArgs& la, float2* Y);

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
// with demod_waves in {2,4,8} wavefronts per demod workgroup and est_jobs in
// {2,4,8} jobs per estimate wavefront.  False if unsupported.
bool batch_kernels(int N, int max_u, int demod_waves, int est_jobs, BatchKernel& dem, BatchKernel& est);
const void* batch_reset_func();

}  // namespace rx
