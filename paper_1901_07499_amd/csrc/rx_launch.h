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

}  // namespace rx
