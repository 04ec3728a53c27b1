// rx_api.cpp -- C ABI of librx.so (declared in include/rx.h).
//
// Argument checks happen first and touch no GPU state, so an error return
// leaves every output untouched and rx_params_check works on a machine
// without a GPU.  A plan holds the parameters plus two small device tables:
// the FFT twiddles exp(-2 pi i k / N) and the LS pilot factors
// conj(Xp[d]) / |Xp[d]|^2 (both evaluated in double, stored as float).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/rx.h"
#include "rx_launch.h"

struct rx_plan_s {
  rx_params p;
  std::vector<float> pilot;  // host copy, 2U floats
  int device = -1;
  float2* tw = nullptr;      // [N]
  float2* pf = nullptr;      // [U]
};

namespace {

bool is_pow2(int32_t n) { return n > 0 && (n & (n - 1)) == 0; }

int spacing(const rx_params& p) { return p.pilot_spacing > 1 ? p.pilot_spacing : 1; }

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

int check_params(const rx_params* p) {
  if (!p) return RX_E_INVALID_ARG;
  if (p->n_users < 1) return RX_E_INVALID_ARG;
  if (p->n_users != 1) return RX_E_UNSUPPORTED;
  if (p->n_ant < 1) return RX_E_INVALID_ARG;
  if (p->n_ant > 65536) return RX_E_UNSUPPORTED;
  if (p->fft_len < 1) return RX_E_INVALID_ARG;
  if (!is_pow2(p->fft_len) || p->fft_len < 64 || p->fft_len > 2048) return RX_E_UNSUPPORTED;
  if (p->cp_len < 0 || p->cp_len >= p->fft_len) return RX_E_INVALID_ARG;
  if (p->n_used < 2 || p->n_used > p->fft_len - 2 || (p->n_used & 1)) return RX_E_INVALID_ARG;
  if (p->n_sym < 2 || p->n_sym > 4096) return RX_E_INVALID_ARG;
  if (p->bits_per_sym != 2 && p->bits_per_sym != 4 && p->bits_per_sym != 6) return RX_E_UNSUPPORTED;
  if ((p->n_used * p->bits_per_sym) % 8) return RX_E_INVALID_ARG;
  if (p->combiner != RX_COMB_MRC && p->combiner != RX_COMB_ZF) return RX_E_UNSUPPORTED;
  if (!p->pilot) return RX_E_INVALID_ARG;
  if (p->pilot_spacing < 0 || p->pilot_spacing > p->n_used) return RX_E_INVALID_ARG;
  if (p->fft_mode < RX_FFT_RADIX_F32 || p->fft_mode > RX_FFT_MFMA_BF16_SPLIT) return RX_E_UNSUPPORTED;
  if (p->fft_mode != RX_FFT_RADIX_F32 &&
      (p->fft_len != 2048 || p->n_used > 1536 || p->combiner != RX_COMB_MRC || p->pilot_spacing > 1))
    return RX_E_UNSUPPORTED;
  for (int d = 0; d < p->n_used; d += spacing(*p)) {
    const float re = p->pilot[2 * d], im = p->pilot[2 * d + 1];
    if (!std::isfinite(re) || !std::isfinite(im) || (re == 0.0f && im == 0.0f)) return RX_E_INVALID_ARG;
  }
  return RX_OK;
}

// Total int16 elements of the input, or -1 on overflow.
int64_t iq_elems(const rx_params& p, int64_t S) {
  const int64_t per_slot = (int64_t)p.n_sym * p.n_ant * (p.fft_len + p.cp_len) * 2;
  if (S > (INT64_C(1) << 62) / per_slot) return -1;
  return per_slot * S;
}

int check_call(rx_plan_t plan, const int16_t* iq, int64_t S) {
  if (!plan) return RX_E_INVALID_ARG;
  if (S < 0) return RX_E_INVALID_ARG;
  if (iq_elems(plan->p, S) < 0) return RX_E_INVALID_ARG;
  // grid sizes are S * (T-1) and S * T * blocks: keep them within 2^31 - 1
  if (S * plan->p.n_sym * (int64_t)((plan->p.n_ant + 3) / 4) > INT64_C(0x7fffffff)) return RX_E_UNSUPPORTED;
  if (S > 0 && (!iq || !aligned(iq, 4))) return RX_E_INVALID_ARG;
  return RX_OK;
}

int check_device(rx_plan_t plan) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return RX_E_HIP;
  return dev == plan->device ? RX_OK : RX_E_INVALID_ARG;
}

rx::LaunchArgs launch_args(rx_plan_t plan, const int16_t* iq, int64_t S, void* stream) {
  rx::LaunchArgs la;
  la.iq = reinterpret_cast<const uint32_t*>(iq);
  la.S = S;
  la.A = plan->p.n_ant;
  la.N = plan->p.fft_len;
  la.CP = plan->p.cp_len;
  la.U = plan->p.n_used;
  la.T = plan->p.n_sym;
  la.B = plan->p.bits_per_sym;
  la.tw = plan->tw;
  la.pf = plan->pf;
  la.ps = spacing(plan->p);
  la.fft_mode = plan->p.fft_mode;
  la.stream = reinterpret_cast<hipStream_t>(stream);
  return la;
}

int hip_status(hipError_t e) { return e == hipSuccess ? RX_OK : RX_E_HIP; }

}  // namespace

extern "C" {

int rx_params_check(const rx_params* p) { return check_params(p); }

int rx_plan_create(const rx_params* p, rx_plan_t* out) {
  if (!out) return RX_E_INVALID_ARG;
  const int st = check_params(p);
  if (st != RX_OK) return st;
  rx_plan_s* plan = new (std::nothrow) rx_plan_s;
  if (!plan) return RX_E_NOMEM;
  plan->p = *p;
  plan->pilot.assign(p->pilot, p->pilot + 2 * p->n_used);
  plan->p.pilot = plan->pilot.data();
  if (hipGetDevice(&plan->device) != hipSuccess) {
    delete plan;
    return RX_E_HIP;
  }
  const int N = p->fft_len, U = p->n_used;
  std::vector<float2> tw(N), pf(U);
  const double two_pi = 6.283185307179586476925286766559;
  for (int k = 0; k < N; k++) {
    const double ang = -two_pi * (double)k / (double)N;
    tw[k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  for (int d = 0; d < U; d++) {
    const double re = p->pilot[2 * d], im = p->pilot[2 * d + 1];
    const double m2 = re * re + im * im;
    // subcarriers off a comb carry no pilot: their factor is never used
    pf[d] = d % spacing(*p) ? make_float2(0.f, 0.f) : make_float2((float)(re / m2), (float)(-im / m2));
  }
  if (hipMalloc(&plan->tw, sizeof(float2) * N) != hipSuccess ||
      hipMalloc(&plan->pf, sizeof(float2) * U) != hipSuccess) {
    (void)hipFree(plan->tw);
    (void)hipFree(plan->pf);
    delete plan;
    return RX_E_NOMEM;
  }
  if (hipMemcpy(plan->tw, tw.data(), sizeof(float2) * N, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(plan->pf, pf.data(), sizeof(float2) * U, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(plan->tw);
    (void)hipFree(plan->pf);
    delete plan;
    return RX_E_HIP;
  }
  *out = plan;
  return RX_OK;
}

int rx_plan_destroy(rx_plan_t plan) {
  if (!plan) return RX_OK;
  int st = RX_OK;
  if (plan->tw && hipFree(plan->tw) != hipSuccess) st = RX_E_HIP;
  if (plan->pf && hipFree(plan->pf) != hipSuccess) st = RX_E_HIP;
  delete plan;
  return st;
}

size_t rx_workspace_bytes(rx_plan_t plan, int64_t n_slots) {
  if (!plan || n_slots <= 0) return 0;
  return (size_t)n_slots * plan->p.n_ant * plan->p.n_used * sizeof(float2);
}

int rx_estimate(rx_plan_t plan, const int16_t* iq, int64_t n_slots, float* H, float* g, void* workspace,
                void* hip_stream) {
  (void)workspace;
  int st = check_call(plan, iq, n_slots);
  if (st != RX_OK || n_slots == 0) return st;
  if (!H || !aligned(H, 8)) return RX_E_INVALID_ARG;
  if (g && !aligned(g, 4)) return RX_E_INVALID_ARG;
  if ((st = check_device(plan)) != RX_OK) return st;
  const rx::LaunchArgs la = launch_args(plan, iq, n_slots, hip_stream);
  float2* H2 = reinterpret_cast<float2*>(H);
  if ((st = hip_status(rx::launch_estimate(la, H2))) != RX_OK) return st;
  if (g) st = hip_status(rx::launch_g(la, H2, g));
  return st;
}

int rx_demod(rx_plan_t plan, const int16_t* iq, const float* H, int64_t n_slots, float* xhat, uint8_t* bits,
             void* workspace, void* hip_stream) {
  (void)workspace;
  int st = check_call(plan, iq, n_slots);
  if (st != RX_OK || n_slots == 0) return st;
  if (!xhat && !bits) return RX_E_INVALID_ARG;
  if (!H || !aligned(H, 8)) return RX_E_INVALID_ARG;
  if (xhat && !aligned(xhat, 8)) return RX_E_INVALID_ARG;
  if ((st = check_device(plan)) != RX_OK) return st;
  const rx::LaunchArgs la = launch_args(plan, iq, n_slots, hip_stream);
  return hip_status(rx::launch_demod(la, plan->p.combiner == RX_COMB_ZF, reinterpret_cast<const float2*>(H),
                                     reinterpret_cast<float2*>(xhat), bits));
}

int rx_process_frame(rx_plan_t plan, const int16_t* iq, int64_t n_slots, float* H, float* xhat, uint8_t* bits,
                     void* workspace, void* hip_stream) {
  int st = check_call(plan, iq, n_slots);
  if (st != RX_OK || n_slots == 0) return st;
  if (!xhat && !bits) return RX_E_INVALID_ARG;
  if (xhat && !aligned(xhat, 8)) return RX_E_INVALID_ARG;
  if (H && !aligned(H, 8)) return RX_E_INVALID_ARG;
  if (!H && (!workspace || !aligned(workspace, 256))) return RX_E_INVALID_ARG;
  if ((st = check_device(plan)) != RX_OK) return st;
  const rx::LaunchArgs la = launch_args(plan, iq, n_slots, hip_stream);
  float2* Hbuf = reinterpret_cast<float2*>(H ? static_cast<void*>(H) : workspace);
  if ((st = hip_status(rx::launch_estimate(la, Hbuf))) != RX_OK) return st;
  return hip_status(rx::launch_demod(la, plan->p.combiner == RX_COMB_ZF, Hbuf, reinterpret_cast<float2*>(xhat), bits));
}

int rx_debug_fft(rx_plan_t plan, const int16_t* iq, int64_t n_slots, float* Y, void* hip_stream) {
  int st = check_call(plan, iq, n_slots);
  if (st != RX_OK || n_slots == 0) return st;
  if (!Y || !aligned(Y, 8)) return RX_E_INVALID_ARG;
  if ((st = check_device(plan)) != RX_OK) return st;
  const rx::LaunchArgs la = launch_args(plan, iq, n_slots, hip_stream);
  return hip_status(rx::launch_fft(la, reinterpret_cast<float2*>(Y)));
}

const char* rx_status_string(int status) {
  switch (status) {
    case RX_OK: return "ok";
    case RX_E_INVALID_ARG: return "invalid argument";
    case RX_E_UNSUPPORTED: return "unsupported parameters";
    case RX_E_HIP: return "HIP runtime error";
    case RX_E_NOMEM: return "out of memory";
    case RX_E_SCRATCH: return "one slot's channel estimate exceeds the library's fixed scratch";
    default: return "unknown status";
  }
}

}  // extern "C"

namespace rx {

// The whole path with the channel estimate kept in a fixed device buffer of
// hbuf_bytes: slots are processed in chunks whose estimates fit it, each
// chunk's estimate written before its demod reads it (one stream, so chunk
// k + 1 overwrites the buffer only after chunk k's demod).  Checks come
// first; nothing is allocated.
int process_frame_in(rx_plan_t plan, const int16_t* iq, int64_t n_slots, float* xhat, uint8_t* bits,
                     float2* hbuf, size_t hbuf_bytes, void* hip_stream) {
  int st = check_call(plan, iq, n_slots);
  if (st != RX_OK || n_slots == 0) return st;
  if (!xhat && !bits) return RX_E_INVALID_ARG;
  if (xhat && !aligned(xhat, 8)) return RX_E_INVALID_ARG;
  const size_t per_slot = (size_t)plan->p.n_ant * plan->p.n_used * sizeof(float2);
  if (per_slot > hbuf_bytes) return RX_E_SCRATCH;
  if ((st = check_device(plan)) != RX_OK) return st;
  if (!hbuf) return RX_E_HIP;
  const int64_t chunk = (int64_t)(hbuf_bytes / per_slot);
  const int64_t slot_iq = (int64_t)plan->p.n_sym * plan->p.n_ant * (plan->p.fft_len + plan->p.cp_len) * 2;
  const int64_t Td = plan->p.n_sym - 1;
  const int64_t row_bytes = (int64_t)plan->p.n_used * plan->p.bits_per_sym / 8;
  for (int64_t s0 = 0; s0 < n_slots; s0 += chunk) {
    const int64_t S = n_slots - s0 < chunk ? n_slots - s0 : chunk;
    const rx::LaunchArgs la = launch_args(plan, iq + s0 * slot_iq, S, hip_stream);
    if ((st = hip_status(rx::launch_estimate(la, hbuf))) != RX_OK) return st;
    float2* x = xhat ? reinterpret_cast<float2*>(xhat) + s0 * Td * plan->p.n_used : nullptr;
    uint8_t* b = bits ? bits + s0 * Td * row_bytes : nullptr;
    if ((st = hip_status(rx::launch_demod(la, plan->p.combiner == RX_COMB_ZF, hbuf, x, b))) != RX_OK) return st;
  }
  return RX_OK;
}

}  // namespace rx
