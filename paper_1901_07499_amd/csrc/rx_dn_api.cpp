// rx_dn_api.cpp -- C ABI of the learned channel-estimate refinement and of
// its training-channel generator (declared in include/rx.h).  Argument checks
// run first and touch no GPU state; kernels live in rx_denoise.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <new>

#include "../../include/rx.h"
#include "rx_launch.h"

static_assert(RX_DN_PARAMS == rx::kParams, "parameter count");

struct rx_dn_s {
  int U = 0;
  int device = -1;
  bool loaded = false;
  float max_corr = 1.0f;     // LS fallback threshold (rx_dn_set_fallback)
  float* theta = nullptr;    // [kParams], the loaded parameters (biases are read from here)
  uint16_t* frag = nullptr;  // [kFragUnits * 8] bf16 operand layout
};

namespace {

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

int check_dn(rx_dn_t dn) {
  if (!dn) return RX_E_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return RX_E_HIP;
  return dev == dn->device ? RX_OK : RX_E_INVALID_ARG;
}

// Workspace carve-up for `rows` rows.
struct Carve {
  int64_t UP = 0;
  size_t off[13] = {0};  // X0 X1 X2 X3 D1 D2 D3 D4 part loss_part M1 M2 M3
  size_t total = 0;
};

Carve carve(int U, int64_t rows) {
  Carve c;
  c.UP = round_up(U, 8);
  const size_t two = (size_t)rows * 2 * c.UP * 2, wide = (size_t)rows * 32 * c.UP * 2;
  const size_t mask = (size_t)rows * c.UP * 4;
  const size_t sizes[13] = {two, wide, wide, wide, wide, wide, wide, two,
                            (size_t)rx::dn_grid(rows) * rx::kParams * 4, (size_t)rx::dn_grid(rows) * 4,
                            mask, mask, mask};
  size_t o = 0;
  for (int i = 0; i < 13; i++) {
    c.off[i] = o;
    o += (size_t)round_up((int64_t)sizes[i], 256);
  }
  c.total = o;
  return c;
}

int check_rows(rx_dn_t dn, int64_t rows) {
  if (rows < 0) return RX_E_INVALID_ARG;
  if (rows > (INT64_C(1) << 40) / (dn->U > 0 ? dn->U : 1)) return RX_E_INVALID_ARG;
  return RX_OK;
}

}  // namespace

extern "C" {

int rx_dn_create(int32_t n_used, rx_dn_t* out) {
  if (!out || n_used < 2 || n_used > 2046) return RX_E_INVALID_ARG;
  rx_dn_s* dn = new (std::nothrow) rx_dn_s;
  if (!dn) return RX_E_NOMEM;
  dn->U = n_used;
  if (hipGetDevice(&dn->device) != hipSuccess) {
    delete dn;
    return RX_E_HIP;
  }
  if (hipMalloc(&dn->theta, sizeof(float) * rx::kParams) != hipSuccess ||
      hipMalloc(&dn->frag, sizeof(uint16_t) * 8 * rx::kFragUnits) != hipSuccess) {
    (void)hipFree(dn->theta);
    (void)hipFree(dn->frag);
    delete dn;
    return RX_E_NOMEM;
  }
  *out = dn;
  return RX_OK;
}

int rx_dn_destroy(rx_dn_t dn) {
  if (!dn) return RX_OK;
  int st = RX_OK;
  if (dn->theta && hipFree(dn->theta) != hipSuccess) st = RX_E_HIP;
  if (dn->frag && hipFree(dn->frag) != hipSuccess) st = RX_E_HIP;
  delete dn;
  return st;
}

int rx_dn_load(rx_dn_t dn, const float* params, void* hip_stream) {
  int st = check_dn(dn);
  if (st != RX_OK) return st;
  if (!params || !aligned(params, 4)) return RX_E_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (hipMemcpyAsync(dn->theta, params, sizeof(float) * rx::kParams, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return RX_E_HIP;
  if (rx::dn_relayout(dn->theta, dn->frag, s) != hipSuccess) return RX_E_HIP;
  dn->loaded = true;
  return RX_OK;
}

int rx_dn_set_fallback(rx_dn_t dn, float max_corr) {
  if (!dn || !(max_corr > 0.f)) return RX_E_INVALID_ARG;  // NaN fails the test too
  dn->max_corr = max_corr;
  return RX_OK;
}

int rx_dn_apply_judged(rx_dn_t dn, const float* H_in, int64_t rows, float* H_out, uint8_t* fell,
                       void* hip_stream) {
  int st = check_dn(dn);
  if (st != RX_OK) return st;
  if ((st = check_rows(dn, rows)) != RX_OK) return st;
  if (rows == 0) return RX_OK;
  if (!H_in || !H_out || !aligned(H_in, 8) || !aligned(H_out, 8)) return RX_E_INVALID_ARG;
  const size_t bytes = (size_t)rows * dn->U * 8;
  const uintptr_t a = (uintptr_t)H_in, b = (uintptr_t)H_out;
  if (a != b && a < b + bytes && b < a + bytes) return RX_E_INVALID_ARG;  // partial overlap
  if (fell) {
    const uintptr_t f = (uintptr_t)fell;
    if ((f < a + bytes && a < f + (size_t)rows) || (f < b + bytes && b < f + (size_t)rows))
      return RX_E_INVALID_ARG;  // flags overlap a row buffer
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (!dn->loaded) {
    // no refinement loaded: every row keeps its LS estimate
    if (a != b && hipMemcpyAsync(H_out, H_in, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) return RX_E_HIP;
    if (fell && rx::fill_u8(fell, 1, rows, s) != hipSuccess) return RX_E_HIP;
    return RX_OK;
  }
  const float mc2 = dn->max_corr * dn->max_corr;
  const hipError_t e = rx::dn_apply(reinterpret_cast<const float2*>(H_in), rows, dn->U, dn->frag, dn->theta,
                                    reinterpret_cast<float2*>(H_out), mc2, fell, s);
  return e == hipSuccess ? RX_OK : RX_E_HIP;
}

int rx_dn_apply(rx_dn_t dn, const float* H_in, int64_t rows, float* H_out, void* hip_stream) {
  return rx_dn_apply_judged(dn, H_in, rows, H_out, nullptr, hip_stream);
}

size_t rx_dn_workspace_bytes(rx_dn_t dn, int64_t rows) {
  if (!dn || rows <= 0 || check_rows(dn, rows) != RX_OK) return 0;
  return carve(dn->U, rows).total;
}

static int train_common(rx_dn_t dn, const float* H_in, const float* H_true, int64_t rows, float* grad, float* loss,
                        const rx::AdamArgs& adam, void* workspace, hipStream_t s) {
  const Carve c = carve(dn->U, rows);
  char* w = static_cast<char*>(workspace);
  rx::DnTrainIo io{};
  io.UP = c.UP;
  io.inv_count = (float)(1.0 / ((double)rows * (double)dn->U));
  uint16_t** bufs[8] = {&io.X0, &io.X1, &io.X2, &io.X3, &io.D1, &io.D2, &io.D3, &io.D4};
  for (int i = 0; i < 8; i++) *bufs[i] = reinterpret_cast<uint16_t*>(w + c.off[i]);
  io.part = reinterpret_cast<float*>(w + c.off[8]);
  io.loss_part = reinterpret_cast<float*>(w + c.off[9]);
  io.M1 = reinterpret_cast<uint32_t*>(w + c.off[10]);
  io.M2 = reinterpret_cast<uint32_t*>(w + c.off[11]);
  io.M3 = reinterpret_cast<uint32_t*>(w + c.off[12]);
  const hipError_t e = rx::dn_train(reinterpret_cast<const float2*>(H_in), reinterpret_cast<const float2*>(H_true),
                                    rows, dn->U, dn->frag, dn->theta, io, grad, loss, adam, s);
  return e == hipSuccess ? RX_OK : RX_E_HIP;
}

static int check_train(rx_dn_t dn, const float* H_in, const float* H_true, int64_t rows, void* workspace) {
  int st = check_dn(dn);
  if (st != RX_OK) return st;
  if ((st = check_rows(dn, rows)) != RX_OK) return st;
  if (rows == 0) return RX_E_INVALID_ARG;  // the loss is a mean over rows
  if (!dn->loaded || !H_in || !H_true || !workspace || !aligned(H_in, 8) || !aligned(H_true, 8) ||
      !aligned(workspace, 256))
    return RX_E_INVALID_ARG;
  return RX_OK;
}

int rx_dn_grad(rx_dn_t dn, const float* H_in, const float* H_true, int64_t rows, float* grad, float* loss,
               void* workspace, void* hip_stream) {
  const int st = check_train(dn, H_in, H_true, rows, workspace);
  if (st != RX_OK) return st;
  if ((grad && !aligned(grad, 4)) || (loss && !aligned(loss, 4))) return RX_E_INVALID_ARG;
  rx::AdamArgs none{};
  return train_common(dn, H_in, H_true, rows, grad, loss, none, workspace, static_cast<hipStream_t>(hip_stream));
}

int rx_dn_train_step(rx_dn_t dn, float* params, float* adam_m, float* adam_v, int64_t step, float lr, float beta1,
                     float beta2, float eps, const float* H_in, const float* H_true, int64_t rows, float* loss,
                     void* workspace, void* hip_stream) {
  int st = check_train(dn, H_in, H_true, rows, workspace);
  if (st != RX_OK) return st;
  if (!params || !adam_m || !adam_v || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f) || !std::isfinite(lr))
    return RX_E_INVALID_ARG;
  if (!aligned(params, 4) || !aligned(adam_m, 4) || !aligned(adam_v, 4) || (loss && !aligned(loss, 4)))
    return RX_E_INVALID_ARG;
  rx::AdamArgs adam{};
  adam.theta = params;
  adam.m = adam_m;
  adam.v = adam_v;
  adam.lr = lr;
  adam.beta1 = beta1;
  adam.beta2 = beta2;
  adam.eps = eps;
  adam.c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
  adam.c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((st = train_common(dn, H_in, H_true, rows, nullptr, loss, adam, workspace, s)) != RX_OK) return st;
  return rx_dn_load(dn, params, hip_stream);
}

int rx_dn_generate(const rx_chan_gen* g, uint64_t seed, int64_t first_row, int64_t rows, float* H_true,
                   float* H_ls, void* hip_stream) {
  if (!g) return RX_E_INVALID_ARG;
  const int N = g->fft_len, U = g->n_used;
  if (N < 64 || N > 2048 || (N & (N - 1)) || U < 2 || U > N - 2 || (U & 1) || g->cp_len < 0 || g->cp_len >= N ||
      g->pilot_spacing < 1 || g->pilot_spacing > U || g->taps_min < 1 || g->taps_max < g->taps_min ||
      g->taps_max > 64 || g->tau_min < 0 || g->tau_max < g->tau_min || !std::isfinite(g->snr_min_db) ||
      !std::isfinite(g->snr_max_db) || !std::isfinite(g->tap_decay_db))
    return RX_E_INVALID_ARG;
  if (rows < 0 || first_row < 0) return RX_E_INVALID_ARG;
  if (rows == 0) return RX_OK;
  if ((!H_true && !H_ls) || (H_true && !aligned(H_true, 8)) || (H_ls && !aligned(H_ls, 8)))
    return RX_E_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return RX_E_HIP;
  rx::GenArgs a{};
  a.N = N;
  a.U = U;
  a.CP = g->cp_len;
  a.ps = g->pilot_spacing;
  a.taps_min = g->taps_min;
  a.taps_max = g->taps_max;
  a.tau_min = g->tau_min;
  a.tau_max = g->tau_max;
  a.snr_min = g->snr_min_db;
  a.snr_max = g->snr_max_db;
  a.decay_db = g->tap_decay_db;
  const hipError_t e = rx::dn_generate(a, seed, first_row, rows, reinterpret_cast<float2*>(H_true),
                                       reinterpret_cast<float2*>(H_ls), static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? RX_OK : RX_E_HIP;
}

}  // extern "C"
