// rx_sync_api.cpp -- C ABI of PN frame synchronisation and slot extraction
// (declared in include/rx.h).  Argument checks run first and touch no GPU
// state; kernels live in rx_sync.hip.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/rx.h"
#include "rx_launch.h"

static_assert(RX_SYNC_MAX_PN == rx::kMaxPn, "PN length limit");

namespace {

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

int check_streams(const int16_t* raw, int32_t n_ant, int64_t n_samples, int64_t stride) {
  if (!raw || !aligned(raw, 4)) return RX_E_INVALID_ARG;
  if (n_ant < 1 || n_ant > 4096 || n_samples < 0 || stride < n_samples || stride < 1) return RX_E_INVALID_ARG;
  if (stride > (INT64_C(1) << 40) / n_ant) return RX_E_INVALID_ARG;
  return RX_OK;
}

}  // namespace

extern "C" {

size_t rx_sync_workspace_bytes(int32_t n_ant, int64_t n_search) {
  if (n_search < 1 || n_ant < 1 || n_ant > 4096 || n_search > (INT64_C(1) << 36)) return 0;
  return rx::sync_workspace(n_ant, n_search);
}

int rx_sync_find(const int16_t* raw, int32_t n_ant, int64_t n_samples, int64_t stride, const int8_t* pn,
                 int32_t pn_len, int64_t n_search, uint64_t* metric, int64_t* offset, uint64_t* peak,
                 void* workspace, void* hip_stream) {
  int st = check_streams(raw, n_ant, n_samples, stride);
  if (st != RX_OK) return st;
  if (!pn || pn_len < 1 || pn_len > RX_SYNC_MAX_PN) return RX_E_INVALID_ARG;
  if (n_search < 1 || n_search > (INT64_C(1) << 36)) return RX_E_INVALID_ARG;
  if (!offset || !aligned(offset, 8) || (metric && !aligned(metric, 8)) || (peak && !aligned(peak, 8)))
    return RX_E_INVALID_ARG;
  if (!workspace || !aligned(workspace, 256)) return RX_E_INVALID_ARG;
  rx::SyncChips ch{};
  ch.L = pn_len;
  for (int m = 0; m < pn_len; m++) {
    if (pn[m] < -1 || pn[m] > 1) return RX_E_INVALID_ARG;
    ch.c[m] = pn[m];
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return RX_E_HIP;
  const hipError_t e = rx::sync_find(reinterpret_cast<const uint32_t*>(raw), n_ant, n_samples, stride, ch, n_search,
                                     metric, offset, peak, workspace, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? RX_OK : RX_E_HIP;
}

int rx_sync_extract(const int16_t* raw, int32_t n_ant, int64_t n_samples, int64_t stride, const int64_t* start,
                    int64_t start_add, int32_t sym_len, int32_t n_sym, int64_t n_slots, int16_t* iq,
                    void* hip_stream) {
  int st = check_streams(raw, n_ant, n_samples, stride);
  if (st != RX_OK) return st;
  if (sym_len < 1 || n_sym < 1 || n_slots < 0 || (start && !aligned(start, 8))) return RX_E_INVALID_ARG;
  if (n_slots == 0) return RX_OK;
  if (n_slots > (INT64_C(1) << 40) / ((int64_t)n_sym * n_ant * sym_len)) return RX_E_INVALID_ARG;
  if (!iq || !aligned(iq, 4)) return RX_E_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return RX_E_HIP;
  const hipError_t e = rx::sync_extract(reinterpret_cast<const uint32_t*>(raw), n_ant, n_samples, stride, start,
                                        start_add, sym_len, n_sym, n_slots, reinterpret_cast<uint32_t*>(iq),
                                        static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? RX_OK : RX_E_HIP;
}

}  // extern "C"
