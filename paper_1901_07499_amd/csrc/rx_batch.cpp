// rx_batch.cpp -- batches of frames with mixed shapes (declared in include/rx.h).
//
// A batch is an ordered list of frames (one slot each) whose antenna count,
// FFT length, CP, used subcarriers, QAM order and pilot may all differ.
// Frames with the same FFT length form a class; each class runs a persistent
// estimate kernel followed by a persistent demod kernel that pull (frame,
// item) tiles from device work queues in frame order.  One graph holds a
// reset node (clears the queues, stamps the start time) and one two-node
// branch per class, the branches independent of each other, so one graph
// launch processes the whole batch.  The autotuner times the launch
// configurations of every class (workgroup shapes and the FFT's radix
// schedule, chosen separately for the estimate and demod kernels) on the
// caller's data, first each class alone and then within the whole graph, and
// keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <initializer_list>
#include <new>
#include <vector>

#include "../../include/rx.h"
#include "rx_launch.h"

namespace {

struct BatchClass {
  int N = 0;
  int max_u = 0;
  std::vector<int> frames;  // batch indices, in batch order
  int demod_waves = 4;      // tuned launch configuration
  int est_jobs = 4;
  int dem_sched = 0, est_sched = 0;  // radix schedules of the two kernels' transforms
  int n_est_tiles = 0, n_dem_tiles = 0;
  rx::FrameDesc* d_desc = nullptr;
  int* d_est_map = nullptr;
  int* d_dem_map = nullptr;
  float2* d_tw = nullptr;
  rx::BatchKernel dem, est;
  size_t dem_lds = 0, est_lds = 0;
  int dem_grid = 0, est_grid = 0;
};

}  // namespace

struct rx_batch_s {
  std::vector<rx_params> p;
  std::vector<std::vector<float>> pilots;
  std::vector<int64_t> iq_off, h_off, x_off, b_off;  // n + 1 entries each
  std::vector<int64_t> pf_off;                       // pilot-factor offset of each frame
  std::vector<BatchClass> cls;
  int device = -1;
  int n_cu = 0;
  float2* d_pf = nullptr;
  int* d_queues = nullptr;  // 2 per class: estimate, demod
  int* d_done_count = nullptr;
  unsigned long long* d_done_time = nullptr;
  unsigned long long* d_start = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  rx::BatchIo graph_io{};
};

namespace {

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

void drop_graph(rx_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

void free_all(rx_batch_s* b) {
  drop_graph(b);
  for (auto& c : b->cls) {
    (void)hipFree(c.d_desc);
    (void)hipFree(c.d_est_map);
    (void)hipFree(c.d_dem_map);
    (void)hipFree(c.d_tw);
  }
  (void)hipFree(b->d_pf);
  (void)hipFree(b->d_queues);
  (void)hipFree(b->d_done_count);
  (void)hipFree(b->d_done_time);
  (void)hipFree(b->d_start);
  delete b;
}

// (Re)build the descriptors, tile maps and launch geometry of class c for
// its current configuration.
int configure_class(rx_batch_s* b, BatchClass& c) {
  if (!rx::batch_kernels(c.N, c.max_u, c.demod_waves, c.est_jobs, c.dem_sched, c.est_sched, c.dem, c.est))
    return RX_E_UNSUPPORTED;
  std::vector<rx::FrameDesc> desc;
  std::vector<int> est_map, dem_map;
  // Queue order: frames with more antennas (longer tiles) first, ties in batch
  // order, so the last tiles of a class are short ones.
  std::vector<int> order = c.frames;
  std::stable_sort(order.begin(), order.end(), [b](int x, int y) { return b->p[x].n_ant > b->p[y].n_ant; });
  for (int i : order) {
    const rx_params& p = b->p[i];
    rx::FrameDesc d;
    d.iq_off = b->iq_off[i] / 2;
    d.h_off = b->h_off[i];
    d.x_off = b->x_off[i];
    d.b_off = b->b_off[i];
    d.pf = b->d_pf + b->pf_off[i];
    d.A = p.n_ant;
    d.T = p.n_sym;
    d.CP = p.cp_len;
    d.U = p.n_used;
    d.B = p.bits_per_sym;
    d.index = i;
    d.est_tile0 = (int)est_map.size();
    d.dem_tile0 = (int)dem_map.size();
    const int local = (int)desc.size();
    const int est_tiles = (p.n_ant + c.est.ants_per_tile - 1) / c.est.ants_per_tile;
    for (int t = 0; t < est_tiles; t++) est_map.push_back(local);
    for (int t = 1; t < p.n_sym; t++) dem_map.push_back(local);
    desc.push_back(d);
  }
  c.n_est_tiles = (int)est_map.size();
  c.n_dem_tiles = (int)dem_map.size();
  (void)hipFree(c.d_desc);
  (void)hipFree(c.d_est_map);
  (void)hipFree(c.d_dem_map);
  c.d_desc = nullptr;
  c.d_est_map = c.d_dem_map = nullptr;
  if (hipMalloc(&c.d_desc, sizeof(rx::FrameDesc) * desc.size()) != hipSuccess ||
      hipMalloc(&c.d_est_map, sizeof(int) * est_map.size()) != hipSuccess ||
      hipMalloc(&c.d_dem_map, sizeof(int) * dem_map.size()) != hipSuccess)
    return RX_E_NOMEM;
  if (hipMemcpy(c.d_desc, desc.data(), sizeof(rx::FrameDesc) * desc.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c.d_est_map, est_map.data(), sizeof(int) * est_map.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c.d_dem_map, dem_map.data(), sizeof(int) * dem_map.size(), hipMemcpyHostToDevice) != hipSuccess)
    return RX_E_HIP;
  c.est_lds = c.est.lds_fft;
  c.dem_lds = std::max(c.dem.lds_fft, c.dem.lds_per_u * (size_t)c.max_u);
  for (auto* k : {&c.est, &c.dem}) {
    const size_t lds = k == &c.est ? c.est_lds : c.dem_lds;
    if (lds > 65536 &&
        hipFuncSetAttribute(k->func, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return RX_E_HIP;
  }
  int occ_e = 0, occ_d = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_e, c.est.func, c.est.block, c.est_lds) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_d, c.dem.func, c.dem.block, c.dem_lds) != hipSuccess)
    return RX_E_HIP;
  c.est_grid = std::max(1, std::min(c.n_est_tiles, b->n_cu * std::max(occ_e, 1)));
  c.dem_grid = std::max(1, std::min(c.n_dem_tiles, b->n_cu * std::max(occ_d, 1)));
  return RX_OK;
}

struct KernelArgs {
  // storage for kernel arguments referenced by kernelParams
  const rx::FrameDesc* desc;
  const int* map;
  int n_tiles;
  rx::BatchIo io;
  const float2* tw;
  int* queue;
  int* done_count;
  unsigned long long* done_time;
  void* ptrs[8];
};

void est_args(rx_batch_s* b, const BatchClass& c, size_t ci, const rx::BatchIo& io, KernelArgs& a) {
  a.desc = c.d_desc;
  a.map = c.d_est_map;
  a.n_tiles = c.n_est_tiles;
  a.io = io;
  a.tw = c.d_tw;
  a.queue = b->d_queues + 2 * ci;
  void* p[] = {&a.desc, &a.map, &a.n_tiles, &a.io, &a.tw, &a.queue};
  std::copy(std::begin(p), std::end(p), a.ptrs);
}

void dem_args(rx_batch_s* b, const BatchClass& c, size_t ci, const rx::BatchIo& io, KernelArgs& a) {
  a.desc = c.d_desc;
  a.map = c.d_dem_map;
  a.n_tiles = c.n_dem_tiles;
  a.io = io;
  a.tw = c.d_tw;
  a.queue = b->d_queues + 2 * ci + 1;
  a.done_count = b->d_done_count;
  a.done_time = b->d_done_time;
  void* p[] = {&a.desc, &a.map, &a.n_tiles, &a.io, &a.tw, &a.queue, &a.done_count, &a.done_time};
  std::copy(std::begin(p), std::end(p), a.ptrs);
}

struct ResetArgs {
  int* queues;
  int n_queues;
  int* done_count;
  int n_frames;
  unsigned long long* start;
  void* ptrs[5];
};

void reset_args(rx_batch_s* b, ResetArgs& r) {
  r.queues = b->d_queues;
  r.n_queues = 2 * (int)b->cls.size();
  r.done_count = b->d_done_count;
  r.n_frames = (int)b->p.size();
  r.start = b->d_start;
  void* p[] = {&r.queues, &r.n_queues, &r.done_count, &r.n_frames, &r.start};
  std::copy(std::begin(p), std::end(p), r.ptrs);
}

int build_graph(rx_batch_s* b, const rx::BatchIo& io) {
  drop_graph(b);
  if (hipGraphCreate(&b->graph, 0) != hipSuccess) return RX_E_HIP;
  ResetArgs ra;
  reset_args(b, ra);
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(rx::batch_reset_func());
  kp.gridDim = dim3(1);
  kp.blockDim = dim3(256);
  kp.sharedMemBytes = 0;
  kp.kernelParams = ra.ptrs;
  kp.extra = nullptr;
  hipGraphNode_t reset;
  if (hipGraphAddKernelNode(&reset, b->graph, nullptr, 0, &kp) != hipSuccess) return RX_E_HIP;
  for (size_t ci = 0; ci < b->cls.size(); ci++) {
    const BatchClass& c = b->cls[ci];
    KernelArgs ea, da;
    est_args(b, c, ci, io, ea);
    dem_args(b, c, ci, io, da);
    hipKernelNodeParams ep{};
    ep.func = const_cast<void*>(c.est.func);
    ep.gridDim = dim3(c.est_grid);
    ep.blockDim = dim3(c.est.block);
    ep.sharedMemBytes = (unsigned)c.est_lds;
    ep.kernelParams = ea.ptrs;
    hipGraphNode_t en, dn;
    if (hipGraphAddKernelNode(&en, b->graph, &reset, 1, &ep) != hipSuccess) return RX_E_HIP;
    hipKernelNodeParams dp{};
    dp.func = const_cast<void*>(c.dem.func);
    dp.gridDim = dim3(c.dem_grid);
    dp.blockDim = dim3(c.dem.block);
    dp.sharedMemBytes = (unsigned)c.dem_lds;
    dp.kernelParams = da.ptrs;
    if (hipGraphAddKernelNode(&dn, b->graph, &en, 1, &dp) != hipSuccess) return RX_E_HIP;
  }
  if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) return RX_E_HIP;
  b->graph_io = io;
  return RX_OK;
}

bool same_io(const rx::BatchIo& a, const rx::BatchIo& b) {
  return a.iq == b.iq && a.H == b.H && a.xhat == b.xhat && a.bits == b.bits;
}

int check_io(rx_batch_t b, const int16_t* iq, float* H, float* xhat, uint8_t* bits, void* workspace,
             rx::BatchIo& io) {
  if (!b) return RX_E_INVALID_ARG;
  if (!iq || !aligned(iq, 4)) return RX_E_INVALID_ARG;
  if (!xhat && !bits) return RX_E_INVALID_ARG;
  if (xhat && !aligned(xhat, 8)) return RX_E_INVALID_ARG;
  if (H && !aligned(H, 8)) return RX_E_INVALID_ARG;
  if (!H && (!workspace || !aligned(workspace, 256))) return RX_E_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return RX_E_HIP;
  if (dev != b->device) return RX_E_INVALID_ARG;
  io.iq = reinterpret_cast<const uint32_t*>(iq);
  io.H = reinterpret_cast<float2*>(H ? static_cast<void*>(H) : workspace);
  io.xhat = reinterpret_cast<float2*>(xhat);
  io.bits = bits;
  return RX_OK;
}

// Direct launches of class ci (reset first), timing each kernel.
int run_class_timed(rx_batch_s* b, size_t ci, const rx::BatchIo& io, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                    hipEvent_t e2, float* est_ms, float* dem_ms) {
  const BatchClass& c = b->cls[ci];
  ResetArgs ra;
  reset_args(b, ra);
  if (hipLaunchKernel(rx::batch_reset_func(), dim3(1), dim3(256), ra.ptrs, 0, st) != hipSuccess) return RX_E_HIP;
  KernelArgs ea, da;
  est_args(b, c, ci, io, ea);
  dem_args(b, c, ci, io, da);
  if (hipEventRecord(e0, st) != hipSuccess) return RX_E_HIP;
  if (hipLaunchKernel(c.est.func, dim3(c.est_grid), dim3(c.est.block), ea.ptrs, c.est_lds, st) != hipSuccess)
    return RX_E_HIP;
  if (hipEventRecord(e1, st) != hipSuccess) return RX_E_HIP;
  if (hipLaunchKernel(c.dem.func, dim3(c.dem_grid), dim3(c.dem.block), da.ptrs, c.dem_lds, st) != hipSuccess)
    return RX_E_HIP;
  if (hipEventRecord(e2, st) != hipSuccess) return RX_E_HIP;
  if (hipEventSynchronize(e2) != hipSuccess) return RX_E_HIP;
  if (hipEventElapsedTime(est_ms, e0, e1) != hipSuccess || hipEventElapsedTime(dem_ms, e1, e2) != hipSuccess)
    return RX_E_HIP;
  return RX_OK;
}

}  // namespace

extern "C" {

int rx_batch_create(const rx_params* frames, int32_t n_frames, rx_batch_t* out) {
  if (!out || !frames || n_frames < 1 || n_frames > 65536) return RX_E_INVALID_ARG;
  for (int i = 0; i < n_frames; i++) {
    const int st = rx_params_check(&frames[i]);
    if (st != RX_OK) return st;
    if (frames[i].combiner != RX_COMB_MRC) return RX_E_UNSUPPORTED;
    if (frames[i].pilot_spacing > 1 || frames[i].fft_mode != 0) return RX_E_UNSUPPORTED;
  }
  rx_batch_s* b = new (std::nothrow) rx_batch_s;
  if (!b) return RX_E_NOMEM;
  b->p.assign(frames, frames + n_frames);
  b->iq_off.assign(n_frames + 1, 0);
  b->h_off.assign(n_frames + 1, 0);
  b->x_off.assign(n_frames + 1, 0);
  b->b_off.assign(n_frames + 1, 0);
  std::vector<float2> pf;
  for (int i = 0; i < n_frames; i++) {
    rx_params& p = b->p[i];
    b->pilots.emplace_back(p.pilot, p.pilot + 2 * p.n_used);
    const int64_t A = p.n_ant, N = p.fft_len, CP = p.cp_len, U = p.n_used, T = p.n_sym;
    b->iq_off[i + 1] = b->iq_off[i] + T * A * (N + CP) * 2;
    b->h_off[i + 1] = b->h_off[i] + A * U;
    b->x_off[i + 1] = b->x_off[i] + (T - 1) * U;
    b->b_off[i + 1] = b->b_off[i] + (T - 1) * U * p.bits_per_sym / 8;
    b->pf_off.push_back((int64_t)pf.size());
    for (int d = 0; d < p.n_used; d++) {
      const double re = p.pilot[2 * d], im = p.pilot[2 * d + 1];
      const double m2 = re * re + im * im;
      pf.push_back(make_float2((float)(re / m2), (float)(-im / m2)));
    }
  }
  for (size_t i = 0; i < b->p.size(); i++) b->p[i].pilot = b->pilots[i].data();
  if (hipGetDevice(&b->device) != hipSuccess ||
      hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) {
    delete b;
    return RX_E_HIP;
  }
  // classes by FFT length, in order of first appearance
  for (int i = 0; i < n_frames; i++) {
    const int N = b->p[i].fft_len;
    auto it = std::find_if(b->cls.begin(), b->cls.end(), [N](const BatchClass& c) { return c.N == N; });
    if (it == b->cls.end()) {
      b->cls.emplace_back();
      it = b->cls.end() - 1;
      it->N = N;
    }
    it->frames.push_back(i);
    it->max_u = std::max(it->max_u, b->p[i].n_used);
  }
  int st = RX_OK;
  if (hipMalloc(&b->d_pf, sizeof(float2) * pf.size()) != hipSuccess ||
      hipMalloc(&b->d_queues, sizeof(int) * 2 * b->cls.size()) != hipSuccess ||
      hipMalloc(&b->d_done_count, sizeof(int) * n_frames) != hipSuccess ||
      hipMalloc(&b->d_done_time, sizeof(unsigned long long) * n_frames) != hipSuccess ||
      hipMalloc(&b->d_start, sizeof(unsigned long long)) != hipSuccess)
    st = RX_E_NOMEM;
  if (st == RX_OK && hipMemcpy(b->d_pf, pf.data(), sizeof(float2) * pf.size(), hipMemcpyHostToDevice) != hipSuccess)
    st = RX_E_HIP;
  const double two_pi = 6.283185307179586476925286766559;
  for (auto& c : b->cls) {
    if (st != RX_OK) break;
    std::vector<float2> tw(c.N);
    for (int k = 0; k < c.N; k++) {
      const double ang = -two_pi * (double)k / (double)c.N;
      tw[k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    if (hipMalloc(&c.d_tw, sizeof(float2) * c.N) != hipSuccess) {
      st = RX_E_NOMEM;
      break;
    }
    if (hipMemcpy(c.d_tw, tw.data(), sizeof(float2) * c.N, hipMemcpyHostToDevice) != hipSuccess) {
      st = RX_E_HIP;
      break;
    }
    st = configure_class(b, c);
  }
  if (st != RX_OK) {
    free_all(b);
    return st;
  }
  *out = b;
  return RX_OK;
}

int rx_batch_destroy(rx_batch_t b) {
  if (b) free_all(b);
  return RX_OK;
}

int rx_batch_layout(rx_batch_t b, int64_t* iq_off, int64_t* h_off, int64_t* x_off, int64_t* b_off) {
  if (!b) return RX_E_INVALID_ARG;
  const size_t n = b->p.size() + 1;
  if (iq_off) std::copy(b->iq_off.begin(), b->iq_off.begin() + n, iq_off);
  if (h_off) std::copy(b->h_off.begin(), b->h_off.begin() + n, h_off);
  if (x_off) std::copy(b->x_off.begin(), b->x_off.begin() + n, x_off);
  if (b_off) std::copy(b->b_off.begin(), b->b_off.begin() + n, b_off);
  return RX_OK;
}

size_t rx_batch_workspace_bytes(rx_batch_t b) {
  return b ? (size_t)b->h_off.back() * sizeof(float2) : 0;
}

int rx_batch_process(rx_batch_t b, const int16_t* iq, float* H, float* xhat, uint8_t* bits, void* workspace,
                     void* hip_stream) {
  rx::BatchIo io;
  int st = check_io(b, iq, H, xhat, bits, workspace, io);
  if (st != RX_OK) return st;
  if (!b->exec || !same_io(io, b->graph_io)) {
    if ((st = build_graph(b, io)) != RX_OK) return st;
  }
  return hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(hip_stream)) == hipSuccess ? RX_OK : RX_E_HIP;
}

int rx_batch_autotune(rx_batch_t b, const int16_t* iq, float* H, float* xhat, uint8_t* bits, void* workspace,
                      int32_t reps, void* hip_stream) {
  rx::BatchIo io;
  int st = check_io(b, iq, H, xhat, bits, workspace, io);
  if (st != RX_OK) return st;
  if (reps < 1) return RX_E_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  hipEvent_t e0, e1, e2;
  if (hipEventCreate(&e0) != hipSuccess) return RX_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return RX_E_HIP;
  }
  if (hipEventCreate(&e2) != hipSuccess) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return RX_E_HIP;
  }
  // Warm-up: a few launches of the whole batch graph, so the first
  // configurations are not timed on an idle GPU whose clocks are still low.
  if ((st = build_graph(b, io)) == RX_OK) {
    for (int r = 0; r < 16 && st == RX_OK; r++)
      if (hipGraphLaunch(b->exec, s) != hipSuccess) st = RX_E_HIP;
    if (st == RX_OK && hipStreamSynchronize(s) != hipSuccess) st = RX_E_HIP;
  }
  drop_graph(b);
  // Pass 1: each class alone, its estimate and demod kernels timed separately
  // (minimum over the timed runs: robust to interference); the estimate's
  // jobs and schedule and the demod's workgroup size and schedule are chosen
  // independently.
  std::vector<float> alone(b->cls.size(), 0.f);
  for (size_t ci = 0; ci < b->cls.size() && st == RX_OK; ci++) {
    BatchClass& c = b->cls[ci];
    const int n_sched = rx::fft_schedule_count(c.N);
    float best_e = 1e30f, best_d = 1e30f;
    int best_w = c.demod_waves, best_j = c.est_jobs, best_sd = c.dem_sched, best_se = c.est_sched;
    for (int sc = 0; sc < n_sched && st == RX_OK; sc++) {
      for (int w : {2, 4, 8}) {
        for (int j : {2, 4, 8}) {
          c.demod_waves = w;
          c.est_jobs = j;
          c.dem_sched = c.est_sched = sc;
          if ((st = configure_class(b, c)) != RX_OK) break;
          float me = 1e30f, md = 1e30f;
          for (int r = 0; r <= reps && st == RX_OK; r++) {  // first run is a warm-up
            float te = 0.f, td = 0.f;
            st = run_class_timed(b, ci, io, s, e0, e1, e2, &te, &td);
            if (r > 0) {
              me = std::min(me, te);
              md = std::min(md, td);
            }
          }
          if (st != RX_OK) break;
          if (me < best_e) {
            best_e = me;
            best_j = j;
            best_se = sc;
          }
          if (md < best_d) {
            best_d = md;
            best_w = w;
            best_sd = sc;
          }
        }
        if (st != RX_OK) break;
      }
    }
    c.demod_waves = best_w;
    c.est_jobs = best_j;
    c.dem_sched = best_sd;
    c.est_sched = best_se;
    alone[ci] = best_e + best_d;
    if (st == RX_OK) st = configure_class(b, c);
  }
  // Pass 2: the classes share the GPU inside one graph launch, so a class's
  // best configuration alone need not be best in the batch.  Class by class,
  // longest first, configurations are timed within the whole graph (the other
  // classes as chosen so far): every workgroup shape with the class's
  // schedules, then every pair of schedules with the best shape.  The
  // incumbent (timed first) is only replaced by a configuration more than 1 %
  // faster, so timing noise does not flip choices that do not matter.
  std::vector<size_t> order(b->cls.size());
  for (size_t i = 0; i < order.size(); i++) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return alone[x] > alone[y]; });
  struct Cfg {
    int w, j, sd, se;
    bool operator==(const Cfg& o) const { return w == o.w && j == o.j && sd == o.sd && se == o.se; }
  };
  auto time_graph = [&](BatchClass& c, const Cfg& g, float* ms) {
    c.demod_waves = g.w;
    c.est_jobs = g.j;
    c.dem_sched = g.sd;
    c.est_sched = g.se;
    int rc = configure_class(b, c);
    if (rc == RX_OK) rc = build_graph(b, io);
    float m = 1e30f;
    for (int r = 0; r <= reps && rc == RX_OK; r++) {  // first run is a warm-up
      float t = 0.f;
      if (hipEventRecord(e0, s) != hipSuccess || hipGraphLaunch(b->exec, s) != hipSuccess ||
          hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&t, e0, e1) != hipSuccess)
        rc = RX_E_HIP;
      else if (r > 0)
        m = std::min(m, t);
    }
    *ms = m;
    return rc;
  };
  for (size_t oi = 0; oi < order.size() && st == RX_OK && b->cls.size() > 1; oi++) {
    BatchClass& c = b->cls[order[oi]];
    const int n_sched = rx::fft_schedule_count(c.N);
    const Cfg inc{c.demod_waves, c.est_jobs, c.dem_sched, c.est_sched};
    Cfg best_cfg = inc;
    float best = 1e30f;
    if ((st = time_graph(c, inc, &best)) != RX_OK) break;
    auto consider = [&](const Cfg& g) {
      if (st != RX_OK || g == best_cfg || g == inc) return;
      float m = 0.f;
      if ((st = time_graph(c, g, &m)) == RX_OK && m < 0.99f * best) {
        best = m;
        best_cfg = g;
      }
    };
    for (int w : {2, 4, 8})
      for (int j : {2, 4, 8}) consider(Cfg{w, j, inc.sd, inc.se});
    const Cfg shape = best_cfg;
    for (int sd = 0; sd < n_sched; sd++)
      for (int se = 0; se < n_sched; se++) consider(Cfg{shape.w, shape.j, sd, se});
    c.demod_waves = best_cfg.w;
    c.est_jobs = best_cfg.j;
    c.dem_sched = best_cfg.sd;
    c.est_sched = best_cfg.se;
    if (st == RX_OK) st = configure_class(b, c);
  }
  drop_graph(b);  // rebuilt for the chosen configurations by the next rx_batch_process
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  return st;
}

int rx_batch_config(rx_batch_t b, int32_t fft_len, int32_t* demod_waves, int32_t* est_jobs) {
  if (!b) return RX_E_INVALID_ARG;
  for (const auto& c : b->cls)
    if (c.N == fft_len) {
      if (demod_waves) *demod_waves = c.demod_waves;
      if (est_jobs) *est_jobs = c.est_jobs;
      return RX_OK;
    }
  return RX_E_INVALID_ARG;
}

int rx_batch_schedules(rx_batch_t b, int32_t fft_len, int32_t* dem_sched, int32_t* est_sched) {
  if (!b) return RX_E_INVALID_ARG;
  for (const auto& c : b->cls)
    if (c.N == fft_len) {
      if (dem_sched) *dem_sched = c.dem_sched;
      if (est_sched) *est_sched = c.est_sched;
      return RX_OK;
    }
  return RX_E_INVALID_ARG;
}

int rx_batch_set_config(rx_batch_t b, int32_t fft_len, int32_t demod_waves, int32_t est_jobs, int32_t dem_sched,
                        int32_t est_sched) {
  if (!b) return RX_E_INVALID_ARG;
  auto it = std::find_if(b->cls.begin(), b->cls.end(), [fft_len](const BatchClass& c) { return c.N == fft_len; });
  if (it == b->cls.end()) return RX_E_INVALID_ARG;
  const auto in = [](int v, std::initializer_list<int> ok) { return std::find(ok.begin(), ok.end(), v) != ok.end(); };
  const int n_sched = rx::fft_schedule_count(fft_len);
  if (!in(demod_waves, {2, 4, 8}) || !in(est_jobs, {2, 4, 8}) || dem_sched < 0 || dem_sched >= n_sched ||
      est_sched < 0 || est_sched >= n_sched)
    return RX_E_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return RX_E_HIP;
  if (dev != b->device) return RX_E_INVALID_ARG;
  BatchClass& c = *it;
  const int old[4] = {c.demod_waves, c.est_jobs, c.dem_sched, c.est_sched};
  c.demod_waves = demod_waves;
  c.est_jobs = est_jobs;
  c.dem_sched = dem_sched;
  c.est_sched = est_sched;
  drop_graph(b);
  int st = configure_class(b, c);
  if (st != RX_OK) {
    c.demod_waves = old[0];
    c.est_jobs = old[1];
    c.dem_sched = old[2];
    c.est_sched = old[3];
    (void)configure_class(b, c);
  }
  return st;
}

int rx_fft_radices(int32_t fft_len, int32_t sched, int32_t* radices) {
  if (!radices) return RX_E_INVALID_ARG;
  const int n = rx::fft_schedule_count(fft_len);
  if (n == 0 || sched < 0 || sched >= n) return RX_E_UNSUPPORTED;
  int r[3];
  rx::fft_schedule_radices(fft_len, sched, r);
  for (int i = 0; i < 3; i++) radices[i] = r[i];
  return RX_OK;
}

int rx_batch_frame_latency(rx_batch_t b, double* ms, void* hip_stream) {
  if (!b || !ms) return RX_E_INVALID_ARG;
  if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(hip_stream)) != hipSuccess) return RX_E_HIP;
  std::vector<unsigned long long> done(b->p.size());
  unsigned long long start = 0;
  if (hipMemcpy(done.data(), b->d_done_time, sizeof(unsigned long long) * done.size(), hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(&start, b->d_start, sizeof(start), hipMemcpyDeviceToHost) != hipSuccess)
    return RX_E_HIP;
  for (size_t i = 0; i < done.size(); i++) ms[i] = (double)(done[i] - start) * 1e-5;  // 100 MHz clock
  return RX_OK;
}

}  // extern "C"
