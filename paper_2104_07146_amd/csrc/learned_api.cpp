// C ABI of the learned starting point: variogram features of fields and the
// start-proposal network (creation, normalisation, forward pass, gradient,
// Adam training step, proposal). The arithmetic runs in learned.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hmle.h"
#include "common.hpp"
#include "learned.hpp"

namespace hmle {
void set_last_error(const std::string& msg);
}

using namespace hmle;

struct hmle_mlp_s {
  hipStream_t stream = nullptr;
  MlpBuffers b{};
  void* state = nullptr;    // params, m, v, grad, norm, loss (one allocation)
  void* act = nullptr;      // activations for b.cap rows
  int64_t step = 0;         // Adam steps taken
  float norm_host[N_NORM];
  std::string err;
  ~hmle_mlp_s() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (state) (void)hipFree(state);
    if (act) (void)hipFree(act);
  }
};

namespace {

hmle_status mfail(hmle_mlp net, hmle_status code, const std::string& msg) {
  if (net) net->err = msg;
  set_last_error(msg);
  return code;
}

#define HIP_OR_FAIL(net, expr)                                                                       \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess)                                                                            \
      return mfail(net, e_ == hipErrorOutOfMemory ? HMLE_E_NOMEM : HMLE_E_HIP,                       \
                   std::string(#expr) + ": " + hipGetErrorString(e_));                               \
  } while (0)

constexpr int64_t ACT_PER_ROW = N_FEAT + 3 * N_HID + N_OUT + N_OUT + 2 * N_HID;

hmle_status ensure_rows(hmle_mlp net, int32_t rows) {
  if (rows <= net->b.cap) return HMLE_OK;
  const int32_t cap = std::max<int32_t>(1024, (rows + 1023) / 1024 * 1024);
  HIP_OR_FAIL(net, hipStreamSynchronize(net->stream));
  if (net->act) HIP_OR_FAIL(net, hipFree(net->act));
  net->act = nullptr;
  net->b.cap = 0;
  HIP_OR_FAIL(net, hipMalloc(&net->act, (size_t)cap * ACT_PER_ROW * sizeof(float)));
  float* a = static_cast<float*>(net->act);
  net->b.X0 = a; a += (int64_t)cap * N_FEAT;
  net->b.H1 = a; a += (int64_t)cap * N_HID;
  net->b.H2 = a; a += (int64_t)cap * N_HID;
  net->b.H3 = a; a += (int64_t)cap * N_HID;
  net->b.Y = a; a += (int64_t)cap * N_OUT;
  net->b.G4 = a; a += (int64_t)cap * N_OUT;
  net->b.Ga = a; a += (int64_t)cap * N_HID;
  net->b.Gb = a;
  net->b.cap = cap;
  return HMLE_OK;
}

// Host check of a device row-index list against the dataset size.
hmle_status check_idx(hmle_mlp net, const int32_t* idx, int32_t rows, int64_t total) {
  if (!idx) return rows <= total ? HMLE_OK : mfail(net, HMLE_E_INVALID, "rows exceed the dataset");
  std::vector<int32_t> h(rows);
  HIP_OR_FAIL(net, hipMemcpyAsync(h.data(), idx, rows * sizeof(int32_t), hipMemcpyDeviceToHost, net->stream));
  HIP_OR_FAIL(net, hipStreamSynchronize(net->stream));
  for (int32_t v : h)
    if (v < 0 || v >= total) return mfail(net, HMLE_E_INVALID, "row index out of range");
  return HMLE_OK;
}

hmle_status grad_pass(hmle_mlp net, const float* x, const float* lt, const int32_t* idx, int32_t rows, int64_t total) {
  if (!x || !lt) return mfail(net, HMLE_E_INVALID, "x and lt must not be NULL");
  if (rows < 1 || rows > (1 << 20)) return mfail(net, HMLE_E_INVALID, "rows must be in [1, 2^20]");
  hmle_status s = check_idx(net, idx, rows, total);
  if (s != HMLE_OK) return s;
  s = ensure_rows(net, rows);
  if (s != HMLE_OK) return s;
  launch_mlp_forward(net->b, x, idx, rows, net->stream);
  launch_mlp_backward(net->b, lt, idx, rows, net->stream);
  HIP_OR_FAIL(net, hmle::launch_status());
  return HMLE_OK;
}

hmle_status read_loss(hmle_mlp net, float* loss) {
  if (!loss) return HMLE_OK;
  HIP_OR_FAIL(net, hipMemcpyAsync(loss, net->b.loss, sizeof(float), hipMemcpyDeviceToHost, net->stream));
  HIP_OR_FAIL(net, hipStreamSynchronize(net->stream));
  return HMLE_OK;
}

// Argument checks shared by the two variogram calls; *max_tiles receives the
// pair-tile count of the largest field.
hmle_status vario_check(const double* pts, const double* z, const int64_t* offsets, int32_t count, int32_t dim,
                        const int32_t* sel, const int64_t* sel_offsets, const float* out, int32_t* max_tiles) {
  if (!pts || !z || !offsets || !out) return mfail(nullptr, HMLE_E_INVALID, "NULL argument");
  if (count < 1) return mfail(nullptr, HMLE_E_INVALID, "count must be >= 1");
  if (dim != 2 && dim != 3) return mfail(nullptr, HMLE_E_INVALID, "dim must be 2 or 3");
  if (sel && !sel_offsets) return mfail(nullptr, HMLE_E_INVALID, "sel needs sel_offsets");
  if (offsets[0] != 0 || (sel && sel_offsets[0] != 0)) return mfail(nullptr, HMLE_E_INVALID, "offsets must start at 0");
  int32_t mt = 1;
  for (int32_t q = 0; q < count; ++q) {
    const int64_t n = offsets[q + 1] - offsets[q];
    const int64_t m = sel ? sel_offsets[q + 1] - sel_offsets[q] : n;
    if (n < 1 || m < 1) return mfail(nullptr, HMLE_E_INVALID, "every field needs at least one point");
    if (m > 65536) return mfail(nullptr, HMLE_E_INVALID, "at most 65536 points per field");
    mt = std::max(mt, variogram_tiles(m));
  }
  if (sel) {   // every selected index must name a point of its own field
    std::vector<int32_t> hsel(sel_offsets[count]);
    if (hipMemcpy(hsel.data(), sel, hsel.size() * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
      return mfail(nullptr, HMLE_E_HIP, "cannot read sel");
    for (int32_t q = 0; q < count; ++q)
      for (int64_t k = sel_offsets[q]; k < sel_offsets[q + 1]; ++k)
        if (hsel[k] < 0 || hsel[k] >= offsets[q + 1] - offsets[q])
          return mfail(nullptr, HMLE_E_INVALID, "sel index out of range of its field");
  }
  *max_tiles = mt;
  return HMLE_OK;
}

// Workspace of one variogram call: the two offset arrays (256-byte aligned
// slots) and the per-tile partial sums.
constexpr size_t vario_slot(int32_t count) { return ((size_t)(count + 1) * sizeof(int64_t) + 255) / 256 * 256; }
size_t vario_bytes(int32_t count, int32_t max_tiles, bool with_sel) {
  return vario_slot(count) * (with_sel ? 2 : 1) + (size_t)count * max_tiles * 64 * sizeof(double);
}

// Offsets to the workspace, the two kernels, and a synchronisation (so the
// workspace may be reused as soon as the call returns). Every partial sum the
// final kernel reads is written first by the tile kernel of the same call, so
// nothing needs clearing.
hmle_status vario_run(const double* pts, const double* z, const int64_t* offsets, int32_t count, int32_t dim,
                      const int32_t* sel, const int64_t* sel_offsets, int32_t max_tiles, void* ws, hipStream_t st,
                      float* out) {
  char* base = static_cast<char*>(ws);
  int64_t* d_offs = reinterpret_cast<int64_t*>(base);
  int64_t* d_soffs = sel ? reinterpret_cast<int64_t*>(base + vario_slot(count)) : nullptr;
  double* d_part = reinterpret_cast<double*>(base + vario_slot(count) * (sel ? 2 : 1));
  hipError_t e = hipMemcpyAsync(d_offs, offsets, (count + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && sel)
    e = hipMemcpyAsync(d_soffs, sel_offsets, (count + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    launch_variogram(pts, z, d_offs, sel, d_soffs, count, dim, max_tiles, d_part, out, st);
    e = hmle::launch_status();
  }
  const hipError_t es = hipStreamSynchronize(st);
  if (e == hipSuccess) e = es;
  if (e != hipSuccess)
    return mfail(nullptr, e == hipErrorOutOfMemory ? HMLE_E_NOMEM : HMLE_E_HIP, hipGetErrorString(e));
  return HMLE_OK;
}

}  // namespace

extern "C" {

int64_t hmle_mlp_param_count(void) { return N_PARAMS; }

hmle_status hmle_variogram(const double* pts, const double* z, const int64_t* offsets, int32_t count, int32_t dim,
                           const int32_t* sel, const int64_t* sel_offsets, void* hip_stream, float* out) {
  int32_t max_tiles = 0;
  const hmle_status vs = vario_check(pts, z, offsets, count, dim, sel, sel_offsets, out, &max_tiles);
  if (vs != HMLE_OK) return vs;
  // a workspace kept per device between calls (grown when a call needs more),
  // so repeated calls do not allocate; the lock spans the call, which ends
  // with a stream synchronisation, so the workspace is free again afterwards
  static std::mutex mu;
  static std::map<int, std::pair<void*, size_t>> cache;
  std::lock_guard<std::mutex> lock(mu);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return mfail(nullptr, HMLE_E_HIP, hipGetErrorString(e));
  const size_t need = vario_bytes(count, max_tiles, sel != nullptr);
  auto& slot = cache[dev];
  if (slot.second < need) {
    if (slot.first) (void)hipFree(slot.first);
    slot = {nullptr, 0};
    e = hipMalloc(&slot.first, need);
    if (e != hipSuccess) return mfail(nullptr, e == hipErrorOutOfMemory ? HMLE_E_NOMEM : HMLE_E_HIP, hipGetErrorString(e));
    slot.second = need;
  }
  return vario_run(pts, z, offsets, count, dim, sel, sel_offsets, max_tiles, slot.first,
                   static_cast<hipStream_t>(hip_stream), out);
}

hmle_status hmle_variogram_noalloc(const double* pts, const double* z, const int64_t* offsets, int32_t count,
                                   int32_t dim, const int32_t* sel, const int64_t* sel_offsets, void* hip_stream,
                                   float* out) {
  int32_t max_tiles = 0;
  const hmle_status vs = vario_check(pts, z, offsets, count, dim, sel, sel_offsets, out, &max_tiles);
  if (vs != HMLE_OK) return vs;
  const size_t need = vario_bytes(count, max_tiles, sel != nullptr);
  if (need > VARIO_SCRATCH_BYTES)
    return mfail(nullptr, HMLE_E_INVALID,
                 "hmle_variogram_noalloc: the fields need " + std::to_string(need) + " bytes of workspace, more than its " +
                     std::to_string(VARIO_SCRATCH_BYTES) + "-byte fixed workspace (use fewer fields per call)");
  void* ws = nullptr;
  const hipError_t e = variogram_scratch(&ws);
  if (e != hipSuccess) return mfail(nullptr, HMLE_E_HIP, std::string("scratch address: ") + hipGetErrorString(e));
  return vario_run(pts, z, offsets, count, dim, sel, sel_offsets, max_tiles, ws, static_cast<hipStream_t>(hip_stream),
                   out);
}

hmle_status hmle_mlp_create(const float* params, void* hip_stream, hmle_mlp* out) {
  if (!params || !out) return mfail(nullptr, HMLE_E_INVALID, "NULL argument");
  *out = nullptr;
  auto* net = new hmle_mlp_s();
  net->stream = static_cast<hipStream_t>(hip_stream);
  const size_t n = (size_t)4 * N_PARAMS + N_NORM + 4;
  hipError_t e = hipMalloc(&net->state, n * sizeof(float));
  if (e == hipSuccess) {
    float* s = static_cast<float*>(net->state);
    net->b.params = s;
    net->b.m = s + N_PARAMS;
    net->b.v = s + 2 * N_PARAMS;
    net->b.grad = s + 3 * N_PARAMS;
    net->b.norm = s + 4 * N_PARAMS;
    net->b.loss = net->b.norm + N_NORM;
    for (int k = 0; k < N_NORM; ++k) net->norm_host[k] = (k < N_FEAT || (k >= 2 * N_FEAT && k < 2 * N_FEAT + N_OUT)) ? 0.0f : 1.0f;
    e = hipMemsetAsync(net->state, 0, n * sizeof(float), net->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(net->b.params, params, N_PARAMS * sizeof(float), hipMemcpyHostToDevice, net->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(net->b.norm, net->norm_host, N_NORM * sizeof(float), hipMemcpyHostToDevice, net->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
  }
  if (e != hipSuccess) {
    const std::string msg = hipGetErrorString(e);
    delete net;
    return mfail(nullptr, e == hipErrorOutOfMemory ? HMLE_E_NOMEM : HMLE_E_HIP, msg);
  }
  *out = net;
  return HMLE_OK;
}

hmle_status hmle_mlp_set_params(hmle_mlp net, const float* params) {
  if (!net || !params) return mfail(net, HMLE_E_INVALID, "NULL argument");
  HIP_OR_FAIL(net, hipMemcpyAsync(net->b.params, params, N_PARAMS * sizeof(float), hipMemcpyHostToDevice, net->stream));
  HIP_OR_FAIL(net, hipMemsetAsync(net->b.m, 0, 2 * N_PARAMS * sizeof(float), net->stream));
  HIP_OR_FAIL(net, hipStreamSynchronize(net->stream));
  net->step = 0;
  return HMLE_OK;
}

hmle_status hmle_mlp_get_params(hmle_mlp net, float* params) {
  if (!net || !params) return mfail(net, HMLE_E_INVALID, "NULL argument");
  HIP_OR_FAIL(net, hipMemcpyAsync(params, net->b.params, N_PARAMS * sizeof(float), hipMemcpyDeviceToHost, net->stream));
  HIP_OR_FAIL(net, hipStreamSynchronize(net->stream));
  return HMLE_OK;
}

hmle_status hmle_mlp_set_norm(hmle_mlp net, const float* norm) {
  if (!net || !norm) return mfail(net, HMLE_E_INVALID, "NULL argument");
  for (int k = 0; k < N_NORM; ++k)
    if (!std::isfinite(norm[k])) return mfail(net, HMLE_E_INVALID, "non-finite normalisation");
  for (int k = 0; k < N_FEAT; ++k)
    if (!(norm[N_FEAT + k] > 0)) return mfail(net, HMLE_E_INVALID, "feature scales must be > 0");
  for (int k = 0; k < N_OUT; ++k)
    if (!(norm[2 * N_FEAT + N_OUT + k] > 0)) return mfail(net, HMLE_E_INVALID, "target scales must be > 0");
  std::copy(norm, norm + N_NORM, net->norm_host);
  HIP_OR_FAIL(net, hipMemcpyAsync(net->b.norm, net->norm_host, N_NORM * sizeof(float), hipMemcpyHostToDevice,
                                  net->stream));
  HIP_OR_FAIL(net, hipStreamSynchronize(net->stream));
  return HMLE_OK;
}

hmle_status hmle_mlp_get_norm(hmle_mlp net, float* norm) {
  if (!net || !norm) return mfail(net, HMLE_E_INVALID, "NULL argument");
  std::copy(net->norm_host, net->norm_host + N_NORM, norm);
  return HMLE_OK;
}

hmle_status hmle_mlp_fit_norm(hmle_mlp net, const float* x, const float* lt, int64_t rows) {
  if (!net || !x || !lt) return mfail(net, HMLE_E_INVALID, "NULL argument");
  if (rows < 1) return mfail(net, HMLE_E_INVALID, "rows must be >= 1");
  // feature statistics into norm[0 .. 2*33), target statistics into norm[66 .. 74);
  // a feature constant over the data is switched off (scale 1e30), a constant
  // target keeps the floor 1e-6
  launch_col_stats(x, rows, N_FEAT, 1e30f, net->b.norm, net->stream);
  launch_col_stats(lt, rows, N_OUT, 1e-6f, net->b.norm + 2 * N_FEAT, net->stream);
  HIP_OR_FAIL(net, hmle::launch_status());
  HIP_OR_FAIL(net, hipMemcpyAsync(net->norm_host, net->b.norm, N_NORM * sizeof(float), hipMemcpyDeviceToHost,
                                  net->stream));
  HIP_OR_FAIL(net, hipStreamSynchronize(net->stream));
  return HMLE_OK;
}

hmle_status hmle_mlp_forward(hmle_mlp net, const float* x, int32_t rows, float* y) {
  if (!net || !x || !y) return mfail(net, HMLE_E_INVALID, "NULL argument");
  if (rows < 1 || rows > (1 << 20)) return mfail(net, HMLE_E_INVALID, "rows must be in [1, 2^20]");
  hmle_status s = ensure_rows(net, rows);
  if (s != HMLE_OK) return s;
  launch_mlp_forward(net->b, x, nullptr, rows, net->stream);
  launch_mlp_output(net->b, rows, y, net->stream);
  HIP_OR_FAIL(net, hmle::launch_status());
  HIP_OR_FAIL(net, hipStreamSynchronize(net->stream));
  return HMLE_OK;
}

hmle_status hmle_mlp_grad(hmle_mlp net, const float* x, const float* lt, const int32_t* idx, int32_t rows,
                          int64_t total, float* grad, float* loss) {
  if (!net || !grad) return mfail(net, HMLE_E_INVALID, "NULL argument");
  hmle_status s = grad_pass(net, x, lt, idx, rows, total);
  if (s != HMLE_OK) return s;
  HIP_OR_FAIL(net, hipMemcpyAsync(grad, net->b.grad, N_PARAMS * sizeof(float), hipMemcpyDeviceToDevice, net->stream));
  s = read_loss(net, loss);
  if (s != HMLE_OK) return s;
  HIP_OR_FAIL(net, hipStreamSynchronize(net->stream));
  return HMLE_OK;
}

hmle_status hmle_mlp_train_step(hmle_mlp net, const float* x, const float* lt, const int32_t* idx, int32_t rows,
                                int64_t total, float lr, float* loss) {
  if (!net) return mfail(nullptr, HMLE_E_INVALID, "network is NULL");
  if (!(lr > 0) || !std::isfinite(lr)) return mfail(net, HMLE_E_INVALID, "lr must be > 0");
  hmle_status s = grad_pass(net, x, lt, idx, rows, total);
  if (s != HMLE_OK) return s;
  net->step += 1;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)net->step));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)net->step));
  launch_adam(net->b, lr, c1, c2, net->stream);
  HIP_OR_FAIL(net, hmle::launch_status());
  return read_loss(net, loss);
}

hmle_status hmle_propose(hmle_mlp net, const float* feat, hmle_theta* start) {
  if (!net || !feat || !start) return mfail(net, HMLE_E_INVALID, "NULL argument");
  hmle_status s = ensure_rows(net, 1);
  if (s != HMLE_OK) return s;
  launch_mlp_forward(net->b, feat, nullptr, 1, net->stream);
  HIP_OR_FAIL(net, hmle::launch_status());
  float y[N_OUT];
  HIP_OR_FAIL(net, hipMemcpyAsync(y, net->b.Y, sizeof(y), hipMemcpyDeviceToHost, net->stream));
  HIP_OR_FAIL(net, hipStreamSynchronize(net->stream));
  double th[N_OUT];
  for (int k = 0; k < N_OUT; ++k) {
    const double lv = (double)y[k] * net->norm_host[2 * N_FEAT + N_OUT + k] + net->norm_host[2 * N_FEAT + k];
    if (!std::isfinite(lv)) return mfail(net, HMLE_E_INVALID, "network output is not finite");
    th[k] = std::exp(lv);
  }
  // into the optimiser's parameter box
  start->sigma2 = std::min(std::max(th[0], 1e-6), 1e6);
  start->range = std::min(std::max(th[1], 1e-4), 10.0);
  start->nu = std::min(std::max(th[2], 0.05), 8.0);
  start->tau2 = std::min(std::max(th[3], 1e-10), 1e3);
  return HMLE_OK;
}

void hmle_mlp_destroy(hmle_mlp net) { delete net; }

}  // extern "C"
