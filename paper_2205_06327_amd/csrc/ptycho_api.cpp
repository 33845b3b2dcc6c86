// ptycho_api.cpp -- C ABI of the multislice ptychography library: contexts,
// FP64-built tables, host validation, tile binning and the stream-ordered
// launches of the fused kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ptycho.h"
#include "ptycho_host.h"
#include "ptycho_kernels.h"

namespace ptycho {
namespace host {

namespace {
thread_local std::string g_err;
}  // namespace

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(PTYCHO_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_err.c_str(); }

// Host-side check of a caller buffer the kernels will address: it must be device memory of the
// context's device, managed memory or pinned host memory, and, where the runtime knows the
// allocation, [p, p + bytes) must lie inside it.  A pageable host pointer, another device's
// memory or an overrun would otherwise reach the kernels as an invalid address.  Memory the
// runtime reports without an address range (e.g. virtual-memory mappings) passes on its type.
int check_buffer(int device, const void* p, size_t bytes, const char* what) {
  if (!p || bytes == 0) return PTYCHO_OK;  // presence is checked by the callers
  hipPointerAttribute_t at{};
  hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess || at.type == hipMemoryTypeUnregistered) {
    (void)hipGetLastError();
    return fail(PTYCHO_E_ARG, "%s is not device-accessible memory (pageable host memory?)", what);
  }
  if (at.type == hipMemoryTypeDevice && at.device != device)
    return fail(PTYCHO_E_ARG, "%s is on device %d, the context on device %d", what, at.device, device);
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) == hipSuccess) {
    const size_t off = static_cast<size_t>(static_cast<const char*>(p) - static_cast<const char*>(base));
    if (off > size || bytes > size - off)
      return fail(PTYCHO_E_SHAPE, "%s: %zu bytes from offset %zu overrun its %zu-byte allocation", what, bytes, off,
                  size);
  } else {
    (void)hipGetLastError();
  }
  return PTYCHO_OK;
}

// Elements spanned by a [S][h][w] view with strides (slice_stride, ld), 0 when empty.  Saturates at
// kSpanCap (beyond any allocation, small enough that byte counts do not wrap), so absurd strides
// fail the allocation check instead of wrapping around to a small span.
constexpr size_t kSpanCap = size_t(1) << 56;
size_t span_elems(int64_t S, int64_t h, int64_t w, int64_t slice_stride, int64_t ld) {
  if (S <= 0 || h <= 0 || w <= 0) return 0;
  if (ld < 0 || (S > 1 && slice_stride < 0)) return kSpanCap;
  const __int128 e = static_cast<__int128>(S - 1) * (S > 1 ? slice_stride : 0) + static_cast<__int128>(h - 1) * ld + w;
  return e > static_cast<__int128>(kSpanCap) ? kSpanCap : static_cast<size_t>(e);
}

}  // namespace host
}  // namespace ptycho

using namespace ptycho::host;

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// fftfreq(M, d)[k]: k/(M d) for k < M/2, (k - M)/(M d) otherwise (M even).
double fft_freq(int k, int M, double d) { return (k < M / 2 ? k : k - M) / (M * d); }

}  // namespace

struct ptycho_ctx {
  int M = 0, S = 0;
  double wavelength = 0, dz = 0, pixel = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  int grid = 0;            // persistent workgroups of the fused kernels
  int capacity = 0;        // positions per call
  float2* d_tw = nullptr;  // W_M^e
  float2* d_h = nullptr;   // separable propagator factor
  float2* d_probe_part = nullptr;  // probe-gradient partial sums, grid * M*M
  ptycho::TileDesc* d_tiles = nullptr;  // tile table of ptycho_tiles_grad (kMaxTiles entries)
  std::vector<ptycho::TileDesc> h_tiles;
  float2* d_ws = nullptr;  // incident-wave store, grid * ws_slots(S, ck) * M*M
  int ck = 1;              // checkpoint interval of the incident waves
  double* d_loss = nullptr;  // per-position losses [capacity]
  unsigned* d_status = nullptr;
  int64_t bytes = 0;
  // kernel timing (ptycho_profile_*)
  bool profiling = false;
  std::vector<hipEvent_t> ev;   // pairs: ev[2k] start, ev[2k+1] stop
  std::vector<int> ev_n;        // positions of launch k
  size_t ev_used = 0;
  int64_t dropped = 0;
};

namespace {

void free_ctx(ptycho_ctx* c) {
  if (!c) return;
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->d_tw) (void)hipFree(c->d_tw);
  if (c->d_h) (void)hipFree(c->d_h);
  if (c->d_ws) (void)hipFree(c->d_ws);
  if (c->d_probe_part) (void)hipFree(c->d_probe_part);
  if (c->d_tiles) (void)hipFree(c->d_tiles);
  if (c->d_loss) (void)hipFree(c->d_loss);
  if (c->d_status) (void)hipFree(c->d_status);
  delete c;
}

int validate_windows_host(const int32_t* pos, int32_t n, int32_t H, int32_t W, int32_t M) {
  for (int32_t i = 0; i < n; ++i) {
    const int32_t y0 = pos[2 * i], x0 = pos[2 * i + 1];
    if (y0 < 0 || x0 < 0 || static_cast<int64_t>(y0) + M > H || static_cast<int64_t>(x0) + M > W)
      return fail(PTYCHO_E_BOUNDS, "position %d: window (%d,%d)+%d leaves the %dx%d object", i, y0, x0, M, H, W);
  }
  return PTYCHO_OK;
}

int check_object_args(const ptycho_ctx* c, const void* obj, int32_t H, int32_t W, int64_t slice_stride, int32_t ld,
                      const void* probe, const int32_t* pos, int32_t n) {
  if (!c) return fail(PTYCHO_E_ARG, "null context");
  if (n < 0) return fail(PTYCHO_E_ARG, "negative position count");
  if (n > 0 && (!obj || !probe || !pos)) return fail(PTYCHO_E_ARG, "null object, probe or positions");
  if (H < c->M || W < c->M) return fail(PTYCHO_E_SHAPE, "object %dx%d smaller than the %d window", H, W, c->M);
  if (ld < W) return fail(PTYCHO_E_SHAPE, "ld %d < W %d", ld, W);
  if (slice_stride < static_cast<int64_t>(H) * ld && c->S > 1)
    return fail(PTYCHO_E_SHAPE, "slice stride %lld < H*ld", static_cast<long long>(slice_stride));
  if (static_cast<int64_t>(ld) * c->M >= (int64_t(1) << 31))
    return fail(PTYCHO_E_SHAPE, "row stride %d too large for a window", ld);
  return PTYCHO_OK;
}

// The object, probe, positions and (optional) patterns of a position call.
int check_position_buffers(const ptycho_ctx* c, const void* obj, int32_t H, int32_t W, int64_t slice_stride,
                           int32_t ld, const void* probe, const int32_t* pos, int32_t n, const float* meas,
                           int64_t probe_stride = 0) {
  if (n == 0) return PTYCHO_OK;
  const size_t M2 = static_cast<size_t>(c->M) * c->M;
  PT_BUF(c->device, obj, span_elems(c->S, H, W, slice_stride, ld) * sizeof(float2), "object");
  PT_BUF(c->device, probe, span_elems(n, 1, static_cast<int64_t>(M2), probe_stride, 0) * sizeof(float2), "probe");
  PT_BUF(c->device, pos, 2 * static_cast<size_t>(n) * sizeof(int32_t), "positions");
  PT_BUF(c->device, meas, static_cast<size_t>(n) * M2 * sizeof(float), "measurements");
  return PTYCHO_OK;
}

ptycho::KernelArgs base_args(const ptycho_ctx* c) {
  ptycho::KernelArgs a{};
  a.M = c->M;
  a.S = c->S;
  a.tw = c->d_tw;
  a.h = c->d_h;
  a.ws = c->d_ws;
  a.ck = c->ck;
  a.loss_work = c->d_loss;
  a.status = c->d_status;
  return a;
}

// Launch of a fused kernel, bracketed by timing events when profiling.
int launch_fused_timed(ptycho_ctx* c, const ptycho::KernelArgs& a, int mode) {
  const int grid = a.n < c->grid ? a.n : c->grid;
  const bool timed = c->profiling && c->ev_used < c->ev_n.size();
  if (c->profiling && !timed) ++c->dropped;
  if (timed) PT_HIP(hipEventRecord(c->ev[2 * c->ev_used], c->stream));
  PT_HIP(ptycho::launch_fused(a, mode, grid, c->stream));
  if (timed) {
    PT_HIP(hipEventRecord(c->ev[2 * c->ev_used + 1], c->stream));
    c->ev_n[c->ev_used++] = a.n;
  }
  return PTYCHO_OK;
}

int run_loss_grad(ptycho_ctx* c, ptycho::KernelArgs a, int32_t gh, int32_t gw, double* loss, uint32_t flags,
                  float2* probe_grad = nullptr) {
  const bool acc = (flags & PTYCHO_ACCUMULATE) != 0;
  if (!acc) PT_HIP(ptycho::launch_zero_slices(a.grad, c->S, gh, gw, a.gslice, a.gld, c->stream));
  if (a.n > 0) {
    a.probe_part = c->d_probe_part;
    int rc = launch_fused_timed(c, a, probe_grad ? ptycho::kModeLossGradProbe : ptycho::kModeLossGrad);
    if (rc != PTYCHO_OK) return rc;
  }
  if (probe_grad) {  // sum the launched workgroups' partial sums (none when n = 0)
    const int parts = a.n < c->grid ? a.n : c->grid;
    PT_HIP(ptycho::launch_probe_reduce(c->d_probe_part, parts, c->M, probe_grad, acc, c->stream));
  }
  PT_HIP(ptycho::launch_finalize_loss(c->d_loss, a.n, loss, acc, c->stream));
  return PTYCHO_OK;
}

}  // namespace

extern "C" {

const char* ptycho_last_error(void) { return ptycho::host::last_error(); }
const char* ptycho_version(void) { return "ptycho-mi355x 0.1 (gfx950)"; }

int ptycho_create(ptycho_ctx** out, int32_t M, int32_t S, double wavelength_A, double dz_A, double pixel_A,
                  int32_t max_positions, void* stream) {
  if (!out) return fail(PTYCHO_E_ARG, "null output pointer");
  *out = nullptr;
  if (M != 64 && M != 128) return fail(PTYCHO_E_UNSUPPORTED, "window size %d not supported (64 or 128)", M);
  if (S < 1 || S > 64) return fail(PTYCHO_E_UNSUPPORTED, "slice count %d not supported (1..64)", S);
  if (!(pixel_A > 0) || !std::isfinite(wavelength_A) || !std::isfinite(dz_A))
    return fail(PTYCHO_E_ARG, "invalid physics (wavelength %g, dz %g, pixel %g)", wavelength_A, dz_A, pixel_A);
  if (max_positions < 0) return fail(PTYCHO_E_ARG, "negative capacity");
  ptycho_ctx* c = new ptycho_ctx();
  c->M = M;
  c->S = S;
  c->wavelength = wavelength_A;
  c->dz = dz_A;
  c->pixel = pixel_A;
  c->stream = static_cast<hipStream_t>(stream);
  hipError_t e = hipGetDevice(&c->device);
  int cus = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
  if (e != hipSuccess) {
    free_ctx(c);
    return hip_fail(e, "device query");
  }
  c->grid = cus > 0 ? cus : 256;  // one workgroup per CU (LDS-bound occupancy)
  c->capacity = max_positions > 0 ? max_positions : 4096;

  // Tables computed in double precision, rounded once to float.
  std::vector<float2> tw(M), h(M);
  for (int e2 = 0; e2 < M; ++e2) {
    const double ang = -2.0 * kPi * e2 / M;
    tw[e2] = make_float2(static_cast<float>(std::cos(ang)), static_cast<float>(std::sin(ang)));
    const double f = fft_freq(e2, M, pixel_A);
    const double ph = -kPi * wavelength_A * dz_A * f * f;
    h[e2] = make_float2(static_cast<float>(std::cos(ph)), static_cast<float>(std::sin(ph)));
  }
  const size_t ws_elems = static_cast<size_t>(c->grid) * ptycho::ws_slots(S, 1) * M * M;
  if ((e = hipMalloc(&c->d_tw, M * sizeof(float2))) != hipSuccess ||
      (e = hipMalloc(&c->d_h, M * sizeof(float2))) != hipSuccess ||
      (e = hipMalloc(&c->d_loss, static_cast<size_t>(c->capacity) * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&c->d_status, sizeof(unsigned))) != hipSuccess ||
      (ws_elems > 0 && (e = hipMalloc(&c->d_ws, ws_elems * sizeof(float2))) != hipSuccess) ||
      (e = hipMalloc(&c->d_probe_part, static_cast<size_t>(c->grid) * M * M * sizeof(float2))) != hipSuccess ||
      (e = hipMalloc(&c->d_tiles, ptycho::kMaxTiles * sizeof(ptycho::TileDesc))) != hipSuccess) {
    free_ctx(c);
    return fail(PTYCHO_E_NOMEM, "device allocation failed: %s", hipGetErrorString(e));
  }
  c->bytes = static_cast<int64_t>(2 * M * sizeof(float2) + c->capacity * sizeof(double) + sizeof(unsigned) +
                                  ws_elems * sizeof(float2) + static_cast<size_t>(c->grid) * M * M * sizeof(float2) +
                                  ptycho::kMaxTiles * sizeof(ptycho::TileDesc));
  if ((e = hipMemcpy(c->d_tw, tw.data(), M * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->d_h, h.data(), M * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(c->d_status, 0, sizeof(unsigned))) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
    free_ctx(c);
    return hip_fail(e, "table upload");
  }
  *out = c;
  return PTYCHO_OK;
}

int ptycho_destroy(ptycho_ctx* ctx) {
  if (!ctx) return PTYCHO_OK;
  (void)hipStreamSynchronize(ctx->stream);
  free_ctx(ctx);
  return PTYCHO_OK;
}

int ptycho_set_stream(ptycho_ctx* ctx, void* stream) {
  if (!ctx) return fail(PTYCHO_E_ARG, "null context");
  ctx->stream = static_cast<hipStream_t>(stream);
  return PTYCHO_OK;
}

int ptycho_reserve(ptycho_ctx* ctx, int32_t max_positions) {
  if (!ctx) return fail(PTYCHO_E_ARG, "null context");
  if (max_positions <= ctx->capacity) return PTYCHO_OK;
  PT_HIP(hipStreamSynchronize(ctx->stream));
  double* p = nullptr;
  hipError_t e = hipMalloc(&p, static_cast<size_t>(max_positions) * sizeof(double));
  if (e != hipSuccess) return fail(PTYCHO_E_NOMEM, "capacity %d: %s", max_positions, hipGetErrorString(e));
  (void)hipFree(ctx->d_loss);
  ctx->d_loss = p;
  ctx->bytes += static_cast<int64_t>(max_positions - ctx->capacity) * static_cast<int64_t>(sizeof(double));
  ctx->capacity = max_positions;
  return PTYCHO_OK;
}

int64_t ptycho_workspace_bytes(const ptycho_ctx* ctx) { return ctx ? ctx->bytes : 0; }

}  // extern "C"

namespace {
int check_probe_stride(const ptycho_ctx* c, int64_t probe_stride) {
  if (probe_stride != 0 && probe_stride < static_cast<int64_t>(c->M) * c->M)
    return fail(PTYCHO_E_SHAPE, "probe stride %lld: 0 (one probe) or >= M*M (one probe per position)",
                static_cast<long long>(probe_stride));
  return PTYCHO_OK;
}

int forward_impl(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride, int32_t ld,
                 const void* probe, int64_t probe_stride, const int32_t* pos, int32_t n, float* intens) {
  int rc = check_object_args(ctx, obj, H, W, slice_stride, ld, probe, pos, n);
  if (rc != PTYCHO_OK) return rc;
  if ((rc = check_probe_stride(ctx, probe_stride)) != PTYCHO_OK) return rc;
  if (n == 0) return PTYCHO_OK;
  if (!intens) return fail(PTYCHO_E_ARG, "null intensity output");
  rc = check_position_buffers(ctx, obj, H, W, slice_stride, ld, probe, pos, n, nullptr, probe_stride);
  if (rc != PTYCHO_OK) return rc;
  PT_BUF(ctx->device, intens, static_cast<size_t>(n) * ctx->M * ctx->M * sizeof(float), "intensities");
  ptycho::KernelArgs a = base_args(ctx);
  a.n = n;
  a.obj = static_cast<const float2*>(obj);
  a.slice_stride = slice_stride;
  a.ld = ld;
  a.bh = H;
  a.bw = W;
  a.oob_flag = PTYCHO_STATUS_BOUNDS;
  a.probe = static_cast<const float2*>(probe);
  a.probe_stride = probe_stride;
  a.pos = pos;
  a.intens = intens;
  return launch_fused_timed(ctx, a, ptycho::kModeIntensity);
}
}  // namespace

extern "C" {

int ptycho_forward(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride, int32_t ld,
                   const void* probe, const int32_t* pos, int32_t n, float* intens) {
  return forward_impl(ctx, obj, H, W, slice_stride, ld, probe, 0, pos, n, intens);
}

int ptycho_forward_stack(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride, int32_t ld,
                         const void* probes, int64_t probe_stride, const int32_t* pos, int32_t n, float* intens) {
  if (ctx && probe_stride == 0) return fail(PTYCHO_E_SHAPE, "a probe stack needs a probe stride >= M*M");
  return forward_impl(ctx, obj, H, W, slice_stride, ld, probes, probe_stride, pos, n, intens);
}

int ptycho_loss_grad(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride, int32_t ld,
                     const void* probe, const int32_t* pos, int32_t n, const float* meas, double* loss,
                     double* loss_per_pos, void* grad, int64_t grad_slice_stride, int32_t grad_ld, uint32_t flags,
                     const double* grad_scale) {
  return ptycho_loss_grad_probe(ctx, obj, H, W, slice_stride, ld, probe, pos, n, meas, loss, loss_per_pos, grad,
                                grad_slice_stride, grad_ld, nullptr, flags, grad_scale);
}

}  // extern "C"

namespace {
int loss_grad_impl(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride, int32_t ld,
                   const void* probe, int64_t probe_stride, const int32_t* pos, int32_t n, const float* meas,
                   double* loss, double* loss_per_pos, void* grad, int64_t grad_slice_stride, int32_t grad_ld,
                   void* probe_grad, uint32_t flags, const double* grad_scale) {
  int rc = check_object_args(ctx, obj, H, W, slice_stride, ld, probe, pos, n);
  if (rc != PTYCHO_OK) return rc;
  if ((rc = check_probe_stride(ctx, probe_stride)) != PTYCHO_OK) return rc;
  if (probe_grad && probe_stride != 0)
    return fail(PTYCHO_E_UNSUPPORTED, "the probe gradient needs one probe shared by all positions");
  if (flags & ~PTYCHO_ACCUMULATE) return fail(PTYCHO_E_ARG, "unknown flags 0x%x", flags);
  if (!loss || !grad) return fail(PTYCHO_E_ARG, "null loss or gradient");
  if (n > 0 && !meas) return fail(PTYCHO_E_ARG, "null measurements");
  if (n > ctx->capacity) return fail(PTYCHO_E_CAPACITY, "%d positions exceed the reserved capacity %d", n, ctx->capacity);
  if (grad_ld < W || (ctx->S > 1 && grad_slice_stride < static_cast<int64_t>(H) * grad_ld))
    return fail(PTYCHO_E_SHAPE, "gradient strides do not cover %dx%d", H, W);
  if (static_cast<int64_t>(grad_ld) * ctx->M >= (int64_t(1) << 31))
    return fail(PTYCHO_E_SHAPE, "gradient row stride too large");  // window row offsets are 32-bit
  if (grad == obj) return fail(PTYCHO_E_ARG, "gradient aliases the object");
  rc = check_position_buffers(ctx, obj, H, W, slice_stride, ld, probe, pos, n, meas, probe_stride);
  if (rc != PTYCHO_OK) return rc;
  PT_BUF(ctx->device, grad, span_elems(ctx->S, H, W, grad_slice_stride, grad_ld) * sizeof(float2), "gradient");
  PT_BUF(ctx->device, loss, sizeof(double), "loss");
  PT_BUF(ctx->device, loss_per_pos, static_cast<size_t>(n) * sizeof(double), "per-position losses");
  PT_BUF(ctx->device, probe_grad, static_cast<size_t>(ctx->M) * ctx->M * sizeof(float2), "probe gradient");
  PT_BUF(ctx->device, grad_scale, sizeof(double), "gradient scale");
  ptycho::KernelArgs a = base_args(ctx);
  a.n = n;
  a.obj = static_cast<const float2*>(obj);
  a.slice_stride = slice_stride;
  a.ld = ld;
  a.bh = H;
  a.bw = W;
  a.oob_flag = PTYCHO_STATUS_BOUNDS;
  a.probe = static_cast<const float2*>(probe);
  a.pos = pos;
  a.meas = meas;
  a.loss_pos = loss_per_pos;
  a.grad = static_cast<float2*>(grad);
  a.gslice = grad_slice_stride;
  a.gld = grad_ld;
  a.grad_scale = grad_scale;
  a.probe_stride = probe_stride;
  if (probe_grad && (probe_grad == grad || probe_grad == probe))
    return fail(PTYCHO_E_ARG, "probe gradient aliases the gradient or the probe");
  return run_loss_grad(ctx, a, H, W, loss, flags, static_cast<float2*>(probe_grad));
}
}  // namespace

extern "C" {

int ptycho_loss_grad_probe(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride,
                           int32_t ld, const void* probe, const int32_t* pos, int32_t n, const float* meas,
                           double* loss, double* loss_per_pos, void* grad, int64_t grad_slice_stride, int32_t grad_ld,
                           void* probe_grad, uint32_t flags, const double* grad_scale) {
  return loss_grad_impl(ctx, obj, H, W, slice_stride, ld, probe, 0, pos, n, meas, loss, loss_per_pos, grad,
                        grad_slice_stride, grad_ld, probe_grad, flags, grad_scale);
}

int ptycho_loss_grad_stack(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride, int32_t ld,
                           const void* probes, int64_t probe_stride, const int32_t* pos, int32_t n, const float* meas,
                           double* loss, double* loss_per_pos, void* grad, int64_t grad_slice_stride, int32_t grad_ld,
                           uint32_t flags, const double* grad_scale) {
  if (ctx && probe_stride == 0) return fail(PTYCHO_E_SHAPE, "a probe stack needs a probe stride >= M*M");
  return loss_grad_impl(ctx, obj, H, W, slice_stride, ld, probes, probe_stride, pos, n, meas, loss, loss_per_pos,
                        grad, grad_slice_stride, grad_ld, nullptr, flags, grad_scale);
}

int ptycho_shift_probes(ptycho_ctx* ctx, const void* probe, const float* shifts, int32_t n, void* out) {
  if (!ctx) return fail(PTYCHO_E_ARG, "null context");
  if (n < 0) return fail(PTYCHO_E_ARG, "negative count");
  if (n == 0) return PTYCHO_OK;
  if (!probe || !shifts || !out) return fail(PTYCHO_E_ARG, "null pointer argument");
  const size_t M2 = static_cast<size_t>(ctx->M) * ctx->M;
  const char* o = static_cast<const char*>(out);
  const char* q = static_cast<const char*>(probe);
  if (q < o + static_cast<size_t>(n) * M2 * sizeof(float2) && o < q + M2 * sizeof(float2))
    return fail(PTYCHO_E_ARG, "the output aliases the probe");
  PT_BUF(ctx->device, probe, M2 * sizeof(float2), "probe");
  PT_BUF(ctx->device, shifts, 2 * static_cast<size_t>(n) * sizeof(float), "shifts");
  PT_BUF(ctx->device, out, static_cast<size_t>(n) * M2 * sizeof(float2), "shifted probes");
  PT_HIP(ptycho::launch_shift_probes(static_cast<const float2*>(probe), shifts, n, ctx->M, ctx->d_tw,
                                     static_cast<float2*>(out), ctx->stream));
  return PTYCHO_OK;
}

}  // extern "C"

namespace {
int loss_impl(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride, int32_t ld,
              const void* probe, int64_t probe_stride, const int32_t* pos, int32_t n, const float* meas, double* loss,
              double* loss_per_pos, uint32_t flags) {
  int rc = check_object_args(ctx, obj, H, W, slice_stride, ld, probe, pos, n);
  if (rc != PTYCHO_OK) return rc;
  if ((rc = check_probe_stride(ctx, probe_stride)) != PTYCHO_OK) return rc;
  if (flags & ~PTYCHO_ACCUMULATE) return fail(PTYCHO_E_ARG, "unknown flags 0x%x", flags);
  if (!loss) return fail(PTYCHO_E_ARG, "null loss");
  if (n > 0 && !meas) return fail(PTYCHO_E_ARG, "null measurements");
  if (n > ctx->capacity) return fail(PTYCHO_E_CAPACITY, "%d positions exceed the reserved capacity %d", n, ctx->capacity);
  rc = check_position_buffers(ctx, obj, H, W, slice_stride, ld, probe, pos, n, meas, probe_stride);
  if (rc != PTYCHO_OK) return rc;
  PT_BUF(ctx->device, loss, sizeof(double), "loss");
  PT_BUF(ctx->device, loss_per_pos, static_cast<size_t>(n) * sizeof(double), "per-position losses");
  ptycho::KernelArgs a = base_args(ctx);
  a.n = n;
  a.obj = static_cast<const float2*>(obj);
  a.slice_stride = slice_stride;
  a.ld = ld;
  a.bh = H;
  a.bw = W;
  a.oob_flag = PTYCHO_STATUS_BOUNDS;
  a.probe = static_cast<const float2*>(probe);
  a.probe_stride = probe_stride;
  a.pos = pos;
  a.meas = meas;
  a.loss_pos = loss_per_pos;
  if (n > 0) {
    rc = launch_fused_timed(ctx, a, ptycho::kModeLoss);
    if (rc != PTYCHO_OK) return rc;
  }
  PT_HIP(ptycho::launch_finalize_loss(ctx->d_loss, n, loss, (flags & PTYCHO_ACCUMULATE) != 0, ctx->stream));
  return PTYCHO_OK;
}
}  // namespace

extern "C" {

int ptycho_loss(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride, int32_t ld,
                const void* probe, const int32_t* pos, int32_t n, const float* meas, double* loss,
                double* loss_per_pos, uint32_t flags) {
  return loss_impl(ctx, obj, H, W, slice_stride, ld, probe, 0, pos, n, meas, loss, loss_per_pos, flags);
}

int ptycho_loss_stack(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride, int32_t ld,
                      const void* probes, int64_t probe_stride, const int32_t* pos, int32_t n, const float* meas,
                      double* loss, double* loss_per_pos, uint32_t flags) {
  if (ctx && probe_stride == 0) return fail(PTYCHO_E_SHAPE, "a probe stack needs a probe stride >= M*M");
  return loss_impl(ctx, obj, H, W, slice_stride, ld, probes, probe_stride, pos, n, meas, loss, loss_per_pos, flags);
}

int ptycho_tile_box(int32_t H, int32_t W, int32_t tiles_y, int32_t tiles_x, int32_t ty, int32_t tx, int32_t halo,
                    int32_t* ty0, int32_t* ty1, int32_t* tx0, int32_t* tx1, int32_t* ey0, int32_t* ey1, int32_t* ex0,
                    int32_t* ex1) {
  if (tiles_y < 1 || tiles_x < 1 || ty < 0 || tx < 0 || ty >= tiles_y || tx >= tiles_x || halo < 0 || H < 1 || W < 1)
    return fail(PTYCHO_E_ARG, "bad tile grid request");
  const int32_t a0 = static_cast<int32_t>(static_cast<int64_t>(ty) * H / tiles_y);
  const int32_t a1 = static_cast<int32_t>(static_cast<int64_t>(ty + 1) * H / tiles_y);
  const int32_t b0 = static_cast<int32_t>(static_cast<int64_t>(tx) * W / tiles_x);
  const int32_t b1 = static_cast<int32_t>(static_cast<int64_t>(tx + 1) * W / tiles_x);
  if (ty0) *ty0 = a0;
  if (ty1) *ty1 = a1;
  if (tx0) *tx0 = b0;
  if (tx1) *tx1 = b1;
  if (ey0) *ey0 = a0 - halo < 0 ? 0 : a0 - halo;
  if (ey1) *ey1 = a1 + halo > H ? H : a1 + halo;
  if (ex0) *ex0 = b0 - halo < 0 ? 0 : b0 - halo;
  if (ex1) *ex1 = b1 + halo > W ? W : b1 + halo;
  return PTYCHO_OK;
}

int ptycho_tile_grad(ptycho_ctx* ctx, const void* obj_ext, int32_t ey0, int32_t ex0, int32_t eh, int32_t ew,
                     int64_t slice_stride, int32_t ld, int32_t ty0, int32_t ty1, int32_t tx0, int32_t tx1,
                     int32_t halo, int32_t H, int32_t W, const void* probe, const int32_t* pos, int32_t n,
                     const float* meas, double* loss, double* loss_per_pos, void* tile_grad, uint32_t flags) {
  if (!ctx) return fail(PTYCHO_E_ARG, "null context");
  if (n < 0) return fail(PTYCHO_E_ARG, "negative position count");
  if (flags & ~PTYCHO_ACCUMULATE) return fail(PTYCHO_E_ARG, "unknown flags 0x%x", flags);
  if (!loss || !tile_grad || (n > 0 && (!obj_ext || !probe || !pos || !meas)))
    return fail(PTYCHO_E_ARG, "null pointer argument");
  if (halo < 0 || ty0 < 0 || tx0 < 0 || ty1 <= ty0 || tx1 <= tx0 || ty1 > H || tx1 > W)
    return fail(PTYCHO_E_SHAPE, "bad tile [%d,%d)x[%d,%d) in %dx%d", ty0, ty1, tx0, tx1, H, W);
  const int32_t wy0 = ty0 - halo < 0 ? 0 : ty0 - halo, wy1 = ty1 + halo > H ? H : ty1 + halo;
  const int32_t wx0 = tx0 - halo < 0 ? 0 : tx0 - halo, wx1 = tx1 + halo > W ? W : tx1 + halo;
  if (ey0 != wy0 || ex0 != wx0 || eh != wy1 - wy0 || ew != wx1 - wx0)
    return fail(PTYCHO_E_SHAPE, "extended box (%d,%d)+(%d,%d) is not the tile grown by halo %d: expected (%d,%d)+(%d,%d)",
                ey0, ex0, eh, ew, halo, wy0, wx0, wy1 - wy0, wx1 - wx0);
  if (eh < ctx->M || ew < ctx->M) return fail(PTYCHO_E_HALO, "extended box smaller than a window");
  if (ld < ew || (ctx->S > 1 && slice_stride < static_cast<int64_t>(eh) * ld))
    return fail(PTYCHO_E_SHAPE, "object strides do not cover the extended box");
  if (static_cast<int64_t>(ld) * ctx->M >= (int64_t(1) << 31)) return fail(PTYCHO_E_SHAPE, "row stride too large");
  if (n > ctx->capacity) return fail(PTYCHO_E_CAPACITY, "%d positions exceed the reserved capacity %d", n, ctx->capacity);
  int rc = check_position_buffers(ctx, obj_ext, eh, ew, slice_stride, ld, probe, pos, n, meas);
  if (rc != PTYCHO_OK) return rc;
  PT_BUF(ctx->device, tile_grad, static_cast<size_t>(ctx->S) * eh * ew * sizeof(float2), "tile gradient");
  PT_BUF(ctx->device, loss, sizeof(double), "loss");
  PT_BUF(ctx->device, loss_per_pos, static_cast<size_t>(n) * sizeof(double), "per-position losses");
  ptycho::KernelArgs a = base_args(ctx);
  a.n = n;
  a.obj = static_cast<const float2*>(obj_ext);
  a.slice_stride = slice_stride;
  a.ld = ld;
  a.bh = eh;
  a.bw = ew;
  a.oy = ey0;
  a.ox = ex0;
  a.check_tile = 1;
  a.ty0 = ty0;
  a.ty1 = ty1;
  a.tx0 = tx0;
  a.tx1 = tx1;
  a.oob_flag = PTYCHO_STATUS_HALO;
  a.probe = static_cast<const float2*>(probe);
  a.pos = pos;
  a.meas = meas;
  a.loss_pos = loss_per_pos;
  a.grad = static_cast<float2*>(tile_grad);
  a.gslice = static_cast<long long>(eh) * ew;
  a.gld = ew;
  return run_loss_grad(ctx, a, eh, ew, loss, flags);
}

}  // extern "C"

namespace {
int tiles_grad_impl(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride, int32_t ld,
                    const ptycho_tile_desc* tiles, int32_t ntiles, int32_t halo, const int32_t* tile_of_pos,
                    const void* probe, int64_t probe_stride, const int32_t* pos, int32_t n, const float* meas,
                    double* loss, double* loss_per_pos, uint32_t flags) {
  int rc = check_object_args(ctx, obj, H, W, slice_stride, ld, probe, pos, n);
  if (rc != PTYCHO_OK) return rc;
  if ((rc = check_probe_stride(ctx, probe_stride)) != PTYCHO_OK) return rc;
  if (flags & ~PTYCHO_ACCUMULATE) return fail(PTYCHO_E_ARG, "unknown flags 0x%x", flags);
  if (!loss || !tiles || (n > 0 && (!meas || !tile_of_pos))) return fail(PTYCHO_E_ARG, "null pointer argument");
  if (ntiles < 1 || ntiles > ptycho::kMaxTiles) return fail(PTYCHO_E_ARG, "tile count %d outside [1, %d]", ntiles,
                                                            ptycho::kMaxTiles);
  if (halo < 0) return fail(PTYCHO_E_ARG, "negative halo");
  if (n > ctx->capacity) return fail(PTYCHO_E_CAPACITY, "%d positions exceed the reserved capacity %d", n, ctx->capacity);
  rc = check_position_buffers(ctx, obj, H, W, slice_stride, ld, probe, pos, n, meas, probe_stride);
  if (rc != PTYCHO_OK) return rc;
  PT_BUF(ctx->device, tile_of_pos, static_cast<size_t>(n) * sizeof(int32_t), "tile indices");
  PT_BUF(ctx->device, loss, sizeof(double), "loss");
  PT_BUF(ctx->device, loss_per_pos, static_cast<size_t>(n) * sizeof(double), "per-position losses");
  std::vector<ptycho::TileDesc> table(ntiles);
  for (int k = 0; k < ntiles; ++k) {
    const ptycho_tile_desc& t = tiles[k];
    if (t.ty0 < 0 || t.tx0 < 0 || t.ty1 > H || t.tx1 > W || t.ty0 >= t.ty1 || t.tx0 >= t.tx1)
      return fail(PTYCHO_E_SHAPE, "tile %d: [%d,%d)x[%d,%d) not inside %dx%d", k, t.ty0, t.ty1, t.tx0, t.tx1, H, W);
    const int ey0 = std::max(t.ty0 - halo, 0), ex0 = std::max(t.tx0 - halo, 0);
    const int ey1 = std::min(t.ty1 + halo, H), ex1 = std::min(t.tx1 + halo, W);
    if (t.ey0 != ey0 || t.ex0 != ex0 || t.eh != ey1 - ey0 || t.ew != ex1 - ex0)
      return fail(PTYCHO_E_SHAPE, "tile %d: extended box is not the tile grown by halo %d", k, halo);
    if (t.eh < ctx->M || t.ew < ctx->M) return fail(PTYCHO_E_HALO, "tile %d: extended box smaller than a window", k);
    if (!t.grad || t.grad == obj) return fail(PTYCHO_E_ARG, "tile %d: bad gradient buffer", k);
    PT_BUF(ctx->device, t.grad, static_cast<size_t>(ctx->S) * t.eh * t.ew * sizeof(float2), "tile gradient");
    ptycho::TileDesc& d = table[k];
    d.ty0 = t.ty0; d.ty1 = t.ty1; d.tx0 = t.tx0; d.tx1 = t.tx1;
    d.ey0 = t.ey0; d.ex0 = t.ex0; d.eh = t.eh; d.ew = t.ew;
    d.grad = static_cast<float2*>(t.grad);
    d.gslice = static_cast<long long>(t.eh) * t.ew;
    d.gld = t.ew;
  }
  // Upload the table only when it changed (a walk passes the same tiles every step).  The copy is
  // stream-ordered after launches that still read the old table, and the host copy it reads is
  // kept unchanged until the stream has passed it.
  const bool same = ctx->h_tiles.size() == table.size() &&
                    std::memcmp(ctx->h_tiles.data(), table.data(), table.size() * sizeof(ptycho::TileDesc)) == 0;
  if (!same) {
    PT_HIP(hipStreamSynchronize(ctx->stream));  // the previous upload has been read
    ctx->h_tiles.swap(table);
    PT_HIP(hipMemcpyAsync(ctx->d_tiles, ctx->h_tiles.data(), ntiles * sizeof(ptycho::TileDesc),
                          hipMemcpyHostToDevice, ctx->stream));
  }
  const bool acc = (flags & PTYCHO_ACCUMULATE) != 0;
  if (!acc) PT_HIP(ptycho::launch_zero_tiles(ctx->d_tiles, ntiles, ctx->S, ctx->stream));
  ptycho::KernelArgs a = base_args(ctx);
  a.n = n;
  a.obj = static_cast<const float2*>(obj);
  a.slice_stride = slice_stride;
  a.ld = ld;
  a.bh = H;
  a.bw = W;
  a.oob_flag = PTYCHO_STATUS_HALO;
  a.probe = static_cast<const float2*>(probe);
  a.pos = pos;
  a.meas = meas;
  a.loss_pos = loss_per_pos;
  a.tiles = ctx->d_tiles;
  a.tile_of_pos = tile_of_pos;
  a.ntiles = ntiles;
  a.probe_stride = probe_stride;
  if (n > 0) {
    rc = launch_fused_timed(ctx, a, ptycho::kModeLossGrad);
    if (rc != PTYCHO_OK) return rc;
  }
  PT_HIP(ptycho::launch_finalize_loss(ctx->d_loss, n, loss, acc, ctx->stream));
  return PTYCHO_OK;
}
}  // namespace

extern "C" {

int ptycho_tiles_grad(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride, int32_t ld,
                      const ptycho_tile_desc* tiles, int32_t ntiles, int32_t halo, const int32_t* tile_of_pos,
                      const void* probe, const int32_t* pos, int32_t n, const float* meas, double* loss,
                      double* loss_per_pos, uint32_t flags) {
  return tiles_grad_impl(ctx, obj, H, W, slice_stride, ld, tiles, ntiles, halo, tile_of_pos, probe, 0, pos, n, meas,
                         loss, loss_per_pos, flags);
}

int ptycho_tiles_grad_stack(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride,
                            int32_t ld, const ptycho_tile_desc* tiles, int32_t ntiles, int32_t halo,
                            const int32_t* tile_of_pos, const void* probes, int64_t probe_stride, const int32_t* pos,
                            int32_t n, const float* meas, double* loss, double* loss_per_pos, uint32_t flags) {
  if (ctx && probe_stride == 0) return fail(PTYCHO_E_SHAPE, "a probe stack needs a probe stride >= M*M");
  return tiles_grad_impl(ctx, obj, H, W, slice_stride, ld, tiles, ntiles, halo, tile_of_pos, probes, probe_stride,
                         pos, n, meas, loss, loss_per_pos, flags);
}

int ptycho_tile_accumulate(ptycho_ctx* ctx, const void* tile_grad, int32_t ey0, int32_t ex0, int32_t eh,
                           int32_t ew, int32_t H, int32_t W, void* grad, int64_t grad_slice_stride,
                           int32_t grad_ld) {
  if (!ctx) return fail(PTYCHO_E_ARG, "null context");
  if (!tile_grad || !grad) return fail(PTYCHO_E_ARG, "null gradient pointer");
  if (eh < 0 || ew < 0 || ey0 < 0 || ex0 < 0 || ey0 + eh > H || ex0 + ew > W)
    return fail(PTYCHO_E_SHAPE, "box (%d,%d)+(%d,%d) outside %dx%d", ey0, ex0, eh, ew, H, W);
  if (grad_ld < W || (ctx->S > 1 && grad_slice_stride < static_cast<int64_t>(H) * grad_ld))
    return fail(PTYCHO_E_SHAPE, "gradient strides do not cover %dx%d", H, W);
  PT_BUF(ctx->device, tile_grad, static_cast<size_t>(ctx->S) * eh * ew * sizeof(float2), "tile gradient");
  PT_BUF(ctx->device, grad, span_elems(ctx->S, H, W, grad_slice_stride, grad_ld) * sizeof(float2), "gradient");
  float2* g = static_cast<float2*>(grad) + static_cast<int64_t>(ey0) * grad_ld + ex0;
  PT_HIP(ptycho::launch_tile_accumulate(static_cast<const float2*>(tile_grad), ctx->S, eh, ew, g, grad_slice_stride,
                                        grad_ld, ctx->stream));
  return PTYCHO_OK;
}

namespace {
int check_plane(const ptycho_ctx* c, int32_t H, int32_t W, int64_t ss, int32_t ld, const void* p, const char* what) {
  if (!p) return fail(PTYCHO_E_ARG, "null %s", what);
  if (ld < W || (c->S > 1 && ss < static_cast<int64_t>(H) * ld))
    return fail(PTYCHO_E_SHAPE, "%s strides do not cover %dx%d", what, H, W);
  return PTYCHO_OK;
}
}  // namespace

int ptycho_potential_transmission(ptycho_ctx* ctx, int32_t H, int32_t W, float sigma, const float* V,
                                  int64_t v_slice_stride, int32_t v_ld, void* t, int64_t t_slice_stride,
                                  int32_t t_ld) {
  if (!ctx) return fail(PTYCHO_E_ARG, "null context");
  if (H < 0 || W < 0 || !std::isfinite(sigma)) return fail(PTYCHO_E_ARG, "bad size or sigma");
  int rc = check_plane(ctx, H, W, v_slice_stride, v_ld, V, "potential");
  if (rc == PTYCHO_OK) rc = check_plane(ctx, H, W, t_slice_stride, t_ld, t, "transmission");
  if (rc != PTYCHO_OK) return rc;
  if (H == 0 || W == 0) return PTYCHO_OK;
  PT_BUF(ctx->device, V, span_elems(ctx->S, H, W, v_slice_stride, v_ld) * sizeof(float), "potential");
  PT_BUF(ctx->device, t, span_elems(ctx->S, H, W, t_slice_stride, t_ld) * sizeof(float2), "transmission");
  PT_HIP(ptycho::launch_potential(0, sigma, ctx->S, H, W, V, v_slice_stride, v_ld, static_cast<float2*>(t), nullptr,
                                  t_slice_stride, t_ld, nullptr, 0, 0, nullptr, 0, 0, ctx->stream));
  return PTYCHO_OK;
}

int ptycho_potential_gradient(ptycho_ctx* ctx, int32_t H, int32_t W, float sigma, const void* t,
                              int64_t t_slice_stride, int32_t t_ld, const void* grad_t, int64_t g_slice_stride,
                              int32_t g_ld, float* grad_V, int64_t gv_slice_stride, int32_t gv_ld) {
  if (!ctx) return fail(PTYCHO_E_ARG, "null context");
  if (H < 0 || W < 0 || !std::isfinite(sigma)) return fail(PTYCHO_E_ARG, "bad size or sigma");
  int rc = check_plane(ctx, H, W, t_slice_stride, t_ld, t, "transmission");
  if (rc == PTYCHO_OK) rc = check_plane(ctx, H, W, g_slice_stride, g_ld, grad_t, "gradient");
  if (rc == PTYCHO_OK) rc = check_plane(ctx, H, W, gv_slice_stride, gv_ld, grad_V, "potential gradient");
  if (rc != PTYCHO_OK) return rc;
  if (H == 0 || W == 0) return PTYCHO_OK;
  PT_BUF(ctx->device, t, span_elems(ctx->S, H, W, t_slice_stride, t_ld) * sizeof(float2), "transmission");
  PT_BUF(ctx->device, grad_t, span_elems(ctx->S, H, W, g_slice_stride, g_ld) * sizeof(float2), "gradient");
  PT_BUF(ctx->device, grad_V, span_elems(ctx->S, H, W, gv_slice_stride, gv_ld) * sizeof(float), "potential gradient");
  PT_HIP(ptycho::launch_potential(1, sigma, ctx->S, H, W, nullptr, 0, 0, nullptr, static_cast<const float2*>(t),
                                  t_slice_stride, t_ld, static_cast<const float2*>(grad_t), g_slice_stride, g_ld,
                                  grad_V, gv_slice_stride, gv_ld, ctx->stream));
  return PTYCHO_OK;
}

int ptycho_copy_box(ptycho_ctx* ctx, int32_t S, int32_t h, int32_t w, const void* src, int64_t src_slice_stride,
                    int32_t src_ld, void* dst, int64_t dst_slice_stride, int32_t dst_ld) {
  if (!ctx) return fail(PTYCHO_E_ARG, "null context");
  if (!src || !dst) return fail(PTYCHO_E_ARG, "null buffer");
  if (S < 0 || h < 0 || w < 0) return fail(PTYCHO_E_SHAPE, "negative box size");
  if (src_ld < w || dst_ld < w ||
      (S > 1 && (src_slice_stride < static_cast<int64_t>(h) * src_ld ||
                 dst_slice_stride < static_cast<int64_t>(h) * dst_ld)))
    return fail(PTYCHO_E_SHAPE, "strides do not cover the box");
  if (S == 0 || h == 0 || w == 0) return PTYCHO_OK;
  const size_t e = sizeof(float2);
  for (int32_t s = 0; s < S; ++s) {
    const char* sp = static_cast<const char*>(src) + static_cast<size_t>(s) * src_slice_stride * e;
    char* dp = static_cast<char*>(dst) + static_cast<size_t>(s) * dst_slice_stride * e;
    PT_HIP(hipMemcpy2DAsync(dp, static_cast<size_t>(dst_ld) * e, sp, static_cast<size_t>(src_ld) * e,
                            static_cast<size_t>(w) * e, static_cast<size_t>(h), hipMemcpyDefault, ctx->stream));
  }
  return PTYCHO_OK;
}

int ptycho_set_checkpoint(ptycho_ctx* ctx, int32_t interval) {
  if (!ctx) return fail(PTYCHO_E_ARG, "null context");
  if (interval < 1 || interval > 64) return fail(PTYCHO_E_ARG, "checkpoint interval %d outside [1, 64]", interval);
  if (interval == ctx->ck) return PTYCHO_OK;
  const size_t old_elems = static_cast<size_t>(ctx->grid) * ptycho::ws_slots(ctx->S, ctx->ck) * ctx->M * ctx->M;
  const size_t new_elems = static_cast<size_t>(ctx->grid) * ptycho::ws_slots(ctx->S, interval) * ctx->M * ctx->M;
  if (new_elems != old_elems) {
    PT_HIP(hipStreamSynchronize(ctx->stream));  // launches in flight may still use the store
    float2* ws = nullptr;
    if (new_elems > 0) {
      hipError_t e = hipMalloc(&ws, new_elems * sizeof(float2));
      if (e != hipSuccess) return fail(PTYCHO_E_NOMEM, "wave store: %s", hipGetErrorString(e));
    }
    float2* old = ctx->d_ws;
    ctx->d_ws = ws;
    ctx->bytes += static_cast<int64_t>(new_elems) * static_cast<int64_t>(sizeof(float2)) -
                  static_cast<int64_t>(old_elems) * static_cast<int64_t>(sizeof(float2));
    ctx->ck = interval;
    if (old) PT_HIP(hipFree(old));  // the context already uses the new store
    return PTYCHO_OK;
  }
  ctx->ck = interval;
  return PTYCHO_OK;
}

namespace {
int box_combine(ptycho_ctx* ctx, int32_t S, const void* src, int32_t sy0, int32_t sx0, int32_t sh, int32_t sw,
                int64_t s_slice_stride, int32_t s_ld, void* dst, int32_t dy0, int32_t dx0, int32_t dh, int32_t dw,
                int64_t d_slice_stride, int32_t d_ld, bool replace, float alpha) {
  if (!ctx) return fail(PTYCHO_E_ARG, "null context");
  if (!src || !dst) return fail(PTYCHO_E_ARG, "null buffer");
  if (!std::isfinite(alpha)) return fail(PTYCHO_E_ARG, "non-finite scale");
  if (S < 1 || S > 65535) return fail(PTYCHO_E_ARG, "slice count %d outside [1, 65535]", S);
  if (sh < 0 || sw < 0 || dh < 0 || dw < 0) return fail(PTYCHO_E_SHAPE, "negative box size");
  if (s_ld < sw || d_ld < dw || (S > 1 && (s_slice_stride < static_cast<int64_t>(sh) * s_ld ||
                                           d_slice_stride < static_cast<int64_t>(dh) * d_ld)))
    return fail(PTYCHO_E_SHAPE, "buffer strides do not cover their boxes");
  const int32_t oy0 = sy0 > dy0 ? sy0 : dy0, ox0 = sx0 > dx0 ? sx0 : dx0;
  const int64_t oy1 = std::min<int64_t>(static_cast<int64_t>(sy0) + sh, static_cast<int64_t>(dy0) + dh);
  const int64_t ox1 = std::min<int64_t>(static_cast<int64_t>(sx0) + sw, static_cast<int64_t>(dx0) + dw);
  // address ranges [first, last element + 1) of the two buffers
  auto span = [&](const void* p, int32_t h, int32_t w, int64_t ss, int32_t ld) {
    const int64_t last = (h > 0 && w > 0) ? (static_cast<int64_t>(S - 1) * (S > 1 ? ss : 0) +
                                             static_cast<int64_t>(h - 1) * ld + w) : 0;
    const uintptr_t b = reinterpret_cast<uintptr_t>(p);
    return std::make_pair(b, b + static_cast<uintptr_t>(last) * sizeof(float2));
  };
  const auto a = span(src, sh, sw, s_slice_stride, s_ld), b = span(dst, dh, dw, d_slice_stride, d_ld);
  if (a.first < b.second && b.first < a.second) return fail(PTYCHO_E_ARG, "source and destination share memory");
  PT_BUF(ctx->device, src, span_elems(S, sh, sw, s_slice_stride, s_ld) * sizeof(float2), "source box");
  PT_BUF(ctx->device, dst, span_elems(S, dh, dw, d_slice_stride, d_ld) * sizeof(float2), "destination box");
  if (oy0 >= oy1 || ox0 >= ox1) return PTYCHO_OK;  // no overlap
  const int oh = static_cast<int>(oy1 - oy0), ow = static_cast<int>(ox1 - ox0);
  const float2* sp = static_cast<const float2*>(src) + static_cast<int64_t>(oy0 - sy0) * s_ld + (ox0 - sx0);
  float2* dp = static_cast<float2*>(dst) + static_cast<int64_t>(oy0 - dy0) * d_ld + (ox0 - dx0);
  PT_HIP(ptycho::launch_box_exchange(sp, s_slice_stride, s_ld, dp, d_slice_stride, d_ld, S, oh, ow, replace, alpha,
                                     ctx->stream));
  return PTYCHO_OK;
}
}  // namespace

int ptycho_box_exchange(ptycho_ctx* ctx, int32_t S, const void* src, int32_t sy0, int32_t sx0, int32_t sh,
                        int32_t sw, int64_t s_slice_stride, int32_t s_ld, void* dst, int32_t dy0, int32_t dx0,
                        int32_t dh, int32_t dw, int64_t d_slice_stride, int32_t d_ld, uint32_t mode) {
  if (mode != PTYCHO_EXCHANGE_ADD && mode != PTYCHO_EXCHANGE_REPLACE) return fail(PTYCHO_E_ARG, "bad mode %u", mode);
  return box_combine(ctx, S, src, sy0, sx0, sh, sw, s_slice_stride, s_ld, dst, dy0, dx0, dh, dw, d_slice_stride, d_ld,
                     mode == PTYCHO_EXCHANGE_REPLACE, 1.0f);
}

int ptycho_box_axpy(ptycho_ctx* ctx, int32_t S, float alpha, const void* src, int32_t sy0, int32_t sx0, int32_t sh,
                    int32_t sw, int64_t s_slice_stride, int32_t s_ld, void* dst, int32_t dy0, int32_t dx0, int32_t dh,
                    int32_t dw, int64_t d_slice_stride, int32_t d_ld) {
  return box_combine(ctx, S, src, sy0, sx0, sh, sw, s_slice_stride, s_ld, dst, dy0, dx0, dh, dw, d_slice_stride, d_ld,
                     false, alpha);
}

int ptycho_zero_gradient(ptycho_ctx* ctx, void* grad, int32_t H, int32_t W, int64_t grad_slice_stride,
                         int32_t grad_ld) {
  if (!ctx) return fail(PTYCHO_E_ARG, "null context");
  if (!grad || H < 0 || W < 0) return fail(PTYCHO_E_ARG, "bad gradient buffer");
  if (grad_ld < W || (ctx->S > 1 && grad_slice_stride < static_cast<int64_t>(H) * grad_ld))
    return fail(PTYCHO_E_SHAPE, "strides do not cover %dx%d", H, W);
  PT_BUF(ctx->device, grad, span_elems(ctx->S, H, W, grad_slice_stride, grad_ld) * sizeof(float2), "gradient");
  PT_HIP(ptycho::launch_zero_slices(static_cast<float2*>(grad), ctx->S, H, W, grad_slice_stride, grad_ld,
                                    ctx->stream));
  return PTYCHO_OK;
}

int ptycho_profile_enable(ptycho_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(PTYCHO_E_ARG, "null context");
  if (enable && ctx->ev.empty()) {
    const size_t pairs = 4096;
    ctx->ev.resize(2 * pairs, nullptr);
    for (auto& e : ctx->ev) PT_HIP(hipEventCreate(&e));
    ctx->ev_n.assign(pairs, 0);
  }
  ctx->profiling = enable != 0;
  return PTYCHO_OK;
}

int ptycho_profile_read(ptycho_ctx* ctx, double* total_ms, int64_t* launches, int64_t* positions) {
  if (!ctx) return fail(PTYCHO_E_ARG, "null context");
  PT_HIP(hipStreamSynchronize(ctx->stream));
  double tot = 0.0;
  int64_t np = 0;
  for (size_t k = 0; k < ctx->ev_used; ++k) {
    float ms = 0.f;
    PT_HIP(hipEventElapsedTime(&ms, ctx->ev[2 * k], ctx->ev[2 * k + 1]));
    tot += ms;
    np += ctx->ev_n[k];
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = static_cast<int64_t>(ctx->ev_used);
  if (positions) *positions = np;
  ctx->ev_used = 0;
  ctx->dropped = 0;
  return PTYCHO_OK;
}

int ptycho_validate_positions(const int32_t* host_pos, int32_t n, int32_t H, int32_t W, int32_t M) {
  if (n < 0 || (n > 0 && !host_pos)) return fail(PTYCHO_E_ARG, "bad position array");
  if (M < 1 || H < 1 || W < 1) return fail(PTYCHO_E_ARG, "bad sizes");
  return validate_windows_host(host_pos, n, H, W, M);
}

int ptycho_bin_positions(const int32_t* host_pos, int32_t n, int32_t H, int32_t W, int32_t M, int32_t tiles_y,
                         int32_t tiles_x, int32_t* host_tile_of_pos) {
  if (n < 0 || (n > 0 && (!host_pos || !host_tile_of_pos))) return fail(PTYCHO_E_ARG, "bad arrays");
  if (tiles_y < 1 || tiles_x < 1 || M < 2 || H < 1 || W < 1) return fail(PTYCHO_E_ARG, "bad tile grid");
  int rc = validate_windows_host(host_pos, n, H, W, M);
  if (rc != PTYCHO_OK) return rc;
  // Tile edges edge_k = floor(k*extent/count); the owner is the tile whose
  // half-open span holds the window centre.
  std::vector<int32_t> ey(tiles_y + 1), ex(tiles_x + 1);
  for (int k = 0; k <= tiles_y; ++k) ey[k] = static_cast<int32_t>(static_cast<int64_t>(k) * H / tiles_y);
  for (int k = 0; k <= tiles_x; ++k) ex[k] = static_cast<int32_t>(static_cast<int64_t>(k) * W / tiles_x);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t cy = host_pos[2 * i] + M / 2, cx = host_pos[2 * i + 1] + M / 2;
    int32_t a = 0, b = tiles_y - 1;  // last edge <= cy
    while (a < b) {
      const int32_t mid = (a + b + 1) / 2;
      if (ey[mid] <= cy) a = mid; else b = mid - 1;
    }
    int32_t c = 0, d = tiles_x - 1;
    while (c < d) {
      const int32_t mid = (c + d + 1) / 2;
      if (ex[mid] <= cx) c = mid; else d = mid - 1;
    }
    host_tile_of_pos[i] = a * tiles_x + c;
  }
  return PTYCHO_OK;
}

int ptycho_gd_step_size(const void* host_probe, int32_t M, const int32_t* host_pos, int32_t n, int32_t H,
                        int32_t W, int32_t S, double* alpha_out) {
  if (!host_probe || !alpha_out || n < 0 || (n > 0 && !host_pos)) return fail(PTYCHO_E_ARG, "bad arguments");
  if (M < 1 || M > 4096 || H < 1 || W < 1 || S < 1) return fail(PTYCHO_E_ARG, "bad sizes");
  int rc = validate_windows_host(host_pos, n, H, W, M);
  if (rc != PTYCHO_OK) return rc;
  // |P|^2 in double from the complex64 values, then the coverage sum_i |P(r - r_i)|^2 per pixel
  const float* p = static_cast<const float*>(host_probe);
  std::vector<double> p2(static_cast<size_t>(M) * M);
  for (size_t q = 0; q < p2.size(); ++q) {
    const double re = p[2 * q], im = p[2 * q + 1];
    p2[q] = re * re + im * im;
  }
  std::vector<double> cover(static_cast<size_t>(H) * W, 0.0);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t y0 = host_pos[2 * i], x0 = host_pos[2 * i + 1];
    for (int32_t y = 0; y < M; ++y) {
      double* row = cover.data() + static_cast<size_t>(y0 + y) * W + x0;
      const double* src = p2.data() + static_cast<size_t>(y) * M;
      for (int32_t x = 0; x < M; ++x) row[x] += src[x];
    }
  }
  double peak = 0.0;
  for (double c : cover) peak = c > peak ? c : peak;
  if (!(peak > 0.0) || !std::isfinite(peak))
    return fail(PTYCHO_E_ARG, "no pixel is covered by a non-zero probe: the step bound is infinite");
  *alpha_out = 1.0 / (2.0 * static_cast<double>(M) * M * S * peak);
  return PTYCHO_OK;
}

// ---------------------------------------------------------------------------
// batched reconstructions
// ---------------------------------------------------------------------------
}  // extern "C"

struct ptycho_batch {
  int nrecon = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 256;
  std::vector<ptycho_recon> host;
  ptycho::BatchRecon* d_recs = nullptr;
  int* d_items = nullptr;
  int nitems = 0;
  double* d_item_loss = nullptr;
  double* d_losses = nullptr;
  double* d_hist = nullptr;
  int hist_rows = 0;
  int* d_iter = nullptr;
  float2* d_h = nullptr;     // nrecon * 128 entries
  float2* d_tw64 = nullptr;
  float2* d_tw128 = nullptr;
  unsigned* d_status = nullptr;
  struct Class {
    int M = 0, item0 = 0, nitems = 0, smax = 1, grid = 0, grid_default = 0, ws_grid = 0;
    float2* ws = nullptr;
  } cls[2];                  // [0] M = 64, [1] M = 128
  hipStream_t side = nullptr;  // the 128-window launch runs here, beside the 64-window one
  hipEvent_t fork = nullptr, join = nullptr;
  int* d_bounds = nullptr;   // per class: 9 item indices splitting its items into 8 parts of equal cost
  int* d_next = nullptr;     // per class: 8 queue counters
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void free_batch(ptycho_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  void* ptrs[] = {b->d_recs, b->d_items, b->d_item_loss, b->d_losses, b->d_hist, b->d_iter, b->d_h,
                  b->d_tw64, b->d_tw128, b->d_status, b->cls[0].ws, b->cls[1].ws, b->d_bounds, b->d_next};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->join) (void)hipEventDestroy(b->join);
  if (b->side) (void)hipStreamDestroy(b->side);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

std::vector<float2> twiddles(int M) {
  std::vector<float2> tw(M);
  for (int e = 0; e < M; ++e) {
    const double ang = -2.0 * kPi * e / M;
    tw[e] = make_float2(static_cast<float>(std::cos(ang)), static_cast<float>(std::sin(ang)));
  }
  return tw;
}

int batch_enqueue_loss_grad(ptycho_batch* b, double* losses) {
  PT_HIP(ptycho::launch_batch_elementwise(b->d_recs, b->nrecon, 0, nullptr, b->stream));
  // the two window sizes run side by side (fork/join through events, also under graph capture)
  const bool both = b->cls[0].nitems > 0 && b->cls[1].nitems > 0;
  if (both) {
    PT_HIP(hipEventRecord(b->fork, b->stream));
    PT_HIP(hipStreamWaitEvent(b->side, b->fork, 0));
  }
  for (auto& c : b->cls) {
    if (c.nitems == 0) continue;
    hipStream_t st = (both && c.M == 128) ? b->side : b->stream;
    ptycho::BatchArgs a{};
    a.recs = b->d_recs;
    a.items = b->d_items;
    a.item0 = c.item0;
    a.nitems = c.nitems;
    a.smax = c.smax;
    a.tw = c.M == 64 ? b->d_tw64 : b->d_tw128;
    a.ws = c.ws;
    a.item_loss = b->d_item_loss;
    a.status = b->d_status;
    const int ci = c.M == 64 ? 0 : 1;
    a.bounds = b->d_bounds + 9 * ci;
    a.next = b->d_next + 8 * ci;
    PT_HIP(ptycho::launch_copy_ints(a.bounds, a.next, 8, st));  // reset the queues (a kernel node)
    PT_HIP(ptycho::launch_batch(a, c.M, c.grid, st));
  }
  if (both) {
    PT_HIP(hipEventRecord(b->join, b->side));
    PT_HIP(hipStreamWaitEvent(b->stream, b->join, 0));
  }
  PT_HIP(ptycho::launch_batch_finalize(b->d_recs, b->d_item_loss, losses ? losses : b->d_losses, b->d_hist, b->d_iter,
                                       b->hist_rows, b->nrecon, b->stream));
  return PTYCHO_OK;
}

int batch_enqueue_update(ptycho_batch* b) {
  PT_HIP(ptycho::launch_batch_elementwise(b->d_recs, b->nrecon, 1, b->d_iter, b->stream));
  return PTYCHO_OK;
}

}  // namespace

extern "C" {

int ptycho_batch_create(ptycho_batch** out, const ptycho_recon* recons, int32_t nrecon, int32_t history_rows) {
  if (!out) return fail(PTYCHO_E_ARG, "null output pointer");
  *out = nullptr;
  if (nrecon < 0 || (nrecon > 0 && !recons)) return fail(PTYCHO_E_ARG, "bad reconstruction array");
  if (history_rows < 0) return fail(PTYCHO_E_ARG, "negative history length");
  int64_t total_items = 0;
  for (int r = 0; r < nrecon; ++r) {
    const ptycho_recon& R = recons[r];
    if (R.M != 64 && R.M != 128) return fail(PTYCHO_E_UNSUPPORTED, "reconstruction %d: window size %d", r, R.M);
    if (R.S < 1 || R.S > 64) return fail(PTYCHO_E_UNSUPPORTED, "reconstruction %d: %d slices", r, R.S);
    if (R.reserved != 0 || R.n < 0) return fail(PTYCHO_E_ARG, "reconstruction %d: bad count", r);
    if (R.H < R.M || R.W < R.M || R.ld < R.W || (R.S > 1 && R.slice_stride < static_cast<int64_t>(R.H) * R.ld))
      return fail(PTYCHO_E_SHAPE, "reconstruction %d: object %dx%d with strides (%lld, %lld)", r, R.H, R.W,
                  static_cast<long long>(R.slice_stride), static_cast<long long>(R.ld));
    if (R.ld * R.M >= (int64_t(1) << 31)) return fail(PTYCHO_E_SHAPE, "reconstruction %d: row stride too large", r);
    if (!R.obj || !R.grad || !R.probe || (R.n > 0 && (!R.pos || !R.meas)))
      return fail(PTYCHO_E_ARG, "reconstruction %d: null pointer", r);
    if (R.obj == R.grad) return fail(PTYCHO_E_ARG, "reconstruction %d: gradient aliases the object", r);
    if (!(R.pixel_A > 0) || !std::isfinite(R.wavelength_A) || !std::isfinite(R.dz_A) || !std::isfinite(R.alpha))
      return fail(PTYCHO_E_ARG, "reconstruction %d: invalid physics or step", r);
    total_items += R.n;
  }
  if (nrecon > 0) {  // the buffers behind the descriptors (needs the device)
    int device = 0;
    PT_HIP(hipGetDevice(&device));
    for (int r = 0; r < nrecon; ++r) {
      const ptycho_recon& R = recons[r];
      const size_t obj_bytes = span_elems(R.S, R.H, R.W, R.slice_stride, R.ld) * sizeof(float2);
      const size_t M2 = static_cast<size_t>(R.M) * R.M;
      PT_BUF(device, R.obj, obj_bytes, "reconstruction object");
      PT_BUF(device, R.grad, obj_bytes, "reconstruction gradient");
      PT_BUF(device, R.probe, M2 * sizeof(float2), "reconstruction probe");
      PT_BUF(device, R.pos, 2 * static_cast<size_t>(R.n) * sizeof(int32_t), "reconstruction positions");
      PT_BUF(device, R.meas, static_cast<size_t>(R.n) * M2 * sizeof(float), "reconstruction measurements");
    }
  }
  if (total_items >= (int64_t(1) << 30)) return fail(PTYCHO_E_CAPACITY, "too many positions");
  ptycho_batch* b = new ptycho_batch();
  b->nrecon = nrecon;
  b->host.assign(recons, recons + nrecon);
  b->hist_rows = history_rows;
  hipError_t e;
  int dev = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess ||
      (e = hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming)) != hipSuccess) {
    free_batch(b);
    return hip_fail(e, "batch stream");
  }
  b->device = dev;
  // work list grouped by window size, then reconstruction, then position
  std::vector<ptycho::BatchRecon> recs(nrecon);
  std::vector<int> bounds(18, 0);
  std::vector<int> items;
  items.reserve(2 * total_items);
  std::vector<float2> htab(static_cast<size_t>(nrecon) * 128);
  for (int ci = 0; ci < 2; ++ci) {
    auto& c = b->cls[ci];
    c.M = ci == 0 ? 64 : 128;
    c.item0 = static_cast<int>(items.size() / 2);
    for (int r = 0; r < nrecon; ++r) {
      const ptycho_recon& R = recons[r];
      if (R.M != c.M) continue;
      ptycho::BatchRecon& D = recs[r];
      D.M = R.M;
      D.S = R.S;
      D.H = R.H;
      D.W = R.W;
      D.n = R.n;
      D.item0 = static_cast<int>(items.size() / 2);
      D.slice_stride = R.slice_stride;
      D.ld = R.ld;
      D.obj = static_cast<float2*>(R.obj);
      D.grad = static_cast<float2*>(R.grad);
      D.probe = static_cast<const float2*>(R.probe);
      D.pos = R.pos;
      D.meas = R.meas;
      D.alpha = static_cast<float>(R.alpha);
      for (int k = 0; k < R.M; ++k) {
        const double f = fft_freq(k, R.M, R.pixel_A);
        const double ph = -kPi * R.wavelength_A * R.dz_A * f * f;
        htab[static_cast<size_t>(r) * 128 + k] = make_float2(static_cast<float>(std::cos(ph)), static_cast<float>(std::sin(ph)));
      }
      for (int p = 0; p < R.n; ++p) {
        items.push_back(r);
        items.push_back(p);
      }
      if (R.S > c.smax) c.smax = R.S;
    }
    c.nitems = static_cast<int>(items.size() / 2) - c.item0;
    // 8 contiguous parts of equal cost, one per XCD queue: an item costs 4S - 2 transforms
    {
      double total = 0.0;
      for (int k = 0; k < c.nitems; ++k) total += 4.0 * recons[items[2 * (c.item0 + k)]].S - 2.0;
      double acc = 0.0;
      int x = 1;
      bounds[9 * ci] = 0;
      for (int k = 0; k < c.nitems && x < 8; ++k) {
        acc += 4.0 * recons[items[2 * (c.item0 + k)]].S - 2.0;
        while (x < 8 && acc >= total * x / 8.0) bounds[9 * ci + x++] = k + 1;
      }
      while (x <= 8) bounds[9 * ci + x++] = c.nitems;
    }
    c.grid_default = b->num_cu * (c.M == 64 ? 2 : 1);
    c.ws_grid = c.grid_default * 2;  // the autotuner may pick up to twice the default
    c.grid = c.nitems < c.grid_default ? c.nitems : c.grid_default;
  }
  b->nitems = static_cast<int>(items.size() / 2);
  const auto tw64 = twiddles(64), tw128 = twiddles(128);
  auto alloc = [&](void** p, size_t bytes) -> bool {
    return bytes == 0 || (e = hipMalloc(p, bytes)) == hipSuccess;
  };
  bool ok = alloc(reinterpret_cast<void**>(&b->d_recs), recs.size() * sizeof(ptycho::BatchRecon)) &&
            alloc(reinterpret_cast<void**>(&b->d_items), items.size() * sizeof(int)) &&
            alloc(reinterpret_cast<void**>(&b->d_item_loss), static_cast<size_t>(b->nitems) * sizeof(double)) &&
            alloc(reinterpret_cast<void**>(&b->d_losses), static_cast<size_t>(nrecon) * sizeof(double)) &&
            alloc(reinterpret_cast<void**>(&b->d_hist), static_cast<size_t>(history_rows) * nrecon * sizeof(double)) &&
            alloc(reinterpret_cast<void**>(&b->d_iter), sizeof(int)) &&
            alloc(reinterpret_cast<void**>(&b->d_h), htab.size() * sizeof(float2)) &&
            alloc(reinterpret_cast<void**>(&b->d_tw64), 64 * sizeof(float2)) &&
            alloc(reinterpret_cast<void**>(&b->d_tw128), 128 * sizeof(float2)) &&
            alloc(reinterpret_cast<void**>(&b->d_status), sizeof(unsigned)) &&
            alloc(reinterpret_cast<void**>(&b->d_bounds), bounds.size() * sizeof(int)) &&
            alloc(reinterpret_cast<void**>(&b->d_next), 16 * sizeof(int));
  for (auto& c : b->cls)
    ok = ok && (c.nitems == 0 || c.smax < 2 ||
                alloc(reinterpret_cast<void**>(&c.ws),
                      static_cast<size_t>(c.ws_grid) * ptycho::ws_slots(c.smax, 1) * c.M * c.M * sizeof(float2)));
  if (!ok) {
    free_batch(b);
    return fail(PTYCHO_E_NOMEM, "batch allocation failed: %s", hipGetErrorString(e));
  }
  for (int r = 0; r < nrecon; ++r) recs[r].h = b->d_h + static_cast<size_t>(r) * 128;
  if (!history_rows) b->d_hist = nullptr;
  const int zero = 0;
  const unsigned uzero = 0;
  if ((!recs.empty() && (e = hipMemcpy(b->d_recs, recs.data(), recs.size() * sizeof(ptycho::BatchRecon),
                                       hipMemcpyHostToDevice)) != hipSuccess) ||
      (!items.empty() &&
       (e = hipMemcpy(b->d_items, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess) ||
      (!htab.empty() &&
       (e = hipMemcpy(b->d_h, htab.data(), htab.size() * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess) ||
      (e = hipMemcpy(b->d_tw64, tw64.data(), 64 * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b->d_tw128, tw128.data(), 128 * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b->d_iter, &zero, sizeof zero, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b->d_bounds, bounds.data(), bounds.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b->d_status, &uzero, sizeof uzero, hipMemcpyHostToDevice)) != hipSuccess) {
    free_batch(b);
    return hip_fail(e, "batch upload");
  }
  *out = b;
  return PTYCHO_OK;
}

int ptycho_batch_destroy(ptycho_batch* b) {
  if (!b) return PTYCHO_OK;
  (void)hipStreamSynchronize(b->stream);
  free_batch(b);
  return PTYCHO_OK;
}

int ptycho_batch_set_grid(ptycho_batch* b, int32_t M, int32_t grid) {
  if (!b) return fail(PTYCHO_E_ARG, "null batch");
  if (M != 64 && M != 128) return fail(PTYCHO_E_UNSUPPORTED, "window size %d", M);
  auto& c = b->cls[M == 64 ? 0 : 1];
  if (grid < 0 || grid > c.ws_grid) return fail(PTYCHO_E_ARG, "grid %d outside [0, %d]", grid, c.ws_grid);
  if (b->exec) return fail(PTYCHO_E_ARG, "the launch shape is frozen once a graph is captured");
  const int g = grid == 0 ? c.grid_default : grid;
  c.grid = c.nitems < g ? c.nitems : g;
  return PTYCHO_OK;
}

int ptycho_batch_get_grid(const ptycho_batch* b, int32_t M) {
  if (!b || (M != 64 && M != 128)) return -1;
  return b->cls[M == 64 ? 0 : 1].grid;
}

int ptycho_batch_loss_grad(ptycho_batch* b, double* losses) {
  if (!b) return fail(PTYCHO_E_ARG, "null batch");
  PT_BUF(b->device, losses, static_cast<size_t>(b->nrecon) * sizeof(double), "losses");
  return batch_enqueue_loss_grad(b, losses);
}

int ptycho_batch_update(ptycho_batch* b) {
  if (!b) return fail(PTYCHO_E_ARG, "null batch");
  return batch_enqueue_update(b);
}

int ptycho_batch_step(ptycho_batch* b) {
  if (!b) return fail(PTYCHO_E_ARG, "null batch");
  int rc = batch_enqueue_loss_grad(b, nullptr);
  return rc != PTYCHO_OK ? rc : batch_enqueue_update(b);
}

int ptycho_batch_capture(ptycho_batch* b) {
  if (!b) return fail(PTYCHO_E_ARG, "null batch");
  if (b->exec) return PTYCHO_OK;
  PT_HIP(hipStreamSynchronize(b->stream));
  PT_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  int rc = batch_enqueue_loss_grad(b, nullptr);
  if (rc == PTYCHO_OK) rc = batch_enqueue_update(b);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (rc != PTYCHO_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t x = nullptr;
  if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(e, "hipGraphInstantiate");
  }
  b->graph = g;
  b->exec = x;
  return PTYCHO_OK;
}

int ptycho_batch_replay(ptycho_batch* b) {
  if (!b) return fail(PTYCHO_E_ARG, "null batch");
  if (!b->exec) return fail(PTYCHO_E_ARG, "no captured graph");
  PT_HIP(hipGraphLaunch(b->exec, b->stream));
  return PTYCHO_OK;
}

int ptycho_batch_sync(ptycho_batch* b) {
  if (!b) return fail(PTYCHO_E_ARG, "null batch");
  PT_HIP(hipStreamSynchronize(b->stream));
  unsigned st = 0;
  PT_HIP(hipMemcpy(&st, b->d_status, sizeof st, hipMemcpyDeviceToHost));
  if (st) {
    const unsigned z = 0;
    PT_HIP(hipMemcpy(b->d_status, &z, sizeof z, hipMemcpyHostToDevice));
    return fail(PTYCHO_E_BOUNDS, "a window left its object (status 0x%x)", st);
  }
  return PTYCHO_OK;
}

int ptycho_batch_history(ptycho_batch* b, double* host_out, int32_t* rows_out) {
  if (!b) return fail(PTYCHO_E_ARG, "null batch");
  PT_HIP(hipStreamSynchronize(b->stream));
  int it = 0;
  PT_HIP(hipMemcpy(&it, b->d_iter, sizeof it, hipMemcpyDeviceToHost));
  const int rows = it < b->hist_rows ? it : b->hist_rows;
  if (rows_out) *rows_out = rows;
  if (host_out && rows > 0)
    PT_HIP(hipMemcpy(host_out, b->d_hist, static_cast<size_t>(rows) * b->nrecon * sizeof(double),
                     hipMemcpyDeviceToHost));
  return PTYCHO_OK;
}

int ptycho_batch_reset_history(ptycho_batch* b) {
  if (!b) return fail(PTYCHO_E_ARG, "null batch");
  PT_HIP(ptycho::launch_set_int(b->d_iter, 0, b->stream));
  return PTYCHO_OK;
}

void* ptycho_batch_stream(const ptycho_batch* b) { return b ? static_cast<void*>(b->stream) : nullptr; }

int ptycho_check(ptycho_ctx* ctx, uint32_t* status_out) {
  if (!ctx) return fail(PTYCHO_E_ARG, "null context");
  PT_HIP(hipStreamSynchronize(ctx->stream));
  unsigned st = 0;
  PT_HIP(hipMemcpy(&st, ctx->d_status, sizeof st, hipMemcpyDeviceToHost));
  if (status_out) *status_out = st;
  if (st) {
    PT_HIP(ptycho::launch_clear_status(ctx->d_status, ctx->stream));
    PT_HIP(hipStreamSynchronize(ctx->stream));
    if (st & PTYCHO_STATUS_BOUNDS) return fail(PTYCHO_E_BOUNDS, "a window left the object (status 0x%x)", st);
    if (st & PTYCHO_STATUS_HALO) return fail(PTYCHO_E_HALO, "a window left the extended tile (status 0x%x)", st);
    return fail(PTYCHO_E_ASSIGN, "a window centre lay outside its tile (status 0x%x)", st);
  }
  return PTYCHO_OK;
}

}  // extern "C"
