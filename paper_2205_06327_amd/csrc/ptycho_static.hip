// ptycho_static.hip -- ptycho_loss_grad_static: the loss and object gradient
// of ptycho_loss_grad without a context and without any device allocation.
//
// Everything the fused kernel needs beyond the caller's inputs and outputs
// (DFT twiddles, propagator factors, the status word, per-position losses and
// the incident-wave store of the adjoint sweep) lives in one file-scope device
// array, `scratch`, of kScratchBytes per GPU.  Its device address is resolved
// once per device with hipGetSymbolAddress and cached; only that address is
// ever handed to kernels or runtime calls.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "../../include/ptycho.h"
#include "ptycho_host.h"
#include "ptycho_kernels.h"

using namespace ptycho::host;

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;
// layout of the array (byte offsets)
constexpr size_t kTwOff = 0;                    // W_M^e, M <= 128 float2
constexpr size_t kHOff = 1024;                  // separable propagator factor, M <= 128 float2
constexpr size_t kStatusOff = 2048;             // device status word
constexpr size_t kLossOff = 4096;               // per-position losses
constexpr int kMaxPositions = 1 << 20;          // 8 MiB of doubles
constexpr size_t kWaveOff = kLossOff + size_t(kMaxPositions) * sizeof(double) + (size_t(64) << 10);
constexpr size_t kWaveBytes = kScratchBytes - kWaveOff;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// The FP32 tables of one window size and slice thickness, computed in FP64 on the device and rounded
// once: tw[e] = exp(-2 pi i e / M) and h[e] = exp(-i pi lambda dz f_e^2), f = fftfreq(M, pixel)
// (the propagator of Section II-B's slice-to-slice step, H[ky,kx] = h[ky] h[kx]).
__global__ void static_tables_kernel(float2* __restrict__ tw, float2* __restrict__ h, int M, double lambda_dz,
                                     double pixel) {
  const int e = static_cast<int>(threadIdx.x);
  if (e >= M) return;
  double s, c;
  sincospi(-2.0 * e / M, &s, &c);
  tw[e] = make_float2(static_cast<float>(c), static_cast<float>(s));
  const double f = (e < M / 2 ? e : e - M) / (M * pixel);
  sincospi(-lambda_dz * f * f, &s, &c);
  h[e] = make_float2(static_cast<float>(c), static_cast<float>(s));
}

struct StaticDevice {
  unsigned char* ptr = nullptr;  // device address of `scratch` on this device
  int cus = 0;
};
std::mutex g_mu;
StaticDevice g_dev[kMaxDevices];

// The array's address and the CU count of the current device, resolved on the first call per device.
int static_device(StaticDevice* out) {
  int dev = 0;
  PT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PTYCHO_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  StaticDevice& d = g_dev[dev];
  if (d.ptr == nullptr) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    d.cus = cus > 0 ? cus : 256;
    d.ptr = static_cast<unsigned char*>(p);
  }
  *out = d;
  return PTYCHO_OK;
}

// Checkpoint interval and workgroup count for which the incident-wave store fits the array: the most
// workgroups (up to one per CU), then the shortest interval (the least recomputation).
void fit_wave_store(int M, int S, int cus, int* ck_out, int* grid_out) {
  const size_t slot = size_t(M) * M * sizeof(float2);
  const size_t slots = kWaveBytes / slot;
  int best_ck = 1, best_grid = 0;
  for (int ck = 1; ck <= S; ++ck) {
    const int per = ptycho::ws_slots(S, ck);
    const size_t g = per == 0 ? size_t(cus) : slots / per;
    const int grid = static_cast<int>(g < size_t(cus) ? g : size_t(cus));
    if (grid > best_grid) {
      best_grid = grid;
      best_ck = ck;
    }
  }
  *ck_out = best_ck;
  *grid_out = best_grid;
}

}  // namespace

extern "C" int ptycho_loss_grad_static(int32_t M, int32_t S, double wavelength_A, double dz_A, double pixel_A,
                                       void* stream, const void* obj, int32_t H, int32_t W, int64_t slice_stride,
                                       int32_t ld, const void* probe, const int32_t* pos, int32_t n,
                                       const float* meas, double* loss, double* loss_per_pos, void* grad,
                                       int64_t grad_slice_stride, int32_t grad_ld, uint32_t flags,
                                       const double* grad_scale) {
  // host validation first: a rejected call touches neither the runtime nor the device
  if (M != 64 && M != 128) return fail(PTYCHO_E_UNSUPPORTED, "window size %d not supported (64 or 128)", M);
  if (S < 1 || S > 64) return fail(PTYCHO_E_UNSUPPORTED, "slice count %d not supported (1..64)", S);
  if (!(pixel_A > 0) || !std::isfinite(pixel_A) || !std::isfinite(wavelength_A) || !std::isfinite(dz_A))
    return fail(PTYCHO_E_ARG, "invalid physics (wavelength %g, dz %g, pixel %g)", wavelength_A, dz_A, pixel_A);
  if (n < 0) return fail(PTYCHO_E_ARG, "negative position count");
  if (n > kMaxPositions)
    return fail(PTYCHO_E_CAPACITY, "%d positions exceed the %d of the static workspace", n, kMaxPositions);
  if (flags & ~PTYCHO_ACCUMULATE) return fail(PTYCHO_E_ARG, "unknown flags 0x%x", flags);
  if (!loss || !grad) return fail(PTYCHO_E_ARG, "null loss or gradient");
  if (n > 0 && (!obj || !probe || !pos || !meas)) return fail(PTYCHO_E_ARG, "null object, probe, positions or measurements");
  if (H < M || W < M) return fail(PTYCHO_E_SHAPE, "object %dx%d smaller than the %d window", H, W, M);
  if (ld < W) return fail(PTYCHO_E_SHAPE, "ld %d < W %d", ld, W);
  if (S > 1 && slice_stride < static_cast<int64_t>(H) * ld)
    return fail(PTYCHO_E_SHAPE, "slice stride %lld < H*ld", static_cast<long long>(slice_stride));
  if (static_cast<int64_t>(ld) * M >= (int64_t(1) << 31)) return fail(PTYCHO_E_SHAPE, "row stride %d too large", ld);
  if (grad_ld < W || (S > 1 && grad_slice_stride < static_cast<int64_t>(H) * grad_ld))
    return fail(PTYCHO_E_SHAPE, "gradient strides do not cover %dx%d", H, W);
  if (static_cast<int64_t>(grad_ld) * M >= (int64_t(1) << 31)) return fail(PTYCHO_E_SHAPE, "gradient row stride too large");
  if (grad == obj) return fail(PTYCHO_E_ARG, "gradient aliases the object");

  StaticDevice sd;
  int rc = static_device(&sd);
  if (rc != PTYCHO_OK) return rc;
  int dev = 0;
  PT_HIP(hipGetDevice(&dev));
  if (stream != nullptr) {  // the array's address is the current device's: the stream must run there too
    hipDevice_t sdev = 0;
    PT_HIP(hipStreamGetDevice(static_cast<hipStream_t>(stream), &sdev));
    if (sdev != dev) return fail(PTYCHO_E_ARG, "stream of device %d, current device %d", sdev, dev);
  }
  const size_t M2 = static_cast<size_t>(M) * M;
  if (n > 0) {
    PT_BUF(dev, obj, span_elems(S, H, W, slice_stride, ld) * sizeof(float2), "object");
    PT_BUF(dev, probe, M2 * sizeof(float2), "probe");
    PT_BUF(dev, pos, 2 * static_cast<size_t>(n) * sizeof(int32_t), "positions");
    PT_BUF(dev, meas, static_cast<size_t>(n) * M2 * sizeof(float), "measurements");
  }
  PT_BUF(dev, grad, span_elems(S, H, W, grad_slice_stride, grad_ld) * sizeof(float2), "gradient");
  PT_BUF(dev, loss, sizeof(double), "loss");
  PT_BUF(dev, loss_per_pos, static_cast<size_t>(n) * sizeof(double), "per-position losses");
  PT_BUF(dev, grad_scale, sizeof(double), "gradient scale");

  int ck = 1, grid = 0;
  fit_wave_store(M, S, sd.cus, &ck, &grid);
  if (grid < 1) return fail(PTYCHO_E_UNSUPPORTED, "%d slices of %dx%d waves do not fit the static workspace", S, M, M);

  hipStream_t st = static_cast<hipStream_t>(stream);
  float2* tw = reinterpret_cast<float2*>(sd.ptr + kTwOff);
  float2* hh = reinterpret_cast<float2*>(sd.ptr + kHOff);
  unsigned* status = reinterpret_cast<unsigned*>(sd.ptr + kStatusOff);
  double* per = reinterpret_cast<double*>(sd.ptr + kLossOff);
  float2* ws = reinterpret_cast<float2*>(sd.ptr + kWaveOff);

  static_tables_kernel<<<1, 128, 0, st>>>(tw, hh, M, wavelength_A * dz_A, pixel_A);
  PT_HIP(hipGetLastError());
  PT_HIP(ptycho::launch_clear_status(status, st));
  const bool acc = (flags & PTYCHO_ACCUMULATE) != 0;
  if (!acc) PT_HIP(ptycho::launch_zero_slices(static_cast<float2*>(grad), S, H, W, grad_slice_stride, grad_ld, st));
  if (n > 0) {
    ptycho::KernelArgs a{};
    a.M = M;
    a.S = S;
    a.n = n;
    a.obj = static_cast<const float2*>(obj);
    a.slice_stride = slice_stride;
    a.ld = ld;
    a.bh = H;
    a.bw = W;
    a.oob_flag = PTYCHO_STATUS_BOUNDS;
    a.probe = static_cast<const float2*>(probe);
    a.pos = pos;
    a.tw = tw;
    a.h = hh;
    a.meas = meas;
    a.loss_work = per;
    a.loss_pos = loss_per_pos;
    a.grad = static_cast<float2*>(grad);
    a.gslice = grad_slice_stride;
    a.gld = grad_ld;
    a.ws = ws;
    a.ck = ck;
    a.status = status;
    a.grad_scale = grad_scale;
    PT_HIP(ptycho::launch_fused(a, ptycho::kModeLossGrad, n < grid ? n : grid, st));
  }
  PT_HIP(ptycho::launch_finalize_loss(per, n, loss, acc, st));
  return PTYCHO_OK;
}
