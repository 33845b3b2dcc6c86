// ptycho_kernels.h -- internal launch interface between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace ptycho {

struct KernelArgs {
  int M, S, n;
  // object window source: element (s, y, x) at obj[s*slice_stride + y*ld + x], y, x local to the box
  const float2* obj;
  long long slice_stride, ld;
  int bh, bw;            // box extent that every window must lie in
  int oy, ox;            // box origin subtracted from the (global) positions
  int check_tile;        // also require the window centre inside [ty0,ty1) x [tx0,tx1)
  int ty0, ty1, tx0, tx1;
  unsigned oob_flag;     // status bit raised for a window outside the box
  const float2* probe;
  const int* pos;        // [n][2] global (y0, x0)
  const float2* tw;      // W_M^e, e in [0, M)
  const float2* h;       // separable propagator factor h[k], k in [0, M)
  float* intens;         // forward output [n][M][M]
  const float* meas;     // [n][M][M]
  double* loss_work;     // [n] per-position losses (always written by the gradient kernel)
  double* loss_pos;      // nullable [n]
  float2* grad;          // gradient, element (s, y, x) at grad[s*gslice + y*gld + x] (box-local)
  long long gslice, gld;
  float2* ws;            // per-block incident-wave store: grid * (S-1) * M*M
  unsigned* status;
};

hipError_t launch_fused(const KernelArgs& a, bool grad, int grid, hipStream_t st);
hipError_t launch_zero_slices(float2* g, int S, int H, int W, long long gslice, long long gld, hipStream_t st);
hipError_t launch_finalize_loss(const double* per, int n, double* loss, bool accumulate, hipStream_t st);
hipError_t launch_clear_status(unsigned* status, hipStream_t st);
hipError_t launch_tile_accumulate(const float2* tile, int S, int eh, int ew, float2* grad, long long gslice,
                                  long long gld, hipStream_t st);

}  // namespace ptycho
