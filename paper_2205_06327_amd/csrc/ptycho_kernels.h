// ptycho_kernels.h -- internal launch interface between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace ptycho {

// what a fused launch produces per position
constexpr int kModeIntensity = 0;  // |Psi|^2
constexpr int kModeLoss = 1;       // f_i only
constexpr int kModeLossGrad = 2;   // f_i and the adjoint gradient
constexpr int kModeLossGradProbe = 3;  // f_i, the object gradient and the probe gradient

// Wave-store slots (M*M complex each) per workgroup for S slices with the
// incident waves checkpointed every ck slices: the checkpoints psi_ck,
// psi_2ck, ..., psi_last (last = the first slice of the last segment), the
// inner waves of one segment, and, when earlier segments are recomputed, one
// slot for the adjoint wave.  ck = 1 keeps all S - 1 waves.
__host__ __device__ constexpr int ws_slots(int S, int ck) {
  return S <= 1 ? 0
                : ((S - 1) / ck) + ((ck < S ? ck : S) - 1) + (((S - 1) / ck) > 0 && ck > 1 ? 1 : 0);
}

// Device copy of a tile descriptor (all tiles of one launch).
struct TileDesc {
  int ty0, ty1, tx0, tx1;  // tile, global pixels
  int ey0, ex0, eh, ew;    // extended box
  float2* grad;            // [S][eh][ew] dense
  long long gslice, gld;
};
constexpr int kMaxTiles = 4096;

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
  long long probe_stride;  // 0: one probe for all positions; else position p uses probe + p*probe_stride
  const int* pos;        // [n][2] global (y0, x0)
  const float2* tw;      // W_M^e, e in [0, M)
  const float2* h;       // separable propagator factor h[k], k in [0, M)
  float* intens;         // forward output [n][M][M]
  const float* meas;     // [n][M][M]
  double* loss_work;     // [n] per-position losses (always written by the gradient kernel)
  double* loss_pos;      // nullable [n]
  float2* grad;          // gradient, element (s, y, x) at grad[s*gslice + y*gld + x] (box-local)
  long long gslice, gld;
  float2* ws;            // per-block incident-wave store: grid * ws_slots(S, ck) * M*M
  int ck;                // checkpoint interval of the incident waves
  unsigned* status;
  const double* grad_scale;  // nullable device scalar multiplying the gradient
  float2* probe_part;    // probe-gradient mode: per-workgroup partial sums, grid * M*M (layout-A order)
  // all-tiles mode (tiles != nullptr): the gradient of position p goes to tiles[tile_of_pos[p]]
  const TileDesc* tiles;
  const int* tile_of_pos;
  int ntiles;
};

// One reconstruction of a batch (device copy of the public descriptor plus
// the position of its items in the work list and its propagator table).
struct BatchRecon {
  int M, S, H, W, n, item0;
  long long slice_stride, ld;
  float2* obj;
  float2* grad;
  const float2* probe;
  const int* pos;
  const float* meas;
  const float2* h;
  float alpha;
};

struct BatchArgs {
  const BatchRecon* recs;
  const int* items;      // (reconstruction, position) pairs, grouped by reconstruction
  int item0, nitems;     // this launch's slice of the list (one window size)
  int smax;              // largest slice count in the slice
  const float2* tw;
  float2* ws;            // grid * ws_slots(smax, 1) * M*M
  double* item_loss;     // one per item of the whole list
  unsigned* status;
  // Work queues: items [bounds[x], bounds[x+1]) of this launch (relative to
  // item0) are served to the workgroups of XCD x through the counter next[x]
  // (reset to bounds[x] before the launch).  The bounds split the items into
  // 8 parts of equal cost ((4S - 2) transforms per item); with fewer than 8
  // workgroups everything is in part 0.
  const int* bounds;     // [9]
  int* next;             // [8]
};

hipError_t launch_fused(const KernelArgs& a, int mode, int grid, hipStream_t st);
hipError_t launch_batch(const BatchArgs& a, int M, int grid, hipStream_t st);
hipError_t launch_batch_finalize(const BatchRecon* recs, const double* item_loss, double* losses, double* hist,
                                 const int* iter, int hist_rows, int nrecon, hipStream_t st);
hipError_t launch_batch_elementwise(const BatchRecon* recs, int nrecon, int mode, int* iter, hipStream_t st);
hipError_t launch_set_int(int* p, int v, hipStream_t st);
hipError_t launch_copy_ints(const int* src, int* dst, int n, hipStream_t st);
hipError_t launch_zero_slices(float2* g, int S, int H, int W, long long gslice, long long gld, hipStream_t st);
hipError_t launch_finalize_loss(const double* per, int n, double* loss, bool accumulate, hipStream_t st);
hipError_t launch_clear_status(unsigned* status, hipStream_t st);
hipError_t launch_shift_probes(const float2* probe, const float* shifts, int n, int M, const float2* tw, float2* out,
                               hipStream_t st);
hipError_t launch_zero_tiles(const TileDesc* tiles, int ntiles, int S, hipStream_t st);
hipError_t launch_probe_reduce(const float2* part, int parts, int M, float2* probe_grad, bool accumulate,
                               hipStream_t st);
hipError_t launch_potential(int mode, float sigma, int S, int H, int W, const float* V, long long vs, long long vld,
                            float2* t_out, const float2* t_in, long long ts, long long tld, const float2* g,
                            long long gs, long long gld, float* gv, long long gvs, long long gvld, hipStream_t st);
hipError_t launch_box_exchange(const float2* src, long long sslice, long long sld, float2* dst, long long dslice,
                               long long dld, int S, int oh, int ow, bool replace, float alpha, hipStream_t st);
hipError_t launch_tile_accumulate(const float2* tile, int S, int eh, int ew, float2* grad, long long gslice,
                                  long long gld, hipStream_t st);

}  // namespace ptycho
