/*
 * ptycho.h -- C ABI of the MI355X (gfx950) multislice ptychography hot path.
 *
 * Problem (Wang et al., "Image Gradient Decomposition for Parallel and
 * Memory-Efficient Ptychographic Reconstruction", SC22):
 *   Section II-B, Eq. 1:  F(V) = sum_i ( |y_i| - |G(p_i, V)| )^2
 *   Section II-B (text after Eq. 1): G runs, slice after slice, a Fourier
 *       transform and an inverse Fourier transform; each slice's output is the
 *       next slice's input; the detector compares magnitudes of the far field.
 *   Section III, Eq. 2: dF/dV = sum_i df_i/dV, each term non-zero only inside
 *       the window of probe location i, so per-position gradients are
 *       scatter-added into the image gradient.
 *   Section III (tiles + halos): the image gradient and the probe locations
 *       are divided into tiles; each tile is extended by a halo that covers its
 *       probe windows; tile gradients of overlapping regions are added.
 *   Section IV: with separately held tile buffers, directional forward (add)
 *       and backward (replace) passes leave the summed gradient on every
 *       tile's box (ptycho_box_exchange); Alg. 1 updates each tile with its
 *       own and its accumulated gradients (ptycho_box_axpy).
 *
 * Model computed by this library (per position i with window top-left (y0, x0)):
 *   psi_0 = probe;  phi_s = psi_s * t_s[y0:y0+M, x0:x0+M]
 *   psi_{s+1} = IDFT( H * DFT(phi_s) ),  H[ky,kx] = exp(-i pi lambda dz (ky^2+kx^2)),
 *               k = fftfreq(M, d = pixel)           (s = 0 .. S-2)
 *   Psi = DFT(phi_{S-1});  I = |Psi|^2   (unnormalised DFT, DC at [0,0], no shift)
 *   f_i = sum_q ( |Psi| - sqrt(meas) )^2
 *   grad = dF/dRe(t) + i dF/dIm(t)      (complex gradient w.r.t. the transmissions)
 *
 * Data types and layouts (all arrays are DEVICE pointers unless marked host):
 *   complex values are interleaved float pairs (re, im) = "float2" below.
 *   object:    slices of complex64, element (s, y, x) at obj[s*slice_stride + y*ld + x]
 *   probe:     complex64 [M][M], row-major
 *   positions: int32 [n][2] = (y0, x0) window top-left corners, in the object's
 *              coordinates (global object coordinates for ptycho_tile_grad)
 *   intensities / measurements: float32 [n][M][M], detector order as above
 *   gradient:  complex64 with its own (slice_stride, ld)
 *
 * Ownership: the caller allocates and frees every array; the library keeps no
 * pointer beyond the call's stream work.  A context owns its device tables and
 * its workspace (allocated in ptycho_create, ptycho_reserve and
 * ptycho_set_checkpoint only), so the hot calls allocate nothing and are
 * stream-ordered and asynchronous.
 *
 * Errors: every call returns PTYCHO_OK (0) or a negative code; a call that
 * fails host validation enqueues nothing.  ptycho_last_error() returns a
 * thread-local message for the last failure.  Host validation includes the
 * caller's buffers: each must be device memory of the context's device,
 * managed memory or pinned host memory (else PTYCHO_E_ARG: a pageable host
 * pointer would reach the kernels as an invalid address), and the bytes a
 * call addresses from it must lie inside its allocation where the runtime
 * knows the allocation (else PTYCHO_E_SHAPE).  ptycho_copy_box is the
 * exception: it also takes pageable host memory.  Windows that leave the object,
 * the extended tile or the tile (conditions only visible on the device because
 * positions live in device memory) are skipped by the kernels without any
 * memory access and recorded in a device status word; ptycho_check()
 * synchronises the context stream and reports it.
 *
 * Thread safety: one context must not be used by several host threads at once.
 */
#ifndef PTYCHO_H
#define PTYCHO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ptycho_ctx ptycho_ctx;

enum {
  PTYCHO_OK = 0,
  PTYCHO_E_ARG = -1,          /* null pointer, negative size, bad flag */
  PTYCHO_E_SHAPE = -2,        /* inconsistent sizes or strides */
  PTYCHO_E_BOUNDS = -3,       /* a window leaves the object */
  PTYCHO_E_HALO = -4,         /* a window leaves the extended tile (halo too small) */
  PTYCHO_E_ASSIGN = -5,       /* a window centre lies outside its tile */
  PTYCHO_E_UNSUPPORTED = -6,  /* unsupported window size or slice count */
  PTYCHO_E_HIP = -7,          /* HIP runtime error */
  PTYCHO_E_NOMEM = -8,        /* device allocation failed (create/reserve only) */
  PTYCHO_E_CAPACITY = -9      /* more positions than the context reserved */
};

/* flags for ptycho_loss_grad / ptycho_tile_grad */
#define PTYCHO_ACCUMULATE 1u   /* add into grad and *loss instead of overwriting them */

/* Status bits reported by ptycho_check (device status word). */
#define PTYCHO_STATUS_BOUNDS 1u
#define PTYCHO_STATUS_HALO 2u
#define PTYCHO_STATUS_ASSIGN 4u

/*
 * ptycho_create: a context for windows of M x M pixels (M in {64, 128}) and
 * S >= 1 slices (S <= 64), with the Fresnel propagator of one slice thickness
 * dz_A for electrons of wavelength wavelength_A on pixels of pixel_A (all in
 * Angstrom).  The FP32 DFT twiddles and the separable propagator factors are
 * computed in FP64 on the host and rounded once.  `stream` is a hipStream_t
 * (NULL = default stream) on which every later call of this context runs.
 * max_positions bounds n of a single loss/gradient call (the context keeps a
 * per-position loss array of that length); 0 picks a default of 4096.
 * The context also owns the incident-wave store of the adjoint sweep:
 * (#CUs) x (S-1) x M*M complex64 (see ptycho_set_checkpoint), and the
 * probe-gradient partial sums, (#CUs) x M*M complex64.
 * Returns PTYCHO_E_UNSUPPORTED for other M or S, PTYCHO_E_NOMEM if the
 * workspace cannot be allocated.
 */
int ptycho_create(ptycho_ctx** out, int32_t M, int32_t S, double wavelength_A, double dz_A,
                  double pixel_A, int32_t max_positions, void* stream);
int ptycho_destroy(ptycho_ctx* ctx);
int ptycho_set_stream(ptycho_ctx* ctx, void* stream);
/* Grow the context's per-call position capacity (allocates; not for hot loops). */
int ptycho_reserve(ptycho_ctx* ctx, int32_t max_positions);
/*
 * ptycho_box_axpy: dst += alpha * src on the overlap of two boxes, with the
 * same buffer conventions and checks as ptycho_box_exchange (E_ARG also for
 * a non-finite alpha).  The tile-local updates of Alg. 1 use it:
 * AccBuf_k += dF/dV_k (alpha = 1) and V_k -= step * dF/dV_k (alpha = -step).
 */
int ptycho_box_axpy(ptycho_ctx* ctx, int32_t S, float alpha, const void* src, int32_t sy0, int32_t sx0, int32_t sh,
                    int32_t sw, int64_t s_slice_stride, int32_t s_ld, void* dst, int32_t dy0, int32_t dx0, int32_t dh,
                    int32_t dw, int64_t d_slice_stride, int32_t d_ld);

/*
 * Real-potential parametrisation (Section II-B: V is the sample's scattering
 * potential; the slices enter the model through their transmissions):
 *   ptycho_potential_transmission:  t = exp(i sigma V)
 *   ptycho_potential_gradient:      dF/dV = sigma * Im(conj(t) * G), with
 *       G = dF/dRe t + i dF/dIm t the gradient of ptycho_loss_grad (the chain
 *       rule through t = exp(i sigma V)).
 * V and dF/dV are float32 [S][H][W] (ctx->S slices) with (slice_stride, ld)
 * in floats; t and G complex64 likewise.  Device arrays owned by the caller;
 * stream-ordered; E_ARG / E_SHAPE on null pointers, non-finite sigma or
 * strides that do not cover H x W.
 */
int ptycho_potential_transmission(ptycho_ctx* ctx, int32_t H, int32_t W, float sigma, const float* V,
                                  int64_t v_slice_stride, int32_t v_ld, void* t, int64_t t_slice_stride,
                                  int32_t t_ld);
int ptycho_potential_gradient(ptycho_ctx* ctx, int32_t H, int32_t W, float sigma, const void* t,
                              int64_t t_slice_stride, int32_t t_ld, const void* grad_t, int64_t g_slice_stride,
                              int32_t g_ld, float* grad_V, int64_t gv_slice_stride, int32_t gv_ld);

/*
 * ptycho_copy_box: copies an h x w box of S complex64 slices between two
 * arrays, either of which may be host memory (pinned for asynchronous
 * transfers) or device memory: element (s, y, x) from
 * src[s*src_slice_stride + y*src_ld + x] to dst[s*dst_slice_stride + y*dst_ld + x].
 * One pitched copy per slice on the context stream (hipMemcpy2DAsync); the
 * streaming tile walk moves extended tiles of a host-resident object and
 * gradient with it.  E_ARG on null pointers, E_SHAPE on negative sizes or
 * strides that do not cover the box.
 */
int ptycho_copy_box(ptycho_ctx* ctx, int32_t S, int32_t h, int32_t w, const void* src, int64_t src_slice_stride,
                    int32_t src_ld, void* dst, int64_t dst_slice_stride, int32_t dst_ld);

/*
 * ptycho_set_checkpoint: how the gradient call obtains the incident waves
 * psi_s of its adjoint sweep (Eq. 2 needs psi_s at slice s, in reverse order).
 * The call always recomputes them from the probe and the object (nothing is
 * kept between calls); within a position, interval 1 (the default) parks every
 * wave of the forward sweep in the context's store, and interval k > 1 parks
 * only the wave entering every k-th slice plus the last segment's waves and
 * recomputes each earlier segment's inner waves from its checkpoint during the
 * adjoint sweep: ws_slots(S, k) instead of S - 1 slots of M*M complex per
 * workgroup (S = 16, k = 4: 7 instead of 15), for (k - 1)/k of the forward
 * transforms again.  Results equal those of interval 1 up to the order of the
 * gradient atomics.  Reallocates the store (synchronising the context stream);
 * E_ARG outside [1, 64].
 */
int ptycho_set_checkpoint(ptycho_ctx* ctx, int32_t interval);

/* Device bytes owned by the context (tables + workspace). */
int64_t ptycho_workspace_bytes(const ptycho_ctx* ctx);

/*
 * ptycho_forward: simulated far-field intensities I_i = |G(p_i, V)|^2
 * (Section II-B) for n positions; writes intens[n][M][M] (overwritten).
 * obj has H x W pixels per slice with the given strides (ld >= W,
 * slice_stride >= H*ld).  Windows outside [0,H)x[0,W) are skipped (their
 * intensities are left untouched) and flagged PTYCHO_STATUS_BOUNDS.
 * n == 0 is a no-op.
 */
int ptycho_forward(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride,
                   int32_t ld, const void* probe, const int32_t* pos, int32_t n, float* intens);

/*
 * ptycho_loss_grad: amplitude cost F (Eq. 1) and its gradient (Eq. 2).
 *   loss:         device double scalar; set to F (or F added when ACCUMULATE)
 *   loss_per_pos: nullable device double [n]; f_i per position (overwritten)
 *   grad:         device complex64 with (grad_slice_stride, grad_ld) over the
 *                 same H x W x S extent as obj; set to dF/dRe t + i dF/dIm t
 *                 (or added into it when ACCUMULATE).  It must not alias obj.
 *   meas:         measured intensities float32 [n][M][M] (non-negative).
 *   grad_scale:   nullable device double; when given, the gradient (not the
 *                 loss) is multiplied by it (the upstream factor of a chain rule).
 * Where |Psi| = 0 the direction Psi/|Psi| is taken as 0.
 * n must not exceed the context's reserved capacity (PTYCHO_E_CAPACITY).
 */
int ptycho_loss_grad(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride,
                     int32_t ld, const void* probe, const int32_t* pos, int32_t n, const float* meas,
                     double* loss, double* loss_per_pos, void* grad, int64_t grad_slice_stride,
                     int32_t grad_ld, uint32_t flags, const double* grad_scale);

/*
 * ptycho_loss_grad_static: ptycho_loss_grad without a context and without any
 * device allocation, for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc).
 * The arguments mean what they mean for ptycho_create (M, S, wavelength_A,
 * dz_A, pixel_A, stream) and ptycho_loss_grad (the rest, one probe for all
 * positions); results equal ptycho_loss_grad's up to the order of the
 * gradient atomics (and the last bit of the FP32 tables, which are built in
 * FP64 on the device here).
 *
 * Workspace: one device array of 256 MiB per GPU, built into the library and
 * held from the first call on that GPU until the process ends (the first call
 * on a device resolves its address; make it outside graph capture).  It holds
 * the tables, the status word, the per-position losses (hence at most 2^20
 * positions per call: PTYCHO_E_CAPACITY beyond) and the incident-wave store;
 * the checkpoint interval (see ptycho_set_checkpoint) and the number of
 * workgroups are chosen so that the store fits (M = 128, S = 16: interval 4).
 * Every call on a GPU uses the same array: calls that overlap on one GPU (two
 * streams, two host threads) race and must be serialised by the caller.  The
 * call runs on the current device; a stream of another device is E_ARG.
 * Windows outside the object are skipped (loss 0) but cannot be reported
 * here: validate positions first (ptycho_validate_positions).
 * Errors as for ptycho_create / ptycho_loss_grad (the caller's buffers are
 * checked the same way); a call rejected by its size, shape, flag or pointer
 * checks makes no HIP call at all.
 */
int ptycho_loss_grad_static(int32_t M, int32_t S, double wavelength_A, double dz_A, double pixel_A,
                            void* stream, const void* obj, int32_t H, int32_t W, int64_t slice_stride,
                            int32_t ld, const void* probe, const int32_t* pos, int32_t n, const float* meas,
                            double* loss, double* loss_per_pos, void* grad, int64_t grad_slice_stride,
                            int32_t grad_ld, uint32_t flags, const double* grad_scale);

/*
 * ptycho_loss_grad_probe: ptycho_loss_grad plus the gradient with respect to
 * the probe, probe_grad = dF/dRe P + i dF/dIm P = sum_i chi_{0,i} conj(t_0[window_i])
 * (chi_0 the adjoint wave at the first slice, Eq. 2 applied to psi_0 = P),
 * complex64 [M][M] on the device, overwritten (added with PTYCHO_ACCUMULATE;
 * the flag applies to grad, loss and probe_grad alike) and scaled like grad.
 * Each workgroup sums its positions into a partial buffer owned by the
 * context; the partial sums are added in workgroup order, so probe_grad does
 * not depend on timing.  E_ARG if probe_grad aliases grad or the probe;
 * otherwise the errors of ptycho_loss_grad.  probe_grad = NULL is
 * ptycho_loss_grad.
 */
int ptycho_loss_grad_probe(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride,
                           int32_t ld, const void* probe, const int32_t* pos, int32_t n, const float* meas,
                           double* loss, double* loss_per_pos, void* grad, int64_t grad_slice_stride, int32_t grad_ld,
                           void* probe_grad, uint32_t flags, const double* grad_scale);

/*
 * Sub-pixel positions (the probe function p_i of Section II-B translated to
 * the i-th location by a fraction of a pixel).  A position (y, x) splits into
 * the integer window corner (floor y, floor x), passed in pos as usual, and
 * the fraction d = (y - floor y, x - floor x); the probe at the position is
 * P_d = F^-1[F(P) exp(-2 pi i (q_y d_y + q_x d_x)/M)] on the periodic M x M
 * window grid, q the integer frequencies (-M/2 at the Nyquist bin), i.e. P
 * translated by d.  Everything after the probe is the integer-position model.
 *
 * ptycho_shift_probes: out[i] = P translated by shifts[i] = (d_y, d_x), for
 * i < n.  probe: device complex64 [M][M]; shifts: device float32 [n][2] (any
 * finite values; the fraction is the intended use); out: device complex64
 * [n][M][M], overwritten, must not overlap the probe (E_ARG).  Non-finite
 * shifts give non-finite probes (no other effect).
 *
 * ptycho_forward_stack / ptycho_loss_stack / ptycho_loss_grad_stack:
 * ptycho_forward, ptycho_loss and ptycho_loss_grad with one probe per
 * position: position i uses
 * probes + i*probe_stride (complex64 [M][M] each), probe_stride >= M*M
 * (else E_SHAPE).  With the probes from ptycho_shift_probes and the integer
 * corners in pos they compute the sub-pixel model.  The object gradient is
 * as in ptycho_loss_grad; the probe gradient is not offered for stacks.
 */
int ptycho_shift_probes(ptycho_ctx* ctx, const void* probe, const float* shifts, int32_t n, void* out);
int ptycho_forward_stack(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride,
                         int32_t ld, const void* probes, int64_t probe_stride, const int32_t* pos, int32_t n,
                         float* intens);
int ptycho_loss_stack(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride, int32_t ld,
                      const void* probes, int64_t probe_stride, const int32_t* pos, int32_t n, const float* meas,
                      double* loss, double* loss_per_pos, uint32_t flags);
int ptycho_loss_grad_stack(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride,
                           int32_t ld, const void* probes, int64_t probe_stride, const int32_t* pos, int32_t n,
                           const float* meas, double* loss, double* loss_per_pos, void* grad,
                           int64_t grad_slice_stride, int32_t grad_ld, uint32_t flags,
                           const double* grad_scale);

/*
 * ptycho_loss: the amplitude cost F (Eq. 1) alone -- the forward sweep and
 * the detector-plane residual, without the adjoint.  loss / loss_per_pos /
 * flags as for ptycho_loss_grad.
 */
int ptycho_loss(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride, int32_t ld,
                const void* probe, const int32_t* pos, int32_t n, const float* meas, double* loss,
                double* loss_per_pos, uint32_t flags);

/*
 * ptycho_tile_grad: the gradient of one tile (Section III): the summed
 * gradient of the positions assigned to tile [ty0,ty1) x [tx0,tx1) (global
 * object pixels, half-open), held on its extended box
 * [ey0, ey0+eh) x [ex0, ex0+ew), which must equal the tile grown by `halo`
 * and clipped to the H x W object (else PTYCHO_E_SHAPE).
 *   obj_ext:   the extended box of the object: element (s, y, x) of the box
 *              (box-local y, x) at obj_ext[s*slice_stride + y*ld + x]; it may
 *              be a view into the full object.
 *   pos:       this tile's positions in GLOBAL object coordinates.
 *   tile_grad: complex64 [S][eh][ew] (dense, box-local), overwritten unless
 *              ACCUMULATE.
 * Device-side checks: a window leaving the box is skipped and flagged
 * PTYCHO_STATUS_HALO; a window whose centre (y0+M/2, x0+M/2) is outside the
 * tile is skipped and flagged PTYCHO_STATUS_ASSIGN.
 * Summing the tile gradients of all tiles (embedded at their boxes) gives the
 * undecomposed gradient.
 */
int ptycho_tile_grad(ptycho_ctx* ctx, const void* obj_ext, int32_t ey0, int32_t ex0, int32_t eh,
                     int32_t ew, int64_t slice_stride, int32_t ld, int32_t ty0, int32_t ty1, int32_t tx0,
                     int32_t tx1, int32_t halo, int32_t H, int32_t W, const void* probe,
                     const int32_t* pos, int32_t n, const float* meas, double* loss,
                     double* loss_per_pos, void* tile_grad, uint32_t flags);

/*
 * Host helpers (host pointers).
 * ptycho_bin_positions: tile index (row-major, tiles_y x tiles_x even split,
 * edge_k = floor(k*extent/count)) of every position: the tile containing the
 * window centre (y0 + M/2, x0 + M/2).  Returns PTYCHO_E_BOUNDS if a window
 * leaves the object.
 * ptycho_validate_positions: PTYCHO_OK iff every window lies inside H x W.
 * ptycho_tile_box: the extended box of tile (ty, tx) for a halo.
 */
int ptycho_bin_positions(const int32_t* host_pos, int32_t n, int32_t H, int32_t W, int32_t M,
                         int32_t tiles_y, int32_t tiles_x, int32_t* host_tile_of_pos);
int ptycho_validate_positions(const int32_t* host_pos, int32_t n, int32_t H, int32_t W, int32_t M);
int ptycho_tile_box(int32_t H, int32_t W, int32_t tiles_y, int32_t tiles_x, int32_t ty, int32_t tx,
                    int32_t halo, int32_t* ty0, int32_t* ty1, int32_t* tx0, int32_t* tx1, int32_t* ey0,
                    int32_t* ey1, int32_t* ex0, int32_t* ex1);

/*
 * ptycho_gd_step_size: step length alpha of the gradient-descent update
 * t <- t - alpha * grad (Section II-B, last paragraph of the formulation; the
 * tile updates of Alg. 1).  The paper states no step length; this library's
 * reading is the inverse of a bound on the Gauss-Newton curvature of the
 * amplitude cost over S unit-modulus slices:
 *   alpha = 1 / (2 M^2 S max_r sum_i |P(r - r_i)|^2),
 * the maximum over the object pixels r, the sum over the windows i covering r
 * (P the probe translated to window i).
 *   host_probe: HOST complex64 [M][M] (interleaved float pairs), M in [1, 4096]
 *   host_pos:   HOST int32 [n][2] window corners (y0, x0), every window inside H x W
 *   S:          slice count, >= 1
 *   alpha_out:  HOST double, written on success only
 * Errors: PTYCHO_E_ARG (a null pointer, n < 0, a bad size, or no object pixel
 * with non-zero coverage -- n = 0 or a zero probe -- where the bound is
 * infinite), PTYCHO_E_BOUNDS (a window leaves the object).  Host only: it uses
 * an H x W host coverage map and touches no device.
 */
int ptycho_gd_step_size(const void* host_probe, int32_t M, const int32_t* host_pos, int32_t n, int32_t H,
                        int32_t W, int32_t S, double* alpha_out);

/*
 * ptycho_tiles_grad: the gradients of all tiles of a decomposition in one
 * persistent launch (Section III): every position adds its window's gradient
 * into the gradient buffer of the tile that owns it, on that tile's extended
 * box, exactly as ptycho_tile_grad does tile by tile -- the per-device work of
 * a tile mesh, run side by side on one GPU.
 *   tiles:       HOST array of ntiles descriptors (copied into the context,
 *                at most 4096); tile.grad is a device complex64 [S][eh][ew]
 *                dense buffer (overwritten unless PTYCHO_ACCUMULATE)
 *   tile_of_pos: device int32 [n], the owning tile of each position
 *   pos:         device int32 [n][2], global window corners; obj is the whole
 *                H x W object.
 * Host validation as in ptycho_tile_grad for every descriptor (tile inside
 * the object, box = tile grown by halo and clipped, box >= M, non-null
 * buffer); on the device a window outside its tile's box raises
 * PTYCHO_STATUS_HALO, a centre outside its tile or a bad tile index
 * PTYCHO_STATUS_ASSIGN, and the position is skipped.  *loss is the sum over
 * all positions (per position in loss_per_pos if non-NULL).
 */
typedef struct ptycho_tile_desc {
  int32_t ty0, ty1, tx0, tx1; /* the tile, global pixels, half-open */
  int32_t ey0, ex0, eh, ew;   /* its extended box */
  void* grad;                 /* device complex64 [S][eh][ew] tile gradient (dense) */
} ptycho_tile_desc;
int ptycho_tiles_grad(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride, int32_t ld,
                      const ptycho_tile_desc* tiles, int32_t ntiles, int32_t halo, const int32_t* tile_of_pos,
                      const void* probe, const int32_t* pos, int32_t n, const float* meas, double* loss,
                      double* loss_per_pos, uint32_t flags);
/*
 * ptycho_tiles_grad_stack: ptycho_tiles_grad with one probe per position
 * (position i uses probes + i*probe_stride, probe_stride >= M*M, in the
 * order of pos), e.g. the sub-pixel probes of ptycho_shift_probes.
 */
int ptycho_tiles_grad_stack(ptycho_ctx* ctx, const void* obj, int32_t H, int32_t W, int64_t slice_stride,
                            int32_t ld, const ptycho_tile_desc* tiles, int32_t ntiles, int32_t halo,
                            const int32_t* tile_of_pos, const void* probes, int64_t probe_stride, const int32_t* pos,
                            int32_t n, const float* meas, double* loss, double* loss_per_pos, uint32_t flags);

/*
 * ptycho_tile_accumulate: the stitch step of the decomposition (Section III,
 * and the final stitch of Alg. 1): adds a tile gradient [S][eh][ew] (dense)
 * into the global gradient at its extended box (ey0, ex0):
 *   grad[s*grad_slice_stride + (ey0+y)*grad_ld + ex0 + x] += tile_grad[s][y][x].
 * Overlapping boxes therefore sum, which is exactly the neighbour-tile gradient
 * addition of the paper on one device.  The box must lie inside H x W.
 */
int ptycho_tile_accumulate(ptycho_ctx* ctx, const void* tile_grad, int32_t ey0, int32_t ex0, int32_t eh,
                           int32_t ew, int32_t H, int32_t W, void* grad, int64_t grad_slice_stride,
                           int32_t grad_ld);

/*
 * ptycho_box_exchange: one exchange of the accumulation passes between two
 * tiles' separately held gradient buffers (Section IV; the buffers stand for
 * the accumulated-gradient buffers that neighbouring devices exchange).  On
 * the overlap of the two boxes, in global pixel coordinates,
 *   PTYCHO_EXCHANGE_ADD:     dst += src   (the forward passes, and the
 *                                          neighbour add of Section III)
 *   PTYCHO_EXCHANGE_REPLACE: dst  = src   (the backward passes).
 * src holds the box with top-left (sy0, sx0) and size sh x sw:
 * element (s, y, x) of the box at src[s*s_slice_stride + y*s_ld + x]; dst
 * likewise.  Both are device complex64 arrays owned by the caller; they must
 * not share memory (E_ARG if the address ranges intersect).  S slices.
 * Boxes that do not overlap enqueue nothing.  Stream-ordered on the context
 * stream; allocates nothing.
 */
#define PTYCHO_EXCHANGE_ADD 0u
#define PTYCHO_EXCHANGE_REPLACE 1u
int ptycho_box_exchange(ptycho_ctx* ctx, int32_t S, const void* src, int32_t sy0, int32_t sx0, int32_t sh,
                        int32_t sw, int64_t s_slice_stride, int32_t s_ld, void* dst, int32_t dy0, int32_t dx0,
                        int32_t dh, int32_t dw, int64_t d_slice_stride, int32_t d_ld, uint32_t mode);

/*
 * ptycho_zero_gradient: sets S slices of an H x W complex64 array with the
 * given strides to zero on the context stream (the reset of a gradient or
 * accumulation buffer; a plain fill kernel, so it may be graph-captured).
 */
int ptycho_zero_gradient(ptycho_ctx* ctx, void* grad, int32_t H, int32_t W, int64_t grad_slice_stride,
                         int32_t grad_ld);

/*
 * Kernel timing.  While enabled, every launch of the fused forward or
 * loss/gradient kernel of this context is bracketed by HIP events on the
 * context stream (a pool of 4096 pairs allocated by the enable call).
 * ptycho_profile_read synchronises, returns the summed kernel time in ms, the
 * number of timed launches and the positions they processed, and resets the
 * counters.
 */
int ptycho_profile_enable(ptycho_ctx* ctx, int32_t enable);
int ptycho_profile_read(ptycho_ctx* ctx, double* total_ms, int64_t* launches, int64_t* positions);

/*
 * Batched reconstructions.  Many independent problems of uneven size (object,
 * slice count, scan, window size 64 or 128, dose) are served by one persistent
 * launch per window size that walks a work list of (reconstruction, position)
 * items; the two window sizes' launches run side by side (the batch stream
 * and a second stream of the batch, joined by events), and each launch's
 * items are split into 8 parts of equal cost ((4S - 2) transforms per item),
 * one per XCD, served to its workgroups through a device counter.  One
 * full-batch gradient-descent iteration t <- t - alpha * dF/dt (Section II-B,
 * last paragraph of the formulation; the tile update of Alg. 1) can be
 * recorded once in a hipGraph and replayed.
 */
typedef struct ptycho_recon {
  int32_t M;              /* window side, 64 or 128 */
  int32_t S;              /* slices, 1..64 */
  int32_t H, W;           /* object rows and columns (>= M) */
  int32_t n;              /* positions (>= 0) */
  int32_t reserved;       /* must be 0 */
  int64_t slice_stride;   /* object and gradient: element (s,y,x) at [s*slice_stride + y*ld + x] */
  int64_t ld;             /* >= W; slice_stride >= H*ld when S > 1 */
  void* obj;              /* device complex64 transmissions, updated in place by the update step */
  void* grad;             /* device complex64 gradient (same strides), overwritten by each loss/gradient */
  const void* probe;      /* device complex64 [M][M] */
  const int32_t* pos;     /* device int32 [n][2] window corners; windows must lie inside H x W */
  const float* meas;      /* device float32 [n][M][M] measured intensities */
  double wavelength_A, dz_A, pixel_A;  /* propagator of this reconstruction */
  double alpha;           /* gradient-descent step */
} ptycho_recon;

typedef struct ptycho_batch ptycho_batch;

/*
 * ptycho_batch_create: copies the descriptors (host array of nrecon), builds
 * the work list and the per-reconstruction propagator tables, and allocates
 * everything the batch needs (work list, per-item and per-reconstruction
 * losses, a loss history of history_rows iterations, the incident-wave store
 * of each window size).  The batch owns a stream of its own (default priority,
 * non-blocking, ptycho_batch_stream); every batch call is enqueued there, so
 * callers order their own work against it: ptycho_batch_sync, or events on
 * that stream (the Python binding makes the batch stream wait for the
 * caller's current stream before each call, and the caller's stream wait for
 * the batch stream after it).  The arrays the descriptors point to stay owned
 * by the caller and must outlive the batch.
 */
int ptycho_batch_create(ptycho_batch** out, const ptycho_recon* recons, int32_t nrecon, int32_t history_rows);
int ptycho_batch_destroy(ptycho_batch* b);
/* Persistent workgroups of the launch for window size M (the autotuner's knob); 0 restores the default. */
int ptycho_batch_set_grid(ptycho_batch* b, int32_t M, int32_t grid);
int ptycho_batch_get_grid(const ptycho_batch* b, int32_t M);
/* Gradient of every reconstruction (each grad overwritten) and its loss; losses: nullable device double[nrecon]
 * on the batch's device (E_ARG otherwise; nothing is enqueued then). */
int ptycho_batch_loss_grad(ptycho_batch* b, double* losses);
/* t <- t - alpha * grad for every reconstruction; advances the history row. */
int ptycho_batch_update(ptycho_batch* b);
/* One iteration: ptycho_batch_loss_grad then ptycho_batch_update. */
int ptycho_batch_step(ptycho_batch* b);
/* Record one iteration in a hipGraph (no allocation inside); replay it with ptycho_batch_replay. */
int ptycho_batch_capture(ptycho_batch* b);
int ptycho_batch_replay(ptycho_batch* b);
/* Synchronise the batch stream; reports out-of-object windows (PTYCHO_E_BOUNDS) and HIP errors. */
int ptycho_batch_sync(ptycho_batch* b);
/* Copies the loss history (rows x nrecon doubles, row k = loss before the k-th update) to host memory. */
int ptycho_batch_history(ptycho_batch* b, double* host_out, int32_t* rows_out);
int ptycho_batch_reset_history(ptycho_batch* b);
/* The batch stream (a hipStream_t), for callers that enqueue their own work on it. */
void* ptycho_batch_stream(const ptycho_batch* b);

/* Synchronise the context stream; PTYCHO_OK, or the first HIP error, or a
 * negative code for the device status word (which is then cleared). */
int ptycho_check(ptycho_ctx* ctx, uint32_t* status_out);

const char* ptycho_last_error(void);
const char* ptycho_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PTYCHO_H */
