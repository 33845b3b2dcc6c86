// ptycho_kernels.hip -- fused multislice forward / amplitude loss / adjoint
// kernels for CDNA4 (gfx950), one probe position per workgroup iteration.
//
// Per position (Section II-B and Eq. 1-2 of Wang et al., SC22):
//   psi_0 = probe, phi_s = psi_s * t_s[window], psi_{s+1} = IDFT(H DFT(phi_s)),
//   Psi = DFT(phi_{S-1}), f = sum (|Psi| - sqrt(meas))^2,
//   chi_{S-1} = DFT^H(2 (|Psi| - a) Psi / |Psi|), grad_s += chi_s conj(psi_s),
//   chi_{s-1} = IDFT(conj(H) DFT(chi_s conj(t_s))).
// The wave of a position stays in registers of one workgroup for the whole
// slice loop; LDS is used only for the two transposing exchanges of every
// 2D DFT (see fft_lds.hpp).  The incident waves psi_s of the forward sweep
// are kept in a per-workgroup workspace in HBM and re-read in reverse order by
// the adjoint sweep.  Gradient patches are added to the caller's gradient with
// hardware float atomics, laid out so that every atomic instruction covers 32
// contiguous complex values.
#include "fft_lds.hpp"
#include "ptycho_kernels.h"

namespace ptycho {

// A zero the compiler cannot see through.  Adding it to LDS and table
// addresses inside the slice loops keeps loop-invariant address arithmetic and
// table reads from being hoisted into long-lived registers.
__device__ __forceinline__ int opaque_zero() {
  int z;
  asm volatile("s_mov_b32 %0, 0" : "=s"(z));
  return z;
}

// Position index of the j-th job of this workgroup, or -1 when done.  Blocks
// are dispatched round-robin over the 8 XCDs; the positions are cut into 8
// contiguous chunks and chunk x is walked by the blocks of XCD x, so blocks
// sharing an L2 work on neighbouring (overlapping) windows.
__device__ __forceinline__ int job_position(int j, int n, int grid) {
  const int b = static_cast<int>(blockIdx.x);
  if (grid < 8) {
    int p = b + j * grid;
    return p < n ? p : -1;
  }
  const int x = b & 7;
  const int gx = (grid - x + 7) >> 3;              // blocks on this XCD
  const int lo = static_cast<int>((static_cast<long long>(x) * n) >> 3);
  const int hi = static_cast<int>((static_cast<long long>(x + 1) * n) >> 3);
  int p = lo + (b >> 3) + j * gx;
  return p < hi ? p : -1;
}

template <class G>
struct Lanes {
  int tid, n2, x;       // layout A
  int k1, m2;           // layout B
  int ky, jh;           // layout C
  __device__ __forceinline__ Lanes() {
    tid = static_cast<int>(threadIdx.x);
    n2 = __builtin_amdgcn_readfirstlane(tid / G::M);
    x = tid % G::M;
    k1 = tid / G::X2;
    m2 = tid % G::X2;
    ky = tid / G::Y2;
    jh = tid % G::Y2;
  }
};

// One full propagation IDFT(Hs * DFT(v)) in place, v in layout A at entry and
// exit.  Hs = (hy * hx[kx]) for the forward propagator or its conjugate for
// the adjoint, hy already carrying the 1/M^2 of the inverse transform.
template <class G, bool ADJ>
__device__ __forceinline__ void propagate(float2 (&v)[G::R], float2* lds, const float2* hx_lds,
                                          const float2 (&twb)[G::X1], float2 hy, const Lanes<G>& L) {
  const int z = opaque_zero();
  lds += z;
  hx_lds += z;
  pass_a_fwd<G>(v, L.n2);
  __syncthreads();
  e1_write_a<G>(lds, v, L.n2, L.x);
  __syncthreads();
  e1_read_b<G>(lds, v, L.k1, L.m2);
  pass_b_fwd<G>(v, twb);
  __syncthreads();
  e2_write_b<G>(lds, v, L.k1, L.m2);
  __syncthreads();
  e2_read_c<G>(lds, v, L.ky, L.jh);
  pass_c<G, false>(v);
  sfor<G::CJ>([&](auto lc) {
    sfor<G::X2>([&](auto jc) {
      constexpr int jl = decltype(lc)::value, j2 = decltype(jc)::value;
      const int kx = L.jh * G::CJ + jl + G::X1 * j2;
      float2 h = cmul(hy, hx_lds[kx]);
      float2& e = v[jl * G::X2 + j2];
      e = ADJ ? cmulc(e, h) : cmul(e, h);
    });
  });
  pass_c<G, true>(v);
  __syncthreads();
  e2_write_c<G>(lds, v, L.ky, L.jh);
  __syncthreads();
  e2_read_b<G>(lds, v, L.k1, L.m2);
  pass_b_inv<G>(v, twb);
  __syncthreads();
  e1_write_b<G>(lds, v, L.k1, L.m2);
  __syncthreads();
  e1_read_a<G>(lds, v, L.n2, L.x);
  pass_a_inv<G>(v, L.n2);
}

// Forward 2D DFT, layout A -> layout C.
template <class G>
__device__ __forceinline__ void dft2_a_to_c(float2 (&v)[G::R], float2* lds, const float2 (&twb)[G::X1],
                                            const Lanes<G>& L) {
  lds += opaque_zero();
  pass_a_fwd<G>(v, L.n2);
  __syncthreads();
  e1_write_a<G>(lds, v, L.n2, L.x);
  __syncthreads();
  e1_read_b<G>(lds, v, L.k1, L.m2);
  pass_b_fwd<G>(v, twb);
  __syncthreads();
  e2_write_b<G>(lds, v, L.k1, L.m2);
  __syncthreads();
  e2_read_c<G>(lds, v, L.ky, L.jh);
  pass_c<G, false>(v);
}

// Unnormalised inverse 2D DFT (the adjoint DFT^H), layout C -> layout A.
template <class G>
__device__ __forceinline__ void idft2_c_to_a(float2 (&v)[G::R], float2* lds, const float2 (&twb)[G::X1],
                                             const Lanes<G>& L) {
  lds += opaque_zero();
  pass_c<G, true>(v);
  __syncthreads();
  e2_write_c<G>(lds, v, L.ky, L.jh);
  __syncthreads();
  e2_read_b<G>(lds, v, L.k1, L.m2);
  pass_b_inv<G>(v, twb);
  __syncthreads();
  e1_write_b<G>(lds, v, L.k1, L.m2);
  __syncthreads();
  e1_read_a<G>(lds, v, L.n2, L.x);
  pass_a_inv<G>(v, L.n2);
}

// Window of the current position in layout A: row y = Y2*r + n2, column x.
// `base` is uniform across the workgroup; each row pointer is computed on the
// scalar unit and the lane offset is the column, so the loads use the
// scalar-base + 32-bit lane-offset addressing form.
template <class G, class F>
__device__ __forceinline__ void for_window_rows(const float2* __restrict__ base, long long ld, const Lanes<G>& L,
                                                F&& f) {
  const int ldz = static_cast<int>(ld) + opaque_zero();
  base += static_cast<long long>(L.n2) * ldz;
  sfor<G::R>([&](auto rc) {
    constexpr int r = decltype(rc)::value;
    const float2* __restrict__ row = base + static_cast<long long>(r * G::Y2 * ldz);
    f(rc, row[L.x]);
  });
}
template <class G>
__device__ __forceinline__ void load_window(float2 (&t)[G::R], const float2* __restrict__ base, long long ld,
                                            const Lanes<G>& L) {
  for_window_rows<G>(base, ld, L, [&](auto rc, float2 e) { t[decltype(rc)::value] = e; });
}
// v *= window (conj_window: v *= conj(window)).  All loads are issued before
// the first multiply (the scheduling fence keeps the compiler from
// interleaving them), so the window costs one memory latency, not R.
template <class G, bool CONJ>
__device__ __forceinline__ void mul_window(float2 (&v)[G::R], const float2* __restrict__ base, long long ld,
                                           const Lanes<G>& L) {
  float2 t[G::R];
  load_window<G>(t, base, ld, L);
  __builtin_amdgcn_sched_barrier(0);
  sfor<G::R>([&](auto rc) {
    constexpr int r = decltype(rc)::value;
    v[r] = CONJ ? cmulc(v[r], t[r]) : cmul(v[r], t[r]);
  });
}

// Adds g (layout A) into the complex gradient rows.  permlane32_swap pairs
// lanes l and l+32 so that each atomic instruction covers 32 consecutive
// complex values (256 contiguous bytes) instead of every other float of 64.
template <class G>
__device__ __forceinline__ void scatter_add(float2* __restrict__ gbase, long long gld, const float2 (&g)[G::R],
                                            const Lanes<G>& L) {
  const int lane = L.tid & 63;
  const int xb = L.x - lane;  // first column of this wave's 64 columns (uniform)
  const int off0 = 2 * (lane & 31) + (lane >> 5);
  const int gldz = static_cast<int>(gld) + opaque_zero();
  gbase += static_cast<long long>(L.n2) * gldz + xb;
  sfor<G::R>([&](auto rc) {
    constexpr int r = decltype(rc)::value;
    auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(g[r].x), __float_as_uint(g[r].y), false, false);
    float* __restrict__ row = reinterpret_cast<float*>(gbase + static_cast<long long>(r * G::Y2 * gldz));
    unsafeAtomicAdd(row + off0, __uint_as_float(sw[0]));
    unsafeAtomicAdd(row + 64 + off0, __uint_as_float(sw[1]));
  });
}

template <class G>
__device__ __forceinline__ void load_hx_table(float2* hx_lds, const float2* __restrict__ h) {
  for (int i = threadIdx.x; i < G::M; i += G::T) hx_lds[i] = h[i];
}

template <class G>
__device__ __forceinline__ void load_twb(float2 (&twb)[G::X1], const float2* __restrict__ tw, int m2) {
  sfor<G::X1>([&](auto jc) {
    constexpr int j1 = decltype(jc)::value;
    twb[j1] = tw[(m2 * j1) % G::M];
  });
}

// Returns true when the window of position p is usable; otherwise flags the
// status word (one lane) and returns false.  Uniform across the workgroup.
__device__ __forceinline__ bool check_window(const KernelArgs& a, int y0, int x0, int gy0, int gx0) {
  const int M = a.M;
  bool ok = y0 >= 0 && x0 >= 0 && y0 + M <= a.bh && x0 + M <= a.bw;
  unsigned flag = a.oob_flag;
  if (ok && a.check_tile) {
    const int cy = gy0 + M / 2, cx = gx0 + M / 2;
    ok = cy >= a.ty0 && cy < a.ty1 && cx >= a.tx0 && cx < a.tx1;
    flag = 4u;
  }
  if (!ok && threadIdx.x == 0) atomicOr(a.status, flag);
  return ok;
}

template <int M, bool GRAD>
__global__ void __launch_bounds__(Geo<M>::T) fused_kernel(KernelArgs a) {
  using G = Geo<M>;
  __shared__ float2 lds[G::LDS_ELEMS];
  __shared__ float2 hx_lds[G::M];
  __shared__ double red[G::T / 64];

  const Lanes<G> L;
  float2 twb[G::X1];
  load_twb<G>(twb, a.tw, L.m2);
  load_hx_table<G>(hx_lds, a.h);
  const float2 hky = a.h[L.ky];
  const float inv_n = 1.0f / float(G::M * G::M);
  const float2 hy = make_float2(hky.x * inv_n, hky.y * inv_n);
  __syncthreads();

  const int S = a.S;
  const long long ld = a.ld;
  const long long sstride = a.slice_stride;
  float2* __restrict__ ws = a.ws + static_cast<long long>(blockIdx.x) * (S > 1 ? S - 1 : 0) * (G::M * G::M);

  for (int j = 0;; ++j) {
    const int p = job_position(j, a.n, static_cast<int>(gridDim.x));
    if (p < 0) break;
    const int gy = a.pos[2 * p], gx = a.pos[2 * p + 1];
    const int y0 = gy - a.oy, x0 = gx - a.ox;
    if (!check_window(a, y0, x0, gy, gx)) {
      if (GRAD && threadIdx.x == 0) {
        a.loss_work[p] = 0.0;
        if (a.loss_pos != nullptr) a.loss_pos[p] = 0.0;
      }
      continue;
    }
    const float2* __restrict__ win = a.obj + static_cast<long long>(y0) * ld + x0;

    float2 v[G::R];
    load_window<G>(v, a.probe, G::M, L);
    for (int s = 0; s < S; ++s) {
      if (GRAD && s >= 1) {
        float2* __restrict__ w = ws + static_cast<long long>(s - 1 + opaque_zero()) * (G::M * G::M);
        sfor<G::R>([&](auto rc) { w[decltype(rc)::value * G::T + L.tid] = v[decltype(rc)::value]; });
      }
      mul_window<G, false>(v, win + s * sstride, ld, L);
      if (s + 1 < S) propagate<G, false>(v, lds, hx_lds, twb, hy, L);
    }
    dft2_a_to_c<G>(v, lds, twb, L);

    // ---- detector plane, layout C: element (ky, kx = jh*CJ + jl + X1*j2)
    const long long pat = static_cast<long long>(p) * (G::M * G::M) + static_cast<long long>(L.ky) * G::M;
    if (!GRAD) {
      float* __restrict__ out = a.intens + pat;
      sfor<G::CJ>([&](auto lc) {
        sfor<G::X2>([&](auto jc) {
          constexpr int jl = decltype(lc)::value, j2 = decltype(jc)::value;
          const float2 e = v[jl * G::X2 + j2];
          out[L.jh * G::CJ + jl + G::X1 * j2] = e.x * e.x + e.y * e.y;
        });
      });
      continue;
    }
    double acc = 0.0;
    const float* __restrict__ mrow = a.meas + pat;
    float amp[G::R];
    sfor<G::CJ>([&](auto lc) {
      sfor<G::X2>([&](auto jc) {
        constexpr int jl = decltype(lc)::value, j2 = decltype(jc)::value;
        amp[jl * G::X2 + j2] = mrow[L.jh * G::CJ + jl + G::X1 * j2];
      });
    });
    __builtin_amdgcn_sched_barrier(0);
    sfor<G::R>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      float2& e = v[i];
      const float a_i = sqrtf(amp[i]);
      const float mod = sqrtf(e.x * e.x + e.y * e.y);
      const float d = mod - a_i;
      acc += static_cast<double>(d) * static_cast<double>(d);
      const float sc = mod > 0.0f ? 2.0f * d / mod : 0.0f;
      e = make_float2(sc * e.x, sc * e.y);
    });
    // position loss: wave reduction then across the waves through LDS
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((L.tid & 63) == 0) red[L.tid >> 6] = acc;

    // ---- adjoint sweep
    idft2_c_to_a<G>(v, lds, twb, L);  // chi_{S-1} = DFT^H g (contains barriers: red[] is visible after it)
    if (L.tid == 0) {
      double f = 0.0;
      for (int w = 0; w < G::T / 64; ++w) f += red[w];
      a.loss_work[p] = f;
      if (a.loss_pos != nullptr) a.loss_pos[p] = f;
    }
    for (int s = S - 1; s >= 0; --s) {
      // psi_s and the transmission window are loaded together and consumed
      // before the gradient atomics are issued: memory operations retire in
      // order, so loads issued behind the atomics would wait for them.  The
      // atomics then drain while the next propagation runs on LDS and VALU.
      float2 g[G::R];
      if (s == 0) {
        load_window<G>(g, a.probe, G::M, L);
        __builtin_amdgcn_sched_barrier(0);
        sfor<G::R>([&](auto rc) { g[decltype(rc)::value] = cmulc(v[decltype(rc)::value], g[decltype(rc)::value]); });
      } else {
        float2 t[G::R];
        const float2* __restrict__ w = ws + static_cast<long long>(s - 1 + opaque_zero()) * (G::M * G::M);
        sfor<G::R>([&](auto rc) { g[decltype(rc)::value] = w[decltype(rc)::value * G::T + L.tid]; });
        load_window<G>(t, win + s * sstride, ld, L);
        __builtin_amdgcn_sched_barrier(0);
        sfor<G::R>([&](auto rc) {
          constexpr int r = decltype(rc)::value;
          g[r] = cmulc(v[r], g[r]);
          v[r] = cmulc(v[r], t[r]);
        });
      }
      __builtin_amdgcn_sched_barrier(0);
      scatter_add<G>(a.grad + s * a.gslice + static_cast<long long>(y0) * a.gld + x0, a.gld, g, L);
      if (s > 0) propagate<G, true>(v, lds, hx_lds, twb, hy, L);
    }
    __syncthreads();  // red[] and lds reuse by the next position
  }
}

// ---------------------------------------------------------------------------
// small helper kernels
// ---------------------------------------------------------------------------
__global__ void zero_slices_kernel(float2* __restrict__ g, int S, int H, int W, long long gslice, long long gld) {
  const long long total = static_cast<long long>(S) * H * W;
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<long long>(gridDim.x) * blockDim.x) {
    const long long s = i / (static_cast<long long>(H) * W);
    const long long r = i - s * H * W;
    const long long y = r / W, x = r - y * W;
    g[s * gslice + y * gld + x] = make_float2(0.f, 0.f);
  }
}

// Sums the per-position losses in a fixed order (deterministic) and writes or
// adds the total.
__global__ void __launch_bounds__(1024) finalize_loss_kernel(const double* __restrict__ per, int n,
                                                             double* __restrict__ loss, int accumulate) {
  __shared__ double part[1024];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += per[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = accumulate ? *loss + part[0] : part[0];
}

__global__ void clear_status_kernel(unsigned* status) { *status = 0u; }

// grad[s, ey0 + y, ex0 + x] += tile[s, y, x]; one thread per complex element.
__global__ void tile_accumulate_kernel(const float2* __restrict__ tile, int S, int eh, int ew, float2* __restrict__ grad,
                                       long long gslice, long long gld) {
  const long long total = static_cast<long long>(S) * eh * ew;
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<long long>(gridDim.x) * blockDim.x) {
    const long long s = i / (static_cast<long long>(eh) * ew);
    const long long r = i - s * eh * ew;
    const long long y = r / ew, x = r - y * ew;
    float2* g = grad + s * gslice + y * gld + x;
    const float2 t = tile[i];
    *g = make_float2(g->x + t.x, g->y + t.y);
  }
}

// ---------------------------------------------------------------------------
// launchers (host side)
// ---------------------------------------------------------------------------
template <int M, bool GRAD>
static hipError_t launch_fused_t(const KernelArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((fused_kernel<M, GRAD>), dim3(grid), dim3(Geo<M>::T), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fused(const KernelArgs& a, bool grad, int grid, hipStream_t st) {
  if (a.M == 128) return grad ? launch_fused_t<128, true>(a, grid, st) : launch_fused_t<128, false>(a, grid, st);
  if (a.M == 64) return grad ? launch_fused_t<64, true>(a, grid, st) : launch_fused_t<64, false>(a, grid, st);
  return hipErrorInvalidValue;
}

hipError_t launch_zero_slices(float2* g, int S, int H, int W, long long gslice, long long gld, hipStream_t st) {
  const long long total = static_cast<long long>(S) * H * W;
  if (total == 0) return hipSuccess;
  long long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(zero_slices_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, g, S, H, W, gslice,
                     gld);
  return hipGetLastError();
}

hipError_t launch_finalize_loss(const double* per, int n, double* loss, bool accumulate, hipStream_t st) {
  hipLaunchKernelGGL(finalize_loss_kernel, dim3(1), dim3(1024), 0, st, per, n, loss, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_tile_accumulate(const float2* tile, int S, int eh, int ew, float2* grad, long long gslice,
                                  long long gld, hipStream_t st) {
  const long long total = static_cast<long long>(S) * eh * ew;
  if (total == 0) return hipSuccess;
  long long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(tile_accumulate_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, tile, S, eh, ew,
                     grad, gslice, gld);
  return hipGetLastError();
}

hipError_t launch_clear_status(unsigned* status, hipStream_t st) {
  hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(1), 0, st, status);
  return hipGetLastError();
}

}  // namespace ptycho
