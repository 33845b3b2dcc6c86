// ptycho_kernels.hip -- fused multislice forward / amplitude loss / adjoint
// kernels for CDNA4 (gfx950), one probe position per workgroup iteration.
//
// Per position (Section II-B and Eq. 1-2 of Wang et al., SC22):
//   psi_0 = probe, phi_s = psi_s * t_s[window], psi_{s+1} = IDFT(H DFT(phi_s)),
//   Psi = DFT(phi_{S-1}), f = sum (|Psi| - sqrt(meas))^2,
//   chi_{S-1} = DFT^H(2 (|Psi| - a) Psi / |Psi|), grad_s += chi_s conj(psi_s),
//   chi_{s-1} = IDFT(conj(H) DFT(chi_s conj(t_s))).
// The wave of a position stays in registers of one workgroup for the whole
// slice loop; LDS holds the two transposing exchanges of every 2D DFT (see
// fft_lds.hpp) and, between propagations, the gradient window being added.
// The incident waves psi_s of the forward sweep are kept in a per-workgroup
// workspace in HBM (all of them, or checkpoints from which the adjoint sweep
// recomputes the rest) and re-read in reverse order by the adjoint sweep.
// Gradient windows are added to the caller's gradient with hardware float
// atomics, each instruction covering whole 128-byte lines (128-windows) or 32
// contiguous complex values (64-windows and the batched launch).  Optional
// outputs: the probe gradient (per-workgroup partial sums).
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

// A wave in a wave-store slot.  Streaming (non-temporal) accesses: each stored
// wave is read back once, so it should not displace the object windows and
// gradient rows that neighbouring positions reuse from the caches.  Register
// pair (2q, 2q+1) of thread tid sits at complex offset 2*(q*T + tid), so each
// access moves 16 bytes per lane, contiguous across the wave: half the memory
// instructions of 8-byte accesses (measured 2.4 % faster over the whole
// position-parallel launch).
typedef float f4v __attribute__((ext_vector_type(4)));
template <int R, int T>
__device__ __forceinline__ void store_slot(float2* slot, const float2 (&v)[R], int tid) {
  f4v* p = reinterpret_cast<f4v*>(slot) + tid;
  sfor<R / 2>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    __builtin_nontemporal_store(f4v{v[2 * q].x, v[2 * q].y, v[2 * q + 1].x, v[2 * q + 1].y}, p + q * T);
  });
}
template <int R, int T>
__device__ __forceinline__ void load_slot(float2 (&v)[R], const float2* slot, int tid) {
  const f4v* p = reinterpret_cast<const f4v*>(slot) + tid;
  sfor<R / 2>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    const f4v e = __builtin_nontemporal_load(p + q * T);
    v[2 * q] = make_float2(e.x, e.y);
    v[2 * q + 1] = make_float2(e.z, e.w);
  });
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
    ky = layout_c_ky<G>(tid);
    jh = tid % G::Y2;
  }
};

struct NoHook {
  __device__ __forceinline__ void operator()() const {}
};
// One full propagation IDFT(Hs * DFT(v)) in place, v in layout A at entry and
// exit.  Hs = (hy * hx[kx]) for the forward propagator or its conjugate for
// the adjoint, hy already carrying the 1/M^2 of the inverse transform.  `late`
// runs after the last exchange write, where the caller can issue loads for
// its next step that then travel during the last barrier and pass.
template <class G, bool ADJ, class Hook = NoHook>
__device__ __forceinline__ void propagate(float2 (&v)[G::R], float2* lds, const float2* hx_lds,
                                          const float2 (&twb)[G::X1], float2 hy, const Lanes<G>& L,
                                          bool own_reads_last = false, const Hook& late = Hook{}) {
  const int z = opaque_zero();
  lds += z;
  hx_lds += z;
  pass_a_fwd<G>(v, L.n2);
  if (!own_reads_last) __syncthreads();  // the buffer may have served another purpose
  e1_write_a<G>(lds, v, L.n2, L.x);
  __syncthreads();
  e1_read_b<G>(lds, v, L.k1, L.m2);
  pass_b_fwd<G>(v, twb);
  e2_write_b<G>(lds, v, L.k1, L.m2);
  wave_sync();
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
  e2_write_c<G>(lds, v, L.ky, L.jh);
  wave_sync();
  e2_read_b<G>(lds, v, L.k1, L.m2);
  pass_b_inv<G>(v, twb);
  e1_write_b<G>(lds, v, L.k1, L.m2);
  late();  // the wave's values sit in LDS here: the fewest registers are live
  __syncthreads();
  e1_read_a<G>(lds, v, L.n2, L.x);
  pass_a_inv<G>(v, L.n2);
}

// Forward 2D DFT, layout A -> layout C.
template <class G>
__device__ __forceinline__ void dft2_a_to_c(float2 (&v)[G::R], float2* lds, const float2 (&twb)[G::X1],
                                            const Lanes<G>& L, bool own_reads_last = false) {
  lds += opaque_zero();
  pass_a_fwd<G>(v, L.n2);
  if (!own_reads_last) __syncthreads();
  e1_write_a<G>(lds, v, L.n2, L.x);
  __syncthreads();
  e1_read_b<G>(lds, v, L.k1, L.m2);
  pass_b_fwd<G>(v, twb);
  e2_write_b<G>(lds, v, L.k1, L.m2);
  wave_sync();
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
  wave_sync();
  e2_read_b<G>(lds, v, L.k1, L.m2);
  pass_b_inv<G>(v, twb);
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

// Adds a gradient window staged in LDS (row-major, row stride RS1, written by
// e1_write_a) into the complex gradient rows so that every atomic instruction
// covers two whole 128-byte lines: a row of M complex values starting at an
// arbitrary column touches M/16 + 1 lines, and instructions aligned to the
// lines touch each of them once instead of splitting lines between
// instructions.  Each wave takes rows wave, wave + T/64, ...; the lines of a
// row are taken in pairs (lanes 0-31 and 32-63), lanes outside the window are
// inactive.
template <class G>
__device__ __forceinline__ void scatter_add_lines(float2* __restrict__ gbase, long long gld, const float2* lds,
                                                  const Lanes<G>& L) {
  constexpr int NW = G::T / 64;
  constexpr int JMAX = (G::M / 16 + 2) / 2;  // instructions per row when the row is not line-aligned
  const int lane = L.tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(L.tid >> 6);
  const int half = lane >> 5;
  const int e = lane & 31;
  const float* __restrict__ lf = reinterpret_cast<const float*>(lds + opaque_zero());
  const int gldz = static_cast<int>(gld) + opaque_zero();
#pragma unroll 1  // one row at a time: measured faster than 2 or 4 (fewer atomics in flight per wave)
  for (int k = 0; k < G::M / NW; ++k) {
    const int y = wave + NW * k;
    float* row = reinterpret_cast<float*>(gbase + static_cast<long long>(y) * gldz);
    const int delta = static_cast<int>((reinterpret_cast<unsigned long long>(row) >> 3) & 15);
    const int nline = (delta + G::M + 15) >> 4;
    float* line0 = row - 2 * delta;  // 128-byte aligned; only in-window floats are touched
    const float* src = lf + 2 * y * G::RS1;
    float val[JMAX];
    bool ok[JMAX];
    sfor<JMAX>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      const int c = 2 * j + half;
      const int w2 = 32 * c + e - 2 * delta;
      ok[j] = c < nline && w2 >= 0 && w2 < 2 * G::M;
      val[j] = ok[j] ? src[w2] : 0.0f;
    });
    sfor<JMAX>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      if (ok[j]) unsafeAtomicAdd(line0 + 32 * (2 * j + half) + e, val[j]);
    });
  }
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

// Everything one position needs, resolved by the caller (uniform across the
// workgroup).
struct PositionJob {
  const float2* win;     // object window origin: element (s, y, x) at win[s*sstride + y*ld + x]
  long long ld, sstride;
  int S;
  const float2* probe;
  const float* meas;     // this position's pattern [M][M]
  float* intens;         // this position's output pattern [M][M]
  float2* grad;          // gradient window origin, element (s, y, x) at grad[s*gslice + y*gld + x]
  long long gld, gslice;
  float gscale;          // 2 x the upstream gradient factor
  int ck;                // checkpoint interval of the incident waves (1: all kept)
  float2* probe_part;    // probe-gradient mode: this workgroup's partial sum (layout A)
};

// Per-workgroup state shared by all positions a workgroup processes.
template <class G>
struct Shared {
  float2 lds[G::LDS_ELEMS];
  float2 hx[G::M];
  double red[G::T / 64];
};

// Loads the separable propagator factor of a reconstruction: the x part into
// LDS, the y part of this thread's layout-C row (with the 1/M^2 of the inverse
// transform) into registers.  Contains no barrier.
template <class G>
__device__ __forceinline__ float2 load_propagator(Shared<G>& sh, const float2* __restrict__ h, const Lanes<G>& L) {
  load_hx_table<G>(sh.hx, h);
  const float2 hky = h[L.ky];
  const float inv_n = 1.0f / float(G::M * G::M);
  return make_float2(hky.x * inv_n, hky.y * inv_n);
}

// The whole per-position path (Section II-B and Eq. 1-2): multislice forward,
// detector plane (intensities, or the amplitude residual and its direction),
// and for the gradient mode the adjoint sweep with the scatter-add.  Returns
// the position loss in thread 0 (LOSS modes).  Starts and ends at a point where
// every LDS read of the previous position has completed.
// LINES: gradient atomics staged through LDS and aligned to 128-byte lines
// (scatter_add_lines); otherwise lanes are paired in registers (scatter_add).
// The staging costs an LDS round trip and two barriers per slice, which pays
// off for 128-windows over many slices (the tile walk) but not for 64-windows
// or the short slice stacks of the batched launch.
// AHEAD: the adjoint sweep requests each stored incident wave one propagation
// early (measured faster in the position-parallel launch, no faster in the
// batched one).
template <class G, int MODE, bool LINES = false, bool CKPT = false, bool AHEAD = false>
__device__ __forceinline__ double run_position(const PositionJob& jb, Shared<G>& sh, const float2 (&twb)[G::X1],
                                               float2 hy, float2* __restrict__ ws, const Lanes<G>& L) {
  constexpr bool GRAD = MODE == kModeLossGrad || MODE == kModeLossGradProbe;
  constexpr bool LOSS = MODE != kModeIntensity;
  const int S = jb.S;
  // Incident waves for the adjoint sweep.  The slices are cut into segments of
  // ck; the forward sweep keeps the wave entering every segment (a
  // checkpoint, psi_ck, psi_2ck, ...) and every wave of the last segment; the
  // adjoint sweep recomputes the inner waves of each earlier segment from its
  // checkpoint just before sweeping it (ck = 1: every wave is kept, nothing is
  // recomputed).  Slots: the checkpoints, then the inner waves of the segment
  // being swept, then one slot holding the adjoint wave while a segment is
  // recomputed (ws_slots(S, ck) in all).
  const int ck = CKPT ? jb.ck : 1;  // without CKPT the segment logic folds away at compile time
  const int last = ((S - 1) / ck) * ck;  // first slice of the last segment
  const int nck = last / ck;
  auto wave_slot = [&](int s, int seg) -> float2* {  // psi_s, s >= 1, of the segment starting at seg
    const int k = s == seg ? s / ck - 1 : nck + (s - seg - 1);
    return ws + static_cast<long long>(k + opaque_zero()) * (G::M * G::M);
  };
  float2 v[G::R];
  float2 t[G::R];  // the next slice's transmission window, loaded one propagation ahead
  load_window<G>(v, jb.probe, G::M, L);
  load_window<G>(t, jb.win, jb.ld, L);
  for (int s = 0; s < S; ++s) {
    if (GRAD && s >= 1 && (s % ck == 0 || s > last)) {
      float2* __restrict__ w = wave_slot(s, s % ck == 0 ? s : last);
      store_slot<G::R, G::T>(w, v, L.tid);
    }
    __builtin_amdgcn_sched_barrier(0);
    sfor<G::R>([&](auto rc) { v[decltype(rc)::value] = cmul(v[decltype(rc)::value], t[decltype(rc)::value]); });
    if (s + 1 < S) {
      load_window<G>(t, jb.win + (s + 1) * jb.sstride, jb.ld, L);  // in flight during the propagation
      // after the first slice the buffer was last read by the previous propagation's layout-A reads,
      // the slots each thread writes first
      propagate<G, false>(v, sh.lds, sh.hx, twb, hy, L, s > 0);
    }
  }
  dft2_a_to_c<G>(v, sh.lds, twb, L, S > 1);

  // ---- detector plane, layout C: element (ky, kx = jh*CJ + jl + X1*j2)
  const long long row = static_cast<long long>(L.ky) * G::M;
  if (!LOSS) {
    float* __restrict__ out = jb.intens + row;
    sfor<G::CJ>([&](auto lc) {
      sfor<G::X2>([&](auto jc) {
        constexpr int jl = decltype(lc)::value, j2 = decltype(jc)::value;
        const float2 e = v[jl * G::X2 + j2];
        out[L.jh * G::CJ + jl + G::X1 * j2] = e.x * e.x + e.y * e.y;
      });
    });
    return 0.0;
  }
  double acc = 0.0;
  const float* __restrict__ mrow = jb.meas + row;
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
    const float sc = mod > 0.0f ? jb.gscale * d / mod : 0.0f;
    e = make_float2(sc * e.x, sc * e.y);
  });
  // position loss: wave reduction, then across the waves through LDS
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((L.tid & 63) == 0) sh.red[L.tid >> 6] = acc;
  double f = 0.0;
  if (!GRAD) {
    __syncthreads();
    if (L.tid == 0)
      for (int w = 0; w < G::T / 64; ++w) f += sh.red[w];
    return f;  // the next position's first LDS write is preceded by a barrier
  }
  // ---- adjoint sweep
  idft2_c_to_a<G>(v, sh.lds, twb, L);  // chi_{S-1} = DFT^H g (its barriers make red[] visible)
  if (L.tid == 0)
    for (int w = 0; w < G::T / 64; ++w) f += sh.red[w];
  // One adjoint step at slice s of the segment starting at seg, with psi_s
  // from the store or the probe (s = 0).  psi_s and the transmission window
  // are consumed before the gradient atomics are issued: a wave's memory
  // operations retire in order, so its loads issued behind the atomics would
  // wait for them.  The atomics then drain while the propagation runs on LDS
  // and VALU; near its end (after its last exchange write) the loads of the
  // next step's psi_{s-1}, when the store already holds it, are issued so that
  // their latency overlaps the propagation's last barrier and pass.  (The
  // window as well would not fit the registers there: it spills.)
  float2 g[G::R];
  bool pre = false;  // g holds psi_s, requested by the previous step
  auto adjoint_step = [&](int s, int seg) {
    if (s == 0) {
      if constexpr (MODE == kModeLossGradProbe) {
        // dF/dP += chi_0 conj(t_0[window]) into this workgroup's partial sum (only this
        // thread touches these elements, so a plain read-modify-write is race-free)
        load_window<G>(g, jb.win, jb.ld, L);
        float2* __restrict__ pp = jb.probe_part + opaque_zero();
        float2 acc[G::R];
        sfor<G::R>([&](auto rc) { acc[decltype(rc)::value] = pp[decltype(rc)::value * G::T + L.tid]; });
        __builtin_amdgcn_sched_barrier(0);
        sfor<G::R>([&](auto rc) {
          constexpr int r = decltype(rc)::value;
          pp[r * G::T + L.tid] = cadd(acc[r], cmulc(v[r], g[r]));
        });
        __builtin_amdgcn_sched_barrier(0);
      }
      load_window<G>(g, jb.probe, G::M, L);
      __builtin_amdgcn_sched_barrier(0);
      sfor<G::R>([&](auto rc) { g[decltype(rc)::value] = cmulc(v[decltype(rc)::value], g[decltype(rc)::value]); });
    } else {
      if (!pre) {
        const float2* __restrict__ w = wave_slot(s, seg);
        load_slot<G::R, G::T>(g, w, L.tid);
      }
      load_window<G>(t, jb.win + s * jb.sstride, jb.ld, L);
      __builtin_amdgcn_sched_barrier(0);
      sfor<G::R>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        g[r] = cmulc(v[r], g[r]);
        v[r] = cmulc(v[r], t[r]);
      });
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (LINES) {
      // no barrier: the last LDS access before this was the layout-A read that ends every transform,
      // of the slots each thread now writes
      e1_write_a<G>(sh.lds + opaque_zero(), g, L.n2, L.x);
      __syncthreads();
      scatter_add_lines<G>(jb.grad + s * jb.gslice, jb.gld, sh.lds, L);
    } else {
      scatter_add<G>(jb.grad + s * jb.gslice, jb.gld, g, L);
    }
    if (s > 0) {
      if constexpr (!AHEAD) {
        propagate<G, true>(v, sh.lds, sh.hx, twb, hy, L);
      } else {
        // psi_{s-1} is in the store now if it belongs to this segment or is a checkpoint (the inner
        // waves of an earlier segment are recomputed first); slice 0 takes the probe at its own step
        const int s1 = s - 1;
        const bool nxt = s1 >= 1 && (s1 >= seg || s1 % ck == 0);
        const float2* __restrict__ nw = nxt ? wave_slot(s1, s1 >= seg ? seg : s1) : ws;
        propagate<G, true>(v, sh.lds, sh.hx, twb, hy, L, false, [&]() {
          // both branches define g, so it is not live across the propagation
          if (nxt) {
            load_slot<G::R, G::T>(g, nw, L.tid);
          } else {
            sfor<G::R>([&](auto rc) { g[decltype(rc)::value] = make_float2(0.f, 0.f); });
          }
        });
        pre = nxt;
      }
    }
  };
  if constexpr (!CKPT) {
    for (int s = S - 1; s >= 0; --s) adjoint_step(s, s);
  } else {
    for (int seg = last; seg >= 0; seg -= ck) {
      const int seg_end = seg + ck < S ? seg + ck : S;
      if (seg < last && seg_end - seg > 1) {
        // recompute psi_{seg+1 .. seg_end-1} from the checkpoint; the adjoint wave waits in its slot
        float2* __restrict__ park = ws + static_cast<long long>(nck + (ck < S ? ck : S) - 1 + opaque_zero()) *
                                             (G::M * G::M);
        store_slot<G::R, G::T>(park, v, L.tid);
        if (seg == 0) {
          load_window<G>(v, jb.probe, G::M, L);
        } else {
          const float2* __restrict__ w = wave_slot(seg, seg);
          load_slot<G::R, G::T>(v, w, L.tid);
        }
        for (int s = seg; s + 1 < seg_end; ++s) {
          load_window<G>(t, jb.win + s * jb.sstride, jb.ld, L);
          __builtin_amdgcn_sched_barrier(0);
          sfor<G::R>([&](auto rc) { v[decltype(rc)::value] = cmul(v[decltype(rc)::value], t[decltype(rc)::value]); });
          propagate<G, false>(v, sh.lds, sh.hx, twb, hy, L);
          float2* __restrict__ w = wave_slot(s + 1, seg);
          store_slot<G::R, G::T>(w, v, L.tid);
        }
        const float2* __restrict__ pk = park + opaque_zero();
        load_slot<G::R, G::T>(v, pk, L.tid);
        if constexpr (AHEAD) {
          // the step below loads psi itself (nothing was requested across a segment boundary);
          // defining g here keeps it from being live across the recomputation
          sfor<G::R>([&](auto rc) { g[decltype(rc)::value] = make_float2(0.f, 0.f); });
          pre = false;
        }
      }
      for (int s = seg_end - 1; s >= seg; --s) adjoint_step(s, seg);
    }
  }
  __syncthreads();  // red[] and lds reuse by the next position
  return f;
}

// Waves per SIMD the position kernels are compiled for: a 128-window workgroup
// (8 waves, 136 KB of LDS) fills a CU alone; three 64-window workgroups (4
// waves, 35 KB of LDS each) share one, which caps the registers at 168 per lane.
template <int M>
constexpr int kWavesPerSimd = M == 64 ? 3 : 2;

template <int M, int MODE>
__global__ void __launch_bounds__(Geo<M>::T, kWavesPerSimd<M>) fused_kernel(KernelArgs a) {
  using G = Geo<M>;
  constexpr bool LOSS = MODE != kModeIntensity;
  __shared__ Shared<G> sh;
  const Lanes<G> L;
  float2 twb[G::X1];
  load_twb<G>(twb, a.tw, L.m2);
  const float2 hy = load_propagator<G>(sh, a.h, L);
  __syncthreads();

  const int S = a.S;
  float2* __restrict__ ws = a.ws + static_cast<long long>(blockIdx.x) * ws_slots(S, a.ck) * (G::M * G::M);
  PositionJob jb;
  jb.ld = a.ld;
  jb.sstride = a.slice_stride;
  jb.S = S;
  jb.probe = a.probe;
  jb.gld = a.gld;
  jb.gslice = a.gslice;
  jb.gscale = 2.0f * (a.grad_scale != nullptr ? static_cast<float>(*a.grad_scale) : 1.0f);
  jb.ck = a.ck;
  jb.probe_part = nullptr;
  if constexpr (MODE == kModeLossGradProbe) {
    jb.probe_part = a.probe_part + static_cast<long long>(blockIdx.x) * (G::M * G::M);
    sfor<G::R>([&](auto rc) { jb.probe_part[decltype(rc)::value * G::T + L.tid] = make_float2(0.f, 0.f); });
  }

  for (int j = 0;; ++j) {
    const int p = job_position(j, a.n, static_cast<int>(gridDim.x));
    if (p < 0) break;
    const int gy = a.pos[2 * p], gx = a.pos[2 * p + 1];
    const int y0 = gy - a.oy, x0 = gx - a.ox;
    bool ok;
    if (a.tiles != nullptr) {  // all-tiles mode: the owning tile's box and gradient buffer (uniform)
      const int tk = a.tile_of_pos[p];
      ok = tk >= 0 && tk < a.ntiles;
      unsigned flag = 4u;
      if (ok) {
        const TileDesc& T = a.tiles[tk];
        const int cy = gy + M / 2, cx = gx + M / 2;
        ok = cy >= T.ty0 && cy < T.ty1 && cx >= T.tx0 && cx < T.tx1;
        if (ok) {
          ok = gy >= T.ey0 && gx >= T.ex0 && gy + M <= T.ey0 + T.eh && gx + M <= T.ex0 + T.ew;
          flag = 2u;
        }
        if (ok) {
          jb.grad = T.grad + static_cast<long long>(gy - T.ey0) * T.gld + (gx - T.ex0);
          jb.gld = T.gld;
          jb.gslice = T.gslice;
        }
      }
      if (!ok && threadIdx.x == 0) atomicOr(a.status, flag);
    } else {
      ok = check_window(a, y0, x0, gy, gx);
      jb.grad = a.grad + static_cast<long long>(y0) * a.gld + x0;
    }
    if (!ok) {
      if (LOSS && threadIdx.x == 0) {
        a.loss_work[p] = 0.0;
        if (a.loss_pos != nullptr) a.loss_pos[p] = 0.0;
      }
      continue;
    }
    jb.win = a.obj + static_cast<long long>(y0) * a.ld + x0;
    jb.probe = a.probe + static_cast<long long>(p) * a.probe_stride;
    jb.meas = a.meas + static_cast<long long>(p) * (G::M * G::M);
    jb.intens = a.intens + static_cast<long long>(p) * (G::M * G::M);
    const double f = run_position<G, MODE, G::M == 128, true, true>(jb, sh, twb, hy, ws, L);
    if (LOSS && L.tid == 0) {
      a.loss_work[p] = f;
      if (a.loss_pos != nullptr) a.loss_pos[p] = f;
    }
  }
}

// ---------------------------------------------------------------------------
// Batched persistent launch: a work list of (reconstruction, position) items
// over many independent reconstructions with the same window size (uneven
// objects, slice counts and scans), one workgroup per CU walking the list.
// ---------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(Geo<M>::T, kWavesPerSimd<M>) batch_kernel(BatchArgs a) {
  using G = Geo<M>;
  __shared__ Shared<G> sh;
  __shared__ int job;
  const Lanes<G> L;
  float2 twb[G::X1];
  load_twb<G>(twb, a.tw, L.m2);
  float2* __restrict__ ws = a.ws + static_cast<long long>(blockIdx.x) * ws_slots(a.smax, 1) * (G::M * G::M);
  int cur = -1;
  float2 hy = make_float2(0.f, 0.f);
  PositionJob jb;
  // this workgroup's queue: blocks are dispatched round-robin over the 8 XCDs
  const int x = gridDim.x >= 8 ? static_cast<int>(blockIdx.x & 7) : 0;
  const int end = gridDim.x >= 8 ? a.bounds[x + 1] : a.bounds[8];  // parts are contiguous
  for (;;) {
    __syncthreads();  // every lane has read the previous job index
    if (threadIdx.x == 0) job = atomicAdd(&a.next[x], 1);
    __syncthreads();
    const int k = job;
    if (k >= end) break;
    const int item = a.item0 + k;
    const int r = a.items[2 * item];
    const int p = a.items[2 * item + 1];
    const BatchRecon& R = a.recs[r];
    if (r != cur) {  // uniform: a new reconstruction's propagator
      __syncthreads();
      hy = load_propagator<G>(sh, R.h, L);
      __syncthreads();
      cur = r;
    }
    const int y0 = R.pos[2 * p], x0 = R.pos[2 * p + 1];
    if (!(y0 >= 0 && x0 >= 0 && y0 + M <= R.H && x0 + M <= R.W)) {
      if (threadIdx.x == 0) {
        atomicOr(a.status, 1u);
        a.item_loss[item] = 0.0;
      }
      continue;
    }
    jb.win = R.obj + static_cast<long long>(y0) * R.ld + x0;
    jb.ld = R.ld;
    jb.sstride = R.slice_stride;
    jb.S = R.S;
    jb.probe = R.probe;
    jb.meas = R.meas + static_cast<long long>(p) * (G::M * G::M);
    jb.intens = nullptr;
    jb.grad = R.grad + static_cast<long long>(y0) * R.ld + x0;
    jb.gld = R.ld;
    jb.gslice = R.slice_stride;
    jb.gscale = 2.0f;
    jb.ck = 1;
    const double f = run_position<G, kModeLossGrad, G::M == 128>(jb, sh, twb, hy, ws, L);
    if (L.tid == 0) a.item_loss[item] = f;
  }
}

__global__ void copy_ints_kernel(const int* __restrict__ src, int* __restrict__ dst, int n) {
  const int i = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) dst[i] = src[i];
}

// losses[r] = sum of the item losses of reconstruction r in item order; also
// appends it to the history row *iter (when the history is enabled).
__global__ void __launch_bounds__(256) batch_finalize_kernel(const BatchRecon* __restrict__ recs,
                                                             const double* __restrict__ item_loss,
                                                             double* __restrict__ losses, double* __restrict__ hist,
                                                             const int* __restrict__ iter, int hist_rows, int nrecon) {
  __shared__ double part[256];
  const int r = blockIdx.x;
  const BatchRecon& R = recs[r];
  double s = 0.0;
  for (int i = threadIdx.x; i < R.n; i += blockDim.x) s += item_loss[R.item0 + i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    losses[r] = part[0];
    if (hist != nullptr) {
      const int it = *iter;
      if (it >= 0 && it < hist_rows) hist[static_cast<long long>(it) * nrecon + r] = part[0];
    }
  }
}

// mode 0: grad = 0 for every reconstruction; mode 1: obj -= alpha * grad, and
// the history row counter advances by one.
__global__ void batch_elementwise_kernel(const BatchRecon* __restrict__ recs, int mode, int* __restrict__ iter) {
  const BatchRecon& R = recs[blockIdx.y];
  const long long total = static_cast<long long>(R.S) * R.H * R.W;
  const float al = R.alpha;
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<long long>(gridDim.x) * blockDim.x) {
    const long long s = i / (static_cast<long long>(R.H) * R.W);
    const long long q = i - s * R.H * R.W;
    const long long y = q / R.W, x = q - y * R.W;
    const long long o = s * R.slice_stride + y * R.ld + x;
    if (mode == 0) {
      R.grad[o] = make_float2(0.f, 0.f);
    } else {
      const float2 g = R.grad[o];
      float2 t = R.obj[o];
      t.x -= al * g.x;
      t.y -= al * g.y;
      R.obj[o] = t;
    }
  }
  if (mode == 1 && iter != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *iter += 1;
}

__global__ void set_int_kernel(int* p, int v) { *p = v; }

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

// One exchange of the accumulation passes: dst = src, or dst += alpha * src,
// over an oh x ow region of S slices (both pointers at the region's top-left).  Workgroups walk rows
// of one slice (blockIdx.y), threads walk columns: row segments are
// contiguous, so loads and stores coalesce.
__global__ void box_exchange_kernel(const float2* __restrict__ src, long long sslice, long long sld,
                                    float2* __restrict__ dst, long long dslice, long long dld, int oh, int ow,
                                    int replace, float alpha) {
  const long long s = blockIdx.y;
  for (int y = blockIdx.x; y < oh; y += gridDim.x) {
    const float2* __restrict__ sp = src + s * sslice + y * sld;
    float2* __restrict__ dp = dst + s * dslice + y * dld;
    for (int x = threadIdx.x; x < ow; x += blockDim.x) {
      const float2 v = sp[x];
      if (replace) {
        dp[x] = v;
      } else {
        const float2 d = dp[x];
        dp[x] = make_float2(d.x + alpha * v.x, d.y + alpha * v.y);
      }
    }
  }
}

// Real-potential parametrisation of the slices, t = exp(i sigma V): the
// transmission from the potential (mode 0) and the chain rule of the complex
// gradient G = dF/dRe t + i dF/dIm t to the potential, dF/dV = sigma Im(conj(t) G)
// (mode 1).  Workgroups walk rows of one slice (blockIdx.y), threads columns.
__global__ void potential_kernel(int mode, float sigma, int H, int W, const float* __restrict__ V, long long vs,
                                 long long vld, float2* __restrict__ t_out, const float2* __restrict__ t_in,
                                 long long ts, long long tld, const float2* __restrict__ g, long long gs,
                                 long long gld, float* __restrict__ gv, long long gvs, long long gvld) {
  const long long s = blockIdx.y;
  for (int y = blockIdx.x; y < H; y += gridDim.x) {
    for (int x = threadIdx.x; x < W; x += blockDim.x) {
      if (mode == 0) {
        float sn, cs;
        sincosf(sigma * V[s * vs + y * vld + x], &sn, &cs);
        t_out[s * ts + y * tld + x] = make_float2(cs, sn);
      } else {
        const float2 t = t_in[s * ts + y * tld + x];
        const float2 d = g[s * gs + y * gld + x];
        gv[s * gvs + y * gvld + x] = sigma * (t.x * d.y - t.y * d.x);
      }
    }
  }
}

// Zeroes every tile gradient of an all-tiles launch (blockIdx.y = tile).
__global__ void zero_tiles_kernel(const TileDesc* __restrict__ tiles, int S) {
  const TileDesc& T = tiles[blockIdx.y];
  const long long total = static_cast<long long>(S) * T.eh * T.ew;  // dense buffers
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    T.grad[i] = make_float2(0.f, 0.f);
}

// probe_grad[y][x] (+)= sum over the workgroups' partial sums, which hold pixel
// (y, x) = (Y2*r + n2, x) at index r*T + n2*M + x (layout A).  The sum runs in
// workgroup order, so the result does not depend on timing.
template <int M>
__global__ void probe_reduce_kernel(const float2* __restrict__ part, int parts, float2* __restrict__ out,
                                    int accumulate) {
  using G = Geo<M>;
  const int i = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= M * M) return;
  const int r = i / G::T, tid = i % G::T;
  const int y = G::Y2 * r + tid / M, x = tid % M;
  float sx = 0.f, sy = 0.f;
  for (int b = 0; b < parts; ++b) {
    const float2 v = part[static_cast<long long>(b) * (M * M) + i];
    sx += v.x;
    sy += v.y;
  }
  float2& o = out[y * M + x];
  o = accumulate ? make_float2(o.x + sx, o.y + sy) : make_float2(sx, sy);
}

// ---------------------------------------------------------------------------
// launchers (host side)
// ---------------------------------------------------------------------------
template <int M, int MODE>
static hipError_t launch_fused_t(const KernelArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((fused_kernel<M, MODE>), dim3(grid), dim3(Geo<M>::T), 0, st, a);
  return hipGetLastError();
}

template <int M>
static hipError_t launch_fused_m(const KernelArgs& a, int mode, int grid, hipStream_t st) {
  switch (mode) {
    case kModeIntensity: return launch_fused_t<M, kModeIntensity>(a, grid, st);
    case kModeLoss: return launch_fused_t<M, kModeLoss>(a, grid, st);
    case kModeLossGrad: return launch_fused_t<M, kModeLossGrad>(a, grid, st);
    case kModeLossGradProbe: return launch_fused_t<M, kModeLossGradProbe>(a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Sub-pixel probe translation: out[p] = F^-1[F(probe) exp(-2 pi i (q_y d_y + q_x d_x)/M)]
// with (d_y, d_x) = shifts[p] and integer frequencies q (-M/2 at the Nyquist bin),
// one workgroup per position, on the same register/LDS transforms as the
// fused kernels.
// ---------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(Geo<M>::T) shift_probe_kernel(const float2* __restrict__ probe,
                                                                const float* __restrict__ shifts, int n,
                                                                const float2* __restrict__ tw,
                                                                float2* __restrict__ out) {
  using G = Geo<M>;
  __shared__ float2 lds[G::LDS_ELEMS];
  const Lanes<G> L;
  const int p = static_cast<int>(blockIdx.x);
  if (p >= n) return;
  float2 twb[G::X1];
  load_twb<G>(twb, tw, L.m2);
  float2 v[G::R];
  load_window<G>(v, probe, G::M, L);
  dft2_a_to_c<G>(v, lds, twb, L);
  const float dy = shifts[2 * p], dx = shifts[2 * p + 1];
  const int qy = L.ky < M / 2 ? L.ky : L.ky - M;
  const float inv_n = 1.0f / float(M * M);
  sfor<G::CJ>([&](auto lc) {
    sfor<G::X2>([&](auto jc) {
      constexpr int jl = decltype(lc)::value, j2 = decltype(jc)::value;
      const int kx = L.jh * G::CJ + jl + G::X1 * j2;
      const int qx = kx < M / 2 ? kx : kx - M;
      // phase -2 pi (qy dy + qx dx)/M, in units of pi, reduced to [-1, 1] before the sine/cosine
      float t = -2.0f * (static_cast<float>(qy) * dy + static_cast<float>(qx) * dx) / float(M);
      t -= 2.0f * rintf(0.5f * t);
      float sn, cs;
      sincospif(t, &sn, &cs);
      float2& e = v[jl * G::X2 + j2];
      e = cmul(e, make_float2(cs * inv_n, sn * inv_n));
    });
  });
  idft2_c_to_a<G>(v, lds, twb, L);
  float2* __restrict__ o = out + static_cast<long long>(p) * (M * M) + L.n2 * M + L.x;
  sfor<G::R>([&](auto rc) { o[decltype(rc)::value * G::Y2 * M] = v[decltype(rc)::value]; });
}

hipError_t launch_shift_probes(const float2* probe, const float* shifts, int n, int M, const float2* tw, float2* out,
                               hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (M == 128) {
    hipLaunchKernelGGL((shift_probe_kernel<128>), dim3(n), dim3(Geo<128>::T), 0, st, probe, shifts, n, tw, out);
  } else if (M == 64) {
    hipLaunchKernelGGL((shift_probe_kernel<64>), dim3(n), dim3(Geo<64>::T), 0, st, probe, shifts, n, tw, out);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fused(const KernelArgs& a, int mode, int grid, hipStream_t st) {
  if (a.M == 128) return launch_fused_m<128>(a, mode, grid, st);
  if (a.M == 64) return launch_fused_m<64>(a, mode, grid, st);
  return hipErrorInvalidValue;
}

hipError_t launch_batch(const BatchArgs& a, int M, int grid, hipStream_t st) {
  if (M == 128) {
    hipLaunchKernelGGL((batch_kernel<128>), dim3(grid), dim3(Geo<128>::T), 0, st, a);
  } else if (M == 64) {
    hipLaunchKernelGGL((batch_kernel<64>), dim3(grid), dim3(Geo<64>::T), 0, st, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_finalize(const BatchRecon* recs, const double* item_loss, double* losses, double* hist,
                                 const int* iter, int hist_rows, int nrecon, hipStream_t st) {
  if (nrecon == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_finalize_kernel, dim3(nrecon), dim3(256), 0, st, recs, item_loss, losses, hist, iter,
                     hist_rows, nrecon);
  return hipGetLastError();
}

hipError_t launch_batch_elementwise(const BatchRecon* recs, int nrecon, int mode, int* iter, hipStream_t st) {
  if (nrecon == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_elementwise_kernel, dim3(512, nrecon), dim3(256), 0, st, recs, mode, iter);
  return hipGetLastError();
}

hipError_t launch_set_int(int* p, int v, hipStream_t st) {
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, st, p, v);
  return hipGetLastError();
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

hipError_t launch_box_exchange(const float2* src, long long sslice, long long sld, float2* dst, long long dslice,
                               long long dld, int S, int oh, int ow, bool replace, float alpha, hipStream_t st) {
  const unsigned rows = static_cast<unsigned>(oh < 1024 ? oh : 1024);
  hipLaunchKernelGGL(box_exchange_kernel, dim3(rows, static_cast<unsigned>(S)), dim3(256), 0, st, src, sslice, sld,
                     dst, dslice, dld, oh, ow, replace ? 1 : 0, alpha);
  return hipGetLastError();
}

hipError_t launch_copy_ints(const int* src, int* dst, int n, hipStream_t st) {
  hipLaunchKernelGGL(copy_ints_kernel, dim3(static_cast<unsigned>((n + 63) / 64)), dim3(64), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_potential(int mode, float sigma, int S, int H, int W, const float* V, long long vs, long long vld,
                            float2* t_out, const float2* t_in, long long ts, long long tld, const float2* g,
                            long long gs, long long gld, float* gv, long long gvs, long long gvld, hipStream_t st) {
  const unsigned rows = static_cast<unsigned>(H < 1024 ? H : 1024);
  hipLaunchKernelGGL(potential_kernel, dim3(rows, static_cast<unsigned>(S)), dim3(256), 0, st, mode, sigma, H, W, V,
                     vs, vld, t_out, t_in, ts, tld, g, gs, gld, gv, gvs, gvld);
  return hipGetLastError();
}

hipError_t launch_zero_tiles(const TileDesc* tiles, int ntiles, int S, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_tiles_kernel, dim3(256, static_cast<unsigned>(ntiles)), dim3(256), 0, st, tiles, S);
  return hipGetLastError();
}

hipError_t launch_probe_reduce(const float2* part, int parts, int M, float2* probe_grad, bool accumulate,
                               hipStream_t st) {
  const unsigned blocks = static_cast<unsigned>((M * M + 255) / 256);
  if (M == 128) {
    hipLaunchKernelGGL(probe_reduce_kernel<128>, dim3(blocks), dim3(256), 0, st, part, parts, probe_grad,
                       accumulate ? 1 : 0);
  } else if (M == 64) {
    hipLaunchKernelGGL(probe_reduce_kernel<64>, dim3(blocks), dim3(256), 0, st, part, parts, probe_grad,
                       accumulate ? 1 : 0);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_clear_status(unsigned* status, hipStream_t st) {
  hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(1), 0, st, status);
  return hipGetLastError();
}

}  // namespace ptycho
