// fft_lds.hpp -- register/LDS 2D DFT building blocks for CDNA4 (gfx950, wave64).
//
// A window of M x M complex64 values (M = 64 or 128) is spread over the
// registers of one workgroup: T = 4*M threads, each holding R = M/4 points.
// A 2D DFT is three register passes separated by two LDS exchanges:
//
//   y = Y2*n1 + n2, ky = k1 + Y1*k2          (Y1 = R, Y2 = 4)
//   x = X2*m1 + m2, kx = j1 + X1*j2          (X2 = 16, X1 = M/16)
//
//   layout A  thread (n2, x)   registers n1 -> k1 : DFT-Y1 along y, twiddle W_M^(n2 k1)
//   layout B  thread (k1, m2)  registers (n2, m1) : DFT-4 along y (n2 -> k2),
//                              DFT-X1 along x (m1 -> j1), twiddle W_M^(m2 j1)
//   layout C  thread (ky, jh)  registers (jl, m2) : DFT-16 along x (m2 -> j2),
//                              j1 = jh*CJ + jl, CJ = X1/4
//
// In layout C, thread t = Y2*c + jh takes ky = 4*(c/16) + c%4 + Y1*((c/4)%4)
// (layout_c_ky), so that a wave reads and writes only the exchange rows that
// the same wave writes and reads in layout B (see the exchanges below).
//
// The inverse runs the same passes backwards with conjugate twiddles, so a
// forward DFT, a pointwise multiply in layout C and an inverse DFT need no
// reordering in between, and the inverse ends in layout A, where the next
// slice's transmission is applied with coalesced loads along x.
//
// This is plain mixed-radix Cooley-Tukey (decimation in time within each
// small DFT); all twiddles of the small DFTs are compile-time constants
// computed in double precision and rounded once to float.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

namespace ptycho {

// ---------------------------------------------------------------------------
// compile-time helpers
// ---------------------------------------------------------------------------
template <class F, int... Is>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double cx_sin_series(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double cx_cos_series(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
// cos and sin of 2*pi*num/den, with the angle reduced to |x| <= pi/4 using
// exact integer arithmetic before the series.
constexpr double cx_cos2pi(long num, long den) {
  num %= den;
  if (num < 0) num += den;
  long k = (4 * num + den / 2) / den;
  long r = 4 * num - k * den;
  double x = (kPi / 2.0) * double(r) / double(den);
  double s = cx_sin_series(x), c = cx_cos_series(x);
  switch (k & 3) {
    case 0: return c;
    case 1: return -s;
    case 2: return -c;
    default: return s;
  }
}
constexpr double cx_sin2pi(long num, long den) {
  num %= den;
  if (num < 0) num += den;
  long k = (4 * num + den / 2) / den;
  long r = 4 * num - k * den;
  double x = (kPi / 2.0) * double(r) / double(den);
  double s = cx_sin_series(x), c = cx_cos_series(x);
  switch (k & 3) {
    case 0: return s;
    case 1: return c;
    case 2: return -s;
    default: return -c;
  }
}

// ---------------------------------------------------------------------------
// complex arithmetic on float2
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 mul_i(float2 a) { return make_float2(-a.y, a.x); }    // *(+i)
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }   // *(-i)

// a * W_N^E with W_N = exp(-2 pi i / N) (forward) or exp(+2 pi i / N) (INV).
template <int E, int N, bool INV>
__device__ __forceinline__ float2 twiddle(float2 a) {
  constexpr int e = ((E % N) + N) % N;
  if constexpr (e == 0) {
    return a;
  } else if constexpr (2 * e == N) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (4 * e == N) {
    return INV ? mul_i(a) : mul_mi(a);
  } else if constexpr (4 * e == 3 * N) {
    return INV ? mul_mi(a) : mul_i(a);
  } else if constexpr ((8 * e) % N == 0) {
    // odd multiples of 45 degrees: (+-1 +- i)/sqrt(2)
    constexpr float h = 0.70710678118654752440f;
    constexpr float c = float(cx_cos2pi(e, N)) > 0.f ? h : -h;
    constexpr float s0 = float(cx_sin2pi(e, N)) > 0.f ? h : -h;
    constexpr float s = INV ? s0 : -s0;  // imaginary part of the twiddle
    return make_float2(c * a.x - s * a.y, c * a.y + s * a.x);
  } else {
    constexpr float c = float(cx_cos2pi(e, N));
    constexpr float s = INV ? float(cx_sin2pi(e, N)) : float(-cx_sin2pi(e, N));
    return make_float2(c * a.x - s * a.y, c * a.y + s * a.x);
  }
}

// In-register DFT of N points (power of two), natural order in and out.
// Radix-4 decimation in time, recursing on the four decimated subsequences.
template <int N, bool INV>
__device__ __forceinline__ void dft(float2 (&v)[N]) {
  if constexpr (N == 1) {
    return;
  } else if constexpr (N == 2) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (N == 4) {
    float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    float2 t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    float2 r = INV ? mul_i(t3) : mul_mi(t3);
    v[1] = cadd(t1, r);
    v[3] = csub(t1, r);
  } else {
    constexpr int K = N / 4;
    float2 s0[K], s1[K], s2[K], s3[K];
    sfor<K>([&](auto mc) {
      constexpr int m = decltype(mc)::value;
      s0[m] = v[4 * m + 0];
      s1[m] = v[4 * m + 1];
      s2[m] = v[4 * m + 2];
      s3[m] = v[4 * m + 3];
    });
    dft<K, INV>(s0);
    dft<K, INV>(s1);
    dft<K, INV>(s2);
    dft<K, INV>(s3);
    sfor<K>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      float2 a0 = s0[k];
      float2 a1 = twiddle<1 * k, N, INV>(s1[k]);
      float2 a2 = twiddle<2 * k, N, INV>(s2[k]);
      float2 a3 = twiddle<3 * k, N, INV>(s3[k]);
      float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
      float2 t2 = cadd(a1, a3), t3 = csub(a1, a3);
      float2 r = INV ? mul_i(t3) : mul_mi(t3);
      v[k] = cadd(t0, t2);
      v[k + 2 * K] = csub(t0, t2);
      v[k + K] = cadd(t1, r);
      v[k + 3 * K] = csub(t1, r);
    });
  }
}

// DFT over registers v[OFF + i*STR], i = 0..N-1.
template <int N, int OFF, int STR, bool INV, int R>
__device__ __forceinline__ void dft_strided(float2 (&v)[R]) {
  float2 t[N];
  sfor<N>([&](auto ic) { t[decltype(ic)::value] = v[OFF + decltype(ic)::value * STR]; });
  dft<N, INV>(t);
  sfor<N>([&](auto ic) { v[OFF + decltype(ic)::value * STR] = t[decltype(ic)::value]; });
}

// ---------------------------------------------------------------------------
// geometry of one window size
// ---------------------------------------------------------------------------
template <int M_>
struct Geo {
  static constexpr int M = M_;
  static constexpr int Y2 = 4;
  static constexpr int Y1 = M / Y2;        // registers per thread
  static constexpr int R = Y1;
  static constexpr int X2 = 16;
  static constexpr int X1 = M / X2;
  static constexpr int CJ = X1 / Y2;       // j1 values per thread in layout C
  static constexpr int T = Y2 * M;         // threads per workgroup
  static constexpr int PAD1 = 3;           // row padding of the exchanges (complex; odd, see below)
  static constexpr int RS1 = M + PAD1;
  static constexpr int PAD2 = PAD1;        // the two exchanges share rows
  static constexpr int RS2 = M + PAD2;
  static constexpr int LDS_ELEMS = M * (RS1 > RS2 ? RS1 : RS2);
  static_assert(X1 % Y2 == 0, "layout C needs X1 divisible by 4");
  static_assert(Y1 * X2 == T && Y2 * X1 == R && CJ * X2 == R, "inconsistent layout");
};

// ---------------------------------------------------------------------------
// pass A: DFT along y over the registers, then (forward) the twiddle
// W_M^(n2*k1); n2 is uniform in a wave, so the twiddles are compile-time
// constants selected by a uniform branch.
// ---------------------------------------------------------------------------
template <class G, bool INV, int N2>
__device__ __forceinline__ void twiddle_a_fixed(float2 (&v)[G::R]) {
  sfor<G::R>([&](auto kc) {
    constexpr int k1 = decltype(kc)::value;
    v[k1] = twiddle<N2 * k1, G::M, INV>(v[k1]);
  });
}
template <class G, bool INV>
__device__ __forceinline__ void twiddle_a(float2 (&v)[G::R], int n2) {
  static_assert(G::Y2 == 4, "twiddle_a is written for Y2 = 4");
  switch (n2) {
    case 1: twiddle_a_fixed<G, INV, 1>(v); break;
    case 2: twiddle_a_fixed<G, INV, 2>(v); break;
    case 3: twiddle_a_fixed<G, INV, 3>(v); break;
    default: break;
  }
}
template <class G>
__device__ __forceinline__ void pass_a_fwd(float2 (&v)[G::R], int n2) {
  dft<G::R, false>(v);
  twiddle_a<G, false>(v, n2);
}
template <class G>
__device__ __forceinline__ void pass_a_inv(float2 (&v)[G::R], int n2) {
  twiddle_a<G, true>(v, n2);
  dft<G::R, true>(v);
}

// ---------------------------------------------------------------------------
// pass B: registers b[n2*X1 + m1] (forward input) / b[k2*X1 + j1] (output).
// tw[j1] = W_M^(m2*j1) for this thread's m2 (forward values).
// ---------------------------------------------------------------------------
template <class G>
__device__ __forceinline__ void pass_b_fwd(float2 (&b)[G::R], const float2 (&tw)[G::X1]) {
  sfor<G::X1>([&](auto mc) { dft_strided<G::Y2, decltype(mc)::value, G::X1, false>(b); });
  sfor<G::Y2>([&](auto kc) { dft_strided<G::X1, decltype(kc)::value * G::X1, 1, false>(b); });
  sfor<G::Y2>([&](auto kc) {
    sfor<G::X1 - 1>([&](auto jc) {
      constexpr int j1 = decltype(jc)::value + 1;
      constexpr int i = decltype(kc)::value * G::X1 + j1;
      b[i] = cmul(b[i], tw[j1]);
    });
  });
}
template <class G>
__device__ __forceinline__ void pass_b_inv(float2 (&b)[G::R], const float2 (&tw)[G::X1]) {
  sfor<G::Y2>([&](auto kc) {
    sfor<G::X1 - 1>([&](auto jc) {
      constexpr int j1 = decltype(jc)::value + 1;
      constexpr int i = decltype(kc)::value * G::X1 + j1;
      b[i] = cmulc(b[i], tw[j1]);
    });
  });
  sfor<G::Y2>([&](auto kc) { dft_strided<G::X1, decltype(kc)::value * G::X1, 1, true>(b); });
  sfor<G::X1>([&](auto mc) { dft_strided<G::Y2, decltype(mc)::value, G::X1, true>(b); });
}

// pass C: registers c[jl*X2 + m2] -> c[jl*X2 + j2]
template <class G, bool INV>
__device__ __forceinline__ void pass_c(float2 (&c)[G::R]) {
  sfor<G::CJ>([&](auto lc) { dft_strided<G::X2, decltype(lc)::value * G::X2, 1, INV>(c); });
}

// ---------------------------------------------------------------------------
// LDS exchanges.  E1 holds element (k1, n2, x) at (k1*Y2 + n2)*RS1 + x.
// E2 holds element (ky, j1, m2) in row Y2*(ky % Y1) + ky / Y1 at column
// j1*X2 + (m2 ^ jh), jh = j1 / CJ.  The row order puts the E2 data of
// layout-B thread (k1, m2) in the rows Y2*k1 .. Y2*k1 + 3 that hold its E1
// data, so wave w of layout B (k1 = 4w .. 4w+3) reads and writes the same 16
// whole rows 16w .. 16w+15 in both exchanges.  Those rows hold
// ky = 4w + a + Y1*b (a, b = 0..3), which are exactly the ky of wave w in
// layout C (layout_c_ky): the B <-> C exchange never crosses a wave.
// Banks: the row stride is odd (M + 3 complex), so the four consecutive ky
// of a 16-lane layout-C access (a = 0..3), Y2 rows apart, start 8 banks apart
// (of 32), and the xor with jh spreads its four jh lanes within those 8;
// every other access runs along a row.
//
// Barriers.  A thread that writes an exchange only overwrites slots that it,
// or its own wave, read last:
//   * layout B: the E1 rows of a wave are its E2 rows (B -> C after A -> B,
//     and B -> A after C -> B), and every value written depends on all
//     values the thread read, so the writes follow the reads in the wave's
//     instruction stream, and LDS operations of one wave complete in order;
//   * layout C writes exactly the slots it read (C -> B after B -> C);
//   * layout A writes exactly the slots it read (A -> B after B -> A).
// So the barrier before such a write is not needed.  Between the writes and
// the reads of an exchange, A <-> B needs a workgroup barrier; B <-> C stays
// within each wave and needs only wave_sync, which keeps the compiler from
// moving LDS accesses across it (the hardware already runs one wave's LDS
// operations in order).  The first write of a transform (layout A) keeps its
// barrier unless its caller knows that the last access to the buffer was the
// layout-A read ending the previous transform; otherwise the buffer may have
// served another purpose since.
// ---------------------------------------------------------------------------
template <class G>
__device__ __forceinline__ int layout_c_ky(int tid) {
  static_assert(G::Y2 == 4 && G::T % 64 == 0, "layout C pairing is written for Y2 = 4, whole waves");
  const int c = tid / G::Y2;
  return 4 * (c >> 4) + (c & 3) + G::Y1 * ((c >> 2) & 3);
}
// Orders the LDS accesses of one wave before and after this point (a
// compiler fence at wavefront scope; no instruction is emitted).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// ---------------------------------------------------------------------------
template <class G>
__device__ __forceinline__ void e1_write_a(float2* lds, const float2 (&v)[G::R], int n2, int x) {
  float2* p = lds + n2 * G::RS1 + x;
  sfor<G::R>([&](auto kc) { p[decltype(kc)::value * G::Y2 * G::RS1] = v[decltype(kc)::value]; });
}
template <class G>
__device__ __forceinline__ void e1_read_a(const float2* lds, float2 (&v)[G::R], int n2, int x) {
  const float2* p = lds + n2 * G::RS1 + x;
  sfor<G::R>([&](auto kc) { v[decltype(kc)::value] = p[decltype(kc)::value * G::Y2 * G::RS1]; });
}
template <class G>
__device__ __forceinline__ void e1_read_b(const float2* lds, float2 (&b)[G::R], int k1, int m2) {
  const float2* p = lds + k1 * G::Y2 * G::RS1 + m2;
  sfor<G::Y2>([&](auto nc) {
    sfor<G::X1>([&](auto mc) {
      constexpr int n2 = decltype(nc)::value, m1 = decltype(mc)::value;
      b[n2 * G::X1 + m1] = p[n2 * G::RS1 + m1 * G::X2];
    });
  });
}
template <class G>
__device__ __forceinline__ void e1_write_b(float2* lds, const float2 (&b)[G::R], int k1, int m2) {
  float2* p = lds + k1 * G::Y2 * G::RS1 + m2;
  sfor<G::Y2>([&](auto nc) {
    sfor<G::X1>([&](auto mc) {
      constexpr int n2 = decltype(nc)::value, m1 = decltype(mc)::value;
      p[n2 * G::RS1 + m1 * G::X2] = b[n2 * G::X1 + m1];
    });
  });
}
// layout B: ky = k1 + Y1*k2, so the row is Y2*k1 + k2
template <class G>
__device__ __forceinline__ void e2_write_b(float2* lds, const float2 (&b)[G::R], int k1, int m2) {
  static_assert(G::RS1 == G::RS2, "E1 and E2 share rows");
  float2* p = lds + k1 * G::Y2 * G::RS2;
  sfor<G::Y2>([&](auto kc) {
    sfor<G::X1>([&](auto jc) {
      constexpr int k2 = decltype(kc)::value, j1 = decltype(jc)::value;
      constexpr int jh = j1 / G::CJ;
      p[k2 * G::RS2 + j1 * G::X2 + (m2 ^ jh)] = b[k2 * G::X1 + j1];
    });
  });
}
template <class G>
__device__ __forceinline__ void e2_read_b(const float2* lds, float2 (&b)[G::R], int k1, int m2) {
  const float2* p = lds + k1 * G::Y2 * G::RS2;
  sfor<G::Y2>([&](auto kc) {
    sfor<G::X1>([&](auto jc) {
      constexpr int k2 = decltype(kc)::value, j1 = decltype(jc)::value;
      constexpr int jh = j1 / G::CJ;
      b[k2 * G::X1 + j1] = p[k2 * G::RS2 + j1 * G::X2 + (m2 ^ jh)];
    });
  });
}
// layout C: row Y2*(ky % Y1) + ky / Y1
template <class G>
__device__ __forceinline__ const float2* e2_row_c(const float2* lds, int ky, int jh) {
  return lds + (G::Y2 * (ky % G::Y1) + ky / G::Y1) * G::RS2 + jh * G::CJ * G::X2;
}
template <class G>
__device__ __forceinline__ void e2_read_c(const float2* lds, float2 (&c)[G::R], int ky, int jh) {
  const float2* p = e2_row_c<G>(lds, ky, jh);
  sfor<G::CJ>([&](auto lc) {
    sfor<G::X2>([&](auto mc) {
      constexpr int jl = decltype(lc)::value, m2 = decltype(mc)::value;
      c[jl * G::X2 + m2] = p[jl * G::X2 + (m2 ^ jh)];
    });
  });
}
template <class G>
__device__ __forceinline__ void e2_write_c(float2* lds, const float2 (&c)[G::R], int ky, int jh) {
  float2* p = const_cast<float2*>(e2_row_c<G>(lds, ky, jh));
  sfor<G::CJ>([&](auto lc) {
    sfor<G::X2>([&](auto mc) {
      constexpr int jl = decltype(lc)::value, m2 = decltype(mc)::value;
      p[jl * G::X2 + (m2 ^ jh)] = c[jl * G::X2 + m2];
    });
  });
}

}  // namespace ptycho
