// Device-side FFT building blocks for gfx950: register DFT codelets
// (2, 3, 4, 8, 16 by Cooley-Tukey with constant twiddles; 6, 12, 24 by the
// prime-factor mapping) and a two-phase line FFT of length N = R1 R2 with
// one LDS exchange.  Twiddles come from a table W_N^j = exp(-2 pi i j / N)
// computed in FP64 on the host (and rounded once to the working
// precision); the inverse transform uses their conjugates.  No device
// transcendental is evaluated.
#pragma once

#include <hip/hip_runtime.h>

namespace pb3 {

template <typename T> struct Cx;
template <> struct Cx<float> { using type = float2; };
template <> struct Cx<double> { using type = double2; };

template <typename C> __device__ __forceinline__ C cx(decltype(C::x) re, decltype(C::x) im) {
  C r;
  r.x = re;
  r.y = im;
  return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cx<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cx<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return cx<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  return cx<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return cx<C>(a.x, -a.y); }
// multiply by s*i, s = +1 or -1
template <int S, typename C> __device__ __forceinline__ C mul_si(C a) {
  return S > 0 ? cx<C>(-a.y, a.x) : cx<C>(a.y, -a.x);
}
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return cx<C>(a.x * s, a.y * s); }

// ---------------------------------------------------------------- codelets
// In-place R-point DFT of v[0..R): X_k = sum_n x_n exp(S * 2 pi i n k / R),
// S = -1 (forward) or +1 (inverse).

template <int S, typename C> __device__ __forceinline__ void dft2(C& a, C& b) {
  C t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int S, typename C> __device__ __forceinline__ void dft3(C* v) {
  using R = decltype(C::x);
  const R c = R(-0.5);
  const R s = R(S) * R(0.866025403784438646763723170752936183);
  C a = v[0], b = v[1], d = v[2];
  C t1 = cadd(b, d);
  C t2 = csub(b, d);
  C m = cx<C>(a.x + c * t1.x, a.y + c * t1.y);
  // s * i * t2
  C r = cx<C>(-s * t2.y, s * t2.x);
  v[0] = cadd(a, t1);
  v[1] = cadd(m, r);
  v[2] = csub(m, r);
}

template <int S, typename C> __device__ __forceinline__ void dft4(C& x0, C& x1, C& x2, C& x3) {
  C a = cadd(x0, x2), b = csub(x0, x2);
  C c = cadd(x1, x3), d = mul_si<S>(csub(x1, x3));
  x0 = cadd(a, c);
  x2 = csub(a, c);
  x1 = cadd(b, d);
  x3 = csub(b, d);
}

template <int S, typename C> __device__ __forceinline__ void dft8(C* v) {
  using R = decltype(C::x);
  const R h = R(0.707106781186547524400844362104849039);
  // even / odd 4-point DFTs
  dft4<S>(v[0], v[2], v[4], v[6]);
  dft4<S>(v[1], v[3], v[5], v[7]);
  // twiddles w^k, w = exp(S i pi / 4), applied to the odd outputs
  C o1 = v[3], o2 = v[5], o3 = v[7];
  // w^1 = h (1 + S i)
  o1 = cx<C>(h * (o1.x - R(S) * o1.y), h * (o1.y + R(S) * o1.x));
  // w^2 = S i
  o2 = mul_si<S>(o2);
  // w^3 = h (-1 + S i)
  o3 = cx<C>(h * (-o3.x - R(S) * o3.y), h * (-o3.y + R(S) * o3.x));
  C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1];
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

template <int S, typename C> __device__ __forceinline__ void dft16(C* v) {
  using R = decltype(C::x);
  const R c1 = R(0.923879532511286756128183189396788933);  // cos(pi/8)
  const R s1 = R(0.382683432365089771728459984030398866);  // sin(pi/8)
  const R h = R(0.707106781186547524400844362104849039);
  // n = 4 n1 + n2: 4-point DFTs over n1 for each n2
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<S>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
  // now v[4 k1 + n2] = Y_{n2}[k1]; twiddle by w16^(n2 k1), w16 = exp(S i pi/8)
  auto tw = [&](C a, R cr, R si) { return cx<C>(a.x * cr - R(S) * si * a.y, a.y * cr + R(S) * si * a.x); };
  // k1 = 1: n2 = 1,2,3 -> angles 1,2,3 (units pi/8)
  v[5] = tw(v[5], c1, s1);
  v[6] = tw(v[6], h, h);
  v[7] = tw(v[7], s1, c1);
  // k1 = 2: angles 2,4,6
  v[9] = tw(v[9], h, h);
  v[10] = mul_si<S>(v[10]);
  v[11] = tw(v[11], -h, h);
  // k1 = 3: angles 3,6,9
  v[13] = tw(v[13], s1, c1);
  v[14] = tw(v[14], -h, h);
  v[15] = tw(v[15], -c1, -s1);
  // 4-point DFTs over n2 for each k1; output index k1 + 4 k2
  C o[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    C a = v[4 * k1 + 0], b = v[4 * k1 + 1], c = v[4 * k1 + 2], d = v[4 * k1 + 3];
    dft4<S>(a, b, c, d);
    o[k1] = a;
    o[k1 + 4] = b;
    o[k1 + 8] = c;
    o[k1 + 12] = d;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = o[i];
}

template <int R, int S, typename C> __device__ __forceinline__ void dft(C* v);

// Good-Thomas prime-factor DFT of length N1*N2 (coprime): input n =
// (N2 n1 + N1 n2) mod N, output k with k = k1 (mod N1), k = k2 (mod N2);
// no twiddles between the two short DFTs.
constexpr int crt_index(int n1, int n2, int k1, int k2) {
  for (int k = 0; k < n1 * n2; ++k)
    if (k % n1 == k1 && k % n2 == k2) return k;
  return -1;
}
template <int N1, int N2, int S, typename C> __device__ __forceinline__ void dft_pfa(C* v) {
  constexpr int N = N1 * N2;
  C w[N];
#pragma unroll
  for (int n2 = 0; n2 < N2; ++n2) {
    C a[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) a[n1] = v[(N2 * n1 + N1 * n2) % N];
    dft<N1, S>(a);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) w[k1 * N2 + n2] = a[k1];
  }
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) {
    C b[N2];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) b[n2] = w[k1 * N2 + n2];
    dft<N2, S>(b);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) v[crt_index(N1, N2, k1, k2)] = b[k2];
  }
}

template <int R, int S, typename C> __device__ __forceinline__ void dft(C* v) {
  if constexpr (R == 1) {
  } else if constexpr (R == 6) {
    dft_pfa<2, 3, S>(v);
  } else if constexpr (R == 12) {
    dft_pfa<4, 3, S>(v);
  } else if constexpr (R == 24) {
    dft_pfa<8, 3, S>(v);
  } else if constexpr (R == 2) {
    dft2<S>(v[0], v[1]);
  } else if constexpr (R == 3) {
    dft3<S>(v);
  } else if constexpr (R == 4) {
    dft4<S>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    dft8<S>(v);
  } else if constexpr (R == 16) {
    dft16<S>(v);
  } else {
    static_assert(R == 2, "unsupported radix");
  }
}

// ------------------------------------------------- two-phase line FFT
// Length N = R1 * R2.  Phase 1: thread t < R2 of the line takes inputs
// n = t + R2 j (j < R1) in registers, runs a DFT of length R1 over j,
// multiplies output k1 by exp(S 2 pi i t k1 / N) and writes it to the
// line's LDS scratch s[k1 RS + t].  Phase 2: thread k1 < R1 reads
// s[k1 RS + t] (t < R2), runs a DFT of length R2 over t and delivers
// output k = k1 + R1 k2.  One LDS exchange, one barrier (every thread of
// the work-group must call it).  tw holds W_N^m = exp(-2 pi i m / N).
// The exchange rows sit RS = R2 + PAD apart and s holds R1 RS elements:
// where a line's threads are consecutive lanes, PAD = 1 puts phase 2's
// reads (stride RS) in distinct LDS banks, which rows of a power-of-two
// R2 would not.
constexpr int fft2_r1(int n) {
  return n == 16 ? 4 : n == 24 ? 8 : n == 32 ? 8 : n == 64 ? 8 : 16;
}
constexpr int fft2_r2(int n) { return n / fft2_r1(n); }
constexpr int fft2_threads(int n) { return fft2_r1(n) > fft2_r2(n) ? fft2_r1(n) : fft2_r2(n); }

// OVER: phase 2 reads its inputs, then a second work-group barrier lets
// store() write into s itself (the caller may alias its output with s).
// R1F, when set, replaces the default first radix fft2_r1(N) (R2 = N / R1F).
template <int N, int S, bool OVER = false, int PAD = 0, int R1F = 0, typename C, typename LoadF, typename StoreF>
__device__ __forceinline__ void fft2_line(C* s, int tl, const C* __restrict__ tw, LoadF&& load, StoreF&& store) {
  constexpr int R1 = R1F ? R1F : fft2_r1(N), R2 = N / R1, RS = R2 + PAD;
  static_assert(R1 * R2 == N, "bad factorisation");
  if (tl < R2) {
    C v[R1];
#pragma unroll
    for (int j = 0; j < R1; ++j) v[j] = load(tl + R2 * j);
    dft<R1, S>(v);
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) {
      C w = tw[tl * k1];
      v[k1] = (S < 0) ? cmul(v[k1], w) : cmulc(v[k1], w);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) s[k1 * RS + tl] = v[k1];
  }
  __syncthreads();
  C u[R2];
  if (tl < R1) {
#pragma unroll
    for (int t = 0; t < R2; ++t) u[t] = s[tl * RS + t];
  }
  if constexpr (OVER) __syncthreads();
  if (tl < R1) {
    dft<R2, S>(u);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) store(tl + R1 * k2, u[k2]);
  }
}

// Wave-synchronous variant for lines whose max(R1, R2) threads sit in one
// wavefront: the LDS exchange is ordered by a wavefront-scope fence instead
// of a work-group barrier, so other waves of the group never wait on it.
// load(j, n) gives input n = tl + R2 j of thread tl < R2; mid() runs on
// every thread once phase 1 has taken its inputs (a caller can issue the
// next line's loads there).  Phase 2 hands thread k1 its whole row u[k2]
// (output index k1 + R1 k2).  The exchange rows are R2 + 1 apart so that
// phase 2's strided reads fall in distinct LDS banks; s holds R1 (R2 + 1)
// elements.  R1F, when set, replaces the default first radix fft2_r1(N)
// (R2 = N / R1F); the caller's slot of lanes must hold max(R1, R2) of them
// inside one wavefront.
template <int N, int S, int R1F = 0, typename C, typename LoadF, typename MidF, typename RowF>
__device__ __forceinline__ void fft2_line_wave(C* s, int tl, const C* __restrict__ tw, LoadF&& load, MidF&& mid,
                                               RowF&& row) {
  constexpr int R1 = R1F ? R1F : fft2_r1(N), R2 = N / R1, RP = R2 + 1;
  static_assert(R1 * R2 == N && R1 <= 64 && R2 <= 64, "line must fit in one wavefront");
  C v[R1];
  if (tl < R2) {
#pragma unroll
    for (int j = 0; j < R1; ++j) v[j] = load(j, tl + R2 * j);
  }
  mid();
  if (tl < R2) {
    dft<R1, S>(v);
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) {
      C w = tw[tl * k1];
      v[k1] = (S < 0) ? cmul(v[k1], w) : cmulc(v[k1], w);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) s[k1 * RP + tl] = v[k1];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (tl < R1) {
    C u[R2];
#pragma unroll
    for (int t = 0; t < R2; ++t) u[t] = s[tl * RP + t];
    dft<R2, S>(u);
    row(tl, u);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace pb3
