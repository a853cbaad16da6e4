// Device-side FFT building blocks for gfx950: register DFT codelets and a
// Stockham (self-sorting) multi-stage FFT on lines held in LDS.
//
// A line of length N (N = 2^a 3^b) is transformed by radix stages taken
// greedily from {16, 8, 4, 3, 2}; each stage reads R values per butterfly
// from LDS, applies the inter-stage twiddle, runs an R-point DFT in
// registers and writes back in Stockham order, so the result is in natural
// order.  Twiddles come from a table W_N^j = exp(-2 pi i j / N) computed in
// FP64 on the host (and rounded once to the working precision); the inverse
// transform uses their conjugates.  No device transcendental is evaluated.
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

template <int R, int S, typename C> __device__ __forceinline__ void dft(C* v) {
  if constexpr (R == 2) {
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

// ------------------------------------------------------- radix schedule
constexpr int next_radix(int rem) {
  return (rem % 16 == 0) ? 16 : (rem % 8 == 0) ? 8 : (rem % 4 == 0) ? 4 : (rem % 3 == 0) ? 3 : (rem % 2 == 0) ? 2 : 1;
}
constexpr int radix_at(int n, int stage) {
  int rem = n;
  for (int s = 0; s < stage; ++s) rem /= next_radix(rem);
  return next_radix(rem);
}
constexpr bool fft_len_ok(int n) {
  int rem = n;
  while (rem > 1) {
    int r = next_radix(rem);
    if (r == 1) return false;
    rem /= r;
  }
  return n >= 2;
}
// threads per line: one radix-R0 butterfly each in the first stage
constexpr int fft_threads(int n) { return n / radix_at(n, 0); }
// radix of the stage that follows LS points already transformed
constexpr int radix_at_ls(int n, int ls) { return next_radix(n / ls); }

// LDS layout of a line: element i lives at px(i) = i + i/16, one pad slot
// per 16 elements, so the first stage's stride-16 writes fall on distinct
// banks.  Lines are line_pitch() apart: at least the padded span and
// congruent to the threads per line modulo 32, so that neighbouring lines
// of a wave do not alias onto the same banks.
__host__ __device__ constexpr int px(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int line_span(int n) { return n + (n >> 4); }
__host__ __device__ constexpr int line_pitch(int n, int t) {
  return line_span(n) + (((t - line_span(n)) % 32) + 32) % 32;
}

// One Stockham stage on a line in LDS (layout px), executed by T threads
// (index t) of the line; every thread of the work-group must call it (it
// contains barriers).  LS = product of the radices already applied.
template <int N, int S, int LS, int T, typename C>
__device__ __forceinline__ void stockham_stage(C* buf, int t, const C* __restrict__ tw) {
  constexpr int R = radix_at_ls(N, LS);
  constexpr int NB = N / R;                  // butterflies
  constexpr int IT = (NB + T - 1) / T;       // butterflies per thread
  C v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    int j = t + it * T;
    if (NB % T == 0 || j < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = buf[px(j + r * NB)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    int j = t + it * T;
    if (NB % T == 0 || j < NB) {
      int k = (LS == 1) ? 0 : (j % LS);
      if constexpr (LS > 1) {
        constexpr int STEP = N / (LS * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C w = tw[r * k * STEP];
          v[it][r] = (S < 0) ? cmul(v[it][r], w) : cmulc(v[it][r], w);
        }
      }
      dft<R, S>(v[it]);
      int base = (j / LS) * LS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[px(base + r * LS)] = v[it][r];
    }
  }
  __syncthreads();
}

// Full Stockham FFT (all stages) of one LDS line of length N.
template <int N, int S, int T, int LS = 1, typename C>
__device__ __forceinline__ void stockham(C* buf, int t, const C* __restrict__ tw) {
  if constexpr (LS < N) {
    stockham_stage<N, S, LS, T>(buf, t, tw);
    stockham<N, S, T, LS * radix_at_ls(N, LS)>(buf, t, tw);
  }
}

}  // namespace pb3
