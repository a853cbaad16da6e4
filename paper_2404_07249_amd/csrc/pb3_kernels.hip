// HIP kernels (gfx950) for the idealized binned power spectrum and
// bispectrum: pruned forward r2c FFT, shell-binned power, per-bin shell
// filter + pruned inverse c2r FFT, triplet contraction and the fixed-order
// reduction.  Launch wrappers at the bottom are called by pb3_host.cpp.
//
// Data layout in HBM (all C order, last index fastest):
//   delta  float  [N][N][N]
//   f1     float2 [N][N][Kz]         after the z pass (kz in [0, Kz))
//   f2     float2 [N][Lc][Kz]        after the y pass (ky centred-compact)
//   dc     float2 [Lc][Lc][Kz]       compact spectrum D(n), |n_i| <= K
//   a1_b   float2 [M][ly_b][kzn_b]   bin b after the inverse x pass
//   a2_b   float2 [M][M][kzn_b]      bin b after the inverse y pass
//   g      float  [nb_pad][M][M][M]  filtered fields G_b on the contraction grid
// A centred-compact index c holds frequency f = c - Kc.

#include <hip/hip_runtime.h>

#include "fft_dev.h"
#include "pb3_internal.h"

namespace pb3 {

constexpr int kLdsBudget = 48 * 1024;

__host__ __device__ constexpr int lines_per_wg(int t, int lp_bytes) {
  int tb = 256 / t;
  if (tb < 1) tb = 1;
  while (tb > 1 && tb * lp_bytes > kLdsBudget) --tb;
  return tb;
}

// Work-group shapes, shared by the kernels and their launchers.
// z passes: TB contiguous lines of T threads each.
template <int N> struct FwdZGeom {
  static constexpr int H = N / 2;
  static constexpr int T = fft_threads(H);
  static constexpr int LP = line_pitch(H, T);
  static constexpr int TB = lines_per_wg(T, LP * 8);
};
// strided passes: TB columns (consecutive inner indices) of T threads; CS =
// bytes per complex element
template <int N, int CS> struct ColGeom {
  static constexpr int T = fft_threads(N);
  static constexpr int LP = line_pitch(N, T);
  static constexpr int TB0 = 256 / T < 16 ? 16 : 256 / T;
  static constexpr int TB = (TB0 * LP * CS > 64 * 1024) ? (64 * 1024) / (LP * CS) : TB0;
};
template <int M, int CS> struct InvZGeom {
  static constexpr int H = M / 2;
  static constexpr int T = fft_threads(H);
  static constexpr int LX = H + 2;  // X_0..X_{M/2} plus pad
  static constexpr int LZ = line_pitch(H, T);
  static constexpr int TB = lines_per_wg(T, (LX + LZ) * CS);
};

// ------------------------------------------------------------ forward z
// r2c along z of N^2 contiguous lines, keeping kz in [0, Kz).  A real line
// of length N is transformed as a complex line of length N/2
// (z_n = x_{2n} + i x_{2n+1}) and untangled:
//   X_k = E_k + W_N^k O_k,  E_k = (Z_k + conj Z_{N/2-k})/2,
//   O_k = -i (Z_k - conj Z_{N/2-k})/2.
template <int N>
__global__ void __launch_bounds__(512) k_fwd_z(const float* __restrict__ delta, float2* __restrict__ f1, int n_lines,
                                               int Kz, const float2* __restrict__ tw_h, const float2* __restrict__ tw_n) {
  using Gm = FwdZGeom<N>;
  constexpr int H = Gm::H, T = Gm::T, LP = Gm::LP, TB = Gm::TB;
  __shared__ float2 buf[TB * LP];
  __shared__ float2 twh[H];
  __shared__ float2 twn[N];
  const int tid = threadIdx.x;
  const int l0 = blockIdx.x * TB;
  const float2* in2 = reinterpret_cast<const float2*>(delta);
  for (int e = tid; e < H; e += TB * T) twh[e] = tw_h[e];
  for (int e = tid; e < N; e += TB * T) twn[e] = tw_n[e];
  for (int e = tid; e < TB * H; e += TB * T) {
    int line = e / H, p = e % H;
    float2 v = make_float2(0.f, 0.f);
    if (l0 + line < n_lines) v = in2[(size_t)(l0 + line) * H + p];
    buf[line * LP + px(p)] = v;
  }
  __syncthreads();
  const int line = tid / T, t = tid % T;
  stockham<H, -1, T>(buf + line * LP, t, twh);
  if (l0 + line < n_lines) {
    const float2* z = buf + line * LP;
    for (int k = t; k < Kz; k += T) {
      float2 zk = z[px(k % H)];
      float2 zc = z[px((H - k) % H)];
      zc.y = -zc.y;  // conj Z_{N/2-k}
      float2 e = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
      float2 d = make_float2(zk.x - zc.x, zk.y - zc.y);
      float2 o = make_float2(0.5f * d.y, -0.5f * d.x);  // -i d / 2
      float2 w = twn[k % N];
      float2 x = make_float2(e.x + w.x * o.x - w.y * o.y, e.y + w.x * o.y + w.y * o.x);
      f1[(size_t)(l0 + line) * Kz + k] = x;
    }
  }
}

// --------------------------------------------------- forward strided c2c
// Forward FFT along a strided axis of length N, output kept in
// centred-compact order: out index c <- frequency c - Ko.
template <int N>
__global__ void __launch_bounds__(512) k_fwd_col(const float2* __restrict__ in, float2* __restrict__ out, int n_inner,
                                                 long in_outer, long out_outer, int Lo, int Ko,
                                                 const float2* __restrict__ tw) {
  using Gm = ColGeom<N, 8>;
  constexpr int T = Gm::T, LP = Gm::LP, TB = Gm::TB;
  __shared__ float2 buf[TB * LP];
  __shared__ float2 tws[N];
  const int tid = threadIdx.x;
  const int nth = TB * T;
  const int i0 = blockIdx.x * TB;
  for (int e = tid; e < N; e += nth) tws[e] = tw[e];
  const float2* src = in + (size_t)blockIdx.y * in_outer;
  for (int e = tid; e < N * TB; e += nth) {
    int p = e / TB, col = e % TB;
    float2 v = make_float2(0.f, 0.f);
    if (i0 + col < n_inner) v = src[(size_t)p * n_inner + i0 + col];
    buf[col * LP + px(p)] = v;
  }
  __syncthreads();
  stockham<N, -1, T>(buf + (tid / T) * LP, tid % T, tws);
  float2* dst = out + (size_t)blockIdx.y * out_outer;
  for (int e = tid; e < Lo * TB; e += nth) {
    int c = e / TB, col = e % TB;
    if (i0 + col < n_inner) {
      int f = c - Ko;
      int p = f < 0 ? f + N : f;
      dst[(size_t)c * n_inner + i0 + col] = buf[col * LP + px(p)];
    }
  }
}

// ------------------------------------------------------------------ power
// Each work-group sums w |D|^2 over one chunk of one bin's mode list in
// FP64 (w = 2 for modes whose conjugate partner is not stored, bit 31 of
// the index marks w = 1), then reduces with a fixed tree.
__global__ void __launch_bounds__(256) k_power_chunks(const float2* __restrict__ dc, const int32_t* __restrict__ modes,
                                                      const int32_t* __restrict__ chunks, double* __restrict__ part) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  const int start = chunks[3 * c + 1], end = chunks[3 * c + 2];
  double acc = 0.0;
  for (int i = start + threadIdx.x; i < end; i += 256) {
    int32_t m = modes[i];
    double w = (m < 0) ? 1.0 : 2.0;
    float2 v = dc[m & 0x7fffffff];
    double re = v.x, im = v.y;
    acc += w * (re * re + im * im);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[c] = red[0];
}

__global__ void k_power_final(const double* __restrict__ part, const int32_t* __restrict__ chunks, int n_chunks, int nb,
                              const double* __restrict__ scale, double* __restrict__ pk) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  double s = 0.0;
  for (int c = 0; c < n_chunks; ++c)
    if (chunks[3 * c] == b) s += part[c];
  pk[b] = s * scale[b];
}

// ---------------------------------------------------------- inverse x
// Per bin b: columns (ky, kz) of the bin's rectangle; gather the kx line of
// Theta_b D (or Theta_b alone when UNIT) into an M-point line and inverse
// transform it.  Output a1_b[x][jy][jz].
template <int M, typename Rl, bool UNIT>
__global__ void __launch_bounds__(512) k_inv_x(const float2* __restrict__ dc, typename Cx<Rl>::type* __restrict__ a1,
                                               const BinGeom* __restrict__ geom, const BinTile* __restrict__ tiles,
                                               const int8_t* __restrict__ lut, int Kc, int Lc, int Kz,
                                               const typename Cx<Rl>::type* __restrict__ tw) {
  using C = typename Cx<Rl>::type;
  using Gm = ColGeom<M, (int)sizeof(C)>;
  constexpr int T = Gm::T, LP = Gm::LP, TB = Gm::TB;
  __shared__ C buf[TB * LP];
  __shared__ C tws[M];
  const int tid = threadIdx.x;
  const int nth = TB * T;
  for (int e = tid; e < M; e += nth) tws[e] = tw[e];
  const BinTile tile = tiles[blockIdx.x];
  const int b = tile.bin;
  const BinGeom g = geom[b];
  const int ncol = g.ly * g.kzn;
  for (int e = tid; e < M * TB; e += nth) {
    int p = e / TB, col = e % TB;
    int q = tile.col0 + col;
    C v = cx<C>(Rl(0), Rl(0));
    int kx = p <= g.kpos ? p : (p >= M - g.kneg ? p - M : 0x40000000);
    if (q < ncol && kx != 0x40000000) {
      int ky = q / g.kzn - g.kneg;
      int kz = q % g.kzn;
      int n2 = kx * kx + ky * ky + kz * kz;
      if (lut[n2] == b) {
        if constexpr (UNIT) {
          v = cx<C>(Rl(1), Rl(0));
        } else {
          float2 d = dc[((size_t)(kx + Kc) * Lc + (ky + Kc)) * Kz + kz];
          v = cx<C>(Rl(d.x), Rl(d.y));
        }
      }
    }
    buf[col * LP + px(p)] = v;
  }
  __syncthreads();
  stockham<M, 1, T>(buf + (tid / T) * LP, tid % T, tws);
  C* dst = a1 + g.a1_off;
  for (int e = tid; e < M * TB; e += nth) {
    int x = e / TB, col = e % TB;
    int q = tile.col0 + col;
    if (q < ncol) dst[(size_t)x * ncol + q] = buf[col * LP + px(x)];
  }
}

// ---------------------------------------------------------- inverse y
// Per bin: columns (x, kz); inverse transform along y.  a2_b[x][y][jz].
template <int M, typename Rl>
__global__ void __launch_bounds__(512) k_inv_y(const typename Cx<Rl>::type* __restrict__ a1,
                                               typename Cx<Rl>::type* __restrict__ a2,
                                               const BinGeom* __restrict__ geom, const BinTile* __restrict__ tiles,
                                               const typename Cx<Rl>::type* __restrict__ tw) {
  using C = typename Cx<Rl>::type;
  using Gm = ColGeom<M, (int)sizeof(C)>;
  constexpr int T = Gm::T, LP = Gm::LP, TB = Gm::TB;
  __shared__ C buf[TB * LP];
  __shared__ C tws[M];
  const int tid = threadIdx.x;
  const int nth = TB * T;
  for (int e = tid; e < M; e += nth) tws[e] = tw[e];
  const BinTile tile = tiles[blockIdx.x];
  const BinGeom g = geom[tile.bin];
  const int ncol = M * g.kzn;
  const C* src = a1 + g.a1_off;
  for (int e = tid; e < M * TB; e += nth) {
    int p = e / TB, col = e % TB;
    int q = tile.col0 + col;
    C v = cx<C>(Rl(0), Rl(0));
    int ky = p <= g.kpos ? p : (p >= M - g.kneg ? p - M : 0x40000000);
    if (q < ncol && ky != 0x40000000) {
      int x = q / g.kzn, jz = q % g.kzn;
      v = src[((size_t)x * g.ly + (ky + g.kneg)) * g.kzn + jz];
    }
    buf[col * LP + px(p)] = v;
  }
  __syncthreads();
  stockham<M, 1, T>(buf + (tid / T) * LP, tid % T, tws);
  C* dst = a2 + g.a2_off;
  for (int e = tid; e < M * TB; e += nth) {
    int y = e / TB, col = e % TB;
    int q = tile.col0 + col;
    if (q < ncol) {
      int x = q / g.kzn, jz = q % g.kzn;
      dst[((size_t)x * M + y) * g.kzn + jz] = buf[col * LP + px(y)];
    }
  }
}

// ---------------------------------------------------------- inverse z
// Per bin: lines (x, y) hold kz in [0, kzn); c2r to M reals through an
// M/2-point complex inverse FFT:
//   Z_k = (X_k + conj X_{M/2-k}) + i (X_k - conj X_{M/2-k}) conj(W_M^k),
//   z = IDFT_{M/2}(Z),  g_{2n} = Re z_n,  g_{2n+1} = Im z_n,
// scaled by 1/M^3 (numpy's inverse normalisation on the M^3 grid).
template <int M, typename Rl>
__global__ void __launch_bounds__(512) k_inv_z(const typename Cx<Rl>::type* __restrict__ a2, Rl* __restrict__ gout,
                                               const BinGeom* __restrict__ geom, const BinTile* __restrict__ tiles,
                                               const typename Cx<Rl>::type* __restrict__ tw_h,
                                               const typename Cx<Rl>::type* __restrict__ tw_m, Rl scale) {
  using C = typename Cx<Rl>::type;
  using Gm = InvZGeom<M, (int)sizeof(C)>;
  constexpr int H = Gm::H, T = Gm::T, LX = Gm::LX, LZ = Gm::LZ, TB = Gm::TB;
  __shared__ C xb[TB * LX];
  __shared__ C zb[TB * LZ];
  __shared__ C twh[H];
  __shared__ C twm[M];
  const int tid = threadIdx.x;
  const int nth = TB * T;
  for (int e = tid; e < H; e += nth) twh[e] = tw_h[e];
  for (int e = tid; e < M; e += nth) twm[e] = tw_m[e];
  const BinTile tile = tiles[blockIdx.x];
  const BinGeom g = geom[tile.bin];
  const int nlines = M * M;
  const C* src = a2 + g.a2_off;
  for (int e = tid; e < TB * (H + 1); e += nth) {
    int line = e / (H + 1), k = e % (H + 1);
    int l = tile.col0 + line;
    C v = cx<C>(Rl(0), Rl(0));
    if (l < nlines && k < g.kzn) v = src[(size_t)l * g.kzn + k];
    xb[line * LX + k] = v;
  }
  __syncthreads();
  for (int e = tid; e < TB * H; e += nth) {
    int line = e / H, k = e % H;
    const C* X = xb + line * LX;
    C a = X[k];
    C b = X[H - k];
    b.y = -b.y;  // conj X_{M/2-k}
    C s = cadd(a, b);
    C d = csub(a, b);
    C w = twm[k];  // W_M^k; multiply by its conjugate
    C dw = cmulc(d, w);
    // Z = s + i dw
    zb[line * LZ + px(k)] = cx<C>(s.x - dw.y, s.y + dw.x);
  }
  __syncthreads();
  stockham<H, 1, T>(zb + (tid / T) * LZ, tid % T, twh);
  Rl* dst = gout + (size_t)tile.bin * ((size_t)M * M * M);
  for (int e = tid; e < TB * H; e += nth) {
    int line = e / H, n = e % H;
    int l = tile.col0 + line;
    if (l < nlines) {
      C z = zb[line * LZ + px(n)];
      typename Cx<Rl>::type o = cx<C>(z.x * scale, z.y * scale);
      reinterpret_cast<typename Cx<Rl>::type*>(dst + (size_t)l * M)[n] = o;
    }
  }
}

// ------------------------------------------------ simple triplet contraction
// Reference-structure contraction: every work-group takes a contiguous
// voxel range, stages VT voxels of all bins in LDS and each thread
// accumulates up to TPT triplets sum_x G_a G_b G_c.  Each VT-voxel tile is
// summed in the working precision and flushed into an FP64 running sum, so
// the rounding error does not grow with the number of voxels per thread.
// partial[wg][t] (FP64) for every candidate triplet t.
template <typename Rl, int TPT>
__global__ void __launch_bounds__(256) k_contract_simple(const Rl* __restrict__ g, int nb, long mvox,
                                                         const int32_t* __restrict__ trips, int n_trip,
                                                         long vox_per_wg, double* __restrict__ part) {
  constexpr int VT = 64;
  extern __shared__ unsigned char smem_raw[];
  Rl* tileg = reinterpret_cast<Rl*>(smem_raw);  // [nb][VT]
  const int tid = threadIdx.x;
  double acc[TPT];
  int ta[TPT], tbb[TPT], tc[TPT];
#pragma unroll
  for (int i = 0; i < TPT; ++i) {
    acc[i] = 0.0;
    int t = tid + i * 256;
    if (t < n_trip) {
      ta[i] = trips[3 * t];
      tbb[i] = trips[3 * t + 1];
      tc[i] = trips[3 * t + 2];
    } else {
      ta[i] = tbb[i] = tc[i] = -1;
    }
  }
  const long v_begin = (long)blockIdx.x * vox_per_wg;
  long v_end = v_begin + vox_per_wg;
  if (v_end > mvox) v_end = mvox;
  for (long v0 = v_begin; v0 < v_end; v0 += VT) {
    __syncthreads();
    for (int e = tid; e < nb * VT; e += 256) {
      int b = e / VT, j = e % VT;
      long v = v0 + j;
      tileg[e] = (v < v_end) ? g[(size_t)b * mvox + v] : Rl(0);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
      if (ta[i] >= 0) {
        const Rl* pa = tileg + ta[i] * VT;
        const Rl* pb = tileg + tbb[i] * VT;
        const Rl* pc = tileg + tc[i] * VT;
        Rl s = Rl(0);
        for (int j = 0; j < VT; ++j) s += pa[j] * pb[j] * pc[j];
        acc[i] += (double)s;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < TPT; ++i) {
    int t = tid + i * 256;
    if (t < n_trip) part[(size_t)blockIdx.x * n_trip + t] = acc[i];
  }
}

// ------------------------------------------------------------- reduction
// Fixed-order FP64 sum of the per-work-group partials for every kept
// triplet, times scale/T (scale = V^2 M^6 / N^9).
template <typename Rl>
__global__ void k_reduce(const Rl* __restrict__ part, int n_wg, int part_len, const int32_t* __restrict__ map,
                         const double* __restrict__ fac, int n_out, double* __restrict__ out) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_out) return;
  int idx = map[t];
  double s = 0.0;
  for (int w = 0; w < n_wg; ++w) s += (double)part[(size_t)w * part_len + idx];
  out[t] = fac ? s * fac[t] : s;
}

// Two-stage form for the MFMA partials: slice s of the work-groups is
// summed per element (FP64), then the slices per kept triplet.
__global__ void k_reduce_slices(const float* __restrict__ part, int n_wg, int part_len, double* __restrict__ rsl) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= part_len) return;
  int s = blockIdx.y;
  int w0 = (int)((long)n_wg * s / kReduceSlices), w1 = (int)((long)n_wg * (s + 1) / kReduceSlices);
  double acc = 0.0;
  for (int w = w0; w < w1; ++w) acc += (double)part[(size_t)w * part_len + e];
  rsl[(size_t)s * part_len + e] = acc;
}

__global__ void k_reduce_final(const double* __restrict__ rsl, int part_len, const int32_t* __restrict__ map,
                               const double* __restrict__ fac, int n_out, double* __restrict__ out) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_out) return;
  int idx = map[t];
  double acc = 0.0;
#pragma unroll
  for (int s = 0; s < kReduceSlices; ++s) acc += rsl[(size_t)s * part_len + idx];
  out[t] = acc * fac[t];
}

// ================================================================ launchers

#define PB3_DISPATCH_LEN(len, FN, ...)           \
  switch (len) {                                 \
    case 8: return FN<8>(__VA_ARGS__);           \
    case 12: return FN<12>(__VA_ARGS__);         \
    case 16: return FN<16>(__VA_ARGS__);         \
    case 24: return FN<24>(__VA_ARGS__);         \
    case 32: return FN<32>(__VA_ARGS__);         \
    case 48: return FN<48>(__VA_ARGS__);         \
    case 64: return FN<64>(__VA_ARGS__);         \
    case 96: return FN<96>(__VA_ARGS__);         \
    case 128: return FN<128>(__VA_ARGS__);       \
    case 192: return FN<192>(__VA_ARGS__);       \
    case 256: return FN<256>(__VA_ARGS__);       \
    case 384: return FN<384>(__VA_ARGS__);       \
    default: return hipErrorInvalidValue;        \
  }

template <int N>
static hipError_t fwd_z_impl(const pb3_plan& p, const float* delta, hipStream_t s) {
  if constexpr (N < 16) {
    return hipErrorInvalidValue;
  } else {
    constexpr int T = FwdZGeom<N>::T, TB = FwdZGeom<N>::TB;
    int n_lines = N * N;
    dim3 grid((n_lines + TB - 1) / TB);
    hipLaunchKernelGGL(k_fwd_z<N>, grid, dim3(TB * T), 0, s, delta, p.ws.f1, n_lines, p.Kz, p.d.tw_n2, p.d.tw_n);
    return hipGetLastError();
  }
}
hipError_t launch_fwd_z(const pb3_plan& p, const float* delta, hipStream_t s) {
  PB3_DISPATCH_LEN(p.N, fwd_z_impl, p, delta, s);
}

template <int N>
static hipError_t fwd_col_impl(const float2* in, float2* out, int n_inner, long in_outer, long out_outer, int n_outer,
                               int Lo, int Ko, const float2* tw, hipStream_t s) {
  constexpr int T = ColGeom<N, 8>::T, TB = ColGeom<N, 8>::TB;
  dim3 grid((n_inner + TB - 1) / TB, n_outer);
  hipLaunchKernelGGL(k_fwd_col<N>, grid, dim3(TB * T), 0, s, in, out, n_inner, in_outer, out_outer, Lo, Ko, tw);
  return hipGetLastError();
}
hipError_t launch_fwd_y(const pb3_plan& p, hipStream_t s) {
  // f1[x][y][kz] -> f2[x][kyc][kz]
  PB3_DISPATCH_LEN(p.N, fwd_col_impl, p.ws.f1, p.ws.f2, p.Kz, (long)p.N * p.Kz, (long)p.Lc * p.Kz, p.N, p.Lc, p.Kc,
                   p.d.tw_n, s);
}
hipError_t launch_fwd_x(const pb3_plan& p, hipStream_t s) {
  // f2[x][kyc][kz] -> dc[kxc][kyc][kz]
  PB3_DISPATCH_LEN(p.N, fwd_col_impl, p.ws.f2, p.ws.dc, p.Lc * p.Kz, 0L, 0L, 1, p.Lc, p.Kc, p.d.tw_n, s);
}

hipError_t launch_power(const pb3_plan& p, double* pk, hipStream_t s) {
  hipLaunchKernelGGL(k_power_chunks, dim3(p.n_chunks), dim3(256), 0, s, p.ws.dc, p.d.modes, p.d.chunk, p.ws.ppart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_power_final, dim3((p.nb + 63) / 64), dim3(64), 0, s, p.ws.ppart, p.d.chunk, p.n_chunks, p.nb,
                     p.d.pk_scale, pk);
  return hipGetLastError();
}

template <int M, typename Rl, bool UNIT>
static hipError_t inv_x_impl2(const pb3_plan& p, typename Cx<Rl>::type* a1, const typename Cx<Rl>::type* tw,
                              const TileSet& ts, hipStream_t s) {
  using Gm = ColGeom<M, (int)sizeof(typename Cx<Rl>::type)>;
  constexpr int T = Gm::T, TB = Gm::TB;
  if (TB != ts.tb) return hipErrorInvalidConfiguration;
  if (ts.n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_inv_x<M, Rl, UNIT>), dim3(ts.n), dim3(TB * T), 0, s, p.ws.dc, a1, p.d.geom, ts.d, p.d.lut,
                     p.Kc, p.Lc, p.Kz, tw);
  return hipGetLastError();
}

template <int M, typename Rl>
static hipError_t inv_y_impl2(const pb3_plan& p, const typename Cx<Rl>::type* a1, typename Cx<Rl>::type* a2,
                              const typename Cx<Rl>::type* tw, const TileSet& ts, hipStream_t s) {
  using Gm = ColGeom<M, (int)sizeof(typename Cx<Rl>::type)>;
  constexpr int T = Gm::T, TB = Gm::TB;
  if (TB != ts.tb) return hipErrorInvalidConfiguration;
  if (ts.n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_inv_y<M, Rl>), dim3(ts.n), dim3(TB * T), 0, s, a1, a2, p.d.geom, ts.d, tw);
  return hipGetLastError();
}

template <int M, typename Rl>
static hipError_t inv_z_impl2(const pb3_plan& p, const typename Cx<Rl>::type* a2, Rl* gout,
                              const typename Cx<Rl>::type* tw_h, const typename Cx<Rl>::type* tw_m, const TileSet& ts,
                              hipStream_t s) {
  if constexpr (M < 16) {
    return hipErrorInvalidValue;
  } else {
    using Gm = InvZGeom<M, (int)sizeof(typename Cx<Rl>::type)>;
    constexpr int T = Gm::T, TB = Gm::TB;
    if (TB != ts.tb) return hipErrorInvalidConfiguration;
    if (ts.n == 0) return hipSuccess;
    Rl scale = Rl(1.0 / ((double)M * M * M));
    hipLaunchKernelGGL((k_inv_z<M, Rl>), dim3(ts.n), dim3(TB * T), 0, s, a2, gout, p.d.geom, ts.d, tw_h, tw_m, scale);
    return hipGetLastError();
  }
}

// tile widths the host needs to build the tile tables (same formulas)
template <int M> static int tb_x_of(bool dbl) { return dbl ? ColGeom<M, 16>::TB : ColGeom<M, 8>::TB; }
template <int M> static int tb_z_of(bool dbl) {
  if constexpr (M < 16) {
    return 0;
  } else {
    return dbl ? InvZGeom<M, 16>::TB : InvZGeom<M, 8>::TB;
  }
}

#define PB3_DISPATCH_M(len, EXPR_T)             \
  switch (len) {                                \
    case 16: { constexpr int MM = 16; EXPR_T; } \
    case 24: { constexpr int MM = 24; EXPR_T; } \
    case 32: { constexpr int MM = 32; EXPR_T; } \
    case 48: { constexpr int MM = 48; EXPR_T; } \
    case 64: { constexpr int MM = 64; EXPR_T; } \
    case 96: { constexpr int MM = 96; EXPR_T; } \
    case 128: { constexpr int MM = 128; EXPR_T; } \
    case 192: { constexpr int MM = 192; EXPR_T; } \
    case 256: { constexpr int MM = 256; EXPR_T; } \
    case 384: { constexpr int MM = 384; EXPR_T; } \
    default: break;                             \
  }

int tile_width_x(int M, bool dbl) {
  PB3_DISPATCH_M(M, return tb_x_of<MM>(dbl));
  return 0;
}
int tile_width_z(int M, bool dbl) {
  PB3_DISPATCH_M(M, return tb_z_of<MM>(dbl));
  return 0;
}

hipError_t launch_inv_x(const pb3_plan& p, hipStream_t s) {
  PB3_DISPATCH_M(p.M, return (inv_x_impl2<MM, float, false>(p, p.ws.a1, p.d.tw_m, p.tx, s)));
  return hipErrorInvalidValue;
}
hipError_t launch_inv_y(const pb3_plan& p, hipStream_t s) {
  PB3_DISPATCH_M(p.M, return (inv_y_impl2<MM, float>(p, p.ws.a1, p.ws.a2, p.d.tw_m, p.ty, s)));
  return hipErrorInvalidValue;
}
hipError_t launch_inv_z(const pb3_plan& p, hipStream_t s) {
  PB3_DISPATCH_M(p.M, return (inv_z_impl2<MM, float>(p, p.ws.a2, p.ws.g, p.d.tw_m2, p.d.tw_m, p.tz, s)));
  return hipErrorInvalidValue;
}

static int tpt_for(int n) {
  int per = (n + 255) / 256;
  if (per <= 4) return 4;
  if (per <= 8) return 8;
  if (per <= 16) return 16;
  if (per <= 32) return 32;
  return -1;
}

template <typename Rl>
static hipError_t contract_simple(const Rl* g, int nb, long mvox, const int32_t* trips, int n_trip, int n_wg,
                                  double* part, hipStream_t s) {
  long per = (mvox + n_wg - 1) / n_wg;
  size_t sh = (size_t)nb * 64 * sizeof(Rl);
  switch (tpt_for(n_trip)) {
    case 4:
      hipLaunchKernelGGL((k_contract_simple<Rl, 4>), dim3(n_wg), dim3(256), sh, s, g, nb, mvox, trips, n_trip, per, part);
      break;
    case 8:
      hipLaunchKernelGGL((k_contract_simple<Rl, 8>), dim3(n_wg), dim3(256), sh, s, g, nb, mvox, trips, n_trip, per, part);
      break;
    case 16:
      hipLaunchKernelGGL((k_contract_simple<Rl, 16>), dim3(n_wg), dim3(256), sh, s, g, nb, mvox, trips, n_trip, per,
                         part);
      break;
    case 32:
      hipLaunchKernelGGL((k_contract_simple<Rl, 32>), dim3(n_wg), dim3(256), sh, s, g, nb, mvox, trips, n_trip, per,
                         part);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_contract(const pb3_plan& p, pb3_precision prec, hipStream_t s) {
  return launch_contract_mfma(p, prec == PB3_MIXED_BF16X3, s);
}

hipError_t launch_reduce(const pb3_plan& p, pb3_precision prec, double* bk, hipStream_t s) {
  (void)prec;
  int n_out = (int)(p.trip.size() / 3);
  if (n_out == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_slices, dim3((p.part_len + 255) / 256, kReduceSlices), dim3(256), 0, s, p.ws.part,
                     p.contract_wgs, p.part_len, p.ws.rsl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3((n_out + 255) / 256), dim3(256), 0, s, p.ws.rsl, p.part_len, p.d.out_map,
                     p.d.inv_counts, n_out, bk);
  return hipGetLastError();
}

// -------------------------------------------------------- FP64 counts
// T_abc = M^6 sum_x H_a H_b H_c on the contraction grid, H_b = IDFT[Theta_b],
// all in FP64 (N_0 of eq. N-ell-def with P_fid = 1), once per plan.
pb3_status compute_counts_fp64(pb3_plan& p, std::vector<double>& counts_out) {
  const int n_cand = (int)(p.trip_all.size() / 3);
  counts_out.assign(n_cand, 0.0);
  if (n_cand == 0) return PB3_OK;
  const long mvox = (long)p.M * p.M * p.M;
  const int nwg = 512;
  double2 *a1 = nullptr, *a2 = nullptr;
  double *h = nullptr, *part = nullptr, *out = nullptr;
  int32_t* map = nullptr;
  BinTile* tiles = nullptr;
  TileSet tsx{}, tsy{}, tsz{};
  hipError_t e;
  pb3_status st = PB3_OK;
  auto alloc = [&](void** ptr, size_t bytes) {
    e = hipMalloc(ptr, bytes);
    return e == hipSuccess;
  };
  std::vector<int32_t> idmap(n_cand);
  for (int i = 0; i < n_cand; ++i) idmap[i] = i;
  if (!alloc((void**)&a1, sizeof(double2) * p.a1_len) || !alloc((void**)&a2, sizeof(double2) * p.a2_len) ||
      !alloc((void**)&h, sizeof(double) * (size_t)p.nb * mvox) ||
      !alloc((void**)&part, sizeof(double) * (size_t)nwg * n_cand) || !alloc((void**)&out, sizeof(double) * n_cand) ||
      !alloc((void**)&map, sizeof(int32_t) * n_cand)) {
    st = PB3_ENOMEM;
    set_error("device allocation failed while computing triangle counts");
    goto done;
  }
  e = hipMemset(h, 0, sizeof(double) * (size_t)p.nb * mvox);
  if (e != hipSuccess) { st = hip_fail(e, "hipMemset"); goto done; }
  e = hipMemcpy(map, idmap.data(), sizeof(int32_t) * n_cand, hipMemcpyHostToDevice);
  if (e != hipSuccess) { st = hip_fail(e, "hipMemcpy"); goto done; }
  {
    // FP64 lines take twice the LDS: the count pass has its own tile tables
    int tbx = tile_width_x(p.M, true), tbz = tile_width_z(p.M, true);
    std::vector<BinTile> vx, vy, vz;
    build_tiles(p, tbx, tbx, tbz, vx, vy, vz);
    size_t nt = vx.size() + vy.size() + vz.size();
    if (!alloc((void**)&tiles, sizeof(BinTile) * (nt ? nt : 1))) {
      st = PB3_ENOMEM;
      set_error("device allocation failed while computing triangle counts");
      goto done;
    }
    std::vector<BinTile> all(vx);
    all.insert(all.end(), vy.begin(), vy.end());
    all.insert(all.end(), vz.begin(), vz.end());
    e = hipMemcpy(tiles, all.data(), sizeof(BinTile) * nt, hipMemcpyHostToDevice);
    if (e != hipSuccess) { st = hip_fail(e, "hipMemcpy"); goto done; }
    tsx = TileSet{tiles, (int)vx.size(), tbx};
    tsy = TileSet{tiles + vx.size(), (int)vy.size(), tbx};
    tsz = TileSet{tiles + vx.size() + vy.size(), (int)vz.size(), tbz};
  }
  {
    hipError_t r = hipErrorInvalidValue;
    PB3_DISPATCH_M(p.M, r = (inv_x_impl2<MM, double, true>(p, a1, p.d.tw_m_d, tsx, nullptr)); break);
    if (r != hipSuccess) { st = hip_fail(r, "count inverse x pass"); goto done; }
    r = hipErrorInvalidValue;
    PB3_DISPATCH_M(p.M, r = (inv_y_impl2<MM, double>(p, a1, a2, p.d.tw_m_d, tsy, nullptr)); break);
    if (r != hipSuccess) { st = hip_fail(r, "count inverse y pass"); goto done; }
    r = hipErrorInvalidValue;
    PB3_DISPATCH_M(p.M, r = (inv_z_impl2<MM, double>(p, a2, h, p.d.tw_m2_d, p.d.tw_m_d, tsz, nullptr)); break);
    if (r != hipSuccess) { st = hip_fail(r, "count inverse z pass"); goto done; }
    r = contract_simple<double>(h, p.nb, mvox, p.d.trip_all, n_cand, nwg, part, nullptr);
    if (r != hipSuccess) { st = hip_fail(r, "count contraction"); goto done; }
    hipLaunchKernelGGL((k_reduce<double>), dim3((n_cand + 255) / 256), dim3(256), 0, nullptr, part, nwg, n_cand, map,
                       (const double*)nullptr, n_cand, out);
    r = hipGetLastError();
    if (r != hipSuccess) { st = hip_fail(r, "count reduce"); goto done; }
    r = hipMemcpy(counts_out.data(), out, sizeof(double) * n_cand, hipMemcpyDeviceToHost);
    if (r != hipSuccess) { st = hip_fail(r, "count copy"); goto done; }
    double m6 = (double)p.M * p.M * p.M;
    m6 *= m6;
    for (auto& v : counts_out) v *= m6;
  }
done:
  hipFree(a1);
  hipFree(a2);
  hipFree(h);
  hipFree(part);
  hipFree(out);
  hipFree(map);
  hipFree(tiles);
  return st;
}

}  // namespace pb3
