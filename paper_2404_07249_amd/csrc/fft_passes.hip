// FFT passes of the estimator (gfx950), built on the two-phase register FFT
// fft2_line (fft_dev.h):
//
//   forward  z  r2c  delta[x][y][:]            -> f1[x][y][kz < Kz]        (length Nz)
//   forward  y  c2c  f1[x][:][kz]              -> f2[x][kyc][kz]   (Ny; centred-compact rows kept)
//   forward  x  c2c  f2[:][kyc][kz]            -> dc[kxc][kyc][kz]         (Nx)
//   inverse  x  c2c  Theta_b D, gathered per bin -> a1_b[x][jy][jz]        (Mx)
//   inverse  y  c2c  a1_b[x][:][jz]            -> a2_b[x][y][jz]           (My)
//   inverse  z  c2r  a2_b[x][y][:]             -> G_b[x][y][z]  (Mz; scaled by 1/(Mx My Mz))
//
// The z passes transform two real lines with one complex FFT: forward,
// z = x_A + i x_B and X_A = (Z_k + conj Z_{N-k})/2, X_B = (Z_k - conj Z_{N-k})/(2i);
// inverse, Y = F_A + i F_B (each extended by Hermitian symmetry), whose
// transform has G_A as real part and G_B as imaginary part.  Strided passes
// take TB neighbouring columns per work-group so that every global access
// is coalesced across the columns.

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_dev.h"
#include "job.h"
#include "pb3_internal.h"

namespace pb3 {

// Work-groups go to the 8 XCDs of the chip round-robin, each XCD with its
// own L2.  The per-bin passes number their tiles so that neighbours share
// cache lines (the column chunks of one row); this maps consecutive tiles
// to work-groups of one XCD (b, b + 8, b + 16, ...), launched as 8 * per
// work-groups of which those past the last tile return at once.
constexpr int kXcds = 8;
__host__ __device__ inline int xcd_tiles(int n) { return kXcds * ((n + kXcds - 1) / kXcds); }
__device__ __forceinline__ int xcd_tile(int b, int n) { return (b % kXcds) * ((n + kXcds - 1) / kXcds) + b / kXcds; }

// Strided passes: TB columns per work-group, TL threads per column.
template <int N, int CS> struct ColShape {
  static constexpr int TL = fft2_threads(N);
  static constexpr int TB = CS == 8 ? 16 : 8;
  static constexpr int LS = N + 1;  // odd LDS stride between columns
  static constexpr int NT = TB * TL;
};
// z passes: TP pairs of lines per work-group, TL threads per pair.
template <int N, int CS> struct PairShape {
  static constexpr int TL = fft2_threads(N);
  static constexpr int TP = ((CS == 8 ? 256 : 128) / TL) < 1 ? 1 : ((CS == 8 ? 256 : 128) / TL);
  static constexpr int LS = N + 1;
  static constexpr int NT = TP * TL;
};

// ------------------------------------------------------------ forward z
// Pair form, for the short lines (N < 64): two real lines as one complex
// line of length N.
template <int N>
__global__ void __launch_bounds__(512) k_fwd_z2(const JobIO io, float2* __restrict__ f1, size_t wstride,
                                                int n_pairs, int Kz, const float2* __restrict__ tw) {
  const float* __restrict__ delta = io.delta[blockIdx.z];
  f1 = job_ptr(f1, wstride);
  using S = PairShape<N, 8>;
  constexpr int TL = S::TL, TP = S::TP, LS = S::LS;
  __shared__ float2 tws[N];
  __shared__ float2 scr[TP * LS];  // the FFT exchange, then the spectra
  const int tid = threadIdx.x;
  for (int e = tid; e < N; e += S::NT) tws[e] = tw[e];
  __syncthreads();
  const int pl = tid / TL, tl = tid % TL;
  const int pair = blockIdx.x * TP + pl;
  const bool live = pair < n_pairs;
  const size_t off = (size_t)(2 * (live ? pair : 0)) * N;
  const float* xa = delta + off;
  const float* xb = xa + N;
  const float* wa = io.window ? io.window + off : nullptr;  // optional window multiplying the field
  float2* z = scr + pl * LS;
  fft2_line<N, -1, true>(
      scr + pl * LS, tl, tws,
      [&](int n) {
        if (!live) return make_float2(0.f, 0.f);
        float2 v = make_float2(xa[n], xb[n]);
        if (wa) {
          v.x *= wa[n];
          v.y *= wa[N + n];
        }
        return v;
      },
      [&](int k, float2 v) { z[k] = v; });
  __syncthreads();
  const int line0 = 2 * blockIdx.x * TP;
  int nl = 2 * n_pairs - line0;
  if (nl > 2 * TP) nl = 2 * TP;
  for (int e = tid; e < nl * Kz; e += S::NT) {
    int ll = e / Kz, k = e % Kz;
    const float2* zz = scr + (ll >> 1) * LS;
    float2 a = zz[k % N], b = zz[(N - k) % N];
    float2 o = (ll & 1) == 0 ? make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y))
                             : make_float2(0.5f * (a.y + b.y), 0.5f * (b.x - a.x));
    f1[(size_t)(line0 + ll) * Kz + k] = o;
  }
}

// Half-length form, for N = 32 H' with H' in {2, 3, 4, 6, 8, 12}: a real
// line x of length N is the complex line z[m] = x[2m] + i x[2m+1] of length
// H = N/2.  With Z = DFT_H[z] (indices mod H), the even and odd samples
// have the spectra E[k] = (Z[k] + conj Z[H-k]) / 2 and
// O[k] = -i (Z[k] - conj Z[H-k]) / 2, and X[k] = E[k] + W_N^k O[k] for
// k < Kz.  The line FFT takes R2 = 16 loaders, so the 16 threads of a line
// read 128 contiguous bytes per load (the pair form reads 64), and its
// exchange rows are padded (PAD = 1) so that phase 2's reads fall in
// distinct LDS banks.  16 lines per work-group.
template <int N> struct HalfShape {
  static constexpr int H = N / 2, R2 = 16, R1 = H / 16;
  static constexpr int TL = 16, NL = 16, NT = TL * NL;
  static constexpr int EX = R1 * (R2 + 1);
  static constexpr int LS = (EX > H ? EX : H) + 1;
};
constexpr bool half_form(int n) { return n == 64 || n == 96 || n == 128 || n == 192 || n == 256 || n == 384; }
template <int N>
__global__ void __launch_bounds__(256) k_fwd_zh(const JobIO io, float2* __restrict__ f1, size_t wstride, int n_lines,
                                                int Kz, const float2* __restrict__ tw) {
  const float* __restrict__ delta = io.delta[blockIdx.z];
  f1 = job_ptr(f1, wstride);
  using S = HalfShape<N>;
  constexpr int H = S::H, TL = S::TL, NL = S::NL, LS = S::LS;
  __shared__ float2 tws[N];  // W_N^m
  __shared__ float2 twh[H];  // W_H^m = W_N^(2m)
  __shared__ float2 scr[NL * LS];  // the FFT exchange, then Z
  const int tid = threadIdx.x;
  for (int e = tid; e < N; e += S::NT) {
    const float2 w = tw[e];
    tws[e] = w;
    if (!(e & 1)) twh[e >> 1] = w;
  }
  __syncthreads();
  const int ln = tid / TL, tl = tid % TL;
  const int line = blockIdx.x * NL + ln;
  const bool live = line < n_lines;
  const size_t off = (size_t)(live ? line : 0) * N;
  const float2* z = reinterpret_cast<const float2*>(delta + off);
  const float2* wz = io.window ? reinterpret_cast<const float2*>(io.window + off) : nullptr;  // optional window
  float2* zl = scr + ln * LS;
  fft2_line<H, -1, true, 1, S::R1>(
      zl, tl, twh,
      [&](int m) {
        if (!live) return make_float2(0.f, 0.f);
        float2 v = z[m];
        if (wz) {
          const float2 w = wz[m];
          v.x *= w.x;
          v.y *= w.y;
        }
        return v;
      },
      [&](int k, float2 v) { zl[k] = v; });
  __syncthreads();
  const int line0 = blockIdx.x * NL;
  int nl = n_lines - line0;
  if (nl > NL) nl = NL;
  for (int e = tid; e < nl * Kz; e += S::NT) {
    const int ll = e / Kz, k = e % Kz;
    const float2* zz = scr + ll * LS;
    const int kh = k % H;
    const float2 a = zz[kh], b = zz[(H - kh) % H];
    const float ex = 0.5f * (a.x + b.x), ey = 0.5f * (a.y - b.y);   // E[k]
    const float ox = 0.5f * (a.y + b.y), oy = -0.5f * (a.x - b.x);  // O[k]
    const float2 w = tws[k];                                        // k < Kz <= N/2 + 1
    f1[(size_t)(line0 + ll) * Kz + k] = make_float2(ex + w.x * ox - w.y * oy, ey + w.x * oy + w.y * ox);
  }
}

// --------------------------------------------------- forward strided c2c
// out row c <- frequency f = c - Ko (kept when 0 <= c < Lo).
template <int N>
__global__ void __launch_bounds__(512) k_fwd_col2(const float2* __restrict__ in, float2* __restrict__ out, int n_inner,
                                                  int n_outer, long in_outer, long out_outer, int Lo, int Ko,
                                                  const float2* __restrict__ tw, size_t wstride) {
  in = job_ptr(in, wstride);
  out = job_ptr(out, wstride);
  using S = ColShape<N, 8>;
  constexpr int TB = S::TB, LS = S::LS;
  __shared__ float2 tws[N];
  __shared__ float2 scr[TB * LS];
  // tiles (outer, chunk of TB inner columns), chunks of one outer row next to
  // each other and on one XCD (rows shorter than a cache line multiple share lines)
  const int n_ck = (n_inner + TB - 1) / TB, n_t = n_ck * n_outer;
  const int t = xcd_tile(blockIdx.x, n_t);
  if (t >= n_t) return;  // whole work-group
  const int ck = t % n_ck, outer = t / n_ck;
  const int tid = threadIdx.x;
  for (int e = tid; e < N; e += S::NT) tws[e] = tw[e];
  __syncthreads();
  const int tl = tid / TB, col = tid % TB;
  const int inner = ck * TB + col;
  const bool live = inner < n_inner;
  const float2* src = in + (size_t)outer * in_outer + (live ? inner : 0);
  float2* dst = out + (size_t)outer * out_outer + inner;
  fft2_line<N, -1>(
      scr + col * LS, tl, tws, [&](int n) { return live ? src[(size_t)n * n_inner] : make_float2(0.f, 0.f); },
      [&](int k, float2 v) {
        int f = k >= N - Ko ? k - N : k;
        int c = f + Ko;
        if (live && c >= 0 && c < Lo) dst[(size_t)c * n_inner] = v;
      });
}

// ---------------------------------------------------------- inverse x
// Per bin b, one work-group per chunk of TB consecutive columns jy * kzn +
// kz of the bin's (ky, kz) rectangle, taken in row-major order so that no
// lane idles at the end of a short row; consecutive chunks have consecutive
// tile indices, so they run together and their partial cache lines combine.
// The kx line of Theta_b D (Theta_b alone when UNIT) enters at FFT
// positions kx mod M.  A mode belongs to the bin when the plan's per-mode
// table bin3 says so; bin3 carries one more entry, "no bin", at index nb3.
// In a cubic box the plain path tests n2lo <= |n|^2 < n2hi instead.
// Output a1_b[x][jy][jz].  Tile col0 = first column.
struct WinOff {
  int x, y, z;  // offsets of k = 0 of each axis in the window table
};

__device__ __forceinline__ double legendre_m2(int l, double m2) {
  switch (l) {
    case 2: return 1.5 * m2 - 0.5;
    case 4: return (35.0 * m2 * m2 - 30.0 * m2 + 3.0) * 0.125;
    default: return 1.0;
  }
}
__device__ __forceinline__ double ipow(double x, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

template <int M, typename Rl, bool UNIT>
__global__ void __launch_bounds__(512) k_inv_x2(const float2* __restrict__ dc, typename Cx<Rl>::type* __restrict__ a1,
                                                const BinGeom* __restrict__ geom, const BinTile* __restrict__ tiles,
                                                int n_tiles, const int8_t* __restrict__ bin3, int Kcx, int Kcy,
                                                int Lcy, int Kz,
                                                const typename Cx<Rl>::type* __restrict__ tw, size_t wstride,
                                                int ell, const float* __restrict__ winv, WinOff wo, float sx,
                                                float sy, const float* __restrict__ pinv,
                                                const double* __restrict__ uw, AngW aw, size_t nb3,
                                                double* __restrict__ ppart, int kz_nyq) {
  dc = job_ptr(dc, wstride);
  a1 = job_ptr(a1, wstride);
  using C = typename Cx<Rl>::type;
  using S = ColShape<M, (int)sizeof(C)>;
  constexpr int TB = S::TB, LS = S::LS;
  __shared__ C tws[M];
  __shared__ C scr[TB * LS];
  const int tid = threadIdx.x;
  for (int e = tid; e < M; e += S::NT) tws[e] = tw[e];
  __syncthreads();
  const int tl = tid / TB, col = tid % TB;
  const int ti = xcd_tile(blockIdx.x, n_tiles);
  if (ti >= n_tiles) return;  // whole work-group
  const BinTile tile = tiles[ti];
  const int b = tile.bin;
  const BinGeom g = geom[b];
  const int ncol = g.ly * g.kzn;
  {
    const int c = tile.col0 + col;  // column jy * kzn + kz of the bin's block
    const bool live = c < ncol;
    const int jy = c / g.kzn, kz = c - jy * g.kzn;
    const int ky = jy - g.knegy;
    C* dst = a1 + g.a1_off + c;
    auto store = [&](int x, C v) {
      if (live) dst[(size_t)x * ncol] = v;
    };
    if constexpr (!UNIT) {
      if (!winv && !pinv && !ell) {
        // Plain spectra: every lane makes both lookups unconditionally (off
        // the bin's rectangle it reads the table's trailing "no bin" entry
        // and value 0) and masks the value by a multiplication, so the
        // loads of a line are in flight together rather than one element
        // after another.  The forward pass writes every compact entry, so
        // a masked-out value is finite whenever the field is.
        // With ppart, the lanes also sum |Theta_b D|^2 over the modes they
        // gather: each of the bin's modes lies in exactly one column of
        // one of its tiles, so the tiles' sums are the power spectrum's
        // numerator (eq. pk-limit), weight 2 for the half spectrum's
        // modes whose conjugate is not stored.
        // In a cubic box the membership is the integer test n2lo <= |n|^2 <
        // n2hi, the same modes as the table's, with no table reads.
        double pacc = 0.0;
        const int r2 = ky * ky + kz * kz;
        auto gather = [&](auto by_n2) {
          fft2_line<M, 1>(
              scr + col * LS, tl, tws,
              [&](int n) {
                const int kx = n <= g.kposx ? n : (n >= M - g.knegx ? n - M : 0x40000000);
                const bool in = live && kx != 0x40000000;
                const size_t ci = in ? ((size_t)(kx + Kcx) * Lcy + (ky + Kcy)) * Kz + kz : 0;
                bool inb;
                if constexpr (decltype(by_n2)::value) {
                  const int kxi = in ? kx : 0;
                  const int n2 = kxi * kxi + r2;
                  inb = in && n2 >= g.n2lo && n2 < g.n2hi;
                } else {
                  inb = bin3[in ? ci : nb3] == b;
                }
                const float2 d = dc[ci];
                const float m = inb ? 1.f : 0.f;
                const float vx = fmaf(d.x, m, 0.f), vy = fmaf(d.y, m, 0.f);
                if (ppart) pacc += (double)vx * vx + (double)vy * vy;
                return cx<C>(Rl(vx), Rl(vy));
              },
              store);
        };
        if (g.n2lo >= 0)
          gather(std::true_type{});
        else
          gather(std::false_type{});
        if (ppart) {
          // fixed-order sum over the work-group: butterfly within each
          // wave, then the waves in order
          static_assert(S::NT % 64 == 0, "whole wavefronts");
          __shared__ double wsum[S::NT / 64];
          double v = pacc * ((kz == 0 || kz == kz_nyq) ? 1.0 : 2.0);
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
          if ((tid & 63) == 0) wsum[tid >> 6] = v;
          __syncthreads();
          if (tid == 0) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < S::NT / 64; ++w) t += wsum[w];
            job_ptr(ppart, wstride)[ti] = t;
          }
        }
        return;
      }
    }
    fft2_line<M, 1>(
        scr + col * LS, tl, tws,
        [&](int n) {
          C v = cx<C>(Rl(0), Rl(0));
          int kx = n <= g.kposx ? n : (n >= M - g.knegx ? n - M : 0x40000000);
          const size_t ci = kx != 0x40000000 ? ((size_t)(kx + Kcx) * Lcy + (ky + Kcy)) * Kz + kz : 0;
          if (live && kx != 0x40000000 && bin3[ci] == b) {
            if constexpr (UNIT) {
              double w = uw ? uw[kx * kx + ky * ky + kz * kz] : 1.0;  // 1 / P_fid in the weighted count
              if (aw.l1 | aw.l2 | aw.ex | aw.ey | aw.ez) {
                // physical wave-vector in units of k_f,z (exact integers for equal box sides)
                const double fx = sqrt((double)sx) * kx, fy = sqrt((double)sy) * ky, fz = (double)kz;
                const double k2 = fx * fx + fy * fy + fz * fz, r = sqrt(k2);
                w *= legendre_m2(aw.l1, fz * fz / k2) * legendre_m2(aw.l2, fz * fz / k2);
                w *= ipow(fx / r, aw.ex) * ipow(fy / r, aw.ey) * ipow(fz / r, aw.ez);
                if (((aw.ex & 1) && abs(kx) == aw.hx) || ((aw.ey & 1) && abs(ky) == aw.hy) ||
                    ((aw.ez & 1) && kz == aw.hz))
                  w = 0.0;
              }
              v = cx<C>(Rl(w), Rl(0));
            } else {
              float2 d = dc[ci];
              if (winv || pinv) {  // weighted estimator: D / (m P_fid)
                float u = pinv ? pinv[kx * kx + ky * ky + kz * kz] : 1.f;
                if (winv) u *= winv[wo.x + kx] * winv[wo.y + ky] * winv[wo.z + kz];
                d.x *= u;
                d.y *= u;
              }
              if (ell) {  // Legendre weight L_ell(mu), mu = k_z / |k| (line of sight along z)
                // k^2 / k_f,z^2 with the axis scales (exact integers for a cubic box)
                const float k2 = sx * (float)(kx * kx) + sy * (float)(ky * ky) + (float)(kz * kz);
                const float m2 = k2 > 0.f ? (float)(kz * kz) / k2 : 0.f;
                const float L = ell == 2 ? 1.5f * m2 - 0.5f : (35.f * m2 * m2 - 30.f * m2 + 3.f) * 0.125f;
                d.x *= L;
                d.y *= L;
              }
              v = cx<C>(Rl(d.x), Rl(d.y));
            }
          }
          return v;
        },
        store);
  }
}

// ---------------------------------------------------------- inverse y
// Per bin, one work-group per chunk of TB consecutive columns x * kzn + jz
// of the bin's mx planes (a chunk may span two planes, so no lane idles at
// the end of a plane); consecutive chunks on one XCD.  Inverse transform
// along y.  Tile col0 = first column.
template <int M, typename Rl>
__global__ void __launch_bounds__(512) k_inv_y2(const typename Cx<Rl>::type* __restrict__ a1,
                                                typename Cx<Rl>::type* __restrict__ a2,
                                                const BinGeom* __restrict__ geom, const BinTile* __restrict__ tiles,
                                                int n_tiles, const typename Cx<Rl>::type* __restrict__ tw,
                                                size_t wstride, int mx) {
  a1 = job_ptr(a1, wstride);
  a2 = job_ptr(a2, wstride);
  using C = typename Cx<Rl>::type;
  using S = ColShape<M, (int)sizeof(C)>;
  constexpr int TB = S::TB, LS = S::LS;
  __shared__ C tws[M];
  __shared__ C scr[TB * LS];
  const int tid = threadIdx.x;
  for (int e = tid; e < M; e += S::NT) tws[e] = tw[e];
  __syncthreads();
  const int tl = tid / TB, col = tid % TB;
  const int ti = xcd_tile(blockIdx.x, n_tiles);
  if (ti >= n_tiles) return;  // whole work-group
  const BinTile tile = tiles[ti];
  const BinGeom g = geom[tile.bin];
  {
    const int c = tile.col0 + col;  // column x * kzn + jz
    const bool live = c < mx * g.kzn;
    const int x = c / g.kzn, jz = c - x * g.kzn;
    const C* src = a1 + g.a1_off + ((size_t)x * g.ly + g.knegy) * g.kzn + jz;  // ky = 0 row
    C* dst = a2 + g.a2_off + (size_t)x * M * g.kzn + jz;
    fft2_line<M, 1>(
        scr + col * LS, tl, tws,
        [&](int n) {
          int ky = n <= g.kposy ? n : (n >= M - g.knegy ? n - M : 0x40000000);
          return (live && ky != 0x40000000) ? src[(long)ky * g.kzn] : cx<C>(Rl(0), Rl(0));
        },
        [&](int y, C v) {
          if (live) dst[(size_t)y * g.kzn] = v;
        });
  }
}

// ---------------------------------------------------------- inverse z
// Per bin: 2*TP consecutive lines (x, y) per work-group, kz in [0, kzn).
// The input block is staged in LDS with coalesced loads; each pair of
// lines is one complex inverse FFT; the real outputs are staged in LDS and
// written back as one contiguous block.
template <int M, typename Rl>
__global__ void __launch_bounds__(512) k_inv_z2(const typename Cx<Rl>::type* __restrict__ a2, Rl* __restrict__ gout,
                                                const BinGeom* __restrict__ geom, const BinTile* __restrict__ tiles,
                                                int n_tiles, const typename Cx<Rl>::type* __restrict__ tw, Rl scale,
                                                int nlines, size_t wstride) {
  a2 = job_ptr(a2, wstride);
  gout = job_ptr(gout, wstride);
  using C = typename Cx<Rl>::type;
  using S = PairShape<M, (int)sizeof(C)>;
  constexpr int TL = S::TL, TP = S::TP, LS = S::LS;
  __shared__ C tws[M];
  __shared__ C scr[TP * LS];
  __shared__ C stage[TP * (M + 2)];  // input 2TP x kzn complex, then output 2TP x M reals
  const int tid = threadIdx.x;
  for (int e = tid; e < M; e += S::NT) tws[e] = tw[e];
  const int ti = xcd_tile(blockIdx.x, n_tiles);
  if (ti >= n_tiles) return;  // whole work-group
  const BinTile tile = tiles[ti];
  const BinGeom g = geom[tile.bin];
  const int kzn = g.kzn;
  const int line0 = tile.col0;
  int nl = nlines - line0;
  if (nl > 2 * TP) nl = 2 * TP;
  const C* src = a2 + g.a2_off + (size_t)line0 * kzn;
  for (int e = tid; e < nl * kzn; e += S::NT) stage[e] = src[e];
  __syncthreads();
  const int pl = tid / TL, tl = tid % TL;
  const bool has_a = 2 * pl < nl, has_b = 2 * pl + 1 < nl;
  const C* xa = stage + 2 * pl * kzn;
  const C* xb = xa + kzn;
  Rl* outr = reinterpret_cast<Rl*>(stage);
  fft2_line<M, 1>(
      scr + pl * LS, tl, tws,
      [&](int k) {
        C a = cx<C>(Rl(0), Rl(0)), b = cx<C>(Rl(0), Rl(0));
        if (k < kzn) {
          if (has_a) a = xa[k];
          if (has_b) b = xb[k];
          return cx<C>(a.x - b.y, a.y + b.x);  // F_A + i F_B
        }
        int m = M - k;
        if (m < kzn) {
          if (has_a) a = xa[m];
          if (has_b) b = xb[m];
          return cx<C>(a.x + b.y, b.x - a.y);  // conj F_A(m) + i conj F_B(m)
        }
        return cx<C>(Rl(0), Rl(0));
      },
      [&](int z, C v) {
        outr[(2 * pl) * M + z] = v.x * scale;
        outr[(2 * pl + 1) * M + z] = v.y * scale;
      });
  __syncthreads();
  Rl* dst = gout + (size_t)tile.bin * ((size_t)nlines * M) + (size_t)line0 * M;
  for (int e = tid; e < nl * M / 2; e += S::NT)
    reinterpret_cast<C*>(dst)[e] = reinterpret_cast<const C*>(outr)[e];
}

// ------------------------------------------- z round trip (masked power)
// For the Monte Carlo Fisher matrix of the masked power spectrum: per z
// line and bin, the inverse z transform of the inverse y pass's output (the
// filtered field g_b on the full grid), times the window w on the line,
// then the forward z transform of w g_b kept at kz < Kz: the forward z pass
// of DFT[w g_b] without g_b ever leaving the chip.  Both transforms take
// the half-length form (N = 2H, real lines as complex lines of H points):
//   inverse: with X[k + H] = conj X[H - k] (X real-valued in z),
//     Z[k] = (X[k] + conj X[H - k]) + i W_N^-k (X[k] - conj X[H - k]),
//     z = IDFT_H[Z] (unnormalised) gives x[2m] = Re z[m], x[2m + 1] = Im z[m];
//   forward: as in the forward z pass above.
// A slot of 16 lanes owns one line for all bins; the window of its line is
// read once into registers, and the next bin's inputs are fetched while the
// current bin is transformed.  Output f1 [nb][lines][Kz].
template <int N>
__global__ void __launch_bounds__(256) k_zround(const float2* __restrict__ a2, float2* __restrict__ f1,
                                                const float* __restrict__ w, const BinGeom* __restrict__ geom, int nb,
                                                const float2* __restrict__ tw, float scale, int nlines, int Kz) {
  constexpr int H = N / 2, R2 = 16, R1 = H / 16, TL = 16, NL = 16, EX = R1 * (R2 + 1);
  static_assert(R1 * 16 == H && R1 <= 16, "half-length lines of 16 x R1 points");
  __shared__ float2 tws[N];  // W_N^m
  __shared__ float2 twh[H];  // W_H^m = W_N^(2m)
  __shared__ float2 xs[NL * EX];  // per line: the FFT exchange
  __shared__ float2 ys[NL * EX];  // per line: w x between the transforms, then the spectrum Z
  const int tid = threadIdx.x;
  for (int e = tid; e < N; e += NL * TL) {
    const float2 v = tw[e];
    tws[e] = v;
    if (!(e & 1)) twh[e >> 1] = v;
  }
  __syncthreads();
  const int ln = tid / TL, tl = tid % TL;
  const int line = blockIdx.x * NL + ln;
  if (line >= nlines) return;  // whole slot; no work-group barrier follows
  float2* xl = xs + ln * EX;
  float2* yl = ys + ln * EX;
  // the window at x[2m], x[2m + 1] for this lane's forward inputs m = tl + 16 j
  float2 wv[R1];
  const float2* wl = reinterpret_cast<const float2*>(w + (size_t)line * N);
#pragma unroll
  for (int j = 0; j < R1; ++j) wv[j] = wl[tl + R2 * j];
  // X[m] and X[H - m] of this lane's inverse inputs m = tl + 16 j (zero past the bin's planes)
  float2 xa[R1], xc[R1];
  auto fetch = [&](int b) {
    const BinGeom g = geom[b];
    const int kzn = g.kzn;
    const float2* X = a2 + g.a2_off + (size_t)line * kzn;
#pragma unroll
    for (int j = 0; j < R1; ++j) {
      const int m = tl + R2 * j;
      xa[j] = m < kzn ? X[m] : make_float2(0.f, 0.f);
      xc[j] = H - m < kzn ? X[H - m] : make_float2(0.f, 0.f);
    }
  };
  fetch(0);
  for (int b = 0; b < nb; ++b) {
    fft2_line_wave<H, 1, R1>(
        xl, tl, twh,
        [&](int j, int m) {
          const float2 a = xa[j], c = xc[j];                    // conj of c taken below
          const float2 e = make_float2(a.x + c.x, a.y - c.y);  // X[m] + conj X[H - m]
          const float2 d = make_float2(a.x - c.x, a.y + c.y);  // X[m] - conj X[H - m]
          const float2 t = tws[m];                              // W_N^m; times its conjugate below
          const float2 o = make_float2(d.x * t.x + d.y * t.y, d.y * t.x - d.x * t.y);
          return make_float2(e.x - o.y, e.y + o.x);  // E' + i O'
        },
        [&] {
          if (b + 1 < nb) fetch(b + 1);
        },
        [&](int k1, const float2 (&u)[R2]) {
#pragma unroll
          for (int k2 = 0; k2 < R2; ++k2) yl[k1 + R1 * k2] = make_float2(u[k2].x * scale, u[k2].y * scale);
        });
    fft2_line_wave<H, -1, R1>(
        xl, tl, twh,
        [&](int j, int m) {
          const float2 v = yl[m];
          return make_float2(v.x * wv[j].x, v.y * wv[j].y);
        },
        [] {},
        [&](int k1, const float2 (&u)[R2]) {
#pragma unroll
          for (int k2 = 0; k2 < R2; ++k2) yl[k1 + R1 * k2] = u[k2];
        });
    float2* dst = f1 + (size_t)b * ((size_t)nlines * Kz) + (size_t)line * Kz;
    for (int k = tl; k < Kz; k += TL) {
      const int kh = k % H;
      const float2 a = yl[kh], c = yl[(H - kh) % H];
      const float ex = 0.5f * (a.x + c.x), ey = 0.5f * (a.y - c.y);   // E[k]
      const float ox = 0.5f * (a.y + c.y), oy = -0.5f * (a.x - c.x);  // O[k]
      const float2 t = tws[k];                                        // k < Kz <= N/2 + 1
      dst[k] = make_float2(ex + t.x * ox - t.y * oy, ey + t.x * oy + t.y * ox);
    }
    // the next bin's transforms write these rows again
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// ================================================================ launchers

#define PB3_FFT_LEN(len, ...)                          \
  switch (len) {                                       \
    case 16: { constexpr int LL = 16; __VA_ARGS__; }   \
    case 24: { constexpr int LL = 24; __VA_ARGS__; }   \
    case 32: { constexpr int LL = 32; __VA_ARGS__; }   \
    case 48: { constexpr int LL = 48; __VA_ARGS__; }   \
    case 64: { constexpr int LL = 64; __VA_ARGS__; }   \
    case 96: { constexpr int LL = 96; __VA_ARGS__; }   \
    case 128: { constexpr int LL = 128; __VA_ARGS__; } \
    case 192: { constexpr int LL = 192; __VA_ARGS__; } \
    case 256: { constexpr int LL = 256; __VA_ARGS__; } \
    case 384: { constexpr int LL = 384; __VA_ARGS__; } \
    default: break;                                    \
  }

int tile_width_x(int M, bool dbl) {
  PB3_FFT_LEN(M, return dbl ? ColShape<LL, 16>::TB : ColShape<LL, 8>::TB);
  return 0;
}
int tile_width_z(int M, bool dbl) {
  PB3_FFT_LEN(M, return 2 * (dbl ? PairShape<LL, 16>::TP : PairShape<LL, 8>::TP));
  return 0;
}

hipError_t launch_fwd_z(const pb3_plan& p, const Exec& x, hipStream_t s) {
  const int n_pairs = p.Nx * p.Ny / 2;
  PB3_FFT_LEN(p.Nz, {
    if constexpr (half_form(LL)) {
      const int n_lines = p.Nx * p.Ny;
      using S = HalfShape<LL>;
      hipLaunchKernelGGL(k_fwd_zh<LL>, dim3((n_lines + S::NL - 1) / S::NL, 1, x.n_jobs), dim3(S::NT), 0, s, x.io,
                         x.ws.f1, x.wstride, n_lines, p.Kz, p.d.tw_n[2]);
      return hipGetLastError();
    }
    break;
  });
  PB3_FFT_LEN(p.Nz, {
    if constexpr (!half_form(LL)) {
      using S = PairShape<LL, 8>;
      hipLaunchKernelGGL(k_fwd_z2<LL>, dim3((n_pairs + S::TP - 1) / S::TP, 1, x.n_jobs), dim3(S::NT), 0, s, x.io,
                         x.ws.f1, x.wstride, n_pairs, p.Kz, p.d.tw_n[2]);
      return hipGetLastError();
    }
    break;
  });
  return hipErrorInvalidValue;
}

// transform of length len along one axis keeping the centred-compact rows [0, Lo)
static hipError_t fwd_col(const Exec& x, int len, const float2* tw, int Lo, int Ko, const float2* in, float2* out,
                          int n_inner, long in_outer, long out_outer, int n_outer, hipStream_t s) {
  PB3_FFT_LEN(len, {
    using S = ColShape<LL, 8>;
    dim3 grid(xcd_tiles((n_inner + S::TB - 1) / S::TB * n_outer), 1, x.n_jobs);
    hipLaunchKernelGGL(k_fwd_col2<LL>, grid, dim3(S::NT), 0, s, in, out, n_inner, n_outer, in_outer, out_outer, Lo, Ko,
                       tw, x.wstride);
    return hipGetLastError();
  });
  return hipErrorInvalidValue;
}
hipError_t launch_fwd_y(const pb3_plan& p, const Exec& x, hipStream_t s) {
  // f1[x][y][kz] -> f2[x][kyc][kz]
  return fwd_col(x, p.Ny, p.d.tw_n[1], p.Lcy, p.Kcy, x.ws.f1, x.ws.f2, p.Kz, (long)p.Ny * p.Kz, (long)p.Lcy * p.Kz,
                 p.Nx, s);
}
hipError_t launch_fwd_x(const pb3_plan& p, const Exec& x, hipStream_t s) {
  // f2[x][kyc][kz] -> dc[kxc][kyc][kz]
  return fwd_col(x, p.Nx, p.d.tw_n[0], p.Lcx, p.Kcx, x.ws.f2, x.ws.dc, p.Lcy * p.Kz, 0L, 0L, 1, s);
}

hipError_t run_inv_x(const pb3_plan& p, bool dbl, bool unit, const float2* dc, void* a1, const TileSet& ts,
                     int n_jobs, size_t wstride, hipStream_t s, int ell, const double* unit_w, bool weighted,
                     AngW aw, double* ppart) {
  const float* winv = weighted ? p.d.win_inv : nullptr;
  const float* pinv = weighted ? p.d.pfid_inv : nullptr;
  const WinOff wo{p.Nx / 2, p.Nx + 1 + p.Ny / 2, p.Nx + p.Ny + 2 + p.Nz / 2};
  const float sx = (float)p.msc[0], sy = (float)p.msc[1];
  const void* tw = dbl ? (const void*)p.d.tw_m_d[0] : (const void*)p.d.tw_m[0];
  if (ts.n == 0) return hipSuccess;
  PB3_FFT_LEN(p.Mx, {
    if (dbl) {
      using S = ColShape<LL, 16>;
      if (unit)
        hipLaunchKernelGGL((k_inv_x2<LL, double, true>), dim3(xcd_tiles(ts.n), 1, n_jobs), dim3(S::NT), 0, s, dc,
                           (double2*)a1, p.d.geom, ts.d, ts.n, p.d.bin3, p.Kcx, p.Kcy, p.Lcy, p.Kz, (const double2*)tw,
                           wstride, 0, (const float*)nullptr, wo, sx, sy, (const float*)nullptr, unit_w, aw, ncompact(p),
                           (double*)nullptr, -1);
      else
        return hipErrorInvalidValue;
    } else {
      using S = ColShape<LL, 8>;
      if (unit) return hipErrorInvalidValue;
      if (ppart && (winv || pinv || ell)) return hipErrorInvalidValue;  // the power sums take plain spectra
      hipLaunchKernelGGL((k_inv_x2<LL, float, false>), dim3(xcd_tiles(ts.n), 1, n_jobs), dim3(S::NT), 0, s, dc,
                         (float2*)a1, p.d.geom, ts.d, ts.n, p.d.bin3, p.Kcx, p.Kcy, p.Lcy, p.Kz, (const float2*)tw,
                         wstride, ell, winv, wo, sx, sy, pinv, (const double*)nullptr, AngW{}, ncompact(p), ppart,
                         p.fullz ? p.Nz / 2 : -1);
    }
    return hipGetLastError();
  });
  return hipErrorInvalidValue;
}

hipError_t run_inv_y(const pb3_plan& p, bool dbl, const void* a1, void* a2, const TileSet& ts, int n_jobs,
                     size_t wstride, hipStream_t s) {
  const void* tw = dbl ? (const void*)p.d.tw_m_d[1] : (const void*)p.d.tw_m[1];
  if (ts.n == 0) return hipSuccess;
  PB3_FFT_LEN(p.My, {
    if (dbl) {
      using S = ColShape<LL, 16>;
      hipLaunchKernelGGL((k_inv_y2<LL, double>), dim3(xcd_tiles(ts.n), 1, n_jobs), dim3(S::NT), 0, s, (const double2*)a1,
                         (double2*)a2, p.d.geom, ts.d, ts.n, (const double2*)tw, wstride, p.Mx);
    } else {
      using S = ColShape<LL, 8>;
      hipLaunchKernelGGL((k_inv_y2<LL, float>), dim3(xcd_tiles(ts.n), 1, n_jobs), dim3(S::NT), 0, s, (const float2*)a1,
                         (float2*)a2, p.d.geom, ts.d, ts.n, (const float2*)tw, wstride, p.Mx);
    }
    return hipGetLastError();
  });
  return hipErrorInvalidValue;
}

hipError_t run_inv_z(const pb3_plan& p, bool dbl, const void* a2, void* gout, const TileSet& ts, int n_jobs,
                     size_t wstride, hipStream_t s) {
  const void* tw = dbl ? (const void*)p.d.tw_m_d[2] : (const void*)p.d.tw_m[2];
  const int nlines = p.Mx * p.My;
  if (ts.n == 0) return hipSuccess;
  const double sc = 1.0 / ((double)p.Mx * p.My * p.Mz);
  PB3_FFT_LEN(p.Mz, {
    if (dbl) {
      using S = PairShape<LL, 16>;
      if (ts.tb != 2 * S::TP) return hipErrorInvalidConfiguration;
      hipLaunchKernelGGL((k_inv_z2<LL, double>), dim3(xcd_tiles(ts.n), 1, n_jobs), dim3(S::NT), 0, s, (const double2*)a2,
                         (double*)gout, p.d.geom, ts.d, ts.n, (const double2*)tw, sc, nlines, wstride);
    } else {
      using S = PairShape<LL, 8>;
      if (ts.tb != 2 * S::TP) return hipErrorInvalidConfiguration;
      hipLaunchKernelGGL((k_inv_z2<LL, float>), dim3(xcd_tiles(ts.n), 1, n_jobs), dim3(S::NT), 0, s, (const float2*)a2,
                         (float*)gout, p.d.geom, ts.d, ts.n, (const float2*)tw, (float)sc, nlines, wstride);
    }
    return hipGetLastError();
  });
  return hipErrorInvalidValue;
}

bool zround_supported(const pb3_plan& p) {
  return p.Mx == p.Nx && p.My == p.Ny && p.Mz == p.Nz && half_form(p.Nz);
}

hipError_t run_zround(const pb3_plan& p, const float2* a2, const float* window, float2* f1, hipStream_t s) {
  if (!zround_supported(p)) return hipErrorInvalidValue;
  const int nlines = p.Nx * p.Ny;
  const float sc = (float)(1.0 / ((double)p.Mx * p.My * p.Mz));
  PB3_FFT_LEN(p.Nz, {
    if constexpr (half_form(LL)) {
      hipLaunchKernelGGL(k_zround<LL>, dim3((nlines + 15) / 16), dim3(256), 0, s, a2, f1, window, p.d.geom, p.nb,
                         p.d.tw_n[2], sc, nlines, p.Kz);
      return hipGetLastError();
    }
    break;
  });
  return hipErrorInvalidValue;
}

hipError_t launch_inv_x(const pb3_plan& p, const Exec& x, hipStream_t s, double* ppart) {
  return run_inv_x(p, false, false, x.ws.dc, x.ws.a1, p.tx, x.n_jobs, x.wstride, s, 0, nullptr, true, AngW{}, ppart);
}
hipError_t launch_inv_y(const pb3_plan& p, const Exec& x, hipStream_t s) {
  return run_inv_y(p, false, x.ws.a1, x.ws.a2, p.ty, x.n_jobs, x.wstride, s);
}
hipError_t launch_inv_z(const pb3_plan& p, const Exec& x, hipStream_t s) {
  return run_inv_z(p, false, x.ws.a2, x.ws.g, p.tz, x.n_jobs, x.wstride, s);
}

}  // namespace pb3
