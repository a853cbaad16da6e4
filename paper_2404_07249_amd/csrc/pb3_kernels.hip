// HIP kernels (gfx950) for the idealized binned power spectrum and
// bispectrum, apart from the FFT passes (fft_passes.hip) and the MFMA
// contraction (contract_mfma.hip): shell-binned power, the FP64 triplet
// contraction of the count pass, the fixed-order reductions and the count
// pass driver.  Launch wrappers at the bottom are called by pb3_host.cpp.
//
// Data layout in HBM (all C order, last index fastest):
//   delta  float  [N][N][N]
//   f1     float2 [N][N][Kz]         after the z pass (kz in [0, Kz))
//   f2     float2 [N][Lc][Kz]        after the y pass (ky centred-compact)
//   dc     float2 [Lc][Lc][Kz]       compact spectrum D(n), |n_i| <= K
//   a1_b   float2 [M][ly_b][kzn_b]   bin b after the inverse x pass
//   a2_b   float2 [M][M][kzn_b]      bin b after the inverse y pass
//   g      float  [nb][M][M][M]      filtered fields G_b on the contraction grid (separate z pass)
// A centred-compact index c holds frequency f = c - Kc.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "job.h"
#include "pb3_internal.h"

namespace pb3 {

// ------------------------------------------------------------------ power
// Each work-group sums w |D|^2 over one chunk of one bin's mode list in
// FP64 (w = 2 for modes whose conjugate partner is not stored, bit 31 of
// the index marks w = 1), then reduces with a fixed tree.
__global__ void __launch_bounds__(256) k_power_chunks(const float2* __restrict__ dc, const int32_t* __restrict__ modes,
                                                      const int32_t* __restrict__ chunks, double* __restrict__ part,
                                                      size_t wstride, const double* __restrict__ mw) {
  dc = job_ptr(dc, wstride);
  part = job_ptr(part, wstride);
  __shared__ double red[256];
  const int c = blockIdx.x;
  const int start = chunks[3 * c + 1], end = chunks[3 * c + 2];
  double acc = 0.0;
  for (int i = start + threadIdx.x; i < end; i += 256) {
    int32_t m = modes[i];
    double w = (m < 0) ? 1.0 : 2.0;
    if (mw) w *= mw[i];  // 1 / (m^2 P_fid^2) of the weighted estimator
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

// One work-group of 256 threads per bin: thread l sums the bin's partials
// l, l + 256, ..., four loads in flight per round, and the threads combine
// in a fixed-order tree in red[256].  The bins with the most partials have
// a few hundred, so one round of loads covers them.
__device__ __forceinline__ void power_bin_final(const double* __restrict__ part, const int32_t* __restrict__ chunk_first,
                                                int b, double* red, const double* __restrict__ scale, double shift,
                                                double* __restrict__ pk) {
  constexpr int NT = 256;
  const int l = threadIdx.x;
  const int first = chunk_first[b], last = chunk_first[b + 1];
  double s = 0.0;
  for (int c = first + l; c < last; c += 4 * NT) {
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = c + k * NT < last ? part[c + k * NT] : 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) s += v[k];
  }
  red[l] = s;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (l < h) red[l] += red[l + h];
    __syncthreads();
  }
  if (l == 0) pk[b] = red[0] * scale[b] - shift;
}

__global__ void __launch_bounds__(256) k_power_final(const double* __restrict__ part,
                                                     const int32_t* __restrict__ chunk_first, int nb,
                                                     const double* __restrict__ scale, const JobIO io, size_t wstride,
                                                     double shift) {
  __shared__ double red[256];
  power_bin_final(job_ptr(part, wstride), chunk_first, blockIdx.x, red, scale, shift, io.pk[blockIdx.z]);
}

// The power spectrum's last step inside the bispectrum's slice reduction,
// when one call computes both: rows of blocks past the slices take one bin
// each.
struct PowerFinal {
  const double* part = nullptr;  // chunk partials (per job at the workspace stride)
  const int32_t* chunk_first = nullptr;
  const double* scale = nullptr;
  double shift = 0.0;
  int nb = 0;
};

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
  constexpr int VS = VT + 1;  // odd row stride: threads reading different rows hit different banks
  extern __shared__ unsigned char smem_raw[];
  Rl* tileg = reinterpret_cast<Rl*>(smem_raw);  // [nb][VS]
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
      tileg[b * VS + j] = (v < v_end) ? g[(size_t)b * mvox + v] : Rl(0);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TPT; ++i) {
      if (ta[i] >= 0) {
        const Rl* pa = tileg + ta[i] * VS;
        const Rl* pb = tileg + tbb[i] * VS;
        const Rl* pc = tileg + tc[i] * VS;
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
                         const double* __restrict__ fac, int n_out, double* __restrict__ out,
                         const double* __restrict__ bias = nullptr) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_out) return;
  int idx = map[t];
  double s = 0.0;
  for (int w = 0; w < n_wg; ++w) s += (double)part[(size_t)w * part_len + idx];
  out[t] = (fac ? s * fac[t] : s) - (bias ? bias[t] : 0.0);
}

// Two-stage form for the MFMA partials: slice s of the work-groups is
// summed per element (FP64), then the slices per kept triplet.
// Each thread takes four neighbouring elements (one 16-byte load per
// work-group partial; part_len is a multiple of 256), each summed over the
// slice's work-groups in order.  With inv (element -> kept triplet or -1)
// the slice sums are stored in triplet order, rsl[s][t], so that the final
// launch reads them without a gather; otherwise every element, rsl[s][e].
// Rows of blocks past the slices finish the power spectrum (one bin per
// block), whose per-tile partials are complete when this launch starts.
__global__ void __launch_bounds__(256) k_reduce_slices(const float* __restrict__ part, int n_wg, int part_len,
                                                       double* __restrict__ rsl, size_t wstride,
                                                       const int32_t* __restrict__ inv, int n_out, PowerFinal pf,
                                                       const JobIO io) {
  if ((int)blockIdx.y >= kReduceSlices) {
    const int b = ((int)blockIdx.y - kReduceSlices) * (int)gridDim.x + (int)blockIdx.x;
    if (b >= pf.nb) return;  // whole work-group
    __shared__ double red[256];
    power_bin_final(job_ptr(pf.part, wstride), pf.chunk_first, b, red, pf.scale, pf.shift, io.pk[blockIdx.z]);
    return;
  }
  part = job_ptr(part, wstride);
  rsl = job_ptr(rsl, wstride);
  const int e = 4 * (blockIdx.x * blockDim.x + threadIdx.x);
  if (e >= part_len) return;
  const int s = blockIdx.y;
  const int w0 = (int)((long)n_wg * s / kReduceSlices), w1 = (int)((long)n_wg * (s + 1) / kReduceSlices);
  double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int w = w0; w < w1; ++w) {
    const float4 v = *reinterpret_cast<const float4*>(part + (size_t)w * part_len + e);
    a[0] += (double)v.x;
    a[1] += (double)v.y;
    a[2] += (double)v.z;
    a[3] += (double)v.w;
  }
  if (inv) {
    const int4 t = *reinterpret_cast<const int4*>(inv + e);
    double* __restrict__ o = rsl + (size_t)s * n_out;
    if (t.x >= 0) o[t.x] = a[0];
    if (t.y >= 0) o[t.y] = a[1];
    if (t.z >= 0) o[t.z] = a[2];
    if (t.w >= 0) o[t.w] = a[3];
  } else {
    double* __restrict__ o = rsl + (size_t)s * part_len + e;
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = a[k];
  }
}

// Per kept triplet t: the slices in order, rsl[s][map[t]] (map given, slice
// stride part_len) or rsl[s][t] (no map, slice stride n_out).
__global__ void __launch_bounds__(256) k_reduce_final(const double* __restrict__ rsl, int stride,
                                                      const int32_t* __restrict__ map, const double* __restrict__ fac,
                                                      int n_out, const JobIO io, size_t wstride,
                                                      const double* __restrict__ bias) {
  rsl = job_ptr(rsl, wstride);
  double* __restrict__ out = io.bk[blockIdx.z];
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_out) return;
  const int idx = map ? map[t] : t;
  double acc = 0.0;
#pragma unroll
  for (int s = 0; s < kReduceSlices; ++s) acc += rsl[(size_t)s * stride + idx];
  out[t] = acc * fac[t] - (bias ? bias[t] : 0.0);
}

// ---------------------------------------------------- window moments
// Conventional normalisation of masked data: sums of w^2 and w^3 over the
// grid (FP64; each block a contiguous range and a fixed tree, then the
// blocks in order), and P / <w^2>, B / <w^3> in place.
__global__ void __launch_bounds__(256) k_window_partial(const float* __restrict__ w, long n, long per_block,
                                                        double* __restrict__ part) {
  __shared__ double r2[256], r3[256];
  const long v0 = (long)blockIdx.x * per_block;
  long v1 = v0 + per_block;
  if (v1 > n) v1 = n;
  double s2 = 0.0, s3 = 0.0;
  for (long v = v0 + threadIdx.x; v < v1; v += 256) {
    double x = w[v];
    double x2 = x * x;
    s2 += x2;
    s3 += x2 * x;
  }
  r2[threadIdx.x] = s2;
  r3[threadIdx.x] = s3;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      r2[threadIdx.x] += r2[threadIdx.x + s];
      r3[threadIdx.x] += r3[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r2[0];
    part[2 * blockIdx.x + 1] = r3[0];
  }
}

__global__ void __launch_bounds__(256) k_window_apply(const double* __restrict__ part, int nblk, double npix,
                                                      double* __restrict__ pk, int nb, double* __restrict__ bk,
                                                      int nt, double* __restrict__ moments) {
  __shared__ double m[2];
  if (threadIdx.x == 0) {
    double s2 = 0.0, s3 = 0.0;
    for (int i = 0; i < nblk; ++i) {
      s2 += part[2 * i];
      s3 += part[2 * i + 1];
    }
    m[0] = s2 / npix;
    m[1] = s3 / npix;
    if (moments) {
      moments[0] = m[0];
      moments[1] = m[1];
    }
  }
  __syncthreads();
  if (pk)
    for (int i = threadIdx.x; i < nb; i += 256) pk[i] /= m[0];
  if (bk)
    for (int i = threadIdx.x; i < nt; i += 256) bk[i] /= m[1];
}

// ------------------------------------------- masked power spectrum (MC)
// Cross spectrum of two compact spectra per bin: each work-group sums
// w Re(conj(V) A) over one chunk of one bin's mode list in FP64 (w as in
// the power kernel), then per bin over its chunks in order, accumulated
// into row[b].
// Row blockIdx.y of a group of Fisher rows: its compact spectrum dv_stride
// values after the previous row's, its chunk partials gridDim.x after.
__global__ void __launch_bounds__(256) k_cross_chunks(const float2* __restrict__ dv, size_t dv_stride,
                                                      const float2* __restrict__ da,
                                                      const int32_t* __restrict__ modes,
                                                      const int32_t* __restrict__ chunks, double* __restrict__ part) {
  __shared__ double red[256];
  dv += (size_t)blockIdx.y * dv_stride;
  part += (size_t)blockIdx.y * gridDim.x;
  const int c = blockIdx.x;
  const int start = chunks[3 * c + 1], end = chunks[3 * c + 2];
  double acc = 0.0;
  for (int i = start + threadIdx.x; i < end; i += 256) {
    const int32_t m = modes[i];
    const double w = (m < 0) ? 1.0 : 2.0;
    const float2 v = dv[m & 0x7fffffff], a = da[m & 0x7fffffff];
    acc += w * ((double)v.x * a.x + (double)v.y * a.y);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[c] = red[0];
}

// Row a = blockIdx.y of the Fisher sums: part holds n_chunks partials per row.
__global__ void k_cross_final(const double* __restrict__ part, int n_chunks, const int32_t* __restrict__ chunk_first,
                              int nb, double* __restrict__ acc) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x, a = blockIdx.y;
  if (b >= nb) return;
  const double* pa = part + (size_t)a * n_chunks;
  double s = 0.0;
  for (int c = chunk_first[b]; c < chunk_first[b + 1]; ++c) s += pa[c];
  acc[(size_t)a * nb + b] += s;
}

__global__ void k_fill_zero(double* __restrict__ x, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// F = scale * acc (nb x nb), p_b = N_b P_box_b / 2, solve F x = p by
// Gaussian elimination with partial pivoting in FP64 (one work-group).
__global__ void __launch_bounds__(64) k_masked_solve(const double* __restrict__ acc, double scale,
                                                     const double* __restrict__ pbox,
                                                     const double* __restrict__ nmodes, int nb,
                                                     double* __restrict__ pk_out, double* __restrict__ f_out) {
  extern __shared__ double A[];  // [nb][nb + 1]
  __shared__ int piv;
  const int ld = nb + 1, tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 64) {
    const int r = e / nb, c = e % nb;
    const double v = scale * acc[e];
    A[r * ld + c] = v;
    if (f_out) f_out[e] = v;
  }
  for (int r = tid; r < nb; r += 64) A[r * ld + nb] = 0.5 * nmodes[r] * pbox[r];
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    if (tid == 0) {
      int best = k;
      for (int r = k + 1; r < nb; ++r)
        if (fabs(A[r * ld + k]) > fabs(A[best * ld + k])) best = r;
      piv = best;
    }
    __syncthreads();
    const int pr = piv;
    if (pr != k)
      for (int c = tid; c <= nb; c += 64) {
        const double t = A[k * ld + c];
        A[k * ld + c] = A[pr * ld + c];
        A[pr * ld + c] = t;
      }
    __syncthreads();
    const double d = A[k * ld + k];
    for (int r = k + 1 + tid; r < nb; r += 64) {
      const double f = A[r * ld + k] / d;
      for (int c = k; c <= nb; ++c) A[r * ld + c] -= f * A[k * ld + c];
    }
    __syncthreads();
  }
  if (tid == 0) {
    for (int r = nb - 1; r >= 0; --r) {
      double v = A[r * ld + nb];
      for (int c = r + 1; c < nb; ++c) v -= A[r * ld + c] * A[c * ld + nb];
      A[r * ld + nb] = v / A[r * ld + r];
    }
  }
  __syncthreads();
  for (int r = tid; r < nb; r += 64) pk_out[r] = A[r * ld + nb];
}

// ------------------------------------------------------------ multipoles
// Power multipoles (line of sight along z): per chunk of one bin's modes,
// sum_n w L_l(mu_n) |D(n)|^2 for l = 0, 2, .. (FP64), mu decoded from the
// compact index; then per bin P_l = sum_l' Finv[l][l'] p_l'.
__global__ void __launch_bounds__(256) k_power_ml_chunks(const float2* __restrict__ dc,
                                                         const int32_t* __restrict__ modes,
                                                         const int32_t* __restrict__ chunks, int Lcy, int Kz,
                                                         int Kcx, int Kcy, double sx, double sy, int ne,
                                                         double* __restrict__ part, const double* __restrict__ mw) {
  __shared__ double red[3][256];
  const int c = blockIdx.x;
  const int start = chunks[3 * c + 1], end = chunks[3 * c + 2];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int i = start + threadIdx.x; i < end; i += 256) {
    const int32_t m = modes[i];
    const double w = (m < 0) ? 1.0 : 2.0;
    const int idx = m & 0x7fffffff;
    const int kz = idx % Kz, cxy = idx / Kz;
    const int ky = cxy % Lcy - Kcy, kx = cxy / Lcy - Kcx;
    // k^2 / k_f,z^2 with the axis scales (exact integers for a cubic box)
    const double n2 = sx * kx * kx + sy * ky * ky + (double)kz * kz;
    const double m2 = n2 > 0 ? (double)kz * kz / n2 : 0.0;
    const float2 v = dc[idx];
    const double p2 = w * (mw ? mw[i] : 1.0) * ((double)v.x * v.x + (double)v.y * v.y);
    acc[0] += p2;
    acc[1] += p2 * (1.5 * m2 - 0.5);
    acc[2] += p2 * ((35.0 * m2 * m2 - 30.0 * m2 + 3.0) * 0.125);
  }
  for (int l = 0; l < 3; ++l) red[l][threadIdx.x] = acc[l];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int l = 0; l < 3; ++l) red[l][threadIdx.x] += red[l][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < ne) part[(size_t)c * ne + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_power_ml_final(const double* __restrict__ part, const int32_t* __restrict__ chunk_first, int nb,
                                 int ne, const double* __restrict__ finv, double* __restrict__ out, double shift) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  double p[3] = {0.0, 0.0, 0.0};
  for (int c = chunk_first[b]; c < chunk_first[b + 1]; ++c)
    for (int l = 0; l < ne; ++l) p[l] += part[(size_t)c * ne + l];
  for (int l = 0; l < ne; ++l) {
    double v = 0.0;
    for (int j = 0; j < ne; ++j) v += finv[((size_t)b * ne + l) * ne + j] * p[j];
    out[(size_t)l * nb + b] = l == 0 ? v - shift : v;  // Poisson noise is isotropic: monopole only
  }
}

// ================================================================ launchers

hipError_t launch_window(long n, const float* w, double* pk, int nb, double* bk, int nt, double* scratch,
                         hipStream_t s) {
  const long per = (n + kWindowBlocks - 1) / kWindowBlocks;
  hipLaunchKernelGGL(k_window_partial, dim3(kWindowBlocks), dim3(256), 0, s, w, n, per, scratch + 2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_window_apply, dim3(1), dim3(256), 0, s, (const double*)(scratch + 2), kWindowBlocks,
                     (double)n, pk, nb, bk, nt, scratch);
  return hipGetLastError();
}

hipError_t launch_power(const pb3_plan& p, const Exec& x, hipStream_t s, bool final) {
  hipLaunchKernelGGL(k_power_chunks, dim3(p.n_chunks, 1, x.n_jobs), dim3(256), 0, s, x.ws.dc, p.d.modes, p.d.chunk,
                     x.ws.ppart, x.wstride, (const double*)p.d.mode_w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !final) return e;
  hipLaunchKernelGGL(k_power_final, dim3(p.nb, 1, x.n_jobs), dim3(256), 0, s, x.ws.ppart, p.d.chunk_first, p.nb,
                     p.d.pk_scale, x.io, x.wstride, p.pk_shift);
  return hipGetLastError();
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
  size_t sh = (size_t)nb * 65 * sizeof(Rl);
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

hipError_t launch_contract(const pb3_plan& p, const Exec& x, pb3_precision prec, hipStream_t s) {
  return launch_contract_mfma(p, x, prec == PB3_MIXED_BF16X3, s);
}

hipError_t launch_reduce(const pb3_plan& p, const Exec& x, hipStream_t s, bool with_pk, bool pk_folded) {
  int n_out = (int)(p.trip.size() / 3);
  if (n_out == 0) return hipSuccess;
  PowerFinal pf;
  // the power partials are per chunk of a bin's mode list, or per inverse-x tile when that pass took them
  if (with_pk) pf = PowerFinal{x.ws.ppart, pk_folded ? p.d.xtile_first : p.d.chunk_first, p.d.pk_scale, p.pk_shift, p.nb};
  const int gx = (p.part_len / 4 + 255) / 256;
  const int pk_rows = (pf.nb + gx - 1) / gx;
  hipLaunchKernelGGL(k_reduce_slices, dim3(gx, kReduceSlices + pk_rows, x.n_jobs), dim3(256), 0, s, x.ws.part,
                     p.contract_wgs, p.part_len, x.ws.rsl, x.wstride, (const int32_t*)p.d.out_inv, n_out, pf, x.io);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3((n_out + 255) / 256, 1, x.n_jobs), dim3(256), 0, s, x.ws.rsl, n_out,
                     (const int32_t*)nullptr, p.d.inv_counts, n_out, x.io, x.wstride, (const double*)p.d.bk_bias);
  return hipGetLastError();
}

// ------------------------------------------- masked power spectrum (MC)
// Per random field a:  g_b = IDFT[Theta_b DFT[w a]] for every bin (inverse
// passes on the full grid), A = DFT[a] (compact), and for every bin a the
// compact DFT of w g_a, whose cross spectrum with A over bin b's modes is
// the Fourier-space dot product of the Fisher estimate
// (Q^asym_b[a] = Theta_b A).  The z direction of g_a -> DFT[w g_a] is one
// kernel over all bins (inverse z, window, forward z kept at kz < Kz), so
// the fields g_a never go to HBM; the y and x forward passes follow per bin.
// (z lengths without the half-length form write g_a [nb][N^3] and run the
// windowed forward z pass per bin instead.)
// The y and x forward passes and the cross spectra of up to kMaskedGroup
// bins share launches (grid z, resp. y, is the bin), each bin's arrays one
// field slot apart.
// Workspace: the plan's workspace, the z-transformed w g_b [nb][Nx Ny][Kz]
// (or g_b), the y and x pass outputs of a group of bins, the compact A,
// chunk partials, the Fisher sums [nb^2] and the data's box P [nb].
constexpr int kMaskedGroup = 8;

static size_t masked_field_bytes(const pb3_plan& p) {
  return zround_supported(p) ? sizeof(float2) * (size_t)p.Nx * p.Ny * p.Kz : sizeof(float) * npix(p);
}

static size_t masked_group_bytes(const pb3_plan& p) {
  return zround_supported(p) ? 2 * (size_t)std::min(kMaskedGroup, p.nb) * masked_field_bytes(p) : 0;
}

size_t masked_workspace_bytes(const pb3_plan& p) {
  const size_t A = 256, nb = (size_t)p.nb;
  auto up = [&](size_t b) { return (b + A - 1) / A * A; };
  const size_t dc = ncompact(p);
  return up(workspace_bytes(&p)) + up(nb * masked_field_bytes(p)) + up(masked_group_bytes(p)) +
         up(sizeof(float2) * dc) + up(sizeof(double) * nb * std::max(p.n_chunks, 1)) + up(sizeof(double) * nb * nb) +
         up(sizeof(double) * nb);
}

static pb3_status masked_tables(pb3_plan& p) {
  if (p.d.nmodes_d) return PB3_OK;
  std::vector<double> nm(p.nmodes.begin(), p.nmodes.end());
  double* t = nullptr;
  hipError_t e = dev_malloc((void**)&t, sizeof(double) * p.nb);
  if (e == hipSuccess) e = hipMemcpy(t, nm.data(), sizeof(double) * p.nb, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (t) hipFree(t);
    return hip_fail(e, "masked power tables");
  }
  p.d.nmodes_d = t;
  return PB3_OK;
}

pb3_status run_masked_power(pb3_plan& p, const float* data, const float* window, const float* const* grfs, int n_grf,
                            double* pk_out, double* f_out, void* workspace, hipStream_t s) {
  pb3_status st = masked_tables(p);
  if (st != PB3_OK) return st;
  const size_t A = 256, n3 = npix(p), dcn = ncompact(p), fb = masked_field_bytes(p);
  const int nb = p.nb, nt = nb * nb;
  const bool zr = zround_supported(p);
  auto up = [&](size_t b) { return (b + A - 1) / A * A; };
  char* c = (char*)workspace;
  Exec x;
  x.ws = carve(&p, c, workspace_bytes(&p));
  c += up(workspace_bytes(&p));
  char* fields = c;  // per bin: w g_b after the z round trip, or g_b
  c += up(nb * fb);
  char* grp = c;  // the y pass outputs of a group of bins, then their compact spectra
  c += up(masked_group_bytes(p));
  float2* dca = (float2*)c;
  c += up(sizeof(float2) * dcn);
  double* cpart = (double*)c;  // per row a: the chunk partials of its cross spectrum
  c += up(sizeof(double) * nb * std::max(p.n_chunks, 1));
  double* acc = (double*)c;
  c += up(sizeof(double) * nt);
  double* pbox = (double*)c;
  auto chk = [&](hipError_t r, const char* what) {
    if (r != hipSuccess) st = hip_fail(r, what);
    return r == hipSuccess;
  };
  auto forward = [&](const float* f, const float* w) {
    x.io.delta[0] = f;
    x.io.window = w;
    return chk(launch_fwd_z(p, x, s), "masked power: fwd_z") && chk(launch_fwd_y(p, x, s), "masked power: fwd_y") &&
           chk(launch_fwd_x(p, x, s), "masked power: fwd_x");
  };
  hipLaunchKernelGGL(k_fill_zero, dim3((nt + 255) / 256), dim3(256), 0, s, acc, nt);
  if (!chk(hipGetLastError(), "masked power: clear")) return st;
  for (int i = 0; i < n_grf; ++i) {
    // A = DFT[a], kept aside
    if (!forward(grfs[i], nullptr)) return st;
    if (!chk(hipMemcpyAsync(dca, x.ws.dc, sizeof(float2) * dcn, hipMemcpyDeviceToDevice, s), "masked power: copy"))
      return st;
    // g_b = IDFT[Theta_b DFT[w a]] on the full grid; with the round trip, w g_b through z both ways
    if (!forward(grfs[i], window) || !chk(launch_inv_x(p, x, s), "masked power: inv_x") ||
        !chk(launch_inv_y(p, x, s), "masked power: inv_y"))
      return st;
    if (zr ? !chk(run_zround(p, x.ws.a2, window, (float2*)fields, s), "masked power: z round trip")
           : !chk(run_inv_z(p, false, x.ws.a2, (float*)fields, p.tz, 1, 0, s), "masked power: inv_z"))
      return st;
    // rows a: cross spectra of DFT[w g_a] with A per bin
    if (zr) {
      for (int a0 = 0; a0 < nb; a0 += kMaskedGroup) {
        Exec xg = x;
        xg.n_jobs = std::min(kMaskedGroup, nb - a0);
        xg.wstride = fb;
        xg.ws.f1 = (float2*)(fields + (size_t)a0 * fb);
        xg.ws.f2 = (float2*)grp;
        xg.ws.dc = (float2*)(grp + (size_t)xg.n_jobs * fb);
        if (!chk(launch_fwd_y(p, xg, s), "masked power: fwd_y") || !chk(launch_fwd_x(p, xg, s), "masked power: fwd_x"))
          return st;
        hipLaunchKernelGGL(k_cross_chunks, dim3(p.n_chunks, xg.n_jobs), dim3(256), 0, s, (const float2*)xg.ws.dc,
                           fb / sizeof(float2), (const float2*)dca, p.d.modes, p.d.chunk,
                           cpart + (size_t)a0 * p.n_chunks);
        if (!chk(hipGetLastError(), "masked power: cross")) return st;
      }
    } else {
      for (int a = 0; a < nb; ++a) {
        if (!forward((const float*)(fields + (size_t)a * fb), window)) return st;
        hipLaunchKernelGGL(k_cross_chunks, dim3(p.n_chunks), dim3(256), 0, s, (const float2*)x.ws.dc, (size_t)0,
                           (const float2*)dca, p.d.modes, p.d.chunk, cpart + (size_t)a * p.n_chunks);
        if (!chk(hipGetLastError(), "masked power: cross")) return st;
      }
    }
    // all rows' per-bin sums at once, each in the order of its chunks
    hipLaunchKernelGGL(k_cross_final, dim3((nb + 63) / 64, nb), dim3(64), 0, s, cpart, p.n_chunks, p.d.chunk_first, nb,
                       acc);
    if (!chk(hipGetLastError(), "masked power: cross")) return st;
  }
  // numerator from the data's box power spectrum, then the solve
  x.io.pk[0] = pbox;
  if (!forward(data, nullptr) || !chk(launch_power(p, x, s, true), "masked power: power")) return st;
  const double scale = 0.5 / ((double)n3 * n_grf);
  hipLaunchKernelGGL(k_masked_solve, dim3(1), dim3(64), sizeof(double) * nb * (nb + 1), s, acc, scale, pbox,
                     p.d.nmodes_d, nb, pk_out, f_out);
  if (!chk(hipGetLastError(), "masked power: solve")) return st;
  return PB3_OK;
}

// ------------------------------------------------------------ multipoles
// Bispectrum multipoles: the Legendre-weighted filtered fields
// g_{c,l} = IDFT_M[Theta_c L_l(mu) D] for l = 0, 2, .. (l = 0 is G),
// then sum_x G_a G_b g_{c,l}: mixed precision on the MFMA contraction
// (pairs of G, columns of g_l), FP32 by the simple contraction (FP32
// tiles flushed to FP64); (2l + 1) V^2 M^6 / (N^9 T) per triplet.
// Workspace: the plan's, fields [n_ell][nb][M^3], partials
// [kMlWgs][n_trip], power-multipole chunk partials [n_chunks][n_ell].
constexpr int kMlWgs = 512;

size_t multipoles_workspace_bytes(const pb3_plan& p) {
  const size_t A = 256, m3 = mpix(p), ne = (size_t)(p.lmax / 2 + 1);
  const size_t nt = p.trip.size() / 3;
  auto up = [&](size_t b) { return (b + A - 1) / A * A; };
  return up(workspace_bytes(&p)) + up(sizeof(float) * ne * p.nb * m3) + up(sizeof(double) * kMlWgs * std::max<size_t>(nt, 1)) +
         up(sizeof(double) * std::max(p.n_chunks, 1) * ne);
}

__global__ void k_ml_mix(double* __restrict__ bk, const double* __restrict__ R, int nt, int ne);

pb3_status run_multipoles(pb3_plan& p, const float* delta, double* pk_out, double* bk_out, pb3_precision prec,
                          void* workspace, hipStream_t s) {
  const size_t A = 256, m3 = mpix(p);
  const int ne = p.lmax / 2 + 1, nt = (int)(p.trip.size() / 3);
  auto up = [&](size_t b) { return (b + A - 1) / A * A; };
  char* c = (char*)workspace;
  Exec x;
  x.ws = carve(&p, c, workspace_bytes(&p));
  c += up(workspace_bytes(&p));
  float* fields = (float*)c;
  c += up(sizeof(float) * ne * p.nb * m3);
  double* part = (double*)c;
  c += up(sizeof(double) * kMlWgs * std::max(nt, 1));
  double* mpart = (double*)c;
  pb3_status st = PB3_OK;
  auto chk = [&](hipError_t r, const char* what) {
    if (r != hipSuccess) st = hip_fail(r, what);
    return r == hipSuccess;
  };
  x.io.delta[0] = delta;
  if (!chk(launch_fwd_z(p, x, s), "multipoles: fwd_z") || !chk(launch_fwd_y(p, x, s), "multipoles: fwd_y") ||
      !chk(launch_fwd_x(p, x, s), "multipoles: fwd_x"))
    return st;
  if (pk_out) {
    hipLaunchKernelGGL(k_power_ml_chunks, dim3(p.n_chunks), dim3(256), 0, s, x.ws.dc, p.d.modes, p.d.chunk, p.Lcy,
                       p.Kz, p.Kcx, p.Kcy, p.msc[0], p.msc[1], ne, mpart, (const double*)p.d.mode_w);
    if (!chk(hipGetLastError(), "multipoles: power")) return st;
    hipLaunchKernelGGL(k_power_ml_final, dim3((p.nb + 63) / 64), dim3(64), 0, s, mpart, p.d.chunk_first, p.nb, ne,
                       p.d.pml_inv, pk_out, p.pk_shift);
    if (!chk(hipGetLastError(), "multipoles: power")) return st;
  }
  if (!bk_out || nt == 0) return PB3_OK;
  for (int l = 0; l < ne; ++l) {
    float* gl = fields + (size_t)l * p.nb * m3;
    if (!chk(run_inv_x(p, false, false, x.ws.dc, x.ws.a1, p.tx, 1, 0, s, 2 * l, nullptr, true),
             "multipoles: inv_x") ||
        !chk(launch_inv_y(p, x, s), "multipoles: inv_y") ||
        !chk(run_inv_z(p, false, x.ws.a2, gl, p.tz, 1, 0, s), "multipoles: inv_z"))
      return st;
  }
  if (prec == PB3_MIXED_BF16X3) {
    // MFMA: pairs of G against columns of g_l, the plan's reduction with (2l + 1) / T
    for (int l = 0; l < ne; ++l) {
      if (!chk(launch_contract_cols(p, x, fields, l ? fields + (size_t)l * p.nb * m3 : nullptr, true, true, s),
               "multipoles: contraction"))
        return st;
      hipLaunchKernelGGL(k_reduce_slices, dim3((p.part_len_ab / 4 + 255) / 256, kReduceSlices, 1), dim3(256), 0, s,
                         x.ws.part, p.contract_wgs, p.part_len_ab, x.ws.rsl, (size_t)0, (const int32_t*)nullptr, 0,
                         PowerFinal{}, JobIO{});
      if (!chk(hipGetLastError(), "multipoles: reduce")) return st;
      JobIO io{};
      io.bk[0] = bk_out + (size_t)l * nt;
      hipLaunchKernelGGL(k_reduce_final, dim3((nt + 255) / 256, 1, 1), dim3(256), 0, s, x.ws.rsl, p.part_len_ab,
                         (const int32_t*)p.d.out_map_ab, p.d.ml_fac + (size_t)l * nt, nt, io, (size_t)0,
                         l == 0 ? (const double*)p.d.bk_bias : nullptr);
      if (!chk(hipGetLastError(), "multipoles: reduce")) return st;
    }
  } else {
    for (int l = 0; l < ne; ++l) {
      if (!chk(contract_simple<float>(fields, ne * p.nb, (long)m3, p.d.ml_trips + (size_t)3 * l * nt, nt, kMlWgs,
                                      part, s),
               "multipoles: contraction"))
        return st;
      hipLaunchKernelGGL((k_reduce<double>), dim3((nt + 255) / 256), dim3(256), 0, s, part, kMlWgs, nt, p.d.ml_map,
                         p.d.ml_fac + (size_t)l * nt, nt, bk_out + (size_t)l * nt,
                         l == 0 ? (const double*)p.d.bk_bias : nullptr);
      if (!chk(hipGetLastError(), "multipoles: reduce")) return st;
    }
  }
  if (p.d.bk_mix) {  // the discrete Fisher matrix of the bispectrum multipoles
    hipLaunchKernelGGL(k_ml_mix, dim3((nt + 255) / 256), dim3(256), 0, s, bk_out, (const double*)p.d.bk_mix, nt, ne);
    if (!chk(hipGetLastError(), "multipoles: Fisher")) return st;
  }
  return PB3_OK;
}

// ----------------------------------------------- bispectrum linear term
// The linear term of the bispectrum numerator, averaged over fields Delta_i
// with (about) the data's covariance:
//   S_lin(d; D) = sum_x (G_a[d] G_b[D] G_c[D] + G_a[D] G_b[d] G_c[D] + G_a[D] G_b[D] G_c[d]).
// S is cubic and G linear in the field, so the part of S(D + d) with one
// factor of d is  S_lin = [S(D + d) - S(D - d)] / 2 - S(d);  the fields D +- d
// run through the plan's own launch sequence, two jobs per Delta_i and up
// to kMaxJobs jobs per launch, and the normalised results combine in FP64:
//   B = B(d) - (1/n) sum_i B_lin,i = 2 B(d) - (1/(2n)) sum_i [B(D_i + d) - B(D_i - d)].
struct LinIO {
  const float* sim[kMaxJobs / 2];
};

__global__ void __launch_bounds__(256) k_lin_fields(const float* __restrict__ d, const LinIO io, size_t n3,
                                                    float* __restrict__ out) {
  const float* __restrict__ e = io.sim[blockIdx.y];
  float* __restrict__ plus = out + (size_t)(2 * blockIdx.y) * n3;
  float* __restrict__ minus = plus + n3;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += stride) {
    const float dv = d[i], ev = e[i];
    plus[i] = ev + dv;
    minus[i] = ev - dv;
  }
}

// acc[t] (+)= sum_j (B(D_j + d) - B(D_j - d)), jobs in order
__global__ void k_lin_acc(const double* __restrict__ bt, int n_s, int nt, double* __restrict__ acc, int first) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  double s = first ? 0.0 : acc[t];
  for (int j = 0; j < n_s; ++j) s += bt[(size_t)(2 * j) * nt + t] - bt[(size_t)(2 * j + 1) * nt + t];
  acc[t] = s;
}

__global__ void k_lin_final(double* __restrict__ bk, const double* __restrict__ acc, int nt, double inv2n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  bk[t] = 2.0 * bk[t] - acc[t] * inv2n;
}

static int lin_jobs(int n_sim) { return std::min(kMaxJobs, 2 * std::max(n_sim, 1)); }

size_t linear_workspace_bytes(const pb3_plan& p, int n_sim) {
  const size_t A = 256, n3 = npix(p), nt = std::max<size_t>(p.trip.size() / 3, 1);
  auto up = [&](size_t b) { return (b + A - 1) / A * A; };
  const size_t J = (size_t)lin_jobs(n_sim);
  return J * up(workspace_bytes(&p)) + up(sizeof(float) * J * n3) + up(sizeof(double) * J * nt) +
         up(sizeof(double) * nt);
}

pb3_status run_bispectrum_linear(pb3_plan& p, const float* data, const float* const* sims, int n_sim, double* bk_out,
                                 pb3_precision prec, void* workspace, hipStream_t s) {
  const size_t A = 256, n3 = npix(p);
  const int nt = (int)(p.trip.size() / 3);
  auto up = [&](size_t b) { return (b + A - 1) / A * A; };
  const int J = lin_jobs(n_sim);
  const size_t stride = up(workspace_bytes(&p));
  char* c = (char*)workspace;
  char* wsb = c;
  c += (size_t)J * stride;
  float* fields = (float*)c;
  c += up(sizeof(float) * J * n3);
  double* bt = (double*)c;
  c += up(sizeof(double) * J * std::max(nt, 1));
  double* acc = (double*)c;
  if (nt == 0) return PB3_OK;
  pb3_status st;
  Exec x0;
  x0.ws = carve(&p, wsb, stride);
  x0.wstride = stride;
  x0.n_jobs = 1;
  x0.io.delta[0] = data;
  x0.io.bk[0] = bk_out;
  if ((st = enqueue(p, x0, false, true, prec, s)) != PB3_OK) return st;
  const int per = J / 2;
  const unsigned blocks = (unsigned)std::min<size_t>((n3 + 255) / 256, 2048);
  for (int i0 = 0; i0 < n_sim; i0 += per) {
    const int ns = std::min(per, n_sim - i0);
    LinIO io{};
    for (int j = 0; j < ns; ++j) io.sim[j] = sims[i0 + j];
    hipLaunchKernelGGL(k_lin_fields, dim3(blocks, ns), dim3(256), 0, s, data, io, n3, fields);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "linear term: fields");
    Exec x;
    x.ws = carve(&p, wsb, stride);
    x.wstride = stride;
    x.n_jobs = 2 * ns;
    for (int k = 0; k < 2 * ns; ++k) {
      x.io.delta[k] = fields + (size_t)k * n3;
      x.io.bk[k] = bt + (size_t)k * nt;
    }
    if ((st = enqueue(p, x, false, true, prec, s)) != PB3_OK) return st;
    hipLaunchKernelGGL(k_lin_acc, dim3((nt + 255) / 256), dim3(256), 0, s, (const double*)bt, ns, nt, acc,
                       i0 == 0 ? 1 : 0);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "linear term: accumulate");
  }
  hipLaunchKernelGGL(k_lin_final, dim3((nt + 255) / 256), dim3(256), 0, s, bk_out, (const double*)acc, nt,
                     0.5 / n_sim);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? PB3_OK : hip_fail(e, "linear term: combine");
}

// -------------------------------------------------------- FP64 counts
// T_abc = M^6 sum_x H_a H_b H_c on the contraction grid, H_b = IDFT[Theta_b],
// all in FP64 (N_0 of eq. N-ell-def with P_fid = 1), once per plan.
pb3_status compute_counts_fp64(pb3_plan& p, std::vector<double>& counts_out, std::vector<double>* q_out) {
  const int n_cand = (int)(p.trip_all.size() / 3);
  counts_out.assign(n_cand, 0.0);
  if (q_out) q_out->assign(n_cand, 0.0);
  if (n_cand == 0) return PB3_OK;
  // fields: the (weighted) unit fields, then, for the shot-noise sums, the
  // unweighted ones; the triplet table of each extra sum moves one leg
  const int nf = q_out ? 2 * p.nb : p.nb;
  int32_t* qtrips = nullptr;
  const long mvox = (long)mpix(p);
  const int nwg = 512;
  double2 *a1 = nullptr, *a2 = nullptr;
  double *h = nullptr, *part = nullptr, *out = nullptr;
  int32_t* map = nullptr;
  BinTile* tiles = nullptr;
  TileSet tsx{}, tsy{}, tsz{};
  hipError_t e;
  pb3_status st = PB3_OK;
  auto alloc = [&](void** ptr, size_t bytes) {
    e = dev_malloc(ptr, bytes);
    return e == hipSuccess;
  };
  std::vector<int32_t> idmap(n_cand);
  for (int i = 0; i < n_cand; ++i) idmap[i] = i;
  if (!alloc((void**)&a1, sizeof(double2) * p.a1_len) || !alloc((void**)&a2, sizeof(double2) * p.a2_len) ||
      !alloc((void**)&h, sizeof(double) * (size_t)nf * mvox) ||
      (q_out && !alloc((void**)&qtrips, sizeof(int32_t) * 9 * (size_t)n_cand)) ||
      !alloc((void**)&part, sizeof(double) * (size_t)nwg * n_cand) || !alloc((void**)&out, sizeof(double) * n_cand) ||
      !alloc((void**)&map, sizeof(int32_t) * n_cand)) {
    st = PB3_ENOMEM;
    set_error("device allocation failed while computing triangle counts");
    goto done;
  }
  e = hipMemset(h, 0, sizeof(double) * (size_t)nf * mvox);
  if (e != hipSuccess) { st = hip_fail(e, "hipMemset"); goto done; }
  e = hipMemcpy(map, idmap.data(), sizeof(int32_t) * n_cand, hipMemcpyHostToDevice);
  if (e != hipSuccess) { st = hip_fail(e, "hipMemcpy"); goto done; }
  {
    // FP64 lines take twice the LDS: the count pass has its own tile tables
    int tbx = tile_width_x(p.Mx, true), tbz = tile_width_z(p.Mz, true);
    if (tbx <= 0 || tbz <= 0) {
      st = PB3_EUNSUPPORTED;
      set_error("contraction grid not implemented");
      goto done;
    }
    std::vector<BinTile> vx, vy, vz;
    build_tiles(p, tbx, tbz, vx, vy, vz);
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
    hipError_t r = hipSuccess;
    for (int set = 0; set < (q_out ? 2 : 1); ++set) {
      const double* uw = set == 0 ? p.d.pfid_inv_d : nullptr;  // set 0: 1 / P_fid (null: unit), set 1: unit
      double* hs = h + (size_t)set * p.nb * mvox;
      r = run_inv_x(p, true, true, nullptr, a1, tsx, 1, 0, nullptr, 0, uw);
      if (r != hipSuccess) { st = hip_fail(r, "count inverse x pass"); goto done; }
      r = run_inv_y(p, true, a1, a2, tsy, 1, 0, nullptr);
      if (r != hipSuccess) { st = hip_fail(r, "count inverse y pass"); goto done; }
      r = run_inv_z(p, true, a2, hs, tsz, 1, 0, nullptr);
      if (r != hipSuccess) { st = hip_fail(r, "count inverse z pass"); goto done; }
    }
    if (q_out) {
      // Q = sum_x (H_a Hw_b Hw_c + Hw_a H_b Hw_c + Hw_a Hw_b H_c)
      std::vector<int32_t> qt(9 * (size_t)n_cand);
      for (int leg = 0; leg < 3; ++leg)
        for (int t = 0; t < n_cand; ++t)
          for (int k = 0; k < 3; ++k)
            qt[((size_t)leg * n_cand + t) * 3 + k] = p.trip_all[3 * t + k] + (k == leg ? p.nb : 0);
      r = hipMemcpy(qtrips, qt.data(), sizeof(int32_t) * qt.size(), hipMemcpyHostToDevice);
      if (r != hipSuccess) { st = hip_fail(r, "hipMemcpy"); goto done; }
      std::vector<double> tmp(n_cand);
      for (int leg = 0; leg < 3; ++leg) {
        r = contract_simple<double>(h, nf, mvox, qtrips + (size_t)3 * leg * n_cand, n_cand, nwg, part, nullptr);
        if (r != hipSuccess) { st = hip_fail(r, "shot-noise contraction"); goto done; }
        hipLaunchKernelGGL((k_reduce<double>), dim3((n_cand + 255) / 256), dim3(256), 0, nullptr, part, nwg, n_cand,
                           map, (const double*)nullptr, n_cand, out, (const double*)nullptr);
        r = hipMemcpy(tmp.data(), out, sizeof(double) * n_cand, hipMemcpyDeviceToHost);
        if (r != hipSuccess) { st = hip_fail(r, "shot-noise copy"); goto done; }
        for (int t = 0; t < n_cand; ++t) (*q_out)[t] += tmp[t];
      }
    }
    r = contract_simple<double>(h, nf, mvox, p.d.trip_all, n_cand, nwg, part, nullptr);
    if (r != hipSuccess) { st = hip_fail(r, "count contraction"); goto done; }
    hipLaunchKernelGGL((k_reduce<double>), dim3((n_cand + 255) / 256), dim3(256), 0, nullptr, part, nwg, n_cand, map,
                       (const double*)nullptr, n_cand, out, (const double*)nullptr);
    r = hipGetLastError();
    if (r != hipSuccess) { st = hip_fail(r, "count reduce"); goto done; }
    r = hipMemcpy(counts_out.data(), out, sizeof(double) * n_cand, hipMemcpyDeviceToHost);
    if (r != hipSuccess) { st = hip_fail(r, "count copy"); goto done; }
    double m6 = (double)p.Mx * p.My * p.Mz;
    m6 *= m6;
    for (auto& v : counts_out) v *= m6;
    if (q_out)
      for (auto& v : *q_out) v *= m6;
  }
done:
  hipFree(qtrips);
  hipFree(a1);
  hipFree(a2);
  hipFree(h);
  hipFree(part);
  hipFree(out);
  hipFree(map);
  hipFree(tiles);
  return st;
}


// ------------------------------------- bispectrum multipole Fisher matrix
// Per kept triplet t = (a, b, c) and l, l' in {0, 2, .., lmax}, sums over
// the closed triangles n1 + n2 + n3 = 0 (mod M) with n1 in a, n2 in b,
// n3 in c (mu_i = n_i,z / |n_i|, u_i = n_i / |n_i|):
// * the discrete ideal Fisher block of eq. (bk-fish-ideal) without its
//   1 / (Delta_l Delta_l'): Ft_{l l'} = sum L_l(mu_3) P_l' with, from the
//   permutations of the k's that keep every k_i in its bin,
//   P_l' = L_l'(mu_3) (a < b < c), 2 L_l'(mu_3) (a = b < c),
//   L_l'(mu_3) + L_l'(mu_2) (a < b = c), 2 [L_l'(mu_1) + L_l'(mu_2) + L_l'(mu_3)] (a = b = c);
// * the degeneracy factors of eq. (Delta-alpha-def), Delta_l = 1, 2,
//   1 + N_l/N_0, 2 (1 + 2 N_l/N_0) in the same cases, N_l = sum L_l(u_2 . u_3)
//   (eq. N-ell-def on the grid), N_0 = T.
// Every sum is separable: sum w1(n1) w2(n2) w3(n3) = M^6 sum_x H1_a H2_b H3_c
// with FP64 unit fields H_b = IDFT[Theta_b w]; N_l goes through
// (u_2 . u_3)^p = sum_{|alpha| = p} p!/alpha! u_2^alpha u_3^alpha, a mode
// with a Nyquist component taking the average over its representatives.  Both
// cross terms of a = b = c equal the (mu_3, mu_2) one (relabel n1 <-> n2).
// Output per triplet: R = Delta Ft^+ diag(T / (2l'+1)), Ft^+ the
// pseudo-inverse of the symmetric block (eigenvalues below 1e-12 of the
// largest dropped), so that b = F^-1 b^num = R y maps the eq. (ideal-bk)
// multipoles y_l = (2l+1) nt_l / T to the Fisher-normalised ones.

// Eigen-decomposition of a symmetric n x n matrix (n <= 3) by cyclic Jacobi
// rotations, then the pseudo-inverse.
static void pinv_sym(int n, const double* F, double* out) {
  double A[9], V[9];
  for (int i = 0; i < n * n; ++i) A[i] = 0.5 * (F[i] + F[(i % n) * n + i / n]);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0.0) continue;
        const double th = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A J
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - sn * akq;
          A[k * n + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^T A
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - sn * aqk;
          A[q * n + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {  // V <- V J
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - sn * vkq;
          V[k * n + q] = sn * vkp + c * vkq;
        }
      }
  }
  double big = 0.0;
  for (int i = 0; i < n; ++i) big = std::max(big, std::fabs(A[i * n + i]));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int k = 0; k < n; ++k) {
        const double w = A[k * n + k];
        if (std::fabs(w) > 1e-12 * big) acc += V[i * n + k] * V[j * n + k] / w;
      }
      out[i * n + j] = acc;
    }
}

pb3_status compute_bk_mixing(pb3_plan& p, std::vector<double>& mix_out) {
  const int nt = (int)(p.trip.size() / 3), nb = p.nb, ne = p.lmax / 2 + 1;
  mix_out.assign((size_t)nt * ne * ne, 0.0);
  if (nt == 0) return PB3_OK;
  const long mvox = (long)mpix(p);
  const int nwg = 512;
  double2 *a1 = nullptr, *a2 = nullptr;
  double *h = nullptr, *part = nullptr, *out = nullptr;
  int32_t *map = nullptr, *trips = nullptr;
  BinTile* tiles = nullptr;
  TileSet tsx{}, tsy{}, tsz{};
  hipError_t e;
  pb3_status st = PB3_OK;
  double m6 = (double)p.Mx * p.My * p.Mz;
  m6 *= m6;
  const int ells[3] = {0, 2, 4};
  std::vector<double> d33((size_t)ne * ne * nt), x32((size_t)ne * ne * nt), c2(nt, 0.0), c4(nt, 0.0), tmp(nt);
  auto alloc = [&](void** ptr, size_t bytes) {
    e = dev_malloc(ptr, bytes);
    return e == hipSuccess;
  };
  // three field sets: unit fields, and two weighted ones
  auto slot = [&](int k) { return h + (size_t)k * nb * mvox; };
  auto build = [&](int k, AngW aw) -> pb3_status {
    hipError_t r = run_inv_x(p, true, true, nullptr, a1, tsx, 1, 0, nullptr, 0, nullptr, false, aw);
    if (r != hipSuccess) return hip_fail(r, "Fisher inverse x pass");
    r = run_inv_y(p, true, a1, a2, tsy, 1, 0, nullptr);
    if (r != hipSuccess) return hip_fail(r, "Fisher inverse y pass");
    r = run_inv_z(p, true, a2, slot(k), tsz, 1, 0, nullptr);
    if (r != hipSuccess) return hip_fail(r, "Fisher inverse z pass");
    return PB3_OK;
  };
  // M^6 sum_x H_{sa}[a] H_{sb}[b] H_{sc}[c] for every kept triplet
  auto sum3 = [&](int sa, int sb, int sc, std::vector<double>& res) -> pb3_status {
    std::vector<int32_t> tb(3 * (size_t)nt);
    for (int t = 0; t < nt; ++t) {
      tb[3 * t] = sa * nb + p.trip[3 * t];
      tb[3 * t + 1] = sb * nb + p.trip[3 * t + 1];
      tb[3 * t + 2] = sc * nb + p.trip[3 * t + 2];
    }
    hipError_t r = hipMemcpy(trips, tb.data(), sizeof(int32_t) * tb.size(), hipMemcpyHostToDevice);
    if (r != hipSuccess) return hip_fail(r, "hipMemcpy");
    r = contract_simple<double>(h, 3 * nb, mvox, trips, nt, nwg, part, nullptr);
    if (r != hipSuccess) return hip_fail(r, "Fisher contraction");
    hipLaunchKernelGGL((k_reduce<double>), dim3((nt + 255) / 256), dim3(256), 0, nullptr, part, nwg, nt, map,
                       (const double*)nullptr, nt, out, (const double*)nullptr);
    r = hipGetLastError();
    if (r != hipSuccess) return hip_fail(r, "Fisher reduce");
    r = hipMemcpy(res.data(), out, sizeof(double) * nt, hipMemcpyDeviceToHost);
    if (r != hipSuccess) return hip_fail(r, "Fisher copy");
    for (auto& v : res) v *= m6;
    return PB3_OK;
  };
  std::vector<int32_t> idmap(nt);
  for (int i = 0; i < nt; ++i) idmap[i] = i;
  if (!alloc((void**)&a1, sizeof(double2) * p.a1_len) || !alloc((void**)&a2, sizeof(double2) * p.a2_len) ||
      !alloc((void**)&h, sizeof(double) * 3 * (size_t)nb * mvox) ||
      !alloc((void**)&trips, sizeof(int32_t) * 3 * (size_t)nt) ||
      !alloc((void**)&part, sizeof(double) * (size_t)nwg * nt) || !alloc((void**)&out, sizeof(double) * nt) ||
      !alloc((void**)&map, sizeof(int32_t) * nt)) {
    st = PB3_ENOMEM;
    set_error("device allocation failed while computing the bispectrum multipole Fisher matrix");
    goto done;
  }
  e = hipMemcpy(map, idmap.data(), sizeof(int32_t) * nt, hipMemcpyHostToDevice);
  if (e != hipSuccess) { st = hip_fail(e, "hipMemcpy"); goto done; }
  {
    int tbx = tile_width_x(p.Mx, true), tbz = tile_width_z(p.Mz, true);
    if (tbx <= 0 || tbz <= 0) {
      st = PB3_EUNSUPPORTED;
      set_error("contraction grid not implemented");
      goto done;
    }
    std::vector<BinTile> vx, vy, vz;
    build_tiles(p, tbx, tbz, vx, vy, vz);
    size_t ntile = vx.size() + vy.size() + vz.size();
    if (!alloc((void**)&tiles, sizeof(BinTile) * (ntile ? ntile : 1))) {
      st = PB3_ENOMEM;
      set_error("device allocation failed while computing the bispectrum multipole Fisher matrix");
      goto done;
    }
    std::vector<BinTile> all(vx);
    all.insert(all.end(), vy.begin(), vy.end());
    all.insert(all.end(), vz.begin(), vz.end());
    e = hipMemcpy(tiles, all.data(), sizeof(BinTile) * ntile, hipMemcpyHostToDevice);
    if (e != hipSuccess) { st = hip_fail(e, "hipMemcpy"); goto done; }
    tsx = TileSet{tiles, (int)vx.size(), tbx};
    tsy = TileSet{tiles + vx.size(), (int)vy.size(), tbx};
    tsz = TileSet{tiles + vx.size() + vy.size(), (int)vz.size(), tbz};
  }
  if ((st = build(0, AngW{})) != PB3_OK) goto done;
  // Legendre products on the third leg (d33) and the (mu_3, mu_2) cross terms (x32)
  for (int i = 0; i < ne && st == PB3_OK; ++i)
    for (int j = i; j < ne && st == PB3_OK; ++j) {
      double* dij = d33.data() + ((size_t)i * ne + j) * nt;
      double* xij = x32.data() + ((size_t)i * ne + j) * nt;
      if (i == 0 && j == 0) {
        for (int t = 0; t < nt; ++t) dij[t] = xij[t] = p.counts[t];
        continue;
      }
      AngW w;
      w.l1 = ells[i];
      w.l2 = ells[j];
      if ((st = build(1, w)) != PB3_OK) break;
      if ((st = sum3(0, 0, 1, tmp)) != PB3_OK) break;
      std::copy(tmp.begin(), tmp.end(), dij);
      // legs: unit on a, L_l' on b, L_l on c
      AngW wi, wj;
      wi.l1 = ells[i];
      wj.l1 = ells[j];
      int si = 0, sj;
      if (i > 0) {
        if ((st = build(1, wi)) != PB3_OK) break;
        si = 1;
      }
      if (j == i) {
        sj = si;
      } else {
        if ((st = build(2, wj)) != PB3_OK) break;
        sj = 2;
      }
      if ((st = sum3(0, sj, si, tmp)) != PB3_OK) break;
      std::copy(tmp.begin(), tmp.end(), xij);
    }
  if (st != PB3_OK) goto done;
  // sum (u_2 . u_3)^p for p = 2 (and 4)
  for (int pw = 2; pw <= (ne > 2 ? 4 : 2) && st == PB3_OK; pw += 2)
    for (int ex = 0; ex <= pw && st == PB3_OK; ++ex)
      for (int ey = 0; ex + ey <= pw && st == PB3_OK; ++ey) {
        const int ez = pw - ex - ey;
        AngW w;
        w.ex = ex;
        w.ey = ey;
        w.ez = ez;
        w.hx = p.Mx / 2;
        w.hy = p.My / 2;
        w.hz = p.Mz / 2;
        auto fact = [](int k) {
          double f = 1.0;
          for (int i = 2; i <= k; ++i) f *= i;
          return f;
        };
        const double coef = fact(pw) / (fact(ex) * fact(ey) * fact(ez));
        if ((st = build(1, w)) != PB3_OK) break;
        if ((st = sum3(0, 1, 1, tmp)) != PB3_OK) break;
        std::vector<double>& acc = pw == 2 ? c2 : c4;
        for (int t = 0; t < nt; ++t) acc[t] += coef * tmp[t];
      }
  if (st != PB3_OK) goto done;
  for (int t = 0; t < nt; ++t) {
    const int a = p.trip[3 * t], b = p.trip[3 * t + 1], c = p.trip[3 * t + 2];
    const int cs = (a == b && b == c) ? 3 : (a == b) ? 1 : (b == c) ? 2 : 0;
    const double T = p.counts[t];
    double F[9], Fi[9], Dl[3];
    for (int i = 0; i < ne; ++i) {
      const double nl = ells[i] == 0 ? T : ells[i] == 2 ? 1.5 * c2[t] - 0.5 * T
                                                        : (35.0 * c4[t] - 30.0 * c2[t] + 3.0 * T) / 8.0;
      const double r = nl / T;
      Dl[i] = cs == 0 ? 1.0 : cs == 1 ? 2.0 : cs == 2 ? 1.0 + r : 2.0 * (1.0 + 2.0 * r);
      for (int j = 0; j < ne; ++j) {
        const int lo = std::min(i, j), hi = std::max(i, j);
        const double dd = d33[((size_t)lo * ne + hi) * nt + t], xx = x32[((size_t)lo * ne + hi) * nt + t];
        F[i * ne + j] = cs == 0 ? dd : cs == 1 ? 2.0 * dd : cs == 2 ? dd + xx : 2.0 * (dd + 2.0 * xx);
      }
    }
    pinv_sym(ne, F, Fi);
    for (int i = 0; i < ne; ++i)
      for (int j = 0; j < ne; ++j)
        mix_out[((size_t)t * ne + i) * ne + j] = Dl[i] * Fi[i * ne + j] * T / (2.0 * ells[j] + 1.0);
  }
done:
  hipFree(a1);
  hipFree(a2);
  hipFree(h);
  hipFree(part);
  hipFree(out);
  hipFree(map);
  hipFree(trips);
  hipFree(tiles);
  return st;
}

// b[l][t] <- sum_l' R[t][l][l'] y[l'][t] in place (one thread per triplet).
__global__ void k_ml_mix(double* __restrict__ bk, const double* __restrict__ R, int nt, int ne) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  double y[3], b[3];
  for (int l = 0; l < ne; ++l) y[l] = bk[(size_t)l * nt + t];
  for (int l = 0; l < ne; ++l) {
    double acc = 0.0;
    for (int j = 0; j < ne; ++j) acc += R[((size_t)t * ne + l) * ne + j] * y[j];
    b[l] = acc;
  }
  for (int l = 0; l < ne; ++l) bk[(size_t)l * nt + t] = b[l];
}

}  // namespace pb3
