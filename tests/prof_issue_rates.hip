// Issue-rate probe for gfx950 (not collected by pytest): cycles per
// iteration of short register-only instruction patterns (plain and DPP
// multiplies, v_dot2c_f32_bf16, v_cvt_pk_bf16_f32, 16x16x32 bf16 MFMA, and
// MFMA interleaved with independent multiplies) on one work-group of 4 or 8
// waves (one or two waves per SIMD), timed with the shader clock.  Each
// thread stores one value in bounds; no memory is read.
//
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         tests/prof_issue_rates.hip -o /tmp/prof_issue_rates && /tmp/prof_issue_rates
#include <hip/hip_runtime.h>
#include <cstdio>
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
constexpr int IT = 2048;

template <int P>
__global__ void __launch_bounds__(512) k(float seed, float* out, long long* cyc) {
  float x0 = seed + threadIdx.x, x1 = x0 + 1, x2 = x0 + 2, x3 = x0 + 3, x4 = x0 + 4, x5 = x0 + 5, x6 = x0 + 6, x7 = x0 + 7;
  float x8 = x0 + 8;
  unsigned h0 = threadIdx.x * 77u, h1 = h0 + 1, h2 = h0 + 2, h3 = h0 + 3;
  f4 a0 = {x0, x1, x2, x3}, a1 = a0, a2 = a0, a3 = a0, a4 = a0, a5 = a0, a6 = a0, a7 = a0;
  s8 m = {1, 2, 3, 4, 5, 6, 7, 8};
  long long t0 = clock64();
  for (int it = 0; it < IT; ++it) {
    if constexpr (P == 0) {  // 8 v_mul_f32
      asm volatile("v_mul_f32 %0, %0, %1" : "+v"(x0) : "v"(x1)); asm volatile("v_mul_f32 %0, %0, %1" : "+v"(x2) : "v"(x1));
      asm volatile("v_mul_f32 %0, %0, %1" : "+v"(x3) : "v"(x1)); asm volatile("v_mul_f32 %0, %0, %1" : "+v"(x4) : "v"(x1));
      asm volatile("v_mul_f32 %0, %0, %1" : "+v"(x5) : "v"(x1)); asm volatile("v_mul_f32 %0, %0, %1" : "+v"(x6) : "v"(x1));
      asm volatile("v_mul_f32 %0, %0, %1" : "+v"(x7) : "v"(x1)); asm volatile("v_mul_f32 %0, %0, %1" : "+v"(h0) : "v"(x1));
    } else if constexpr (P == 1) {  // 8 v_dot2c_f32_bf16
      asm volatile("v_dot2c_f32_bf16 %0, %1, %2" : "+v"(x0) : "v"(h1), "v"(h2)); asm volatile("v_dot2c_f32_bf16 %0, %1, %2" : "+v"(x2) : "v"(h1), "v"(h2));
      asm volatile("v_dot2c_f32_bf16 %0, %1, %2" : "+v"(x3) : "v"(h1), "v"(h2)); asm volatile("v_dot2c_f32_bf16 %0, %1, %2" : "+v"(x4) : "v"(h1), "v"(h2));
      asm volatile("v_dot2c_f32_bf16 %0, %1, %2" : "+v"(x5) : "v"(h1), "v"(h2)); asm volatile("v_dot2c_f32_bf16 %0, %1, %2" : "+v"(x6) : "v"(h1), "v"(h2));
      asm volatile("v_dot2c_f32_bf16 %0, %1, %2" : "+v"(x7) : "v"(h1), "v"(h2)); asm volatile("v_dot2c_f32_bf16 %0, %1, %2" : "+v"(h0) : "v"(h1), "v"(h2));
    } else if constexpr (P == 2) {  // 8 v_cvt_pk_bf16_f32
      asm volatile("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(h0) : "v"(x1), "v"(x2)); asm volatile("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(h1) : "v"(x1), "v"(x2));
      asm volatile("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(h2) : "v"(x1), "v"(x2)); asm volatile("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(h3) : "v"(x1), "v"(x2));
      asm volatile("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(h0) : "v"(x3), "v"(x2)); asm volatile("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(h1) : "v"(x3), "v"(x2));
      asm volatile("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(h2) : "v"(x3), "v"(x2)); asm volatile("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(h3) : "v"(x3), "v"(x2));
    } else if constexpr (P == 3) {  // 8 v_mul_f32_dpp row_ror
      asm volatile("v_mul_f32_dpp %0, %1, %2 row_ror:1 row_mask:0xf bank_mask:0xf bound_ctrl:1" : "=v"(x0) : "v"(x1), "v"(x2));
      asm volatile("v_mul_f32_dpp %0, %1, %2 row_ror:2 row_mask:0xf bank_mask:0xf bound_ctrl:1" : "=v"(x3) : "v"(x1), "v"(x2));
      asm volatile("v_mul_f32_dpp %0, %1, %2 row_ror:3 row_mask:0xf bank_mask:0xf bound_ctrl:1" : "=v"(x4) : "v"(x1), "v"(x2));
      asm volatile("v_mul_f32_dpp %0, %1, %2 row_ror:4 row_mask:0xf bank_mask:0xf bound_ctrl:1" : "=v"(x5) : "v"(x1), "v"(x2));
      asm volatile("v_mul_f32_dpp %0, %1, %2 row_ror:5 row_mask:0xf bank_mask:0xf bound_ctrl:1" : "=v"(x6) : "v"(x1), "v"(x2));
      asm volatile("v_mul_f32_dpp %0, %1, %2 row_ror:6 row_mask:0xf bank_mask:0xf bound_ctrl:1" : "=v"(x7) : "v"(x1), "v"(x2));
      asm volatile("v_mul_f32_dpp %0, %1, %2 row_ror:7 row_mask:0xf bank_mask:0xf bound_ctrl:1" : "=v"(x0) : "v"(x1), "v"(x2));
      asm volatile("v_mul_f32_dpp %0, %1, %2 row_ror:8 row_mask:0xf bank_mask:0xf bound_ctrl:1" : "=v"(x3) : "v"(x1), "v"(x2));
    } else if constexpr (P == 4) {  // 8 independent MFMA 16x16x32 bf16
      asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %1, %0" : "+v"(a0) : "v"(m)); asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %1, %0" : "+v"(a1) : "v"(m));
      asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %1, %0" : "+v"(a2) : "v"(m)); asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %1, %0" : "+v"(a3) : "v"(m));
      asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %1, %0" : "+v"(a4) : "v"(m)); asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %1, %0" : "+v"(a5) : "v"(m));
      asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %1, %0" : "+v"(a6) : "v"(m)); asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %1, %0" : "+v"(a7) : "v"(m));
    } else if constexpr (P >= 5 && P <= 9) {  // 8 x (1 MFMA + K independent v_mul), K = 2 (P-5)
      constexpr int K = 2 * (P - 5);
#define MF(A) asm volatile("v_mfma_f32_16x16x32_bf16 %0, %1, %1, %0" : "+v"(A) : "v"(m));
#define VM(X) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(X) : "v"(x1));
#define VK if constexpr (K >= 1) { VM(x0) } if constexpr (K >= 2) { VM(x2) } if constexpr (K >= 3) { VM(x3) } if constexpr (K >= 4) { VM(x4) } \
           if constexpr (K >= 5) { VM(x5) } if constexpr (K >= 6) { VM(x6) } if constexpr (K >= 7) { VM(x7) } if constexpr (K >= 8) { VM(x8) }
      MF(a0) VK MF(a1) VK MF(a2) VK MF(a3) VK MF(a4) VK MF(a5) VK MF(a6) VK MF(a7) VK
    }
  }
  long long t1 = clock64();
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  out[g] = x0 + x8 + x2 + x3 + x4 + x5 + x6 + x7 + __uint_as_float(h0 ^ h1 ^ h2 ^ h3) + a0[0] + a1[1] + a2[2] + a3[3] + a4[0] + a5[1] + a6[2] + a7[3];
  if ((threadIdx.x & 63) == 0) cyc[g / 64] = t1 - t0;
}

template <int P> void run(int threads, float* out, long long* cyc, const char* name, int insts) {
  hipLaunchKernelGGL(k<P>, dim3(1), dim3(threads), 0, 0, 1.0f, out, cyc);
  long long h[8];
  if (hipDeviceSynchronize() != hipSuccess) { printf("fail\n"); return; }
  hipMemcpy(h, cyc, sizeof(long long) * (threads / 64), hipMemcpyDeviceToHost);
  double mx = 0;
  for (int w = 0; w < threads / 64; ++w) mx = h[w] > mx ? h[w] : mx;
  printf("%-28s waves=%d  cycles/iter=%7.1f  cycles/inst=%5.2f\n", name, threads / 64, mx / IT, mx / IT / insts);
}
int main() {
  float* out; long long* cyc;
  hipMalloc(&out, 512 * 4); hipMalloc(&cyc, 8 * 8);
  for (int th : {256, 512}) {
    run<0>(th, out, cyc, "8 v_mul_f32", 8);
    run<3>(th, out, cyc, "8 v_mul_f32_dpp", 8);
    run<1>(th, out, cyc, "8 v_dot2c_f32_bf16", 8);
    run<2>(th, out, cyc, "8 v_cvt_pk_bf16_f32", 8);
    run<4>(th, out, cyc, "8 mfma16x16x32bf16", 8);
    run<5>(th, out, cyc, "8x(mfma + 0 mul)", 8);
    run<6>(th, out, cyc, "8x(mfma + 2 mul)", 8);
    run<7>(th, out, cyc, "8x(mfma + 4 mul)", 8);
    run<8>(th, out, cyc, "8x(mfma + 6 mul)", 8);
    run<9>(th, out, cyc, "8x(mfma + 8 mul)", 8);
  }
  return 0;
}
