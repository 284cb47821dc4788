// In-bounds probe of the lane layout of the FP64 / FP32 16x16x4 MFMA
// builtins: one wave of 64 lanes, inputs of 64 values, outputs of 256.
#include <hip/hip_runtime.h>
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// A[i][0] = i + 1, A[i][1] = 1; B[0][j] = 1000, B[1][j] = j + 1 (k >= 2: 0)
// so D[i][j] = 1000 (i + 1) + (j + 1) names its row and column
__device__ inline double aval(int l) { return l / 16 == 0 ? (double)(l % 16 + 1) : (l / 16 == 1 ? 1.0 : 0.0); }
__device__ inline double bval(int l) { return l / 16 == 0 ? 1000.0 : (l / 16 == 1 ? (double)(l % 16 + 1) : 0.0); }
__global__ void probe64(double* out) {
  const int l = threadIdx.x;
  double a = aval(l);  // A[l%16][l/16]
  double b = bval(l);  // B[l/16][l%16]
  d4 acc = {0, 0, 0, 0};
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  for (int i = 0; i < 4; ++i) out[l * 4 + i] = acc[i];
}
__global__ void probe32(float* out) {
  const int l = threadIdx.x;
  float a = (float)aval(l);
  float b = (float)bval(l);
  f4 acc = {0, 0, 0, 0};
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  for (int i = 0; i < 4; ++i) out[l * 4 + i] = acc[i];
}
extern "C" int run_probe(double* h64, float* h32) {
  double* d64; float* d32;
  if (hipMalloc(&d64, 256 * 8) != hipSuccess) return 1;
  if (hipMalloc(&d32, 256 * 4) != hipSuccess) return 1;
  hipLaunchKernelGGL(probe64, dim3(1), dim3(64), 0, 0, d64);
  hipLaunchKernelGGL(probe32, dim3(1), dim3(64), 0, 0, d32);
  if (hipMemcpy(h64, d64, 256 * 8, hipMemcpyDeviceToHost) != hipSuccess) return 2;
  if (hipMemcpy(h32, d32, 256 * 4, hipMemcpyDeviceToHost) != hipSuccess) return 2;
  if (hipFree(d64) != hipSuccess || hipFree(d32) != hipSuccess) return 3;
  return 0;
}
