// Block product Y = A S (paper §5.1: the O(n^2 m) term of one LOBPCG
// iteration), A symmetric n x n in FP64, FP32 or BF16, S an orthonormal
// n x k trial basis in FP64, Y in FP64.
//
// Reference tiling (this file): each workgroup computes 64 rows x 16 columns
// of Y; A is read along its columns (coalesced), S through LDS.  The low-
// precision variants round S to the product precision and accumulate in
// FP32, which is what the matrix cores do.
#include <type_traits>

#include "common.h"

namespace psdp {

constexpr int kPR = 64;   // rows per workgroup
constexpr int kPQ = 16;   // columns per workgroup
constexpr int kPK = 32;   // k chunk

template <int PREC>
__device__ inline double load_a(const void* A, size_t idx) {
  if (PREC == 0) return ((const double*)A)[idx];
  if (PREC == 1) return (double)((const float*)A)[idx];
  return (double)bf16_to_f32(((const uint16_t*)A)[idx]);
}

template <int PREC>
__device__ inline double round_s(double v) {
  if (PREC == 0) return v;
  if (PREC == 1) return (double)(float)v;
  return (double)bf16_to_f32(f32_to_bf16_rne((float)v));
}

template <int PREC>
__global__ __launch_bounds__(256) void k_product_ref(const void* __restrict__ A, int lda, int n,
                                                     const double* __restrict__ S, int lds,
                                                     double* __restrict__ Y, int ldy,
                                                     const int* cols_dev, int cols_host,
                                                     const int* stop) {
  if (stop && *stop) return;
  using acc_t = typename std::conditional<PREC == 0, double, float>::type;
  __shared__ acc_t sA[kPK][kPR + 1];
  __shared__ acc_t sS[kPK][kPQ + 1];
  const int cols = cols_dev ? *cols_dev : cols_host;
  const int row0 = blockIdx.x * kPR, col0 = blockIdx.y * kPQ;
  if (col0 >= cols) return;
  const int r = threadIdx.x % kPR, cg = threadIdx.x / kPR;
  acc_t acc[4] = {0, 0, 0, 0};
  for (int k0 = 0; k0 < n; k0 += kPK) {
    for (int e = threadIdx.x; e < kPK * kPR; e += 256) {
      int rr = e % kPR, kc = e / kPR;
      int row = row0 + rr, k = k0 + kc;
      sA[kc][rr] = (row < n && k < n) ? (acc_t)load_a<PREC>(A, row + (size_t)k * lda) : (acc_t)0;
    }
    for (int e = threadIdx.x; e < kPK * kPQ; e += 256) {
      int kc = e % kPK, c = e / kPK;
      int k = k0 + kc, j = col0 + c;
      sS[kc][c] = (k < n && j < cols) ? (acc_t)round_s<PREC>(S[k + (size_t)j * lds]) : (acc_t)0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kc = 0; kc < kPK; ++kc) {
      acc_t a = sA[kc][r];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = fma(a, sS[kc][cg * 4 + c], acc[c]);
    }
    __syncthreads();
  }
  int row = row0 + r;
  if (row < n) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int j = col0 + cg * 4 + c;
      if (j < cols) Y[row + (size_t)j * ldy] = (double)acc[c];
    }
  }
}

hipError_t launch_product(const ProductArgs& a, hipStream_t st) {
  if (a.cols_max <= 0 || a.n <= 0) return hipSuccess;
  dim3 grid((a.n + kPR - 1) / kPR, (a.cols_max + kPQ - 1) / kPQ);
  const int* stop = a.stop;
  if (a.prec == 1)
    hipLaunchKernelGGL(k_product_ref<1>, grid, dim3(256), 0, st, a.A, a.lda, a.n, a.S, a.lds, a.Y,
                       a.ldy, a.cols_dev, a.cols_max, stop);
  else if (a.prec == 2)
    hipLaunchKernelGGL(k_product_ref<2>, grid, dim3(256), 0, st, a.A, a.lda, a.n, a.S, a.lds, a.Y,
                       a.ldy, a.cols_dev, a.cols_max, stop);
  else
    hipLaunchKernelGGL(k_product_ref<0>, grid, dim3(256), 0, st, a.A, a.lda, a.n, a.S, a.lds, a.Y,
                       a.ldy, a.cols_dev, a.cols_max, stop);
  return hipGetLastError();
}

}  // namespace psdp
