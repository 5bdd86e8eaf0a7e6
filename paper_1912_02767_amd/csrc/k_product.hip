// Block product Y = A S (paper §5.1: the O(n^2 m) term of one LOBPCG
// iteration), A symmetric n x n in FP64, FP32 or BF16, S an orthonormal
// n x k trial basis in FP64, Y in FP64.
//
// Reference tiling (this file): each workgroup computes 64 rows x 16 columns
// of Y; A is read along its columns (coalesced), S through LDS.  The low-
// precision variants round S to the product precision and accumulate in
// FP32, which is what the matrix cores do.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "common.h"

namespace psdp {

hipError_t launch_product_ref(const ProductArgs& a, hipStream_t st);

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

// ----------------------------------------------------------- MFMA path --
// Y = A S on the matrix cores, split over K (rows of S) into `splitk`
// slices whose partial products are summed afterwards in a fixed order.
// Workgroup: 4 waves, 64 rows of Y (16 per wave) and every column of S
// (up to kMaxN, 16 per MFMA tile); S is staged through LDS in the product
// precision, k-contiguous per column; A is read straight from HBM.
//   FP64: v_mfma_f64_16x16x4f64   A[i][k]: lane -> (l % 16, l / 16)
//   FP32: v_mfma_f32_16x16x4f32   same operand layout, FP32 accumulate
//   BF16: v_mfma_f32_16x16x32_bf16 lane holds 8 consecutive k: (l % 16,
//         8 (l / 16) + 0..7); A is symmetric, so A[i][k] is read as A[k][i]
//         (k contiguous in memory)
// D[i][j]: lane -> column l % 16; rows 4 (l / 16) + r for the FP32
// accumulating shapes and l / 16 + 4 r for FP64 (register r = 0..3).
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int kMT = 12;  // column tiles of 16 (up to 192 columns)

template <int PREC>
struct MfmaCfg;
template <>
struct MfmaCfg<0> {
  using acc_t = d4_t;
  using part_t = double;
  static constexpr int KC = 32;   // k per staged chunk
  static constexpr int KS = 4;    // k per MFMA
};
template <>
struct MfmaCfg<1> {
  using acc_t = f4_t;
  using part_t = float;
  static constexpr int KC = 32;
  static constexpr int KS = 4;
};
template <>
struct MfmaCfg<2> {
  using acc_t = f4_t;
  using part_t = float;
  static constexpr int KC = 64;
  static constexpr int KS = 32;
};

template <int PREC>
__global__ __launch_bounds__(256) void k_product_mfma(const void* __restrict__ A, int lda, int n,
                                                      const double* __restrict__ S, int lds,
                                                      void* __restrict__ part, int ldp,
                                                      size_t part_stride, const int* cols_dev,
                                                      int cols_host, int kslice,
                                                      const int* stop) {
  if (stop && *stop) return;
  using C = MfmaCfg<PREC>;
  using acc_t = typename C::acc_t;
  using part_t = typename C::part_t;
  constexpr int KC = C::KC;
  const int cols = cols_dev ? *cols_dev : cols_host;
  const int nct = (cols + 15) / 16;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row0 = blockIdx.x * 64 + wv * 16;
  const int kbeg = blockIdx.y * kslice, kend = min(n, kbeg + kslice);
  // S chunk in LDS: [column j][k], k contiguous, padded leading dim
  constexpr int LDK = (PREC == 2) ? KC + 8 : KC + 1;
  __shared__ __align__(16) unsigned char sraw[kMT * 16 * LDK * (PREC == 0 ? 8 : (PREC == 1 ? 4 : 2))];
  acc_t acc[kMT];
#pragma unroll
  for (int t = 0; t < kMT; ++t) acc[t] = acc_t{0, 0, 0, 0};
  const int li = lane & 15, lk = lane >> 4;
  for (int k0 = kbeg; k0 < kend; k0 += KC) {
    // stage S[k0 : k0 + KC, 0 : 16 nct]
    for (int e = threadIdx.x; e < KC * 16 * nct; e += 256) {
      const int kk = e % KC, j = e / KC;
      const int k = k0 + kk;
      const double v = (k < kend && j < cols) ? S[k + (size_t)j * lds] : 0.0;
      if constexpr (PREC == 0) ((double*)sraw)[j * LDK + kk] = v;
      else if constexpr (PREC == 1) ((float*)sraw)[j * LDK + kk] = (float)v;
      else ((uint16_t*)sraw)[j * LDK + kk] = f32_to_bf16_rne((float)v);
    }
    __syncthreads();
    const int ksteps = (min(KC, kend - k0) + C::KS - 1) / C::KS;
    for (int ks = 0; ks < ksteps; ++ks) {
      const int kb = k0 + ks * C::KS;
      if constexpr (PREC == 0) {
        const int k = kb + lk;
        const double av = (k < kend) ? ((const double*)A)[(row0 + li) + (size_t)k * lda] : 0.0;
        const double* sb = (const double*)sraw;
#pragma unroll
        for (int t = 0; t < kMT; ++t)
          if (t < nct) {
            const double bv = sb[(t * 16 + li) * LDK + ks * 4 + lk];
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
          }
      } else if constexpr (PREC == 1) {
        const int k = kb + lk;
        const float av = (k < kend) ? ((const float*)A)[(row0 + li) + (size_t)k * lda] : 0.0f;
        const float* sb = (const float*)sraw;
#pragma unroll
        for (int t = 0; t < kMT; ++t)
          if (t < nct) {
            const float bv = sb[(t * 16 + li) * LDK + ks * 4 + lk];
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0, 0, 0);
          }
      } else {
        // A[row0 + li][kb + 8 lk .. +7] read as A[k][i] (symmetric), 16 bytes
        const int kq = kb + 8 * lk;
        bf8_t av;
        if (kq + 8 <= kend) {
          av = *(const bf8_t*)((const uint16_t*)A + kq + (size_t)(row0 + li) * lda);
        } else {
          uint16_t tmp[8];
          for (int q = 0; q < 8; ++q)
            tmp[q] = (kq + q < kend) ? ((const uint16_t*)A)[kq + q + (size_t)(row0 + li) * lda] : 0;
          av = __builtin_bit_cast(bf8_t, *(const uint4*)tmp);
        }
        const uint16_t* sb = (const uint16_t*)sraw;
#pragma unroll
        for (int t = 0; t < kMT; ++t)
          if (t < nct) {
            const bf8_t bv = *(const bf8_t*)(sb + (t * 16 + li) * LDK + ks * 32 + 8 * lk);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[t], 0, 0, 0);
          }
      }
    }
    __syncthreads();
  }
  // partial tile -> part[slice]
  part_t* out = (part_t*)part + (size_t)blockIdx.y * part_stride;
#pragma unroll
  for (int t = 0; t < kMT; ++t)
    if (t < nct) {
      const int j = t * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // FP64 16x16x4: register r of lane l holds row l/16 + 4r; the FP32
        // accumulating shapes hold row 4(l/16) + r (checked on gfx950)
        const int i = (PREC == 0) ? row0 + lk + 4 * r : row0 + 4 * lk + r;
        if (j < cols) out[i + (size_t)j * ldp] = (part_t)acc[t][r];
      }
    }
}

template <typename part_t>
__global__ __launch_bounds__(256) void k_product_reduce(const part_t* __restrict__ part, int nsl,
                                                        size_t part_stride, int ldp, int n,
                                                        const int* cols_dev, int cols_host,
                                                        double* __restrict__ Y, int ldy,
                                                        const int* stop) {
  if (stop && *stop) return;
  const int cols = cols_dev ? *cols_dev : cols_host;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int i = (int)(e % (size_t)n), j = (int)(e / (size_t)n);
  if (j >= cols) return;
  double s = 0.0;
  for (int q = 0; q < nsl; ++q) s += (double)part[(size_t)q * part_stride + i + (size_t)j * ldp];
  Y[i + (size_t)j * ldy] = s;
}

static int g_force_ref = -1;

hipError_t launch_product(const ProductArgs& a, hipStream_t st) {
  if (a.cols_max <= 0 || a.n <= 0) return hipSuccess;
  if (g_force_ref < 0) {
    const char* e = getenv("PSDP_PRODUCT_REF");
    g_force_ref = (e && atoi(e) == 1) ? 1 : 0;
  }
  const bool mfma_ok = a.partial && a.cols_max <= kMT * 16 && a.lda % 64 == 0 && !g_force_ref;
  if (mfma_ok) {
    const int rt = (a.n + 63) / 64;
    // K slices: enough workgroups to cover the chip, at least 256 k each
    int sk = std::max(1, std::min((512 + rt - 1) / rt, a.n / 256));
    sk = std::min(sk, a.max_slices);
    const int kslice = ((a.n + sk - 1) / sk + 63) / 64 * 64;
    sk = (a.n + kslice - 1) / kslice;
    const size_t pstride = (size_t)a.lda * a.cols_max;
    const size_t elem = a.prec == 0 ? 8 : 4;
    if ((size_t)sk * pstride * elem > a.partial_bytes) return hipErrorInvalidValue;
    dim3 grid(rt, sk);
    if (a.prec == 0)
      hipLaunchKernelGGL(k_product_mfma<0>, grid, dim3(256), 0, st, a.A, a.lda, a.n, a.S, a.lds,
                         (void*)a.partial, a.lda, pstride, a.cols_dev, a.cols_max, kslice, a.stop);
    else if (a.prec == 1)
      hipLaunchKernelGGL(k_product_mfma<1>, grid, dim3(256), 0, st, a.A, a.lda, a.n, a.S, a.lds,
                         (void*)a.partial, a.lda, pstride, a.cols_dev, a.cols_max, kslice, a.stop);
    else
      hipLaunchKernelGGL(k_product_mfma<2>, grid, dim3(256), 0, st, a.A, a.lda, a.n, a.S, a.lds,
                         (void*)a.partial, a.lda, pstride, a.cols_dev, a.cols_max, kslice, a.stop);
    const size_t total = (size_t)a.n * a.cols_max;
    dim3 rg((unsigned)((total + 255) / 256));
    if (a.prec == 0)
      hipLaunchKernelGGL(k_product_reduce<double>, rg, dim3(256), 0, st, (const double*)a.partial,
                         sk, pstride, a.lda, a.n, a.cols_dev, a.cols_max, a.Y, a.ldy, a.stop);
    else
      hipLaunchKernelGGL(k_product_reduce<float>, rg, dim3(256), 0, st, (const float*)a.partial,
                         sk, pstride, a.lda, a.n, a.cols_dev, a.cols_max, a.Y, a.ldy, a.stop);
    return hipGetLastError();
  }
  return launch_product_ref(a, st);
}

hipError_t launch_product_ref(const ProductArgs& a, hipStream_t st) {
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
