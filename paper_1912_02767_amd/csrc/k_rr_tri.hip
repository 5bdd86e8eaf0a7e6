// Rayleigh-Ritz kernels for the single-cone pipeline (bodies in rr_body.h
// and rr_fast.h).
#include "rr_body.h"
#include "rr_fast.h"

namespace psdp {

template <bool FULL>
__global__ __launch_bounds__(kTriThreads) void k_rr_tri(RRArgs a) {
  extern __shared__ double lds[];
  __shared__ double s_lo[kMaxM], s_hi[kMaxM];
  __shared__ int s_npos;
  __shared__ double s_tnorm, s_pivmin;
  if (a.st->stop) return;
  RRShared sh{s_lo, s_hi, &s_npos, &s_tnorm, &s_pivmin};
  rr_tri_body<FULL>(a, lds, sh);
}

constexpr int kFastThreads = 512;
constexpr int kFastThreadsS = 256;  // trial bases up to 80: 16 x 16 grid, 5 x 5 per thread

__global__ __launch_bounds__(kFastThreads) void k_rr_fast(RRArgs a) {
  extern __shared__ double lds[];
  __shared__ double s_lo[kMaxM], s_hi[kMaxM];
  __shared__ int s_npos;
  __shared__ double s_tnorm, s_pivmin;
  if (a.st->stop) return;
  RRShared sh{s_lo, s_hi, &s_npos, &s_tnorm, &s_pivmin};
  // 32 x 16 thread grid, N <= 144; the reflectors go to a.scratch
  rr_fast_body<5, 9, kFastThreads, true>(a, lds, sh);
}

// the same for N <= 80: fewer waves, shorter chains per step
__global__ __launch_bounds__(kFastThreadsS) void k_rr_fast_s(RRArgs a) {
  extern __shared__ double lds[];
  __shared__ double s_lo[kMaxM], s_hi[kMaxM];
  __shared__ int s_npos;
  __shared__ double s_tnorm, s_pivmin;
  if (a.st->stop) return;
  RRShared sh{s_lo, s_hi, &s_npos, &s_tnorm, &s_pivmin};
  rr_fast_body<5, 5, kFastThreadsS, true>(a, lds, sh);
}

// Back-transformation of the Ritz vectors of the tridiagonal matrix (C, in
// place) by the reflectors k_rr_fast left in a.scratch (packed lower
// triangle, then tau): one workgroup per 16 columns of C.
constexpr int kBackThreads = kWYDenseThreads;
constexpr int kBackCols = 16;

__host__ __device__ inline int rr_back_nbc(int N) { return N <= 80 ? 5 : 9; }

__host__ __device__ inline size_t rr_back_lds_doubles(int N) {
  const size_t n = N, ldy = (N & 1) ? n : n + 1;
  const size_t vb = 16 * (size_t)(16 * rr_back_nbc(N) + 1);
  return n * (n + 1) / 2 + n + ldy * kBackCols + kWYBlock * kWYBlock + kWYLd * kBackCols + vb;
}

template <int NBC>
__global__ __launch_bounds__(kBackThreads) void k_rr_back(RRArgs a) {
  double* lds = lds_base();
  State* st = a.st;
  if (st->stop) return;
  const int N = st->Np, mk = min(a.mtarget, N);
  const int j0 = blockIdx.x * kBackCols;
  if (j0 >= mk) return;
  const int nc = min(kBackCols, mk - j0);
  const int ldy = (N & 1) ? N : N + 1;
  const size_t n2 = (size_t)N * (N + 1) / 2;
  double* P = lds;
  double* tau = P + n2;
  double* Y = tau + N;
  double* Tb = Y + (size_t)ldy * kBackCols;
  double* Wb = Tb + kWYBlock * kWYBlock;
  double* Vb = Wb + kWYLd * kBackCols;
  // P and tau, then the 16 columns of C: eight loads in flight per thread
  const size_t np = n2 + N;
  for (size_t x0 = 0; x0 < np; x0 += 8 * kBackThreads) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = a.scratch[min(x0 + threadIdx.x + (size_t)u * kBackThreads, np - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const size_t x = x0 + threadIdx.x + (size_t)u * kBackThreads;
      if (x < np) P[x] = v[u];
    }
  }
  for (int x0 = 0; x0 < ldy * kBackCols; x0 += 8 * kBackThreads) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int x = x0 + threadIdx.x + u * kBackThreads;
      const int i = min(x % ldy, N - 1), j = min(x / ldy, nc - 1);
      v[u] = a.C[i + (size_t)(j0 + j) * a.ldc];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int x = x0 + threadIdx.x + u * kBackThreads;
      const int i = x % ldy, j = x / ldy;
      if (x < ldy * kBackCols) Y[x] = (i < N && j < nc) ? v[u] : 0.0;
    }
  }
  __syncthreads();
  wy_back_dense<NBC>(N, P, tau, Y, ldy, nc, Tb, Wb, Vb,
                     (blockIdx.x == 0 && a.trace) ? st : nullptr);
  for (int x = threadIdx.x; x < N * nc; x += kBackThreads) {
    const int i = x % N, j = x / N;
    a.C[i + (size_t)(j0 + j) * a.ldc] = Y[i + (size_t)j * ldy];
  }
}

static int g_tri_lds_limit = 56 * 1024;

hipError_t launch_rr_fast(const RRArgs& a_in, int Np_host, int mk_host, hipStream_t st) {
  RRArgs a = a_in;
  if (Np_host > 144 || std::min(mk_host, Np_host) > kMaxM) return hipErrorInvalidValue;
  const bool small = Np_host <= 80;
  const size_t doubles =
      small ? rr_fast_lds_doubles(Np_host, std::min(mk_host, Np_host), kFastThreadsS, 5, 5)
            : rr_fast_lds_doubles(Np_host, std::min(mk_host, Np_host), kFastThreads, 5, 9);
  if (doubles * 8 > (size_t)g_tri_lds_limit) return hipErrorInvalidValue;
  if (rr_back_lds_doubles(Np_host) * 8 > (size_t)g_tri_lds_limit) return hipErrorInvalidValue;
  a.lds_cap = doubles;
  if (small)
    hipLaunchKernelGGL(k_rr_fast_s, dim3(1), dim3(kFastThreadsS), doubles * 8, st, a);
  else
    hipLaunchKernelGGL(k_rr_fast, dim3(1), dim3(kFastThreads), doubles * 8, st, a);
  return hipGetLastError();
}

hipError_t launch_rr_back(const RRArgs& a, int Np_host, int mk_host, hipStream_t st) {
  const size_t back = rr_back_lds_doubles(Np_host);
  if (Np_host > 144 || back * 8 > (size_t)g_tri_lds_limit) return hipErrorInvalidValue;
  const int mk = std::min(mk_host, Np_host);
  if (mk <= 0) return hipSuccess;
  if (rr_back_nbc(Np_host) == 5)
    hipLaunchKernelGGL(k_rr_back<5>, dim3((mk + kBackCols - 1) / kBackCols), dim3(kBackThreads),
                       back * 8, st, a);
  else
    hipLaunchKernelGGL(k_rr_back<9>, dim3((mk + kBackCols - 1) / kBackCols), dim3(kBackThreads),
                       back * 8, st, a);
  return hipGetLastError();
}

hipError_t launch_rr_tri(const RRArgs& a_in, int Np_host, int mk_host, hipStream_t st) {
  RRArgs a = a_in;
  const size_t N = Np_host, mk = std::min(mk_host, Np_host);
  const bool full = Np_host <= kFullMaxN;
  const size_t hsz = full ? N * N : N * (N + 1) / 2;
  const size_t base = hsz + 14 * N + (N + 1) * mk + (kTriThreads + 2) / 2 + 2;
  const size_t cap = (size_t)g_tri_lds_limit / 8;
  if (base > cap) return hipErrorInvalidValue;
  const size_t want = base + 3 * N * mk;  // U factors in LDS as well
  const size_t doubles = want <= cap ? want : base;
  a.lds_cap = doubles;
  if (full)
    hipLaunchKernelGGL(k_rr_tri<true>, dim3(1), dim3(kTriThreads), doubles * 8, st, a);
  else
    hipLaunchKernelGGL(k_rr_tri<false>, dim3(1), dim3(kTriThreads), doubles * 8, st, a);
  return hipGetLastError();
}

hipError_t rr_tri_init() {
  int dev = 0, lim = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
  if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    lim = 64 * 1024;
  const int dyn = lim - 2 * 1024;  // static LDS of k_rr_tri is below 2 KB
  if (dyn > 0) {
    g_tri_lds_limit = dyn;
    (void)hipFuncSetAttribute((const void*)k_rr_tri<true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void*)k_rr_tri<false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void*)k_rr_fast, hipFuncAttributeMaxDynamicSharedMemorySize,
                              dyn);
    (void)hipFuncSetAttribute((const void*)k_rr_fast_s,
                              hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void*)k_rr_back<5>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void*)k_rr_back<9>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
  }
  (void)hipGetLastError();
  return hipSuccess;
}

}  // namespace psdp
