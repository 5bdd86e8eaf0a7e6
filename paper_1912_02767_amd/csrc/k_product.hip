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
// Y = A S on the matrix cores, split over K (rows of S) into slices whose
// partial products are summed afterwards in a fixed order.  Workgroup: four
// waves, 16 rows of Y each, every column of S (up to kPMaxCols, 16 per MFMA
// tile).  A is symmetric, so row i of A is read as column i: each lane loads
// 16 contiguous bytes of one row per step, which feed TPL MFMAs:
//   FP64 v_mfma_f64_16x16x4f64   2 k per lane, slot g = l / 16 <-> k = kb + 2 g + t
//   FP32 v_mfma_f32_16x16x4f32   4 k per lane, slot g <-> k = kb + 4 g + t
//   BF16 v_mfma_f32_16x16x32_bf16 8 k per lane (the instruction's own layout)
// (row l % 16 of the tile); B takes the same k for the same slot, so the
// lane's B values of one step are 16 contiguous bytes of a column of the S
// chunk in LDS (k contiguous, padded).  The A loads of the next chunk are in
// flight while the current chunk is multiplied (a ring of KC / KPL loads).
// D[i][j]: lane -> column l % 16; rows 4 (l / 16) + r for the FP32
// accumulating shapes and l / 16 + 4 r for FP64 (register r = 0..3).
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef float f2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int kPMaxCols = 192;  // 12 column tiles

template <int PREC>
struct PCfg;
template <>
struct PCfg<0> {
  using el = double;
  using acc_t = d4_t;
  using part_t = double;
  static constexpr int KPL = 8, TPL = 2, KC = 32, PAD = 2;
};
template <>
struct PCfg<1> {
  using el = float;
  using acc_t = f4_t;
  using part_t = float;
  static constexpr int KPL = 16, TPL = 4, KC = 64, PAD = 4;
};
template <>
struct PCfg<2> {
  using el = uint16_t;
  using acc_t = f4_t;
  using part_t = float;
  static constexpr int KPL = 32, TPL = 1, KC = 128, PAD = 8;
};

template <int PREC>
__device__ inline void mfma_step(const uint4& av, const uint4& bv, typename PCfg<PREC>::acc_t& acc) {
  if constexpr (PREC == 0) {
    const double2 a2 = __builtin_bit_cast(double2, av), b2 = __builtin_bit_cast(double2, bv);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a2.x, b2.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a2.y, b2.y, acc, 0, 0, 0);
  } else if constexpr (PREC == 1) {
    const f4_t a4 = __builtin_bit_cast(f4_t, av), b4 = __builtin_bit_cast(f4_t, bv);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[0], b4[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[1], b4[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[2], b4[2], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[3], b4[3], acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8_t, av),
                                                  __builtin_bit_cast(bf8_t, bv), acc, 0, 0, 0);
  }
}

// zero the entries of a 16-byte fragment whose k (first = k0) is at or past kend
template <int PREC>
__device__ inline uint4 mask_k(uint4 v, int k0, int kend) {
  using el = typename PCfg<PREC>::el;
  constexpr int E = 16 / (int)sizeof(el);
  el x[E];
  __builtin_memcpy(x, &v, 16);
#pragma unroll
  for (int q = 0; q < E; ++q)
    if (k0 + q >= kend) x[q] = (el)0;
  __builtin_memcpy(&v, x, 16);
  return v;
}

// FULL: the launch's width (known on the host) fills all NCT column tiles
template <int PREC, int NCT, bool FULL>
__global__ __launch_bounds__(256) void k_product_mfma(const void* __restrict__ A, int lda, int n,
                                                      const double* __restrict__ S, int lds,
                                                      int cols_alloc, void* __restrict__ part,
                                                      int ldp, size_t part_stride,
                                                      const int* cols_dev, int cols_host,
                                                      int kslice, const int* stop) {
  if (stop && *stop) return;
  using C = PCfg<PREC>;
  using el = typename C::el;
  using acc_t = typename C::acc_t;
  using part_t = typename C::part_t;
  constexpr int KC = C::KC, LDK = KC + C::PAD, KPL = C::KPL, NL = KC / KPL;
  constexpr int EPL = 16 / (int)sizeof(el);  // elements per 16-byte fragment
  const int cols = min(cols_dev ? *cols_dev : cols_host, NCT * 16);
  const int colsr = (cols + 15) / 16 * 16;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, li = lane & 15, g = lane >> 4;
  const int row0 = blockIdx.x * 64 + wv * 16;
  const int kbeg = blockIdx.y * kslice, kend = min(n, kbeg + kslice);
  __shared__ __align__(16) el sB[NCT * 16 * LDK];
  acc_t acc[NCT];
#pragma unroll
  for (int t = 0; t < NCT; ++t) acc[t] = acc_t{0, 0, 0, 0};
  // this lane's row of A, read as a column; loads past the slice stay inside
  // the row (clamped) and are never used
  const el* arow = (const el*)A + (size_t)(row0 + li) * lda + EPL * g;
  const int kmax = lda - KPL;
  uint4 ring[NL];
#pragma unroll
  for (int s = 0; s < NL; ++s) ring[s] = *(const uint4*)(arow + min(kbeg + s * KPL, kmax));
  // S[kc0 : kc0 + KC, 0 : colsr], two FP64 values per load, is fetched into
  // registers one chunk ahead (in flight while the current chunk is
  // multiplied) and stored to LDS in the product precision (rows past kend
  // are zero)
  constexpr int PFN = (NCT * 16 * (KC / 2) + 255) / 256;
  double2 pf[PFN];
  const int nfe = colsr * (KC / 2);
  auto fetch = [&](int kc0) {
#pragma unroll
    for (int u = 0; u < PFN; ++u) {
      const int e = min(tid + 256 * u, nfe - 1);
      const int j = e / (KC / 2), kk = 2 * (e % (KC / 2));
      pf[u] = *(const double2*)(S + min(kc0 + kk, lda - 2) + (size_t)min(j, cols_alloc - 1) * lds);
    }
  };
  fetch(kbeg);
  for (int kc0 = kbeg; kc0 < kend; kc0 += KC) {
#pragma unroll
    for (int u = 0; u < PFN; ++u) {
      const int e = tid + 256 * u;
      if (e < nfe) {
        const int j = e / (KC / 2), kk = 2 * (e % (KC / 2));
        const int k = kc0 + kk;
        const double v0 = (k < kend) ? pf[u].x : 0.0, v1 = (k + 1 < kend) ? pf[u].y : 0.0;
        el* dst = sB + j * LDK + kk;
        if constexpr (PREC == 0) {
          dst[0] = v0;
          dst[1] = v1;
        } else if constexpr (PREC == 1) {
          *(f2_t*)dst = f2_t{(float)v0, (float)v1};
        } else {
          dst[0] = f32_to_bf16_rne((float)v0);
          dst[1] = f32_to_bf16_rne((float)v1);
        }
      }
    }
    __syncthreads();
    if (kc0 + KC < kend) fetch(kc0 + KC);
    const bool tail = kc0 + KC > kend;  // uniform
#pragma unroll
    for (int s = 0; s < NL; ++s) {
      const int kb = kc0 + s * KPL;
      uint4 av = ring[s];
      ring[s] = *(const uint4*)(arow + min(kb + KC, kmax));  // next chunk, same step
      if (tail) av = mask_k<PREC>(av, kb + EPL * g, kend);
      const el* bcol = sB + li * LDK + s * KPL + EPL * g;
      if constexpr (FULL) {
        // every tile in use: each tile's B fragment read before the first
        // MFMA uses one
        uint4 bv[NCT];
#pragma unroll
        for (int t = 0; t < NCT; ++t) bv[t] = *(const uint4*)(bcol + 16 * t * LDK);
#pragma unroll
        for (int t = 0; t < NCT; ++t) mfma_step<PREC>(av, bv[t], acc[t]);
      } else {
        // the width is read on the device (columns dropped or converged):
        // the tiles past it are skipped
#pragma unroll
        for (int t = 0; t < NCT; ++t)
          if (16 * t < colsr) mfma_step<PREC>(av, *(const uint4*)(bcol + 16 * t * LDK), acc[t]);
      }
    }
    __syncthreads();
  }
  // partial tile -> part[slice]
  part_t* out = (part_t*)part + (size_t)blockIdx.y * part_stride;
#pragma unroll
  for (int t = 0; t < NCT; ++t)
    if (16 * t < cols) {
      const int j = t * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = (PREC == 0) ? row0 + g + 4 * r : row0 + 4 * g + r;
        if (j < cols) out[i + (size_t)j * ldp] = (part_t)acc[t][r];
      }
    }
}

template <typename part_t>
__global__ __launch_bounds__(256) void k_product_reduce(const part_t* __restrict__ part, int nsl,
                                                        size_t part_stride, int ldp, int n,
                                                        const int* cols_dev, int cols_host,
                                                        double* __restrict__ Y, int ldy,
                                                        const int* stop, ProductComb cb) {
  if (stop && *stop) return;
  const int cols = cols_dev ? *cols_dev : cols_host;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int i = (int)(e % (size_t)n), j = (int)(e / (size_t)n);
  if (j >= cols) return;
  // the slices' loads issued 16 at a time before they are added (in slice order)
  const part_t* p = part + i + (size_t)j * ldp;
  double s = 0.0;
  for (int q0 = 0; q0 < nsl; q0 += 16) {
    part_t v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = p[(size_t)min(q0 + u, nsl - 1) * part_stride];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (q0 + u < nsl) s += (double)v[u];
  }
  if (cb.b1) {
    // fused three-term combination: Y = ca (A S) + cb B1 + cc B0
    double v = cb.ca * s + cb.cb * cb.b1[i + (size_t)j * cb.ld];
    if (cb.b0) v += cb.cc * cb.b0[i + (size_t)j * cb.ld];
    s = v;
  }
  Y[i + (size_t)j * ldy] = s;
}

static int g_force_ref = -1;

hipError_t launch_product(const ProductArgs& a, hipStream_t st) {
  if (a.cols_max <= 0 || a.n <= 0) return hipSuccess;
  if (g_force_ref < 0) {
    const char* e = getenv("PSDP_PRODUCT_REF");
    g_force_ref = (e && atoi(e) == 1) ? 1 : 0;
  }
  const bool mfma_ok = a.partial && a.cols_max <= kPMaxCols && a.lda % 8 == 0 &&
                       a.lds % 2 == 0 && a.lds >= a.lda && !g_force_ref;
  if (mfma_ok) {
    const int rt = (a.n + 63) / 64;
    // K slices: up to two resident workgroups per compute unit (512), each
    // slice at least two staging chunks of the precision and a multiple of
    // one (small n: more slices fill the device)
    const int kc = a.prec == 0 ? PCfg<0>::KC : (a.prec == 1 ? PCfg<1>::KC : PCfg<2>::KC);
    int sk = std::max(1, std::min(512 / rt, a.n / (2 * kc)));
    sk = std::min(sk, a.max_slices);
    const int kslice = ((a.n + sk - 1) / sk + kc - 1) / kc * kc;
    sk = (a.n + kslice - 1) / kslice;
    const size_t pstride = (size_t)a.lda * a.cols_max;
    const size_t elem = a.prec == 0 ? 8 : 4;
    if ((size_t)sk * pstride * elem > a.partial_bytes) return hipErrorInvalidValue;
    dim3 grid(rt, sk);
    const int nct = (a.cols_max + 15) / 16;
#define PSDP_LAUNCH_PRODUCT(P, T)                                                              \
  if (!a.cols_dev && (a.cols_max + 15) / 16 == T)                                              \
    hipLaunchKernelGGL((k_product_mfma<P, T, true>), grid, dim3(256), 0, st, a.A, a.lda, a.n,   \
                       a.S, a.lds, a.cols_max, (void*)a.partial, a.lda, pstride, a.cols_dev,    \
                       a.cols_max, kslice, a.stop);                                            \
  else                                                                                         \
    hipLaunchKernelGGL((k_product_mfma<P, T, false>), grid, dim3(256), 0, st, a.A, a.lda, a.n,  \
                       a.S, a.lds, a.cols_max, (void*)a.partial, a.lda, pstride, a.cols_dev,    \
                       a.cols_max, kslice, a.stop)
#define PSDP_LAUNCH_PREC(P)                        \
  if (nct <= 3) PSDP_LAUNCH_PRODUCT(P, 3);         \
  else if (nct <= 6) PSDP_LAUNCH_PRODUCT(P, 6);    \
  else if (nct <= 9) PSDP_LAUNCH_PRODUCT(P, 9);    \
  else PSDP_LAUNCH_PRODUCT(P, 12);
    if (a.prec == 0) {
      PSDP_LAUNCH_PREC(0)
    } else if (a.prec == 1) {
      PSDP_LAUNCH_PREC(1)
    } else {
      PSDP_LAUNCH_PREC(2)
    }
#undef PSDP_LAUNCH_PREC
#undef PSDP_LAUNCH_PRODUCT
    const size_t total = (size_t)a.n * a.cols_max;
    dim3 rg((unsigned)((total + 255) / 256));
    if (a.prec == 0)
      hipLaunchKernelGGL(k_product_reduce<double>, rg, dim3(256), 0, st, (const double*)a.partial,
                         sk, pstride, a.lda, a.n, a.cols_dev, a.cols_max, a.Y, a.ldy, a.stop,
                         a.comb);
    else
      hipLaunchKernelGGL(k_product_reduce<float>, rg, dim3(256), 0, st, (const float*)a.partial,
                         sk, pstride, a.lda, a.n, a.cols_dev, a.cols_max, a.Y, a.ldy, a.stop,
                         a.comb);
    return hipGetLastError();
  }
  hipError_t e = launch_product_ref(a, st);
  if (e != hipSuccess || !a.comb.b1) return e;
  if (a.cols_dev) return hipErrorInvalidValue;  // the combination takes a host column count
  return launch_axpby3(a.n, a.cols_max, a.comb.ca, a.Y, a.ldy, a.comb.cb, a.comb.b1, a.comb.ld,
                       a.comb.cc, a.comb.b0, a.comb.ld, a.Y, a.ldy, st);
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
