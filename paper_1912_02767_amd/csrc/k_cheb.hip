// Kernels of the Chebyshev-filtered subspace iteration behind
// PSDP_METHOD_CHEBYSHEV (a polynomial subspace-extraction variant of the
// block eigensolver, paper §1 on polynomial subspace extraction and §5 on
// block Krylov methods):
//
//  * k_axpby3: out = ca Y + cb B1 + cc B0 on n x cols column blocks, the
//    three-term recurrence of the Chebyshev polynomials where the product
//    A B1 is already in Y (the MFMA path folds the same combination into its
//    split-K reduction instead);
//  * k_lanczos_vec: one step of the plain Lanczos recurrence on a single
//    vector (one workgroup), and after the last step the smallest eigenvalue
//    of the tridiagonal by Sturm multisection and the residual norm of its
//    Ritz pair, from which the lower end of the spectrum is estimated
//    (theta_min less twice that residual and 1 %, never below theta_min -
//    beta_k, the Zhou-Saad estimator).
#include "common.h"

namespace psdp {

__global__ __launch_bounds__(256) void k_axpby3(int n, int cols, double ca,
                                                const double* __restrict__ Y, int ldy, double cb,
                                                const double* __restrict__ B1, int ld1, double cc,
                                                const double* __restrict__ B0, int ld0,
                                                double* out, int ldo) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int i = (int)(e % (size_t)n), j = (int)(e / (size_t)n);
  if (j >= cols) return;
  double v = ca * Y[i + (size_t)j * ldy] + cb * B1[i + (size_t)j * ld1];
  if (B0) v += cc * B0[i + (size_t)j * ld0];
  out[i + (size_t)j * ldo] = v;
}

hipError_t launch_axpby3(int n, int cols, double ca, const double* Y, int ldy, double cb,
                         const double* B1, int ld1, double cc, const double* B0, int ld0,
                         double* out, int ldo, hipStream_t st) {
  if (n <= 0 || cols <= 0) return hipSuccess;
  const size_t total = (size_t)n * cols;
  hipLaunchKernelGGL(k_axpby3, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n, cols,
                     ca, Y, ldy, cb, B1, ld1, cc, B0, ld0, out, ldo);
  return hipGetLastError();
}

constexpr int kLzThreads = 1024;
constexpr int kLzReg = 8;  // elements per thread kept in registers (n <= 8192)

__device__ inline double lz_block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < kLzThreads / 64; ++q) s += red[q];  // same order in every thread
  return s;
}

// Sturm count: eigenvalues of the k x k tridiagonal (alpha, beta[1..k-1])
// below x
__device__ inline int sturm_below(const double* al, const double* be, int k, double x) {
  int cnt = 0;
  double q = 1.0;
  for (int i = 0; i < k; ++i) {
    const double b2 = i > 0 ? be[i] * be[i] : 0.0;
    q = (al[i] - x) - (i > 0 ? b2 / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// Smallest eigenvalue of the k x k tridiagonal (A, B[1..k-1]) by
// multisection on one wave: each round the 64 lanes count at 64 interior
// points of [lo, hi] and the bracket shrinks to the 1/65 in which the count
// first reaches 1 (the largest x with no eigenvalue below it is lo).
__device__ inline double tridiag_min_wave(const double* A, const double* B, int k) {
  const int lane = threadIdx.x & 63;
  double lo = A[0], hi = A[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? fabs(B[i]) : 0.0) + (i + 1 < k ? fabs(B[i + 1]) : 0.0);
    lo = fmin(lo, A[i] - r);
    hi = fmax(hi, A[i] + r);
  }
  for (int it = 0; it < 40 && hi - lo > 1e-15 * fmax(fabs(lo), fabs(hi)); ++it) {
    const double w = (hi - lo) / 65.0;
    const double x = lo + w * (lane + 1);
    const unsigned long long above = __ballot(sturm_below(A, B, k, x) >= 1);
    // points at and right of the first lane with a count >= 1 bound from above
    const int first = above ? __builtin_ctzll(above) : 64;
    const double nlo = lo + w * first, nhi = first < 64 ? lo + w * (first + 1) : hi;
    lo = nlo;
    hi = fmax(nhi, nlo);
  }
  return lo;
}

// coef: alpha[0..31], beta[32..64] (beta[32 + j] = beta_j, beta_0 = 0),
// out[0] = lower end, out[1] = theta_min, out[2] = last beta, out[3] = the
// residual norm of the Ritz pair for theta_min.
//   step < 0 : v <- v / ||v||
//   step j   : w <- w - beta_j vprev; alpha_j = w.v; w <- w - alpha_j v;
//              beta_{j+1} = ||w||; w <- w / beta_{j+1}  (the next v)
//   last     : bound from T_{j+1}
// For n <= kLzReg * kLzThreads each thread keeps its elements (i = tid +
// 1024 u) in registers between the passes: one read and one write of each
// vector element per step.
__global__ __launch_bounds__(kLzThreads) void k_lanczos_vec(int n, int step, int last,
                                                            double* __restrict__ w,
                                                            const double* __restrict__ v,
                                                            const double* __restrict__ vprev,
                                                            double* coef, double* out) {
  __shared__ double red[kLzThreads / 64];
  __shared__ double tri[2 * 32];  // the tridiagonal T_{step+1} for the bound
  const int tid = threadIdx.x;
  const bool reg = n <= kLzReg * kLzThreads;
  if (step < 0) {
    double s = 0.0;
    for (int i = tid; i < n; i += kLzThreads) s += w[i] * w[i];
    s = lz_block_sum(s, red);
    const double sc = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    for (int i = tid; i < n; i += kLzThreads) w[i] *= sc;
    return;
  }
  const double bj = step > 0 ? coef[32 + step] : 0.0;
  double al, b;
  if (reg) {
    double x[kLzReg], vv[kLzReg];
#pragma unroll
    for (int u = 0; u < kLzReg; ++u) {
      const int i = tid + kLzThreads * u;
      const bool in = i < n;
      x[u] = in ? w[i] : 0.0;
      vv[u] = in ? v[i] : 0.0;
      const double p = (in && step > 0) ? vprev[i] : 0.0;
      x[u] = fma(-bj, p, x[u]);
    }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kLzReg; ++u) s = fma(x[u], vv[u], s);
    al = lz_block_sum(s, red);
    double s2 = 0.0;
#pragma unroll
    for (int u = 0; u < kLzReg; ++u) {
      x[u] = fma(-al, vv[u], x[u]);
      s2 = fma(x[u], x[u], s2);
    }
    b = sqrt(lz_block_sum(s2, red));
    // breakdown (an invariant subspace): the next vector is zero, so later
    // steps add zero rows whose eigenvalue 0 only loosens the bound
    const double sc = b > 1e-300 ? 1.0 / b : 0.0;
#pragma unroll
    for (int u = 0; u < kLzReg; ++u) {
      const int i = tid + kLzThreads * u;
      if (i < n) w[i] = x[u] * sc;
    }
  } else {
    double s = 0.0;
    for (int i = tid; i < n; i += kLzThreads) {
      const double x = w[i] - (step > 0 ? bj * vprev[i] : 0.0);
      w[i] = x;
      s += x * v[i];
    }
    al = lz_block_sum(s, red);
    double s2 = 0.0;
    for (int i = tid; i < n; i += kLzThreads) {
      const double x = w[i] - al * v[i];
      w[i] = x;
      s2 += x * x;
    }
    b = sqrt(lz_block_sum(s2, red));
    const double sc = b > 1e-300 ? 1.0 / b : 0.0;
    for (int i = tid; i < n; i += kLzThreads) w[i] *= sc;
  }
  if (tid == 0) {
    coef[step] = al;
    coef[32 + step + 1] = b;
  }
  if (last) {
    // T_{step+1} into LDS: this step's coefficients from registers (every
    // thread holds them), the earlier ones written by earlier launches
    const int k = step + 1;
    if (tid < k) {
      tri[tid] = tid == step ? al : coef[tid];
      tri[32 + tid] = tid == 0 ? 0.0 : coef[32 + tid];
    }
    __syncthreads();
    if (tid < 64) {
      const double th = tridiag_min_wave(tri, tri + 32, k);
      if (tid == 0) {
        // residual norm of the Ritz pair for theta_min: beta_k |z_k|, z the
        // unit eigenvector of T_k (its last component by the three-term
        // recurrence of T_k's rows from z_1 = 1, rescaled as it grows)
        const double* A = tri;
        const double* B = tri + 32;
        double y0 = 0.0, y1 = 1.0, s2 = 1.0;
        bool ok = true;
        for (int i = 0; i + 1 < k; ++i) {
          const double bn = B[i + 1];
          if (!(fabs(bn) > 0.0)) {
            ok = false;
            break;
          }
          const double y2 = ((th - A[i]) * y1 - B[i] * y0) / bn;
          y0 = y1;
          y1 = y2;
          s2 += y2 * y2;
          if (s2 > 1e200) {
            y0 *= 1e-100;
            y1 *= 1e-100;
            s2 *= 1e-200;
          }
        }
        const double zl = fabs(y1) / sqrt(s2);
        const double rho = (ok && zl <= 1.0) ? b * zl : b;
        out[1] = th;
        out[2] = b;
        out[3] = rho;
        // twice the residual below theta_min (an eigenvalue lies within rho
        // of it) and 1 % of its size; a lower end slightly inside the
        // spectrum only lets the filter grow the lowest eigenvalues by a
        // small factor, far below the wanted ones
        out[0] = th - fmin(b, 2.0 * rho + 1e-2 * fabs(th));
      }
    }
  }
}

hipError_t launch_lanczos_vec(int n, int step, int last, double* w, const double* v,
                              const double* vprev, double* coef, double* out, hipStream_t st) {
  if (step > 30) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lanczos_vec, dim3(1), dim3(kLzThreads), 0, st, n, step, last, w, v, vprev,
                     coef, out);
  return hipGetLastError();
}

}  // namespace psdp
