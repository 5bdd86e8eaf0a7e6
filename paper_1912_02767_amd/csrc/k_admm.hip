// Kernels of the ADMM loop for standard-form SDPs (paper §2, Alg. 1):
//
//   minimize <C, Y>  s.t.  <A_i, Y> = b_i,  Y psd,
//
// in the form (P) with x = Y, q = C, A x = (A_eq(Y), Y), cone {b} x S_+.
// The constraint matrices have disjoint supports, so A_eq^* A_eq acts on
// each A_i as s_i = ||A_i||_F^2 and as zero on their orthogonal complement,
// and the linear system of Alg. 1's first line,
//   ((sigma + rho) I + rho A_eq^* A_eq) x~ = sigma x - q + A^T (rho z - y),
// has the closed-form solution
//   x~ = r / (sigma + rho) + sum_i (<A_i, r> / s_i) (1 / (sigma + rho + rho s_i)
//                                                 - 1 / (sigma + rho)) A_i.
// Every n x n matrix is column-major with leading dimension n; a dense map
// gives, for each position, the constraint whose support holds it (or -1)
// and that constraint's entry there.
#include "admm.h"

namespace psdp {

namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace

// symmetric copy of the lower triangle of C (ldc) into Cs (ld n)
__global__ __launch_bounds__(256) void k_admm_sym(const double* __restrict__ C, int ldc, int n,
                                                  double* __restrict__ Cs) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int i = (int)(e % n), j = (int)(e / n);
  Cs[e] = (i >= j) ? C[i + (size_t)j * ldc] : C[j + (size_t)i * ldc];
}

// map: -1 everywhere, then each entry at (r, c) and (c, r)
__global__ __launch_bounds__(256) void k_admm_map_clear(int* __restrict__ con_of, size_t total) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e < total) con_of[e] = -1;
}

__global__ __launch_bounds__(256) void k_admm_map_fill(const AdmmConstraints c, int n,
                                                       int* __restrict__ con_of,
                                                       double* __restrict__ aval) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= c.nnz) return;
  const int r = c.row[e], k = c.col[e];
  const size_t p1 = r + (size_t)k * n, p2 = k + (size_t)r * n;
  con_of[p1] = c.con[e];
  con_of[p2] = c.con[e];
  aval[p1] = c.val[e];
  aval[p2] = c.val[e];
}

// One wavefront per constraint i: t = <A_i, M> (off-diagonal entries count
// twice), or s = ||A_i||_F^2 when M is null; then, by mode,
//   kDotStore  out[i] = t
//   kDotNorm   out[i] = s
//   kDotSolve  coef[i] = (t / s_i)(1/(sigma + rho + rho s_i) - 1/(sigma + rho)),
//              z~_i = t / (sigma + rho) + coef[i] s_i (= <A_i, x~>), and the
//              multiplier update y_i += rho alpha (z~_i - b_i) (the {b} part
//              of z is b before and after the projection)
__global__ __launch_bounds__(256) void k_admm_cdot(const AdmmConstraints c, const double* M, int n,
                                                   int mode, AdmmParams prm, double* __restrict__ out,
                                                   double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= c.p) return;
  const int e0 = c.off[i], e1 = c.off[i + 1];
  double acc = 0.0;
  for (int e = e0 + lane; e < e1; e += 64) {
    const int r = c.row[e], k = c.col[e];
    const double w = (r == k) ? 1.0 : 2.0;
    const double v = c.val[e];
    acc += w * v * (M ? M[r + (size_t)k * n] : v);
  }
  acc = wave_sum(acc);
  if (lane != 0) return;
  if (mode == kDotStore || mode == kDotNorm) {
    out[i] = acc;
    return;
  }
  const double s = c.s[i], sr = prm.sigma + prm.rho;
  const double coef = (acc / s) * (1.0 / (sr + prm.rho * s) - 1.0 / sr);
  out[i] = coef;
  const double zt = acc / sr + coef * s;
  y[i] += prm.rho * prm.alpha * (zt - c.b[i]);
}

// R = sigma Y - C + rho Z - W + sum_i (rho b_i - y_i) A_i
__global__ __launch_bounds__(256) void k_admm_rhs(int n, AdmmParams prm, const double* __restrict__ Y,
                                                  const double* __restrict__ C,
                                                  const double* __restrict__ Z,
                                                  const double* __restrict__ W,
                                                  const int* __restrict__ con_of,
                                                  const double* __restrict__ aval,
                                                  const double* __restrict__ b,
                                                  const double* __restrict__ y,
                                                  double* __restrict__ R) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)n * n) return;
  double r = prm.sigma * Y[e] - C[e] + prm.rho * Z[e] - W[e];
  const int ci = con_of[e];
  if (ci >= 0) r += (prm.rho * b[ci] - y[ci]) * aval[e];
  R[e] = r;
}

// x~ = R / (sigma + rho) + coef[con] A_con; then the relaxation
//   V = alpha x~ + (1 - alpha) Z + W / rho   (the point projected onto S_+)
//   Y = alpha x~ + (1 - alpha) Y
__global__ __launch_bounds__(256) void k_admm_xt(int n, AdmmParams prm, const double* __restrict__ R,
                                                 const int* __restrict__ con_of,
                                                 const double* __restrict__ aval,
                                                 const double* __restrict__ coef,
                                                 const double* __restrict__ Z,
                                                 const double* __restrict__ W,
                                                 double* __restrict__ V, double* __restrict__ Y) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)n * n) return;
  double xt = R[e] / (prm.sigma + prm.rho);
  const int ci = con_of[e];
  if (ci >= 0) xt += coef[ci] * aval[e];
  V[e] = prm.alpha * xt + (1.0 - prm.alpha) * Z[e] + W[e] / prm.rho;
  Y[e] = prm.alpha * xt + (1.0 - prm.alpha) * Y[e];
}

// W = W + rho (alpha x~ + (1 - alpha) Z_old - Z) = rho (V - Z)
__global__ __launch_bounds__(256) void k_admm_dual(int n, double rho, const double* __restrict__ V,
                                                   const double* __restrict__ Z,
                                                   double* __restrict__ W) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)n * n) return;
  W[e] = rho * (V[e] - Z[e]);
}

// D = P - Q (successive differences for the infeasibility tests)
__global__ __launch_bounds__(256) void k_admm_diff(size_t total, const double* __restrict__ P,
                                                   const double* __restrict__ Q,
                                                   double* __restrict__ D) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e < total) D[e] = P[e] - Q[e];
}

// Per-workgroup partial sums over the n x n positions (kNorms entries):
//   0 ||Y - Z||^2, 1 ||Y||^2, 2 ||Z||^2, 3 ||C + A^*y + W||^2,
//   4 ||A^*y + W||^2, 5 <C, Y>, 6 ||C||^2, 7 ||W||^2
__global__ __launch_bounds__(256) void k_admm_norms(int n, const double* __restrict__ Y,
                                                    const double* __restrict__ Z,
                                                    const double* __restrict__ C,
                                                    const double* __restrict__ W,
                                                    const int* __restrict__ con_of,
                                                    const double* __restrict__ aval,
                                                    const double* __restrict__ y,
                                                    double* __restrict__ part) {
  __shared__ double red[kNorms][4];
  double a[kNorms];
#pragma unroll
  for (int q = 0; q < kNorms; ++q) a[q] = 0.0;
  const size_t total = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const double yv = Y[e], zv = Z[e], cv = C[e], wv = W[e];
    const int ci = con_of[e];
    const double aty = (ci >= 0 ? y[ci] * aval[e] : 0.0) + wv;
    a[0] += (yv - zv) * (yv - zv);
    a[1] += yv * yv;
    a[2] += zv * zv;
    a[3] += (cv + aty) * (cv + aty);
    a[4] += aty * aty;
    a[5] += cv * yv;
    a[6] += cv * cv;
    a[7] += wv * wv;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kNorms; ++q) {
    const double s = wave_sum(a[q]);
    if (lane == 0) red[q][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x < kNorms) {
    const int q = threadIdx.x;
    part[(size_t)blockIdx.x * kNorms + q] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
  }
}

// ------------------------------------------------------------- launch ----
namespace {
inline dim3 grid_for(size_t total) { return dim3((unsigned)((total + 255) / 256)); }
}  // namespace

hipError_t launch_admm_sym(const double* C, int ldc, int n, double* Cs, hipStream_t st) {
  hipLaunchKernelGGL(k_admm_sym, grid_for((size_t)n * n), dim3(256), 0, st, C, ldc, n, Cs);
  return hipGetLastError();
}

hipError_t launch_admm_map(const AdmmConstraints& c, int n, int* con_of, double* aval,
                           hipStream_t st) {
  const size_t total = (size_t)n * n;
  hipLaunchKernelGGL(k_admm_map_clear, grid_for(total), dim3(256), 0, st, con_of, total);
  if (c.nnz > 0)
    hipLaunchKernelGGL(k_admm_map_fill, grid_for((size_t)c.nnz), dim3(256), 0, st, c, n, con_of,
                       aval);
  return hipGetLastError();
}

hipError_t launch_admm_cdot(const AdmmConstraints& c, const double* M, int n, int mode,
                            const AdmmParams& prm, double* out, double* y, hipStream_t st) {
  if (c.p <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_admm_cdot, dim3((c.p + 3) / 4), dim3(256), 0, st, c, M, n, mode, prm, out, y);
  return hipGetLastError();
}

hipError_t launch_admm_rhs(int n, const AdmmParams& prm, const double* Y, const double* C,
                           const double* Z, const double* W, const int* con_of, const double* aval,
                           const double* b, const double* y, double* R, hipStream_t st) {
  hipLaunchKernelGGL(k_admm_rhs, grid_for((size_t)n * n), dim3(256), 0, st, n, prm, Y, C, Z, W,
                     con_of, aval, b, y, R);
  return hipGetLastError();
}

hipError_t launch_admm_xt(int n, const AdmmParams& prm, const double* R, const int* con_of,
                          const double* aval, const double* coef, const double* Z, const double* W,
                          double* V, double* Y, hipStream_t st) {
  hipLaunchKernelGGL(k_admm_xt, grid_for((size_t)n * n), dim3(256), 0, st, n, prm, R, con_of, aval,
                     coef, Z, W, V, Y);
  return hipGetLastError();
}

hipError_t launch_admm_dual(int n, double rho, const double* V, const double* Z, double* W,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_admm_dual, grid_for((size_t)n * n), dim3(256), 0, st, n, rho, V, Z, W);
  return hipGetLastError();
}

hipError_t launch_admm_diff(size_t total, const double* P, const double* Q, double* D,
                            hipStream_t st) {
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_admm_diff, grid_for(total), dim3(256), 0, st, total, P, Q, D);
  return hipGetLastError();
}

hipError_t launch_admm_norms(int n, const double* Y, const double* Z, const double* C,
                             const double* W, const int* con_of, const double* aval,
                             const double* y, double* part, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_admm_norms, dim3(nblk), dim3(256), 0, st, n, Y, Z, C, W, con_of, aval, y,
                     part);
  return hipGetLastError();
}

}  // namespace psdp
