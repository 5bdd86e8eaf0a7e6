// Exact projection of many small cones at once (paper §1: full
// eigendecomposition, clip, rebuild), the exact fallback of the batched
// engine.  Cones of uneven order are zero-padded to a common bucket order
// nb: the padded matrix is diag(X_i, 0), whose eigenpairs are those of X_i
// plus zero eigenvalues with eigenvectors outside X_i's coordinates, so the
// projection restricted to the leading n_i x n_i block is Pi(X_i).
#include <algorithm>

#include "batched.h"

namespace psdp {

// A_b = diag(sym(X_i), 0) in an nb x nb slot; flags non-finite input
__global__ void k_eig_pad(const EigCone* cones, double* A, int nb, int* bad) {
  const EigCone c = cones[blockIdx.y];
  double* Ab = A + (size_t)blockIdx.y * nb * nb;
  int nonfin = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nb * nb; e += gridDim.x * blockDim.x) {
    const int i = e % nb, j = e / nb;
    double v = 0.0;
    if (i < c.n && j < c.n) v = (i >= j) ? c.X[i + (size_t)j * c.n] : c.X[j + (size_t)i * c.n];
    nonfin |= !isfinite(v);
    Ab[e] = v;
  }
  if (nonfin) atomicOr(bad + blockIdx.y, 1);
}

// Pi_i = sum over lambda_k > 0 of lambda_k v_k v_k^T on the leading n_i rows
// and columns; 32 x 32 lower tiles, mirrored.
__global__ __launch_bounds__(256) void k_eig_rebuild(const EigCone* cones, const double* A,
                                                     const double* D, int nb) {
  const EigCone c = cones[blockIdx.y];
  const int n = c.n;
  const int nt = (n + 31) / 32;
  int t = blockIdx.x, ti = 0;
  while (t >= ti + 1) { t -= ti + 1; ++ti; }  // lower tile (ti, tj = t)
  const int tj = t;
  if (ti >= nt) return;
  const double* Vb = A + (size_t)blockIdx.y * nb * nb;
  const double* lam = D + (size_t)blockIdx.y * nb;
  __shared__ double sr[32][33], sc[32][33], sl[32];
  __shared__ int s_first;
  // eigenvalues ascending: the positive ones are the last columns
  if (threadIdx.x == 0) {
    int f = nb;
    while (f > 0 && lam[f - 1] > 0.0) --f;
    s_first = f;
  }
  __syncthreads();
  const int first = s_first;
  const int r = threadIdx.x & 31, q = threadIdx.x >> 5;  // 8 row groups of 4 columns
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = first; k0 < nb; k0 += 32) {
    for (int e = threadIdx.x; e < 32 * 32; e += 256) {
      const int rr = e & 31, kk = e >> 5, k = k0 + kk;
      const int gi = ti * 32 + rr, gj = tj * 32 + rr;
      sr[kk][rr] = (k < nb && gi < n) ? Vb[gi + (size_t)k * nb] : 0.0;
      sc[kk][rr] = (k < nb && gj < n) ? Vb[gj + (size_t)k * nb] : 0.0;
    }
    if (threadIdx.x < 32) sl[threadIdx.x] = (k0 + threadIdx.x < nb) ? lam[k0 + threadIdx.x] : 0.0;
    __syncthreads();
    for (int kk = 0; kk < 32; ++kk) {
      const double a = sr[kk][r] * sl[kk];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = fma(a, sc[kk][q * 4 + u], acc[u]);
    }
    __syncthreads();
  }
  const int gi = ti * 32 + r;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int gj = tj * 32 + q * 4 + u;
    if (gi < n && gj < n && gj <= gi) {
      c.Pi[gi + (size_t)gj * n] = acc[u];
      c.Pi[gj + (size_t)gi * n] = acc[u];
    }
  }
}

// Leading eigenpairs (largest first) whose vectors live in X_i's
// coordinates: the positive ones plus max(4, ceil(0.2 p)) guard columns, at
// most m_cap.  out[2 i] = p (positive count), out[2 i + 1] = columns written.
__global__ __launch_bounds__(256) void k_eig_leading(const EigCone* cones, const double* A,
                                                     const double* D, int nb, int* out) {
  const EigCone c = cones[blockIdx.x];
  const int n = c.n;
  const double* Vb = A + (size_t)blockIdx.x * nb * nb;
  const double* lam = D + (size_t)blockIdx.x * nb;
  __shared__ double nrm[256];
  __shared__ int pick[256];
  __shared__ int s_k, s_p;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += Vb[i + (size_t)k * nb] * Vb[i + (size_t)k * nb];
    nrm[k] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int p = 0;
    for (int k = nb - 1; k >= 0; --k)
      if (nrm[k] > 0.5 && lam[k] > 0.0) ++p;
    const int want = min(min(c.m_cap, n), p + max(4, (p * 2 + 9) / 10));
    int got = 0;
    for (int k = nb - 1; k >= 0 && got < want; --k)
      if (nrm[k] > 0.5) pick[got++] = k;
    s_k = (c.V && c.lam) ? got : 0;
    s_p = p;
  }
  __syncthreads();
  const int kk = s_k;
  for (int e = threadIdx.x; e < n * kk; e += blockDim.x) {
    const int i = e % n, j = e / n;
    c.V[i + (size_t)j * n] = Vb[i + (size_t)pick[j] * nb];
  }
  for (int j = threadIdx.x; j < kk; j += blockDim.x) c.lam[j] = lam[pick[j]];
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = s_p;
    out[2 * blockIdx.x + 1] = kk;
  }
}

__global__ void k_zero_ints(int* p, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0;
}

hipError_t launch_eig_pad(const EigCone* cones, int count, double* A, int nb, int* bad,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(256), 0, st, bad, count);
  const int bx = std::min(64, (nb * nb + 255) / 256);
  hipLaunchKernelGGL(k_eig_pad, dim3(bx, count), dim3(256), 0, st, cones, A, nb, bad);
  return hipGetLastError();
}

hipError_t launch_eig_rebuild(const EigCone* cones, int count, const double* A, const double* D,
                              int nb, hipStream_t st) {
  const int nt = (nb + 31) / 32;
  hipLaunchKernelGGL(k_eig_rebuild, dim3(nt * (nt + 1) / 2, count), dim3(256), 0, st, cones, A, D,
                     nb);
  return hipGetLastError();
}

hipError_t launch_eig_leading(const EigCone* cones, int count, const double* A, const double* D,
                              int nb, int* out, hipStream_t st) {
  hipLaunchKernelGGL(k_eig_leading, dim3(count), dim3(256), 0, st, cones, A, D, nb, out);
  return hipGetLastError();
}

}  // namespace psdp
