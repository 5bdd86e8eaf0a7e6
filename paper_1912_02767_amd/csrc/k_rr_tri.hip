// Rayleigh-Ritz step (paper §5, Alg. 2) for one small projected matrix
// H = S^T A S (S orthonormal), one workgroup, FP64 throughout:
//   1. Householder tridiagonalization H = Q T Q^T in LDS (packed lower
//      triangle; Golub & Van Loan §8.3.1), reflectors kept in place
//   2. the largest mk eigenvalues of T by multisection on Sturm counts
//      (every thread evaluates one LDL^T inertia count per round), plus the
//      count of positive eigenvalues of H
//   3. eigenvectors of T by inverse iteration (two steps) with modified
//      Gram-Schmidt inside clusters of close eigenvalues
//   4. back-transformation Z = Q Y and Rayleigh quotients for the values
// The outputs are the coefficients C (Np x mk) of the kept Ritz vectors in
// the basis S and their Ritz values in descending order.
#include <algorithm>

#include "common.h"

namespace psdp {

constexpr int kTriThreads = 512;

__device__ inline int tri_row2(int e) {
  int r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= e) ++r;
  while (r * (r + 1) / 2 > e) --r;
  return r;
}
// packed lower triangle, row-major: (i, j), j <= i
__device__ inline int pl(int i, int j) { return i * (i + 1) / 2 + j; }
// symmetric access in the packed lower triangle
__device__ inline int ps(int i, int j) { return i >= j ? pl(i, j) : pl(j, i); }

__device__ inline double wg_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x / 64;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)blockDim.x / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

// number of eigenvalues of T (d, e2 = e^2) below x, LDL^T inertia with a
// floor on the pivots (pivmin)
__device__ inline int sturm_count(const double* d, const double* e2, int N, double x,
                                  double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += (q < 0.0);
  for (int i = 1; i < N; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
  }
  return cnt;
}

// deterministic start vector entries for inverse iteration
__device__ inline double start_entry(int i, int j) {
  uint32_t h = (uint32_t)i * 0x9E3779B1u ^ ((uint32_t)j * 0x85EBCA77u + 0x1912u);
  h ^= h >> 15; h *= 0x2C1B3C6Du; h ^= h >> 12; h *= 0x297A2D39u; h ^= h >> 15;
  return 1.0 + 0.5 * ((double)(h & 0xFFFFFF) / 16777216.0 - 0.5);
}

__global__ __launch_bounds__(kTriThreads) void k_rr_tri(RRArgs a) {
  extern __shared__ double lds[];
  __shared__ double red[kTriThreads / 64];
  __shared__ double s_lo[kMaxM], s_hi[kMaxM];
  __shared__ int s_npos;
  __shared__ double s_tnorm, s_pivmin;
  State* st = a.st;
  if (st->stop) return;
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int N = st->Np;
  const int mk = min(a.mtarget, N);
  // ---- LDS layout
  double* Hp = lds;                              // N(N+1)/2
  double* d = Hp + N * (N + 1) / 2;              // N
  double* e = d + N;                             // N   (sub-diagonal)
  double* e2 = e + N;                            // N
  double* tau = e2 + N;                          // N
  double* pv = tau + N;                          // N   (p, then w)
  double* part = pv + N;                         // 8 N (segment partial sums)
  double* Y = part + 8 * N;                      // N x mk eigenvectors (col-major)
  double* cnt_buf = Y + (size_t)N * mk;          // nt counts / dot products

  if (tid == 0) st->t_phase[0] = wall_clock64();
  // load the symmetric part of K into the packed lower triangle
  for (int x = tid; x < N * (N + 1) / 2; x += nt) {
    int i = tri_row2(x), j = x - i * (i + 1) / 2;
    Hp[x] = 0.5 * (a.K[i + (size_t)j * a.ldk] + a.K[j + (size_t)i * a.ldk]);
  }
  __syncthreads();

  // ---- 1. tridiagonalization (lower): H_k = I - tau v v^T, v(0) = 1 at row k+1
  for (int k = 0; k + 2 < N; ++k) {
    const int m = N - k - 1;  // length of x = H[k+1:N, k]
    double part_sq = 0.0;
    for (int i = k + 2 + tid; i < N; i += nt) {
      double x = Hp[pl(i, k)];
      part_sq += x * x;
    }
    const double xnorm2 = wg_sum(part_sq, red);
    const double alpha = Hp[pl(k + 1, k)];
    double t = 0.0, beta = alpha, scale = 0.0;
    if (xnorm2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    // v into column k (v(0) = 1 stored explicitly)
    for (int i = k + 1 + tid; i < N; i += nt)
      Hp[pl(i, k)] = (i == k + 1) ? 1.0 : Hp[pl(i, k)] * scale;
    if (tid == 0) { tau[k] = t; e[k] = beta; }
    __syncthreads();
    if (t != 0.0) {
      // p = t * A22 v, A22 = H[k+1:, k+1:]; rows split into 4 segments of j
      const int seg = (m + 3) / 4;
      for (int x = tid; x < 4 * m; x += nt) {
        int r = x % m, sgi = x / m;
        int i = k + 1 + r;
        int j0 = k + 1 + sgi * seg, j1 = min(N, j0 + seg);
        double s = 0.0;
        for (int j = j0; j < j1; ++j) s += Hp[ps(i, j)] * Hp[pl(j, k)];
        part[sgi * N + i] = s;
      }
      __syncthreads();
      double dot_part = 0.0;
      for (int i = k + 1 + tid; i < N; i += nt) {
        double p = t * (part[i] + part[N + i] + part[2 * N + i] + part[3 * N + i]);
        pv[i] = p;
        dot_part += p * Hp[pl(i, k)];
      }
      const double pdotv = wg_sum(dot_part, red);
      const double al = -0.5 * t * pdotv;
      for (int i = k + 1 + tid; i < N; i += nt) pv[i] += al * Hp[pl(i, k)];
      __syncthreads();
      // A22 -= v w^T + w v^T (lower part)
      const int cnt = m * (m + 1) / 2;
      for (int x = tid; x < cnt; x += nt) {
        int r = tri_row2(x), c = x - r * (r + 1) / 2;
        int i = k + 1 + r, j = k + 1 + c;
        double vi = Hp[pl(i, k)], vj = Hp[pl(j, k)];
        Hp[pl(i, j)] -= vi * pv[j] + pv[i] * vj;
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < N; i += nt) d[i] = Hp[pl(i, i)];
  if (tid == 0) st->t_phase[1] = wall_clock64();
  if (tid == 0 && N >= 2) { e[N - 2] = Hp[pl(N - 1, N - 2)]; tau[N - 2] = 0.0; }
  __syncthreads();
  for (int i = tid; i + 1 < N; i += nt) e2[i] = e[i] * e[i];
  // norm and pivot floor
  if (tid == 0) {
    double tn = 0.0, emax2 = 0.0;
    for (int i = 0; i < N; ++i) {
      double r = fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < N ? fabs(e[i]) : 0.0);
      tn = fmax(tn, r);
      if (i + 1 < N) emax2 = fmax(emax2, e[i] * e[i]);
    }
    s_tnorm = tn;
    s_pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  }
  __syncthreads();
  const double tnorm = s_tnorm, pivmin = s_pivmin;

  // ---- 2. multisection for the top mk eigenvalues (+ count of positives)
  {
    double gl = 0.0, gu = 0.0;
    for (int i = 0; i < N; ++i) {
      double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < N ? fabs(e[i]) : 0.0);
      gl = (i == 0) ? d[i] - r : fmin(gl, d[i] - r);
      gu = (i == 0) ? d[i] + r : fmax(gu, d[i] + r);
    }
    const double pad = 2.2e-16 * tnorm * 4.0 * N + 2.0 * pivmin;
    gl -= pad;
    gu += pad;
    for (int j = tid; j < mk; j += nt) { s_lo[j] = gl; s_hi[j] = gu; }
    if (tid == 0) s_npos = N - sturm_count(d, e2, N, 0.0, pivmin);
    __syncthreads();
    const int per = max(1, nt / max(mk, 1));  // threads per eigenvalue
    const int j_me = tid / per, s_me = tid % per;
    int* cnts = (int*)cnt_buf;
    for (int round = 0; round < 40; ++round) {
      // all intervals narrow enough?
      // the shifts only need to be close enough for inverse iteration; the
      // values themselves come from Rayleigh quotients afterwards
      bool done = true;
      for (int j = 0; j < mk; ++j) {
        double w = s_hi[j] - s_lo[j];
        double tolj = 1e-12 * tnorm + 4.0 * 2.2e-16 * fmax(fabs(s_lo[j]), fabs(s_hi[j])) + 4.0 * pivmin;
        if (w > tolj) { done = false; break; }
      }
      if (done) break;
      if (j_me < mk) {
        double lo = s_lo[j_me], hi = s_hi[j_me];
        double x = lo + (hi - lo) * (double)(s_me + 1) / (double)(per + 1);
        cnts[tid] = sturm_count(d, e2, N, x, pivmin);
      }
      __syncthreads();
      if (tid < mk) {
        const int j = tid;
        const int target = N - 1 - j;  // ascending index of the j-th largest
        double lo = s_lo[j], hi = s_hi[j];
        double nlo = lo, nhi = hi;
        // points x_s (s = 0..per-1); count(x) = #eigenvalues < x
        for (int s2 = 0; s2 < per; ++s2) {
          double x = lo + (hi - lo) * (double)(s2 + 1) / (double)(per + 1);
          int c = cnts[j * per + s2];
          if (c <= target) nlo = x;                 // eigenvalue >= x
          else { nhi = x; break; }                  // eigenvalue < x
        }
        s_lo[j] = nlo;
        s_hi[j] = nhi;
      }
      __syncthreads();
    }
  }

  if (tid == 0) st->t_phase[2] = wall_clock64();
  // ---- 3. inverse iteration on T, one thread per eigenvector: Gaussian
  // elimination with partial pivoting of the tridiagonal T - sigma I (row
  // interchanges add a second super-diagonal), zero pivots replaced by
  // eps ||T||.  Factors live in global scratch, interleaved by eigenvector.
  double* fdl = a.scratch;                        // N x mk each: element i of j at i*mk + j
  double* fdd = fdl + (size_t)N * mk;
  double* fdu = fdd + (size_t)N * mk;
  double* fdu2 = fdu + (size_t)N * mk;
  double* fpiv = fdu2 + (size_t)N * mk;
  const double pfloor = fmax(2.2e-16 * tnorm, 1e-300);
  if (tid < mk) {
    const int j = tid;
    const double sigma = 0.5 * (s_lo[j] + s_hi[j]);
#define F(arr, i) arr[(size_t)(i) * mk + j]
    for (int i = 0; i < N; ++i) {
      F(fdd, i) = d[i] - sigma;
      F(fdl, i) = (i + 1 < N) ? e[i] : 0.0;
      F(fdu, i) = (i + 1 < N) ? e[i] : 0.0;
      F(fdu2, i) = 0.0;
    }
    for (int i = 0; i + 1 < N; ++i) {
      double di = F(fdd, i), li = F(fdl, i);
      if (fabs(di) >= fabs(li)) {
        if (di == 0.0) { di = pfloor; F(fdd, i) = di; }
        double fact = li / di;
        F(fdl, i) = fact;
        F(fdd, i + 1) -= fact * F(fdu, i);
        F(fpiv, i) = 0.0;
      } else {
        double fact = di / li;
        F(fdd, i) = li;
        F(fdl, i) = fact;
        double tmp = F(fdu, i);
        F(fdu, i) = F(fdd, i + 1);
        F(fdd, i + 1) = tmp - fact * F(fdd, i + 1);
        if (i + 2 < N) {
          F(fdu2, i) = F(fdu, i + 1);
          F(fdu, i + 1) = -fact * F(fdu, i + 1);
        }
        F(fpiv, i) = 1.0;
      }
    }
    if (F(fdd, N - 1) == 0.0) F(fdd, N - 1) = pfloor;
    for (int i = 0; i < N; ++i) {
      if (fabs(F(fdd, i)) < pfloor) F(fdd, i) = copysign(pfloor, F(fdd, i));
      Y[i + (size_t)j * N] = start_entry(i, j);
    }
#undef F
  }
  __syncthreads();
  const double ortol = 1e-3 * tnorm;
  for (int itn = 0; itn < 2; ++itn) {
    if (tid < mk) {
      const int j = tid;
      double* y = Y + (size_t)j * N;
#define F(arr, i) arr[(size_t)(i) * mk + j]
      // forward: apply the row interchanges and multipliers
      for (int i = 0; i + 1 < N; ++i) {
        if (F(fpiv, i) != 0.0) {
          double t0 = y[i];
          y[i] = y[i + 1];
          y[i + 1] = t0 - F(fdl, i) * y[i];
        } else {
          y[i + 1] -= F(fdl, i) * y[i];
        }
      }
      // backward with the three diagonals of U
      y[N - 1] /= F(fdd, N - 1);
      if (N >= 2) y[N - 2] = (y[N - 2] - F(fdu, N - 2) * y[N - 1]) / F(fdd, N - 2);
      for (int i = N - 3; i >= 0; --i)
        y[i] = (y[i] - F(fdu, i) * y[i + 1] - F(fdu2, i) * y[i + 2]) / F(fdd, i);
#undef F
      double nn = 0.0, mx = 0.0;
      for (int i = 0; i < N; ++i) mx = fmax(mx, fabs(y[i]));
      double sc = mx > 0.0 ? 1.0 / mx : 1.0;
      for (int i = 0; i < N; ++i) { y[i] *= sc; nn += y[i] * y[i]; }
      double inv = 1.0 / sqrt(nn);
      for (int i = 0; i < N; ++i) y[i] *= inv;
    }
    __syncthreads();
    // modified Gram-Schmidt inside clusters of close eigenvalues
    for (int j = 1; j < mk; ++j) {
      double mid_j = 0.5 * (s_lo[j] + s_hi[j]);
      double mid_p = 0.5 * (s_lo[j - 1] + s_hi[j - 1]);
      if (mid_p - mid_j > ortol) continue;   // uniform: not in a cluster with j-1
      int c0 = j - 1;
      while (c0 > 0 && 0.5 * (s_lo[c0 - 1] + s_hi[c0 - 1]) - 0.5 * (s_lo[c0] + s_hi[c0]) <= ortol) --c0;
      double* yj = Y + (size_t)j * N;
      for (int i0 = c0; i0 < j; ++i0) {
        const double* yi = Y + (size_t)i0 * N;
        double dp = 0.0;
        for (int r = tid; r < N; r += nt) dp += yi[r] * yj[r];
        dp = wg_sum(dp, red);
        for (int r = tid; r < N; r += nt) yj[r] -= dp * yi[r];
        __syncthreads();
      }
      double nn = 0.0;
      for (int r = tid; r < N; r += nt) nn += yj[r] * yj[r];
      nn = wg_sum(nn, red);
      double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
      for (int r = tid; r < N; r += nt) yj[r] *= inv;
      __syncthreads();
    }
  }
  if (tid == 0) st->t_phase[3] = wall_clock64();
  // Rayleigh quotients y^T T y (eigenvalues of H to second order)
  double* theta = cnt_buf;  // mk doubles (the counts are no longer needed)
  if (tid < mk) {
    const double* y = Y + (size_t)tid * N;
    double rq = 0.0;
    for (int i = 0; i < N; ++i) {
      double ty = d[i] * y[i];
      if (i > 0) ty += e[i - 1] * y[i - 1];
      if (i + 1 < N) ty += e[i] * y[i + 1];
      rq += y[i] * ty;
    }
    theta[tid] = rq;
  }
  __syncthreads();

  // ---- 4. back-transformation Z = H_0 H_1 ... H_{N-3} Y
  for (int k = N - 3; k >= 0; --k) {
    const double t = tau[k];
    if (t == 0.0) continue;  // uniform
    const int m = N - k - 1;
    // w_j = v^T Y[k+1:, j], rows split into 8 segments
    const int seg = (m + 7) / 8;
    for (int x = tid; x < 8 * mk; x += nt) {
      int j = x % mk, sgi = x / mk;
      int r0 = k + 1 + sgi * seg, r1 = min(N, r0 + seg);
      double s = 0.0;
      for (int r = r0; r < r1; ++r) s += Hp[pl(r, k)] * Y[r + (size_t)j * N];
      part[sgi * mk + j] = s;
    }
    __syncthreads();
    for (int x = tid; x < m * mk; x += nt) {
      int r = k + 1 + x % m, j = x / m;
      double wj = part[j] + part[mk + j] + part[2 * mk + j] + part[3 * mk + j] +
                  part[4 * mk + j] + part[5 * mk + j] + part[6 * mk + j] + part[7 * mk + j];
      Y[r + (size_t)j * N] -= t * Hp[pl(r, k)] * wj;
    }
    __syncthreads();
  }
  if (tid == 0) st->t_phase[4] = wall_clock64();
  // ---- outputs: C = Z (N x mk), Ritz values descending
  for (int x = tid; x < N * mk; x += nt) {
    int i = x % N, j = x / N;
    a.C[i + (size_t)j * a.ldc] = Y[x];
  }
  for (int j = tid; j < mk; j += nt) st->theta[j] = theta[j];
  if (tid == 0) {
    st->npos_rr = s_npos;
    st->mk = mk;
    st->expand_req = (s_npos > a.mtarget) ? 1 : 0;
    st->jacobi_rounds = 0;
    if (a.count_iter) st->iter += 1;
  }
}

static int g_tri_lds_limit = 56 * 1024;

hipError_t launch_rr_tri(const RRArgs& a, int Np_host, int mk_host, hipStream_t st) {
  size_t N = Np_host, mk = std::min(mk_host, Np_host);
  size_t need = N * (N + 1) / 2 + 13 * N + N * mk + kTriThreads / 2 + 16;
  size_t bytes = sizeof(double) * need;
  if (bytes > (size_t)g_tri_lds_limit) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rr_tri, dim3(1), dim3(kTriThreads), bytes, st, a);
  return hipGetLastError();
}

hipError_t rr_tri_init() {
  int dev = 0, lim = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
  if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    lim = 64 * 1024;
  int dyn = lim - 2 * 1024;  // static LDS of k_rr_tri is below 2 KB
  if (dyn > 0) {
    g_tri_lds_limit = dyn;
    (void)hipFuncSetAttribute((const void*)k_rr_tri, hipFuncAttributeMaxDynamicSharedMemorySize,
                              dyn);
  }
  (void)hipGetLastError();
  return hipSuccess;
}

}  // namespace psdp
