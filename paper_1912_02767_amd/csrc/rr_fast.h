// Device bodies of the Rayleigh-Ritz step on the N x N projected matrix
// (N <= 144 in one workgroup):
//   1. Householder tridiagonalization with the matrix in registers on an
//      RG x 16 thread grid (tridiag_reg), two barriers per column; the
//      reflectors, unit entry included, in a packed column-major lower
//      triangle (column j starts at cb(j) + j, cb(j) = j N - j (j + 1) / 2);
//   2. multisection with Sturm counts for the mk largest eigenvalues: one
//      shared round over the Gershgorin interval, then per-eigenvalue shifts,
//      to a few ulps of ||T||;
//   3. eigenvectors of T by the twisted factorization of T - sigma I (top-down
//      and bottom-up pivots, twist at the smallest |gamma|), one thread per
//      vector; classical Gram-Schmidt, twice, inside clusters (with inverse
//      iteration from a fixed start vector when a vector collapses onto its
//      predecessors, as for exactly repeated eigenvalues); Rayleigh quotients;
//   4. back-transformation by blocks of 16 reflectors in compact WY form
//      (wy_back), in the same workgroup (batched engine) or in a separate
//      kernel over column tiles of the vectors (single cone).
// Included by the single-cone kernels and the batched persistent kernel;
// needs blockDim.x >= N.
#pragma once
#include "rr_body.h"

namespace psdp {

constexpr int kWYBlock = 16;
constexpr int kWYLd = 17;  // leading dimension of W in LDS (odd: no bank conflicts)

__host__ __device__ inline int pk_cb(int j, int N) { return j * N - (j * (j + 1)) / 2; }

// dynamic LDS doubles of rr_fast_body for order N and mk vectors
// Tb + Wb region: the block reflector factor and V^T Y, or the three
// factor diagonals of one inverse-iteration solve
__host__ __device__ inline size_t rr_fast_tbw(int N, int mk) {
  const size_t wy = (size_t)kWYBlock * kWYBlock + (size_t)kWYLd * mk;
  return wy > 3 * (size_t)N ? wy : 3 * (size_t)N;
}

// The Y region also hosts the six LP-vectors of phase 1 and the Sturm
// counts of phase 2.
// LP: padded length of the phase-1 vectors (rows covered by the thread grid)
__host__ __device__ inline size_t rr_fast_lp(int nthreads, int nbr, int nbc) {
  const size_t a = (size_t)(nthreads / 16) * nbr, b = 16 * (size_t)nbc;
  return a > b ? a : b;
}

__host__ __device__ inline size_t rr_fast_yspace(int N, int mk, int nthreads, size_t lp) {
  const size_t n = N;
  const size_t ldy = (N & 1) ? n : n + 1;
  size_t y = ldy * (size_t)mk;
  if (y < 6 * lp) y = 6 * lp;
  if (y < (size_t)nthreads) y = nthreads;
  return y;
}

__host__ __device__ inline size_t rr_fast_lds_doubles(int N, int mk, int nthreads, int nbr,
                                                      int nbc) {
  const size_t n = N, nw = nthreads / 64;
  return n * (n + 1) / 2 + 5 * n + rr_fast_yspace(N, mk, nthreads, rr_fast_lp(nthreads, nbr, nbc)) +
         rr_fast_tbw(N, mk) + nw + 4;
}

// Twisted-factorization eigenvector of the tridiagonal T (d, e, e2 = e^2)
// for the shift sigma, written to y (length N, stride 1, not normalized);
// pivots of magnitude below pfloor are replaced by -pfloor.  The loops load
// four entries ahead of the pivot recurrences.
__device__ inline double tw_piv(double dd, double ee2, double prev, double pfloor) {
  double q = dd - fast_div(ee2, prev);
  return (fabs(q) < pfloor) ? -pfloor : q;
}

__device__ inline void twisted_vector(const double* d, const double* e, const double* e2, int N,
                                      double sigma, double pfloor, double* y) {
  if (N == 1) { y[0] = 1.0; return; }
  // top-down pivots D+ into y
  double dp = d[0] - sigma;
  if (fabs(dp) < pfloor) dp = -pfloor;
  y[0] = dp;
  int i = 1;
  for (; i + 3 < N; i += 4) {
    const double d0 = d[i] - sigma, d1 = d[i + 1] - sigma, d2 = d[i + 2] - sigma, d3 = d[i + 3] - sigma;
    const double f0 = e2[i - 1], f1 = e2[i], f2 = e2[i + 1], f3 = e2[i + 2];
    dp = tw_piv(d0, f0, dp, pfloor); y[i] = dp;
    dp = tw_piv(d1, f1, dp, pfloor); y[i + 1] = dp;
    dp = tw_piv(d2, f2, dp, pfloor); y[i + 2] = dp;
    dp = tw_piv(d3, f3, dp, pfloor); y[i + 3] = dp;
  }
  for (; i < N; ++i) { dp = tw_piv(d[i] - sigma, e2[i - 1], dp, pfloor); y[i] = dp; }
  // bottom-up pivots D-, twist index at the smallest |gamma_i|,
  // gamma_i = D+_i + D-_i - (d_i - sigma)
  double dm = d[N - 1] - sigma;
  if (fabs(dm) < pfloor) dm = -pfloor;
  int r = N - 1;
  double gbest = fabs(y[N - 1]);
  i = N - 2;
  for (; i - 3 >= 0; i -= 4) {
    const double d0 = d[i] - sigma, d1 = d[i - 1] - sigma, d2 = d[i - 2] - sigma, d3 = d[i - 3] - sigma;
    const double f0 = e2[i], f1 = e2[i - 1], f2 = e2[i - 2], f3 = e2[i - 3];
    const double y0 = y[i], y1 = y[i - 1], y2 = y[i - 2], y3 = y[i - 3];
    double g;
    dm = tw_piv(d0, f0, dm, pfloor); g = fabs(y0 + dm - d0); if (g < gbest) { gbest = g; r = i; }
    dm = tw_piv(d1, f1, dm, pfloor); g = fabs(y1 + dm - d1); if (g < gbest) { gbest = g; r = i - 1; }
    dm = tw_piv(d2, f2, dm, pfloor); g = fabs(y2 + dm - d2); if (g < gbest) { gbest = g; r = i - 2; }
    dm = tw_piv(d3, f3, dm, pfloor); g = fabs(y3 + dm - d3); if (g < gbest) { gbest = g; r = i - 3; }
  }
  for (; i >= 0; --i) {
    const double di = d[i] - sigma;
    dm = tw_piv(di, e2[i], dm, pfloor);
    const double g = fabs(y[i] + dm - di);
    if (g < gbest) { gbest = g; r = i; }
  }
  // D- again below the twist (y[i], i > r, is no longer needed as D+)
  dm = d[N - 1] - sigma;
  if (fabs(dm) < pfloor) dm = -pfloor;
  if (r < N - 1) y[N - 1] = dm;
  for (i = N - 2; i > r; --i) {
    dm = tw_piv(d[i] - sigma, e2[i], dm, pfloor);
    y[i] = dm;
  }
  // the vector: z_r = 1, upward through L (D+), downward through U (D-)
  double z = 1.0;
  for (i = r - 1; i >= 0; --i) {
    z = -fast_div(e[i], y[i]) * z;
    y[i] = z;
  }
  z = 1.0;
  for (i = r + 1; i < N; ++i) {
    z = -fast_div(e[i - 1], y[i]) * z;
    y[i] = z;
  }
  y[r] = 1.0;
}

// The twisted factorization split over two threads of a vector: the
// top-down pivots D+ (into y) and the bottom-up pivots D- (into w) run at
// once; then both threads find the twist and build the two halves of the
// vector (the same values as twisted_vector).
__device__ inline void twisted_top(const double* d, const double* e2, int N, double sigma,
                                   double pfloor, double* y) {
  double dp = d[0] - sigma;
  if (fabs(dp) < pfloor) dp = -pfloor;
  y[0] = dp;
  int i = 1;
  for (; i + 3 < N; i += 4) {
    const double d0 = d[i] - sigma, d1 = d[i + 1] - sigma, d2 = d[i + 2] - sigma, d3 = d[i + 3] - sigma;
    const double f0 = e2[i - 1], f1 = e2[i], f2 = e2[i + 1], f3 = e2[i + 2];
    dp = tw_piv(d0, f0, dp, pfloor); y[i] = dp;
    dp = tw_piv(d1, f1, dp, pfloor); y[i + 1] = dp;
    dp = tw_piv(d2, f2, dp, pfloor); y[i + 2] = dp;
    dp = tw_piv(d3, f3, dp, pfloor); y[i + 3] = dp;
  }
  for (; i < N; ++i) { dp = tw_piv(d[i] - sigma, e2[i - 1], dp, pfloor); y[i] = dp; }
}

__device__ inline void twisted_bottom(const double* d, const double* e2, int N, double sigma,
                                      double pfloor, double* w) {
  double dm = d[N - 1] - sigma;
  if (fabs(dm) < pfloor) dm = -pfloor;
  w[N - 1] = dm;
  int i = N - 2;
  for (; i - 3 >= 0; i -= 4) {
    const double d0 = d[i] - sigma, d1 = d[i - 1] - sigma, d2 = d[i - 2] - sigma, d3 = d[i - 3] - sigma;
    const double f0 = e2[i], f1 = e2[i - 1], f2 = e2[i - 2], f3 = e2[i - 3];
    dm = tw_piv(d0, f0, dm, pfloor); w[i] = dm;
    dm = tw_piv(d1, f1, dm, pfloor); w[i - 1] = dm;
    dm = tw_piv(d2, f2, dm, pfloor); w[i - 2] = dm;
    dm = tw_piv(d3, f3, dm, pfloor); w[i - 3] = dm;
  }
  for (; i >= 0; --i) { dm = tw_piv(d[i] - sigma, e2[i], dm, pfloor); w[i] = dm; }
}

// twist index: the smallest |gamma_i| = |D+_i + D-_i - (d_i - sigma)|, the
// last row first and the larger index kept on ties
__device__ inline int twisted_index(const double* d, int N, double sigma, const double* y,
                                   const double* w) {
  int r = N - 1;
  double gbest = fabs(y[N - 1]);
  for (int i = N - 2; i >= 0; --i) {
    const double di = d[i] - sigma;
    const double g = fabs(y[i] + w[i] - di);
    if (g < gbest) { gbest = g; r = i; }
  }
  return r;
}

// z_r = 1; upward through L (D+ in y), written over y
__device__ inline void twisted_up(const double* e, int r, double* y) {
  double z = 1.0;
  for (int i = r - 1; i >= 0; --i) {
    z = -fast_div(e[i], y[i]) * z;
    y[i] = z;
  }
  y[r] = 1.0;
}

// downward through U (D- in w), into y below the twist
__device__ inline void twisted_down(const double* e, int N, int r, const double* w, double* y) {
  double z = 1.0;
  for (int i = r + 1; i < N; ++i) {
    z = -fast_div(e[i - 1], w[i]) * z;
    y[i] = z;
  }
}

// a / b with the reciprocal estimate refined by one Newton step (relative
// error about 1e-14: the counts below are those of a matrix whose squared
// off-diagonal entries are perturbed by that much)
__device__ inline double div_n1(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  return a * r;
}

// sturm_count with div_n1: the multisection is bound by instruction
// throughput (every thread runs one count), so the shorter division pays
__device__ inline int sturm_count_n1(const double* d, const double* e2, int N, double x,
                                     double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += (q < 0.0);
  for (int i = 1; i < N; ++i) {
    q = d[i] - x - div_n1(e2[i - 1], q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
  }
  return cnt;
}

// Sturm count of T - x I by the three-term recurrence of its leading
// principal minors, p_{i+1} = (d_i - x) p_i - e_{i-1}^2 p_{i-1} with p_0 = 1,
// p_1 = d_0 - x: the number of sign changes along p_0 .. p_N is the number of
// eigenvalues below x, a zero minor taking the sign opposite to its
// predecessor (the limit of the ratio form's -pivmin).  ds, e2s and xs are d,
// e^2 and x scaled by a power of two that brings ||T|| below one, so |p|
// grows at most threefold per step; every 8 steps the pair (p_i, p_{i+1}) is
// rescaled by a power of two.  The same backward error as the ratio form
// (relative perturbations of d_i - x and e_i^2 of a few ulps), with one
// dependent FMA per step in place of a division chain.  Returns -1 when the
// pair fell below 2^-900, became zero or non-finite; the caller then counts
// with the ratio form.
__device__ inline void sturm_poly_step(double dsi, double e2m, double xs, double& a, double& b,
                                       bool& sb, int& cnt) {
  const double c = fma(dsi - xs, b, -e2m * a);
  const bool sc = (c < 0.0) | ((c == 0.0) & !sb);  // no short circuit: no branches
  cnt += (sc != sb) ? 1 : 0;
  sb = sc;
  a = b;
  b = c;
}

__device__ inline int sturm_count_poly(const double* ds, const double* e2s, int N, double xs) {
  double a = 1.0, b = ds[0] - xs;
  bool sb = !(b > 0.0);  // p_0 = 1 > 0: a zero p_1 counts as negative
  int cnt = sb ? 1 : 0, emin = 0;
  // blocks of 8 steps; the next block's entries are loaded during the current one
  double dn[8], en[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    dn[u] = ds[min(1 + u, N - 1)];
    en[u] = e2s[min(u, N - 1)];
  }
  int i = 1;
  for (; i + 8 <= N; i += 8) {
    double dc[8], ec[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      dc[u] = dn[u];
      ec[u] = en[u];
      dn[u] = ds[min(i + 8 + u, N - 1)];
      en[u] = e2s[min(i + 7 + u, N - 1)];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) sturm_poly_step(dc[u], ec[u], xs, a, b, sb, cnt);
    const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(a), fabs(b)));
    emin = min(emin, ex);
    a = __builtin_amdgcn_ldexp(a, -ex);
    b = __builtin_amdgcn_ldexp(b, -ex);
  }
  // the last partial block from the values already prefetched (rows i .. N - 1)
#pragma unroll
  for (int u = 0; u < 8; ++u)
    if (i + u < N) sturm_poly_step(dn[u], en[u], xs, a, b, sb, cnt);
  const double m = fmax(fabs(a), fabs(b));
  emin = min(emin, __builtin_amdgcn_frexp_exp(m));
  const bool bad = !(m > 0.0) || !(m < 1e300) || emin < -900;
  return bad ? -1 : cnt;
}

// The count for the shift x: the scaled recurrence, or the ratio form when
// it reports underflow (d, e2 unscaled; sh the scaling exponent).
__device__ inline int sturm_count_fast(const double* ds, const double* e2s, const double* d,
                                       const double* e2, int N, double x, int sh, double pivmin) {
  const int c = sturm_count_poly(ds, e2s, N, __builtin_amdgcn_ldexp(x, -sh));
  return c >= 0 ? c : sturm_count_n1(d, e2, N, x, pivmin);
}

// An eigenvalue bracket [lo, hi] is still open above a few ulps of ||T||.
__device__ inline bool bracket_open(double lo, double hi, double tnorm, double pivmin) {
  return hi - lo > 4.4e-16 * (tnorm + fmax(fabs(lo), fabs(hi))) + 4.0 * pivmin;
}

// Reflector scalars of a column with leading entry alpha and squared norm
// xn of the entries below it (LAPACK dlarfg convention, beta = -sign(alpha) |x|).
__device__ inline void reflector(double alpha, double xn, double& t, double& beta, double& scale) {
  t = 0.0;
  beta = alpha;
  scale = 0.0;
  if (xn > 0.0) {
    beta = -copysign(sqrt(alpha * alpha + xn), alpha);
    t = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
}

// Sum over each row of 16 lanes (every lane of the row gets the sum).
__device__ inline double row16_sum(double v) {
  v += dpp_d<0xB1>(v);   // lane ^ 1
  v += dpp_d<0x4E>(v);   // lane ^ 2
  v += dpp_d<0x141>(v);  // other quad of each 8
  v += dpp_d<0x140>(v);  // other 8 of each 16
  return v;
}

// lane ^ 16 (within 32) and lane ^ 32 partners' values added
__device__ inline double add_x16_x32(double v) {
  int2 x = __builtin_bit_cast(int2, v);
  x.x = __builtin_amdgcn_ds_swizzle(x.x, 0x401F);
  x.y = __builtin_amdgcn_ds_swizzle(x.y, 0x401F);
  v += __builtin_bit_cast(double, x);
  return v + __shfl_xor(v, 32, 64);
}

template <int NB>
__device__ inline double sel(const double (&row)[NB], int q) {
  double v = row[0];
#pragma unroll
  for (int t = 1; t < NB; ++t) v = (t == q) ? row[t] : v;
  return v;
}

// Householder tridiagonalization with the matrix in registers.  The NT
// threads form an RG x 16 grid (RG = NT / 16 row groups, 16 column groups):
// thread (r, c) = (tid >> 4, tid & 15) holds A(r NBR + li, c + 16 lj) for
// li < NBR, lj < NBC (both triangles): contiguous row blocks, so the 16
// threads of one row group are 16 lanes of one wave and each wave owns 4 NBR
// consecutive rows.  LDS vectors (LP entries, zero-padded) hold the current
// column x (rows <= k zero), w (rows <= k zero), A x and column k + 1 before
// the update.  Per step k:
//   (a) every thread loads x on its columns and forms |x|^2 over the 16 lanes
//       of its row group (DPP); waves that own a row below k form their
//       rows of A x (summed over the row group) and their part of x^T A x;
//       the owners of column k + 1 publish it; every thread forms the
//       reflector scalars (dlarfg convention);
//   (b) with v = scale x + g e_{k+1} (g = 1 - scale x_{k+1}), A v and v^T A v
//       follow from A x, x^T A x and column k + 1; one thread per trailing row
//       forms w = t A v - (t^2 / 2)(v^T A v) v, stores w, keeps the reflector
//       in P, and forms column k + 1 after the update (the next column
//       buffer) and its diagonal entry;
//   (c) waves that own a row below k apply A -= v w^T + w v^T to their block,
//       v formed again from the x of (a) in the registers (entries in
//       finished rows or columns see zero v and w and stay put).
// Two barriers per step.  On return: d, e (N - 1 entries), tau, and the
// reflectors (unit entry at row k + 1 included) in the packed column-major
// lower triangle P.
template <int NBR, int NBC, int NT>
__device__ inline void tridiag_reg(const RRArgs& a, int N, double* P, double* d, double* e,
                                   double* tau, double* buf, double* red) {
  constexpr int RG = NT / 16, nw = NT / 64;
  constexpr int LP = (RG * NBR > 16 * NBC) ? RG * NBR : 16 * NBC;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = tid >> 4, c = tid & 15;
  const int row0 = r * NBR;
  const int wave_last_row = (4 * wv + 4) * NBR - 1;
  // LDS vectors: two column buffers at buf and buf + LP (addressed by offset:
  // a pointer picked from an array loses its LDS address space), w, A x,
  // column k + 1
  double* wb = buf + 2 * LP;
  double* pf = buf + 3 * LP;
  double* cpre = buf + 4 * LP;
  double A[NBR][NBC];
  // one row of the block at a time: both triangles' entries loaded
  // unconditionally (indices clamped) before the selects
#pragma unroll
  for (int li = 0; li < NBR; ++li) {
    double ka[NBC], kb[NBC];
    const int i = row0 + li, ic = min(i, N - 1);
#pragma unroll
    for (int lj = 0; lj < NBC; ++lj) {
      const int jc = min(c + 16 * lj, N - 1);
      ka[lj] = a.K[ic + (size_t)jc * a.ldk];
      kb[lj] = a.K[jc + (size_t)ic * a.ldk];
    }
#pragma unroll
    for (int lj = 0; lj < NBC; ++lj) {
      const int j = c + 16 * lj;
      A[li][lj] = (i < N && j < N) ? 0.5 * (ka[lj] + kb[lj]) : 0.0;
    }
  }
  // column 0 below the diagonal, and d[0]
  for (int i = tid; i < LP; i += NT) {
    buf[i] = (i >= 1 && i < N) ? 0.5 * (a.K[i] + a.K[(size_t)i * a.ldk]) : 0.0;
    buf[LP + i] = 0.0;  // rows at or beyond N stay zero in every vector
    wb[i] = 0.0;
    pf[i] = 0.0;
    cpre[i] = 0.0;
  }
  if (tid == 0) d[0] = a.K[0];
  __syncthreads();
  const bool tr = a.trace != 0 && tid == 0;  // per-step clock totals (tracing only)
  long long tl = tr ? wall_clock64() : 0, tacc0 = 0, tacc1 = 0;
  for (int k = 0; k + 2 < N; ++k) {
    const double* col = buf + (k & 1) * LP;
    double* coln = buf + ((k + 1) & 1) * LP;
    const bool live = wave_last_row > k;  // uniform: this wave owns a row below k
    // ---- (a)
    double xc[NBC];
#pragma unroll
    for (int q = 0; q < NBC; ++q) xc[q] = col[c + 16 * q];
    // short dependent chains: FP64 latency, not issue, bounds this kernel
    double xs3[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NBC; ++q) xs3[q % 3] = fma(xc[q], xc[q], xs3[q % 3]);
    double xs = row16_sum((xs3[0] + xs3[1]) + xs3[2]);  // |x|^2, x_{k+1} included
    const double alpha = col[k + 1];
    double xax = 0.0;
    double xr[NBR];  // x on this thread's rows (also gives v there in (c))
    if (live) {
#pragma unroll
      for (int q = 0; q < NBR; ++q) xr[q] = col[row0 + q];
#pragma unroll
      for (int li = 0; li < NBR; ++li) {
        double s3[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int lj = 0; lj < NBC; ++lj) s3[lj % 3] = fma(A[li][lj], xc[lj], s3[lj % 3]);
        const double s0 = row16_sum((s3[0] + s3[1]) + s3[2]);  // (A x) for row row0 + li
        if (c == 0) pf[row0 + li] = s0;
        xax = fma(xr[li], s0, xax);
      }
    }
    // the owners of column k + 1 publish it (before this step's update)
    {
      const int lj1 = (k + 1) >> 4;
#pragma unroll
      for (int q = 0; q < NBC; ++q)
        if (q == lj1 && c == ((k + 1) & 15)) {
#pragma unroll
          for (int li = 0; li < NBR; ++li) cpre[row0 + li] = A[li][q];
        }
    }
    // x^T A x of the wave: the four row groups (equal over their 16 lanes)
    {
      int2 v2 = __builtin_bit_cast(int2, xax);
      double s4 = 0.0;
#pragma unroll
      for (int g4 = 0; g4 < 4; ++g4) {
        int2 u;
        u.x = __builtin_amdgcn_readlane(v2.x, 16 * g4);
        u.y = __builtin_amdgcn_readlane(v2.y, 16 * g4);
        s4 += __builtin_bit_cast(double, u);
      }
      if (lane == 0) red[wv] = s4;
    }
    // reflector scalars (dlarfg convention), branch-free so that they overlap
    // the products above: r = 1 / sqrt(|x|^2) by reciprocal square root and
    // two Newton steps, beta = -sign(alpha) |x|, t = (beta - alpha) / beta =
    // 1 + |alpha| r, scale = 1 / (alpha - beta) = sign(alpha) / (|alpha| + |x|)
    double t, beta, scale;
    {
      const bool refl = xs - alpha * alpha > 0.0;
      const double xq = refl ? xs : 1.0;
      double rs = __builtin_amdgcn_rsq(xq);
      rs = rs * fma(-0.5 * xq * rs, rs, 1.5);
      rs = rs * fma(-0.5 * xq * rs, rs, 1.5);
      const double nx = xq * rs, aa = fabs(alpha);
      const double den = aa + nx;
      double q = __builtin_amdgcn_rcp(den);
      q = fma(fma(-den, q, 1.0), q, q);
      q = fma(fma(-den, q, 1.0), q, q);
      t = refl ? fma(aa, rs, 1.0) : 0.0;
      beta = refl ? -copysign(nx, alpha) : alpha;
      scale = refl ? copysign(q, alpha) : 0.0;
    }
    __syncthreads();
    if (tr) { const long long tn = wall_clock64(); tacc0 += tn - tl; tl = tn; }
    // ---- (b) v and w, the reflector kept in P, the next column
    // (threads past the last trailing row skip the phase)
    if (k + 1 + tid < N) {
      const double g = 1.0 - scale * alpha;
      double rw[nw];
  #pragma unroll
      for (int q = 0; q < nw; ++q) rw[q] = red[q];
  #pragma unroll
      for (int h = 1; h < nw; h *= 2)  // pairwise: log2(nw) dependent adds
  #pragma unroll
        for (int q = 0; q + h < nw; q += 2 * h) rw[q] += rw[q + h];
      const double xaxs = rw[0];
      const double ax1 = pf[k + 1], a11 = cpre[k + 1];
      // v^T A v = scale^2 x^T A x + 2 scale g (A x)_{k+1} + g^2 A(k+1, k+1)
      const double vav = scale * scale * xaxs + 2.0 * scale * g * ax1 + g * g * a11;
      const double alf = -0.5 * t * t * vav;
      // (A v)_i = scale (A x)_i + g A(i, k+1)
      const double w1 = (t != 0.0) ? t * (scale * ax1 + g * a11) + alf : 0.0;  // v_{k+1} = 1
      if (tid == 0) {
        tau[k] = t;
        e[k] = beta;
        coln[k] = 0.0;  // rows <= k + 1 of the next column, v and w are zero
        wb[k] = 0.0;
      }
      const int ck = pk_cb(k, N);
      for (int i = k + 1 + tid; i < N; i += NT) {
        const double x = col[i];
        const double vi = (i == k + 1) ? 1.0 : x * scale;
        const double ci = cpre[i];
        const double wi = (t != 0.0) ? t * (scale * pf[i] + g * ci) + alf * vi : 0.0;
        wb[i] = wi;
        // reflector kept below the diagonal of column k (identity if t = 0)
        P[ck + i] = (t != 0.0) ? vi : ((i == k + 1) ? 1.0 : 0.0);
        // column k + 1 after the update: A(i, k+1) - v_i w_{k+1} - w_i v_{k+1}
        const double upd = (t != 0.0) ? vi * w1 + wi : 0.0;
        if (i == k + 1) d[k + 1] = ci - ((t != 0.0) ? 2.0 * w1 : 0.0);
        coln[i] = (i >= k + 2) ? ci - upd : 0.0;
      }
    }
    __syncthreads();
    if (tr) { const long long tn = wall_clock64(); tacc1 += tn - tl; tl = tn; }
    // ---- (c) rank-2 update of this thread's block; v comes from x in the
    // registers (v = scale x below row k + 1, v_{k+1} = 1, the same products
    // as in (b)), w from LDS
    if (live && t != 0.0) {
      double vr[NBR], vc[NBC], wr[NBR], wc[NBC];
#pragma unroll
      for (int q = 0; q < NBR; ++q) {
        wr[q] = wb[row0 + q];
        vr[q] = (row0 + q == k + 1) ? 1.0 : xr[q] * scale;
      }
#pragma unroll
      for (int q = 0; q < NBC; ++q) {
        wc[q] = wb[c + 16 * q];
        vc[q] = (c + 16 * q == k + 1) ? 1.0 : xc[q] * scale;
      }
#pragma unroll
      for (int li = 0; li < NBR; ++li)
#pragma unroll
        for (int lj = 0; lj < NBC; ++lj)
          A[li][lj] = fma(-vr[li], wc[lj], fma(-wr[li], vc[lj], A[li][lj]));
    }
  }
  // last diagonal entry and last off-diagonal from the registers
#pragma unroll
  for (int li = 0; li < NBR; ++li)
#pragma unroll
    for (int lj = 0; lj < NBC; ++lj) {
      const int i = row0 + li, j = c + 16 * lj;
      if (N >= 2 && i == N - 1 && j == N - 1) d[N - 1] = A[li][lj];
      if (N >= 2 && i == N - 1 && j == N - 2) e[N - 2] = A[li][lj];
    }
  if (tid == 0) {
    tau[max(N - 2, 0)] = 0.0;
    if (N == 1) d[0] = a.K[0];
    a.st->t_sub[0] = tacc0;
    a.st->t_sub[1] = tacc1;
  }
  __syncthreads();
}

// tridiag_reg on the smallest thread-grid blocking that covers N: the work
// of a step is issue-bound (every thread updates its whole block), so a
// trial basis well below the kernel's largest order takes a smaller block
// per thread.  The choice is uniform (N from the device state).
template <int NBR, int NBC, int NT>
__device__ inline void tridiag_fit(const RRArgs& a, int N, double* P, double* d, double* e,
                                   double* tau, double* buf, double* red) {
  constexpr int RG = NT / 16;
  if constexpr (NBR >= 3 && NBC >= 3 && (NBR > 3 || NBC > 3)) {
    if (N <= 3 * RG && N <= 48) {
      tridiag_reg<3, 3, NT>(a, N, P, d, e, tau, buf, red);
      return;
    }
  }
  if constexpr (NBR >= 4 && NBC >= 4 && (NBR > 4 || NBC > 4)) {
    if (N <= 4 * RG && N <= 64) {
      tridiag_reg<4, 4, NT>(a, N, P, d, e, tau, buf, red);
      return;
    }
  }
  if constexpr (NBR >= 3 && NBC >= 6 && (NBR > 3 || NBC > 6)) {
    if (N <= 3 * RG && N <= 96) {
      tridiag_reg<3, 6, NT>(a, N, P, d, e, tau, buf, red);
      return;
    }
  }
  if constexpr (NBR >= 4 && NBC >= 8 && (NBR > 4 || NBC > 8)) {
    if (N <= 4 * RG && N <= 128) {
      tridiag_reg<4, 8, NT>(a, N, P, d, e, tau, buf, red);
      return;
    }
  }
  tridiag_reg<NBR, NBC, NT>(a, N, P, d, e, tau, buf, red);
}

// Back-transformation Z = H_0 H_1 ... H_{N-3} Y by blocks of
// reflectors, last block first, on ncols <= 16 (NTQ - 1) columns of Y:
// Y <- (I - V T V^T) Y with V the block's reflectors (unit at row k + 1,
// zero above) and T = U^{-1}, U = diag(1 / tau) + strictly upper part of
// V^T V (a zero tau gives a zero row and column of T).  Per block:
//   (i)   G = V^T [V, Y] (16 x (16 + ncols)): each 16-lane row group forms an
//         LPG x 16 tile over rows b0 + 1 + s + 16 u (lane s), summed over
//         the row group (DPP);
//   (ii)  W <- T W by back substitution with U = T^{-1}, one thread per column;
//   (iii) Y -= V W in the RG x 16 thread grid, rows b0 + 1 + r + RG li,
//         columns c + 16 lj.
template <int NT, int NBC, int NTQ>
__device__ inline void wy_back(int N, const double* P, const double* tau, double* Y, int ldy,
                               int ncols, double* Tb, double* Wb, State* st) {
  const int tid = threadIdx.x;
  {
    constexpr int RG = NT / 16;            // 16-lane row groups
    constexpr int LPG = 16 * NTQ / RG;     // reflectors per group in (i)
    static_assert(16 * NTQ % RG == 0 && 16 % (16 * NTQ / RG) == 0, "row groups per target tile");
    constexpr int LQ = kWYBlock / LPG;     // groups per target quarter
    constexpr int NCW = NTQ - 1;           // column tiles of Y (ncols <= 16 NCW)
    const int g = tid >> 4, s16 = tid & 15, r = tid >> 4, c = tid & 15;
    const int nref = N - 2;  // reflectors 0 .. N - 3
    long long tw = st ? wall_clock64() : 0, twa[4] = {0, 0, 0, 0};
    for (int b0 = nref > 0 ? ((nref - 1) / kWYBlock) * kWYBlock : -1; b0 >= 0; b0 -= kWYBlock) {
      const int bs = min(kWYBlock, nref - b0);
      {
        const int lq = g % LQ, tq = g / LQ;  // reflectors lq LPG .., targets 16 tq ..
        double acc[LPG][16];
#pragma unroll
        for (int x = 0; x < LPG; ++x)
#pragma unroll
          for (int tt = 0; tt < 16; ++tt) acc[x][tt] = 0.0;
#pragma unroll 1
        for (int u = 0; u < NBC; ++u) {
          const int i = b0 + 1 + s16 + 16 * u, ic = min(i, N - 1);
          double vx[LPG];
#pragma unroll
          for (int x = 0; x < LPG; ++x) {
            const int l = lq * LPG + x, kl = b0 + l;
            const double pv_ = P[pk_cb(min(kl, N - 3), N) + ic];
            vx[x] = (l < bs && i >= kl + 1 && i < N) ? ((i == kl + 1) ? 1.0 : pv_) : 0.0;
          }
          if (tq == 0) {  // V^T V (uniform per wave)
#pragma unroll
            for (int tt = 0; tt < 16; ++tt) {
              const int kq = b0 + tt;
              const double pq = P[pk_cb(min(kq, N - 3), N) + ic];
              const double vq = (tt < bs && i >= kq + 1 && i < N) ? ((i == kq + 1) ? 1.0 : pq) : 0.0;
#pragma unroll
              for (int x = 0; x < LPG; ++x) acc[x][tt] = fma(vx[x], vq, acc[x][tt]);
            }
          } else {  // V^T Y on columns 16 (tq - 1) .. (v is zero past N)
#pragma unroll
            for (int tt = 0; tt < 16; ++tt) {
              const int jc = min(16 * (tq - 1) + tt, ncols - 1);
              const double yv = Y[ic + (size_t)jc * ldy];
#pragma unroll
              for (int x = 0; x < LPG; ++x) acc[x][tt] = fma(vx[x], yv, acc[x][tt]);
            }
          }
        }
#pragma unroll
        for (int x = 0; x < LPG; ++x)
#pragma unroll
          for (int tt = 0; tt < 16; ++tt) acc[x][tt] = row16_sum(acc[x][tt]);
        if (s16 == 0) {
#pragma unroll
          for (int x = 0; x < LPG; ++x) {
            const int l = lq * LPG + x;
#pragma unroll
            for (int tt = 0; tt < 16; ++tt) {
              if (tq == 0) {
                Tb[l + kWYBlock * tt] = acc[x][tt];
              } else {
                const int j = 16 * (tq - 1) + tt;
                if (j < ncols) Wb[l + kWYLd * j] = acc[x][tt];
              }
            }
          }
        }
      }
      __syncthreads();
      if (tid == 0 && st) { const long long tn = wall_clock64(); twa[0] += tn - tw; tw = tn; }
      // W <- T W with T = U^{-1}, U = diag(1 / tau) + strictly upper part of
      // V^T V: back substitution U W' = W, one thread per column of W,
      // W'(l) = tau_l (W(l) - sum_{m > l} G(l, m) W'(m)) (zero when tau_l = 0)
      for (int j = tid; j < ncols; j += NT) {
        double w[kWYBlock];
#pragma unroll
        for (int l = 0; l < kWYBlock; ++l) {
          const double wl = Wb[l + kWYLd * j];
          w[l] = (l < bs) ? wl : 0.0;
        }
#pragma unroll
        for (int l = kWYBlock - 1; l >= 0; --l) {
          double s = w[l];
#pragma unroll
          for (int m = l + 1; m < kWYBlock; ++m) s = fma(-Tb[l + kWYBlock * m], w[m], s);
          const double tl = (l < bs) ? tau[b0 + min(l, bs - 1)] : 0.0;
          w[l] = tl * s;
          asm volatile("" ::: "memory");  // one row of G in flight at a time
        }
#pragma unroll
        for (int l = 0; l < kWYBlock; ++l) Wb[l + kWYLd * j] = w[l];
      }
      __syncthreads();
      if (tid == 0 && st) {
        const long long tn = wall_clock64();
        twa[1] += tn - tw;
        tw = tn;
      }
      // Y -= V W on rows b0 + 1 .. N - 1
      {
        const int i0 = b0 + 1;
        double wr3[NCW][kWYBlock];  // this thread's columns of W (rows >= bs are zero)
#pragma unroll
        for (int lj = 0; lj < NCW; ++lj) {
          const int jc = min(c + 16 * lj, ncols - 1);
#pragma unroll
          for (int l = 0; l < kWYBlock; ++l) {
            const double wl = Wb[l + kWYLd * jc];
            wr3[lj][l] = (l < bs) ? wl : 0.0;
          }
        }
        for (int li = 0; i0 + r + RG * li < N; ++li) {
          const int i = i0 + r + RG * li;
          double vr[kWYBlock];
#pragma unroll
          for (int l = 0; l < kWYBlock; ++l) {
            const int kl = b0 + l;
            const double pl = P[pk_cb(min(kl, N - 3), N) + i];  // in range for every l
            vr[l] = (l < bs && i >= kl + 1) ? ((i == kl + 1) ? 1.0 : pl) : 0.0;
          }
#pragma unroll
          for (int lj = 0; lj < NCW; ++lj) {
            const int j = c + 16 * lj, jc = min(j, ncols - 1);
            double s = Y[i + (size_t)jc * ldy];
#pragma unroll
            for (int l = 0; l < kWYBlock; ++l) s = fma(-vr[l], wr3[lj][l], s);
            if (j < ncols) Y[i + (size_t)j * ldy] = s;
          }
        }
      }
      __syncthreads();
      if (tid == 0 && st) { const long long tn = wall_clock64(); twa[3] += tn - tw; tw = tn; }
    }
    if (tid == 0 && st)
      for (int q = 0; q < 4; ++q) st->t_sub[2 + q] = twa[q];
  }
}

// The back-transformation of wy_back for 256 threads and up to 16 columns of
// Y, with each block's reflectors first expanded into a dense zero-padded
// 16 x ldv array Vb (ldv = 16 NBC + 1, rows b0 + 1 + i' at i', the unit
// entries and the zeros above them written out).  Every load of the three
// stages is then unconditional, and the row loops stop at the block's last
// row instead of running over the whole trial basis.
constexpr int kWYDenseThreads = 256;
template <int NBC>
__host__ __device__ constexpr int wy_dense_ldv() { return 16 * NBC + 1; }

template <int NBC>
__device__ inline void wy_back_dense(int N, const double* P, const double* tau, double* Y, int ldy,
                                     int ncols, double* Tb, double* Wb, double* Vb, State* st) {
  constexpr int NT = kWYDenseThreads;
  constexpr int LDV = wy_dense_ldv<NBC>();
  constexpr int LPG = 2;   // reflectors per 16-lane group in (i)
  constexpr int LQ = 8;    // groups per target tile: groups 0-7 form V^T V, 8-15 V^T Y
  const int tid = threadIdx.x;
  const int g = tid >> 4, s16 = tid & 15;
  const int nref = N - 2;  // reflectors 0 .. N - 3
  long long tw = st ? wall_clock64() : 0, twa[4] = {0, 0, 0, 0};
  for (int b0 = nref > 0 ? ((nref - 1) / kWYBlock) * kWYBlock : -1; b0 >= 0; b0 -= kWYBlock) {
    const int bs = min(kWYBlock, nref - b0);
    const int nrow = N - 1 - b0;          // rows b0 + 1 .. N - 1
    const int nu = (nrow + 15) >> 4;      // 16-row chunks
    // (0) Vb: thread (l = g, s16) fills rows s16 + 16 u of reflector b0 + l
    {
      const int l = g, kl = b0 + l, kc = min(kl, N - 3);
      const int base = pk_cb(kc, N);
      double pv[NBC];
#pragma unroll
      for (int u = 0; u < NBC; ++u) pv[u] = P[base + min(b0 + 1 + s16 + 16 * u, N - 1)];
      asm volatile("" ::: "memory");  // all loads issued before the selects
#pragma unroll
      for (int u = 0; u < NBC; ++u) {
        const int i = b0 + 1 + s16 + 16 * u;
        const double v = (l < bs && i < N && i > kl) ? ((i == kl + 1) ? 1.0 : pv[u]) : 0.0;
        Vb[l * LDV + s16 + 16 * u] = v;
      }
    }
    __syncthreads();
    // (i) G = V^T [V, Y]
    {
      const int lq = g % LQ, tq = g / LQ;
      double acc[LPG][16];
#pragma unroll
      for (int x = 0; x < LPG; ++x)
#pragma unroll
        for (int tt = 0; tt < 16; ++tt) acc[x][tt] = 0.0;
#pragma unroll 1
      for (int u = 0; u < nu; ++u) {
        const int ip = s16 + 16 * u;
        double vx[LPG], tv[16];
#pragma unroll
        for (int x = 0; x < LPG; ++x) vx[x] = Vb[(lq * LPG + x) * LDV + ip];
        if (tq == 0) {  // uniform per wave
#pragma unroll
          for (int tt = 0; tt < 16; ++tt) tv[tt] = Vb[tt * LDV + ip];
        } else {
          const int ic = min(b0 + 1 + ip, N - 1);  // v is zero past the last row
#pragma unroll
          for (int tt = 0; tt < 16; ++tt) tv[tt] = Y[ic + (size_t)min(tt, ncols - 1) * ldy];
        }
#pragma unroll
        for (int tt = 0; tt < 16; ++tt)
#pragma unroll
          for (int x = 0; x < LPG; ++x) acc[x][tt] = fma(vx[x], tv[tt], acc[x][tt]);
      }
#pragma unroll
      for (int x = 0; x < LPG; ++x)
#pragma unroll
        for (int tt = 0; tt < 16; ++tt) acc[x][tt] = row16_sum(acc[x][tt]);
      if (s16 == 0) {
#pragma unroll
        for (int x = 0; x < LPG; ++x) {
          const int l = lq * LPG + x;
#pragma unroll
          for (int tt = 0; tt < 16; ++tt) {
            if (tq == 0)
              Tb[l + kWYBlock * tt] = acc[x][tt];
            else if (tt < ncols)
              Wb[l + kWYLd * tt] = acc[x][tt];
          }
        }
      }
    }
    __syncthreads();
    if (tid == 0 && st) { const long long tn = wall_clock64(); twa[0] += tn - tw; tw = tn; }
    // (ii) W <- T W by back substitution with U = T^{-1}, one thread per
    // column: W'(l) = tau_l (W(l) - sum_{m > l} G(l, m) W'(m)); rows l >= bs
    // of G and W are zero, and tau_l = 0 there
    if (tid < ncols) {
      const int j = tid;
      double w[kWYBlock];
#pragma unroll
      for (int l = 0; l < kWYBlock; ++l) {
        const double wl = Wb[l + kWYLd * j];
        w[l] = (l < bs) ? wl : 0.0;
      }
#pragma unroll
      for (int l = kWYBlock - 1; l >= 0; --l) {
        double s = w[l];
#pragma unroll
        for (int m = l + 1; m < kWYBlock; ++m) s = fma(-Tb[l + kWYBlock * m], w[m], s);
        const double tl = tau[b0 + min(l, bs - 1)];
        w[l] = (l < bs) ? tl * s : 0.0;
        asm volatile("" ::: "memory");  // one row of G in flight at a time
      }
#pragma unroll
      for (int l = 0; l < kWYBlock; ++l) Wb[l + kWYLd * j] = w[l];
    }
    __syncthreads();
    if (tid == 0 && st) { const long long tn = wall_clock64(); twa[1] += tn - tw; tw = tn; }
    // (iii) Y -= V W: thread (r, c) on rows b0 + 1 + r + 16 li of column c
    {
      const int r = tid >> 4, c = tid & 15, jc = min(c, ncols - 1);
      double wr[kWYBlock];
#pragma unroll
      for (int l = 0; l < kWYBlock; ++l) wr[l] = Wb[l + kWYLd * jc];
#pragma unroll 1
      for (int ip = r; ip < nrow; ip += 16) {
        double vr[kWYBlock];
#pragma unroll
        for (int l = 0; l < kWYBlock; ++l) vr[l] = Vb[l * LDV + ip];
        double* yp = Y + (b0 + 1 + ip) + (size_t)jc * ldy;
        double s = *yp;
#pragma unroll
        for (int l = 0; l < kWYBlock; ++l) s = fma(-vr[l], wr[l], s);
        if (c < ncols) *yp = s;
      }
    }
    __syncthreads();
    if (tid == 0 && st) { const long long tn = wall_clock64(); twa[3] += tn - tw; tw = tn; }
  }
  if (tid == 0 && st)
    for (int q = 0; q < 4; ++q) st->t_sub[2 + q] = twa[q];
}

template <int NBR, int NBC, int NT, bool EXPORT>
__device__ inline void rr_fast_body(const RRArgs& a, double* lds, const RRShared& sh) {
  lds = lds_base();  // callers pass the dynamic LDS base; keep its address space
  double* s_lo = sh.lo;
  double* s_hi = sh.hi;
  int& s_npos = *sh.npos;
  double& s_tnorm = *sh.tnorm;
  double& s_pivmin = *sh.pivmin;
  State* st = a.st;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int N = st->Np;
  const int mk = min(a.mtarget, N);
  // ---- LDS layout
  const int ldy = (N & 1) ? N : N + 1;  // odd: threads over columns hit distinct banks
  double* P = lds;                                   // N(N+1)/2 packed lower, column-major
  double* d = P + (size_t)N * (N + 1) / 2;           // N
  double* e = d + N;                                 // N
  double* e2 = e + N;                                // N
  double* tau = e2 + N;                              // N
  double* pv = tau + N;                              // N: Ritz values
  double* Y = pv + N;                                // ldy x mk (phase 3, 4)
  double* tbuf = Y;                                  // phase-1 vectors and partial products
  int* cnts = (int*)Y;                               // nt Sturm counts (phase 2)
  double* Tb = Y + rr_fast_yspace(N, mk, nt, rr_fast_lp(nt, NBR, NBC));  // 16 x 16 WY factor
  double* Wb = Tb + kWYBlock * kWYBlock;             // 16 x mk
  double* red = Tb + rr_fast_tbw(N, mk);             // nw
  if (tid == 0) st->t_phase[0] = wall_clock64();

  // ---- 1. tridiagonalization (matrix in registers)
  tridiag_fit<NBR, NBC, NT>(a, N, P, d, e, tau, tbuf, red);
  if (EXPORT) {
    // reflectors and tau to the global scratch for the back-transformation
    // kernel; the reflector region is free for the vectors' D- afterwards
    const size_t n2 = (size_t)N * (N + 1) / 2;
    for (size_t x = tid; x < n2; x += nt) a.scratch[x] = P[x];
    for (int x = tid; x < N; x += nt) a.scratch[n2 + x] = tau[x];
  }
  // e^2, and in one parallel pass the row-sum norm ||T||, max e^2 and the
  // Gershgorin interval (max / min reductions: the same values as a serial loop)
  double s_gl, s_gu;
  {
    double tn = 0.0, em = 0.0, gl = 0.0, gu = 0.0;
    bool any = false;
    for (int i = tid; i < N; i += nt) {
      const double ea = (i > 0) ? fabs(e[i - 1]) : 0.0;
      const double eb = (i + 1 < N) ? fabs(e[i]) : 0.0;
      if (i + 1 < N) {
        const double q = e[i] * e[i];
        e2[i] = q;
        em = fmax(em, q);
      }
      tn = fmax(tn, fabs(d[i]) + ea + eb);
      const double rr = ea + eb;
      gl = any ? fmin(gl, d[i] - rr) : d[i] - rr;
      gu = any ? fmax(gu, d[i] + rr) : d[i] + rr;
      any = true;
    }
    if (!any) {  // neutral elements for the reductions
      gl = __builtin_inf();
      gu = -__builtin_inf();
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      tn = fmax(tn, __shfl_xor(tn, o, 64));
      em = fmax(em, __shfl_xor(em, o, 64));
      gl = fmin(gl, __shfl_xor(gl, o, 64));
      gu = fmax(gu, __shfl_xor(gu, o, 64));
    }
    double* part = s_lo;  // 4 per wave (the brackets are written later)
    if (lane == 0) {
      part[4 * wv] = tn;
      part[4 * wv + 1] = em;
      part[4 * wv + 2] = gl;
      part[4 * wv + 3] = gu;
    }
    __syncthreads();
    for (int q = 0; q < nt / 64; ++q) {
      tn = fmax(tn, part[4 * q]);
      em = fmax(em, part[4 * q + 1]);
      gl = fmin(gl, part[4 * q + 2]);
      gu = fmax(gu, part[4 * q + 3]);
    }
    s_gl = gl;
    s_gu = gu;
    if (tid == 0) {
      s_tnorm = tn;
      s_pivmin = 2.2250738585072014e-308 * fmax(1.0, em);
    }
  }
  __syncthreads();
  const double tnorm = s_tnorm, pivmin = s_pivmin;
  // d and e^2 scaled by 2^-tsh (||T|| below one) for the polynomial Sturm
  // counts, after the counts in the Y region (nt ints; the region holds
  // max(nt, 6 lp) doubles with lp >= N)
  const int tsh = tnorm > 0.0 ? __builtin_amdgcn_frexp_exp(tnorm) : 0;
  double* dsc = Y + nt / 2;
  double* e2sc = dsc + N;
  for (int i = tid; i < N; i += nt) {
    dsc[i] = __builtin_amdgcn_ldexp(d[i], -tsh);
    e2sc[i] = (i + 1 < N) ? __builtin_amdgcn_ldexp(e2[i], -2 * tsh) : 0.0;
  }
  __syncthreads();
  if (tid == 0) st->t_phase[1] = wall_clock64();

  // ---- 2. multisection for the top mk eigenvalues (+ count of positives)
  {
    double gl = s_gl, gu = s_gu;
    const double pad = 2.2e-16 * tnorm * 4.0 * N + 2.0 * pivmin;
    gl -= pad;
    gu += pad;
    // shared first round: nt - 1 equispaced shifts over [gl, gu] for all
    // the eigenvalues at once, and the count below zero; each eigenvalue's
    // bracket follows by binary search over the counts, keeping
    // count(lo) <= target < count(hi)
    // open brackets: per-wave ballots in LDS (the tridiagonalization's
    // reduction slots), read by every thread after the next barrier
    int* oflag = reinterpret_cast<int*>(red);
    bool open = false;
    {
      const int ng = nt - 1;
      const double x = (tid < ng) ? gl + (gu - gl) * (double)(tid + 1) / (double)(ng + 1) : 0.0;
      cnts[tid] = sturm_count_fast(dsc, e2sc, d, e2, N, x, tsh, pivmin);
      __syncthreads();
      if (tid == nt - 1) s_npos = N - cnts[tid];
      for (int j = tid; j < mk; j += nt) {
        const int target = N - 1 - j;
        int a0 = -1, a1 = ng;  // virtual counts: cnt(-1) = 0 at gl, cnt(ng) = N at gu
        while (a1 - a0 > 1) {
          const int mid = (a0 + a1) >> 1;
          if (cnts[mid] <= target) a0 = mid;
          else a1 = mid;
        }
        const double lo = (a0 < 0) ? gl : gl + (gu - gl) * (double)(a0 + 1) / (double)(ng + 1);
        const double hi = (a1 >= ng) ? gu : gl + (gu - gl) * (double)(a1 + 1) / (double)(ng + 1);
        s_lo[j] = lo;
        s_hi[j] = hi;
        open = open || bracket_open(lo, hi, tnorm, pivmin);
      }
    }
    {
      const unsigned long long bal = __ballot(open);
      if (lane == 0) oflag[wv] = bal != 0ull;
    }
    __syncthreads();
    const int per = max(1, nt / max(mk, 1));  // shifts per eigenvalue per round
    const int j_me = tid / per, s_me = tid % per;
    // shift s of a bracket [lo, hi]: lo + (hi - lo) (s + 1) rp; the counts
    // and the bracket update use this same expression
    const double rp = 1.0 / (double)(per + 1);
    int rounds = 1;
    for (int round = 0; round < 64; ++round) {
      int anyi = 0;
#pragma unroll
      for (int q = 0; q < NT / 64; ++q) anyi |= oflag[q];
      if (anyi == 0) break;
      ++rounds;
      if (j_me < mk) {
        const double lo = s_lo[j_me], hi = s_hi[j_me];
        const double x = lo + (hi - lo) * ((double)(s_me + 1) * rp);
        cnts[tid] = sturm_count_fast(dsc, e2sc, d, e2, N, x, tsh, pivmin);
      }
      __syncthreads();
      // new bracket: the first shift whose count exceeds the target (counts
      // loaded 16 at a time ahead of the selects, no early exit)
      open = false;
      if (tid < mk) {
        const int j = tid;
        const int target = N - 1 - j;  // ascending index of the j-th largest
        const double lo = s_lo[j], hi = s_hi[j];
        int first = per;
        for (int s0 = 0; s0 < per; s0 += 16) {
          int cv[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) cv[u] = cnts[j * per + min(s0 + u, per - 1)];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int s2 = s0 + u;
            first = (s2 < first && s2 < per && cv[u] > target) ? s2 : first;
          }
        }
        const double nlo = (first > 0) ? lo + (hi - lo) * ((double)first * rp) : lo;
        const double nhi = (first < per) ? lo + (hi - lo) * ((double)(first + 1) * rp) : hi;
        s_lo[j] = nlo;
        s_hi[j] = nhi;
        open = bracket_open(nlo, nhi, tnorm, pivmin);
      }
      {
        const unsigned long long bal = __ballot(open);
        if (lane == 0) oflag[wv] = bal != 0ull;
      }
      __syncthreads();
    }
    if (tid == 0) st->t_sub[6] = rounds;
  }
  if (tid == 0) st->t_phase[2] = wall_clock64();
  long long t_mgs = wall_clock64();

  // ---- 3. eigenvectors: twisted factorization, one thread per vector
  const double pfloor = fmax(2.2e-16 * tnorm, 1e-300);
  const double ortol = 1e-3 * tnorm;
  if (EXPORT && mk <= 64 && nt >= 128 && 2 * mk <= N + 1) {
    // wave 0 forms the top-down pivots of vector `lane`, wave 1 its
    // bottom-up pivots (D- in the reflector region, exported already, which
    // holds N (N + 1) / 2 >= mk N doubles); both
    // find the twist, then wave 0 builds the part above it and wave 1 the
    // part below
    const int j = lane, half = wv;
    const bool act = wv < 2 && j < mk;
    const double sigma = act ? 0.5 * (s_lo[j] + s_hi[j]) : 0.0;
    double* y = Y + (size_t)min(j, mk - 1) * ldy;
    double* dmv = P + (size_t)min(j, mk - 1) * N;
    if (act) {
      if (N == 1) {
        if (half == 0) y[0] = 1.0;
      } else if (half == 0) {
        twisted_top(d, e2, N, sigma, pfloor, y);
      } else {
        twisted_bottom(d, e2, N, sigma, pfloor, dmv);
      }
    }
    __syncthreads();
    const int r = (act && N > 1) ? twisted_index(d, N, sigma, y, dmv) : 0;
    __syncthreads();  // every twist is known before either part is written
    if (act && N > 1) {
      if (half == 0)
        twisted_up(e, r, y);
      else
        twisted_down(e, N, r, dmv, y);
    }
  } else {
    for (int j = tid; j < mk; j += nt)
      twisted_vector(d, e, e2, N, 0.5 * (s_lo[j] + s_hi[j]), pfloor, Y + (size_t)j * ldy);
  }
  __syncthreads();
  // normalization, one wave per vector: scaled by the largest entry first
  for (int j = wv; j < mk; j += nt / 64) {
    double* y = Y + (size_t)j * ldy;
    double mx = 0.0;
    for (int i = lane; i < N; i += 64) mx = fmax(mx, fabs(y[i]));
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    const double sc = mx > 0.0 ? 1.0 / mx : 1.0;
    double nn = 0.0;
    for (int i = lane; i < N; i += 64) { const double v = y[i] * sc; nn += v * v; }
    nn = wave_sum(nn);
    const double inv = 1.0 / sqrt(nn);
    for (int i = lane; i < N; i += 64) y[i] = (y[i] * sc) * inv;
  }
  __syncthreads();
  if (tid == 0) t_mgs = wall_clock64();
  // Gram-Schmidt inside clusters, block-wide: classical, applied twice per
  // vector (every dot product of a pass at once, one wave each), then the
  // norm by a block reduction; dot products in Tb
  {
    double* dots = Tb;
    for (int j = 1; j < mk; ++j) {
      const double mid_j = 0.5 * (s_lo[j] + s_hi[j]);
      const double mid_p = 0.5 * (s_lo[j - 1] + s_hi[j - 1]);
      if (mid_p - mid_j > ortol) continue;
      int c0 = j - 1;
      while (c0 > 0 && 0.5 * (s_lo[c0 - 1] + s_hi[c0 - 1]) - 0.5 * (s_lo[c0] + s_hi[c0]) <= ortol)
        --c0;
      double* yj = Y + (size_t)j * ldy;
      for (int attempt = 0; attempt < 2; ++attempt) {
        for (int pass = 0; pass < 2; ++pass) {
          for (int i0 = c0 + wv; i0 < j; i0 += nt / 64) {
            const double* yi = Y + (size_t)i0 * ldy;
            double dp = 0.0;
            for (int q = lane; q < N; q += 64) dp += yi[q] * yj[q];
            dp = wave_sum(dp);
            if (lane == 0) dots[i0 - c0] = dp;
          }
          __syncthreads();
          for (int q = tid; q < N; q += nt) {
            double v = yj[q];
            for (int i0 = c0; i0 < j; ++i0) v -= dots[i0 - c0] * Y[q + (size_t)i0 * ldy];
            yj[q] = v;
          }
          __syncthreads();
        }
        double nn = 0.0;
        for (int q = tid; q < N; q += nt) nn += yj[q] * yj[q];
        nn = wave_sum(nn);
        if (lane == 0) red[wv] = nn;
        __syncthreads();
        nn = 0.0;
        for (int q = 0; q < nt / 64; ++q) nn += red[q];
        if (nn > 0.25 || attempt == 1) {
          const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
          for (int q = tid; q < N; q += nt) yj[q] *= inv;
          __syncthreads();
          break;
        }
        // the vector collapsed onto its predecessors (repeated eigenvalue):
        // inverse iteration from a fixed start vector, factors in Tb
        if (tid == 0) {
          for (int i = 0; i < N; ++i) yj[i] = start_entry(i, j);
          double* U0 = Tb;
          tri_solve(d, e, N, mid_j, pfloor, yj, U0, U0 + N, U0 + 2 * N, 1);
          double mx = 0.0;
          for (int i = 0; i < N; ++i) mx = fmax(mx, fabs(yj[i]));
          const double sc = mx > 0.0 ? 1.0 / mx : 1.0;
          for (int i = 0; i < N; ++i) yj[i] *= sc;
        }
        __syncthreads();
      }
    }
  }
  if (tid == 0) st->t_sub[7] = wall_clock64() - t_mgs;
  // Rayleigh quotients y^T T y, one wave per vector
  for (int j = wv; j < mk; j += nt / 64) {
    const double* y = Y + (size_t)j * ldy;
    double rq = 0.0;
    for (int i = lane; i < N; i += 64) {
      double ty = d[i] * y[i];
      if (i > 0) ty += e[i - 1] * y[i - 1];
      if (i + 1 < N) ty += e[i] * y[i + 1];
      rq += y[i] * ty;
    }
    rq = wave_sum(rq);
    if (lane == 0) pv[j] = rq;
  }
  __syncthreads();
  if (tid == 0) st->t_phase[3] = wall_clock64();

  if (!EXPORT) wy_back<NT, NBC, 4>(N, P, tau, Y, ldy, mk, Tb, Wb, a.trace ? st : nullptr);
  if (tid == 0) st->t_phase[4] = wall_clock64();
  // ---- outputs: C = Z (N x mk), Ritz values descending
  for (int x = tid; x < N * mk; x += nt) {
    const int i = x % N, j = x / N;
    a.C[i + (size_t)j * a.ldc] = Y[i + (size_t)j * ldy];
  }
  for (int j = tid; j < mk; j += nt) st->theta[j] = pv[j];
  if (tid == 0) {
    st->npos_rr = s_npos;
    st->mk = mk;
    st->expand_req = (s_npos > a.mtarget) ? 1 : 0;
    st->jacobi_rounds = 0;
    if (a.count_iter) st->iter += 1;
  }
}

}  // namespace psdp
