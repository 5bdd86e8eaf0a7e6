// Certificate of the tail term of the a-posteriori bound (paper §5.2,
// Thm `bound`): forming M = s I - P A P + c Vt Vt^T and its FP64 Cholesky
// factorization on 64 x 64 tiles (see cert.h for what success proves).
//
// Rounding (Higham, Accuracy and Stability of Numerical Algorithms, Thm 10.3
// and §3.5): a Cholesky factorization that completes with positive pivots
// gives L L^T = M + dM with |dM| <= gamma_{L+1} |L| |L^T|, hence
// ||dM||_2 <= gamma_{L+1} tr(M) / (1 - gamma_{L+1}); the factorization here
// scales by a refined reciprocal square root and divides through rounded
// reciprocals, a few more roundings per entry, which gamma_{L+8} covers (the
// bound holds for any order of each entry's inner product, so it covers the
// substitutions, the FMA updates and the matrix-core updates alike).  The
// formation of M is bounded the same way from the norms the kernels
// measure; eta is twice the sum of these terms.
#include "cert.h"
#include "common.h"

namespace psdp {

namespace {

constexpr int kT = kCertTile;  // 64
constexpr int kLd = kT + 1;     // LDS row stride of a row-major 64 x 64 tile

__device__ inline bool cert_failed(const CertState* cs) {
  return *(const volatile int*)&cs->fail != 0;
}

// lower-triangular tile index b -> (ii, jj), ii >= jj
__device__ inline void tri_index(int b, int& ii, int& jj) {
  int i = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= b) ++i;
  while (i * (i + 1) / 2 > b) --i;
  ii = i;
  jj = b - i * (i + 1) / 2;
}

// 1 / sqrt(d) for d > 0: the hardware estimate (relative error about 2^-24)
// refined by one third-order step y (1 + e / 2 + 3 e^2 / 8), e = 1 - d y^2
// (the first terms of (1 - e)^(-1/2)); measured within 1.3 units of
// roundoff, which the margin eta allows for.
__device__ inline double rsqrt_nr(double d) {
  const double y = __builtin_amdgcn_rsq(d);
  const double e = fma(-d * y, y, 1.0);
  const double p = fma(0.375, e, 0.5);
  return fma(y * e, p, y);
}

// v of lane `src` (a constant) on every lane
__device__ inline double bcast_lane(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// v of lane N of this lane's sixteen-lane row (DPP row broadcast)
template <int N>
__device__ inline double row_bcast(double v) {
  // one 64-bit DPP move (row_newbcast is a DPP64 control); every lane has a
  // source, so the old value is never kept
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + N, 0xF, 0xF, true);
}

// row_bcast with the lane given at run time (a constant once unrolled)
__device__ inline double row_bcast_n(double v, int n) {
  switch (n) {
    case 0: return row_bcast<0>(v);
    case 1: return row_bcast<1>(v);
    case 2: return row_bcast<2>(v);
    case 3: return row_bcast<3>(v);
    case 4: return row_bcast<4>(v);
    case 5: return row_bcast<5>(v);
    case 6: return row_bcast<6>(v);
    case 7: return row_bcast<7>(v);
    case 8: return row_bcast<8>(v);
    case 9: return row_bcast<9>(v);
    case 10: return row_bcast<10>(v);
    case 11: return row_bcast<11>(v);
    case 12: return row_bcast<12>(v);
    case 13: return row_bcast<13>(v);
    case 14: return row_bcast<14>(v);
    default: return row_bcast<15>(v);
  }
}

// Right-looking Cholesky of the 16 x 16 diagonal block at (o, o) of the
// 64 x 64 tile held row-major (stride 65) in LDS, by the first wave: lane i
// < 16 keeps row o + i in registers (the sixteen lanes of one DPP row); at
// column j the pivot comes from lane j by readlane, every lane forms
// 1 / sqrt(pivot) itself and its l_ij, and updates its row with l_cj, c > j,
// received from lane c by a DPP row broadcast (the entries right of its
// diagonal take junk updates that are never read).  Afterwards lane i writes
// the block's transposed strict lower triangle (lt[c * 16 + i] = l_ic for
// i > c, zero elsewhere) and 1 / l_ii (rinv) for the solves below the block.
// Returns 0 when a pivot is not positive and finite (the same on every
// lane).
__device__ __attribute__((always_inline)) inline int chol16_wave(double* a, double* lt,
                                                                double* rinv, int o) {
  constexpr int B = 16;
  const int lane = threadIdx.x;
  // lanes past the block repeat the rows of lanes 0..15 in their own DPP
  // rows (their results are neither broadcast nor stored), so every load is
  // unconditional
  double r[B];
#pragma unroll
  for (int c = 0; c < B; ++c) r[c] = a[(o + (lane & (B - 1))) * kLd + o + c];
  // No branch per column: a failed pivot clears `ok` (the same on every
  // lane) and is replaced by 1 so the remaining arithmetic stays finite.
  // The next pivot is lane j + 1's own update of its diagonal entry,
  // a_{j+1,j+1} - l_{j+1,j}^2 (the same FMA the column update below applies
  // there), read before the rest of the column's updates so that its
  // reciprocal square root overlaps them.
  int ok = 1;
  double d = bcast_lane(r[0], 0);
#pragma unroll
  for (int j = 0; j < B; ++j) {
    ok &= (d > 0.0 && d < INFINITY) ? 1 : 0;
    d = ok ? d : 1.0;
    const double inv = rsqrt_nr(d);
    const double l = r[j] * inv;
    r[j] = (lane == j) ? d * inv : l;
    const double dn = (j + 1 < B) ? bcast_lane(fma(-l, l, r[(j + 1) & (B - 1)]), (j + 1) & (B - 1)) : 0.0;
#pragma unroll
    for (int c = j + 1; c < B; ++c) r[c] = fma(-l, row_bcast_n(l, c), r[c]);
    d = dn;
  }
  if (lane < B) {
#pragma unroll
    for (int c = 0; c < B; ++c) {
      a[(o + lane) * kLd + o + c] = r[c];
      lt[c * B + lane] = (lane > c) ? r[c] : 0.0;
    }
    rinv[lane] = 1.0 / r[lane];
  }
  return ok;
}

// L_ik = A_ik L_kk^{-T} for the 16-row blocks i > K below the diagonal block
// K of the tile in LDS: sixteen lanes per row (one DPP row), lane g owning
// column 16 K + g, each lane 3 - K rows (three register slots, the unused
// ones repeating the last row and never stored).  At column c the owning
// lane forms x_c = a_c / l_cc by the rounded reciprocal, the row's lanes
// receive it by a DPP row broadcast and update their columns with l_gc from
// lt (zero on and above the diagonal, so every lane applies every update
// unconditionally): the column-ordered substitution of the standard
// algorithm.
__device__ __attribute__((always_inline)) inline void trsm16_tile(double* a, const double* lt,
                                                                 const double* rinv, int K) {
  const int nr = 3 - K;
  const int t = threadIdx.x, g = t & 15, gr = t >> 4;
  const int col = 16 * K + g;
  double x[3], w[16];
#pragma unroll
  for (int u = 0; u < 3; ++u) x[u] = a[(16 * (K + 1) + gr + 16 * min(u, nr - 1)) * kLd + col];
#pragma unroll
  for (int c = 0; c < 16; ++c) w[c] = lt[c * 16 + g];
  const double rv = rinv[g];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const double v = row_bcast_n(x[u] * rv, c);
      x[u] = (g == c) ? v : x[u];
      x[u] = fma(-v, w[c], x[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < 3; ++u)
    if (u < nr) a[(16 * (K + 1) + gr + 16 * u) * kLd + col] = x[u];
}

// A_IJ -= L_IK L_JK^T for the 16 x 16 blocks K < J <= I < 4 of the tile in
// LDS, on the matrix cores (v_mfma_f64_16x16x4f64, four k-steps of the
// panel's 16 columns): wave w takes the blocks w, w + 4, ...  Operands:
// A[row][k] = -l(16 I + row, 16 K + k) on lane (row + 16 k'), B[k][col] =
// l(16 J + col, 16 K + k); D: lane -> column l % 16, rows l / 16 + 4 r.
// Diagonal blocks are updated whole (their upper halves are never read).
__device__ __attribute__((always_inline)) inline void update16_tile(double* a, int K) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int nt = 3 - K;  // trailing blocks
  const int nb = nt * (nt + 1) / 2;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, li = lane & 15, gq = lane >> 4;
  for (int p = wv; p < nb; p += 4) {
    // block p of the trailing lower triangle, column by column
    int J = K + 1, q = p;
    while (q >= 4 - J) {
      q -= 4 - J;
      ++J;
    }
    const int I = J + q;
    d4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = a[(16 * I + gq + 4 * r) * kLd + 16 * J + li];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const double av = -a[(16 * I + li) * kLd + 16 * K + 4 * s4 + gq];
      const double bv = a[(16 * J + li) * kLd + 16 * K + 4 * s4 + gq];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) a[(16 * I + gq + 4 * r) * kLd + 16 * J + li] = acc[r];
  }
}

// Cholesky of the lower triangle of the 64 x 64 tile in LDS, blocked 4 x 4
// on 16-column blocks: for K = 0..3 the diagonal block by the first wave,
// the blocks below it by substitution, then the trailing blocks' update on
// the matrix cores.  The block loop is kept rolled so that the code a
// workgroup runs once per panel stays small (instruction fetch, not
// arithmetic, dominated the fully unrolled form).  Every entry is the
// standard algorithm's inner product in some order.  Called by every thread
// of the workgroup; lt and rinv are 272 doubles of LDS scratch.  Returns
// false, on every thread, when a pivot is not positive and finite; on
// success the lower triangle holds the factor.
__device__ __attribute__((always_inline)) inline bool chol_tile_lds(double* a, double* lt,
                                                                   double* rinv, int* flag) {
#pragma nounroll
  for (int K = 0; K < 4; ++K) {
    if (threadIdx.x < 64) {
      const int ok = chol16_wave(a, lt, rinv, 16 * K);
      if (threadIdx.x == 0) *flag = ok;
    }
    __syncthreads();
    if (!*flag) return false;
    if (K < 3) {
      trsm16_tile(a, lt, rinv, K);
      __syncthreads();
      update16_tile(a, K);
      __syncthreads();
    }
  }
  return true;
}

// tile (row block bi, column block bj) of column-major M <-> row-major LDS
__device__ inline void load_tile(const double* M, int L, int bi, int bj, double* a) {
  const int t = threadIdx.x;
#pragma unroll 4
  for (int u = 0; u < kT * kT / 256; ++u) {
    const int e = t + 256 * u, r = e & 63, c = e >> 6;
    a[r * kLd + c] = M[(size_t)(bi * kT + r) + (size_t)(bj * kT + c) * L];
  }
}

__device__ inline void store_tile(double* M, int L, int bi, int bj, const double* a) {
  const int t = threadIdx.x;
#pragma unroll 4
  for (int u = 0; u < kT * kT / 256; ++u) {
    const int e = t + 256 * u, r = e & 63, c = e >> 6;
    M[(size_t)(bi * kT + r) + (size_t)(bj * kT + c) * L] = a[r * kLd + c];
  }
}

}  // namespace

// ------------------------------------------------------------ formation --
// One workgroup per 64 rows; thread (r = t % 64, g = t / 64) computes the
// columns q = g, g + 4, ... of row r:  U = W + (c/2) Vt - Vt H / 2.
constexpr int kCertMaxM = kMaxM;

__global__ __launch_bounds__(256) void k_cert_prep(const double* __restrict__ V,
                                                   const double* __restrict__ W, int ld,
                                                   const double* __restrict__ H, int ldh, int mt,
                                                   int n, double c, double* __restrict__ U,
                                                   double* __restrict__ part) {
  __shared__ double hs[kCertMaxM * (kCertMaxM + 1)];
  __shared__ double vs[kCertMaxM * kT];  // vs[p * 64 + r]
  __shared__ double red[2 * 256];
  const int t = threadIdx.x, r = t & 63, g = t >> 6;
  const int row = blockIdx.x * kT + r;
  const bool ok = row < n;
  for (int e = t; e < mt * mt; e += 256) {
    const int p = e % mt, q = e / mt;
    hs[p * (kCertMaxM + 1) + q] = H[p + (size_t)q * ldh];
  }
  for (int e = t; e < mt * kT; e += 256) {
    const int rr = e & 63, p = e >> 6;
    const int rw = blockIdx.x * kT + rr;
    vs[p * kT + rr] = (rw < n) ? V[rw + (size_t)p * ld] : 0.0;
  }
  __syncthreads();
  double su = 0.0, sw = 0.0;
  for (int q = g; q < mt; q += 4) {
    const double w = ok ? W[row + (size_t)q * ld] : 0.0;
    double s = 0.0;
    for (int p = 0; p < mt; ++p) s = fma(vs[p * kT + r], hs[p * (kCertMaxM + 1) + q], s);
    const double u = ok ? (w + 0.5 * c * vs[q * kT + r]) - 0.5 * s : 0.0;
    U[row + (size_t)q * ld] = u;
    su = fma(u, u, su);
    sw = fma(w, w, sw);
  }
  red[t] = su;
  red[256 + t] = sw;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      red[t] += red[t + s];
      red[256 + t] += red[256 + t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[2 * blockIdx.x] = red[0];
    part[2 * blockIdx.x + 1] = red[256];
  }
}

// M0 = -A + [Vt U] [U Vt]^T on lower tiles; thread (tr = t % 16, tc = t / 16)
// owns rows 4 tr .. 4 tr + 3 and columns 4 tc .. 4 tc + 3 of the tile.  The
// rank-2m~ inner dimension is staged in LDS in chunks of 32, k-major.
constexpr int kFK = 32;

__global__ __launch_bounds__(256) void k_cert_form(const double* __restrict__ A, int lda,
                                                   const double* __restrict__ V,
                                                   const double* __restrict__ U, int ld, int mt,
                                                   int n, int L, double* __restrict__ M,
                                                   double* __restrict__ diag_part) {
  __shared__ __align__(16) double pt[kFK * kT];
  __shared__ __align__(16) double qt[kFK * kT];
  __shared__ double red[256];
  int bi, bj;
  tri_index(blockIdx.x, bi, bj);
  const int t = threadIdx.x, tr = t & 15, tc = t >> 4;
  const int i0 = bi * kT, j0 = bj * kT;
  double acc[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) acc[a][b] = -A[(size_t)(i0 + 4 * tr + a) + (size_t)(j0 + 4 * tc + b) * lda];
  const int K = 2 * mt;
  for (int k0 = 0; k0 < K; k0 += kFK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kFK * kT / 256; ++u) {
      const int e = t + 256 * u, r = e & 63, kk = e >> 6, k = k0 + kk;
      double pv = 0.0, qv = 0.0;
      if (k < mt) {
        pv = V[(size_t)(i0 + r) + (size_t)k * ld];
        qv = U[(size_t)(j0 + r) + (size_t)k * ld];
      } else if (k < K) {
        pv = U[(size_t)(i0 + r) + (size_t)(k - mt) * ld];
        qv = V[(size_t)(j0 + r) + (size_t)(k - mt) * ld];
      }
      pt[kk * kT + r] = pv;
      qt[kk * kT + r] = qv;
    }
    __syncthreads();
    const int kn = min(kFK, K - k0);
    for (int kk = 0; kk < kn; ++kk) {
      const double2 p01 = *(const double2*)&pt[kk * kT + 4 * tr];
      const double2 p23 = *(const double2*)&pt[kk * kT + 4 * tr + 2];
      const double2 q01 = *(const double2*)&qt[kk * kT + 4 * tc];
      const double2 q23 = *(const double2*)&qt[kk * kT + 4 * tc + 2];
      const double p[4] = {p01.x, p01.y, p23.x, p23.y};
      const double q[4] = {q01.x, q01.y, q23.x, q23.y};
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int a = 0; a < 4; ++a) acc[a][b] = fma(p[a], q[b], acc[a][b]);
    }
  }
  double dsum = 0.0;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = i0 + 4 * tr + a, j = j0 + 4 * tc + b;
      double v = acc[a][b];
      if (i >= n || j >= n) v = (i == j) ? 1.0 : 0.0;
      else if (i == j) dsum += v;
      M[(size_t)i + (size_t)j * L] = v;
    }
  if (bi == bj) {
    red[t] = dsum;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) red[t] += red[t + s];
      __syncthreads();
    }
    if (t == 0) diag_part[bi] = red[0];
  }
}

// ------------------------------------------------------------- margins ---
__device__ inline double gam(double k) {
  const double u = 1.1102230246251565e-16;  // 2^-53
  return k * u / (1.0 - k * u);
}

__global__ __launch_bounds__(256) void k_cert_shift(const double* __restrict__ G, int ldg,
                                                    const double* __restrict__ prep_part, int nprep,
                                                    const double* __restrict__ diag_part,
                                                    double* __restrict__ M, CertState* cs) {
  __shared__ double red[4 * 256];
  __shared__ double s_shift;
  const int t = threadIdx.x;
  const int n = cs->n, L = cs->L, mt = cs->mt, T = L / kT;
  double tr = 0.0, su = 0.0, sw = 0.0, sv = 0.0, sp = 0.0;
  for (int b = t; b < T; b += 256) tr += diag_part[b];
  for (int b = t; b < nprep; b += 256) {
    su += prep_part[2 * b];
    sw += prep_part[2 * b + 1];
  }
  for (int e = t; e < mt * mt; e += 256) {
    const int p = e % mt, q = e / mt;
    const double gv = G[p + (size_t)q * ldg];
    if (p == q) sv += gv;
    const double d = gv - (p == q ? 1.0 : 0.0);
    sp = fma(d, d, sp);
  }
  red[t] = tr;
  red[256 + t] = su;
  red[512 + t] = sw;
  red[768 + t] = sv;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      red[t] += red[t + s];
      red[256 + t] += red[256 + t + s];
      red[512 + t] += red[512 + t + s];
      red[768 + t] += red[768 + t + s];
    }
    __syncthreads();
  }
  const double trace = red[0], ufro2 = red[256], wfro2 = red[512], vfro2 = red[768];
  __syncthreads();
  red[t] = sp;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  if (t == 0) {
    const double phi = sqrt(red[0]);
    const double fa = cs->fro_a, c = cs->c;
    const double vn = sqrt(fmax(vfro2, 0.0)), wn = sqrt(fmax(wfro2, 0.0));
    const double f = (1.0 + phi) * (1.0 + phi);
    // every term but the factorization's does not depend on delta
    const double e_form = gam(2.0 * mt + 1.0) * (fa + vfro2 + ufro2);
    const double e_w = 3.0 * gam((double)n) * fa * vn * f + gam((double)n) * vn * wn * f +
                       2.0 * (1.0 + phi) * gam(mt + 2.0) * (wn + 0.5 * vn * wn * (1.0 + phi) + 0.5 * c * vn);
    const double e_orth = (2.0 * phi + phi * phi) * fa + c * phi;
    const double gl = gam(L + 8.0);
    double delta = cs->delta, eta = 0.0;
    for (int it = 0; it < 3; ++it) {
      const double tr_m = fmax(trace + n * delta + (double)(L - n), 0.0);
      const double e_chol = gl * tr_m / (1.0 - gl);
      const double e_diag = 1.1102230246251565e-16 * (fa + c + delta);
      eta = 2.0 * (e_chol + e_form + e_w + e_orth + e_diag);
      if (delta < 4.0 * eta) delta = 4.0 * eta;
    }
    cs->trace = trace;
    cs->ufro2 = ufro2;
    cs->wfro2 = wfro2;
    cs->vfro2 = vfro2;
    cs->phi = phi;
    cs->eta = eta;
    cs->delta_eff = delta;
    cs->shift = delta - eta;
    s_shift = delta - eta;
    if (!(trace + n * delta + (double)(L - n) > 0.0)) cs->fail = -2;
  }
  __syncthreads();
  const double sh = s_shift;
  for (int i = t; i < n; i += 256) M[(size_t)i + (size_t)i * L] += sh;
}

// ----------------------------------------------------------- Cholesky ----
__global__ __launch_bounds__(256) void k_chol_diag(double* __restrict__ M, int L, int k,
                                                   CertState* cs) {
  if (cert_failed(cs)) return;
  __shared__ double a[kT * kLd];
  __shared__ double lt[16 * 16 + 16];
  __shared__ int flag;
  const long long t0 = wall_clock64();
  load_tile(M, L, k, k, a);
  __syncthreads();
  const long long t1 = wall_clock64();
  if (!chol_tile_lds(a, lt, lt + 256, &flag)) {
    if (threadIdx.x == 0) cs->fail = 1 + k;
    return;
  }
  const long long t2 = wall_clock64();
  store_tile(M, L, k, k, a);
  if (threadIdx.x == 0) {
    cs->t_diag[0] = t0;
    cs->t_diag[1] = t1;
    cs->t_diag[2] = t2;
    cs->t_diag[3] = wall_clock64();
  }
}

// L_ik = A_ik L_kk^{-T} for the row blocks i > k, sixteen rows per
// workgroup: the sixteen lanes of a row each own four of its columns (lane g
// of the row: columns 4g .. 4g + 3).  At column c the owning lane forms
// x_c = a_c / l_cc by the rounded reciprocal, the row's lanes receive it by a
// DPP row broadcast and update their columns q > c with l_qc, read from L_kk staged
// transposed in LDS and zero on and above its diagonal (so every lane
// applies every update unconditionally).  The arithmetic is the column-
// ordered substitution of the standard algorithm.
__global__ __launch_bounds__(256) void k_chol_trsm(double* __restrict__ M, int L, int k,
                                                   CertState* cs) {
  if (cert_failed(cs)) return;
  __shared__ __align__(16) double lt[kT * kT];  // lt[c * 64 + q] = L_kk(q, c), q > c
  __shared__ double rinv[kT];
  const int t = threadIdx.x;
  const int g = t & 15;  // this lane's place in its sixteen-lane DPP row
  const int row = (k + 1) * kT + blockIdx.x * 16 + (t >> 4);
  double* rowp = M + (size_t)row + (size_t)(k * kT + 4 * g) * L;
  double x[4], rv[4];
  // the row's loads and all of L_kk's are issued before any is used
#pragma unroll
  for (int q = 0; q < 4; ++q) x[q] = rowp[(size_t)q * L];
  {
    const double* src = M + (size_t)(k * kT) + (size_t)(k * kT) * L;
    constexpr int U = kT * kT / 256;
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = t + 256 * u, q = e & 63, c = e >> 6;
      v[u] = src[q + (size_t)c * L];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = t + 256 * u, q = e & 63, c = e >> 6;
      if (q == c) rinv[c] = 1.0 / v[u];
      lt[c * kT + q] = (q > c) ? v[u] : 0.0;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) rv[q] = rinv[4 * g + q];
#pragma unroll
  for (int c = 0; c < kT; ++c) {
    const int own = c >> 2, qq = c & 3;
    const double v = row_bcast_n(x[qq] * rv[qq], own);
    x[qq] = (g == own) ? v : x[qq];
    const double2 w0 = *(const double2*)(lt + c * kT + 4 * g);
    const double2 w1 = *(const double2*)(lt + c * kT + 4 * g + 2);
    x[0] = fma(-v, w0.x, x[0]);
    x[1] = fma(-v, w0.y, x[1]);
    x[2] = fma(-v, w1.x, x[2]);
    x[3] = fma(-v, w1.y, x[3]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) rowp[(size_t)q * L] = x[q];
}

// Trailing update A_ij -= L_ik L_jk^T for k < j <= i; workgroup 0 takes the
// tile (k + 1, k + 1) and then factors it (one-panel lookahead).
__global__ __launch_bounds__(256) void k_chol_syrk(double* __restrict__ M, int L, int k,
                                                   CertState* cs) {
  if (cert_failed(cs)) return;
  __shared__ __align__(16) double sm[2 * kT * kT];
  int* flag = (int*)(sm + kT * kLd);
  double* lt = sm + kT * kLd + 8;  // 256 + 16 doubles: L_KK^T and 1 / l_ii
  double* pt = sm;            // pt[q * 64 + r] = L_ik(r, q)
  double* qt = sm + kT * kT;  // qt[q * 64 + c] = L_jk(c, q)
  int ii, jj;
  tri_index(blockIdx.x, ii, jj);
  const int bi = k + 1 + ii, bj = k + 1 + jj;
  const int i0 = bi * kT, j0 = bj * kT, k0 = k * kT;
  const int t = threadIdx.x, tr = t & 15, tc = t >> 4;
  // every global load (both panel tiles and the target tile) is issued
  // before the first is used
  constexpr int U = kT * kT / 256;
  double pv[U], qv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = t + 256 * u, r = e & 63, q = e >> 6;
    pv[u] = M[(size_t)(i0 + r) + (size_t)(k0 + q) * L];
    qv[u] = M[(size_t)(j0 + r) + (size_t)(k0 + q) * L];
  }
  double acc[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) acc[a][b] = M[(size_t)(i0 + 4 * tr + a) + (size_t)(j0 + 4 * tc + b) * L];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = t + 256 * u, r = e & 63, q = e >> 6;
    pt[q * kT + r] = pv[u];
    qt[q * kT + r] = qv[u];
  }
  __syncthreads();
#pragma unroll 4
  for (int q = 0; q < kT; ++q) {
    const double2 p01 = *(const double2*)&pt[q * kT + 4 * tr];
    const double2 p23 = *(const double2*)&pt[q * kT + 4 * tr + 2];
    const double2 q01 = *(const double2*)&qt[q * kT + 4 * tc];
    const double2 q23 = *(const double2*)&qt[q * kT + 4 * tc + 2];
    const double p[4] = {p01.x, p01.y, p23.x, p23.y};
    const double w[4] = {q01.x, q01.y, q23.x, q23.y};
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int a = 0; a < 4; ++a) acc[a][b] = fma(-p[a], w[b], acc[a][b]);
  }
  if (blockIdx.x != 0) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int a = 0; a < 4; ++a) M[(size_t)(i0 + 4 * tr + a) + (size_t)(j0 + 4 * tc + b) * L] = acc[a][b];
    return;
  }
  // lookahead: the updated diagonal tile (k + 1, k + 1) is factored here
  double* a = sm;  // 64 x 65 row-major, over pt (no longer read)
  __syncthreads();
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int q = 0; q < 4; ++q) a[(4 * tr + q) * kLd + 4 * tc + b] = acc[q][b];
  __syncthreads();
  if (!chol_tile_lds(a, lt, lt + 256, flag)) {
    if (t == 0) cs->fail = 1 + bi;
    return;
  }
  store_tile(M, L, bi, bi, a);
}

// ------------------------------------------------------------- launch ----
hipError_t launch_cert_prep(const double* V, const double* W, int ld, const double* H, int ldh,
                            int mt, int n, int L, double c, double* U, double* part,
                            hipStream_t st) {
  if (mt <= 0) return hipSuccess;
  if (mt > kCertMaxM) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cert_prep, dim3(L / kT), dim3(256), 0, st, V, W, ld, H, ldh, mt, n, c, U,
                     part);
  return hipGetLastError();
}

hipError_t launch_cert_form(const double* A, int lda, const double* V, const double* U, int ld,
                            int mt, int n, int L, double* M, double* diag_part, hipStream_t st) {
  if (L % kT != 0 || mt < 0) return hipErrorInvalidValue;
  const int T = L / kT;
  hipLaunchKernelGGL(k_cert_form, dim3(T * (T + 1) / 2), dim3(256), 0, st, A, lda, V, U, ld, mt,
                     n, L, M, diag_part);
  return hipGetLastError();
}

hipError_t launch_cert_shift(const double* G, int ldg, const double* prep_part, int nprep,
                             const double* diag_part, double* M, CertState* cs, hipStream_t st) {
  hipLaunchKernelGGL(k_cert_shift, dim3(1), dim3(256), 0, st, G, ldg, prep_part, nprep, diag_part,
                     M, cs);
  return hipGetLastError();
}

hipError_t launch_cert_chol(double* M, int L, CertState* cs, hipStream_t st) {
  if (L % kT != 0 || L <= 0) return hipErrorInvalidValue;
  const int T = L / kT;
  hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, st, M, L, 0, cs);
  for (int k = 0; k + 1 < T; ++k) {
    const int R = T - k - 1;
    hipLaunchKernelGGL(k_chol_trsm, dim3(4 * R), dim3(256), 0, st, M, L, k, cs);
    hipLaunchKernelGGL(k_chol_syrk, dim3(R * (R + 1) / 2), dim3(256), 0, st, M, L, k, cs);
  }
  return hipGetLastError();
}

}  // namespace psdp
