// Device body of the one-workgroup Rayleigh-Ritz step (tridiagonalization,
// multisection, inverse iteration, back-transformation); included by the
// single-cone kernel and the batched persistent kernel.
#pragma once
#include <algorithm>

#include "common.h"

namespace psdp {


constexpr int kTriThreads = 256;
constexpr int kFullMaxN = 112;  // full storage of H up to this order

__device__ inline int tri_row2(int e) {
  int r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= e) ++r;
  while (r * (r + 1) / 2 > e) --r;
  return r;
}

template <bool FULL>
struct SymStore {
  double* a;
  int ld;
  __device__ inline double& at(int i, int j) const {  // any (i, j)
    if (FULL) return a[i + (size_t)j * ld];
    return (i >= j) ? a[i * (i + 1) / 2 + j] : a[j * (j + 1) / 2 + i];
  }
  __device__ inline double& low(int i, int j) const {  // i >= j
    if (FULL) return a[i + (size_t)j * ld];
    return a[i * (i + 1) / 2 + j];
  }
};

// Sum over the 64 lanes of a wave, result in every lane: DPP within rows
// of 16 lanes (quad permutes and mirrors), a swizzle across the two rows of
// each half, and two lane reads across the halves.
template <int CTRL>
__device__ inline double dpp_d(double v) {
  int2 x = __builtin_bit_cast(int2, v);
  x.x = __builtin_amdgcn_mov_dpp(x.x, CTRL, 0xF, 0xF, false);
  x.y = __builtin_amdgcn_mov_dpp(x.y, CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, x);
}
__device__ inline double wave_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
  v += dpp_d<0x141>(v);  // row_half_mirror: the other quad of each 8
  v += dpp_d<0x140>(v);  // row_mirror: the other 8 of each 16
  int2 x = __builtin_bit_cast(int2, v);
  x.x = __builtin_amdgcn_ds_swizzle(x.x, 0x401F);  // lane ^ 16 within 32
  x.y = __builtin_amdgcn_ds_swizzle(x.y, 0x401F);
  v += __builtin_bit_cast(double, x);
  int2 y = __builtin_bit_cast(int2, v);
  int2 lo, hi;
  lo.x = __builtin_amdgcn_readlane(y.x, 0);
  lo.y = __builtin_amdgcn_readlane(y.y, 0);
  hi.x = __builtin_amdgcn_readlane(y.x, 32);
  hi.y = __builtin_amdgcn_readlane(y.y, 32);
  return __builtin_bit_cast(double, lo) + __builtin_bit_cast(double, hi);
}

// a / b through the hardware reciprocal and one Newton step (relative error
// a few units in the last place; used in the Sturm and inverse-iteration
// recurrences, where the result only steers inertia counts and directions)
__device__ inline double fast_div(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  r = fma(fma(-b, r, 1.0), r, r);
  return a * r;
}

// number of eigenvalues of T (d, e2 = e^2) below x, LDL^T inertia with a
// floor on the pivots
__device__ inline int sturm_count(const double* d, const double* e2, int N, double x,
                                  double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += (q < 0.0);
  for (int i = 1; i < N; ++i) {
    q = d[i] - x - fast_div(e2[i - 1], q);
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

// One inverse-iteration solve (T - sigma I) y_new = y: Gaussian elimination
// with partial pivoting fused with the forward substitution, U's three
// diagonals in U0/U1/U2 (stride us between entries), then back
// substitution.  Pivots below pfloor in magnitude are replaced by pfloor.
__device__ inline void tri_solve(const double* d, const double* e, int N, double sigma,
                                 double pfloor, double* y, double* U0, double* U1, double* U2,
                                 size_t us) {
  double di = d[0] - sigma;                 // current row i: (di, ui) after elimination
  double ui = (N > 1) ? e[0] : 0.0;
  double bi = y[0];
  for (int i = 0; i + 1 < N; ++i) {
    const double li = e[i];                 // entry (i+1, i)
    const double dn = d[i + 1] - sigma;     // entry (i+1, i+1)
    const double un = (i + 2 < N) ? e[i + 1] : 0.0;  // entry (i+1, i+2)
    const double bn = y[i + 1];
    if (fabs(di) >= fabs(li)) {
      const double piv = (di == 0.0) ? pfloor : di;
      const double f = fast_div(li, piv);
      U0[i * us] = piv;
      U1[i * us] = ui;
      U2[i * us] = 0.0;
      y[i] = bi;
      di = dn - f * ui;
      ui = un;
      bi = bn - f * bi;
    } else {
      // interchange rows i and i+1
      const double f = fast_div(di, li);
      U0[i * us] = li;
      U1[i * us] = dn;
      U2[i * us] = un;
      y[i] = bn;
      di = ui - f * dn;
      ui = -f * un;
      bi = bi - f * bn;
    }
  }
  if (fabs(di) < pfloor) di = (di < 0.0) ? -pfloor : pfloor;
  U0[(size_t)(N - 1) * us] = di;
  y[N - 1] = bi / di;
  for (int i = N - 2; i >= 0; --i) {
    double u0 = U0[i * us];
    if (fabs(u0) < pfloor) u0 = (u0 < 0.0) ? -pfloor : pfloor;
    double s = y[i] - U1[i * us] * y[i + 1];
    if (i + 2 < N) s -= U2[i * us] * y[i + 2];
    y[i] = fast_div(s, u0);
  }
}

// Body shared by the single-cone kernel and the batched persistent kernel:
// `lds` is the dynamic LDS (a.lds_cap doubles), `sh` the small static
// arrays, 256 threads.
template <bool FULL>
__device__ inline void rr_tri_body(const RRArgs& a, double* lds, const RRShared& sh) {
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
  const size_t hsz = FULL ? (size_t)N * N : (size_t)N * (N + 1) / 2;
  double* Hraw = lds;
  double* d = Hraw + hsz;         // N
  double* e = d + N;              // N (sub-diagonal)
  double* e2 = e + N;             // N
  double* tau = e2 + N;           // N
  double* pv = tau + N;           // N (p, then w; then the Ritz values)
  double* vbuf = pv + N;          // N (current reflector)
  double* wbuf = vbuf + N;        // 4 N (per-wave w)
  double* part = wbuf + 4 * N;    // 4 N (per-wave partial products)
  const int ldy = N + 1;          // odd leading dimension: lanes over columns
  double* Y = part + 4 * N;       // ldy x mk eigenvectors, column-major
  int* cnts = (int*)(Y + (size_t)ldy * mk);           // nt ints
  double* ufac = (double*)(cnts + nt + (nt & 1));     // 3 N mk in LDS when it fits
  const bool fac_lds = a.lds_cap >= (size_t)(ufac - lds) + 3 * (size_t)N * mk;
  SymStore<FULL> H{Hraw, N};
  if (tid == 0) st->t_phase[0] = wall_clock64();
  if (FULL) {
    for (int x = tid; x < N * N; x += nt) {
      int i = x % N, j = x / N;
      Hraw[x] = 0.5 * (a.K[i + (size_t)j * a.ldk] + a.K[j + (size_t)i * a.ldk]);
    }
  } else {
    for (int x = tid; x < N * (N + 1) / 2; x += nt) {
      int i = tri_row2(x), j = x - i * (i + 1) / 2;
      Hraw[x] = 0.5 * (a.K[i + (size_t)j * a.ldk] + a.K[j + (size_t)i * a.ldk]);
    }
  }
  __syncthreads();

  // ---- 1. tridiagonalization: lanes over rows, the four waves over column
  // segments of each step.  Per step: every wave forms the reflector v
  // (redundantly), partial products of its column segment go to LDS
  // (barrier), every wave combines them into p and w = p - (t/2)(p.v) v in
  // its own copy, then updates its column segment of the trailing rows
  // (barrier).  Reflectors stay in column k.
  {
    const int nw = nt / 64;
    double* __restrict__ vv = vbuf;                  // N, written by wave 0
    double* __restrict__ ww = wbuf + (size_t)wv * N; // per-wave copy of w
    double* __restrict__ pp = part;                  // nw x N partial products
    for (int k = 0; k + 2 < N; ++k) {
      const int m = N - k - 1;
      double xs = 0.0;
      for (int i = k + 2 + lane; i < N; i += 64) {
        const double x = H.low(i, k);
        xs += x * x;
      }
      const double xnorm2 = wave_sum(xs);
      const double alpha = H.low(k + 1, k);
      double t = 0.0, beta = alpha, scale = 0.0;
      if (xnorm2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
        t = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      // the reflector, in registers of every wave and in vv (wave 0 writes)
      if (t == 0.0) {
        // column k is already reduced: no reflection (same decision in
        // every wave, so the whole workgroup skips the step)
        if (wv == 0 && lane == 0) { tau[k] = 0.0; e[k] = beta; }
        continue;
      }
      const int seg = (m + nw - 1) / nw;
      const int j0 = k + 1 + wv * seg, j1 = min(N, j0 + seg);
      for (int i = k + 1 + lane; i < N; i += 64) {
        const double v = (i == k + 1) ? 1.0 : H.low(i, k) * scale;
        if (wv == 0) vv[i] = v;
      }
      __syncthreads();  // vv complete; everybody has read column k
      if (wv == 0) {
        for (int i = k + 1 + lane; i < N; i += 64) H.low(i, k) = vv[i];
        if (lane == 0) { tau[k] = t; e[k] = beta; }
      }
      // partial products over this wave's column segment
      for (int i = k + 1 + lane; i < N; i += 64) {
        double s0 = 0.0, s1 = 0.0;
        int j = j0;
        for (; j + 1 < j1; j += 2) {
          s0 += H.at(i, j) * vv[j];
          s1 += H.at(i, j + 1) * vv[j + 1];
        }
        if (j < j1) s0 += H.at(i, j) * vv[j];
        pp[(size_t)wv * N + i] = s0 + s1;
      }
      __syncthreads();
      // p and w for all rows, in this wave's copy
      double dp = 0.0;
      for (int i = k + 1 + lane; i < N; i += 64) {
        double sum = 0.0;
        for (int q = 0; q < nw; ++q) sum += pp[(size_t)q * N + i];
        const double p = t * sum;
        ww[i] = p;
        dp += p * vv[i];
      }
      const double al = -0.5 * t * wave_sum(dp);
      for (int i = k + 1 + lane; i < N; i += 64) ww[i] += al * vv[i];
      __threadfence_block();
      // A22 -= v w^T + w v^T on this wave's column segment (both triangles
      // when stored full, the lower one otherwise)
      for (int i = k + 1 + lane; i < N; i += 64) {
        const double vi = vv[i], wi = ww[i];
        const int jb = j0, je = FULL ? j1 : min(j1, i + 1);
        for (int j = jb; j < je; ++j) H.at(i, j) -= vi * ww[j] + wi * vv[j];
      }
      __syncthreads();
    }
  }
  if (wv == 0) {
    for (int i = lane; i < N; i += 64) d[i] = H.low(i, i);
    if (lane == 0 && N >= 2) { e[N - 2] = H.low(N - 1, N - 2); tau[N - 2] = 0.0; }
    __threadfence_block();
    for (int i = lane; i + 1 < N; i += 64) e2[i] = e[i] * e[i];
    __threadfence_block();
    if (lane == 0) {
      double tn = 0.0, emax2 = 0.0;
      for (int i = 0; i < N; ++i) {
        double r = fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < N ? fabs(e[i]) : 0.0);
        tn = fmax(tn, r);
        if (i + 1 < N) emax2 = fmax(emax2, e2[i]);
      }
      s_tnorm = tn;
      s_pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
    }
  }
  __syncthreads();
  const double tnorm = s_tnorm, pivmin = s_pivmin;
  if (tid == 0) st->t_phase[1] = wall_clock64();

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
    if (tid == nt - 1) s_npos = N - sturm_count(d, e2, N, 0.0, pivmin);
    __syncthreads();
    const int per = max(1, nt / max(mk, 1));
    const int j_me = tid / per, s_me = tid % per;
    for (int round = 0; round < 48; ++round) {
      // the shifts only need to be close for inverse iteration; the values
      // come from Rayleigh quotients afterwards
      bool done = true;
      for (int j = 0; j < mk; ++j) {
        double w = s_hi[j] - s_lo[j];
        double tolj = 1e-12 * tnorm + 8.8e-16 * fmax(fabs(s_lo[j]), fabs(s_hi[j])) + 4.0 * pivmin;
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
        for (int s2 = 0; s2 < per; ++s2) {
          double x = lo + (hi - lo) * (double)(s2 + 1) / (double)(per + 1);
          if (cnts[j * per + s2] <= target) nlo = x;
          else { nhi = x; break; }
        }
        s_lo[j] = nlo;
        s_hi[j] = nhi;
      }
      __syncthreads();
    }
  }
  if (tid == 0) st->t_phase[2] = wall_clock64();

  // ---- 3. inverse iteration (one lane per vector; mk <= 64 so all lanes
  // are in wave 0), Gram-Schmidt inside clusters by the same wave
  const double pfloor = fmax(2.2e-16 * tnorm, 1e-300);
  const double ortol = 1e-3 * tnorm;
  if (wv == 0) {
    for (int j = lane; j < mk; j += 64)
      for (int i = 0; i < N; ++i) Y[i + (size_t)j * ldy] = start_entry(i, j);
    __threadfence_block();
    for (int itn = 0; itn < 2; ++itn) {
      for (int j = lane; j < mk; j += 64) {
        const double sigma = 0.5 * (s_lo[j] + s_hi[j]);
        double* y = Y + (size_t)j * ldy;
        double *U0, *U1, *U2;
        size_t us;
        if (fac_lds) {
          U0 = ufac + (size_t)j * 3 * N; U1 = U0 + N; U2 = U1 + N; us = 1;
        } else {
          U0 = a.scratch + j; U1 = U0 + (size_t)N * mk; U2 = U1 + (size_t)N * mk; us = mk;
        }
        tri_solve(d, e, N, sigma, pfloor, y, U0, U1, U2, us);
        double mx = 0.0;
        for (int i = 0; i < N; ++i) mx = fmax(mx, fabs(y[i]));
        const double sc = mx > 0.0 ? 1.0 / mx : 1.0;
        double nn = 0.0;
        for (int i = 0; i < N; ++i) { y[i] *= sc; nn += y[i] * y[i]; }
        const double inv = 1.0 / sqrt(nn);
        for (int i = 0; i < N; ++i) y[i] *= inv;
      }
      __threadfence_block();
      for (int j = 1; j < mk; ++j) {
        const double mid_j = 0.5 * (s_lo[j] + s_hi[j]);
        const double mid_p = 0.5 * (s_lo[j - 1] + s_hi[j - 1]);
        if (mid_p - mid_j > ortol) continue;
        int c0 = j - 1;
        while (c0 > 0 && 0.5 * (s_lo[c0 - 1] + s_hi[c0 - 1]) - 0.5 * (s_lo[c0] + s_hi[c0]) <= ortol)
          --c0;
        double* yj = Y + (size_t)j * ldy;
        for (int i0 = c0; i0 < j; ++i0) {
          const double* yi = Y + (size_t)i0 * ldy;
          double dp = 0.0;
          for (int r = lane; r < N; r += 64) dp += yi[r] * yj[r];
          dp = wave_sum(dp);
          for (int r = lane; r < N; r += 64) yj[r] -= dp * yi[r];
          __threadfence_block();
        }
        double nn = 0.0;
        for (int r = lane; r < N; r += 64) nn += yj[r] * yj[r];
        nn = wave_sum(nn);
        const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        for (int r = lane; r < N; r += 64) yj[r] *= inv;
        __threadfence_block();
      }
    }
    // Rayleigh quotients y^T T y
    for (int j = lane; j < mk; j += 64) {
      const double* y = Y + (size_t)j * ldy;
      double rq = 0.0;
      for (int i = 0; i < N; ++i) {
        double ty = d[i] * y[i];
        if (i > 0) ty += e[i - 1] * y[i - 1];
        if (i + 1 < N) ty += e[i] * y[i + 1];
        rq += y[i] * ty;
      }
      pv[j] = rq;
    }
  }
  __syncthreads();
  if (tid == 0) st->t_phase[3] = wall_clock64();

  // ---- 4. back-transformation Z = H_0 ... H_{N-3} Y.  Columns are
  // independent: each column is owned by a group of 8 lanes of one wave
  // (row segments), reflectors applied in order with a 3-step shuffle sum.
  {
    const int g = lane >> 3, sl = lane & 7;  // 8 groups of 8 lanes per wave
    const int ncg = (nt / 64) * 8;           // column groups in the workgroup
    for (int j = wv * 8 + g; j - g < mk; j += ncg) {
      const bool act = j < mk;
      double* __restrict__ y = Y + (size_t)(act ? j : 0) * ldy;
      for (int k = N - 3; k >= 0; --k) {
        const double t = tau[k];
        if (t == 0.0) continue;
        double dp = 0.0;
        if (act)
          for (int r = k + 1 + sl; r < N; r += 8) dp += H.low(r, k) * y[r];
        dp += __shfl_xor(dp, 1, 64);
        dp += __shfl_xor(dp, 2, 64);
        dp += __shfl_xor(dp, 4, 64);
        dp *= t;
        if (act)
          for (int r = k + 1 + sl; r < N; r += 8) y[r] -= dp * H.low(r, k);
      }
    }
  }
  __syncthreads();
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
