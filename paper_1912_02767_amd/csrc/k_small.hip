// One-workgroup kernels on the small (<= 192 x 192) matrices of one
// LOBPCG iteration:
//   k_decide_chol : convergence / stall / expansion decisions, active set,
//                   and Cholesky-QR with column dropping of the trial basis
//                   (paper §5.1: Cholesky QR instead of Householder QR)
//   k_rr          : Rayleigh-Ritz on an orthonormal basis (paper §5, Alg. 2):
//                   parallel cyclic Jacobi on H = S^T A S in LDS, selection of
//                   the largest Ritz values, eigenvectors by replaying the
//                   rotation log on unit vectors.
#include <algorithm>

#include "common.h"

namespace psdp {

constexpr int kSmallThreads = 512;
constexpr int kRRThreads = 256;
static int g_lds_limit = 56 * 1024;  // dynamic LDS bytes per workgroup (set at init)

__device__ inline double block_sum(double v, double* red) {
  // red: kSmallThreads / 64 doubles of LDS
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  int nw = blockDim.x / 64;
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

__device__ inline double block_max(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = -INFINITY;
  int nw = blockDim.x / 64;
  for (int i = 0; i < nw; ++i) s = fmax(s, red[i]);
  __syncthreads();
  return s;
}

// e -> (row, col) of a packed triangle: row r with r(r+1)/2 <= e < (r+1)(r+2)/2
__device__ inline int tri_row(int e) {
  int r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= e) ++r;
  while (r * (r + 1) / 2 > e) --r;
  return r;
}

// packed lower triangle, row-major: (i, j) with j <= i  ->  i(i+1)/2 + j
__device__ inline int plo(int i, int j) { return i * (i + 1) / 2 + j; }
// packed upper triangle, column-major: (i, j) with i <= j  ->  j(j+1)/2 + i
__device__ inline int pup(int i, int j) {
  return (i <= j) ? (j * (j + 1) / 2 + i) : (i * (i + 1) / 2 + j);
}



// Dynamic LDS: packed lower triangle of the scaled Gram (N(N+1)/2 doubles)
// + row buffer (N) + scale (N) + misc.
__global__ __launch_bounds__(kSmallThreads) void k_decide_chol(DecideArgs a) {
  extern __shared__ double lds[];
  __shared__ double red[kSmallThreads / 64];
  __shared__ int s_list[kMaxN];   // logical trial column -> candidate index in G
  __shared__ int s_kind[kMaxN];
  __shared__ int s_col[kMaxN];
  __shared__ int s_keep[kMaxN];
  __shared__ int s_N, s_Np, s_nx, s_stop;
  State* st = a.st;
  const int tid = threadIdx.x;
  const int m = a.m;

  if (a.mode == kModeFull || a.mode == kModeXR || a.mode == kModeEval) {
    // ---- decisions from the residual norms (paper §5.2 / §6 stopping rule)
    if (tid < m) st->rnorm[tid] = sqrt(fmax(a.G[(m + tid) + (size_t)(m + tid) * a.ldg], 0.0));
    __syncthreads();
    if (tid == 0) {
      double tol = st->tol;
      int npos = 0;
      for (int i = 0; i < m; ++i) npos += (st->theta[i] > 0.0);
      st->npos_blk = npos;
      double rmax = 0.0, rfro = 0.0;
      for (int i = 0; i < npos; ++i) {
        rmax = fmax(rmax, st->rnorm[i]);
        rfro += st->rnorm[i] * st->rnorm[i];
      }
      st->res_max_pos = rmax;
      st->res_fro_pos = sqrt(rfro);
      st->theta_min_pos = npos > 0 ? st->theta[npos - 1] : 0.0;
      int stop = kRunning;
      bool nonfin = !isfinite(rfro);
      for (int i = 0; i < m; ++i) nonfin |= !isfinite(st->theta[i]) || !isfinite(st->rnorm[i]);
      // guard: largest non-positive Ritz pair, resolved to half its gap
      double q;  // progress metric, <= 1 when converged
      bool guard_ok = false;
      if (npos < m) {
        int g = npos;
        double delta = npos > 0 ? (st->theta[npos - 1] - st->theta[g]) : fabs(st->theta[g]);
        double gtol = fmax(tol, 0.5 * delta);
        st->guard_theta = st->theta[g];
        st->guard_res = st->rnorm[g];
        guard_ok = st->rnorm[g] <= gtol;
        q = fmax(rmax / tol, st->rnorm[g] / gtol);
      } else {
        st->guard_theta = NAN;
        st->guard_res = NAN;
        q = rmax / tol;
      }
      // Below FP64 the products carry rounding noise of order u_p ||A||, so
      // counts of positive Ritz values near zero are unreliable: expansion
      // decisions are left to the FP64 phase and a low-precision phase that
      // asks for one ends as stalled.
      const bool lowp = a.phase_lowprec != 0;
      if (nonfin) {
        stop = kNonFinite;
      } else if (st->expand_req) {
        stop = lowp ? kStalled : kExpand;
      } else if (npos == m && rmax <= tol) {
        stop = lowp ? kStalled : kExpand;  // no room left for a non-positive guard pair
      } else if (rmax <= tol && guard_ok) {
        stop = kConverged;
      } else {
        // stalled: no 10% progress within the window; in FP64 a newly found
        // positive pair counts as progress even when the residual jumps
        if ((!lowp && npos != st->last_npos) || q < 0.9 * st->best_res) {
          st->best_res = q;
          st->best_iter = st->iter;
          st->last_npos = npos;
        } else if (st->iter - st->best_iter >= st->stall_window) {
          stop = kStalled;
        }
      }
      st->eval_stop = stop;
      if (a.mode == kModeEval) stop = kEvaluated;
      st->stop = stop;
      s_stop = stop;
      // logical trial basis: X, then active R, then active P
      int N = 0;
      for (int i = 0; i < m; ++i) { s_list[N] = i; s_kind[N] = 0; s_col[N] = i; ++N; }
      if (stop == kRunning) {
        for (int i = 0; i < m; ++i)
          if (st->rnorm[i] > tol) { s_list[N] = m + i; s_kind[N] = 1; s_col[N] = i; ++N; }
        if (a.has_p && a.mode == kModeFull)
          for (int i = 0; i < m; ++i)
            if (st->rnorm[i] > tol) { s_list[N] = 2 * m + i; s_kind[N] = 2; s_col[N] = i; ++N; }
      }
      s_N = N;
    }
    __syncthreads();
    if (s_stop != kRunning) return;
  } else if (a.mode == kModeXOnly || a.mode == kModeXZ) {
    if (tid == 0) {
      int N = 0;
      for (int i = 0; i < m; ++i) { s_list[N] = i; s_kind[N] = 0; s_col[N] = i; ++N; }
      if (a.mode == kModeXZ)
        for (int i = 0; i < a.nz; ++i) { s_list[N] = m + i; s_kind[N] = 3; s_col[N] = i; ++N; }
      s_N = N;
      st->stop = kRunning;
    }
    __syncthreads();
  } else {
    // second Cholesky-QR pass over S1 (columns 0..Ng)
    if (st->stop) return;
    const int ng = st->Np;
    if (tid == 0) s_N = ng;
    __syncthreads();
    for (int i = tid; i < ng; i += blockDim.x) { s_list[i] = i; s_kind[i] = 4; s_col[i] = i; }
    __syncthreads();
  }
  const int N = s_N;
  if (a.mode == -1) {
    // Second pass: S1 is orthonormal to first order, G = I + E.  When
    // max|E| <= 1e-6 the Cholesky factor is I + F + O(E^2) with F the strict
    // lower part of E plus half its diagonal, so T = L^-T = I - F^T up to
    // O(E^2) <= 1e-12: no sequential factorization is needed.
    double em = 0.0;
    for (int x = tid; x < N * N; x += blockDim.x) {
      int i = x % N, j = x / N;
      em = fmax(em, fabs(a.G[i + (size_t)j * a.ldg] - (i == j ? 1.0 : 0.0)));
    }
    em = block_max(em, red);
    if (em <= 1e-6) {
      for (int x = tid; x < N * N; x += blockDim.x) {
        int t = x % N, c = x / N;
        double v = 0.0;
        if (c == t) v = 1.0 - 0.5 * (a.G[t + (size_t)t * a.ldg] - 1.0);
        else if (c > t) v = -a.G[c + (size_t)t * a.ldg];
        a.T[t + (size_t)c * a.ldt] = v;
      }
      for (int t = tid; t < N; t += blockDim.x) {
        a.colptr[t] = a.bases[4] + (size_t)t * a.ld;
        st->keep_col[t] = t;
      }
      if (tid == 0) {
        st->Np1 = N;  // Np and nx unchanged
      }
      return;
    }
  }
  double* Lp = lds;                      // N(N+1)/2
  double* dsc = Lp + N * (N + 1) / 2;    // N scales
  double* row = dsc + N;                 // scratch: inverse blocks + 16 x N
  // scaled Gram into packed lower
  for (int i = tid; i < N; i += blockDim.x) {
    double gii = a.G[s_list[i] + (size_t)s_list[i] * a.ldg];
    dsc[i] = (gii > 0.0 && isfinite(gii)) ? 1.0 / sqrt(gii) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < N * (N + 1) / 2; e += blockDim.x) {
    int i = tri_row(e);
    int j = e - i * (i + 1) / 2;
    double g = a.G[s_list[i] + (size_t)s_list[j] * a.ldg];
    Lp[e] = g * dsc[i] * dsc[j];
  }
  __syncthreads();
  // right-looking Cholesky with dropping on the packed lower triangle: at
  // step j the trailing Schur complement is in place; column j is dropped
  // when its pivot (squared distance of the scaled column to the span of
  // the kept ones) is below tau, and then contributes nothing.
  __shared__ int s_drop;
  __shared__ double s_piv;
  for (int j = 0; j < N; ++j) {
    if (tid == 0) {
      double d = Lp[plo(j, j)];
      bool drop = !(d > a.tau) || dsc[j] == 0.0;
      s_drop = drop;
      s_piv = drop ? 0.0 : sqrt(d);
      Lp[plo(j, j)] = s_piv;
    }
    __syncthreads();
    const bool drop = s_drop;
    const double ljj = s_piv;
    for (int i = j + 1 + tid; i < N; i += blockDim.x)
      Lp[plo(i, j)] = drop ? 0.0 : Lp[plo(i, j)] / ljj;
    if (drop)
      for (int k = tid; k < j; k += blockDim.x) Lp[plo(j, k)] = 0.0;
    __syncthreads();
    if (!drop) {
      // trailing update: G[i,k] -= L[i,j] L[k,j] for j < k <= i
      const int t = N - j - 1;
      const int cnt = t * (t + 1) / 2;
      for (int e = tid; e < cnt; e += blockDim.x) {
        int r = tri_row(e);
        int c = e - r * (r + 1) / 2;
        int i = j + 1 + r, k = j + 1 + c;
        Lp[plo(i, k)] -= Lp[plo(i, j)] * Lp[plo(k, j)];
      }
      __syncthreads();
    }
  }
  // kept list
  if (tid == 0) {
    int np = 0, nx = 0;
    int nxcand = (a.mode == -1) ? st->nx : m;  // candidates that came from X
    for (int j = 0; j < N; ++j)
      if (Lp[plo(j, j)] != 0.0) {
        s_keep[np++] = j;
        if (j < nxcand) ++nx;
      }
    s_Np = np;
    s_nx = nx;
  }
  __syncthreads();
  const int Np = s_Np;
  // in-place inverse of the lower-triangular factor by 16 x 16 block
  // forward substitution (dropped rows/columns are zero and stay zero):
  //   Linv[I,I] = inv(L[I,I]);  Linv[I,J] = -Linv[I,I] sum_{J<=K<I} L[I,K] Linv[K,J]
  // Diagonal blocks are inverted in place first (one wave each, through a
  // per-wave 16 x 16 buffer); block rows then follow in order, each in
  // parallel over its entries.  L[I,I] is not needed once inverted.
  {
    const int NB = (N + 15) / 16;
    double* scratch = row;  // max(waves * 256, 16 * N) doubles
    const int lane = tid % 64, wv = tid / 64, nw = blockDim.x / 64;
    double* D = scratch + (size_t)wv * 256;
    for (int B = wv; B < NB; B += nw) {
      const int o = B * 16, bs = min(16, N - o);
      for (int e = lane; e < 256; e += 64) D[e] = 0.0;
      __threadfence_block();
      for (int j = bs - 1; j >= 0; --j) {
        double ljj = Lp[plo(o + j, o + j)];
        double inv = (ljj != 0.0) ? 1.0 / ljj : 0.0;
        double v = 0.0;
        int i = j + 1 + lane;
        if (i < bs && ljj != 0.0) {
          double sum = 0.0;
          for (int c = j + 1; c <= i; ++c) sum += D[i + 16 * c] * Lp[plo(o + c, o + j)];
          v = -inv * sum;
        }
        if (i < bs) D[i + 16 * j] = v;
        if (lane == 0) D[j + 16 * j] = inv;
        __threadfence_block();
      }
      for (int e = lane; e < bs * bs; e += 64) {
        int r = e % bs, c = e / bs;
        if (c <= r) Lp[plo(o + r, o + c)] = D[r + 16 * c];
      }
      __threadfence_block();
    }
    __syncthreads();
    double* tmp = scratch;  // 16 x N
    for (int I = 1; I < NB; ++I) {
      const int oi = I * 16, bi = min(16, N - oi);
      // tmp[r, c] = sum_{c <= k < oi} L[oi + r, k] Linv[k, c]   (c < oi)
      for (int e = tid; e < bi * oi; e += blockDim.x) {
        int r = e % bi, c = e / bi;
        double sum = 0.0;
        for (int k = c; k < oi; ++k) sum += Lp[plo(oi + r, k)] * Lp[plo(k, c)];
        tmp[r + 16 * c] = sum;
      }
      __syncthreads();
      // Linv[oi + r, c] = -sum_{q <= r} Linv[oi + r, oi + q] tmp[q, c]
      for (int e = tid; e < bi * oi; e += blockDim.x) {
        int r = e % bi, c = e / bi;
        double sum = 0.0;
        for (int q = 0; q <= r; ++q) sum += Lp[plo(oi + r, oi + q)] * tmp[q + 16 * c];
        Lp[plo(oi + r, c)] = -sum;
      }
      __syncthreads();
    }
  }
  // T = D Linv^T restricted to kept columns: T[t, c] = d_t * Linv[keep[c], t]
  for (int e = tid; e < N * Np; e += blockDim.x) {
    int t = e % N, c = e / N;
    int kc = s_keep[c];
    double v = (t <= kc) ? Lp[plo(kc, t)] * dsc[t] : 0.0;
    a.T[t + (size_t)c * a.ldt] = v;
  }
  for (int t = tid; t < N; t += blockDim.x) {
    a.colptr[t] = a.bases[s_kind[t]] + (size_t)s_col[t] * a.ld;
    st->src_kind[t] = s_kind[t];
    st->src_col[t] = s_col[t];
  }
  for (int c = tid; c < Np; c += blockDim.x) st->keep_col[c] = s_keep[c];
  if (tid == 0) {
    if (a.mode == -1) {
      st->Np1 = st->Np;
    } else {
      st->N = N;
      st->nr = 0; st->np = 0; st->nz = 0;
      for (int t = 0; t < N; ++t) {
        st->nr += (s_kind[t] == 1);
        st->np += (s_kind[t] == 2);
        st->nz += (s_kind[t] == 3);
      }
    }
    st->Np = Np;
    st->nx = s_nx;
    if (Np == 0) st->stop = kBreakdown;
  }
}

// ---------------------------------------------------------------- RR ----


__device__ inline void rr_pair(int Ne, int r, int k, int* p, int* q) {
  // round-robin: slot 0 pairs the fixed last player with r, slot k > 0 pairs
  // (r + k) and (r - k) modulo Ne - 1
  int x, y;
  const int M = Ne - 1;
  if (k == 0) {
    x = r;
    y = M;
  } else {
    x = r + k;
    if (x >= M) x -= M;
    y = r - k;
    if (y < 0) y += M;
  }
  *p = min(x, y);
  *q = max(x, y);
}

__global__ __launch_bounds__(kRRThreads) void k_rr(RRArgs a) {
  extern __shared__ double lds[];
  __shared__ double red[kRRThreads / 64];
  __shared__ double s_cs[kMaxN + 2];    // c, s per pair
  __shared__ int s_pq[kMaxN + 2];       // p, q per pair
  __shared__ double s_theta[kMaxN];
  __shared__ int s_rank[kMaxN];
  __shared__ int s_rounds;
  State* st = a.st;
  if (st->stop) return;
  const int tid = threadIdx.x;
  const int Np = st->Np;
  const int Ne = Np + (Np & 1);
  const int P = Ne / 2;
  const int mk = min(a.mtarget, Np);
  double* H = lds;  // packed upper, Np(Np+1)/2
  const int NH = Np * (Np + 1) / 2;
  // eigenvectors accumulated in LDS when they fit, else replayed from the log
  const bool vin = (size_t)NH + (size_t)Np * Np <= a.lds_cap;
  double* V = H + NH;
  double fro2 = 0.0;
  for (int e = tid; e < NH; e += blockDim.x) {
    int j = tri_row(e);
    int i = e - j * (j + 1) / 2;
    double h = 0.5 * (a.K[i + (size_t)j * a.ldk] + a.K[j + (size_t)i * a.ldk]);
    H[e] = h;
    fro2 += (i == j ? 1.0 : 2.0) * h * h;
  }
  if (vin)
    for (int e = tid; e < Np * Np; e += blockDim.x) V[e] = (e % Np == e / Np) ? 1.0 : 0.0;
  fro2 = block_sum(fro2, red);
  const double skip = 1e-18 * sqrt(fro2);
  const double stop2 = (a.off_tol * a.off_tol) * fro2;
  // ---- parallel cyclic Jacobi (round-robin order)
  int round_id = 0;
  const size_t per_round = (size_t)2 * P;
  const int nblocks = P * (P + 1) / 2;
  for (int sweep = 0; sweep < a.max_sweeps && Np > 1; ++sweep) {
    double off = 0.0;
    for (int j = 1; j < Np; ++j)
      for (int i = tid; i < j; i += blockDim.x) {
        double v = H[j * (j + 1) / 2 + i];
        off += 2.0 * v * v;
      }
    off = block_sum(off, red);
    if (off <= stop2) break;
    if (!vin && (size_t)(round_id + Ne) * per_round > a.log_cap) break;
    for (int r = 0; r < Ne - 1; ++r) {
      if (tid < P) {
        int p, q;
        rr_pair(Ne, r, tid, &p, &q);
        s_pq[2 * tid] = p;
        s_pq[2 * tid + 1] = q;
        double c = 1.0, s = 0.0;
        if (q < Np) {
          double hpq = H[pup(p, q)];
          if (fabs(hpq) > skip) {
            // t = sign(d) e / (|d| + sqrt(d^2 + e^2)), d = hqq - hpp, e = 2 hpq:
            // the smaller root of the symmetric 2x2 Schur rotation
            double d = H[pup(q, q)] - H[pup(p, p)];
            double e2 = 2.0 * hpq;
            double rr = sqrt(d * d + e2 * e2);
            double t = (d >= 0.0 ? e2 : -e2) / (fabs(d) + rr);
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        s_cs[2 * tid] = c;
        s_cs[2 * tid + 1] = s;
        if (!vin) {
          a.log[(size_t)round_id * per_round + 2 * tid] = c;
          a.log[(size_t)round_id * per_round + 2 * tid + 1] = s;
        }
      }
      __syncthreads();
      // two-sided update of every 2x2 block (k, l), k <= l
      for (int b = tid; b < nblocks; b += blockDim.x) {
        int l = tri_row(b);
        int k = b - l * (l + 1) / 2;
        double ck = s_cs[2 * k], sk = s_cs[2 * k + 1];
        double cl = s_cs[2 * l], sl = s_cs[2 * l + 1];
        if (sk == 0.0 && sl == 0.0) continue;
        int pk = s_pq[2 * k], qk = s_pq[2 * k + 1];
        int pl = s_pq[2 * l], ql = s_pq[2 * l + 1];
        if (k == l) {
          if (qk >= Np) continue;
          double hpp = H[pup(pk, pk)], hqq = H[pup(qk, qk)], hpq = H[pup(pk, qk)];
          double c2 = ck * ck, s2 = sk * sk, cs = ck * sk;
          H[pup(pk, pk)] = c2 * hpp - 2.0 * cs * hpq + s2 * hqq;
          H[pup(qk, qk)] = s2 * hpp + 2.0 * cs * hpq + c2 * hqq;
          H[pup(pk, qk)] = 0.0;
        } else {
          bool vk = qk < Np, vl = ql < Np;
          double b00 = H[pup(pk, pl)];
          double b01 = vl ? H[pup(pk, ql)] : 0.0;
          double b10 = vk ? H[pup(qk, pl)] : 0.0;
          double b11 = (vk && vl) ? H[pup(qk, ql)] : 0.0;
          double m00 = cl * b00 - sl * b01, m01 = sl * b00 + cl * b01;
          double m10 = cl * b10 - sl * b11, m11 = sl * b10 + cl * b11;
          H[pup(pk, pl)] = ck * m00 - sk * m10;
          if (vl) H[pup(pk, ql)] = ck * m01 - sk * m11;
          if (vk) H[pup(qk, pl)] = sk * m00 + ck * m10;
          if (vk && vl) H[pup(qk, ql)] = sk * m01 + ck * m11;
        }
      }
      if (vin) {
        // V <- V J: columns (p, q) of every pair
        for (int e = tid; e < Np * P; e += blockDim.x) {
          int i = e % Np, k = e / Np;
          double c = s_cs[2 * k], s = s_cs[2 * k + 1];
          int p = s_pq[2 * k], q = s_pq[2 * k + 1];
          if (s == 0.0 || q >= Np) continue;
          double vp = V[i + (size_t)p * Np], vq = V[i + (size_t)q * Np];
          V[i + (size_t)p * Np] = c * vp - s * vq;
          V[i + (size_t)q * Np] = s * vp + c * vq;
        }
      }
      __syncthreads();
      ++round_id;
    }
  }
  if (tid == 0) s_rounds = round_id;
  for (int i = tid; i < Np; i += blockDim.x) s_theta[i] = H[pup(i, i)];
  __syncthreads();
  // ranking (descending, ties by index)
  for (int i = tid; i < Np; i += blockDim.x) {
    double ti = s_theta[i];
    int r = 0;
    for (int j = 0; j < Np; ++j) {
      double tj = s_theta[j];
      r += (tj > ti) || (tj == ti && j < i);
    }
    s_rank[i] = r;
  }
  __syncthreads();
  if (vin) {
    for (int e = tid; e < Np * Np; e += blockDim.x) {
      int i = e % Np, j = e / Np;
      int r = s_rank[j];
      if (r < mk) a.C[i + (size_t)r * a.ldc] = V[e];
    }
  } else {
    // W = J_1 ... J_T E_sel: replay the logged rounds backwards on unit
    // vectors (H's LDS is reused)
    double* W = lds;
    for (int e = tid; e < Np * mk; e += blockDim.x) W[e] = 0.0;
    __syncthreads();
    for (int i = tid; i < Np; i += blockDim.x)
      if (s_rank[i] < mk) W[i + (size_t)s_rank[i] * Np] = 1.0;
    __syncthreads();
    const int rounds = s_rounds;
    double* chunk = W + (size_t)Np * mk;
    const int chunk_rounds = 32;
    for (int t_hi = rounds; t_hi > 0; t_hi -= chunk_rounds) {
      int t_lo = max(0, t_hi - chunk_rounds);
      int cnt = t_hi - t_lo;
      for (int e = tid; e < cnt * (int)per_round; e += blockDim.x)
        chunk[e] = a.log[(size_t)t_lo * per_round + e];
      __syncthreads();
      for (int t = t_hi - 1; t >= t_lo; --t) {
        int r = t % (Ne - 1);
        const double* cs = chunk + (size_t)(t - t_lo) * per_round;
        for (int e = tid; e < P * mk; e += blockDim.x) {
          int k = e % P, col = e / P;
          double c = cs[2 * k], s = cs[2 * k + 1];
          if (s == 0.0) continue;
          int p, q;
          rr_pair(Ne, r, k, &p, &q);
          if (q >= Np) continue;
          double wp = W[p + (size_t)col * Np], wq = W[q + (size_t)col * Np];
          W[p + (size_t)col * Np] = c * wp + s * wq;
          W[q + (size_t)col * Np] = -s * wp + c * wq;
        }
        __syncthreads();
      }
    }
    for (int e = tid; e < Np * mk; e += blockDim.x) {
      int i = e % Np, col = e / Np;
      a.C[i + (size_t)col * a.ldc] = W[e];
    }
  }
  int npos = 0;
  for (int i = tid; i < Np; i += blockDim.x) {
    npos += (s_theta[i] > 0.0);
    if (s_rank[i] < mk) st->theta[s_rank[i]] = s_theta[i];
  }
  double npd = block_sum((double)npos, red);
  if (tid == 0) {
    st->npos_rr = (int)npd;
    st->mk = mk;
    st->expand_req = ((int)npd > a.mtarget) ? 1 : 0;
    st->jacobi_rounds = s_rounds;
    if (a.count_iter) st->iter += 1;
  }
}

hipError_t launch_decide_chol(const DecideArgs& a, int N_host, hipStream_t st) {
  size_t scr = std::max((size_t)(kSmallThreads / 64) * 256, (size_t)16 * N_host);
  size_t lds = sizeof(double) * ((size_t)N_host * (N_host + 1) / 2 + (size_t)N_host + scr + 8);
  hipLaunchKernelGGL(k_decide_chol, dim3(1), dim3(kSmallThreads), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_rr(const RRArgs& a_in, int Np_host, int mk_host, hipStream_t st) {
  RRArgs a = a_in;
  size_t h = (size_t)Np_host * (Np_host + 1) / 2;
  size_t w = (size_t)Np_host * mk_host + (size_t)32 * (Np_host + 2) + 64;
  size_t want = h + (size_t)Np_host * Np_host;  // H and V both in LDS
  size_t cap_doubles = (size_t)(g_lds_limit / 8);
  size_t need = std::max(h, w);
  size_t lds_d = want <= cap_doubles ? want : need;
  a.lds_cap = lds_d;
  hipLaunchKernelGGL(k_rr, dim3(1), dim3(kRRThreads), sizeof(double) * lds_d, st, a);
  return hipGetLastError();
}

hipError_t small_kernels_init() {
  // allow up to the device's LDS per workgroup for the dynamic allocations
  int dev = 0, lim = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
  if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    lim = 64 * 1024;
  int dyn = lim - 8 * 1024;  // static LDS of the kernels stays below 8 KB
  if (dyn > 0) g_lds_limit = dyn;
  if (dyn > 0) {
    (void)hipFuncSetAttribute((const void*)k_decide_chol,
                              hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void*)k_rr, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
  }
  (void)hipGetLastError();
  return hipSuccess;
}

}  // namespace psdp
