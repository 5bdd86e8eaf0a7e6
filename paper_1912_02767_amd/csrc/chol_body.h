// Device body of the decision + Cholesky-QR step (convergence, stall and
// expansion decisions, active set, Cholesky with column dropping, inverse
// factor); included by the single-cone kernel and the batched kernel.
#pragma once
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
// Body shared by the single-cone kernel and the batched persistent kernel.
__device__ inline void decide_chol_body(const DecideArgs& a, double* lds, const CholShared& sh) {
  double* red = sh.red;
  int* s_list = sh.list;   // logical trial column -> candidate index in G
  int* s_kind = sh.kind;
  int* s_col = sh.col;
  int* s_keep = sh.keep;
  int& s_N = *sh.N;
  int& s_Np = *sh.Np;
  int& s_nx = *sh.nx;
  int& s_stop = *sh.stop;
  State* st = a.st;
  const int tid = threadIdx.x;
  const int m = a.m;
  if (tid == 0 && a.mode != -1) st->t_phase[5] = wall_clock64();

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
      // Rounding floor of residuals formed with low-precision products:
      // about u_p ||A||_F / sqrt(n) per unit column (entry-wise rounding of A
      // and of the accumulation); a phase ends once its largest positive
      // residual is within a small factor of it.
      const double up = a.phase_lowprec == 2 ? 3.9e-3 : 6.0e-8;
      const double lp_floor = lowp ? 8.0 * up * sqrt(st->fro2_x / (double)max(st->n, 1)) : 0.0;
      if (nonfin) {
        stop = kNonFinite;
      } else if (lowp && npos > 0 && rmax <= lp_floor) {
        stop = kStalled;  // at the floor: continue with the next precision
      } else if (st->expand_req) {
        stop = lowp ? kStalled : kExpand;
      } else if (npos == m && rmax <= tol && m >= st->n) {
        stop = kConverged;  // the block spans the whole space
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
  const bool mark = (a.mode != -1) && tid == 0;
  if (mark) st->t_phase[6] = wall_clock64();
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
  if (mark) st->t_phase[7] = wall_clock64();
  // Blocked right-looking Cholesky with dropping on the packed lower
  // triangle, panels of 16 columns; at the start of panel [o, o + bs) the
  // trailing Schur complement is in place.  A column is dropped when its
  // pivot (squared distance of the scaled column to the span of the kept
  // ones) is below tau: its column and row of L are zero and it contributes
  // nothing to later columns.
  //   (1) one wave factors the diagonal block column by column;
  //   (2) rows below the block solve against it, one row per thread;
  //   (3) the trailing triangle takes the rank-bs update in 4 x 4 tiles.
  {
    double* pinv = row;  // 16 inverse pivots of the panel (0: dropped)
    const int lane = tid & 63;
    for (int o = 0; o < N; o += 16) {
      const int bs = min(16, N - o);
      if (tid < 64) {
        for (int j = 0; j < bs; ++j) {
          const int jj = o + j;
          const double d = Lp[plo(jj, jj)];
          const bool drop = !(d > a.tau) || dsc[jj] == 0.0;
          const double ljj = drop ? 0.0 : sqrt(d);
          __threadfence_block();
          if (lane == 0) {
            Lp[plo(jj, jj)] = ljj;
            pinv[j] = drop ? 0.0 : 1.0 / ljj;
          }
          if (lane < bs - j - 1) {
            const int i = jj + 1 + lane;
            Lp[plo(i, jj)] = drop ? 0.0 : Lp[plo(i, jj)] / ljj;
          }
          if (drop)
            for (int k = lane; k < jj; k += 64) Lp[plo(jj, k)] = 0.0;
          __threadfence_block();
          if (!drop) {
            const int t = bs - j - 1;
            for (int e = lane; e < t * t; e += 64) {
              const int r = e / t, c = e - r * t;
              if (c <= r) {
                const int i = jj + 1 + r, k = jj + 1 + c;
                Lp[plo(i, k)] -= Lp[plo(i, jj)] * Lp[plo(k, jj)];
              }
            }
          }
          __threadfence_block();
        }
      }
      __syncthreads();
      // (2) L[i, o:o+bs] = S[i, o:o+bs] L_D^-T, dropped columns zero
      for (int i = o + bs + tid; i < N; i += blockDim.x) {
        double* Li = Lp + plo(i, o);
        double v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          if (j < bs) {
            const double* Lj = Lp + plo(o + j, o);
            double s = Li[j];
#pragma unroll
            for (int k = 0; k < j; ++k) s = fma(-v[k], Lj[k], s);
            v[j] = s * pinv[j];
          }
        }
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (j < bs) Li[j] = v[j];
      }
      __syncthreads();
      // (3) S[i, k] -= sum_j L[i, o + j] L[k, o + j] for o + bs <= k <= i
      const int b0 = o + bs;
      const int t = N - b0;
      if (t > 0) {
        const int nt = (t + 3) / 4;
        for (int tile = tid; tile < nt * (nt + 1) / 2; tile += blockDim.x) {
          const int ti = tri_row(tile), tj = tile - ti * (ti + 1) / 2;
          const int i0 = b0 + 4 * ti, k0 = b0 + 4 * tj;
          double acc[4][4];
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
          for (int j0 = 0; j0 < bs; j0 += 4) {
            double x[4][4], y[4][4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = min(i0 + r, N - 1), k = min(k0 + r, N - 1);
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const bool in = j0 + q < bs;
                x[r][q] = in ? Lp[plo(i, o + j0 + q)] : 0.0;
                y[r][q] = in ? Lp[plo(k, o + j0 + q)] : 0.0;
              }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
              for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[r][c] = fma(x[r][q], y[c][q], acc[r][c]);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const int i = i0 + r, k = k0 + c;
              if (i < N && k <= i) Lp[plo(i, k)] -= acc[r][c];
            }
        }
      }
      __syncthreads();
    }
  }
  if (mark) st->t_phase[8] = wall_clock64();
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
  if (mark) st->t_phase[9] = wall_clock64();
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
    if (a.mode != -1) st->t_phase[10] = wall_clock64();
  }
}


}  // namespace psdp
