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

// value of lane l (compile-time or uniform) in every lane
__device__ inline double bcast_d(double v, int l) {
  int2 x = __builtin_bit_cast(int2, v);
  x.x = __builtin_amdgcn_readlane(x.x, l);
  x.y = __builtin_amdgcn_readlane(x.y, l);
  return __builtin_bit_cast(double, x);
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
  lds = lds_base();  // callers pass the dynamic LDS base; keep its address space
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
  if (a.spec_m > 0) {
    // queued before the previous iteration was read back: a no-op unless that
    // iteration kept running with the assumed block size.  One thread reads
    // the state and the workgroup takes its verdict, before any thread can
    // change the state.
    if (tid == 0) {
      const int stop0 = st->stop;
      s_stop = (stop0 != kRunning) ? 1 : (st->mk != a.spec_m ? 2 : 0);
      if (s_stop == 2) st->stop = kSpecAbort;
    }
    __syncthreads();
    const int verdict = s_stop;
    __syncthreads();
    if (verdict != 0) return;
  }
  if (tid == 0 && a.mode != -1) st->t_phase[5] = wall_clock64();

  if (a.mode == kModeFull || a.mode == kModeXR || a.mode == kModeEval) {
    // ---- decisions from the residual norms (paper §5.2 / §6 stopping rule),
    // in wave 0 with one lane per block column (m <= 64; theta descending)
    double* s_th = red + blockDim.x / 64;  // 64 + 64 doubles after the reduction slots
    double* s_rn = s_th + 64;
    if (tid < 64) {
      const int i = tid;
      const bool in = i < m;
      const double th = st->theta[min(i, m - 1)];
      const double rn = sqrt(fmax(a.G[(m + min(i, m - 1)) + (size_t)(m + min(i, m - 1)) * a.ldg], 0.0));
      if (in) {
        st->rnorm[i] = rn;
        s_th[i] = th;
        s_rn[i] = rn;
      }
      const unsigned long long posm = __ballot(in && th > 0.0);
      const int npos = __popcll(posm);
      double rm = (in && i < npos) ? rn : 0.0;
      double r2 = rm * rm;
      double ra = in ? rn : 0.0;  // over every pair of the block
      for (int o = 32; o > 0; o >>= 1) {
        rm = fmax(rm, __shfl_xor(rm, o, 64));
        r2 += __shfl_xor(r2, o, 64);
        ra = fmax(ra, __shfl_xor(ra, o, 64));
      }
      const bool bad = in && (!isfinite(th) || !isfinite(rn));
      const bool nonfin_any = __ballot(bad) != 0ull;
      const double tol = st->tol;
      // Active residuals: a positive pair, and the first non-positive (guard)
      // pair, which is the one that rises toward positive eigenvalues not
      // yet in the block, until they meet tol; the further non-positive
      // pairs only while the guard rule (largest non-positive pair within
      // max(tol, gap / 2), the stopping rule below) is unmet: past that
      // they stay in X but their R and P columns leave the trial basis (the
      // top-r variant needs every pair of its block)
      double gtl = tol;
      {
        const int g0 = npos < m ? npos : m - 1;
        const double thp = npos > 0 ? st->theta[npos - 1] : 0.0;
        const double thg = st->theta[g0];
        const double dl = npos > 0 ? (thp - thg) : fabs(thg);
        gtl = fmax(tol, 0.5 * dl);
      }
      const bool act = in && rn > ((i <= npos || st->fixed_block) ? tol : gtl);
      const unsigned long long actm = __ballot(act);
      const int nact = __popcll(actm);
      const int pre = __popcll(actm & ((1ull << i) - 1ull));
      __threadfence_block();  // s_th, s_rn visible to lane 0
      if (i == 0) {
        st->npos_blk = npos;
        const double rmax = rm, rfro = r2;
        st->res_max_pos = rmax;
        st->res_fro_pos = sqrt(rfro);
        st->theta_min_pos = npos > 0 ? s_th[npos - 1] : 0.0;
        int stop = kRunning;
        const bool nonfin = nonfin_any || !isfinite(rfro);
        // guard: largest non-positive Ritz pair, resolved to half its gap
        double q;  // progress metric, <= 1 when converged
        bool guard_ok = false;
        if (npos < m) {
          const int g = npos;
          const double delta = npos > 0 ? (s_th[npos - 1] - s_th[g]) : fabs(s_th[g]);
          const double gtol = fmax(tol, 0.5 * delta);
          st->guard_theta = s_th[g];
          st->guard_res = s_rn[g];
          guard_ok = s_rn[g] <= gtol;
          q = fmax(rmax / tol, s_rn[g] / gtol);
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
        } else if (st->fixed_block && ra <= tol) {
          // top-r: every pair of the block, positive or not, meets tol
          stop = lowp ? kStalled : kConverged;
        } else if (st->expand_req && !st->fixed_block) {
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
      }
      __threadfence_block();  // s_stop visible to the wave
      const int stop = s_stop;
      // logical trial basis: X, then active R, then active P
      if (in) { s_list[i] = i; s_kind[i] = 0; s_col[i] = i; }
      const bool withp = a.has_p && a.mode == kModeFull;
      if (stop == kRunning && act) {
        s_list[m + pre] = m + i; s_kind[m + pre] = 1; s_col[m + pre] = i;
        if (withp) { s_list[m + nact + pre] = 2 * m + i; s_kind[m + nact + pre] = 2; s_col[m + nact + pre] = i; }
      }
      if (i == 0) s_N = (stop == kRunning) ? m + nact * (withp ? 2 : 1) : m;
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
    // both sweeps over G issue kU unconditional loads (indices clamped)
    // before using any: one global-memory round trip per kU elements
    constexpr int kU = 16;
    const int NN = N * N, nb = (int)blockDim.x;
    double em = 0.0;
    for (int x0 = tid; x0 < NN; x0 += kU * nb) {
      double g[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int x = min(x0 + u * nb, NN - 1);
        g[u] = a.G[x % N + (size_t)(x / N) * a.ldg];
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int x = x0 + u * nb;
        const int i = x % N, j = x / N;
        const double dv = fabs(g[u] - (i == j ? 1.0 : 0.0));
        em = fmax(em, (x < NN) ? dv : 0.0);
      }
    }
    em = block_max(em, red);
    if (em <= 1e-6) {
      for (int x0 = tid; x0 < NN; x0 += kU * nb) {
        double g[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int x = min(x0 + u * nb, NN - 1);
          g[u] = a.G[x / N + (size_t)(x % N) * a.ldg];  // G[c, t]
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int x = x0 + u * nb;
          const int t = x % N, c = x / N;
          const double v = (c == t) ? 1.0 - 0.5 * (g[u] - 1.0) : ((c > t) ? -g[u] : 0.0);
          if (x < NN) a.T[t + (size_t)c * a.ldt] = v;
        }
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
  {
    // sixteen independent loads in flight per thread (indices clamped)
    constexpr int kU = 16;
    const int n2 = N * (N + 1) / 2, ntu = kU * blockDim.x;
    for (int e0 = tid; e0 < n2; e0 += ntu) {
      double g[kU];
      int ii[kU], jj[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = min(e0 + u * (int)blockDim.x, n2 - 1);
        ii[u] = tri_row(e);
        jj[u] = e - ii[u] * (ii[u] + 1) / 2;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) g[u] = a.G[s_list[ii[u]] + (size_t)s_list[jj[u]] * a.ldg];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * (int)blockDim.x;
        if (e < n2) Lp[e] = g[u] * dsc[ii[u]] * dsc[jj[u]];
      }
    }
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
  // Lookahead: in (3) wave 0 takes the tiles of the next diagonal block and
  // goes on to factor it (1) while the other waves update the rest, so the
  // sequential factorization of a block is off the critical path.  What the
  // other waves read meanwhile that (1) may change (row L[k, :o] of a column
  // k dropped in the next block) only enters entries of column k, which the
  // solve (2) multiplies by a zero inverse pivot.
  {
    double* pinv = row;  // 16 inverse pivots of the panel (0: dropped)
    const int lane = tid & 63;
    const bool tr = mark && a.trace != 0;  // per-panel clock totals (tracing only)
    long long tc = tr ? wall_clock64() : 0, tca[3] = {0, 0, 0};
    // (1) for the block at o, by wave 0: lane l < bs holds row o + l of the
    // diagonal block; pivots by reciprocal square root (two Newton steps),
    // the block column by lane reads, the rank-1 updates in registers
    auto factor_diag = [&](int o) {
      const int bs = min(16, N - o);
      const int l = lane;
      double rw[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) rw[k] = (l < bs && k <= l) ? Lp[plo(o + min(l, bs - 1), o + min(k, l))] : 0.0;
      const double dsl = dsc[o + min(l, bs - 1)];
      unsigned long long dropm = 0ull;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        if (j < bs) {
          const double d = bcast_d(rw[j], j);
          const double dsj = bcast_d(dsl, j);
          const bool drop = !(d > a.tau) || dsj == 0.0;
          double r = 0.0;
          if (!drop) {
            r = __builtin_amdgcn_rsq(d);
            r = r * fma(-0.5 * d * r, r, 1.5);
            r = r * fma(-0.5 * d * r, r, 1.5);
          }
          if (drop) dropm |= 1ull << j;
          if (l == j) rw[j] = drop ? 0.0 : d * r;  // L(j, j) = sqrt(d)
          if (l > j) rw[j] = drop ? 0.0 : rw[j] * r;
          if (l == 0) pinv[j] = r;
          if (!drop) {
#pragma unroll
            for (int k = j + 1; k < 16; ++k) {
              const double lkj = bcast_d(rw[j], k);  // L(k, j)
              if (k <= l) rw[k] = fma(-rw[j], lkj, rw[k]);
            }
          }
        }
      }
      // rows of dropped columns are zero (in this block and to its left)
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (l == j && ((dropm >> j) & 1ull)) {
#pragma unroll
          for (int k = 0; k < 16; ++k) rw[k] = 0.0;
        }
      if (l < bs)
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (k <= l) Lp[plo(o + l, o + k)] = rw[k];
      for (int j = 0; j < bs; ++j)
        if ((dropm >> j) & 1ull)
          for (int k = lane; k < o; k += 64) Lp[plo(o + j, k)] = 0.0;
    };
    // one 4 x 4 tile of the rank-16 update from panel o (rows i0.., columns k0..)
    auto update_tile = [&](int o, int i0, int k0) {
      double acc[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
#pragma unroll 1
      for (int j0 = 0; j0 < 16; j0 += 4) {
        double x[4][4], y[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = min(i0 + r, N - 1), k = min(k0 + r, N - 1);
#pragma unroll
          for (int q = 0; q < 4; ++q) {  // bs = 16 whenever a trailing block exists
            x[r][q] = Lp[plo(i, o + j0 + q)];
            y[r][q] = Lp[plo(k, o + j0 + q)];
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
    };
    if (tid < 64) factor_diag(0);
    __syncthreads();
    for (int o = 0; o < N; o += 16) {
      const int bs = min(16, N - o);
      if (tr) { const long long tn = wall_clock64(); tca[0] += tn - tc; tc = tn; }
      // (2) L[i, o:o+bs] = S[i, o:o+bs] L_D^-T, dropped columns zero
      // (rows below the block exist only when the block is full: bs = 16)
      for (int i = o + bs + tid; i < N; i += blockDim.x) {
        // right-looking: the dependent chain is one multiply and one fma per column
        double* Li = Lp + plo(i, o);
        double v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = Li[j];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          v[j] *= pinv[j];
#pragma unroll
          for (int k = j + 1; k < 16; ++k) v[k] = fma(-v[j], Lp[plo(o + k, o) + j], v[k]);
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) Li[j] = v[j];
      }
      __syncthreads();
      if (tr) { const long long tn = wall_clock64(); tca[1] += tn - tc; tc = tn; }
      // (3) S[i, k] -= sum_j L[i, o + j] L[k, o + j] for o + bs <= k <= i;
      // tiles 0 .. 9 (rows and columns below b0 + 16) form the next diagonal
      // block: wave 0 updates them and factors that block, the other waves
      // take tiles 10 ..
      const int b0 = o + bs;
      const int t = N - b0;
      if (t > 0) {
        const int nt = (t + 3) / 4;
        const int ntile = nt * (nt + 1) / 2;
        if (tid < 64) {
          if (tid < min(10, ntile)) {
            const int ti = tri_row(tid), tj = tid - ti * (ti + 1) / 2;
            update_tile(o, b0 + 4 * ti, b0 + 4 * tj);
          }
          __threadfence_block();  // the wave's tile updates precede its reads of the block
          factor_diag(b0);
        } else {
          for (int tile = 10 + tid - 64; tile < ntile; tile += blockDim.x - 64) {
            const int ti = tri_row(tile), tj = tile - ti * (ti + 1) / 2;
            update_tile(o, b0 + 4 * ti, b0 + 4 * tj);
          }
        }
      }
      __syncthreads();
      if (tr) { const long long tn = wall_clock64(); tca[2] += tn - tc; tc = tn; }
    }
    if (mark)
      for (int q = 0; q < 3; ++q) st->t_sub[8 + q] = tca[q];
  }
  if (mark) st->t_phase[8] = wall_clock64();
  // kept list, in wave 0: 64 candidates per ballot, prefix counts by popcount
  if (tid < 64) {
    const int nxcand = (a.mode == -1) ? st->nx : m;  // candidates that came from X
    int np = 0, nx = 0;
    for (int j0 = 0; j0 < N; j0 += 64) {
      const int j = j0 + tid;
      const bool kept = j < N && Lp[plo(min(j, N - 1), min(j, N - 1))] != 0.0;
      const unsigned long long km = __ballot(kept);
      if (kept) s_keep[np + __popcll(km & ((1ull << tid) - 1ull))] = j;
      np += __popcll(km);
      nx += __popcll(__ballot(kept && j < nxcand));
    }
    if (tid == 0) {
      s_Np = np;
      s_nx = nx;
    }
  }
  __syncthreads();
  const int Np = s_Np;
  // in-place inverse of the lower-triangular factor by 16 x 16 blocks
  // (dropped rows and columns are zero and stay zero):
  //   (1) diagonal blocks, one wave per block and one lane per column:
  //       forward substitution L x = e_j in registers;
  //   (2) block rows I = 1, 2, ...: wave J forms
  //       Linv[I, J] = -Linv[I, I] sum_{J <= K < I} L[I, K] Linv[K, J]
  //       (a 16 x 16 tile, four entries per lane); all waves have read
  //       L[I, :] before any of them writes its block.
  {
    const int NB = (N + 15) / 16;
    const int lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
    for (int B = wv; B < NB; B += nw) {
      const int o = B * 16, bs = min(16, N - o);
      if (lane < 16) {
        const int j = lane;
        double x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          x[i] = 0.0;
          if (i < bs) {
            const double lii = Lp[plo(o + i, o + i)];
            double inv = 0.0;
            if (lii != 0.0) {
              inv = __builtin_amdgcn_rcp(lii);
              inv = fma(fma(-lii, inv, 1.0), inv, inv);
              inv = fma(fma(-lii, inv, 1.0), inv, inv);
            }
            double s0 = (i == j) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
            for (int k = 0; k < i; ++k) {
              const double l = Lp[plo(o + i, o + k)];
              if (k & 1) s1 = fma(-l, x[k], s1);
              else s0 = fma(-l, x[k], s0);
            }
            x[i] = (i >= j) ? (s0 + s1) * inv : 0.0;
          }
        }
        __threadfence_block();  // the wave has read the block before it is overwritten
        if (j < bs)
#pragma unroll
          for (int i = 0; i < 16; ++i)
            if (i >= j && i < bs) Lp[plo(o + i, o + j)] = x[i];
      }
    }
    __syncthreads();
    if (mark) st->t_sub[11] = wall_clock64() - st->t_phase[8];  // diagonal blocks (and kept list)
    double* Wt = row + (size_t)wv * 256;  // per-wave 16 x 16 tile
    const int r = lane & 15, c4 = lane >> 4;
    for (int I = 1; I < NB; ++I) {
      const int oi = I * 16, bi = min(16, N - oi);
      const int ri = oi + min(r, bi - 1);  // rows past N are computed from a valid row and dropped
      double out[2][4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int J = wv + h * nw;
#pragma unroll
        for (int q = 0; q < 4; ++q) out[h][q] = 0.0;
        if (J < I) {  // uniform per wave
          const int oj = J * 16;
          double acc[4] = {0.0, 0.0, 0.0, 0.0};
          {
            // K = J: the diagonal block of Linv is lower triangular
            const double* lrow = Lp + plo(ri, oj);
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
              const double l = lrow[kk];
              const double* vrow = Lp + plo(oj + kk, oj);  // row oj + kk, columns oj ..
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int c = 4 * c4 + q;
                const double v = vrow[min(c, kk)];
                acc[q] = fma(l, (kk >= c) ? v : 0.0, acc[q]);
              }
            }
          }
          for (int K = J + 1; K < I; ++K) {
            // below the diagonal blocks: contiguous rows, no masks
            const int ok = K * 16;
            const double* lrow = Lp + plo(ri, ok);
            double lv[16];
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) lv[kk] = lrow[kk];
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
              const double* vrow = Lp + plo(ok + kk, oj) + 4 * c4;
#pragma unroll
              for (int q = 0; q < 4; ++q) acc[q] = fma(lv[kk], vrow[q], acc[q]);
            }
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) Wt[r * 16 + 4 * c4 + q] = acc[q];
          __threadfence_block();
#pragma unroll
          for (int qq = 0; qq < 16; ++qq) {
            const double lq = Lp[plo(ri, oi + min(qq, ri - oi))];  // Linv[I, I](r, qq)
            const double lqm = (qq <= ri - oi) ? lq : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) out[h][q] = fma(-lqm, Wt[qq * 16 + 4 * c4 + q], out[h][q]);
          }
          __threadfence_block();  // the tile buffer is reused by the next J of this wave
        }
      }
      __syncthreads();  // every wave has read L[I, :]
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int J = wv + h * nw;
        if (J < I && r < bi) {
#pragma unroll
          for (int q = 0; q < 4; ++q) Lp[plo(oi + r, J * 16 + 4 * c4 + q)] = out[h][q];
        }
      }
      __syncthreads();
    }
  }
  if (mark) st->t_phase[9] = wall_clock64();
  // T = D Linv^T restricted to kept columns: T[t, c] = d_t * Linv[keep[c], t]
  for (int e = tid; e < N * Np; e += blockDim.x) {
    int t = e % N, c = e / N;
    int kc = s_keep[c];
    const double lv = Lp[plo(kc, min(t, kc))] * dsc[t];
    const double v = (t <= kc) ? lv : 0.0;
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
