// Batched projection of many independent cones of uneven size in one
// persistent launch (paper §6.1: SDPs in block-diagonal form split into many
// smaller PSD variables, each projected every ADMM iteration).
//
// Each workgroup takes the next cone from an atomic queue (the host orders
// the queue by decreasing work) and runs the whole warm-started LOBPCG of
// paper §5.1 (Alg. 3) for it alone: the decision/Cholesky-QR and the
// Rayleigh-Ritz steps are the device bodies of the single-cone pipeline,
// the tall-skinny and block products are workgroup GEMMs over the
// workgroup's own scratch.  Products run in FP32 (or FP64), everything else
// in FP64; the run ends with an FP64 refresh and FP64 iterations, the §5.2
// bound statistics and the rebuild.
#include "batched.h"
#include "chol_body.h"
#include "rr_fast.h"

namespace psdp {

// ---------------------------------------------------------- workgroup GEMM
// C (M x N, ldc, FP64) = op(A) (M x K) op(B) (K x N), accumulated in TC.
//   AT = true : op(A)[i, k] = A.col(i)[k]   (Gram S^T Y)
//   AT = false: op(A)[i, k] = A.col(k)[i]   (S M, A S)
//   BT = false: op(B)[k, j] = B[k + j ldb];  BT = true: op(B)[k, j] = B[j + k ldb]
// 64 x 64 output tiles, 4 x 4 per thread, k staged through LDS in chunks.
template <typename TA>
struct ColsT {
  const TA* const* ptr;  // column pointers, or
  const TA* base;        // contiguous columns with leading dim ld
  int ld;
  __device__ inline const TA* col(int k) const { return ptr ? ptr[k] : base + (size_t)k * ld; }
};

template <typename TA, typename TC, bool AT, bool BT>
__device__ void wg_gemm(int M, int N, int K, ColsT<TA> A, const double* B, int ldb, double* C,
                        int ldc, void* smem, int kc) {
  smem = lds_base();            // callers pass the dynamic LDS base; keep its address space
  TC* sA = (TC*)smem;           // kc x 65
  TC* sB = sA + kc * 65;        // kc x 65
  const int tid = threadIdx.x, nt = blockDim.x;
  const int tx = tid & 15, ty = tid >> 4;
  for (int i0 = 0; i0 < M; i0 += 64)
    for (int j0 = 0; j0 < N; j0 += 64) {
      TC acc[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = TC(0);
      for (int k0 = 0; k0 < K; k0 += kc) {
        for (int e = tid; e < kc * 64; e += nt) {
          int kk, ii;
          if (AT) { kk = e % kc; ii = e / kc; } else { ii = e & 63; kk = e >> 6; }
          const int i = i0 + ii, k = k0 + kk;
          TC v = TC(0);
          if (i < M && k < K) v = (TC)(AT ? A.col(i)[k] : A.col(k)[i]);
          sA[kk * 65 + ii] = v;
        }
        for (int e = tid; e < kc * 64; e += nt) {
          int kk, jj;
          if (BT) { jj = e & 63; kk = e >> 6; } else { kk = e % kc; jj = e / kc; }
          const int k = k0 + kk, j = j0 + jj;
          TC v = TC(0);
          if (k < K && j < N) v = (TC)(BT ? B[j + (size_t)k * ldb] : B[k + (size_t)j * ldb]);
          sB[kk * 65 + jj] = v;
        }
        __syncthreads();
        const int kend = min(kc, K - k0);
        for (int kk = 0; kk < kend; ++kk) {
          TC av[4], bv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) av[u] = sA[kk * 65 + ty + 16 * u];
#pragma unroll
          for (int v = 0; v < 4; ++v) bv[v] = sB[kk * 65 + tx + 16 * v];
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
        }
        __syncthreads();
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + ty + 16 * u, j = j0 + tx + 16 * v;
          if (i < M && j < N) C[i + (size_t)j * ldc] = (double)acc[u][v];
        }
    }
  __syncthreads();
}

// ------------------------------------------------------------- scratch ---
struct BScratch {
  double* A64;   // n x n, sign * sym(X)
  float* A32;    // n x n, FP32 copy
  double* XRP;   // [X | R | P], column blocks of m at offsets 0, m, 2m (ld n)
  double* AX;    // n x mmax
  double* Z;     // n x mmax
  double* S1;    // n x 3 mmax
  double* S2;    // n x 3 mmax
  double* AS;    // n x 3 mmax
  double* G;     // NC x NC (NC = 3 mmax)
  double* T;     // NC x NC
  double* C;     // NC x NC
  double* rrs;   // 5 NC mmax (Rayleigh-Ritz factor spill)
  const double** colptr;  // NC
  State* st;
};

__device__ inline BScratch bscratch_at(char* base, int nmax, int mmax) {
  const size_t n = nmax, mc = mmax, nc = 3 * (size_t)mmax;
  BScratch w;
  double* p = (double*)base;
  w.A64 = p; p += n * n;
  w.XRP = p; p += n * 3 * mc;
  w.AX = p; p += n * mc;
  w.Z = p; p += n * mc;
  w.S1 = p; p += n * nc;
  w.S2 = p; p += n * nc;
  w.AS = p; p += n * nc;
  w.G = p; p += nc * nc;
  w.T = p; p += nc * nc;
  w.C = p; p += nc * nc;
  w.rrs = p; p += 5 * nc * mc;
  w.colptr = (const double**)p; p += nc;
  w.A32 = (float*)p; p += (n * n + 1) / 2;
  p = (double*)(((uintptr_t)p + 255) & ~(uintptr_t)255);
  w.st = (State*)p;
  return w;
}

size_t batched_scratch_bytes(int nmax, int mmax) {
  const size_t n = nmax, mc = mmax, nc = 3 * (size_t)mmax;
  const size_t d = n * n + n * 3 * mc + 2 * n * mc + 3 * n * nc + 3 * nc * nc + 5 * nc * mc + nc +
                   (n * n + 1) / 2;
  const size_t b = 8 * d + 256 + sizeof(State);
  return (b + 255) / 256 * 256;
}

// ------------------------------------------------------------ one cone ---
struct BShared {
  RRShared rr;
  CholShared ch;
};

template <bool RRFULL>
struct ConeSolver {
  const BatchArgs& ba;
  BScratch w;
  BShared sh;
  double* lds;
  int n = 0, mcap = 0, m = 0, has_p = 0;
  uint64_t rng = 0;
  __device__ ConeSolver(const BatchArgs& b, BScratch ws, BShared s, double* l)
      : ba(b), w(ws), sh(s), lds(l) {}

  __device__ void gemm_nn(int M, int N, int K, ColsT<double> A, const double* B, int ldb,
                          double* Cp, int ldc) {
    wg_gemm<double, double, false, false>(M, N, K, A, B, ldb, Cp, ldc, lds, ba.kc);
  }
  __device__ void gram(int M, int N, ColsT<double> A, const double* B, int ldb, double* Cp,
                       int ldc) {
    wg_gemm<double, double, true, false>(M, N, n, A, B, ldb, Cp, ldc, lds, ba.kc);
  }

  // One Rayleigh-Ritz step on the trial basis of `mode` (Alg. 3 loop body).
  __device__ void iterate(int mode, int pprec, int mtarget, int nz) {
    State* st = w.st;
    const int ld = n;
    const int NC = 3 * ba.mmax;
    double* X = w.XRP;
    double* R = w.XRP + (size_t)m * ld;
    double* P = w.XRP + (size_t)2 * m * ld;
    int Ng;
    if (mode == kModeXOnly) {
      Ng = m;
    } else if (mode == kModeXZ) {
      // the expansion columns go to the R slot: candidates stay contiguous
      for (int e = threadIdx.x; e < n * nz; e += blockDim.x) R[e] = w.Z[e];
      __syncthreads();
      Ng = m + nz;
    } else {
      Ng = has_p ? 3 * m : 2 * m;
    }
    ColsT<double> cand{nullptr, w.XRP, ld};
    gram(Ng, Ng, cand, w.XRP, ld, w.G, NC);
    DecideArgs da{};
    da.G = w.G; da.ldg = NC; da.Ng = Ng; da.mode = mode; da.m = m; da.nz = nz;
    da.has_p = has_p; da.phase_lowprec = pprec; da.tau = 1e-10;
    da.bases[0] = X; da.bases[1] = R; da.bases[2] = P; da.bases[3] = R; da.bases[4] = w.S1;
    da.ld = ld; da.T = w.T; da.ldt = NC; da.colptr = w.colptr; da.st = st;
    decide_chol_body(da, lds, sh.ch);
    __syncthreads();
    if (st->stop != kRunning) return;
    // first Cholesky-QR pass: S1 = S T1
    {
      ColsT<double> tri{w.colptr, nullptr, ld};
      gemm_nn(n, st->Np, st->N, tri, w.T, NC, w.S1, ld);
    }
    // second pass on S1: S2 = S1 T2
    {
      const int Np = st->Np;
      ColsT<double> s1{nullptr, w.S1, ld};
      gram(Np, Np, s1, w.S1, ld, w.G, NC);
      DecideArgs db = da;
      db.mode = -1;
      db.Ng = Np;
      decide_chol_body(db, lds, sh.ch);
      __syncthreads();
      if (st->stop != kRunning) return;
      gemm_nn(n, st->Np, st->Np1, s1, w.T, NC, w.S2, ld);
    }
    // AS = A S2 in the phase precision, K = S2^T AS
    {
      const int Np = st->Np;
      if (pprec == 0) {
        ColsT<double> a{nullptr, w.A64, ld};
        wg_gemm<double, double, false, false>(n, Np, n, a, w.S2, ld, w.AS, ld, lds, ba.kc);
      } else {
        ColsT<float> a{nullptr, w.A32, ld};
        wg_gemm<float, float, false, false>(n, Np, n, a, w.S2, ld, w.AS, ld, lds, ba.kc);
      }
      ColsT<double> s2{nullptr, w.S2, ld};
      gram(Np, Np, s2, w.AS, ld, w.G, NC);
    }
    // Rayleigh-Ritz (Alg. 2) on K
    {
      RRArgs ra{};
      ra.K = w.G; ra.ldk = NC; ra.mtarget = mtarget; ra.C = w.C; ra.ldc = NC;
      ra.count_iter = (mode == kModeFull || mode == kModeXR) ? 1 : 0;
      ra.lds_cap = ba.lds_doubles;
      ra.scratch = w.rrs;
      ra.st = st;
      rr_fast_body<6, 6, kBThreads, false>(ra, lds, sh.rr);  // 16 x 16 thread grid, N <= 96
      __syncthreads();
    }
    // X = S2 C, AX = AS C, P = S2[:, nx:] C[nx:, :], R = AX - X diag(theta)
    {
      const int Np = st->Np, mk = st->mk, nx = st->nx;
      const int want_p = (mode == kModeFull || mode == kModeXR) ? 1 : 0;
      ColsT<double> s2{nullptr, w.S2, ld}, as{nullptr, w.AS, ld};
      gemm_nn(n, mk, Np, s2, w.C, NC, w.S1, ld);  // new X (S1 is free now)
      gemm_nn(n, mk, Np, as, w.C, NC, w.AX, ld);
      if (want_p && Np > nx) {
        ColsT<double> s2p{nullptr, w.S2 + (size_t)nx * ld, ld};
        gemm_nn(n, mk, Np - nx, s2p, w.C + nx, NC, w.Z, ld);
      }
      double* Xn = w.XRP;
      double* Rn = w.XRP + (size_t)mk * ld;
      double* Pn = w.XRP + (size_t)2 * mk * ld;
      for (int e = threadIdx.x; e < n * mk; e += blockDim.x) {
        const int j = e / n;
        const double x = w.S1[e];
        Xn[e] = x;
        Rn[e] = w.AX[e] - x * st->theta[j];
        if (want_p) Pn[e] = (Np > nx) ? w.Z[e] : 0.0;
      }
      __syncthreads();
      m = mk;
      has_p = want_p;
    }
  }

  // residual statistics of the current block without an update
  __device__ void evaluate() {
    State* st = w.st;
    const int NC = 3 * ba.mmax;
    ColsT<double> cand{nullptr, w.XRP, n};
    gram(2 * m, 2 * m, cand, w.XRP, n, w.G, NC);
    DecideArgs da{};
    da.G = w.G; da.ldg = NC; da.Ng = 2 * m; da.mode = kModeEval; da.m = m; da.nz = 0;
    da.has_p = 0; da.tau = 1e-10;
    for (int b = 0; b < 4; ++b) da.bases[b] = w.XRP;
    da.bases[4] = w.S1;
    da.ld = n; da.T = w.T; da.ldt = NC; da.colptr = w.colptr; da.st = st;
    decide_chol_body(da, lds, sh.ch);
    __syncthreads();
  }

  // seeded N(0,1) columns (Philox4x32-10 + Box-Muller), one stream per call
  __device__ void fill_normal(double* B, int col0, int cols) {
    const uint64_t sid = rng++;
    for (int e = threadIdx.x; e < n * cols; e += blockDim.x) {
      const int i = e % n, j = e / n;
      uint32_t r[4];
      Philox::gen((uint64_t)e + (sid << 32), ba.seed, r);
      const double u1 = ((double)r[0] + 1.0) * (1.0 / 4294967296.0);
      const double u2 = (double)r[1] * (1.0 / 4294967296.0);
      B[i + (size_t)(col0 + j) * n] = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
    }
    __syncthreads();
  }

  __device__ void reset_progress(int window) {
    if (threadIdx.x == 0) {
      w.st->best_res = INFINITY;
      w.st->best_iter = w.st->iter;
      w.st->stall_window = window;
      w.st->last_npos = -1;
    }
    __syncthreads();
  }

  // exact FP64 product on span(X), P dropped (refresh before FP64 sweeps)
  __device__ void refresh() {
    iterate(kModeXOnly, 0, m, 0);
    has_p = 0;
  }

  __device__ void solve(const BatchCone& c, BatchOut* out) {
    State* st = w.st;
    n = c.n;
    mcap = min(min(c.m_cap, ba.mmax), n);
    rng = (uint64_t)c.index << 16;
    const double sign = c.sign;
    // ---- ingest: A = sign * sym(X) from the lower triangle, FP64 + FP32
    double fro = 0.0;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int i = e % n, j = e / n;
      const double v = sign * ((i >= j) ? c.X[i + (size_t)j * n] : c.X[j + (size_t)i * n]);
      fro += v * v;
      w.A64[e] = v;
      w.A32[e] = (float)v;
    }
    fro = block_sum(fro, sh.ch.red);
    if (!isfinite(fro)) {
      if (threadIdx.x == 0) {
        BatchOut o{};
        o.status = -4;
        o.tail_est = NAN;
        o.err_bound = NAN;
        *out = o;
      }
      __syncthreads();
      return;
    }
    const int m_in = max(0, min(c.m_in, mcap));
    const int m0 = m_in > 0 ? m_in : mcap;
    const double tol = ba.tol > 0 ? ba.tol : 1e-8 * sqrt(fro) / sqrt(2.0 * m0);
    if (threadIdx.x == 0) {
      State z{};
      *st = z;
      st->n = n;
      st->tol = tol;
      st->best_res = INFINITY;
      st->last_npos = -1;
      st->stall_window = ba.prec == 0 ? 30 : 8;
      st->fro2_x = fro;
    }
    for (int e = threadIdx.x; e < n * m_in; e += blockDim.x) w.XRP[e] = c.V_in[e];
    __syncthreads();
    if (m0 > m_in) fill_normal(w.XRP, m_in, m0 - m_in);
    m = m0;
    has_p = 0;
    // initial Rayleigh-Ritz on span(X0) with an FP64 product
    for (int attempt = 0; attempt < 4; ++attempt) {
      iterate(kModeXOnly, 0, m0, 0);
      if (st->stop != kRunning) break;
      if (m >= m0) break;
      fill_normal(w.XRP, m, m0 - m);  // rank-deficient start: refill
      m = m0;
    }
    int phase = ba.prec;
    int expansions = 0;
    bool converged = false;
    int guard = 0;
    while (st->stop == kRunning && ++guard < 4 * ba.max_iter + 64) {
      iterate(has_p ? kModeFull : kModeXR, phase, m, 0);
      const int stop = st->stop;
      if (stop == kNonFinite || stop == kBreakdown) break;
      if (stop == kConverged) {
        if (phase != 0) {  // FP64 residual correction, then FP64 iterations
          phase = 0;
          refresh();
          reset_progress(30);
          continue;
        }
        converged = true;
        break;
      }
      if (stop == kStalled) {
        if (phase != 0) {
          phase = 0;
          refresh();
          reset_progress(30);
          continue;
        }
        break;
      }
      if (stop == kExpand) {  // paper §5.1: append random columns
        int e = ba.expand_cols > 0 ? ba.expand_cols : (n + 49) / 50;
        e = min(max(1, e), mcap - m);
        if (e <= 0) break;
        fill_normal(w.Z, 0, e);
        iterate(kModeXZ, phase, m + e, e);
        has_p = 0;
        ++expansions;
        reset_progress(phase == 0 ? 30 : 8);
        continue;
      }
      if (st->iter >= ba.max_iter) break;
    }
    const bool failed = st->stop == kNonFinite || st->stop == kBreakdown;
    if (!failed && !converged && phase != 0) {
      phase = 0;
      refresh();
      if (st->stop == kRunning) {
        iterate(kModeXR, 0, m, 0);
        converged = st->stop == kConverged;
      }
    }
    if (!failed && !converged) {
      evaluate();
      converged = st->eval_stop == kConverged;
    }
    const int npos = failed ? 0 : st->npos_blk;
    // ---- rebuild (eq. projection): Pi = base + Xp diag(theta) Xp^T
    for (int e = threadIdx.x; e < n * npos; e += blockDim.x)
      w.S1[e] = w.XRP[e] * st->theta[e / n];
    __syncthreads();
    {
      ColsT<double> wcols{nullptr, w.S1, n};
      wg_gemm<double, double, false, true>(n, n, npos, wcols, w.XRP, n, c.Pi, n, lds, ba.kc);
    }
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int i = e % n, j = e / n;
      if (i < j) continue;
      double v = c.Pi[e];
      if (sign < 0) v -= w.A64[e];  // Moreau: Pi(X) = X + Pi(-X), A64 = -sym(X)
      c.Pi[e] = v;
      c.Pi[j + (size_t)i * n] = v;
    }
    for (int e = threadIdx.x; e < n * m; e += blockDim.x) c.V_out[e] = w.XRP[e];
    for (int j = threadIdx.x; j < m; j += blockDim.x) c.lam[j] = st->theta[j];
    __syncthreads();
    if (threadIdx.x == 0) {
      double tail = 0.0;
      if (npos < m) {
        // estimate (uncertified): the largest non-positive Ritz value plus
        // its residual norm, an eigenvalue lies within r_g of theta_g
        tail = sqrt((double)(n - npos)) * fmax(st->guard_theta + st->guard_res, 0.0);
      } else if (m < n) {
        tail = INFINITY;  // no non-positive pair in the block to estimate from
      }
      double sp = 0.0;
      for (int k = 0; k < npos; ++k) sp += st->theta[k] * st->theta[k];
      BatchOut o{};
      o.res_fro = st->res_fro_pos;
      o.tail_est = tail;
      o.err_bound = sqrt(2.0 * o.res_fro * o.res_fro + tail * tail);
      o.pi_fro = sign > 0 ? sqrt(sp) : sqrt(fmax(fro - sp, 0.0));
      o.theta_guard = st->guard_theta;
      o.tol_used = tol;
      o.n_pos = npos;
      o.m_out = m;
      o.iters = st->iter;
      o.expansions = expansions;
      o.prec_final = phase;
      o.status = failed ? -4 : (converged ? 0 : 1);
      *out = o;
    }
    __syncthreads();
  }
};

// RRFULL: one workgroup per CU, or (false) registers limited so that two
// workgroups share a CU.
template <bool RRFULL>
__global__ __launch_bounds__(kBThreads, RRFULL ? 1 : 2) void k_batched(BatchArgs ba) {
  extern __shared__ double lds[];
  __shared__ double red[kBThreads / 64 + 128];
  __shared__ int s_list[kMaxN], s_kind[kMaxN], s_col[kMaxN], s_keep[kMaxN];
  __shared__ int s_N, s_Np, s_nx, s_stop, s_next;
  __shared__ double s_lo[kMaxM], s_hi[kMaxM];
  __shared__ int s_npos;
  __shared__ double s_tnorm, s_pivmin;
  BShared sh;
  sh.ch = CholShared{s_list, s_kind, s_col, s_keep, &s_N, &s_Np, &s_nx, &s_stop,
                     red};
  sh.rr = RRShared{s_lo, s_hi, &s_npos, &s_tnorm, &s_pivmin};
  BScratch ws = bscratch_at(ba.scratch + (size_t)blockIdx.x * ba.scratch_stride, ba.nmax, ba.mmax);
  ConeSolver<RRFULL> cs(ba, ws, sh, lds);
  // every workgroup drains the queue and leaves when it is empty
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(ba.counter, 1);
    __syncthreads();
    const int c = s_next;
    __syncthreads();
    if (c >= ba.count) break;
    const BatchCone cone = ba.cones[c];
    cs.solve(cone, ba.outs + cone.index);
  }
}

__global__ void k_fill_int(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

size_t batched_static_lds_bytes() {
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, (const void*)k_batched<true>) != hipSuccess) return 4096;
  return fa.sharedSizeBytes;
}

hipError_t launch_batched(const BatchArgs& a, bool rr_full, int grid, hipStream_t st) {
  // queue head back to 0 with a kernel (capturable, no memset node)
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, a.counter, 0);
  if (rr_full)
    hipLaunchKernelGGL(k_batched<true>, dim3(grid), dim3(kBThreads), a.lds_doubles * 8, st, a);
  else
    hipLaunchKernelGGL(k_batched<false>, dim3(grid), dim3(kBThreads), a.lds_doubles * 8, st, a);
  return hipGetLastError();
}

hipError_t batched_init(int lds_bytes) {
  (void)hipFuncSetAttribute((const void*)k_batched<true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  (void)hipFuncSetAttribute((const void*)k_batched<false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  return hipGetLastError();
}

}  // namespace psdp
