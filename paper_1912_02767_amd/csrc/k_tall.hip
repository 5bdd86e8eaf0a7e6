// Tall-skinny kernels over n-row blocks: ingest, Gram partial sums,
// deterministic reductions, block-times-small-matrix products, the
// Ritz-vector update with its residual, random fills, rebuild.
#include "common.h"

namespace psdp {

// ---------------------------------------------------------------- ingest --
// A = sign * sym(X) from the lower triangle of X, written in FP64 (full,
// zero padded to lda) and in the product precision.  One 32x32 tile of the
// lower triangle per workgroup: the tile is read once (coalesced) and
// written to both (I,J) and, transposed through LDS, (J,I).
// Also per-workgroup partial ||X||_F^2 and a non-finite flag.
constexpr int kTile = 32;

template <int PREC>
__global__ __launch_bounds__(256) void k_ingest(const double* __restrict__ X, int ldx, int n,
                                                double sign, double* __restrict__ A64, int lda,
                                                void* __restrict__ Alp, double* fro_partial,
                                                int* nonfinite) {
  __shared__ double tile[kTile][kTile + 1];
  __shared__ double red[256];
  // map linear block id -> lower-triangular tile (bi >= bj)
  int b = blockIdx.x;
  int bi = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((bi + 1) * (bi + 2) / 2 <= b) ++bi;
  while (bi * (bi + 1) / 2 > b) --bi;
  int bj = b - bi * (bi + 1) / 2;
  int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;  // 32 x 8
  int i0 = bi * kTile, j0 = bj * kTile;
  double fro = 0.0;
  int bad = 0;
  for (int jj = ty; jj < kTile; jj += 8) {
    int i = i0 + tx, j = j0 + jj;
    double v = 0.0;
    if (i < n && j < n) {
      // element (i, j) of the symmetric matrix from the lower triangle
      v = (i >= j) ? X[i + (size_t)j * ldx] : X[j + (size_t)i * ldx];
      if (!isfinite(v)) bad = 1;
      if (bi != bj || i >= j) fro += (i == j ? 1.0 : 2.0) * v * v;
    }
    tile[jj][tx] = sign * v;
  }
  __syncthreads();
  // write (I,J) tile
  for (int jj = ty; jj < kTile; jj += 8) {
    int i = i0 + tx, j = j0 + jj;
    if (i < lda && j < lda) {
      double v = tile[jj][tx];
      A64[i + (size_t)j * lda] = v;
      if (PREC == 1) ((float*)Alp)[i + (size_t)j * lda] = (float)v;
      if (PREC == 2) ((uint16_t*)Alp)[i + (size_t)j * lda] = f32_to_bf16_rne((float)v);
    }
  }
  if (bi != bj) {
    // (J,I) tile = transpose
    for (int ii = ty; ii < kTile; ii += 8) {
      int i = j0 + tx, j = i0 + ii;  // row in J block, column in I block
      if (i < lda && j < lda) {
        double v = tile[tx][ii];
        A64[i + (size_t)j * lda] = v;
        if (PREC == 1) ((float*)Alp)[i + (size_t)j * lda] = (float)v;
        if (PREC == 2) ((uint16_t*)Alp)[i + (size_t)j * lda] = f32_to_bf16_rne((float)v);
      }
    }
  }
  if (bad) atomicOr(nonfinite, 1);
  red[threadIdx.x] = fro;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) fro_partial[blockIdx.x] = red[0];
}

// The kernel writes every element (i, j) with i, j < lda (zero padding
// included): A64 (and Alp) must hold lda x lda elements, i.e. at least lda
// allocated columns (cols_alloc).
hipError_t launch_ingest(const double* X, int ldx, int n, double sign, double* A64, int lda,
                         int cols_alloc, void* Alp, int prec, double* fro_partial, int* nonfinite,
                         hipStream_t st, int* nblocks_out) {
  if (n < 0 || lda < n || cols_alloc < lda) return hipErrorInvalidValue;
  int T = (lda + kTile - 1) / kTile;
  int nb = T * (T + 1) / 2;
  if (nblocks_out) *nblocks_out = nb;
  if (prec == 1)
    hipLaunchKernelGGL(k_ingest<1>, dim3(nb), dim3(256), 0, st, X, ldx, n, sign, A64, lda, Alp,
                       fro_partial, nonfinite);
  else if (prec == 2)
    hipLaunchKernelGGL(k_ingest<2>, dim3(nb), dim3(256), 0, st, X, ldx, n, sign, A64, lda, Alp,
                       fro_partial, nonfinite);
  else
    hipLaunchKernelGGL(k_ingest<0>, dim3(nb), dim3(256), 0, st, X, ldx, n, sign, A64, lda, Alp,
                       fro_partial, nonfinite);
  return hipGetLastError();
}

// out[0] = sum of partial[0..count) in a fixed order (one workgroup).
__global__ __launch_bounds__(256) void k_reduce_sum(const double* partial, int count, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

hipError_t launch_reduce_sum(const double* partial, int count, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, st, partial, count, out);
  return hipGetLastError();
}

// ------------------------------------------------------------ Gram partials --
// For column sets B (nb columns, via column pointers) and Y (ny columns):
//   G_part[blk] = B_blk^T B_blk   (nb x nb)          if Y == nullptr
//   G_part[blk] = B_blk^T Y_blk   (nb x ny)          otherwise
// over row block blk of kGramRows rows.  Partials are reduced later in a
// fixed order, so the result is bitwise reproducible.  Column counts can come
// from device memory (cnt_dev) with host upper bounds for the grid.
// Layout of a partial: column-major nb_max x ny_max with leading dim ldp.
constexpr int kGT = 64;   // output tile 64 x 64 per workgroup, 4x4 per thread
constexpr int kGR = 32;   // rows staged per step

__global__ __launch_bounds__(256) void k_gram_partial(ColMap bptr, ColMap yptr, int has_y,
                                                      const int* __restrict__ nb_dev, int nb_host,
                                                      const int* __restrict__ ny_dev, int ny_host,
                                                      int n, double* __restrict__ part, int ldp,
                                                      size_t part_stride, const int* stop) {
  if (stop && *stop) return;
  const int nb = nb_dev ? *nb_dev : nb_host;
  const int ny = has_y ? (ny_dev ? *ny_dev : ny_host) : nb;
  const int ti = blockIdx.y * kGT, tj = blockIdx.z * kGT;
  if (ti >= nb || tj >= ny) return;
  const bool sym = !has_y;
  if (sym && tj + kGT <= ti) return;  // lower tiles mirrored at the end
  __shared__ double sb[kGR][kGT + 1];
  __shared__ double sy[kGR][kGT + 1];
  __shared__ const double* pb[kGT];
  __shared__ const double* py[kGT];
  __shared__ int okb[kGT], oky[kGT];
  if (threadIdx.x < kGT) {
    // inactive columns alias column 0 (always valid) and are masked to zero
    const int c = threadIdx.x;
    const bool vb = ti + c < nb;
    const bool vy = sym ? (tj + c < nb) : (tj + c < ny);
    pb[c] = bptr.col(vb ? ti + c : 0);
    py[c] = sym ? bptr.col(vy ? tj + c : 0) : yptr.col(vy ? tj + c : 0);
    okb[c] = vb;
    oky[c] = vy;
  }
  __syncthreads();
  const int r0 = blockIdx.x * kGramRows;
  const int r1 = min(n, r0 + kGramRows);
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;  // 16 x 16 threads, 4x4 each
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
  // kGR rows x 64 columns of B and Y per stage, eight values each per thread;
  // the next stage's loads are in flight while this stage is multiplied
  constexpr int PER = kGR * kGT / 256;
  double cb[PER], cy[PER];
  // unconditional loads (rows clamped, global address space), the zero
  // padding applied at the LDS store: no wait between the loads of a stage
  typedef const __attribute__((address_space(1))) double* gptr;
  auto load_stage = [&](int rr) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int r = e % kGR, c = e / kGR;
      const int rowc = min(rr + r, r1 - 1);
      cb[u] = ((gptr)pb[c])[rowc];
      cy[u] = ((gptr)py[c])[rowc];
    }
  };
  load_stage(r0);
  for (int rr = r0; rr < r1; rr += kGR) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int r = e % kGR, c = e / kGR;
      const bool rowok = rr + r < r1;
      sb[r][c] = (rowok && okb[c]) ? cb[u] : 0.0;
      sy[r][c] = (rowok && oky[c]) ? cy[u] : 0.0;
    }
    __syncthreads();
    if (rr + kGR < r1) load_stage(rr + kGR);
#pragma unroll 4
    for (int r = 0; r < kGR; ++r) {
      double bv[4], yv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) bv[a] = sb[r][ty + 16 * a];
#pragma unroll
      for (int c = 0; c < 4; ++c) yv[c] = sy[r][tx + 16 * c];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = fma(bv[a], yv[c], acc[a][c]);
    }
    __syncthreads();
  }
  double* out = part + (size_t)blockIdx.x * part_stride;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int i = ti + ty + 16 * a, j = tj + tx + 16 * c;
      if (i < nb && j < ny) {
        out[i + (size_t)j * ldp] = acc[a][c];
        if (sym && i != j) out[j + (size_t)i * ldp] = acc[a][c];
      }
    }
}

// out[e] = sum_b part[b][e], e over an ldp x cols column-major panel; fixed
// summation order (b ascending) for reproducibility.
__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ part,
                                                         int nblk, size_t part_stride, int ldp,
                                                         const int* rows_dev, int rows_host,
                                                         const int* cols_dev, int cols_host,
                                                         double* __restrict__ out, int ldo,
                                                         const int* stop) {
  if (stop && *stop) return;
  int rows = rows_dev ? *rows_dev : rows_host;
  int cols = cols_dev ? *cols_dev : cols_host;
  int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * cols) return;
  int i = e % rows, j = e / rows;
  // 32 loads in flight (all of a group issued before any is added); the
  // partial sums are combined in a fixed order
  const double* p = part + i + (size_t)j * ldp;
  constexpr int W = 32;
  double s[W];
#pragma unroll
  for (int u = 0; u < W; ++u) s[u] = 0.0;
  for (int b = 0; b < nblk; b += W) {
    double v[W];
#pragma unroll
    for (int u = 0; u < W; ++u) v[u] = p[(size_t)min(b + u, nblk - 1) * part_stride];
#pragma unroll
    for (int u = 0; u < W; ++u) s[u] += (b + u < nblk) ? v[u] : 0.0;
  }
#pragma unroll
  for (int h = W / 2; h > 0; h /= 2)
#pragma unroll
    for (int u = 0; u < h; ++u) s[u] += s[u + h];
  out[i + (size_t)j * ldo] = s[0];
}

// --------------------------------------------------------------- tsmm ---
// Y[:, j] = sum_k src_k * M[k, j] for j < q, k < kk, rows < n.
// Columns of the source via column pointers.  M is kk x q (ldm), FP64.
// Each workgroup: 64 rows x 16 output columns; the source row block is
// staged in LDS in chunks of 32 columns.
constexpr int kTR = 64;
constexpr int kTQ = 16;
constexpr int kTK = 32;

constexpr int kTGroup = 5;  // chunks whose loads are issued together (kk <= 160 in one group)

__device__ inline void tsmm_tile(const ColMap& src, int kk, int q,
                                 const double* __restrict__ M, int ldm, int n,
                                 double* __restrict__ Y, int ldy, int row0, int col0,
                                 double (*sS)[kTR + 1], double (*sM)[kTQ + 1],
                                 const double** sp) {
  // 256 threads: thread -> (row r = tid % 64, col group cg = tid / 64 -> 4 cols)
  const int r = threadIdx.x % kTR;
  const int cg = threadIdx.x / kTR;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // per chunk: 32 source columns x 64 rows (8 values per thread) and 32 x 16
  // of M (2 per thread).  The loads of a whole group of chunks (the full
  // trial basis in one group) are issued before the first chunk is used:
  // one global-memory round trip instead of one per chunk.
  constexpr int PS = kTK * kTR / 256, PM = kTK * kTQ / 256;
  double cs[kTGroup][PS], cm[kTGroup][PM];
  // column pointers of the group in LDS (sp[k - g0]): resolving a column
  // inside the load loop would put a dependent pointer load and a branch in
  // front of every element.  Every load of the group is unconditional (indices
  // clamped); the zero padding is applied when the values reach LDS.
  typedef const __attribute__((address_space(1))) double* gptr;
  for (int g0 = 0; g0 < kk; g0 += kTGroup * kTK) {
    for (int k = g0 + (int)threadIdx.x; k < min(kk, g0 + kTGroup * kTK); k += 256)
      sp[k - g0] = src.col(k);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kTGroup; ++c) {
      const int k0 = g0 + c * kTK;
#pragma unroll
      for (int u = 0; u < PS; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int rr = e % kTR, kc = e / kTR;
        const int k = min(k0 + kc, kk - 1);
        cs[c][u] = ((gptr)sp[k - g0])[min(row0 + rr, n - 1)];
      }
#pragma unroll
      for (int u = 0; u < PM; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int kc = e % kTK, cc = e / kTK;
        cm[c][u] = M[min(k0 + kc, kk - 1) + (size_t)min(col0 + cc, q - 1) * ldm];
      }
    }
#pragma unroll
    for (int c = 0; c < kTGroup; ++c) {
      const int k0 = g0 + c * kTK;
      if (k0 >= kk) break;  // uniform
#pragma unroll
      for (int u = 0; u < PS; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int rr = e % kTR, kc = e / kTR;
        sS[kc][rr] = (row0 + rr < n && k0 + kc < kk) ? cs[c][u] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < PM; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int kc = e % kTK, cc = e / kTK;
        sM[kc][cc] = (k0 + kc < kk && col0 + cc < q) ? cm[c][u] : 0.0;
      }
      __syncthreads();
#pragma unroll 8
      for (int kc = 0; kc < kTK; ++kc) {
        double sv = sS[kc][r];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) acc[cc] = fma(sv, sM[kc][cg * 4 + cc], acc[cc]);
      }
      __syncthreads();
    }
  }
  int row = row0 + r;
  if (row < n) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int j = col0 + cg * 4 + c;
      if (j < q) Y[row + (size_t)j * ldy] = acc[c];
    }
  }
}

__global__ __launch_bounds__(256) void k_tsmm(ColMap src,
                                              const int* kk_dev, int kk_host,
                                              const int* q_dev, int q_host,
                                              const double* __restrict__ M, int ldm, int n,
                                              double* __restrict__ Y, int ldy, const int* stop) {
  if (stop && *stop) return;
  __shared__ double sS[kTK][kTR + 1];
  __shared__ double sM[kTK][kTQ + 1];
  __shared__ const double* sp[kTGroup * kTK];
  int kk = kk_dev ? *kk_dev : kk_host;
  int q = q_dev ? *q_dev : q_host;
  int row0 = blockIdx.x * kTR, col0 = blockIdx.y * kTQ;
  if (col0 >= q) return;
  tsmm_tile(src, kk, q, M, ldm, n, Y, ldy, row0, col0, sS, sM, sp);
}

// ----------------------------------------------------------- Ritz update ---
// X = S C, AX = AS C, P = S[:, nx:] C[nx:, :] (paper §5.1: Delta X in the
// BLOPEX form), R = AX - X diag(theta).  C is Np x mk (ldc), all counts
// from the device state.  One workgroup: 64 rows x 16 columns of all four.
__global__ __launch_bounds__(256) void k_update(const double* __restrict__ S,
                                                const double* __restrict__ AS, int lds,
                                                const double* __restrict__ C, int ldc,
                                                const State* __restrict__ st, int want_p, int n,
                                                double* __restrict__ Xo, double* __restrict__ AXo,
                                                double* __restrict__ Po, double* __restrict__ Ro,
                                                int ldo) {
  if (st->stop) return;
  const int Np = st->Np, mk = st->mk, nx = st->nx;
  const int row0 = blockIdx.x * kTR, col0 = blockIdx.y * kTQ;
  if (col0 >= mk) return;
  const int r = threadIdx.x % kTR;
  const int cg = threadIdx.x / kTR;
  __shared__ double sS[kTK][kTR + 1];
  __shared__ double sA[kTK][kTR + 1];
  __shared__ double sC[kTK][kTQ + 1];
  double ax[4] = {0, 0, 0, 0}, xx[4] = {0, 0, 0, 0}, pp[4] = {0, 0, 0, 0};
  constexpr int PS = kTK * kTR / 256, PC = kTK * kTQ / 256;
  // every chunk of a group (the whole trial basis in one group) is loaded
  // before the first is used, indices clamped; the zero padding is applied
  // when the values reach LDS
  double cs[kTGroup][PS], ca[kTGroup][PS], cc_[kTGroup][PC];
  for (int g0 = 0; g0 < Np; g0 += kTGroup * kTK) {
#pragma unroll
    for (int c = 0; c < kTGroup; ++c) {
      const int k0 = g0 + c * kTK;
#pragma unroll
      for (int u = 0; u < PS; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int rr = e % kTR, kc = e / kTR;
        const size_t o = min(row0 + rr, n - 1) + (size_t)min(k0 + kc, Np - 1) * lds;
        cs[c][u] = S[o];
        ca[c][u] = AS[o];
      }
#pragma unroll
      for (int u = 0; u < PC; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int kc = e % kTK, cc = e / kTK;
        cc_[c][u] = C[min(k0 + kc, Np - 1) + (size_t)min(col0 + cc, mk - 1) * ldc];
      }
    }
#pragma unroll
    for (int c = 0; c < kTGroup; ++c) {
      const int k0 = g0 + c * kTK;
      if (k0 >= Np) break;  // uniform
#pragma unroll
      for (int u = 0; u < PS; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int rr = e % kTR, kc = e / kTR;
        const bool ok = (row0 + rr < n && k0 + kc < Np);
        sS[kc][rr] = ok ? cs[c][u] : 0.0;
        sA[kc][rr] = ok ? ca[c][u] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < PC; ++u) {
        const int e = threadIdx.x + 256 * u;
        const int kc = e % kTK, cc = e / kTK;
        sC[kc][cc] = (k0 + kc < Np && col0 + cc < mk) ? cc_[c][u] : 0.0;
      }
      __syncthreads();
#pragma unroll 8
      for (int kc = 0; kc < kTK; ++kc) {
        double sv = sS[kc][r], a = sA[kc][r];
        bool isp = (k0 + kc) >= nx;
#pragma unroll
        for (int c2 = 0; c2 < 4; ++c2) {
          double cv = sC[kc][cg * 4 + c2];
          xx[c2] = fma(sv, cv, xx[c2]);
          ax[c2] = fma(a, cv, ax[c2]);
          if (isp) pp[c2] = fma(sv, cv, pp[c2]);
        }
      }
      __syncthreads();
    }
  }
  int row = row0 + r;
  if (row < n) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int j = col0 + cg * 4 + c;
      if (j < mk) {
        size_t o = row + (size_t)j * ldo;
        Xo[o] = xx[c];
        AXo[o] = ax[c];
        Ro[o] = ax[c] - xx[c] * st->theta[j];
        if (want_p) Po[o] = pp[c];
      }
    }
  }
}

// --------------------------------------------------------- random fill ---
// B[:, col0 .. col0+cols) = N(0,1) from Philox4x32-10 keyed by (seed,
// stream_id); counter = element index, so the values do not depend on the
// launch shape.
__global__ __launch_bounds__(256) void k_fill_normal(double* B, int ld, int n, int col0, int cols,
                                                     uint64_t seed, uint64_t stream_id) {
  size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  size_t total = (size_t)n * cols;
  if (e >= total) return;
  int i = (int)(e % n), j = (int)(e / n);
  uint32_t r[4];
  Philox::gen((uint64_t)e + (stream_id << 40), seed, r);
  // Box-Muller on two 32-bit uniforms in (0, 1]
  double u1 = ((double)r[0] + 1.0) * (1.0 / 4294967296.0);
  double u2 = ((double)r[1]) * (1.0 / 4294967296.0);
  double z = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
  B[i + (size_t)(col0 + j) * ld] = z;
}

hipError_t launch_fill_normal(double* B, int ld, int n, int col0, int cols, uint64_t seed,
                              uint64_t stream_id, hipStream_t st) {
  size_t total = (size_t)n * cols;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_normal, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, B,
                     ld, n, col0, cols, seed, stream_id);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_copy_cols(const double* src, int lds, double* dst,
                                                   int ldd, int n, int cols) {
  size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)n * cols) return;
  int i = (int)(e % n), j = (int)(e / n);
  dst[i + (size_t)j * ldd] = src[i + (size_t)j * lds];
}

hipError_t launch_copy_cols(const double* src, int lds, double* dst, int ldd, int n, int cols,
                            hipStream_t st) {
  size_t total = (size_t)n * cols;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, src,
                     lds, dst, ldd, n, cols);
  return hipGetLastError();
}

// ----------------------------------------------------------- rebuild ---
// Pi = base + W W^T with W = V diag(sqrt(lt)) over the positive pairs
// (paper §1 eq. `projection`; the negative side adds X by the Moreau
// identity).  base = 0 (positive side) or sym(X) read from the FP64 copy
// (negative side; A64 holds -sym(X) there, so base = -A64).  Each
// workgroup computes one 64 x 64 tile (i, j), i >= j, of the lower triangle
// on the matrix cores (v_mfma_f64_16x16x4f64: wave w takes rows 16w .. 16w +
// 15 of the tile, four 16 x 16 column tiles), K = the pairs in chunks of 16
// staged in LDS (V diag(lt) for the rows, V for the columns), and writes it
// and its transpose through an LDS copy of the tile so that both stores are
// coalesced: the result is symmetric by construction.
constexpr int kRB = 64;
constexpr int kRK = 16;       // pairs per LDS chunk
constexpr int kRLd = kRB + 1;  // padded LDS row
typedef double rb_d4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_rebuild(const double* __restrict__ V, int ldv,
                                                 const double* __restrict__ lt, int mt, int n,
                                                 const double* __restrict__ base, int ldb,
                                                 double base_sign, double* __restrict__ Pi,
                                                 int ldpi) {
  __shared__ double sa[kRK * kRLd];  // sa[k * 65 + r] = V(i0 + r, k) lt[k]
  __shared__ double sb[kRK * kRLd];  // sb[k * 65 + c] = V(j0 + c, k)
  __shared__ double tile[kRB * kRLd];
  // lower-triangular tile index -> (ti, tj), ti >= tj
  int ti = (int)((sqrt(8.0 * blockIdx.x + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= (int)blockIdx.x) ++ti;
  while (ti * (ti + 1) / 2 > (int)blockIdx.x) --ti;
  const int tj = (int)blockIdx.x - ti * (ti + 1) / 2;
  const int i0 = ti * kRB, j0 = tj * kRB;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, li = lane & 15, g = lane >> 4;
  rb_d4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = rb_d4{0.0, 0.0, 0.0, 0.0};
  // 2 x 16 x 64 values per chunk, four per thread per side, fetched into
  // registers one chunk ahead (in flight while the current chunk is
  // multiplied); rows past n and pairs past mt are zero
  constexpr int PU = kRK * kRB / 256;
  double pa[PU], pb[PU], pw[PU];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int e = t + 256 * u, r = e & 63, kk = e >> 6, k = k0 + kk;
      const bool kin = k < mt;
      pw[u] = kin ? lt[k] : 0.0;
      pa[u] = (kin && i0 + r < n) ? V[(i0 + r) + (size_t)k * ldv] : 0.0;
      pb[u] = (kin && j0 + r < n) ? V[(j0 + r) + (size_t)k * ldv] : 0.0;
    }
  };
  if (mt > 0) fetch(0);
  for (int k0 = 0; k0 < mt; k0 += kRK) {
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int e = t + 256 * u, r = e & 63, kk = e >> 6;
      sa[kk * kRLd + r] = pa[u] * pw[u];
      sb[kk * kRLd + r] = pb[u];
    }
    __syncthreads();
    if (k0 + kRK < mt) fetch(k0 + kRK);
#pragma unroll
    for (int ks = 0; ks < kRK; ks += 4) {
      const double a = sa[(ks + g) * kRLd + 16 * wv + li];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double b = sb[(ks + g) * kRLd + 16 * c + li];
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // D[row][col] of column tile c: lane -> col 16 c + li, rows g + 4 r
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) tile[(16 * wv + g + 4 * r) * kRLd + 16 * c + li] = acc[c][r];
  __syncthreads();
  // Pi(i0 + r, j0 + c) for consecutive r, then the transpose Pi(j0 + r, i0 + c)
#pragma unroll 4
  for (int u = 0; u < kRB * kRB / 256; ++u) {
    const int e = t + 256 * u, r = e & 63, c = e >> 6;
    const int i = i0 + r, j = j0 + c;
    if (i < n && j < n) {
      double v = tile[r * kRLd + c];
      if (base) v += base_sign * base[i + (size_t)j * ldb];
      Pi[i + (size_t)j * ldpi] = v;
    }
  }
  if (ti != tj) {
#pragma unroll 4
    for (int u = 0; u < kRB * kRB / 256; ++u) {
      const int e = t + 256 * u, r = e & 63, c = e >> 6;
      const int i = j0 + r, j = i0 + c;  // element (i, j) of Pi = tile(c, r)
      if (i < n && j < n) {
        double v = tile[c * kRLd + r];
        if (base) v += base_sign * base[i + (size_t)j * ldb];
        Pi[i + (size_t)j * ldpi] = v;
      }
    }
  }
}

}  // namespace psdp

// C-linkage launchers used by the driver (kept inside the library).
namespace psdp {
hipError_t launch_gram_partial(const ColMap& bptr, const ColMap* yptr,
                               const int* nb_dev, int nb_host, const int* ny_dev, int ny_host,
                               int n, double* part, int ldp, size_t part_stride, int* nblk_out,
                               const int* stop, hipStream_t st) {
  int nblk = (n + kGramRows - 1) / kGramRows;
  if (nblk_out) *nblk_out = nblk;
  int tb = (nb_host + kGT - 1) / kGT;
  int ty = yptr ? (ny_host + kGT - 1) / kGT : tb;
  if (tb == 0 || ty == 0) return hipSuccess;
  ColMap ym = yptr ? *yptr : bptr;
  hipLaunchKernelGGL(k_gram_partial, dim3(nblk, tb, ty), dim3(256), 0, st, bptr, ym,
                     yptr ? 1 : 0, nb_dev,
                     nb_host, ny_dev, ny_host, n, part, ldp, part_stride, stop);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* part, int nblk, size_t part_stride, int ldp,
                                  const int* rows_dev, int rows_host, const int* cols_dev,
                                  int cols_host, double* out, int ldo, const int* stop,
                                  hipStream_t st) {
  int total = rows_host * cols_host;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_partials, dim3((total + 255) / 256), dim3(256), 0, st, part, nblk,
                     part_stride, ldp, rows_dev, rows_host, cols_dev, cols_host, out, ldo, stop);
  return hipGetLastError();
}

__global__ void k_set_stop(State* st, int v) {
  if (threadIdx.x == 0) st->stop = v;
}

hipError_t launch_set_stop(State* st, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_stop, dim3(1), dim3(64), 0, s, st, v);
  return hipGetLastError();
}

__global__ void k_set_int(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_tsmm(const ColMap& src, const int* kk_dev, int kk_host, const int* q_dev,
                       int q_host, const double* M, int ldm, int n, double* Y, int ldy,
                       const int* stop, hipStream_t st) {
  if (q_host <= 0 || n <= 0) return hipSuccess;
  dim3 grid((n + kTR - 1) / kTR, (q_host + kTQ - 1) / kTQ);
  hipLaunchKernelGGL(k_tsmm, grid, dim3(256), 0, st, src, kk_dev, kk_host, q_dev, q_host, M, ldm,
                     n, Y, ldy, stop);
  return hipGetLastError();
}

hipError_t launch_update(const double* S, const double* AS, int lds, const double* C, int ldc,
                         const State* stt, int want_p, int n, int mk_host, double* Xo,
                         double* AXo, double* Po, double* Ro, int ldo, hipStream_t st) {
  if (mk_host <= 0) return hipSuccess;
  dim3 grid((n + kTR - 1) / kTR, (mk_host + kTQ - 1) / kTQ);
  hipLaunchKernelGGL(k_update, grid, dim3(256), 0, st, S, AS, lds, C, ldc, stt, want_p, n, Xo,
                     AXo, Po, Ro, ldo);
  return hipGetLastError();
}

hipError_t launch_rebuild(const double* V, int ldv, const double* lt, int mt, int n,
                          const double* base, int ldb, double base_sign, double* Pi, int ldpi,
                          hipStream_t st) {
  const int T = (n + kRB - 1) / kRB;
  dim3 grid((unsigned)(T * (T + 1) / 2));
  hipLaunchKernelGGL(k_rebuild, grid, dim3(256), 0, st, V, ldv, lt, mt, n, base, ldb, base_sign,
                     Pi, ldpi);
  return hipGetLastError();
}
}  // namespace psdp
