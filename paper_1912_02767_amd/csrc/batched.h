// Shared declarations of the batched persistent engine (kernel side and
// host side).
#pragma once
#include <stddef.h>

#include "common.h"

namespace psdp {

constexpr int kBThreads = 256;    // threads per workgroup (four waves)
constexpr int kBatchMaxN = 256;   // largest cone order of the batched engine
constexpr int kBatchMaxM = 32;    // largest block of the batched engine

// One cone of the queue (device array, host-ordered by decreasing work).
struct BatchCone {
  int n;           // order; every matrix of the cone has leading dimension n
  int m_cap;       // column capacity of V_out / lam
  int m_in;        // warm-start columns in V_in (0: cold start with m_cap columns)
  int index;       // position in the caller's arrays (output slot, RNG stream)
  double sign;     // +1 positive side, -1 negative side (Moreau)
  const double* X; // n x n, lower triangle read
  const double* V_in;
  double* V_out;   // may equal V_in (read completely before written)
  double* lam;
  double* Pi;      // n x n, both triangles written
};

// Per-cone result (device array indexed by BatchCone::index).
struct BatchOut {
  double err_bound, res_fro, tail_est, pi_fro, theta_guard, tol_used;
  int n_pos, m_out, iters, status, expansions, prec_final;
};

struct BatchArgs {
  const BatchCone* cones;
  BatchOut* outs;
  int count;
  int* counter;            // queue head, set to 0 by the launch sequence
  char* scratch;           // grid x scratch_stride bytes
  size_t scratch_stride;
  int nmax, mmax;          // scratch sizing (largest n and block in the batch)
  int prec;                // product precision of the first phase: 0 FP64, 1 FP32
  double tol;              // <= 0: 1e-8 ||X||_F / sqrt(2 m) per cone
  int max_iter;
  unsigned long long seed;
  int expand_cols;         // 0: ceil(n / 50)
  size_t lds_doubles;      // dynamic LDS of the launch
  int kc;                  // k-chunk of the workgroup GEMM
};

// One cone of the batched exact path (zero-padded full eigendecomposition).
struct EigCone {
  const double* X;  // n x n, lower triangle read
  double* Pi;       // n x n output
  double* V;        // n x m_cap leading eigenvectors, or nullptr
  double* lam;      // m_cap leading eigenvalues, or nullptr
  int n, m_cap;
};
hipError_t launch_eig_pad(const EigCone* cones, int count, double* A, int nb, int* bad,
                          hipStream_t st);
hipError_t launch_eig_rebuild(const EigCone* cones, int count, const double* A, const double* D,
                              int nb, hipStream_t st);
hipError_t launch_eig_leading(const EigCone* cones, int count, const double* A, const double* D,
                              int nb, int* out, hipStream_t st);

size_t batched_scratch_bytes(int nmax, int mmax);
size_t batched_static_lds_bytes();
hipError_t launch_batched(const BatchArgs& a, bool rr_full, int grid, hipStream_t st);
hipError_t batched_init(int lds_bytes);

// Dynamic LDS doubles the batched kernel needs for blocks of width <= mmax
// with the given GEMM k-chunk (the Rayleigh-Ritz body, the Cholesky body
// and the GEMM staging share the same space).
inline size_t batched_lds_doubles(int mmax, bool /*one_per_cu*/, int kc) {
  const size_t N = 3 * (size_t)mmax;
  const size_t n2 = N * (N + 1) / 2;
  const size_t ldy = (N & 1) ? N : N + 1;
  const size_t wy = 16 * 16 + 17 * (size_t)mmax;  // rr_fast_tbw: T block + W (ld 17)
  const size_t lp = 96;  // 16 row groups x 6 = 16 column groups x 6
  size_t ysp = ldy * mmax;
  if (ysp < 6 * lp) ysp = 6 * lp;
  if (ysp < (size_t)kBThreads) ysp = kBThreads;
  const size_t rr = n2 + 5 * N + ysp + (wy > 3 * N ? wy : 3 * N) + kBThreads / 64 + 4;
  const size_t chol = n2 + N + (N * 16 > 1024 ? N * 16 : 1024) + 8;
  const size_t gemm = 2 * (size_t)kc * 65;
  size_t m = rr > chol ? rr : chol;
  return m > gemm ? m : gemm;
}

}  // namespace psdp
