// Internal declarations shared by the HIP kernels and the host driver.
// gfx950 only; wavefront size 64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psdp {

constexpr int kWave = 64;
constexpr int kMaxM = 48;             // largest block (X columns) of the single-cone engine
constexpr int kMaxN = 3 * kMaxM;      // largest trial basis [X, R, P]
constexpr int kRowBlk = 256;          // rows per workgroup in the tall-skinny kernels
constexpr int kGramRows = 32;         // rows per partial Gram block

// Why an iteration stopped (device state `stop`).
enum StopReason : int {
  kRunning = 0,
  kConverged = 1,
  kExpand = 2,     // more positive Ritz values than the block holds (paper §5.1)
  kStalled = 3,    // residual no longer decreasing at this product precision
  kNonFinite = 4,
  kBreakdown = 5,  // trial basis lost rank beyond recovery
  kEvaluated = 6,  // evaluation pass only (statistics of the current block)
  kSpecAbort = 7,  // a speculatively queued iteration found the block size changed
};

// Composition of the trial basis of one iteration.
enum IterMode : int {
  kModeFull = 0,   // [X, R_active, P_active]  (paper §5.1 Alg. 3: span(X, R, dX))
  kModeXOnly = 1,  // [X]: Rayleigh-Ritz on span(X) (warm-start RR, refresh)
  kModeXR = 2,     // [X, R_active] (first iteration, P dropped)
  kModeXZ = 3,     // [X, Z]: expansion with random columns (paper §5.1)
  kModeEval = 4,   // residual statistics of the current block, no update
};

// Device-resident state of one single-cone solve.  The host mirrors it
// after each iteration.  Sizes are counts of columns.
struct State {
  // sizes of the current iteration
  int n;
  int m;         // X columns (block size)
  int nr;        // residual columns in the trial basis
  int np;        // P columns in the trial basis
  int nz;        // random expansion columns in the trial basis
  int N;         // m + nr + np + nz
  int Np;        // columns kept by the Cholesky-QR with dropping
  int nx;        // kept columns that came from X
  int mk;        // Ritz pairs kept by the Rayleigh-Ritz (new m)
  int has_p;     // P (paper's Delta X) is valid
  int mode;      // IterMode
  // control
  int iter;
  int stop;      // StopReason
  int npos_rr;   // positive Ritz values among all Np of the last RR
  int npos_blk;  // positive Ritz values among the kept mk
  int best_iter;
  int stall_window;
  int nonfinite;
  double tol;
  double best_res;
  double res_max_pos;   // max residual norm over positive Ritz pairs
  double guard_theta;   // largest non-positive Ritz value in the block
  double guard_res;     // its residual norm
  double res_fro_pos;   // ||R||_F over positive pairs
  double theta_min_pos; // smallest positive Ritz value
  double fro2_x;        // ||X||_F^2 of the symmetrized input
  int expand_req;       // last RR found more positive Ritz values than it kept
  int Np1;              // kept columns of the first Cholesky-QR pass
  int jacobi_rounds;    // rotation rounds of the last RR
  int eval_stop;        // decision an evaluation pass would have taken
  int last_npos;        // positive count at the last progress check
  int fixed_block;      // truncated top-r variant: converged once every pair of the
                        // block meets tol, never expanded
  long long t_phase[12]; // device clock at phase boundaries of the last RR (0-4)
                         // and of the last first-pass Cholesky-QR (6-10)
  long long t_sub[12];    // device clock ticks inside the last RR: tridiagonalization
                          // (a)+(c), (b); back-transformation stages (i), (ii) T,
                          // (ii) T W, (iii); multisection rounds; cluster
                          // orthogonalization; and inside the last first-pass
                          // Cholesky factorization: diagonal blocks, panels, trailing
  // per column data (block order = descending Ritz value)
  double theta[kMaxM];
  double rnorm[kMaxM];
  // logical trial basis column -> source: kind (0 X, 1 R, 2 P, 3 Z) and column
  int src_kind[kMaxN];
  int src_col[kMaxN];
  int keep_col[kMaxN];   // logical columns kept after dropping (Np entries)
};

// Base of the launch's dynamic LDS.  The device bodies take their LDS
// pointer from here rather than from a parameter: a pointer that passed
// through a struct in memory loses its address space, and every access
// through it becomes a flat access.
__device__ inline double* lds_base() {
  extern __shared__ double psdp_dyn_lds[];
  return psdp_dyn_lds;
}

// Bit-cast helpers for BF16 (round to nearest even from float).
__host__ __device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) {           // inf / nan
    uint16_t h = (uint16_t)(u >> 16);
    if (u & 0x007fffffu) h |= 0x0040;                  // keep NaN quiet
    return h;
  }
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  uint32_t u = ((uint32_t)h) << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

__host__ __device__ inline int round_up(int x, int a) { return (x + a - 1) / a * a; }

// Counter-based Philox4x32-10 (Salmon et al., SC'11), used for the cold-start
// block and the expansion columns.  Normal deviates via Box-Muller.
struct Philox {
  __host__ __device__ static inline void round(uint32_t ctr[4], uint32_t key[2]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    uint64_t p0 = (uint64_t)M0 * ctr[0];
    uint64_t p1 = (uint64_t)M1 * ctr[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ ctr[1] ^ key[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ ctr[3] ^ key[1];
    uint32_t n3 = lo0;
    ctr[0] = n0; ctr[1] = n1; ctr[2] = n2; ctr[3] = n3;
  }
  __host__ __device__ static inline void gen(uint64_t counter, uint64_t seed, uint32_t out[4]) {
    uint32_t ctr[4] = {(uint32_t)counter, (uint32_t)(counter >> 32), 0x1912u, 0x2767u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int r = 0; r < 10; ++r) {
      round(ctr, key);
      key[0] += 0x9E3779B9u;
      key[1] += 0xBB67AE85u;
    }
    out[0] = ctr[0]; out[1] = ctr[1]; out[2] = ctr[2]; out[3] = ctr[3];
  }
};

// Logical column list: either a device array of column pointers, or the
// concatenation of up to four column-major segments sharing a leading dim.
struct ColMap {
  const double* const* ptrs;
  const double* base[4];
  int len[4];
  int ld;
  __device__ inline const double* col(int j) const {
    if (ptrs) return ptrs[j];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (j < len[s]) return base[s] + (size_t)j * ld;
      j -= len[s];
    }
    return base[0];
  }
};

inline ColMap colmap_ptrs(const double* const* p) {
  ColMap c{};
  c.ptrs = p;
  return c;
}
inline ColMap colmap_seg(const double* b0, int l0, int ld, const double* b1 = nullptr, int l1 = 0,
                         const double* b2 = nullptr, int l2 = 0) {
  ColMap c{};
  c.ptrs = nullptr;
  c.base[0] = b0; c.len[0] = l0;
  c.base[1] = b1; c.len[1] = l1;
  c.base[2] = b2; c.len[2] = l2;
  c.base[3] = nullptr; c.len[3] = 0;
  c.ld = ld;
  return c;
}

// Arguments of the one-workgroup kernels (k_small.hip).
struct DecideArgs {
  const double* G;      // Ng x Ng Gram of the candidate columns, leading dim ldg
  int ldg;
  int Ng;               // candidate columns (host bound; mode -1 reads st->Np)
  int mode;             // IterMode; -1 = second Cholesky-QR pass (no decisions)
  int m;                // block size
  int nz;               // expansion columns (mode XZ)
  int has_p;
  int phase_lowprec;    // product precision of the phase: 0 FP64, 1 FP32, 2 BF16
  int spec_m;           // > 0: queued before the previous iteration was read back,
                        // assuming it kept running with block size spec_m
  double tau;           // dropping threshold on the scaled pivot
  const double* bases[5];  // X, R, P, Z, S1 column bases
  int ld;               // leading dim of the bases
  double* T;            // out: N x Np (ldt)
  int ldt;
  const double** colptr;  // out: N column pointers of the logical trial basis
  int trace;            // 1: per-panel clock totals into st->t_sub
  State* st;
};

struct RRArgs {
  const double* K;   // Np x Np projected matrix S^T A S, leading dim ldk
  int ldk;
  int mtarget;       // Ritz pairs to keep
  double* C;         // out: Np x mk coefficients (eigenvectors), ldc
  int ldc;
  double* log;       // rotation log (c, s) per pair per round
  size_t log_cap;    // doubles available
  int max_sweeps;
  int count_iter;    // 1: this RR is a LOBPCG iteration (increments st->iter)
  double off_tol;    // Jacobi stops when off(H) <= off_tol * ||H||_F
  size_t lds_cap;    // dynamic LDS doubles of the launch (set by launch_rr)
  double* scratch;   // global scratch, >= 5 * Np * mk doubles (tridiagonal path)
  int trace;         // 1: per-step clock totals into st->t_sub
  State* st;
};

struct RRShared {
  double* lo;
  double* hi;
  int* npos;
  double* tnorm;
  double* pivmin;
};
struct CholShared {
  int* list;
  int* kind;
  int* col;
  int* keep;
  int* N;
  int* Np;
  int* nx;
  int* stop;
  double* red;  // blockDim.x / 64 + 128 doubles: reduction slots, then the
                // block's Ritz values and residual norms (64 each)
};
hipError_t launch_decide_chol(const DecideArgs& a, int N_host, hipStream_t st);
hipError_t launch_rr(const RRArgs& a, int Np_host, int mk_host, hipStream_t st);
hipError_t launch_rr_tri(const RRArgs& a, int Np_host, int mk_host, hipStream_t st);
hipError_t launch_rr_fast(const RRArgs& a, int Np_host, int mk_host, hipStream_t st);
// back-transformation of the Ritz vectors left by launch_rr_fast (C in place)
hipError_t launch_rr_back(const RRArgs& a, int Np_host, int mk_host, hipStream_t st);
hipError_t rr_tri_init();
hipError_t small_kernels_init();

// ------------------------------------------------------------------ launch
// Host-side launch helpers (defined in the kernel files).
// Optional epilogue of a block product: Y = ca (A S) + cb B1 + cc B0 (B0 may
// be null), B1 and B0 n x cols with leading dim ld, neither aliasing Y.
struct ProductComb {
  const double* b1;
  const double* b0;
  int ld;
  double ca, cb, cc;
};

struct ProductArgs {
  const void* A;     // FP64 / FP32 / BF16 matrix, column-major, leading dim lda
  int lda;
  int n;             // order
  int prec;          // 0 fp64, 1 fp32, 2 bf16
  const double* S;   // n x cols, leading dim lds
  int lds;
  double* Y;         // n x cols, leading dim ldy
  int ldy;
  const int* cols_dev;  // device pointer to the column count (or nullptr)
  int cols_max;         // grid bound on columns
  void* scratch;        // low-precision copy of S (bf16/fp32), size lds*cols_max*4 bytes
  void* partial;        // split-K partial sums (FP64 for FP64 products, else FP32)
  size_t partial_bytes;
  int max_slices;       // split-K slices the partial buffer holds
  const int* stop;      // device stop flag: the launch is a no-op when set
  ProductComb comb;     // b1 == nullptr: plain product
};

hipError_t launch_ingest(const double* X, int ldx, int n, double sign, double* A64, int lda,
                         int cols_alloc, void* Alp, int prec, double* fro_partial, int* nonfinite,
                         hipStream_t st, int* nblocks_out);
hipError_t launch_reduce_sum(const double* partial, int count, double* out, hipStream_t st);
hipError_t launch_product(const ProductArgs& a, hipStream_t st);
hipError_t launch_axpby3(int n, int cols, double ca, const double* Y, int ldy, double cb,
                         const double* B1, int ld1, double cc, const double* B0, int ld0,
                         double* out, int ldo, hipStream_t st);
hipError_t launch_lanczos_vec(int n, int step, int last, double* w, const double* v,
                              const double* vprev, double* coef, double* out, hipStream_t st);
hipError_t launch_fill_normal(double* B, int ld, int n, int col0, int cols, uint64_t seed,
                              uint64_t stream_id, hipStream_t st);
hipError_t launch_copy_cols(const double* src, int lds, double* dst, int ldd, int n, int cols,
                            hipStream_t st);
// st->stop = v (one thread)
hipError_t launch_set_stop(State* st, int v, hipStream_t s);
// *p = v (one thread)
hipError_t launch_set_int(int* p, int v, hipStream_t s);

}  // namespace psdp
