// Internal declarations of the ADMM loop for standard-form SDPs (paper §2,
// Alg. 1): device views of the constraint data and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

namespace psdp {

// Constraint data on the device: entries sorted by constraint, off[i] ..
// off[i+1] the entries of constraint i, s[i] = ||A_i||_F^2.
struct AdmmConstraints {
  int p, nnz;
  const int* con;
  const int* row;
  const int* col;
  const double* val;
  const int* off;
  const double* s;
  const double* b;
};

struct AdmmParams {
  double rho, sigma, alpha;
};

enum AdmmDotMode : int { kDotStore = 0, kDotNorm = 1, kDotSolve = 2 };
constexpr int kNorms = 8;

hipError_t launch_admm_sym(const double* C, int ldc, int n, double* Cs, hipStream_t st);
hipError_t launch_admm_map(const AdmmConstraints& c, int n, int* con_of, double* aval,
                           hipStream_t st);
hipError_t launch_admm_cdot(const AdmmConstraints& c, const double* M, int n, int mode,
                            const AdmmParams& prm, double* out, double* y, hipStream_t st);
hipError_t launch_admm_rhs(int n, const AdmmParams& prm, const double* Y, const double* C,
                           const double* Z, const double* W, const int* con_of, const double* aval,
                           const double* b, const double* y, double* R, hipStream_t st);
hipError_t launch_admm_xt(int n, const AdmmParams& prm, const double* R, const int* con_of,
                          const double* aval, const double* coef, const double* Z, const double* W,
                          double* V, double* Y, hipStream_t st);
hipError_t launch_admm_dual(int n, double rho, const double* V, const double* Z, double* W,
                            hipStream_t st);
hipError_t launch_admm_diff(size_t total, const double* P, const double* Q, double* D,
                            hipStream_t st);
hipError_t launch_admm_norms(int n, const double* Y, const double* Z, const double* C,
                             const double* W, const int* con_of, const double* aval,
                             const double* y, double* part, int nblk, hipStream_t st);

}  // namespace psdp
