// Certificate of the tail term of the a-posteriori bound (paper §5.2,
// Thm `bound`, second term ||Pi(Vt_perp^T A Vt_perp)||_F).
//
// With P = I - Vt Vt^T (Vt: the m~ positive Ritz vectors, orthonormal) the
// matrix
//     M = s I - P A P + c Vt Vt^T
// is block diagonal in the basis [Vt, Vt_perp]: (s + c) I on range(Vt) and
// s I - Vt_perp^T A Vt_perp on its complement.  An FP64 Cholesky
// factorization of M that runs to completion with positive pivots therefore
// proves, once the rounding of forming and factoring M is bounded by eta and
// s = delta - eta, that every eigenvalue of Vt_perp^T A Vt_perp is below
// delta, so the tail term is at most sqrt(n - m~) * delta.
//
// Layout: M is L x L FP64 column-major (L = n rounded up to 64), rows and
// columns n..L-1 hold the identity, so the factorization runs on 64 x 64
// tiles with no bounds checks.
#pragma once

#include <hip/hip_runtime.h>

namespace psdp {

constexpr int kCertTile = 64;

struct CertState {
  // inputs, written by the host before the launches
  double delta;  // requested threshold (> 0)
  double c;      // eigenvalue given to range(Vt) (> 0)
  double fro_a;  // ||A||_F
  int n, L, mt;  // order, padded order, columns of Vt
  int pad0;
  // outputs
  double trace;   // tr(M0), M0 = -P A P + c Vt Vt^T over the first n rows
  double ufro2;   // ||U||_F^2, U = W - Vt H / 2 + c Vt / 2
  double wfro2;   // ||W||_F^2, W = A Vt (FP64 product)
  double vfro2;   // tr(Vt^T Vt) as computed
  double phi;     // ||Vt^T Vt - I||_F as computed
  double eta;     // bound on the rounding of forming and factoring M
  double delta_eff;  // max(delta, 4 eta): the threshold actually certified
  double shift;   // delta_eff - eta, added to the diagonal of M0
  int fail;       // 0: every pivot so far positive; 1 + p: a pivot of diagonal
                  // tile p was not positive and finite; -2: tr(M) < 0
  int pad1;
  long long t_diag[4];  // device clock (100 MHz) in the first diagonal tile's
                        // factorization: start, loaded, factored, stored
};

// U = W - Vt H / 2 + (c / 2) Vt (rows < n; zero below), per-workgroup
// partial sums of ||U||^2 and ||W||^2 into part[2 * blk + {0, 1}].
hipError_t launch_cert_prep(const double* V, const double* W, int ld, const double* H, int ldh,
                            int mt, int n, int L, double c, double* U, double* part,
                            hipStream_t st);
// M0 = -A + Vt U^T + U Vt^T on the lower 64 x 64 tiles of the L x L matrix
// (identity on the padding); diagonal sums of each diagonal tile into
// diag_part[tile].
hipError_t launch_cert_form(const double* A, int lda, const double* V, const double* U, int ld,
                            int mt, int n, int L, double* M, double* diag_part, hipStream_t st);
// Sums the partials, computes eta and delta_eff from G = Vt^T Vt (ldg),
// adds the shift to the diagonal of M.
hipError_t launch_cert_shift(const double* G, int ldg, const double* prep_part, int nprep,
                             const double* diag_part, double* M, CertState* cs, hipStream_t st);
// Blocked right-looking Cholesky of M (L x L, lower) on 64 x 64 tiles; a
// non-positive pivot sets cs->fail and the remaining launches return at once.
hipError_t launch_cert_chol(double* M, int L, CertState* cs, hipStream_t st);

}  // namespace psdp
