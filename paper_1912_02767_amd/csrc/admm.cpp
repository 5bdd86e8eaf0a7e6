// psdp_admm_solve: approximate ADMM (paper §2, Alg. 1) for standard-form
// SDPs with the PSD projections of the library (paper §6: LOBPCG on the
// side chosen from the previous iterate's inertia, warm-started from its
// Ritz block, stopped at residual tol_scale / k^tol_power), or exact ones.
// Termination by the primal and dual residuals of (P); infeasibility by the
// successive-difference certificates of §6.2.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <unordered_set>
#include <vector>

#include "../../include/psdp.h"
#include "admm.h"
#include "common.h"
#include "internal.h"

using namespace psdp;

namespace {

#define ADMM_TRY(expr)                         \
  do {                                         \
    if ((expr) != hipSuccess) {                \
      rc = PSDP_ERR_HIP;                       \
      goto done;                               \
    }                                          \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

psdp_status validate(const psdp_sdp* pr, std::vector<int>& off, std::vector<double>& sq) {
  if (!pr || pr->n < 1 || pr->p < 0 || pr->nnz < pr->p || !pr->C || pr->ldc < pr->n)
    return PSDP_ERR_INVALID_ARG;
  if (pr->p > 0 && (!pr->con || !pr->row || !pr->col || !pr->val || !pr->b))
    return PSDP_ERR_INVALID_ARG;
  const int n = pr->n, p = pr->p;
  off.assign(p + 1, 0);
  sq.assign(p, 0.0);
  std::unordered_set<long long> seen;
  seen.reserve((size_t)pr->nnz * 2 + 1);
  int prev = 0;
  for (int e = 0; e < pr->nnz; ++e) {
    const int c = pr->con[e], r = pr->row[e], k = pr->col[e];
    const double v = pr->val[e];
    if (c < prev || c >= p || k < 0 || r < k || r >= n || !std::isfinite(v) || v == 0.0)
      return PSDP_ERR_INVALID_ARG;
    if (!seen.insert((long long)r * n + k).second) return PSDP_ERR_INVALID_ARG;  // supports overlap
    prev = c;
    off[c + 1] += 1;
    sq[c] += (r == k ? 1.0 : 2.0) * v * v;
  }
  for (int i = 0; i < p; ++i) {
    if (off[i + 1] == 0 || !std::isfinite(pr->b[i])) return PSDP_ERR_INVALID_ARG;
    off[i + 1] += off[i];
  }
  return PSDP_OK;
}

}  // namespace

extern "C" void psdp_admm_default_options(psdp_admm_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->rho = 0.1;
  o->sigma = 1e-6;
  o->alpha = 1.6;
  o->max_iter = 2500;
  o->check_every = 40;
  o->eps_abs = 1e-5;
  o->eps_rel = 1e-5;
  o->eps_inf = 1e-5;
  o->exact = 0;
  o->tol_scale = 10.0;
  o->tol_power = 1.01;
  o->prec = PSDP_PREC_FP64;
  o->m_cap = 48;
  o->method = PSDP_METHOD_LOBPCG;
}

extern "C" psdp_status psdp_admm_solve(psdp_handle h, const psdp_sdp* pr,
                                       const psdp_admm_options* opt_in, double* Y, int ldy,
                                       double* y, double* W, int ldw, psdp_admm_info* info) {
  psdp_admm_options opt;
  if (opt_in) opt = *opt_in; else psdp_admm_default_options(&opt);
  psdp_admm_info dummy;
  if (!info) info = &dummy;
  std::memset(info, 0, sizeof(*info));
  info->status = PSDP_ADMM_MAX_ITER;
  std::vector<int> off;
  std::vector<double> sq;
  if (!h || !Y || ldy < (pr ? pr->n : 1) || !W || ldw < (pr ? pr->n : 1))
    return PSDP_ERR_INVALID_ARG;
  psdp_status rc = validate(pr, off, sq);
  if (rc != PSDP_OK) return rc;
  if (pr->p > 0 && !y) return PSDP_ERR_INVALID_ARG;
  if (!(opt.rho > 0.0) || !(opt.sigma > 0.0) || !(opt.alpha > 0.0) || !(opt.alpha < 2.0) ||
      opt.max_iter < 1 || opt.check_every < 1 || !(opt.eps_abs >= 0.0) || !(opt.eps_rel >= 0.0) ||
      !(opt.eps_inf > 0.0) || !(opt.tol_scale > 0.0) || !(opt.tol_power >= 0.0) || opt.prec < 0 ||
      opt.prec > 2 || opt.m_cap < 1 ||
      (opt.method != PSDP_METHOD_LOBPCG && opt.method != PSDP_METHOD_CHEBYSHEV))
    return PSDP_ERR_INVALID_ARG;

  const int n = pr->n, p = pr->p, nnz = pr->nnz;
  const size_t nn = (size_t)n * n;
  const int dev = handle_device(h);
  if (hipSetDevice(dev) != hipSuccess) return PSDP_ERR_HIP;
  hipStream_t s = handle_stream(h);
  const int mcap = std::min(opt.m_cap, n);
  const int nblk = (int)std::min<size_t>(1024, (nn + 255) / 256);
  const AdmmParams prm{opt.rho, opt.sigma, opt.alpha};

  // one device block for every buffer of the solve
  size_t sz = 0;
  auto take = [&](size_t b) { size_t o = sz; sz = align_up(sz + b, 256); return o; };
  const size_t oC = take(8 * nn), oY = take(8 * nn), oZ = take(8 * nn), oW = take(8 * nn),
               oR = take(8 * nn), oV = take(8 * nn), oYp = take(8 * nn), oWp = take(8 * nn),
               oAv = take(8 * nn), oMap = take(4 * nn), oCon = take(4 * (size_t)nnz + 4),
               oRow = take(4 * (size_t)nnz + 4), oCol = take(4 * (size_t)nnz + 4),
               oVal = take(8 * (size_t)nnz + 8), oOff = take(4 * (size_t)(p + 1)),
               oS = take(8 * (size_t)p + 8), oB = take(8 * (size_t)p + 8), oy = take(8 * (size_t)p + 8),
               oyp = take(8 * (size_t)p + 8), oCoef = take(8 * (size_t)p + 8),
               oT = take(8 * (size_t)p + 8), oPart = take(8 * (size_t)nblk * kNorms),
               oVb = take(8 * (size_t)n * mcap), oLam = take(8 * (size_t)mcap + 8);
  char* base = nullptr;
  if (hipMalloc(&base, sz) != hipSuccess) return PSDP_ERR_OUT_OF_MEMORY;
  double *Cs = (double*)(base + oC), *Yb = (double*)(base + oY), *Z = (double*)(base + oZ),
         *Wb = (double*)(base + oW), *R = (double*)(base + oR), *V = (double*)(base + oV),
         *Yp = (double*)(base + oYp), *Wp = (double*)(base + oWp), *aval = (double*)(base + oAv),
         *s_d = (double*)(base + oS), *b_d = (double*)(base + oB), *y_d = (double*)(base + oy),
         *yp_d = (double*)(base + oyp), *coef = (double*)(base + oCoef), *t_d = (double*)(base + oT),
         *part = (double*)(base + oPart), *Vblk = (double*)(base + oVb), *lam = (double*)(base + oLam);
  int *con_of = (int*)(base + oMap), *con_d = (int*)(base + oCon), *row_d = (int*)(base + oRow),
      *col_d = (int*)(base + oCol), *off_d = (int*)(base + oOff);
  double* val_d = (double*)(base + oVal);
  AdmmConstraints cs{p, nnz, con_d, row_d, col_d, val_d, off_d, s_d, b_d};
  std::vector<double> hpart((size_t)nblk * kNorms), ht(p > 0 ? p : 1), hy(p > 0 ? p : 1),
      hyp(p > 0 ? p : 1);
  double b2 = 0.0;
  for (int i = 0; i < p; ++i) b2 += pr->b[i] * pr->b[i];
  const double t0 = now_ms();
  double proj_ms = 0.0;
  int pos_hint = -1, warm_side = PSDP_SIDE_AUTO, m_io = 0;
  double c2 = -1.0;

  // sums over the positions: partials on the device, the last step on the host
  auto norms = [&](const double* Ym, const double* Zm, const double* Wm, const double* ym,
                   double out[kNorms]) -> hipError_t {
    hipError_t e = launch_admm_norms(n, Ym, Zm, Cs, Wm, con_of, aval, ym, part, nblk, s);
    if (e != hipSuccess) return e;
    e = copy_to_host(hpart.data(), part, 8 * (size_t)nblk * kNorms, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (int q = 0; q < kNorms; ++q) out[q] = 0.0;
    for (int bk = 0; bk < nblk; ++bk)
      for (int q = 0; q < kNorms; ++q) out[q] += hpart[(size_t)bk * kNorms + q];
    return hipSuccess;
  };
  // <A_i, M> for every constraint, on the host
  auto cdots = [&](const double* M) -> hipError_t {
    if (p == 0) return hipSuccess;
    hipError_t e = launch_admm_cdot(cs, M, n, kDotStore, prm, t_d, nullptr, s);
    if (e != hipSuccess) return e;
    e = copy_to_host(ht.data(), t_d, 8 * (size_t)p, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
  };
  // exact projection of M (the exact path of the library) into the buffer P
  auto exact_proj = [&](const double* M, double* P) -> psdp_status {
    const double ta = now_ms();
    psdp_status r = psdp_full_eig_project(h, n, M, n, nullptr, P, n);
    proj_ms += now_ms() - ta;
    return r;
  };

  ADMM_TRY(hipMemcpyAsync(con_d, pr->con, 4 * (size_t)nnz, hipMemcpyHostToDevice, s));
  ADMM_TRY(hipMemcpyAsync(row_d, pr->row, 4 * (size_t)nnz, hipMemcpyHostToDevice, s));
  ADMM_TRY(hipMemcpyAsync(col_d, pr->col, 4 * (size_t)nnz, hipMemcpyHostToDevice, s));
  ADMM_TRY(hipMemcpyAsync(val_d, pr->val, 8 * (size_t)nnz, hipMemcpyHostToDevice, s));
  ADMM_TRY(hipMemcpyAsync(off_d, off.data(), 4 * (size_t)(p + 1), hipMemcpyHostToDevice, s));
  ADMM_TRY(hipMemcpyAsync(s_d, sq.data(), 8 * (size_t)p, hipMemcpyHostToDevice, s));
  ADMM_TRY(hipMemcpyAsync(b_d, pr->b, 8 * (size_t)p, hipMemcpyHostToDevice, s));
  ADMM_TRY(hipMemsetAsync(y_d, 0, 8 * (size_t)p + 8, s));
  ADMM_TRY(hipMemsetAsync(Yb, 0, 8 * nn, s));
  ADMM_TRY(hipMemsetAsync(Z, 0, 8 * nn, s));   // z^0 = Pi_C(A x^0) = (b, 0) for x^0 = 0
  ADMM_TRY(hipMemsetAsync(Wb, 0, 8 * nn, s));
  ADMM_TRY(launch_admm_sym(pr->C, pr->ldc, n, Cs, s));
  ADMM_TRY(launch_admm_map(cs, n, con_of, aval, s));

  {
    int k = 1;
    for (; k <= opt.max_iter; ++k) {
      const bool check = (k % opt.check_every == 0) || k == opt.max_iter;
      if (check) {
        ADMM_TRY(hipMemcpyAsync(Yp, Yb, 8 * nn, hipMemcpyDeviceToDevice, s));
        ADMM_TRY(hipMemcpyAsync(Wp, Wb, 8 * nn, hipMemcpyDeviceToDevice, s));
        if (p) ADMM_TRY(hipMemcpyAsync(yp_d, y_d, 8 * (size_t)p, hipMemcpyDeviceToDevice, s));
      }
      // Alg. 1, first line: the linear system, solved in closed form
      ADMM_TRY(launch_admm_rhs(n, prm, Yb, Cs, Z, Wb, con_of, aval, b_d, y_d, R, s));
      ADMM_TRY(launch_admm_cdot(cs, R, n, kDotSolve, prm, coef, y_d, s));
      // second and third lines: relaxation and the point to project
      ADMM_TRY(launch_admm_xt(n, prm, R, con_of, aval, coef, Z, Wb, V, Yb, s));
      // projection onto S_+ (the {b} part of C is b itself)
      if (opt.exact) {
        if ((rc = exact_proj(V, Z)) != PSDP_OK) goto done;
        info->proj_full += 1;
      } else {
        psdp_options po;
        psdp_default_options(&po);
        po.side = PSDP_SIDE_AUTO;
        po.prec = opt.prec;
        po.tol = opt.tol_scale / std::pow((double)k, opt.tol_power);
        po.pos_hint = pos_hint;
        po.warm_side = warm_side;
        po.fallback_full = 1;
        po.method = opt.method;
        psdp_info pi;
        const double ta = now_ms();
        psdp_status r = psdp_project(h, n, V, n, Vblk, n, mcap, &m_io, lam, Z, n, &po, &pi);
        proj_ms += now_ms() - ta;
        if (r < 0) { rc = r; goto done; }
        if (pi.side_used == PSDP_SIDE_FULL) {
          info->proj_full += 1;
          if (pi.iters > 0) info->proj_not_certified += 1;
        } else {
          info->proj_block += 1;
        }
        pos_hint = pi.pos_est;
        warm_side = pi.block_side;
      }
      // fourth line: the multiplier of the PSD block
      ADMM_TRY(launch_admm_dual(n, opt.rho, V, Z, Wb, s));
      if (!check) continue;

      // ---- termination: primal and dual residuals of (P)
      double nm[kNorms];
      ADMM_TRY(norms(Yb, Z, Wb, y_d, nm));
      if (c2 < 0.0) c2 = nm[6];
      ADMM_TRY(cdots(Yb));
      double ax2 = 0.0, res_eq2 = 0.0;
      for (int i = 0; i < p; ++i) {
        ax2 += ht[i] * ht[i];
        res_eq2 += (ht[i] - pr->b[i]) * (ht[i] - pr->b[i]);
      }
      const double r_prim = std::sqrt(res_eq2 + nm[0]);
      const double r_dual = std::sqrt(nm[3]);
      info->r_prim = r_prim;
      info->r_dual = r_dual;
      info->obj = nm[5];
      info->iters = k;
      const double nAx = std::sqrt(ax2 + nm[1]), nz = std::sqrt(b2 + nm[2]);
      const double nq = std::sqrt(c2), nAty = std::sqrt(nm[4]);
      if (!std::isfinite(r_prim) || !std::isfinite(r_dual)) { rc = PSDP_ERR_NUMERICAL; goto done; }
      if (r_prim <= opt.eps_abs + opt.eps_rel * std::max(nAx, nz) &&
          r_dual <= opt.eps_abs + opt.eps_rel * std::max(nq, nAty)) {
        info->status = PSDP_ADMM_SOLVED;
        break;
      }
      // ---- infeasibility (§6.2): successive differences dx, dy
      ADMM_TRY(launch_admm_diff(nn, Yb, Yp, R, s));          // dY
      ADMM_TRY(launch_admm_diff(nn, Wb, Wp, V, s));          // dW
      if (p) ADMM_TRY(launch_admm_diff((size_t)p, y_d, yp_d, yp_d, s));  // dy (into yp)
      double dn[kNorms];
      ADMM_TRY(norms(R, R, V, yp_d, dn));  // 1: ||dY||^2, 5: <C, dY>, 4: ||A^* dy + dW||^2, 7: ||dW||^2
      ADMM_TRY(cdots(R));                  // A_eq dY
      double aeq2 = 0.0;
      for (int i = 0; i < p; ++i) aeq2 += ht[i] * ht[i];
      if (p) {
        ADMM_TRY(copy_to_host(hy.data(), yp_d, 8 * (size_t)p, s));
        ADMM_TRY(hipStreamSynchronize(s));
      }
      double dy2 = 0.0, bdy = 0.0;
      for (int i = 0; i < p; ++i) {
        dy2 += hy[i] * hy[i];
        bdy += pr->b[i] * hy[i];
      }
      const double ndx = std::sqrt(dn[1]), ndy = std::sqrt(dy2 + dn[7]), e = opt.eps_inf;
      if (ndx > 0.0 && std::sqrt(aeq2) <= e * ndx && dn[5] <= -e * ndx) {
        // dual infeasibility: dY / ||dY|| also in the recession cone S_+
        if ((rc = exact_proj(R, Yp)) != PSDP_OK) goto done;
        double pn[kNorms];
        ADMM_TRY(norms(R, Yp, V, yp_d, pn));
        if (std::sqrt(pn[0]) <= e * ndx) {
          info->status = PSDP_ADMM_DUAL_INFEASIBLE;
          break;
        }
      }
      if (ndy > 0.0 && std::sqrt(dn[4]) <= e * ndy && bdy <= -e * ndy) {
        // primal infeasibility: the PSD part of dy / ||dy|| negative semidefinite
        if ((rc = exact_proj(V, Wp)) != PSDP_OK) goto done;
        double pn[kNorms];
        ADMM_TRY(norms(V, Wp, V, yp_d, pn));
        if (std::sqrt(pn[2]) <= e * ndy) {
          info->status = PSDP_ADMM_PRIMAL_INFEASIBLE;
          break;
        }
      }
    }
    if (k > opt.max_iter) info->iters = opt.max_iter;
  }
  // ---- outputs
  ADMM_TRY(launch_copy_cols(Yb, n, Y, ldy, n, n, s));
  ADMM_TRY(launch_copy_cols(Wb, n, W, ldw, n, n, s));
  if (p) ADMM_TRY(hipMemcpyAsync(y, y_d, 8 * (size_t)p, hipMemcpyDeviceToDevice, s));
  ADMM_TRY(hipStreamSynchronize(s));
  rc = PSDP_OK;
done:
  (void)hipStreamSynchronize(s);
  hipFree(base);
  info->proj_ms = proj_ms;
  info->total_ms = now_ms() - t0;
  return rc;
}
