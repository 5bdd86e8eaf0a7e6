// Host driver of the single-cone projection and the C-ABI entry points.
//
// One psdp_project call (paper §5.1, Alg. 3 with the §6 side rule and the
// §5.2 bound):
//   ingest      A = s * sym(X) (s = +1 positive side, -1 negative side), in
//               FP64 and in the product precision
//   start       warm-start block V (or seeded N(0,1) columns), Rayleigh-Ritz
//               on its span with an FP64 product (Alg. 3, initial RR)
//   iterate     trial basis [X, R, P] -> two Cholesky-QR passes -> A S ->
//               S^T A S -> Jacobi -> X, AX, P, R   (Alg. 3 loop)
//   expand      when more positive Ritz values than columns: append seeded
//               random columns (paper §5.1 expansion rule)
//   ladder      low-precision products until the residual stalls, then
//               higher precision; an FP64 refresh + sweep at the end
//   bound       err^2 = 2 ||R||_F^2 + tail^2 (Thm `bound`), tail estimated
//   rebuild     Pi = V diag(l) V^T (+ X on the negative side, Moreau)
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "../../include/psdp.h"
#include "batched.h"
#include "cert.h"
#include "common.h"
#include "internal.h"

namespace psdp {
// launchers defined in the kernel files
hipError_t launch_gram_partial(const ColMap& bptr, const ColMap* yptr, const int* nb_dev,
                               int nb_host, const int* ny_dev, int ny_host, int n, double* part,
                               int ldp, size_t part_stride, int* nblk_out, const int* stop,
                               hipStream_t st);
hipError_t launch_reduce_partials(const double* part, int nblk, size_t part_stride, int ldp,
                                  const int* rows_dev, int rows_host, const int* cols_dev,
                                  int cols_host, double* out, int ldo, const int* stop,
                                  hipStream_t st);
hipError_t launch_tsmm(const ColMap& src, const int* kk_dev, int kk_host, const int* q_dev,
                       int q_host, const double* M, int ldm, int n, double* Y, int ldy,
                       const int* stop, hipStream_t st);
hipError_t launch_update(const double* S, const double* AS, int lds, const double* C, int ldc,
                         const State* stt, int want_p, int n, int mk_host, double* Xo,
                         double* AXo, double* Po, double* Ro, int ldo, hipStream_t st);
hipError_t launch_rebuild(const double* V, int ldv, const double* lt, int mt, int n,
                          const double* base, int ldb, double base_sign, double* Pi, int ldpi,
                          hipStream_t st);
// batched engine (batched_host.cpp)
struct BatchEngine;
BatchEngine* batch_engine_new(int device);
void batch_engine_free(BatchEngine* e);
double batch_engine_last_ms(const BatchEngine* e);
int batch_engine_last_variant(const BatchEngine* e);
psdp_status batch_engine_run(BatchEngine* e, hipStream_t s, int count, const int* n,
                             const double* const* X, double* const* V, const int* m_cap,
                             int* m_inout, double* const* lambda, double* const* Pi,
                             const psdp_options& opt, psdp_info* info);
}  // namespace psdp

using namespace psdp;

namespace {

constexpr int kMaxSweeps = 40;
constexpr int kProductSlices = 16;

struct ProfEntry {
  long launches = 0;
  double ms = 0.0, bytes = 0.0, flops = 0.0;
};

struct PendingEvent {
  std::string family;
  hipEvent_t a, b;
  double bytes, flops;
  int prec = -1;  // block products: 0 FP64, 1 FP32, 2 BF16 (also tallied per precision)
};

struct Workspace {
  int L = 0, MC = 0, NC = 0, prec = -1, nblk = 0;
  size_t bytes = 0;
  char* base = nullptr;
  double *A64 = nullptr;
  void* Alp = nullptr;
  double *X = nullptr, *R = nullptr, *P = nullptr, *AX = nullptr, *Z = nullptr;
  double *S1 = nullptr, *S2 = nullptr, *AS = nullptr;
  double *Gpart = nullptr, *G = nullptr, *T = nullptr, *C = nullptr, *rrs = nullptr;
  void* ppart = nullptr;  // split-K partial products
  size_t ppart_bytes = 0;
  double* log = nullptr;
  size_t log_cap = 0;
  const double** colptr = nullptr;
  double* fro_part = nullptr;
  int fro_nblk = 0;
  double* scal = nullptr;  // [0] fro2
  int* nonfinite = nullptr;
  State* st = nullptr;
  double* lz = nullptr;  // Lanczos bound: three vectors (ld L), coefficients, result,
                         // then the split-K partials of its one-column products
};

}  // namespace

struct psdp_handle_s {
  int device = 0;
  hipStream_t stream = nullptr;
  Workspace ws;
  State* h_state = nullptr;  // pinned mirror
  rocblas_handle rb = nullptr;
  double* eig_d = nullptr;  // full-eig scratch
  double* eig_e = nullptr;
  rocblas_int* eig_info = nullptr;
  double* eig_A = nullptr;
  int eig_cap = 0;
  double* h_pin = nullptr;  // pinned scratch for small readbacks
  size_t h_pin_cap = 0;
  unsigned long long calls = 0;
  int rr_method = 0;  // 0: column-parallel tridiagonal + twisted vectors + WY back-transform,
                      // 1: Jacobi, 2: first tridiagonal design (inverse iteration)
  int trace = 0;      // PSDP_TRACE=1: one line per iteration on stderr (2: RR stages)
  bool prof = false;
  std::set<std::string> prof_only;  // families timed while prof is on (empty: all)
  std::map<std::string, ProfEntry> prof_tab;
  std::vector<PendingEvent> pending;
  std::vector<hipEvent_t> event_pool;
  hipEvent_t sync_ev = nullptr;  // polled by spin_wait
  // second stream (default priority, non-blocking) for the Lanczos bound of
  // the Chebyshev variant, which runs beside the first Rayleigh-Ritz step;
  // its pinned result slot
  hipStream_t aux = nullptr;
  double* h_pin_aux = nullptr;
  State* h_snap = nullptr;         // two pinned state snapshots of queued iterations
  hipEvent_t snap_ev[2] = {nullptr, nullptr};
  psdp::BatchEngine* batch = nullptr;
  char* beig = nullptr;  // batched exact path scratch
  size_t beig_bytes = 0;
  // tail certificate: M (L x L FP64), partial sums, device state
  char* cert_base = nullptr;
  int cert_L = 0;
  double* cert_M = nullptr;
  double* cert_part = nullptr;
  psdp::CertState* cert_dev = nullptr;
  psdp::CertState* cert_host = nullptr;  // pinned
};

namespace {

#define HIP_TRY(expr)                                  \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) return PSDP_ERR_HIP;         \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Waits for the work queued on s by polling an event: the host sees the end
// of a short iteration within microseconds, where a blocking wait can sleep
// for tens of them before the next launches are queued.
hipError_t spin_wait(psdp_handle h, hipStream_t s) {
  if (!h->sync_ev && hipEventCreateWithFlags(&h->sync_ev, hipEventDisableTiming) != hipSuccess) {
    h->sync_ev = nullptr;
    return hipStreamSynchronize(s);
  }
  hipError_t e = hipEventRecord(h->sync_ev, s);
  if (e != hipSuccess) return e;
  while ((e = hipEventQuery(h->sync_ev)) == hipErrorNotReady) {
  }
  return e;
}

// Polls an already recorded event.
hipError_t spin_event(hipEvent_t ev) {
  hipError_t e;
  while ((e = hipEventQuery(ev)) == hipErrorNotReady) {
  }
  return e;
}

hipEvent_t get_event(psdp_handle h) {
  if (!h->event_pool.empty()) {
    hipEvent_t e = h->event_pool.back();
    h->event_pool.pop_back();
    return e;
  }
  // timing only: no system-scope fence (cache write-back and invalidation)
  // when the event is recorded, which would stall the following launches
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

struct ProfScope {
  psdp_handle h;
  const char* fam;
  hipEvent_t a = nullptr, b = nullptr;
  double bytes, flops;
  int prec;
  hipStream_t st;
  ProfScope(psdp_handle h_, const char* f, double by = 0, double fl = 0, int pr = -1,
            hipStream_t s_ = nullptr)
      : h(h_), fam(f), bytes(by), flops(fl), prec(pr), st(s_ ? s_ : h_->stream) {
    if (h->prof && (h->prof_only.empty() || h->prof_only.count(f))) {
      a = get_event(h);
      b = get_event(h);
      if (a) (void)hipEventRecord(a, st);
    }
  }
  ~ProfScope() {
    if (a && b) {
      (void)hipEventRecord(b, st);
      h->pending.push_back({fam, a, b, bytes, flops, prec});
    }
  }
};

void prof_collect(psdp_handle h) {
  if (h->pending.empty()) return;
  (void)hipStreamSynchronize(h->stream);
  if (h->aux) (void)hipStreamSynchronize(h->aux);
  for (auto& p : h->pending) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p.a, p.b);
    auto& e = h->prof_tab[p.family];
    e.launches += 1;
    e.ms += ms;
    e.bytes += p.bytes;
    e.flops += p.flops;
    if (p.prec >= 0 && p.prec <= 2) {
      static const char* const kPrecName[3] = {"product_fp64", "product_fp32", "product_bf16"};
      auto& q = h->prof_tab[kPrecName[p.prec]];
      q.launches += 1;
      q.ms += ms;
      q.bytes += p.bytes;
      q.flops += p.flops;
    }
    h->event_pool.push_back(p.a);
    h->event_pool.push_back(p.b);
  }
  h->pending.clear();
}

size_t product_elem_bytes(int prec) { return prec == 0 ? 8 : (prec == 1 ? 4 : 2); }

psdp_status ensure_workspace(psdp_handle h, int n, int mc, int prec) {
  Workspace& w = h->ws;
  int L = round_up(std::max(n, 1), 64);
  int MC = std::min(std::max(mc, 1), kMaxM);
  int NC = 3 * MC;
  (void)prec;  // the low-precision copy is sized for FP32, which also holds BF16
  if (w.base && L <= w.L && MC <= w.MC) return PSDP_OK;
  // grow
  L = std::max(L, w.L);
  MC = std::max(MC, w.MC);
  NC = 3 * MC;
  int wprec = 1;
  int nblk = (L + kGramRows - 1) / kGramRows;
  int T32 = (L + 31) / 32;
  int fro_nblk = T32 * (T32 + 1) / 2;
  size_t log_cap = (size_t)kMaxSweeps * (NC + 1) * (NC + 2);
  size_t sz = 0;
  auto take = [&](size_t b) {
    size_t off = sz;
    sz = align_up(sz + b, 256);
    return off;
  };
  size_t oA64 = take(sizeof(double) * (size_t)L * L);
  size_t oAlp = take((size_t)L * L * 4);
  size_t oX = take(sizeof(double) * (size_t)L * MC);
  size_t oR = take(sizeof(double) * (size_t)L * MC);
  size_t oP = take(sizeof(double) * (size_t)L * MC);
  size_t oAX = take(sizeof(double) * (size_t)L * MC);
  size_t oZ = take(sizeof(double) * (size_t)L * MC);
  size_t oS1 = take(sizeof(double) * (size_t)L * NC);
  size_t oS2 = take(sizeof(double) * (size_t)L * NC);
  size_t oAS = take(sizeof(double) * (size_t)L * NC);
  size_t oGp = take(sizeof(double) * (size_t)nblk * NC * NC);
  size_t oG = take(sizeof(double) * (size_t)NC * NC);
  size_t oT = take(sizeof(double) * (size_t)NC * NC);
  size_t oC = take(sizeof(double) * (size_t)NC * NC);
  size_t oRrs = take(sizeof(double) * 5 * (size_t)NC * MC);
  const size_t ppart_bytes = sizeof(double) * kProductSlices * (size_t)L * NC;
  size_t oPP = take(ppart_bytes);
  size_t oLog = take(sizeof(double) * log_cap);
  size_t oPtr = take(sizeof(double*) * (size_t)NC);
  size_t oFro = take(sizeof(double) * (size_t)fro_nblk);
  size_t oScal = take(sizeof(double) * 16);
  size_t oNf = take(sizeof(int) * 16);
  size_t oSt = take(sizeof(State));
  size_t oLz = take(sizeof(double) * ((3 + kProductSlices) * (size_t)L + 128));
  if (w.base) {
    (void)hipStreamSynchronize(h->stream);
    hipFree(w.base);
    w.base = nullptr;
  }
  char* base = nullptr;
  if (hipMalloc(&base, sz) != hipSuccess) {
    w = Workspace();
    return PSDP_ERR_OUT_OF_MEMORY;
  }
  w.base = base;
  w.bytes = sz;
  w.L = L; w.MC = MC; w.NC = NC; w.prec = wprec; w.nblk = nblk;
  w.A64 = (double*)(base + oA64);
  w.Alp = (void*)(base + oAlp);
  w.X = (double*)(base + oX);
  w.R = (double*)(base + oR);
  w.P = (double*)(base + oP);
  w.AX = (double*)(base + oAX);
  w.Z = (double*)(base + oZ);
  w.S1 = (double*)(base + oS1);
  w.S2 = (double*)(base + oS2);
  w.AS = (double*)(base + oAS);
  w.Gpart = (double*)(base + oGp);
  w.G = (double*)(base + oG);
  w.T = (double*)(base + oT);
  w.C = (double*)(base + oC);
  w.rrs = (double*)(base + oRrs);
  w.ppart = (void*)(base + oPP);
  w.ppart_bytes = ppart_bytes;
  w.log = (double*)(base + oLog);
  w.log_cap = log_cap;
  w.colptr = (const double**)(base + oPtr);
  w.fro_part = (double*)(base + oFro);
  w.fro_nblk = fro_nblk;
  w.scal = (double*)(base + oScal);
  w.nonfinite = (int*)(base + oNf);
  w.st = (State*)(base + oSt);
  w.lz = (double*)(base + oLz);
  // zero everything once so padded rows are zero
  HIP_TRY(hipMemsetAsync(base, 0, sz, h->stream));
  return PSDP_OK;
}

psdp_status ensure_pinned(psdp_handle h, size_t bytes) {
  if (h->h_pin_cap >= bytes) return PSDP_OK;
  if (h->h_pin) hipHostFree(h->h_pin);
  h->h_pin = nullptr;
  h->h_pin_cap = 0;
  if (hipHostMalloc((void**)&h->h_pin, bytes, hipHostMallocDefault) != hipSuccess)
    return PSDP_ERR_OUT_OF_MEMORY;
  h->h_pin_cap = bytes;
  return PSDP_OK;
}

// ---------------------------------------------------------------- solver --
struct Solver {
  psdp_handle h;
  Workspace& w;
  hipStream_t s;
  int n;
  int m;       // current block
  int mcap;    // capacity (<= kMaxM and the caller's m_cap)
  int has_p = 0;
  int iters = 0;
  int prec;    // product precision of the current phase
  State* hs;   // pinned host mirror
  Solver(psdp_handle h_, int n_, int mcap_)
      : h(h_), w(h_->ws), s(h_->stream), n(n_), m(0), mcap(mcap_), prec(0), hs(h_->h_state) {}

  const void* amat(int p) const { return p == 0 ? (const void*)w.A64 : w.Alp; }

  psdp_status read_state() {
    HIP_TRY(copy_to_host(hs, w.st, sizeof(State), s));
    HIP_TRY(spin_wait(h, s));
    return PSDP_OK;
  }

  // Algorithmic bytes / flops of this iteration's launches, attributed once
  // the device-side widths are known (after the state readback).
  void attribute(size_t first, size_t last, int Ng, int pprec) {
    if (!h->prof) return;
    const State& st = *hs;
    const double nn = n, N = st.N > 0 ? st.N : Ng, N1 = st.Np1, N2 = st.Np, mk = st.mk;
    int gram_i = 0, chol_i = 0, tsmm_i = 0;
    for (size_t i = first; i < last && i < h->pending.size(); ++i) {
      PendingEvent& p = h->pending[i];
      if (p.family == "gram") {
        double c = (gram_i == 0) ? Ng : (gram_i == 1 ? N1 : N2);
        p.bytes = (gram_i == 2 ? 16.0 : 8.0) * nn * c;
        p.flops = (gram_i == 2 ? 2.0 : 1.0) * nn * c * c;
        ++gram_i;
      } else if (p.family == "chol") {
        double c = (chol_i == 0) ? N : N1;
        p.flops = 2.0 * c * c * c / 3.0;  // Cholesky + triangular inverse
        p.bytes = 16.0 * c * c;
        ++chol_i;
      } else if (p.family == "rr") {
        if (h->rr_method == 0) {
          // tridiagonalization (4/3 N^3), eigenvalues and vectors of T
          p.flops = 4.0 / 3.0 * N2 * N2 * N2;
          p.bytes = 8.0 * N2 * N2 + 4.0 * N2 * N2 + 8.0 * N2 * mk;
        } else {
          p.flops = 9.0 * N2 * N2 * N2;  // dense symmetric eigendecomposition
          p.bytes = 8.0 * N2 * N2 + 8.0 * N2 * mk;
        }
      } else if (p.family == "rrback") {
        p.flops = 4.0 * N2 * N2 * mk;  // N - 2 reflectors applied to mk columns
        p.bytes = 4.0 * N2 * N2 + 16.0 * N2 * mk;
      } else if (p.family == "tsmm") {
        if (tsmm_i == 0) { p.flops = 2 * nn * N * N1; p.bytes = 8 * nn * (N + N1); }
        else if (tsmm_i == 1) { p.flops = 2 * nn * N1 * N2; p.bytes = 8 * nn * (N1 + N2); }
        else { p.flops = 6 * nn * N2 * mk; p.bytes = 8 * nn * (2 * N2 + 4 * mk); }
        ++tsmm_i;
      } else if (p.family == "product") {
        p.flops = 2.0 * nn * nn * N2;
        p.bytes = (double)product_elem_bytes(pprec) * nn * nn + 16.0 * nn * N2;
        p.prec = pprec;
      }
    }
  }

  // An iteration whose launches are queued and whose state snapshot is not
  // read yet.  spec_m > 0: queued before the previous iteration was read back,
  // assuming it kept running with block size spec_m; its decision kernel
  // turns it into no-ops otherwise.
  struct Queued {
    int mode = 0, pprec = 0, Ng = 0, want_p = 0, spec_m = 0, slot = 0;
    size_t ev_begin = 0, ev_end = 0;
  };
  int next_slot = 0;

  psdp_status ensure_snapshots() {
    if (!h->h_snap) {
      if (hipHostMalloc((void**)&h->h_snap, 2 * sizeof(State), hipHostMallocDefault) != hipSuccess) {
        h->h_snap = nullptr;
        return PSDP_ERR_OUT_OF_MEMORY;
      }
    }
    for (auto& e : h->snap_ev)
      if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return PSDP_OK;
  }

  // one Rayleigh-Ritz iteration on the trial basis given by `mode`, queued
  // and read back
  psdp_status iterate(int mode, int pprec, int mtarget, int nz) {
    Queued q;
    psdp_status r = enqueue(mode, pprec, mtarget, nz, 0, q);
    if (r != PSDP_OK) return r;
    return complete(q);
  }

  // the launches of one iteration, then the state snapshot into a pinned slot
  psdp_status enqueue(int mode, int pprec, int mtarget, int nz, int spec_m, Queued& q) {
    psdp_status pr = ensure_snapshots();
    if (pr != PSDP_OK) return pr;
    const int L = w.L, NC = w.NC;
    const size_t first_ev = h->pending.size();
    const int* stop = &w.st->stop;
    const int* stop_first = spec_m > 0 ? stop : nullptr;  // a speculative Gram skips when stopped
    const int hp = (mode == kModeFull) ? 1 : (mode == kModeXR ? 0 : has_p);
    // ---- Gram of the candidate columns (gives residual norms too)
    ColMap cand;
    int Ng;
    if (mode == kModeXOnly) {
      cand = colmap_seg(w.X, m, L);
      Ng = m;
    } else if (mode == kModeXZ) {
      cand = colmap_seg(w.X, m, L, w.Z, nz);
      Ng = m + nz;
    } else {
      cand = colmap_seg(w.X, m, L, w.R, m, hp ? w.P : nullptr, hp ? m : 0);
      Ng = hp ? 3 * m : 2 * m;
    }
    int nblk = 0;
    {
      ProfScope ps(h, "gram");
      HIP_TRY(launch_gram_partial(cand, nullptr, nullptr, Ng, nullptr, Ng, n, w.Gpart, NC,
                                  (size_t)NC * NC, &nblk, stop_first, s));
      HIP_TRY(launch_reduce_partials(w.Gpart, nblk, (size_t)NC * NC, NC, nullptr, Ng, nullptr, Ng,
                                     w.G, NC, stop_first, s));
    }
    // ---- decisions + first Cholesky-QR pass
    DecideArgs da{};
    da.G = w.G; da.ldg = NC; da.Ng = Ng; da.mode = mode; da.m = m; da.nz = nz;
    da.has_p = hp; da.phase_lowprec = pprec; da.tau = 1e-10; da.spec_m = spec_m;
    da.bases[0] = w.X; da.bases[1] = w.R; da.bases[2] = w.P; da.bases[3] = w.Z; da.bases[4] = w.S1;
    da.ld = L; da.T = w.T; da.ldt = NC; da.colptr = w.colptr; da.st = w.st;
    da.trace = h->trace > 1 ? 1 : 0;
    int Nmax = Ng;  // upper bound on the trial width
    {
      ProfScope ps(h, "chol");
      HIP_TRY(launch_decide_chol(da, Nmax, s));
    }
    // orth pass 1: S1 = S T1
    {
      ProfScope ps(h, "tsmm");
      HIP_TRY(launch_tsmm(colmap_ptrs(w.colptr), &w.st->N, Nmax, &w.st->Np, Nmax, w.T, NC, n,
                          w.S1, L, stop, s));
    }
    // orth pass 2
    {
      ProfScope ps(h, "gram");
      HIP_TRY(launch_gram_partial(colmap_seg(w.S1, NC, L), nullptr, &w.st->Np, Nmax, nullptr, 0,
                                  n, w.Gpart, NC, (size_t)NC * NC, &nblk, stop, s));
      HIP_TRY(launch_reduce_partials(w.Gpart, nblk, (size_t)NC * NC, NC, &w.st->Np, Nmax,
                                     &w.st->Np, Nmax, w.G, NC, stop, s));
    }
    DecideArgs db = da;
    db.spec_m = 0;
    db.mode = -1;  // second pass: the candidate count is st->Np on the device
    db.Ng = Nmax;
    {
      ProfScope ps(h, "chol");
      HIP_TRY(launch_decide_chol(db, Nmax, s));
    }
    {
      ProfScope ps(h, "tsmm");
      HIP_TRY(launch_tsmm(colmap_seg(w.S1, NC, L), &w.st->Np1, Nmax, &w.st->Np, Nmax, w.T, NC, n,
                          w.S2, L, stop, s));
    }
    // ---- block product AS = A S2 at the phase precision
    {
      ProfScope ps(h, "product");
      ProductArgs pa{};
      pa.A = amat(pprec); pa.lda = L; pa.n = n; pa.prec = pprec;
      pa.S = w.S2; pa.lds = L; pa.Y = w.AS; pa.ldy = L;
      pa.cols_dev = &w.st->Np; pa.cols_max = Nmax; pa.stop = stop;
      pa.partial = w.ppart; pa.partial_bytes = w.ppart_bytes; pa.max_slices = kProductSlices;
      HIP_TRY(launch_product(pa, s));
    }
    // ---- projected matrix K = S2^T A S2
    {
      ProfScope ps(h, "gram");
      ColMap s2 = colmap_seg(w.S2, NC, L), as = colmap_seg(w.AS, NC, L);
      HIP_TRY(launch_gram_partial(s2, &as, &w.st->Np, Nmax, &w.st->Np, Nmax, n, w.Gpart, NC,
                                  (size_t)NC * NC, &nblk, stop, s));
      HIP_TRY(launch_reduce_partials(w.Gpart, nblk, (size_t)NC * NC, NC, &w.st->Np, Nmax,
                                     &w.st->Np, Nmax, w.G, NC, stop, s));
    }
    // ---- Rayleigh-Ritz
    RRArgs ra{};
    ra.K = w.G; ra.ldk = NC; ra.mtarget = mtarget; ra.C = w.C; ra.ldc = NC;
    ra.log = w.log; ra.log_cap = w.log_cap; ra.max_sweeps = kMaxSweeps;
    ra.count_iter = (mode == kModeFull || mode == kModeXR) ? 1 : 0;
    ra.off_tol = 1e-14;
    ra.scratch = w.rrs;
    ra.trace = h->trace > 1 ? 1 : 0;
    ra.st = w.st;
    {
      ProfScope ps(h, "rr");
      if (h->rr_method == 0) {
        HIP_TRY(launch_rr_fast(ra, Nmax, std::min(mtarget, Nmax), s));
      } else if (h->rr_method == 2) {
        HIP_TRY(launch_rr_tri(ra, Nmax, std::min(mtarget, Nmax), s));
      } else {
        HIP_TRY(launch_rr(ra, Nmax, std::min(mtarget, Nmax), s));
      }
    }
    if (h->rr_method == 0) {
      ProfScope ps(h, "rrback");
      HIP_TRY(launch_rr_back(ra, Nmax, std::min(mtarget, Nmax), s));
    }
    // ---- update X, AX, P, R
    int want_p = (mode == kModeFull || mode == kModeXR) ? 1 : 0;
    {
      ProfScope ps(h, "tsmm");
      HIP_TRY(launch_update(w.S2, w.AS, L, w.C, NC, w.st, want_p, n, std::min(mtarget, Nmax),
                            w.X, w.AX, w.P, w.R, L, s));
    }
    q.mode = mode; q.pprec = pprec; q.Ng = Ng; q.want_p = want_p; q.spec_m = spec_m;
    q.slot = next_slot;
    next_slot ^= 1;
    q.ev_begin = first_ev;
    q.ev_end = h->pending.size();
    HIP_TRY(copy_to_host(h->h_snap + q.slot, w.st, sizeof(State), s));
    HIP_TRY(hipEventRecord(h->snap_ev[q.slot], s));
    return PSDP_OK;
  }

  // drops a queued iteration that will not be read back (its timing events
  // are not accumulated)
  void discard(const Queued& q) {
    for (size_t i = q.ev_begin; i < q.ev_end && i < h->pending.size(); ++i) {
      h->event_pool.push_back(h->pending[i].a);
      h->event_pool.push_back(h->pending[i].b);
    }
    if (q.ev_end <= h->pending.size() && q.ev_begin < q.ev_end)
      h->pending.erase(h->pending.begin() + q.ev_begin, h->pending.begin() + q.ev_end);
  }

  // waits for a queued iteration's snapshot, mirrors it and updates the block
  psdp_status complete(const Queued& q) {
    const int mode = q.mode, pprec = q.pprec, Ng = q.Ng, want_p = q.want_p;
    const size_t first_ev = q.ev_begin;
    HIP_TRY(spin_event(h->snap_ev[q.slot]));
    std::memcpy(hs, h->h_snap + q.slot, sizeof(State));
    if (h->trace) {
      double ph[4], pc[5];
      for (int q = 0; q < 4; ++q) ph[q] = (hs->t_phase[q + 1] - hs->t_phase[q]) * 1e-2;  // us
      for (int q = 0; q < 5; ++q) pc[q] = (hs->t_phase[q + 6] - hs->t_phase[q + 5]) * 1e-2;
      std::fprintf(stderr,
                   "psdp: iter %d mode %d prec %d N %d Np %d mk %d npos %d/%d stop %d rmax %.3e "
                   "rguard %.3e tol %.3e rr_us %.0f %.0f %.0f %.0f chol_us %.0f %.0f %.0f %.0f %.0f\n",
                   hs->iter, mode, pprec, hs->N, hs->Np, hs->mk, hs->npos_blk, hs->npos_rr,
                   hs->stop, hs->res_max_pos, hs->guard_res, hs->tol, ph[0], ph[1], ph[2], ph[3],
                   pc[0], pc[1], pc[2], pc[3], pc[4]);
      if (h->trace > 1)
        std::fprintf(stderr,
                     "psdp:   rr_sub_us %.0f %.0f | %.0f %.0f %.0f %.0f | rounds %lld mgs %.0f"
                     " | chol_sub_us %.0f %.0f %.0f | inv_diag_us %.0f\n",
                     hs->t_sub[0] * 1e-2, hs->t_sub[1] * 1e-2, hs->t_sub[2] * 1e-2,
                     hs->t_sub[3] * 1e-2, hs->t_sub[4] * 1e-2, hs->t_sub[5] * 1e-2,
                     hs->t_sub[6], hs->t_sub[7] * 1e-2, hs->t_sub[8] * 1e-2,
                     hs->t_sub[9] * 1e-2, hs->t_sub[10] * 1e-2, hs->t_sub[11] * 1e-2);
    }
    if (h->prof && hs->stop == kRunning) {
      auto& e = h->prof_tab["rr_stats"];  // launches: RR calls, bytes: sum Np, flops: sum rounds
      e.launches += 1;
      e.bytes += hs->Np;
      e.flops += hs->jacobi_rounds;
      for (int ph = 0; ph < 4; ++ph) {
        auto& q = h->prof_tab[std::string("rr_phase") + char('0' + ph)];
        long long dt = hs->t_phase[ph + 1] - hs->t_phase[ph];
        if (dt > 0 && dt < (1ll << 40)) { q.launches += 1; q.ms += dt * 1e-5; }  // 100 MHz clock
      }
    }
    if (hs->stop == kRunning || mode == kModeXOnly || mode == kModeXZ) {
      attribute(first_ev, q.ev_end, Ng, pprec);
    } else if (h->prof) {
      // stopped after the decision pass: only the first Gram and decision ran
      for (size_t i = first_ev; i < q.ev_end && i < h->pending.size(); ++i) {
        PendingEvent& p = h->pending[i];
        if (p.family == "gram" && p.bytes == 0) { p.bytes = 8.0 * n * Ng; p.flops = (double)n * Ng * Ng; }
        if (p.family == "chol" && p.flops == 0) { p.flops = 2.0 * Ng * Ng * (double)Ng / 3.0; p.bytes = 16.0 * Ng * Ng; }
      }
    }
    if (hs->stop == kRunning || mode == kModeXOnly || mode == kModeXZ) {
      if (hs->stop == kBreakdown) return PSDP_ERR_NUMERICAL;
      m = hs->mk;
      has_p = want_p;
    }
    return PSDP_OK;
  }
  // residual statistics of the current block without changing it
  psdp_status evaluate() {
    const int L = w.L, NC = w.NC;
    ColMap cand = colmap_seg(w.X, m, L, w.R, m, has_p ? w.P : nullptr, has_p ? m : 0);
    int Ng = has_p ? 3 * m : 2 * m;
    int nblk = 0;
    {
      ProfScope ps(h, "gram");
      HIP_TRY(launch_gram_partial(cand, nullptr, nullptr, Ng, nullptr, Ng, n, w.Gpart, NC,
                                  (size_t)NC * NC, &nblk, nullptr, s));
      HIP_TRY(launch_reduce_partials(w.Gpart, nblk, (size_t)NC * NC, NC, nullptr, Ng, nullptr, Ng,
                                     w.G, NC, nullptr, s));
    }
    DecideArgs da{};
    da.G = w.G; da.ldg = NC; da.Ng = Ng; da.mode = kModeEval; da.m = m; da.nz = 0;
    da.has_p = has_p; da.tau = 1e-10;
    da.bases[0] = w.X; da.bases[1] = w.R; da.bases[2] = w.P; da.bases[3] = w.Z; da.bases[4] = w.S1;
    da.ld = L; da.T = w.T; da.ldt = NC; da.colptr = w.colptr; da.st = w.st;
    da.trace = h->trace > 1 ? 1 : 0;
    {
      ProfScope ps(h, "chol");
      HIP_TRY(launch_decide_chol(da, Ng, s));
    }
    return read_state();
  }
};


// Lower end of the spectrum of the ingested matrix: `steps` plain Lanczos
// steps from a seeded random vector (products at precision `prec`), then
// theta_min(T) less twice the residual norm of its Ritz pair and 1 % of its
// size, but never below theta_min - beta_steps (Zhou and Saad's estimator):
// the Ritz value lies above the spectrum's lower end and an eigenvalue lies
// within the residual of it.  Used for the damped interval of the Chebyshev
// filter, where an end slightly inside the spectrum costs little (the
// lowest eigenvalues grow by a small factor) and one far outside slows
// every pass.
// lanczos_launch queues the steps on the handle's second stream (the
// ingested copies of A must be complete; only A and the Lanczos region of
// the workspace are touched, so the first Rayleigh-Ritz step can run on the
// main stream meanwhile); lanczos_finish waits for them and reads the bound.
psdp_status lanczos_launch(psdp_handle h, int n, int prec, int steps, uint64_t seed,
                           uint64_t stream_id) {
  Workspace& w = h->ws;
  if (!h->aux && hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) != hipSuccess) {
    h->aux = nullptr;
    return PSDP_ERR_HIP;
  }
  if (!h->h_pin_aux &&
      hipHostMalloc((void**)&h->h_pin_aux, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    h->h_pin_aux = nullptr;
    return PSDP_ERR_OUT_OF_MEMORY;
  }
  hipStream_t s = h->aux;
  const int L = w.L;
  steps = std::max(1, std::min(steps, std::min(n, 30)));
  double* vb[3] = {w.lz, w.lz + L, w.lz + 2 * (size_t)L};
  double* coef = w.lz + 3 * (size_t)L;
  double* out = coef + 96;
  double* part = coef + 128;
  HIP_TRY(launch_fill_normal(vb[0], L, n, 0, 1, seed, stream_id, s));
  HIP_TRY(launch_lanczos_vec(n, -1, 0, vb[0], nullptr, nullptr, coef, out, s));
  int iv = 0, iw = 1, ip = 2;
  for (int j = 0; j < steps; ++j) {
    {
      ProfScope ps(h, "lanczos", (double)product_elem_bytes(prec) * n * (double)n + 16.0 * n,
                   2.0 * n * (double)n, -1, s);
      ProductArgs pa{};
      pa.A = prec == 0 ? (const void*)w.A64 : w.Alp; pa.lda = L; pa.n = n; pa.prec = prec;
      pa.S = vb[iv]; pa.lds = L; pa.Y = vb[iw]; pa.ldy = L;
      pa.cols_dev = nullptr; pa.cols_max = 1; pa.stop = nullptr;
      pa.partial = part; pa.partial_bytes = sizeof(double) * kProductSlices * (size_t)L;
      pa.max_slices = kProductSlices;
      HIP_TRY(launch_product(pa, s));
      HIP_TRY(launch_lanczos_vec(n, j, j == steps - 1, vb[iw], vb[iv], vb[ip], coef, out, s));
    }
    const int t = ip;
    ip = iv;
    iv = iw;
    iw = t;
  }
  HIP_TRY(copy_to_host(h->h_pin_aux, out, 4 * sizeof(double), s));
  return PSDP_OK;
}

psdp_status lanczos_finish(psdp_handle h, double* lo, double* theta_min) {
  HIP_TRY(hipStreamSynchronize(h->aux));
  *lo = h->h_pin_aux[0];
  *theta_min = h->h_pin_aux[1];
  if (h->trace)
    std::fprintf(stderr, "psdp: lanczos theta_min %.6e beta %.3e residual %.3e lower end %.6e\n",
                 h->h_pin_aux[1], h->h_pin_aux[2], h->h_pin_aux[3], h->h_pin_aux[0]);
  return std::isfinite(*lo) ? PSDP_OK : PSDP_ERR_NUMERICAL;
}

// Waits for the second stream when a call leaves while the Lanczos steps
// may still be queued (an error return), so that nothing later overwrites
// A under them.
struct AuxJoin {
  psdp_handle h;
  bool pending = false;
  ~AuxJoin() {
    if (pending && h->aux) (void)hipStreamSynchronize(h->aux);
  }
};

psdp_status ensure_cert(psdp_handle h, int L) {
  if (h->cert_base && h->cert_L >= L) return PSDP_OK;
  if (!h->cert_host &&
      hipHostMalloc((void**)&h->cert_host, sizeof(CertState), hipHostMallocDefault) != hipSuccess) {
    h->cert_host = nullptr;
    return PSDP_ERR_OUT_OF_MEMORY;
  }
  if (h->cert_base) {
    (void)hipStreamSynchronize(h->stream);
    hipFree(h->cert_base);
    h->cert_base = nullptr;
    h->cert_L = 0;
  }
  const int T = L / kCertTile;
  const size_t oM = 0;
  const size_t oP = align_up(oM + sizeof(double) * (size_t)L * L, 256);
  const size_t oS = align_up(oP + sizeof(double) * (size_t)(3 * T + 8), 256);
  const size_t total = align_up(oS + sizeof(CertState), 256);
  char* base = nullptr;
  if (hipMalloc(&base, total) != hipSuccess) return PSDP_ERR_OUT_OF_MEMORY;
  h->cert_base = base;
  h->cert_L = L;
  h->cert_M = (double*)(base + oM);
  h->cert_part = (double*)(base + oP);
  h->cert_dev = (CertState*)(base + oS);
  return PSDP_OK;
}

// Tail certificate (paper §5.2, Thm `bound`: the term ||Pi(Vt_perp^T A
// Vt_perp)||_F) for the first mt columns of the block X, the positive Ritz
// vectors of A = s sym(X) held in A64: an FP64 Cholesky factorization of
// (delta - eta) I - P A P + c Vt Vt^T, P = I - Vt Vt^T.  On success every
// eigenvalue of Vt_perp^T A Vt_perp is below out->delta_eff.  Clobbers the
// work columns AS (W = A Vt), S1 (U), G and T (Vt^T W, Vt^T Vt) and the
// split-K partials; X and A64 are only read.
psdp_status run_certificate(psdp_handle h, int n, int mt, double fro2, double delta, int* certified,
                            CertState* out) {
  Workspace& w = h->ws;
  hipStream_t s = h->stream;
  const int L = w.L, NC = w.NC;
  if (mt < 0 || mt > w.MC) return PSDP_ERR_INVALID_ARG;
  psdp_status ps = ensure_cert(h, L);
  if (ps != PSDP_OK) return ps;
  const double nn = n;
  CertState* hc = h->cert_host;
  std::memset(hc, 0, sizeof(CertState));
  hc->delta = delta;
  hc->fro_a = std::sqrt(std::max(fro2, 0.0));
  hc->c = fro2 > 0.0 ? std::sqrt(fro2 / nn) : 1.0;
  hc->n = n;
  hc->L = L;
  hc->mt = mt;
  {
    // algorithmic work: W = A Vt (2 n^2 mt), the rank-2 mt formation of the
    // lower triangle (2 n^2 mt), the factorization (n^3 / 3); bytes: A read
    // twice (full, then its lower triangle), M written and read (lower)
    ProfScope pscope(h, "cert", 20.0 * nn * nn, 4.0 * nn * nn * mt + nn * nn * nn / 3.0);
    if (mt > 0) {
      ProductArgs pa{};
      pa.A = w.A64; pa.lda = L; pa.n = n; pa.prec = 0;
      pa.S = w.X; pa.lds = L; pa.Y = w.AS; pa.ldy = L;
      pa.cols_dev = nullptr; pa.cols_max = mt; pa.stop = nullptr;
      pa.partial = w.ppart; pa.partial_bytes = w.ppart_bytes; pa.max_slices = kProductSlices;
      HIP_TRY(launch_product(pa, s));
      int nblk = 0;
      const ColMap vx = colmap_seg(w.X, mt, L), wa = colmap_seg(w.AS, mt, L);
      HIP_TRY(launch_gram_partial(vx, &wa, nullptr, mt, nullptr, mt, n, w.Gpart, NC, (size_t)NC * NC,
                                  &nblk, nullptr, s));
      HIP_TRY(launch_reduce_partials(w.Gpart, nblk, (size_t)NC * NC, NC, nullptr, mt, nullptr, mt,
                                     w.G, NC, nullptr, s));
      HIP_TRY(launch_gram_partial(vx, nullptr, nullptr, mt, nullptr, mt, n, w.Gpart, NC,
                                  (size_t)NC * NC, &nblk, nullptr, s));
      HIP_TRY(launch_reduce_partials(w.Gpart, nblk, (size_t)NC * NC, NC, nullptr, mt, nullptr, mt,
                                     w.T, NC, nullptr, s));
  }
    HIP_TRY(hipMemcpyAsync(h->cert_dev, hc, sizeof(CertState), hipMemcpyHostToDevice, s));
    const int T = L / kCertTile;
    double* prep_part = h->cert_part;
    double* diag_part = h->cert_part + 2 * T;
    HIP_TRY(launch_cert_prep(w.X, w.AS, L, w.G, NC, mt, n, L, hc->c, w.S1, prep_part, s));
    HIP_TRY(launch_cert_form(w.A64, L, w.X, w.S1, L, mt, n, L, h->cert_M, diag_part, s));
    HIP_TRY(launch_cert_shift(w.T, NC, prep_part, mt > 0 ? T : 0, diag_part, h->cert_M, h->cert_dev,
                              s));
    HIP_TRY(launch_cert_chol(h->cert_M, L, h->cert_dev, s));
  }
  HIP_TRY(copy_to_host(hc, h->cert_dev, sizeof(CertState), s));
  HIP_TRY(hipStreamSynchronize(s));
  *out = *hc;
  *certified = (hc->fail == 0) ? 1 : 0;
  if (h->trace)
    std::fprintf(stderr, "psdp: cert n %d mt %d fail %d eta %.3e delta %.3e diag_us load %.1f factor %.1f store %.1f\n",
                 n, mt, hc->fail, hc->eta, hc->delta_eff, (hc->t_diag[1] - hc->t_diag[0]) * 1e-2,
                 (hc->t_diag[2] - hc->t_diag[1]) * 1e-2, (hc->t_diag[3] - hc->t_diag[2]) * 1e-2);
  return PSDP_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char* psdp_version(void) { return "psdp 0.1 (gfx950)"; }

const char* psdp_status_str(psdp_status s) {
  switch (s) {
    case PSDP_OK: return "PSDP_OK";
    case PSDP_NOT_CONVERGED: return "PSDP_NOT_CONVERGED";
    case PSDP_PENDING: return "PSDP_PENDING";
    case PSDP_FELL_BACK_FULL_EIG: return "PSDP_FELL_BACK_FULL_EIG";
    case PSDP_ERR_INVALID_ARG: return "PSDP_ERR_INVALID_ARG";
    case PSDP_ERR_HIP: return "PSDP_ERR_HIP";
    case PSDP_ERR_OUT_OF_MEMORY: return "PSDP_ERR_OUT_OF_MEMORY";
    case PSDP_ERR_NUMERICAL: return "PSDP_ERR_NUMERICAL";
    case PSDP_ERR_CAPACITY: return "PSDP_ERR_CAPACITY";
  }
  return "PSDP_UNKNOWN_STATUS";
}

void psdp_default_options(psdp_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->side = PSDP_SIDE_AUTO;
  o->prec = PSDP_PREC_FP64;
  o->tol = 0.0;
  o->max_iter = 300;
  o->refine_fp64 = 1;
  o->ladder = 1;
  o->certify = 1;
  o->seed = 0x1912276700000000ull;
  o->side_threshold = 1.0 / 3.0;
  o->expand_cols = 0;
  o->pos_hint = -1;
  o->fallback_full = 0;
  o->block_guard = 4;
  o->batch_variant = -1;
  o->batch_graph = 1;
  o->bound_rel_max = 0.0;
  o->certify_delta = 0.0;
  o->warm_side = PSDP_SIDE_AUTO;
  o->method = PSDP_METHOD_LOBPCG;
  o->method_param = 0;
}

psdp_status psdp_workspace_bytes(int n, int m_cap, int prec, size_t* bytes) {
  if (!bytes || n < 1 || m_cap < 1 || prec < 0 || prec > 2) return PSDP_ERR_INVALID_ARG;
  size_t L = (size_t)round_up(n, 64);
  size_t MC = (size_t)std::min(m_cap, kMaxM), NC = 3 * MC;
  size_t nblk = (L + kGramRows - 1) / kGramRows;
  size_t T32 = (L + 31) / 32;
  size_t b = 8 * L * L + 4 * L * L + 5 * 8 * L * MC + 3 * 8 * L * NC + 8 * nblk * NC * NC +
             8 * 8 * L * NC +
             3 * 8 * NC * NC + 5 * 8 * NC * MC + 8 * (size_t)kMaxSweeps * (NC + 1) * (NC + 2) + 8 * NC +
             8 * T32 * (T32 + 1) / 2 + sizeof(State) + 4096;
  *bytes = b;
  return PSDP_OK;
}

psdp_status psdp_create(psdp_handle* out, int device, void* stream) {
  if (!out) return PSDP_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return PSDP_ERR_HIP;
  if (device < 0 || device >= count) return PSDP_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return PSDP_ERR_HIP;
  psdp_handle h = new (std::nothrow) psdp_handle_s();
  if (!h) return PSDP_ERR_OUT_OF_MEMORY;
  h->device = device;
  h->stream = (hipStream_t)stream;
  if (small_kernels_init() != hipSuccess || rr_tri_init() != hipSuccess) {
    delete h;
    return PSDP_ERR_HIP;
  }
  if (const char* m = std::getenv("PSDP_RR_METHOD")) {
    const int v = std::atoi(m);
    h->rr_method = (v == 1 || v == 2) ? v : 0;
  }
  if (const char* t = std::getenv("PSDP_TRACE")) h->trace = std::atoi(t);
  if (hipHostMalloc((void**)&h->h_state, sizeof(State), hipHostMallocDefault) != hipSuccess) {
    delete h;
    return PSDP_ERR_OUT_OF_MEMORY;
  }
  *out = h;
  return PSDP_OK;
}

psdp_status psdp_destroy(psdp_handle h) {
  if (!h) return PSDP_ERR_INVALID_ARG;
  hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  prof_collect(h);
  for (auto e : h->event_pool) hipEventDestroy(e);
  if (h->sync_ev) hipEventDestroy(h->sync_ev);
  if (h->aux) {
    (void)hipStreamSynchronize(h->aux);
    hipStreamDestroy(h->aux);
  }
  if (h->h_pin_aux) hipHostFree(h->h_pin_aux);
  for (auto e : h->snap_ev) if (e) hipEventDestroy(e);
  if (h->h_snap) hipHostFree(h->h_snap);
  if (h->ws.base) hipFree(h->ws.base);
  if (h->eig_A) hipFree(h->eig_A);
  if (h->h_state) hipHostFree(h->h_state);
  if (h->h_pin) hipHostFree(h->h_pin);
  if (h->rb) rocblas_destroy_handle(h->rb);
  batch_engine_free(h->batch);
  if (h->beig) hipFree(h->beig);
  if (h->cert_base) hipFree(h->cert_base);
  if (h->cert_host) hipHostFree(h->cert_host);
  delete h;
  return PSDP_OK;
}

psdp_status psdp_set_stream(psdp_handle h, void* stream) {
  if (!h) return PSDP_ERR_INVALID_ARG;
  h->stream = (hipStream_t)stream;
  if (h->rb) rocblas_set_stream(h->rb, h->stream);
  return PSDP_OK;
}

psdp_status psdp_profile_enable(psdp_handle h, int on) {
  if (!h) return PSDP_ERR_INVALID_ARG;
  prof_collect(h);
  h->prof_tab.clear();
  h->prof = on != 0;
  return PSDP_OK;
}

psdp_status psdp_profile_filter(psdp_handle h, const char* families) {
  if (!h) return PSDP_ERR_INVALID_ARG;
  prof_collect(h);
  h->prof_only.clear();
  if (families) {
    std::string cur;
    for (const char* c = families;; ++c) {
      if (*c == ',' || *c == '\0') {
        if (!cur.empty()) h->prof_only.insert(cur);
        cur.clear();
        if (*c == '\0') break;
      } else if (*c != ' ') {
        cur += *c;
      }
    }
  }
  return PSDP_OK;
}

psdp_status psdp_profile_get(psdp_handle h, const char* family, long* launches, double* total_ms,
                             double* bytes, double* flops) {
  if (!h || !family) return PSDP_ERR_INVALID_ARG;
  prof_collect(h);
  auto it = h->prof_tab.find(family);
  ProfEntry e;
  if (it != h->prof_tab.end()) e = it->second;
  if (launches) *launches = e.launches;
  if (total_ms) *total_ms = e.ms;
  if (bytes) *bytes = e.bytes;
  if (flops) *flops = e.flops;
  return PSDP_OK;
}

}  // extern "C"

// ------------------------------------------------------------ full eig ----
static psdp_status full_eig_core(psdp_handle h, int n, const double* X, int ldx, double* lambda_all,
                                 double* Pi, int ldpi, double* V, int ldv, int m_cap, int* m_out,
                                 double* lambda_pos, int* npos_out) {
  hipStream_t s = h->stream;
  if (!h->rb) {
    if (rocblas_create_handle(&h->rb) != rocblas_status_success) return PSDP_ERR_HIP;
  }
  rocblas_set_stream(h->rb, s);
  int lda = round_up(n, 64);
  const int T32 = (lda + 31) / 32;
  const size_t fro_n = (size_t)T32 * (T32 + 1) / 2;
  if (h->eig_cap < lda) {
    if (h->eig_A) hipFree(h->eig_A);
    h->eig_A = nullptr;
    // the ingest writes the zero padding too: the copy is lda x lda
    // d and e are sized for any order up to lda (later calls reuse the buffer)
    size_t b = sizeof(double) * ((size_t)lda * lda + 2 * (size_t)lda + 8 + fro_n + 8) + 64;
    if (hipMalloc(&h->eig_A, b) != hipSuccess) { h->eig_cap = 0; return PSDP_ERR_OUT_OF_MEMORY; }
    h->eig_cap = lda;
  }
  const int cap = h->eig_cap;
  double* A = h->eig_A;
  double* d = A + (size_t)cap * cap;
  double* e = d + cap;
  rocblas_int* info = (rocblas_int*)(e + cap);
  double* fro_part = e + cap + 8;
  int* nonfin = (int*)(fro_part + fro_n);
  // symmetric copy (lower triangle of X) via the ingest kernel, FP64 only
  int nb = 0;
  HIP_TRY(launch_ingest(X, ldx, n, 1.0, A, lda, lda, nullptr, 0, fro_part, nonfin, s, &nb));
  (void)nb;
  {
    ProfScope pscope(h, "fulleig");
    if (rocsolver_dsyevd(h->rb, rocblas_evect_original, rocblas_fill_lower, n, A, lda, d, e, info) !=
        rocblas_status_success)
      return PSDP_ERR_HIP;
  }
  // count positive eigenvalues (ascending order)
  psdp_status pp = ensure_pinned(h, sizeof(double) * (size_t)n + 64);
  if (pp != PSDP_OK) return pp;
  HIP_TRY(copy_to_host(h->h_pin, d, sizeof(double) * n, s));
  HIP_TRY(copy_to_host(h->h_pin + n, info, sizeof(rocblas_int), s));
  HIP_TRY(hipStreamSynchronize(s));
  int infov = 0;
  std::memcpy(&infov, h->h_pin + n, sizeof(rocblas_int));
  int npos = 0;
  bool finite = true;
  for (int i = 0; i < n; ++i) {
    npos += (h->h_pin[i] > 0.0);
    finite &= std::isfinite(h->h_pin[i]);
  }
  if (infov != 0 || !finite) return PSDP_ERR_NUMERICAL;
  if (lambda_all) HIP_TRY(hipMemcpyAsync(lambda_all, d, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  {
    ProfScope pscope(h, "rebuild", 8.0 * n * (double)n, (double)n * n * npos);
    HIP_TRY(launch_rebuild(A + (size_t)(n - npos) * lda, lda, d + (n - npos), npos, n, nullptr, 0,
                           0.0, Pi, ldpi, s));
  }
  if (V && m_out) {
    // the positive pairs plus the next ones as guard columns (a warm start
    // for a later block solve), largest first
    int k = std::min(std::min(m_cap, n), npos + std::max(4, (int)std::ceil(0.2 * npos)));
    for (int j = 0; j < k; ++j) {
      HIP_TRY(hipMemcpyAsync(V + (size_t)j * ldv, A + (size_t)(n - 1 - j) * lda, sizeof(double) * n,
                             hipMemcpyDeviceToDevice, s));
      HIP_TRY(hipMemcpyAsync(lambda_pos + j, d + (n - 1 - j), sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    *m_out = k;
  }
  if (npos_out) *npos_out = npos;
  HIP_TRY(hipStreamSynchronize(s));
  return PSDP_OK;
}

extern "C" psdp_status psdp_full_eig_project(psdp_handle h, int n, const double* X, int ldx,
                                             double* lambda_all, double* Pi, int ldpi) {
  if (!h || n < 1 || !X || !Pi || ldx < n || ldpi < n) return PSDP_ERR_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return PSDP_ERR_HIP;
  return full_eig_core(h, n, X, ldx, lambda_all, Pi, ldpi, nullptr, 0, 0, nullptr, nullptr, nullptr);
}

// --------------------------------------------------------- block product ---
extern "C" psdp_status psdp_block_product(psdp_handle h, int n, const double* X, int ldx,
                                          const double* S, int lds, int k, int prec, double* Y,
                                          int ldy) {
  if (!h || n < 1 || k < 1 || k > kMaxN || !X || !S || !Y || ldx < n || lds < n || ldy < n ||
      prec < 0 || prec > 2)
    return PSDP_ERR_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return PSDP_ERR_HIP;
  psdp_status ps = ensure_workspace(h, n, (k + 2) / 3, prec);
  if (ps != PSDP_OK) return ps;
  Workspace& w = h->ws;
  if (k > w.NC) return PSDP_ERR_CAPACITY;
  hipStream_t s = h->stream;
  int nb = 0;
  HIP_TRY(launch_ingest(X, ldx, n, 1.0, w.A64, w.L, w.L, w.Alp, prec, w.fro_part, w.nonfinite, s, &nb));
  HIP_TRY(launch_copy_cols(S, lds, w.S2, w.L, n, k, s));
  ProductArgs pa{};
  pa.A = prec == 0 ? (const void*)w.A64 : w.Alp; pa.lda = w.L; pa.n = n; pa.prec = prec;
  pa.S = w.S2; pa.lds = w.L; pa.Y = w.AS; pa.ldy = w.L;
  pa.cols_dev = nullptr; pa.cols_max = k; pa.stop = nullptr;
  pa.partial = w.ppart; pa.partial_bytes = w.ppart_bytes; pa.max_slices = kProductSlices;
  {
    ProfScope pscope(h, "product", (double)product_elem_bytes(prec) * n * (double)n + 16.0 * n * k,
                     2.0 * n * (double)n * k);
    HIP_TRY(launch_product(pa, s));
  }
  HIP_TRY(launch_copy_cols(w.AS, w.L, Y, ldy, n, k, s));
  HIP_TRY(hipStreamSynchronize(s));
  return PSDP_OK;
}

// ------------------------------------------------------ tail certificate ---
extern "C" psdp_status psdp_certify_tail(psdp_handle h, int n, const double* X, int ldx,
                                         const double* V, int ldv, int m, double delta,
                                         int* certified, double* delta_eff, double* eta) {
  if (!h || n < 1 || !X || ldx < n || m < 0 || m > kMaxM || m > n || (m > 0 && (!V || ldv < n)) ||
      !(delta > 0.0) || !(delta < INFINITY) || !certified)
    return PSDP_ERR_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return PSDP_ERR_HIP;
  psdp_status ps = ensure_workspace(h, n, std::max(m, 1), 0);
  if (ps != PSDP_OK) return ps;
  ps = ensure_pinned(h, 64);
  if (ps != PSDP_OK) return ps;
  Workspace& w = h->ws;
  hipStream_t s = h->stream;
  HIP_TRY(hipMemsetAsync(w.nonfinite, 0, sizeof(int), s));
  int nb = 0;
  HIP_TRY(launch_ingest(X, ldx, n, 1.0, w.A64, w.L, w.L, w.Alp, 0, w.fro_part, w.nonfinite, s, &nb));
  HIP_TRY(launch_reduce_sum(w.fro_part, nb, w.scal, s));
  HIP_TRY(copy_to_host(h->h_pin, w.scal, sizeof(double), s));
  HIP_TRY(copy_to_host(h->h_pin + 1, w.nonfinite, sizeof(int), s));
  HIP_TRY(hipStreamSynchronize(s));
  const double fro2 = h->h_pin[0];
  int nonfin = 0;
  std::memcpy(&nonfin, h->h_pin + 1, sizeof(int));
  if (nonfin || !std::isfinite(fro2)) return PSDP_ERR_NUMERICAL;
  if (m > 0) HIP_TRY(launch_copy_cols(V, ldv, w.X, w.L, n, m, s));
  CertState cs{};
  int ok = 0;
  ps = run_certificate(h, n, m, fro2, delta, &ok, &cs);
  if (ps != PSDP_OK) return ps;
  *certified = ok;
  if (delta_eff) *delta_eff = cs.delta_eff;
  if (eta) *eta = cs.eta;
  return PSDP_OK;
}

// ---------------------------------------------------------- single cone ---
static void fill_info_defaults(psdp_info* info) {
  std::memset(info, 0, sizeof(*info));
  info->err_bound = NAN;
  info->res_fro = NAN;
  info->tail_est = NAN;
  info->pi_fro = NAN;
  info->theta_guard = NAN;
  info->n_pos_full = -1;
  info->pos_est = -1;
  info->block_side = PSDP_SIDE_POS;
  info->cert_delta = NAN;
  info->cert_eta = NAN;
  info->trunc_bound = NAN;
  info->spec_lower = NAN;
}

// Exact projection of many cones (n <= 256) through zero-padded buckets of
// order round_up(n, 32) and one batched rocSOLVER eigendecomposition per
// bucket.  Outputs per cone i (caller's order): n_pos[i], m_out[i] (leading
// columns written to V[i], 0 when V is null), bad[i] (non-finite input or
// solver failure).
static psdp_status full_eig_batched(psdp_handle h, int count, const int* n,
                                    const double* const* X, double* const* Pi,
                                    double* const* V, const int* m_cap, double* const* lambda,
                                    int* m_out, int* n_pos, int* bad) {
  hipStream_t s = h->stream;
  if (!h->rb && rocblas_create_handle(&h->rb) != rocblas_status_success) return PSDP_ERR_HIP;
  rocblas_set_stream(h->rb, s);
  std::map<int, std::vector<int>> buckets;
  for (int i = 0; i < count; ++i) buckets[round_up(n[i], 32)].push_back(i);
  size_t maxA = 0, maxD = 0;
  for (auto& b : buckets) {
    maxA = std::max(maxA, (size_t)b.first * b.first * b.second.size());
    maxD = std::max(maxD, (size_t)b.first * b.second.size());
  }
  const size_t oA = 0, oD = align_up(oA + 8 * maxA, 256), oE = align_up(oD + 8 * maxD, 256);
  const size_t oC = align_up(oE + 8 * maxD, 256);
  const size_t oI = align_up(oC + sizeof(EigCone) * count, 256);
  const size_t oO = align_up(oI + sizeof(int) * count, 256);
  const size_t oB = align_up(oO + 2 * sizeof(int) * count, 256);
  const size_t total = align_up(oB + sizeof(int) * count, 256);
  if (total > h->beig_bytes) {
    (void)hipStreamSynchronize(s);
    if (h->beig) hipFree(h->beig);
    h->beig = nullptr;
    h->beig_bytes = 0;
    if (hipMalloc(&h->beig, total) != hipSuccess) return PSDP_ERR_OUT_OF_MEMORY;
    h->beig_bytes = total;
  }
  const size_t pin = sizeof(EigCone) * count + 4 * sizeof(int) * count + 64;
  psdp_status pp = ensure_pinned(h, pin);
  if (pp != PSDP_OK) return pp;
  char* base = h->beig;
  double* A = (double*)(base + oA);
  double* D = (double*)(base + oD);
  double* E = (double*)(base + oE);
  EigCone* dc = (EigCone*)(base + oC);
  rocblas_int* dinfo = (rocblas_int*)(base + oI);
  int* dout = (int*)(base + oO);
  int* dbad = (int*)(base + oB);
  EigCone* hc = (EigCone*)h->h_pin;
  int* hint = (int*)(hc + count);  // out (2 count), bad (count), info (count)
  std::vector<int> order;
  order.reserve(count);
  int q = 0;
  for (auto& b : buckets) {
    const int nb = b.first, cnt = (int)b.second.size();
    for (int t = 0; t < cnt; ++t) {
      const int i = b.second[t];
      order.push_back(i);
      EigCone c{};
      c.X = X[i];
      c.Pi = Pi[i];
      c.V = V ? V[i] : nullptr;
      c.lam = lambda ? lambda[i] : nullptr;
      c.n = n[i];
      c.m_cap = m_cap ? m_cap[i] : 0;
      hc[q + t] = c;
    }
    HIP_TRY(hipMemcpyAsync(dc + q, hc + q, sizeof(EigCone) * cnt, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_eig_pad(dc + q, cnt, A, nb, dbad + q, s));
    if (rocsolver_dsyevd_strided_batched(h->rb, rocblas_evect_original, rocblas_fill_lower, nb, A, nb,
                                         (rocblas_stride)nb * nb, D, nb, E, nb, dinfo + q,
                                         cnt) != rocblas_status_success)
      return PSDP_ERR_HIP;
    HIP_TRY(launch_eig_rebuild(dc + q, cnt, A, D, nb, s));
    HIP_TRY(launch_eig_leading(dc + q, cnt, A, D, nb, dout + 2 * q, s));
    q += cnt;
  }
  HIP_TRY(copy_to_host(hint, dout, 2 * sizeof(int) * count, s));
  HIP_TRY(copy_to_host(hint + 2 * count, dbad, sizeof(int) * count, s));
  HIP_TRY(copy_to_host(hint + 3 * count, dinfo, sizeof(int) * count, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int t = 0; t < count; ++t) {
    const int i = order[t];
    n_pos[i] = hint[2 * t];
    m_out[i] = hint[2 * t + 1];
    bad[i] = hint[2 * count + t] != 0 || hint[3 * count + t] != 0;
  }
  return PSDP_OK;
}

static void fill_full_info(psdp_info* f, int npos, int mo, int bad) {
  std::memset(f, 0, sizeof(*f));
  f->side_used = PSDP_SIDE_FULL;
  f->n_pos = npos;
  f->n_pos_full = npos;
  f->m_out = mo;
  f->status = bad ? PSDP_ERR_NUMERICAL : PSDP_OK;
}

extern "C" psdp_status psdp_full_eig_project_batched(psdp_handle h, int count, const int* n,
                                                     const double* const* X, double* const* V,
                                                     const int* m_cap, int* m_inout,
                                                     double* const* lambda, double* const* Pi,
                                                     psdp_info* info) {
  if (!h || count < 0) return PSDP_ERR_INVALID_ARG;
  if (count == 0) return PSDP_OK;
  if (!n || !X || !Pi || !info) return PSDP_ERR_INVALID_ARG;
  const bool want_v = V != nullptr;
  if (want_v && (!m_cap || !m_inout || !lambda)) return PSDP_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > kBatchMaxN || !X[i] || !Pi[i]) return PSDP_ERR_INVALID_ARG;
    if ((const void*)Pi[i] == (const void*)X[i]) return PSDP_ERR_INVALID_ARG;
    if (want_v && (!V[i] || !lambda[i] || m_cap[i] < 1)) return PSDP_ERR_INVALID_ARG;
  }
  if (hipSetDevice(h->device) != hipSuccess) return PSDP_ERR_HIP;
  std::vector<int> mo(count, 0), np(count, 0), bad(count, 0);
  psdp_status rc;
  {
    ProfScope pscope(h, "fulleig");
    rc = full_eig_batched(h, count, n, X, Pi, want_v ? V : nullptr, want_v ? m_cap : nullptr,
                          want_v ? lambda : nullptr, mo.data(), np.data(), bad.data());
  }
  if (rc != PSDP_OK) return rc;
  psdp_status worst = PSDP_OK;
  for (int i = 0; i < count; ++i) {
    fill_full_info(&info[i], np[i], mo[i], bad[i]);
    if (want_v && !bad[i]) m_inout[i] = mo[i];
    if (bad[i]) worst = PSDP_ERR_NUMERICAL;
  }
  return worst;
}

extern "C" psdp_status psdp_project_batched(psdp_handle h, int count, const int* n,
                                            const double* const* X, double* const* V,
                                            const int* m_cap, int* m_inout,
                                            double* const* lambda, double* const* Pi,
                                            const psdp_options* opt_in, psdp_info* info) {
  psdp_options opt;
  if (opt_in) opt = *opt_in; else psdp_default_options(&opt);
  // ---- validation (no launch before this point)
  if (!h || count < 0) return PSDP_ERR_INVALID_ARG;
  if (count == 0) return PSDP_OK;
  if (!n || !X || !V || !m_cap || !m_inout || !lambda || !Pi || !info) return PSDP_ERR_INVALID_ARG;
  if (opt.side < 0 || opt.side > 2 || opt.prec < 0 || opt.prec > 2) return PSDP_ERR_INVALID_ARG;
  if (opt.max_iter < 1 || opt.certify < 0 || opt.certify > 1 || opt.expand_cols < 0 ||
      opt.batch_variant < -1)
    return PSDP_ERR_INVALID_ARG;
  if (opt.prec == PSDP_PREC_BF16) opt.prec = PSDP_PREC_FP32;
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > kBatchMaxN || m_cap[i] < 1) return PSDP_ERR_INVALID_ARG;
    if (m_inout[i] < 0 || m_inout[i] > m_cap[i]) return PSDP_ERR_INVALID_ARG;
    if (!X[i] || !V[i] || !lambda[i] || !Pi[i]) return PSDP_ERR_INVALID_ARG;
    if ((const void*)Pi[i] == (const void*)X[i]) return PSDP_ERR_INVALID_ARG;
  }
  if (hipSetDevice(h->device) != hipSuccess) return PSDP_ERR_HIP;
  if (!h->batch) h->batch = batch_engine_new(h->device);
  if (!h->batch) return PSDP_ERR_OUT_OF_MEMORY;
  h->calls += 1;
  psdp_status rc;
  size_t first = h->pending.size();
  {
    ProfScope pscope(h, "batched");
    rc = batch_engine_run(h->batch, h->stream, count, n, X, V, m_cap, m_inout, lambda, Pi, opt, info);
  }
  if (rc == PSDP_NOT_CONVERGED && opt.fallback_full) {
    // exact path for the cones the block solver did not converge
    std::vector<int> idx;
    for (int i = 0; i < count; ++i)
      if (info[i].status == PSDP_NOT_CONVERGED) idx.push_back(i);
    const int c = (int)idx.size();
    std::vector<int> fn(c), fcap(c), mo(c), np(c), bad(c);
    std::vector<const double*> fX(c);
    std::vector<double*> fV(c), fL(c), fP(c);
    for (int t = 0; t < c; ++t) {
      const int i = idx[t];
      fn[t] = n[i]; fcap[t] = m_cap[i]; fX[t] = X[i]; fV[t] = V[i]; fL[t] = lambda[i]; fP[t] = Pi[i];
    }
    psdp_status r2;
    {
      ProfScope pscope(h, "fulleig");
      r2 = full_eig_batched(h, c, fn.data(), fX.data(), fP.data(), fV.data(), fcap.data(), fL.data(),
                            mo.data(), np.data(), bad.data());
    }
    if (r2 != PSDP_OK) return r2;
    rc = PSDP_OK;
    for (int t = 0; t < c; ++t) {
      const int i = idx[t];
      const int iters = info[i].iters, exps = info[i].expansions;
      fill_full_info(&info[i], np[t], mo[t], bad[t]);
      info[i].iters = iters;
      info[i].expansions = exps;
      if (bad[t]) { rc = PSDP_ERR_NUMERICAL; continue; }
      info[i].status = PSDP_FELL_BACK_FULL_EIG;
      m_inout[i] = mo[t];
    }
    if (rc == PSDP_OK) {
      for (int i = 0; i < count; ++i) {
        if (info[i].status < 0) { rc = (psdp_status)std::min((int)rc, info[i].status); }
        else if (rc >= 0) rc = (psdp_status)std::max((int)rc, info[i].status);
      }
    }
  }
  if (h->prof && h->pending.size() > first) {
    // algorithmic traffic: X read, Pi written, V read and written; flops of
    // the iterations: product 2 n^2 (3m) + Gram/orthogonalization ~ 10 n (3m)^2
    double bytes = 0.0, flops = 0.0;
    for (int i = 0; i < count; ++i) {
      const double nn = n[i], mm = std::min(std::min(m_cap[i], kBatchMaxM), n[i]);
      bytes += 16.0 * nn * nn + 16.0 * nn * mm;
      flops += (double)std::max(info[i].iters, 0) * (6.0 * nn * nn * mm + 90.0 * nn * mm * mm);
    }
    h->pending.back().bytes = bytes;
    h->pending.back().flops = flops;
  }
  return rc;
}

namespace psdp {
namespace {
std::atomic<long long> g_d2h_copies{0}, g_d2h_bytes{0}, g_d2h_max{0};
}  // namespace

hipError_t copy_to_host(void* dst, const void* src, size_t bytes, hipStream_t s) {
  g_d2h_copies.fetch_add(1, std::memory_order_relaxed);
  g_d2h_bytes.fetch_add((long long)bytes, std::memory_order_relaxed);
  long long cur = g_d2h_max.load(std::memory_order_relaxed);
  while ((long long)bytes > cur &&
         !g_d2h_max.compare_exchange_weak(cur, (long long)bytes, std::memory_order_relaxed)) {
  }
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
}

int handle_device(psdp_handle h) { return h->device; }
hipStream_t handle_stream(psdp_handle h) { return h->stream; }

int block_need(int est, const psdp_options& opt) {
  return est + std::max(opt.block_guard, (int)std::ceil(0.2 * est));
}

int auto_side(int n, int pos_hint, int m_cap, const psdp_options& opt) {
  // paper §6: project through the side with fewer than threshold * n
  // eigenvalues; with no estimate, the full eig
  int side;
  if (pos_hint < 0) return PSDP_SIDE_FULL;
  if (pos_hint < opt.side_threshold * n) side = PSDP_SIDE_POS;
  else if (n - pos_hint < opt.side_threshold * n) side = PSDP_SIDE_NEG;
  else return PSDP_SIDE_FULL;
  // cost rule: the block the estimate needs must fit the capacity, and a
  // trial basis of 3m columns must stay well below n (paper §5.1: the
  // O(n^2 m) iteration only pays off for m << n)
  const int need = block_need(side == PSDP_SIDE_POS ? pos_hint : n - pos_hint, opt);
  if (need > std::min(m_cap, kMaxM) || 6 * need >= n) return PSDP_SIDE_FULL;
  return side;
}
}  // namespace psdp

extern "C" psdp_status psdp_transfer_stats(long long* copies, long long* bytes, long long* max_bytes,
                                           int reset) {
  if (copies) *copies = g_d2h_copies.load();
  if (bytes) *bytes = g_d2h_bytes.load();
  if (max_bytes) *max_bytes = g_d2h_max.load();
  if (reset) {
    g_d2h_copies = 0;
    g_d2h_bytes = 0;
    g_d2h_max = 0;
  }
  return PSDP_OK;
}

extern "C" psdp_status psdp_batched_tuning(psdp_handle h, int* variant, double* last_ms) {
  if (!h || !variant || !last_ms) return PSDP_ERR_INVALID_ARG;
  *variant = batch_engine_last_variant(h->batch);
  *last_ms = batch_engine_last_ms(h->batch);
  return PSDP_OK;
}

extern "C" psdp_status psdp_project(psdp_handle h, int n, const double* X, int ldx, double* V,
                                    int ldv, int m_cap, int* m_inout, double* lambda, double* Pi,
                                    int ldpi, const psdp_options* opt_in, psdp_info* info) {
  psdp_info dummy;
  if (!info) info = &dummy;
  fill_info_defaults(info);
  psdp_options opt;
  if (opt_in) opt = *opt_in; else psdp_default_options(&opt);
  // ---- validation (no launch before this point)
  if (!h || n < 1 || !X || !V || !m_inout || !lambda || !Pi) return PSDP_ERR_INVALID_ARG;
  if (ldx < n || ldv < n || ldpi < n || m_cap < 1) return PSDP_ERR_INVALID_ARG;
  if (*m_inout < 0 || *m_inout > m_cap) return PSDP_ERR_INVALID_ARG;
  if (opt.side < 0 || opt.side > 3 || opt.prec < 0 || opt.prec > 2) return PSDP_ERR_INVALID_ARG;
  if (opt.max_iter < 1 || opt.certify < 0 || opt.certify > 1 || !(opt.side_threshold > 0.0) ||
      opt.side_threshold > 0.5 || opt.expand_cols < 0 || opt.pos_hint > n ||
      !(opt.certify_delta >= 0.0) || opt.warm_side < 0 || opt.warm_side > 2 ||
      opt.method < PSDP_METHOD_LOBPCG || opt.method > PSDP_METHOD_CHEBYSHEV ||
      (opt.method == PSDP_METHOD_TOP_R && opt.method_param < 1) || opt.method_param < 0)
    return PSDP_ERR_INVALID_ARG;
  if ((const void*)Pi == (const void*)X) return PSDP_ERR_INVALID_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return PSDP_ERR_HIP;
  h->calls += 1;

  // ---- side (paper §6): fewer than threshold*n positive -> positive side
  int side = opt.side;
  if (side == PSDP_SIDE_AUTO) side = auto_side(n, opt.pos_hint, m_cap, opt);
  const int mcap = std::min(std::min(m_cap, kMaxM), n);
  if (side == PSDP_SIDE_FULL) {
    int mo = 0, npos = 0;
    psdp_status st = full_eig_core(h, n, X, ldx, nullptr, Pi, ldpi, V, ldv, m_cap, &mo, lambda, &npos);
    if (st != PSDP_OK) { info->status = st; return st; }
    *m_inout = mo;
    info->side_used = PSDP_SIDE_FULL;
    info->n_pos = npos;
    info->n_pos_full = npos;
    info->pos_est = npos;
    info->block_side = PSDP_SIDE_POS;
    info->m_out = mo;
    info->err_bound = 0.0;
    info->res_fro = 0.0;
    info->tail_est = 0.0;
    info->certified = 1;
    info->status = PSDP_FELL_BACK_FULL_EIG;
    return PSDP_FELL_BACK_FULL_EIG;
  }
  const double sign = (side == PSDP_SIDE_NEG) ? -1.0 : 1.0;
  // ---- block size; a warm block of the other side is not used
  int m_in = *m_inout;
  if (opt.warm_side != PSDP_SIDE_AUTO && opt.warm_side != side) m_in = 0;
  int m0 = m_in;
  if (m0 == 0) {
    int est = -1;
    if (opt.pos_hint >= 0) est = (side == PSDP_SIDE_POS) ? opt.pos_hint : n - opt.pos_hint;
    if (est >= 0) m0 = est + std::max(opt.block_guard, (int)std::ceil(0.2 * est));
    else m0 = std::max(8, opt.block_guard);
  }
  const bool top_r = opt.method == PSDP_METHOD_TOP_R;
  if (top_r) m0 = opt.method_param;  // the truncation width is the block
  m0 = std::max(1, std::min(m0, mcap));
  int prec0 = opt.prec;
  psdp_status ps = ensure_workspace(h, n, mcap, prec0);
  if (ps != PSDP_OK) { info->status = ps; return ps; }
  Workspace& w = h->ws;
  hipStream_t s = h->stream;
  // ---- ingest
  HIP_TRY(hipMemsetAsync(w.nonfinite, 0, sizeof(int), s));
  int nb = 0;
  {
    ProfScope pscope(h, "ingest", 8.0 * n * (double)n / 2 + (8.0 + product_elem_bytes(prec0)) * n * (double)n, 0);
    HIP_TRY(launch_ingest(X, ldx, n, sign, w.A64, w.L, w.L, w.Alp, prec0, w.fro_part, w.nonfinite, s, &nb));
    HIP_TRY(launch_reduce_sum(w.fro_part, nb, w.scal, s));
  }
  psdp_status pp = ensure_pinned(h, 64);
  if (pp != PSDP_OK) return pp;
  HIP_TRY(copy_to_host(h->h_pin, w.scal, sizeof(double), s));
  HIP_TRY(copy_to_host(h->h_pin + 1, w.nonfinite, sizeof(int), s));
  HIP_TRY(hipStreamSynchronize(s));
  double fro2 = h->h_pin[0];
  int nonfin = 0;
  std::memcpy(&nonfin, h->h_pin + 1, sizeof(int));
  if (nonfin || !std::isfinite(fro2)) { info->status = PSDP_ERR_NUMERICAL; return PSDP_ERR_NUMERICAL; }
  double tol = opt.tol > 0 ? opt.tol : 1e-8 * std::sqrt(fro2) / std::sqrt(2.0 * m0);
  if (tol <= 0) tol = 1e-300;
  // the Chebyshev variant's spectrum bound needs only the ingested A: it
  // runs on the second stream beside the first Rayleigh-Ritz step (queued
  // after that step's launches, which are on the critical path)
  AuxJoin aux_join{h};
  // ---- state init
  State& hs = *h->h_state;
  std::memset(&hs, 0, sizeof(State));
  hs.n = n;
  hs.tol = tol;
  hs.best_res = INFINITY;
  hs.last_npos = -1;
  hs.stall_window = (prec0 == 0) ? 30 : 8;
  hs.fixed_block = top_r ? 1 : 0;
  hs.fro2_x = fro2;
  HIP_TRY(hipMemcpyAsync(w.st, &hs, sizeof(State), hipMemcpyHostToDevice, s));
  // ---- start block: warm start columns, then seeded normals
  HIP_TRY(hipMemset2DAsync(w.X, sizeof(double) * w.L, 0, sizeof(double) * w.L, w.MC, s));
  if (m_in > 0) HIP_TRY(launch_copy_cols(V, ldv, w.X, w.L, n, std::min(m_in, m0), s));
  const uint64_t seed = opt.seed;
  uint64_t rng_stream = (h->calls << 8);
  if (m0 > m_in) HIP_TRY(launch_fill_normal(w.X, w.L, n, m_in, m0 - m_in, seed, rng_stream++, s));
  HIP_TRY(hipStreamSynchronize(s));

  Solver sv(h, n, top_r ? m0 : mcap);
  sv.m = m0;
  sv.has_p = 0;
  psdp_status rc = PSDP_OK;
  int expansions = 0;
  // initial Rayleigh-Ritz on span(X0) with an FP64 product (Alg. 3, first RR)
  for (int attempt = 0; attempt < 4; ++attempt) {
    int want = sv.m;
    if (attempt == 0 && opt.method == PSDP_METHOD_CHEBYSHEV) {
      Solver::Queued q;
      rc = sv.enqueue(kModeXOnly, 0, want, 0, 0, q);
      if (rc != PSDP_OK) { info->status = rc; return rc; }
      rc = lanczos_launch(h, n, prec0, 10, opt.seed, (h->calls << 8) | 0xFF);
      if (rc != PSDP_OK) { info->status = rc; return rc; }
      aux_join.pending = true;
      rc = sv.complete(q);
    } else {
      rc = sv.iterate(kModeXOnly, 0, want, 0);
    }
    if (rc != PSDP_OK) { info->status = rc; return rc; }
    if (sv.m >= std::min(m0, n)) break;
    // rank-deficient start: refill the missing columns with random ones
    int miss = m0 - sv.m;
    HIP_TRY(launch_fill_normal(w.X, w.L, n, sv.m, miss, seed, rng_stream++, s));
    sv.m = m0;
  }
  int phase = prec0;
  bool finished = false;
  bool converged = false;
  int fell_back = 0;
  if (opt.method == PSDP_METHOD_BLOCK_KRYLOV) {
    // Rayleigh-Ritz on span(X, AX) (one block Lanczos iteration from the
    // warm start), method_param times, and no convergence loop
    const int steps = std::max(1, opt.method_param);
    for (int i = 0; i < steps; ++i) {
      rc = sv.iterate(kModeXR, phase, sv.m, 0);
      if (rc != PSDP_OK) { info->status = rc; return rc; }
      const int stp = h->h_state->stop;
      if (stp == kNonFinite) { info->status = PSDP_ERR_NUMERICAL; return PSDP_ERR_NUMERICAL; }
      if (stp == kConverged) converged = true;
      if (stp != kRunning) break;  // converged (or stopped) before the step
      sv.has_p = 0;
    }
    finished = true;
  }
  int cheb_passes = 0, cheb_products = 0;
  double cheb_lo = NAN;
  int pre_cert = -1;  // certificate already run on the final block: its result
  CertState pre_cs{};
  if (opt.method == PSDP_METHOD_CHEBYSHEV) {
    // Chebyshev-filtered subspace iteration: X <- T_d((A - c) / e) X with the
    // interval [lo, theta_m] (the spectrum's lower end to the smallest Ritz
    // value of the block) damped to |T_d| <= 1 and the positive Ritz values
    // amplified by T_d at their scaled position, then Rayleigh-Ritz on
    // span(X) with an FP64 product; repeated until the stopping rule holds.
    double thmin = 0.0;
    rc = lanczos_finish(h, &cheb_lo, &thmin);
    aux_join.pending = false;
    if (rc != PSDP_OK) { info->status = rc; return rc; }
    cheb_lo -= 1e-2 * std::fabs(cheb_lo);  // margin for the rounding of the bound
    cheb_products += 10;
    const int dmax = opt.method_param > 0 ? std::min(opt.method_param, 64) : 24;
    // a pass applies a whole polynomial: max_iter passes, at most 40; and
    // after three certificates failed on blocks that met the stopping rule
    // the positive eigenvalues outside the block are taken as out of reach
    // (eigenvalues clustered at zero): not converged
    const int max_pass = std::max(1, std::min(opt.max_iter, 40));
    int cert_fail = 0;
    const int L = w.L;
    for (;;) {
      rc = sv.evaluate();
      if (rc != PSDP_OK) { info->status = rc; return rc; }
      const State& st = *h->h_state;
      const int ev = st.eval_stop;
      if (ev == kNonFinite) { info->status = PSDP_ERR_NUMERICAL; return PSDP_ERR_NUMERICAL; }
      const int m = sv.m, np = st.npos_blk;
      bool expand = np >= m || ev == kExpand;
      if (ev == kConverged) {
        // the stopping rule judges the guard pair against half its gap to
        // the smallest positive Ritz value, which a block still far from the
        // top of the spectrum can meet: with the certificate on, it decides
        if (!opt.certify || np >= n) { converged = true; break; }
        const double delta = opt.certify_delta > 0.0
                                 ? opt.certify_delta
                                 : std::sqrt(2.0 * std::max(np, 1)) * tol / std::sqrt((double)n);
        rc = run_certificate(h, n, np, fro2, delta, &pre_cert, &pre_cs);
        if (rc != PSDP_OK) { info->status = rc; return rc; }
        if (pre_cert) { converged = true; break; }
        pre_cert = -1;  // a positive eigenvalue outside the block: filter on
        if (++cert_fail >= 3) break;
      }
      if (expand) {
        // no non-positive Ritz pair left in the block: append columns
        int e = opt.expand_cols > 0 ? opt.expand_cols : (n + 49) / 50;
        e = std::min(std::max(1, e), sv.mcap - sv.m);
        if (e <= 0) {
          if (opt.fallback_full) fell_back = 1;
          break;
        }
        HIP_TRY(launch_fill_normal(w.Z, L, n, 0, e, seed, rng_stream++, s));
        rc = sv.iterate(kModeXZ, 0, sv.m + e, e);
        if (rc != PSDP_OK) { info->status = rc; return rc; }
        sv.has_p = 0;
        cheb_products += 1;
        expansions += 1;
        continue;
      }
      if (cheb_passes >= max_pass) break;
      ++cheb_passes;
      // filter degree: enough to bring the largest positive residual below
      // tol (with a factor 4 in hand) at the smallest positive Ritz value's
      // amplification, at most dmax, and with the amplification of the top
      // of the spectrum at most R times that of the smallest positive value,
      // so that the filtered columns stay numerically independent: a column
      // with residual r has components of at most r / (theta_0 - theta_m)
      // along the top eigenvectors, which the filter multiplies by R
      // relative to its own, so R = 1e6 (theta_0 - theta_m) / max r (that
      // bound is far above the components Ritz vectors carry in practice),
      // kept within [1e5, 1e13] (rounding of the products bounds it above);
      // columns that still come out dependent are dropped by the
      // Cholesky-QR and replaced
      const double b = st.theta[m - 1];
      const double a = std::min(cheb_lo, b - 1e-3 * std::max(std::fabs(b), 1e-300));
      const double c = 0.5 * (a + b), e = 0.5 * (b - a);
      const double thp = np > 0 ? st.theta[np - 1] : st.theta[0];
      const double xp = std::max((thp - c) / e, 1.0 + 1e-12);
      const double xmax = std::max((st.theta[0] + st.res_max_pos - c) / e, xp);
      double ratio = st.res_max_pos / tol;
      if (np < m && std::isfinite(st.guard_res)) {
        const double gap = np > 0 ? st.theta[np - 1] - st.guard_theta : std::fabs(st.guard_theta);
        ratio = std::max(ratio, st.guard_res / std::max(tol, 0.5 * gap));
      }
      const double need = 4.0 * std::max(ratio, 2.0);
      const double ap = std::acosh(xp);
      int d = (int)std::ceil(std::acosh(need) / ap);
      const double spread = std::acosh(xmax) - ap;
      double rall = 0.0, rg = 0.0;
      for (int i = 0; i < m; ++i) rall = std::max(rall, st.rnorm[i]);
      for (int i = np; i < m; ++i) rg = std::max(rg, st.rnorm[i]);
      const double R = std::min(1e13, std::max(1e5, 1e6 * (st.theta[0] - b) / std::max(rall, 1e-300)));
      if (spread > 0) d = std::min(d, (int)(std::log(R) / spread));
      // the non-positive (guard) columns sit in the damped interval, so the
      // filter leaves their own direction at most 1 while it multiplies their
      // components along the top eigenvectors, at most r_g / (theta_0 -
      // theta_g), by T_d(x_max).  Past some level the Cholesky-QR drops the
      // guards as dependent, and the random columns that replace them cost a
      // Rayleigh-Ritz pass and spoil the next call's warm start (its damped
      // interval then ends at their Ritz values, far below zero).  The bound
      // overstates the components; guards were kept at a bound of 3.5e9 and
      // dropped at 1.2e12, so it is held to 1e10.
      if (np > 0 && np < m && rg > 0.0) {
        const double gapg = st.theta[0] - st.theta[np];
        const double amax = std::acosh(xmax);
        if (gapg > 0.0 && amax > 0.0)
          d = std::min(d, (int)(std::log(2e10 * gapg / rg) / amax));
      }
      d = std::max(2, std::min(d, dmax));
      // Y0 = X, Y1 = (AX - c X) / e (AX exact from the last Rayleigh-Ritz),
      // Y_{k+1} = 2 (A Y_k - c Y_k) / e - Y_{k-1} through the product epilogue
      double* yb[3] = {w.X, w.R, w.P};
      {
        ProfScope ps(h, "tsmm", 24.0 * n * (double)m, 3.0 * n * (double)m);
        HIP_TRY(launch_axpby3(n, m, 1.0 / e, w.AX, L, -c / e, w.X, L, 0.0, nullptr, L, w.R, L, s));
      }
      // product precision of the pass: the low-precision copy of A while the
      // largest residual is above ten times that precision's rounding floor
      // (about 8 u_p ||A||_F / sqrt(n) per unit column, as for the LOBPCG
      // ladder), FP64 otherwise; the Rayleigh-Ritz after it is FP64
      int fprec = 0;
      if (prec0 != 0) {
        const double up = prec0 == 2 ? 3.9e-3 : 6.0e-8;
        if (st.res_max_pos > 10.0 * 8.0 * up * std::sqrt(fro2 / (double)n)) fprec = prec0;
      }
      int i0 = 0, i1 = 1;
      for (int k = 2; k <= d; ++k) {
        const int i2 = 3 - i0 - i1;
        ProfScope ps(h, "product", (double)product_elem_bytes(fprec) * n * (double)n + 40.0 * n * m,
                     2.0 * n * (double)n * m, fprec);
        ProductArgs pa{};
        pa.A = fprec == 0 ? (const void*)w.A64 : w.Alp; pa.lda = L; pa.n = n; pa.prec = fprec;
        pa.S = yb[i1]; pa.lds = L; pa.Y = yb[i2]; pa.ldy = L;
        pa.cols_dev = nullptr; pa.cols_max = m; pa.stop = nullptr;
        pa.partial = w.ppart; pa.partial_bytes = w.ppart_bytes; pa.max_slices = kProductSlices;
        pa.comb.b1 = yb[i1]; pa.comb.b0 = yb[i0]; pa.comb.ld = L;
        pa.comb.ca = 2.0 / e; pa.comb.cb = -2.0 * c / e; pa.comb.cc = -1.0;
        HIP_TRY(launch_product(pa, s));
        i0 = i1;
        i1 = i2;
      }
      cheb_products += d - 1;
      if (i1 != 0) HIP_TRY(launch_copy_cols(yb[i1], L, w.X, L, n, m, s));
      if (h->trace)
        std::fprintf(stderr, "psdp: chebyshev pass %d degree %d interval [%.4e, %.4e] xp %.6f "
                     "rmax %.3e tol %.3e npos %d m %d prec %d\n", cheb_passes, d, a, b, xp,
                     st.res_max_pos, tol, np, m, fprec);
      // Rayleigh-Ritz on span(X); columns the Cholesky-QR drops as dependent
      // are replaced by seeded random ones
      sv.has_p = 0;
      for (int attempt = 0; attempt < 4; ++attempt) {
        rc = sv.iterate(kModeXOnly, 0, m, 0);
        if (rc != PSDP_OK) { info->status = rc; return rc; }
        cheb_products += 1;
        if (sv.m >= m) break;
        HIP_TRY(launch_fill_normal(w.X, L, n, sv.m, m - sv.m, seed, rng_stream++, s));
        sv.m = m;
      }
    }
    finished = true;
  }
  auto refresh = [&](int pprec) -> psdp_status {
    // Rayleigh-Ritz on span(X) with a fresh product: exact AX at pprec
    psdp_status r = sv.iterate(kModeXOnly, pprec, sv.m, 0);
    sv.has_p = 0;
    hs.best_res = INFINITY;
    return r;
  };
  auto reset_stall = [&]() -> psdp_status {
    State tmp = *h->h_state;
    (void)tmp;
    // best_res / best_iter live on the device: reset them in place
    double inf = INFINITY;
    HIP_TRY(hipMemcpyAsync(&w.st->best_res, &inf, sizeof(double), hipMemcpyHostToDevice, s));
    int it = h->h_state->iter;
    HIP_TRY(hipMemcpyAsync(&w.st->best_iter, &it, sizeof(int), hipMemcpyHostToDevice, s));
    int win = (phase == 0) ? 30 : 8;
    HIP_TRY(hipMemcpyAsync(&w.st->stall_window, &win, sizeof(int), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PSDP_OK;
  };
  int guard_calls = 0;
  // The loop keeps one iteration queued ahead: while the host reads back
  // iteration t, iteration t + 1 (full trial basis, same block size and
  // product precision) is already on the stream.  Its decision kernel makes
  // it a no-op when t stopped or changed the block size; the host then drops
  // it (and after a size change clears the abort flag).
  Solver::Queued cur, nxt;
  bool have_cur = false;
  auto drop_next = [&](bool have, const Solver::Queued& q, bool clear_abort) -> psdp_status {
    if (!have) return PSDP_OK;
    sv.discard(q);
    if (clear_abort) HIP_TRY(launch_set_stop(w.st, kRunning, s));
    return PSDP_OK;
  };
  while (!finished) {
    if (++guard_calls > 4 * opt.max_iter + 64) break;  // hard bound on host steps
    if (!have_cur) {
      int mode = sv.has_p ? kModeFull : kModeXR;
      rc = sv.enqueue(mode, phase, sv.m, 0, 0, cur);
      if (rc != PSDP_OK) { info->status = rc; return rc; }
    }
    have_cur = false;
    // h_state is still the snapshot before `cur`: two more iterations fit
    bool have_nxt = false;
    if (h->h_state->iter + 2 <= opt.max_iter) {
      rc = sv.enqueue(kModeFull, phase, sv.m, 0, sv.m, nxt);
      if (rc != PSDP_OK) { info->status = rc; return rc; }
      have_nxt = true;
    }
    rc = sv.complete(cur);
    if (rc != PSDP_OK) { info->status = rc; return rc; }
    const State& st = *h->h_state;
    int stop = st.stop;
    if (stop != kRunning) {
      // the queued iteration found `stop` set and did nothing
      drop_next(have_nxt, nxt, false);
      have_nxt = false;
    }
    if (stop == kNonFinite) { info->status = PSDP_ERR_NUMERICAL; return PSDP_ERR_NUMERICAL; }
    if (stop == kBreakdown) {
      if (opt.fallback_full) { fell_back = 1; break; }
      info->status = PSDP_ERR_NUMERICAL;
      return PSDP_ERR_NUMERICAL;
    }
    if (stop == kConverged) {
      if (phase != 0 && opt.refine_fp64) {
        // FP64 residual-correction: exact AX, then keep iterating in FP64
        // until the exact residuals meet tol
        phase = 0;
        rc = refresh(0);
        if (rc != PSDP_OK) return rc;
        rc = reset_stall();
        continue;
      }
      converged = true;
      finished = true;
      break;
    }
    if (stop == kStalled) {
      if (phase == 2 && opt.ladder) {
        phase = 1;
        // the low-precision copy of A holds BF16: convert it to FP32 again
        int nb2 = 0;
        HIP_TRY(launch_ingest(X, ldx, n, sign, w.A64, w.L, w.L, w.Alp, 1, w.fro_part, w.nonfinite,
                              s, &nb2));
        if ((rc = refresh(1)) != PSDP_OK) return rc;
        reset_stall();
        continue;
      }
      if (phase != 0 && (opt.ladder || opt.refine_fp64)) {
        phase = 0;
        if ((rc = refresh(0)) != PSDP_OK) return rc;
        reset_stall();
        if (!opt.ladder) {
          // raw low-precision path: one FP64 sweep then stop
          rc = sv.iterate(kModeXR, 0, sv.m, 0);
          if (rc != PSDP_OK) return rc;
          rc = refresh(0);
          if (rc != PSDP_OK) return rc;
          finished = true;
          break;
        }
        continue;
      }
      finished = true;  // stalled at FP64
      break;
    }
    if (stop == kExpand) {
      int e = opt.expand_cols > 0 ? opt.expand_cols : (n + 49) / 50;
      e = std::max(1, e);
      e = std::min(e, sv.mcap - sv.m);
      if (e <= 0) {
        if (opt.fallback_full) { fell_back = 1; break; }
        // no room: report what we have
        finished = true;
        break;
      }
      HIP_TRY(launch_fill_normal(w.Z, w.L, n, 0, e, seed, rng_stream++, s));
      rc = sv.iterate(kModeXZ, phase, sv.m + e, e);
      if (rc != PSDP_OK) return rc;
      sv.has_p = 0;
      expansions += 1;
      reset_stall();
      continue;
    }
    if (st.iter >= opt.max_iter) {
      drop_next(have_nxt, nxt, true);
      finished = true;
      break;
    }
    if (have_nxt) {
      if (sv.m == nxt.spec_m && sv.has_p) {
        cur = nxt;  // the queued iteration is the next one
        have_cur = true;
      } else {
        drop_next(true, nxt, true);  // it aborted on the block size
      }
    }
  }
  // the exact path in place of the LOBPCG result
  auto full_instead = [&]() -> psdp_status {
    int mo = 0, npos = 0;
    psdp_status st2 = full_eig_core(h, n, X, ldx, nullptr, Pi, ldpi, V, ldv, m_cap, &mo, lambda, &npos);
    if (st2 != PSDP_OK) { info->status = st2; return st2; }
    *m_inout = mo;
    info->side_used = PSDP_SIDE_FULL;
    info->n_pos = npos;
    info->n_pos_full = npos;
    info->pos_est = npos;
    info->block_side = PSDP_SIDE_POS;
    info->m_out = mo;
    info->err_bound = 0.0; info->res_fro = 0.0; info->tail_est = 0.0;
    info->certified = 1;
    info->iters = h->h_state->iter;
    info->expansions = expansions;
    info->status = PSDP_FELL_BACK_FULL_EIG;
    return PSDP_FELL_BACK_FULL_EIG;
  };
  if (fell_back || (!converged && opt.fallback_full)) return full_instead();
  if (!converged && phase != 0 && opt.refine_fp64) {
    // not converged at a low precision: still finish with exact FP64 pairs
    phase = 0;
    if ((rc = refresh(0)) != PSDP_OK) return rc;
    rc = sv.iterate(kModeXR, 0, sv.m, 0);  // one FP64 sweep on span(X, R)
    if (rc != PSDP_OK) return rc;
    converged = (h->h_state->stop == kConverged);
  }
  // ---- statistics of the final block (exact FP64 residuals)
  if (h->h_state->stop != kConverged) {
    rc = sv.evaluate();
    if (rc != PSDP_OK) return rc;
    converged = converged || (h->h_state->eval_stop == kConverged);
  }
  // ---- bound (Thm `bound`) from the last decision pass
  const State& st = *h->h_state;
  const int m = sv.m;
  int npos = st.npos_blk;
  double rfro = st.res_fro_pos;
  // tail term ||Pi(Vt_perp^T A Vt_perp)||_F
  double tail = 0.0;
  int certified = 0;
  double cert_delta = NAN, cert_eta = NAN;
  if (npos >= n) {
    certified = 1;  // Vt spans the whole space: no complement
  } else if (opt.certify) {
    const double delta = opt.certify_delta > 0.0
                             ? opt.certify_delta
                             : std::sqrt(2.0 * std::max(npos, 1)) * tol / std::sqrt((double)n);
    CertState cs{};
    if (pre_cert >= 0) {
      certified = pre_cert;  // the filtered iteration's stopping test ran it on this block
      cs = pre_cs;
    } else {
      rc = run_certificate(h, n, npos, fro2, delta, &certified, &cs);
      if (rc != PSDP_OK) { info->status = rc; return rc; }
    }
    cert_delta = cs.delta_eff;
    cert_eta = cs.eta;
    if (certified) tail = std::sqrt((double)(n - npos)) * cert_delta;
  }
  if (!certified && npos < n) {
    if (opt.certify) {
      tail = INFINITY;  // the certificate failed: the tail term is not bounded
    } else if (npos < m) {
      // estimate from the largest non-positive Ritz pair: its value plus its
      // residual norm (an eigenvalue lies within r_g of theta_g)
      tail = std::sqrt((double)(n - npos)) * std::max(st.guard_theta + st.guard_res, 0.0);
    } else {
      tail = INFINITY;  // no non-positive pair in the block to estimate from
    }
  }
  // a certificate that was asked for and failed: positive eigenvalues of the
  // complement may exceed the threshold, so the result is not converged
  if (opt.certify && !certified && !top_r) {
    converged = false;
    if (opt.fallback_full) return full_instead();
  }
  double bound = std::sqrt(2.0 * rfro * rfro + tail * tail);
  double sum_pos2 = 0.0;
  for (int i = 0; i < npos; ++i) sum_pos2 += st.theta[i] * st.theta[i];
  double pi_fro = (side == PSDP_SIDE_POS) ? std::sqrt(sum_pos2) : std::sqrt(std::max(fro2 - sum_pos2, 0.0));
  // a bound above the caller's target: the exact path instead (not-a-number
  // bounds included)
  if (opt.fallback_full && opt.bound_rel_max > 0.0 && !(bound <= opt.bound_rel_max * pi_fro))
    return full_instead();
  // ---- rebuild Pi
  {
    ProfScope pscope(h, "rebuild", 8.0 * n * (double)n * (side == PSDP_SIDE_NEG ? 2 : 1),
                     (double)n * n * npos);
    const double* lt = &w.st->theta[0];
    if (side == PSDP_SIDE_POS)
      HIP_TRY(launch_rebuild(w.X, w.L, lt, npos, n, nullptr, 0, 0.0, Pi, ldpi, s));
    else
      HIP_TRY(launch_rebuild(w.X, w.L, lt, npos, n, w.A64, w.L, -1.0, Pi, ldpi, s));
  }
  // ---- outputs: Ritz block and values
  HIP_TRY(launch_copy_cols(w.X, w.L, V, ldv, n, m, s));
  HIP_TRY(hipMemcpyAsync(lambda, &w.st->theta[0], sizeof(double) * m, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  *m_inout = m;
  info->err_bound = bound;
  info->res_fro = rfro;
  info->tail_est = tail;
  info->pi_fro = pi_fro;
  info->theta_guard = st.guard_theta;
  info->tol_used = tol;
  info->n_pos = npos;
  info->m_out = m;
  info->iters = st.iter;
  info->side_used = side;
  info->certified = certified;
  info->cert_delta = cert_delta;
  info->cert_eta = cert_eta;
  info->pos_est = (side == PSDP_SIDE_POS) ? npos : n - npos;
  info->block_side = side;
  if (top_r)
    info->trunc_bound = std::sqrt((double)std::max(n - m, 0)) * std::max(st.theta[m - 1], 0.0);
  if (opt.method == PSDP_METHOD_CHEBYSHEV) {
    info->iters = cheb_passes;
    info->products = cheb_products;
    info->spec_lower = cheb_lo;
  }
  info->expansions = expansions;
  info->prec_final = phase;
  info->status = converged ? PSDP_OK : PSDP_NOT_CONVERGED;
  return (psdp_status)info->status;
}
