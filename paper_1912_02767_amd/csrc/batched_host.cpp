// Host side of the batched persistent engine: queue construction (cones in
// decreasing order of work), scratch sizing, the launch-shape autotuner,
// and hipGraph capture/replay of the launch sequence.
//
// Launch shapes ("variants") differ in the Rayleigh-Ritz storage (full
// square matrix in LDS, one workgroup per CU; or packed triangle, two
// workgroups per CU) and in the k-chunk of the workgroup GEMM.  The first
// call for a batch signature times every variant that fits the device on
// the caller's inputs (results go to internal buffers, so warm starts are
// left untouched) and keeps the fastest; PSDP_TUNE_FILE, when set, names a
// text file that stores and reloads these choices across processes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/psdp.h"
#include "batched.h"
#include "internal.h"

namespace psdp {

struct BatchVariant {
  bool rr_full;
  int wg_per_cu;
  int kc;
};

static const BatchVariant kVariants[] = {
    {true, 1, 16},
    {true, 1, 32},
    {false, 2, 16},
    {false, 2, 8},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

struct BatchEngine {
  int device = 0;
  int cus = 256;
  size_t lds_block = 65536, lds_cu = 65536, lds_static = 4096;
  hipStream_t cap_stream = nullptr;
  BatchCone* d_cones = nullptr;
  BatchOut* d_outs = nullptr;
  int* d_counter = nullptr;
  int cap = 0;
  BatchCone* h_cones = nullptr;
  BatchOut* h_outs = nullptr;
  char* d_scratch = nullptr;
  size_t scratch_bytes = 0;
  double* d_tune = nullptr;  // outputs of tuning runs
  size_t tune_bytes = 0;
  hipGraphExec_t exec = nullptr;
  std::vector<char> exec_key;
  std::map<std::string, int> tuned;
  bool tune_loaded = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0.0;
  int last_variant = -1;
};

#define BT_TRY(expr)                               \
  do {                                             \
    hipError_t _e = (expr);                        \
    if (_e != hipSuccess) return PSDP_ERR_HIP;     \
  } while (0)

BatchEngine* batch_engine_new(int device) {
  BatchEngine* e = new BatchEngine();
  e->device = device;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && v > 0)
    e->cus = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && v > 0)
    e->lds_block = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) ==
          hipSuccess && v > 0)
    e->lds_cu = v;
  else
    e->lds_cu = e->lds_block;
  e->lds_static = batched_static_lds_bytes();
  (void)batched_init((int)(e->lds_block - e->lds_static));
  (void)hipGetLastError();
  return e;
}

void batch_engine_free(BatchEngine* e) {
  if (!e) return;
  if (e->exec) (void)hipGraphExecDestroy(e->exec);
  if (e->cap_stream) (void)hipStreamDestroy(e->cap_stream);
  if (e->d_cones) (void)hipFree(e->d_cones);
  if (e->d_outs) (void)hipFree(e->d_outs);
  if (e->d_counter) (void)hipFree(e->d_counter);
  if (e->d_scratch) (void)hipFree(e->d_scratch);
  if (e->d_tune) (void)hipFree(e->d_tune);
  if (e->h_cones) (void)hipHostFree(e->h_cones);
  if (e->h_outs) (void)hipHostFree(e->h_outs);
  if (e->ev0) (void)hipEventDestroy(e->ev0);
  if (e->ev1) (void)hipEventDestroy(e->ev1);
  delete e;
}

double batch_engine_last_ms(const BatchEngine* e) { return e ? e->last_ms : 0.0; }
int batch_engine_last_variant(const BatchEngine* e) { return e ? e->last_variant : -1; }

// dynamic LDS bytes of a variant, or 0 when it does not fit the device
static size_t variant_lds(const BatchEngine* e, const BatchVariant& v, int mmax) {
  const size_t dyn = 8 * batched_lds_doubles(mmax, v.rr_full, v.kc);
  if (dyn + e->lds_static > e->lds_block) return 0;
  if ((size_t)v.wg_per_cu * (dyn + e->lds_static) > e->lds_cu) return 0;
  return dyn;
}

static psdp_status ensure_queue(BatchEngine* e, int count) {
  if (count <= e->cap) return PSDP_OK;
  if (e->d_cones) (void)hipFree(e->d_cones);
  if (e->d_outs) (void)hipFree(e->d_outs);
  if (e->h_cones) (void)hipHostFree(e->h_cones);
  if (e->h_outs) (void)hipHostFree(e->h_outs);
  e->d_cones = nullptr; e->d_outs = nullptr; e->h_cones = nullptr; e->h_outs = nullptr;
  e->cap = 0;
  if (e->exec) { (void)hipGraphExecDestroy(e->exec); e->exec = nullptr; e->exec_key.clear(); }
  const int c = std::max(count, 64);
  if (hipMalloc(&e->d_cones, sizeof(BatchCone) * c) != hipSuccess) return PSDP_ERR_OUT_OF_MEMORY;
  if (hipMalloc(&e->d_outs, sizeof(BatchOut) * c) != hipSuccess) return PSDP_ERR_OUT_OF_MEMORY;
  if (hipHostMalloc((void**)&e->h_cones, sizeof(BatchCone) * c, hipHostMallocDefault) != hipSuccess)
    return PSDP_ERR_OUT_OF_MEMORY;
  if (hipHostMalloc((void**)&e->h_outs, sizeof(BatchOut) * c, hipHostMallocDefault) != hipSuccess)
    return PSDP_ERR_OUT_OF_MEMORY;
  if (!e->d_counter && hipMalloc(&e->d_counter, 256) != hipSuccess) return PSDP_ERR_OUT_OF_MEMORY;
  e->cap = c;
  return PSDP_OK;
}

static psdp_status ensure_scratch(BatchEngine* e, size_t bytes, hipStream_t s) {
  if (bytes <= e->scratch_bytes) return PSDP_OK;
  (void)hipStreamSynchronize(s);
  if (e->d_scratch) (void)hipFree(e->d_scratch);
  e->d_scratch = nullptr;
  e->scratch_bytes = 0;
  if (e->exec) { (void)hipGraphExecDestroy(e->exec); e->exec = nullptr; e->exec_key.clear(); }
  if (hipMalloc(&e->d_scratch, bytes) != hipSuccess) return PSDP_ERR_OUT_OF_MEMORY;
  e->scratch_bytes = bytes;
  return PSDP_OK;
}

// ---------------------------------------------------------- tune file ----
static void tune_load(BatchEngine* e) {
  if (e->tune_loaded) return;
  e->tune_loaded = true;
  const char* path = std::getenv("PSDP_TUNE_FILE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char key[256];
  int v = -1;
  while (std::fscanf(f, "%255s %d", key, &v) == 2)
    if (v >= 0 && v < kNumVariants) e->tuned[key] = v;
  std::fclose(f);
}

static void tune_store(BatchEngine* e, const std::string& key, int v) {
  e->tuned[key] = v;
  const char* path = std::getenv("PSDP_TUNE_FILE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d\n", key.c_str(), v);
  std::fclose(f);
}

static std::string tune_key(int nmax, int mmax, int count, int prec, int cus) {
  int cb = 1;
  while (cb < count) cb <<= 1;
  char buf[128];
  std::snprintf(buf, sizeof buf, "cu%d_n%d_m%d_c%d_p%d", cus, (nmax + 31) / 32 * 32, mmax, cb, prec);
  return buf;
}

// --------------------------------------------------------------- launch ---
static psdp_status run_variant(BatchEngine* e, BatchArgs a, int vi, int count, bool use_graph,
                               hipStream_t s, float* ms) {
  const BatchVariant& v = kVariants[vi];
  a.kc = v.kc;
  a.lds_doubles = variant_lds(e, v, a.mmax) / 8;
  const int grid = std::max(1, std::min(count, e->cus * v.wg_per_cu));
  const size_t stride = batched_scratch_bytes(a.nmax, a.mmax);
  psdp_status ps = ensure_scratch(e, stride * grid, s);
  if (ps != PSDP_OK) return ps;
  a.scratch = e->d_scratch;
  a.scratch_stride = stride;
  if (!e->ev0) BT_TRY(hipEventCreate(&e->ev0));
  if (!e->ev1) BT_TRY(hipEventCreate(&e->ev1));
  BT_TRY(hipEventRecord(e->ev0, s));
  if (use_graph) {
    std::vector<char> key(sizeof(BatchArgs) + 2 * sizeof(int));
    std::memcpy(key.data(), &a, sizeof(BatchArgs));
    std::memcpy(key.data() + sizeof(BatchArgs), &vi, sizeof(int));
    std::memcpy(key.data() + sizeof(BatchArgs) + sizeof(int), &grid, sizeof(int));
    if (!e->exec || key != e->exec_key) {
      if (e->exec) { (void)hipGraphExecDestroy(e->exec); e->exec = nullptr; }
      if (!e->cap_stream) BT_TRY(hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      BT_TRY(hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t le = launch_batched(a, v.rr_full, grid, e->cap_stream);
      hipError_t ce = hipStreamEndCapture(e->cap_stream, &g);
      if (le != hipSuccess || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return PSDP_ERR_HIP;
      }
      hipError_t ie = hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) { e->exec = nullptr; return PSDP_ERR_HIP; }
      e->exec_key = key;
    }
    BT_TRY(hipGraphLaunch(e->exec, s));
  } else {
    BT_TRY(launch_batched(a, v.rr_full, grid, s));
  }
  BT_TRY(hipEventRecord(e->ev1, s));
  if (ms) {
    BT_TRY(hipEventSynchronize(e->ev1));
    BT_TRY(hipEventElapsedTime(ms, e->ev0, e->ev1));
  }
  return PSDP_OK;
}

psdp_status batch_engine_run(BatchEngine* e, hipStream_t s, int count, const int* n,
                             const double* const* X, double* const* V, const int* m_cap,
                             int* m_inout, double* const* lambda, double* const* Pi,
                             const psdp_options& opt, psdp_info* info) {
  if (hipSetDevice(e->device) != hipSuccess) return PSDP_ERR_HIP;
  psdp_status ps = ensure_queue(e, count);
  if (ps != PSDP_OK) return ps;
  // queue order: decreasing n^2 m (the larger cones start first)
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  auto work = [&](int i) { return (double)n[i] * n[i] * std::min(m_cap[i], kBatchMaxM); };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
  int nmax = 1, mmax = 1;
  const double sign = (opt.side == PSDP_SIDE_NEG) ? -1.0 : 1.0;
  for (int q = 0; q < count; ++q) {
    const int i = order[q];
    BatchCone c{};
    c.n = n[i];
    c.m_cap = std::min(std::min(m_cap[i], kBatchMaxM), n[i]);
    c.m_in = std::min(m_inout[i], c.m_cap);
    c.index = i;
    c.sign = sign;
    c.X = X[i];
    c.V_in = V[i];
    c.V_out = V[i];
    c.lam = lambda[i];
    c.Pi = Pi[i];
    e->h_cones[q] = c;
    nmax = std::max(nmax, c.n);
    mmax = std::max(mmax, c.m_cap);
  }
  BatchArgs a{};
  a.cones = e->d_cones;
  a.outs = e->d_outs;
  a.count = count;
  a.counter = e->d_counter;
  a.nmax = nmax;
  a.mmax = mmax;
  a.prec = opt.prec == PSDP_PREC_FP64 ? 0 : 1;
  a.tol = opt.tol;
  a.max_iter = opt.max_iter;
  a.seed = opt.seed;
  a.expand_cols = opt.expand_cols;

  // ---- launch shape: forced, cached, or tuned now
  int vi = opt.batch_variant;
  if (vi >= 0 && (vi >= kNumVariants || variant_lds(e, kVariants[vi], mmax) == 0))
    return PSDP_ERR_INVALID_ARG;
  if (vi < 0) {
    tune_load(e);
    const std::string key = tune_key(nmax, mmax, count, a.prec, e->cus);
    auto it = e->tuned.find(key);
    if (it != e->tuned.end() && variant_lds(e, kVariants[it->second], mmax) > 0) {
      vi = it->second;
    } else {
      // time every fitting variant on these inputs, outputs redirected
      size_t need = 0;
      for (int q = 0; q < count; ++q) {
        const BatchCone& c = e->h_cones[q];
        need += (size_t)c.n * c.n + (size_t)c.n * c.m_cap + c.m_cap;
      }
      if (need * 8 > e->tune_bytes) {
        (void)hipStreamSynchronize(s);
        if (e->d_tune) (void)hipFree(e->d_tune);
        e->d_tune = nullptr;
        e->tune_bytes = 0;
        if (hipMalloc(&e->d_tune, need * 8) != hipSuccess) return PSDP_ERR_OUT_OF_MEMORY;
        e->tune_bytes = need * 8;
      }
      std::vector<BatchCone> real(e->h_cones, e->h_cones + count);
      double* p = e->d_tune;
      for (int q = 0; q < count; ++q) {
        BatchCone& c = e->h_cones[q];
        c.Pi = p; p += (size_t)c.n * c.n;
        c.V_out = p; p += (size_t)c.n * c.m_cap;
        c.lam = p; p += c.m_cap;
      }
      BT_TRY(hipMemcpyAsync(e->d_cones, e->h_cones, sizeof(BatchCone) * count,
                            hipMemcpyHostToDevice, s));
      float best = INFINITY;
      int bi = -1;
      for (int v = 0; v < kNumVariants; ++v) {
        if (variant_lds(e, kVariants[v], mmax) == 0) continue;
        float ms = 0.f;
        ps = run_variant(e, a, v, count, false, s, &ms);
        if (ps != PSDP_OK) return ps;
        if (ms < best) { best = ms; bi = v; }
      }
      if (bi < 0) return PSDP_ERR_CAPACITY;
      std::copy(real.begin(), real.end(), e->h_cones);
      vi = bi;
      tune_store(e, key, vi);
    }
  }
  BT_TRY(hipMemcpyAsync(e->d_cones, e->h_cones, sizeof(BatchCone) * count, hipMemcpyHostToDevice, s));
  float ms = 0.f;
  ps = run_variant(e, a, vi, count, opt.batch_graph != 0, s, &ms);
  if (ps != PSDP_OK) return ps;
  e->last_ms = ms;
  e->last_variant = vi;
  BT_TRY(copy_to_host(e->h_outs, e->d_outs, sizeof(BatchOut) * count, s));
  BT_TRY(hipStreamSynchronize(s));
  int worst_err = 0, worst = 0;
  for (int i = 0; i < count; ++i) {
    const BatchOut& o = e->h_outs[i];
    psdp_info& f = info[i];
    std::memset(&f, 0, sizeof f);
    f.err_bound = o.err_bound;
    f.res_fro = o.res_fro;
    f.tail_est = o.tail_est;
    f.pi_fro = o.pi_fro;
    f.theta_guard = o.theta_guard;
    f.tol_used = o.tol_used;
    f.n_pos = o.n_pos;
    f.m_out = o.m_out;
    f.iters = o.iters;
    f.side_used = sign > 0 ? PSDP_SIDE_POS : PSDP_SIDE_NEG;
    f.certified = 0;
    f.status = o.status < 0 ? PSDP_ERR_NUMERICAL : o.status;
    f.expansions = o.expansions;
    f.prec_final = o.prec_final;
    f.n_pos_full = -1;
    if (o.status >= 0) m_inout[i] = o.m_out;
    if (f.status < 0) worst_err = std::min(worst_err, f.status);
    else worst = std::max(worst, f.status);
  }
  return (psdp_status)(worst_err < 0 ? worst_err : worst);
}

}  // namespace psdp
