// psdp_block_product_noalloc: the block product entry point for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).  Every buffer beyond the
// caller's inputs and outputs (the FP64 and product-precision copies of A,
// the staged S, the split-K partial sums, the ingest's partial norms and
// flag) lives in `scratch`, a file-scope device array of kScratchBytes.  The
// array's device address is taken once per device with hipGetSymbolAddress
// (its name in host code is only a stand-in) and used for every launch.
// Every call on one GPU shares that GPU's array: calls that overlap on one
// GPU race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/psdp.h"
#include "common.h"
#include "internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;
constexpr int kMaxSlices = 16;  // split-K slices of the single-cone workspace

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
char* g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (the device is current).
psdp_status scratch_address(int device, char** out) {
  if (device < 0 || device >= kMaxDevices) return PSDP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PSDP_ERR_HIP;
    g_scratch[device] = (char*)p;
  }
  *out = g_scratch[device];
  return PSDP_OK;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Layout {
  size_t a64, alp, s, part, fro, flag, total;
  int slices;
};

// Carving of the scratch array for order n, k columns and precision prec:
// the most split-K slices (up to 16) that fit; total > kScratchBytes when
// even one slice does not fit.
Layout layout(int n, int k, int prec) {
  Layout o{};
  const size_t L = (size_t)psdp::round_up(n, 64);
  const size_t el = prec == 0 ? 8 : (prec == 1 ? 4 : 2);
  const size_t pel = prec == 0 ? 8 : 4;
  const size_t T32 = (L + 31) / 32;
  size_t off = 0;
  o.a64 = off;  off = align_up(off + 8 * L * L, 256);
  o.alp = off;  off = align_up(off + (prec == 0 ? 0 : el * L * L), 256);
  o.s = off;    off = align_up(off + 8 * L * (size_t)k, 256);
  o.fro = off;  off = align_up(off + 8 * T32 * (T32 + 1) / 2, 256);
  o.flag = off; off = align_up(off + 64, 256);
  o.part = off;
  const size_t per = pel * L * (size_t)k;
  int sl = kMaxSlices;
  while (sl > 1 && off + per * sl > kScratchBytes) --sl;
  o.slices = sl;
  o.total = off + per * sl;
  return o;
}

}  // namespace

extern "C" psdp_status psdp_block_product_noalloc(psdp_handle h, int n, const double* X, int ldx,
                                                  const double* S, int lds, int k, int prec,
                                                  double* Y, int ldy) {
  using namespace psdp;
  if (!h || n < 1 || k < 1 || k > kMaxN || !X || !S || !Y || ldx < n || lds < n || ldy < n ||
      prec < 0 || prec > 2)
    return PSDP_ERR_INVALID_ARG;
  const Layout lay = layout(n, k, prec);
  if (lay.total > kScratchBytes) return PSDP_ERR_CAPACITY;
  const int device = handle_device(h);
  if (hipSetDevice(device) != hipSuccess) return PSDP_ERR_HIP;
  char* base = nullptr;
  psdp_status ps = scratch_address(device, &base);
  if (ps != PSDP_OK) return ps;
  hipStream_t s = handle_stream(h);
  const int L = round_up(n, 64);
  double* A64 = (double*)(base + lay.a64);
  void* Alp = prec == 0 ? nullptr : (void*)(base + lay.alp);
  double* S2 = (double*)(base + lay.s);
  double* fro = (double*)(base + lay.fro);
  int* nonfinite = (int*)(base + lay.flag);
  // the ingest only ever sets the flag: clear it with a kernel (no memset
  // node in a captured graph)
  if (launch_set_int(nonfinite, 0, s) != hipSuccess) return PSDP_ERR_HIP;
  int nb = 0;
  if (launch_ingest(X, ldx, n, 1.0, A64, L, L, Alp, prec, fro, nonfinite, s, &nb) != hipSuccess)
    return PSDP_ERR_HIP;
  if (launch_copy_cols(S, lds, S2, L, n, k, s) != hipSuccess) return PSDP_ERR_HIP;
  ProductArgs pa{};
  pa.A = prec == 0 ? (const void*)A64 : Alp;
  pa.lda = L;
  pa.n = n;
  pa.prec = prec;
  pa.S = S2;
  pa.lds = L;
  pa.Y = Y;
  pa.ldy = ldy;
  pa.cols_dev = nullptr;
  pa.cols_max = k;
  pa.stop = nullptr;
  pa.partial = base + lay.part;
  pa.partial_bytes = kScratchBytes - lay.part;
  pa.max_slices = lay.slices;
  if (launch_product(pa, s) != hipSuccess) return PSDP_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return PSDP_ERR_HIP;
  return PSDP_OK;
}
