// One-workgroup kernels on the small (<= 192 x 192) matrices of one
// LOBPCG iteration:
//   k_decide_chol : convergence / stall / expansion decisions, active set,
//                   and Cholesky-QR with column dropping of the trial basis
//                   (paper §5.1: Cholesky QR instead of Householder QR)
//   k_rr          : Rayleigh-Ritz on an orthonormal basis (paper §5, Alg. 2):
//                   parallel cyclic Jacobi on H = S^T A S in LDS, selection of
//                   the largest Ritz values, eigenvectors by replaying the
//                   rotation log on unit vectors.
#include "chol_body.h"

namespace psdp {
// ---------------------------------------------------------------- RR ----


__device__ inline void rr_pair(int Ne, int r, int k, int* p, int* q) {
  // round-robin: slot 0 pairs the fixed last player with r, slot k > 0 pairs
  // (r + k) and (r - k) modulo Ne - 1
  int x, y;
  const int M = Ne - 1;
  if (k == 0) {
    x = r;
    y = M;
  } else {
    x = r + k;
    if (x >= M) x -= M;
    y = r - k;
    if (y < 0) y += M;
  }
  *p = min(x, y);
  *q = max(x, y);
}

__global__ __launch_bounds__(kRRThreads) void k_rr(RRArgs a) {
  extern __shared__ double lds[];
  __shared__ double red[kRRThreads / 64];
  __shared__ double s_cs[kMaxN + 2];    // c, s per pair
  __shared__ int s_pq[kMaxN + 2];       // p, q per pair
  __shared__ double s_theta[kMaxN];
  __shared__ int s_rank[kMaxN];
  __shared__ int s_rounds;
  State* st = a.st;
  if (st->stop) return;
  const int tid = threadIdx.x;
  const int Np = st->Np;
  const int Ne = Np + (Np & 1);
  const int P = Ne / 2;
  const int mk = min(a.mtarget, Np);
  double* H = lds;  // packed upper, Np(Np+1)/2
  const int NH = Np * (Np + 1) / 2;
  // eigenvectors accumulated in LDS when they fit, else replayed from the log
  const bool vin = (size_t)NH + (size_t)Np * Np <= a.lds_cap;
  double* V = H + NH;
  double fro2 = 0.0;
  for (int e = tid; e < NH; e += blockDim.x) {
    int j = tri_row(e);
    int i = e - j * (j + 1) / 2;
    double h = 0.5 * (a.K[i + (size_t)j * a.ldk] + a.K[j + (size_t)i * a.ldk]);
    H[e] = h;
    fro2 += (i == j ? 1.0 : 2.0) * h * h;
  }
  if (vin)
    for (int e = tid; e < Np * Np; e += blockDim.x) V[e] = (e % Np == e / Np) ? 1.0 : 0.0;
  fro2 = block_sum(fro2, red);
  const double skip = 1e-18 * sqrt(fro2);
  const double stop2 = (a.off_tol * a.off_tol) * fro2;
  // ---- parallel cyclic Jacobi (round-robin order)
  int round_id = 0;
  const size_t per_round = (size_t)2 * P;
  const int nblocks = P * (P + 1) / 2;
  for (int sweep = 0; sweep < a.max_sweeps && Np > 1; ++sweep) {
    double off = 0.0;
    for (int j = 1; j < Np; ++j)
      for (int i = tid; i < j; i += blockDim.x) {
        double v = H[j * (j + 1) / 2 + i];
        off += 2.0 * v * v;
      }
    off = block_sum(off, red);
    if (off <= stop2) break;
    if (!vin && (size_t)(round_id + Ne) * per_round > a.log_cap) break;
    for (int r = 0; r < Ne - 1; ++r) {
      if (tid < P) {
        int p, q;
        rr_pair(Ne, r, tid, &p, &q);
        s_pq[2 * tid] = p;
        s_pq[2 * tid + 1] = q;
        double c = 1.0, s = 0.0;
        if (q < Np) {
          double hpq = H[pup(p, q)];
          if (fabs(hpq) > skip) {
            // t = sign(d) e / (|d| + sqrt(d^2 + e^2)), d = hqq - hpp, e = 2 hpq:
            // the smaller root of the symmetric 2x2 Schur rotation
            double d = H[pup(q, q)] - H[pup(p, p)];
            double e2 = 2.0 * hpq;
            double rr = sqrt(d * d + e2 * e2);
            double t = (d >= 0.0 ? e2 : -e2) / (fabs(d) + rr);
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        s_cs[2 * tid] = c;
        s_cs[2 * tid + 1] = s;
        if (!vin) {
          a.log[(size_t)round_id * per_round + 2 * tid] = c;
          a.log[(size_t)round_id * per_round + 2 * tid + 1] = s;
        }
      }
      __syncthreads();
      // two-sided update of every 2x2 block (k, l), k <= l
      for (int b = tid; b < nblocks; b += blockDim.x) {
        int l = tri_row(b);
        int k = b - l * (l + 1) / 2;
        double ck = s_cs[2 * k], sk = s_cs[2 * k + 1];
        double cl = s_cs[2 * l], sl = s_cs[2 * l + 1];
        if (sk == 0.0 && sl == 0.0) continue;
        int pk = s_pq[2 * k], qk = s_pq[2 * k + 1];
        int pl = s_pq[2 * l], ql = s_pq[2 * l + 1];
        if (k == l) {
          if (qk >= Np) continue;
          double hpp = H[pup(pk, pk)], hqq = H[pup(qk, qk)], hpq = H[pup(pk, qk)];
          double c2 = ck * ck, s2 = sk * sk, cs = ck * sk;
          H[pup(pk, pk)] = c2 * hpp - 2.0 * cs * hpq + s2 * hqq;
          H[pup(qk, qk)] = s2 * hpp + 2.0 * cs * hpq + c2 * hqq;
          H[pup(pk, qk)] = 0.0;
        } else {
          bool vk = qk < Np, vl = ql < Np;
          double b00 = H[pup(pk, pl)];
          double b01 = vl ? H[pup(pk, ql)] : 0.0;
          double b10 = vk ? H[pup(qk, pl)] : 0.0;
          double b11 = (vk && vl) ? H[pup(qk, ql)] : 0.0;
          double m00 = cl * b00 - sl * b01, m01 = sl * b00 + cl * b01;
          double m10 = cl * b10 - sl * b11, m11 = sl * b10 + cl * b11;
          H[pup(pk, pl)] = ck * m00 - sk * m10;
          if (vl) H[pup(pk, ql)] = ck * m01 - sk * m11;
          if (vk) H[pup(qk, pl)] = sk * m00 + ck * m10;
          if (vk && vl) H[pup(qk, ql)] = sk * m01 + ck * m11;
        }
      }
      if (vin) {
        // V <- V J: columns (p, q) of every pair
        for (int e = tid; e < Np * P; e += blockDim.x) {
          int i = e % Np, k = e / Np;
          double c = s_cs[2 * k], s = s_cs[2 * k + 1];
          int p = s_pq[2 * k], q = s_pq[2 * k + 1];
          if (s == 0.0 || q >= Np) continue;
          double vp = V[i + (size_t)p * Np], vq = V[i + (size_t)q * Np];
          V[i + (size_t)p * Np] = c * vp - s * vq;
          V[i + (size_t)q * Np] = s * vp + c * vq;
        }
      }
      __syncthreads();
      ++round_id;
    }
  }
  if (tid == 0) s_rounds = round_id;
  for (int i = tid; i < Np; i += blockDim.x) s_theta[i] = H[pup(i, i)];
  __syncthreads();
  // ranking (descending, ties by index)
  for (int i = tid; i < Np; i += blockDim.x) {
    double ti = s_theta[i];
    int r = 0;
    for (int j = 0; j < Np; ++j) {
      double tj = s_theta[j];
      r += (tj > ti) || (tj == ti && j < i);
    }
    s_rank[i] = r;
  }
  __syncthreads();
  if (vin) {
    for (int e = tid; e < Np * Np; e += blockDim.x) {
      int i = e % Np, j = e / Np;
      int r = s_rank[j];
      if (r < mk) a.C[i + (size_t)r * a.ldc] = V[e];
    }
  } else {
    // W = J_1 ... J_T E_sel: replay the logged rounds backwards on unit
    // vectors (H's LDS is reused)
    double* W = lds;
    for (int e = tid; e < Np * mk; e += blockDim.x) W[e] = 0.0;
    __syncthreads();
    for (int i = tid; i < Np; i += blockDim.x)
      if (s_rank[i] < mk) W[i + (size_t)s_rank[i] * Np] = 1.0;
    __syncthreads();
    const int rounds = s_rounds;
    double* chunk = W + (size_t)Np * mk;
    const int chunk_rounds = 32;
    for (int t_hi = rounds; t_hi > 0; t_hi -= chunk_rounds) {
      int t_lo = max(0, t_hi - chunk_rounds);
      int cnt = t_hi - t_lo;
      for (int e = tid; e < cnt * (int)per_round; e += blockDim.x)
        chunk[e] = a.log[(size_t)t_lo * per_round + e];
      __syncthreads();
      for (int t = t_hi - 1; t >= t_lo; --t) {
        int r = t % (Ne - 1);
        const double* cs = chunk + (size_t)(t - t_lo) * per_round;
        for (int e = tid; e < P * mk; e += blockDim.x) {
          int k = e % P, col = e / P;
          double c = cs[2 * k], s = cs[2 * k + 1];
          if (s == 0.0) continue;
          int p, q;
          rr_pair(Ne, r, k, &p, &q);
          if (q >= Np) continue;
          double wp = W[p + (size_t)col * Np], wq = W[q + (size_t)col * Np];
          W[p + (size_t)col * Np] = c * wp + s * wq;
          W[q + (size_t)col * Np] = -s * wp + c * wq;
        }
        __syncthreads();
      }
    }
    for (int e = tid; e < Np * mk; e += blockDim.x) {
      int i = e % Np, col = e / Np;
      a.C[i + (size_t)col * a.ldc] = W[e];
    }
  }
  int npos = 0;
  for (int i = tid; i < Np; i += blockDim.x) {
    npos += (s_theta[i] > 0.0);
    if (s_rank[i] < mk) st->theta[s_rank[i]] = s_theta[i];
  }
  double npd = block_sum((double)npos, red);
  if (tid == 0) {
    st->npos_rr = (int)npd;
    st->mk = mk;
    st->expand_req = ((int)npd > a.mtarget) ? 1 : 0;
    st->jacobi_rounds = s_rounds;
    if (a.count_iter) st->iter += 1;
  }
}

__global__ __launch_bounds__(kSmallThreads) void k_decide_chol(DecideArgs a) {
  extern __shared__ double lds[];
  __shared__ double red[kSmallThreads / 64 + 128];
  __shared__ int s_list[kMaxN], s_kind[kMaxN], s_col[kMaxN], s_keep[kMaxN];
  __shared__ int s_N, s_Np, s_nx, s_stop;
  CholShared sh{s_list, s_kind, s_col, s_keep, &s_N, &s_Np, &s_nx, &s_stop, red};
  decide_chol_body(a, lds, sh);
}

hipError_t launch_decide_chol(const DecideArgs& a, int N_host, hipStream_t st) {
  size_t scr = std::max((size_t)(kSmallThreads / 64) * 256, (size_t)16 * N_host);
  size_t lds = sizeof(double) * ((size_t)N_host * (N_host + 1) / 2 + (size_t)N_host + scr + 8);
  hipLaunchKernelGGL(k_decide_chol, dim3(1), dim3(kSmallThreads), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_rr(const RRArgs& a_in, int Np_host, int mk_host, hipStream_t st) {
  RRArgs a = a_in;
  size_t h = (size_t)Np_host * (Np_host + 1) / 2;
  size_t w = (size_t)Np_host * mk_host + (size_t)32 * (Np_host + 2) + 64;
  size_t want = h + (size_t)Np_host * Np_host;  // H and V both in LDS
  size_t cap_doubles = (size_t)(g_lds_limit / 8);
  size_t need = std::max(h, w);
  size_t lds_d = want <= cap_doubles ? want : need;
  a.lds_cap = lds_d;
  hipLaunchKernelGGL(k_rr, dim3(1), dim3(kRRThreads), sizeof(double) * lds_d, st, a);
  return hipGetLastError();
}

hipError_t small_kernels_init() {
  // allow up to the device's LDS per workgroup for the dynamic allocations
  int dev = 0, lim = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
  if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    lim = 64 * 1024;
  int dyn = lim - 8 * 1024;  // static LDS of the kernels stays below 8 KB
  if (dyn > 0) g_lds_limit = dyn;
  if (dyn > 0) {
    (void)hipFuncSetAttribute((const void*)k_decide_chol,
                              hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    (void)hipFuncSetAttribute((const void*)k_rr, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
  }
  (void)hipGetLastError();
  return hipSuccess;
}

}  // namespace psdp
