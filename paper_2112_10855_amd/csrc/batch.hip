// Batched CP-ALS-QR (paper Alg. 2) for many small 3-way tensors in one
// persistent launch.
//
// Design.  One workgroup owns one tensor for the whole run: every sweep's
// Khatri-Rao QR, Multi-TTM, Q_0 application, solve, normalization, factor QR
// and efficient error execute inside that workgroup, with workgroup barriers
// between steps and no dependency on any other workgroup, so a single launch
// carries all sweeps of all tensors.  Tensors are dispatched largest first
// (longest-processing-time order) so the big ones start early.  Per-tensor
// scratch (intermediates, Q_k, R_k, Q_0, R_0) lives in the caller's work
// buffer; the tensor and the factors stay in HBM and the small intermediates
// stay in L2.
//
// Limits: N = 3, R <= 16, I_k <= NT (the factor QR keeps one row per thread),
// R^2 <= NT.  Arithmetic: Multi-TTM in FP32 on the vector ALUs (the tensors are
// small and the contractions short), everything else FP64.

#include <sys/stat.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "wgqr.h"

namespace cpqr {
namespace {

using namespace wgqr;

constexpr int RB = 16;     // register width for factor rows (R <= 16)
constexpr int UROWS = 256; // rows of a contraction operand staged in LDS

struct BItem {
  int64_t I[3];
  int R;
  int pad;
  const float* X;
  double* A[3];
  double* Q[3];
  double* Rf[3];
  double* lam;
  double* relerr;
  float* T;    // first contraction output
  float* T2;   // second contraction output before unfolding
  float* Y;    // Y_(n), I_n x R^2
  double* Q0;  // R^2 x R
  double* R0;  // R x R
  double* xnorm2;
};

template <int NT>
struct BShared {
  Shared<RB, NT> qr;
  union alignas(16) {
    float us[UROWS * RB];     // contraction operand, row-major (i, r) -- Multi-TTM
    double q0s[UROWS * RB];   // Q_0 rows, row-major (rho, c) -- Khatri-Rao QR to solve
  };
  double r0[RB][RB + 1];      // R_0
  double rn[RB][RB + 1];      // R_n of the last factor QR
  double lam[RB];
};

// T'[p, r, s] = sum_i T[p, i, s] U[i, r] with U in LDS (row-major, RB wide).
// One thread per (p, s); R accumulators; RR is R rounded up to a multiple of 4.
template <int NT, int RR>
__device__ void wg_ttm(const float* __restrict__ src, float* __restrict__ dst, int64_t P, int64_t K,
                       int64_t S, int R, const float* us, int tid) {
  const int64_t M = P * S;
  for (int64_t m = tid; m < M; m += NT) {
    const int64_t p = m % P, s = m / P;
    const float* base = src + p + s * P * K;
    float acc[RR];
#pragma unroll
    for (int r = 0; r < RR; ++r) acc[r] = 0.f;
    for (int64_t i = 0; i < K; ++i) {
      const float x = base[i * P];
      const float4* u = reinterpret_cast<const float4*>(us + i * RB);
#pragma unroll
      for (int q = 0; q < RR / 4; ++q) {
        const float4 uv = u[q];
        acc[4 * q] += x * uv.x;
        acc[4 * q + 1] += x * uv.y;
        acc[4 * q + 2] += x * uv.z;
        acc[4 * q + 3] += x * uv.w;
      }
    }
#pragma unroll
    for (int r = 0; r < RR; ++r)
      if (r < R) dst[p + r * P + s * P * R] = acc[r];
  }
}

template <int NT>
__device__ void wg_ttm_r(const float* src, float* dst, int64_t P, int64_t K, int64_t S, int R,
                         const float* us, int tid) {
  if (R <= 4) wg_ttm<NT, 4>(src, dst, P, K, S, R, us, tid);
  else if (R <= 8) wg_ttm<NT, 8>(src, dst, P, K, S, R, us, tid);
  else if (R <= 12) wg_ttm<NT, 12>(src, dst, P, K, S, R, us, tid);
  else wg_ttm<NT, 16>(src, dst, P, K, S, R, us, tid);
}

// Stage Q_k (I_k x R FP64, column-major) as FP32 rows into us; zeros past R.
template <int NT>
__device__ void stage_u(const double* Q, int64_t Ik, int R, float* us, int tid) {
  for (int e = tid; e < Ik * RB; e += NT) {
    const int i = e / RB, r = e % RB;
    us[e] = r < R ? float(Q[i + int64_t(r) * Ik]) : 0.f;
  }
}

// Factor QR of the block held in a[] (one row per thread, m rows): writes
// Q (m x R, ld m) and R (R x R) to global, and R into sh.rn.
template <int NT>
__device__ void wg_qr_store(double (&a)[RB], int m, int R, BShared<NT>& sh, double* Qout, int64_t ldq,
                            double* Rout, int tid) {
  wg_factor<RB, NT>(a, tid, m, R, sh.qr);
  wg_build_t<RB, NT>(tid, R, sh.qr);
  if (tid < R) {
#pragma unroll
    for (int c = 0; c < RB; ++c) {
      const double v = (c >= tid && c < R) ? a[c] : 0.0;
      sh.rn[tid][c] = v;
      if (c < R) Rout[tid + c * R] = v;
    }
  }
  for (int e = tid; e < RB * RB; e += NT) sh.qr.C[e / RB][e % RB] = (e / RB == e % RB) ? 1.0 : 0.0;
  __syncthreads();
  double q[RB];
  wg_form_q<RB, NT>(a, q, tid, m, R, sh.qr);
  if (tid < m) {
#pragma unroll
    for (int c = 0; c < RB; ++c)
      if (c < R) Qout[tid + c * ldq] = q[c];
  }
  __syncthreads();
}

template <int NT>
__device__ double block_sum1(double v, Shared<RB, NT>& q, int tid) {
  double x[1] = {v};
  block_sum_vec<1, NT / WAVE>(x, q.red, q.res, tid);
  return q.res[0];
}

template <int NT>
__global__ __launch_bounds__(NT) void als_batch_kernel(const BItem* __restrict__ items,
                                                       const int* __restrict__ order, int nsweeps,
                                                       int do_init, int sweep_offset) {
  __shared__ BShared<NT> sh;
  const int tid = threadIdx.x;
  const BItem it = items[order[blockIdx.x]];
  const int R = it.R;
  const int64_t I0 = it.I[0], I1 = it.I[1], I2 = it.I[2];

  if (do_init) {
    for (int k = 1; k < 3; ++k) {
      double a[RB];
#pragma unroll
      for (int c = 0; c < RB; ++c) a[c] = (tid < it.I[k] && c < R) ? it.A[k][tid + c * it.I[k]] : 0.0;
      wg_qr_store<NT>(a, int(it.I[k]), R, sh, it.Q[k], it.I[k], it.Rf[k], tid);
    }
    for (int c = tid; c < R; c += NT) it.lam[c] = 1.0;
    double s = 0.0;
    const int64_t cnt = I0 * I1 * I2;
    for (int64_t e = tid; e < cnt; e += NT) {
      const double v = double(it.X[e]);
      s += v * v;
    }
    s = block_sum1<NT>(s, sh.qr, tid);
    if (tid == 0) *it.xnorm2 = s;
    __syncthreads();
  }

  const int64_t K0 = int64_t(R) * R;  // rows of V_n, columns of Y_(n)
  for (int sw = 0; sw < nsweeps; ++sw) {
    for (int n = 0; n < 3; ++n) {
      const int ma = n == 0 ? 1 : 0, mb = n == 2 ? 1 : 2;  // the two other modes, ascending
      // ---- Multi-TTM: Y_(n), first contraction over a mode with P > 1
      int64_t Pn, In, Sn;  // layout of the second contraction's output [Pn, In, Sn]
      if (n == 0) {
        stage_u<NT>(it.Q[1], I1, R, sh.us, tid);
        __syncthreads();
        wg_ttm_r<NT>(it.X, it.T, I0, I1, I2, R, sh.us, tid);  // T[i0, r1, i2]
        __syncthreads();
        stage_u<NT>(it.Q[2], I2, R, sh.us, tid);
        __syncthreads();
        wg_ttm_r<NT>(it.T, it.Y, I0 * R, I2, 1, R, sh.us, tid);  // Y[i0, r1, r2] = Y_(1)
        Pn = 1;
        In = I0;
        Sn = K0;
      } else if (n == 1) {
        stage_u<NT>(it.Q[2], I2, R, sh.us, tid);
        __syncthreads();
        wg_ttm_r<NT>(it.X, it.T, I0 * I1, I2, 1, R, sh.us, tid);  // T[i0, i1, r2]
        __syncthreads();
        stage_u<NT>(it.Q[0], I0, R, sh.us, tid);
        __syncthreads();
        wg_ttm_r<NT>(it.T, it.T2, 1, I0, I1 * R, R, sh.us, tid);  // T2[r0, i1, r2]
        Pn = R;
        In = I1;
        Sn = R;
      } else {
        stage_u<NT>(it.Q[1], I1, R, sh.us, tid);
        __syncthreads();
        wg_ttm_r<NT>(it.X, it.T, I0, I1, I2, R, sh.us, tid);  // T[i0, r1, i2]
        __syncthreads();
        stage_u<NT>(it.Q[0], I0, R, sh.us, tid);
        __syncthreads();
        wg_ttm_r<NT>(it.T, it.T2, 1, I0, R * I2, R, sh.us, tid);  // T2[r0, r1, i2]
        Pn = K0;
        In = I2;
        Sn = 1;
      }
      __syncthreads();
      if (n != 0) {  // Y_(n)[i + In (p + Pn s)] = T2[p + Pn i + Pn In s]
        const int64_t cnt = Pn * In * Sn;
        for (int64_t e = tid; e < cnt; e += NT) {
          const int64_t i = e % In, c = e / In;
          const int64_t p = c % Pn, s = c / Pn;
          it.Y[e] = it.T2[p + Pn * i + Pn * In * s];
        }
        __syncthreads();
      }
      // ---- V_n = R_mb (.) R_ma, QR with Q_0 explicit (rows: index of ma fastest)
      {
        double a[RB];
        const int rho = tid, da = rho % R, db = rho / R;
#pragma unroll
        for (int c = 0; c < RB; ++c)
          a[c] = (rho < K0 && c < R) ? it.Rf[ma][da + c * R] * it.Rf[mb][db + c * R] : 0.0;
        wg_factor<RB, NT>(a, tid, int(K0), R, sh.qr);
        wg_build_t<RB, NT>(tid, R, sh.qr);
        if (tid < R) {
#pragma unroll
          for (int c = 0; c < RB; ++c) sh.r0[tid][c] = (c >= tid && c < R) ? a[c] : 0.0;
        }
        for (int e = tid; e < RB * RB; e += NT) sh.qr.C[e / RB][e % RB] = (e / RB == e % RB) ? 1.0 : 0.0;
        __syncthreads();
        double q[RB];
        wg_form_q<RB, NT>(a, q, tid, int(K0), R, sh.qr);
        if (tid < K0) {
#pragma unroll
          for (int c = 0; c < RB; ++c) sh.q0s[tid * RB + c] = c < R ? q[c] : 0.0;
        }
        __syncthreads();
      }
      // ---- W = Y_(n) Q_0, solve A R_0^T = W, per row; keep rows in registers
      double arow[RB], wrow[RB];
#pragma unroll
      for (int c = 0; c < RB; ++c) arow[c] = wrow[c] = 0.0;
      const int64_t Inn = it.I[n];
      if (tid < Inn) {
        for (int64_t rho = 0; rho < K0; ++rho) {
          const double y = double(it.Y[tid + rho * Inn]);
#pragma unroll
          for (int c = 0; c < RB; ++c) wrow[c] += y * sh.q0s[rho * RB + c];
        }
#pragma unroll
        for (int j = RB - 1; j >= 0; --j) {
          if (j < R) {
            double v = wrow[j];
#pragma unroll
            for (int c = j + 1; c < RB; ++c)
              if (c < R) v -= sh.r0[j][c] * arow[c];
            arow[j] = v / sh.r0[j][j];
          }
        }
      }
      // <W, Ahat R_0^T> of this row, needed by the error after the last mode
      double ip = 0.0;
      if (n == 2 && tid < Inn) {
#pragma unroll
        for (int c = 0; c < RB; ++c) {
          if (c >= R) continue;
          double v = 0.0;
#pragma unroll
          for (int k = 0; k < RB; ++k)
            if (k >= c && k < R) v += arow[k] * sh.r0[c][k];
          ip += wrow[c] * v;
        }
      }
      // ---- normalize: lambda_c = ||A(:, c)||
      {
        double x[RB];
#pragma unroll
        for (int c = 0; c < RB; ++c) x[c] = arow[c] * arow[c];
        block_sum_vec<RB, NT / WAVE>(x, sh.qr.red, sh.qr.res, tid);
        if (tid < RB) sh.lam[tid] = tid < R ? sqrt(sh.qr.res[tid]) : 0.0;
        __syncthreads();
      }
      double anorm[RB];
#pragma unroll
      for (int c = 0; c < RB; ++c) {
        const double l = sh.lam[c];
        anorm[c] = (c < R && l > 0.0) ? arow[c] / l : 0.0;
      }
      if (tid < Inn) {
#pragma unroll
        for (int c = 0; c < RB; ++c)
          if (c < R) it.A[n][tid + c * Inn] = anorm[c];
      }
      for (int c = tid; c < R; c += NT) it.lam[c] = sh.lam[c];
      // ---- factor QR of the normalized A_n
      {
        double a[RB];
#pragma unroll
        for (int c = 0; c < RB; ++c) a[c] = tid < Inn ? anorm[c] : 0.0;
        wg_qr_store<NT>(a, int(Inn), R, sh, it.Q[n], Inn, it.Rf[n], tid);
      }
      // ---- efficient error after the last mode (section 3.3.1)
      if (n == 2) {
        ip = block_sum1<NT>(ip, sh.qr, tid);
        double nn = 0.0;
        for (int e = tid; e < R * R; e += NT) {
          const int a = e % R, b = e / R;
          double g0 = 0.0, gn = 0.0;
          for (int k = 0; k < R; ++k) {
            g0 += sh.r0[k][a] * sh.r0[k][b];
            gn += sh.rn[k][a] * sh.rn[k][b];
          }
          nn += g0 * sh.lam[a] * sh.lam[b] * gn;
        }
        nn = block_sum1<NT>(nn, sh.qr, tid);
        if (tid == 0 && it.relerr) {
          const double x2 = *it.xnorm2;
          const double r2 = x2 - 2.0 * ip + nn;
          it.relerr[sweep_offset + sw] = sqrt((r2 > 0.0 ? r2 : 0.0) / x2);
        }
        __syncthreads();
      }
    }
  }
}

// ------------------------------------------------------------ host side
struct Layout {
  BItem* items;  // device
  int* order;    // device
  int n;
  char* scratch;
};

size_t item_scratch(const cpqr_batch_item& b) {
  const int64_t R = b.R;
  const int64_t i0 = b.I[0], i1 = b.I[1], i2 = b.I[2];
  const int64_t imax = std::max(i0, std::max(i1, i2));
  const int64_t t1 = std::max(i0 * R * i2, i0 * i1 * R);
  const int64_t t2 = R * R * imax;
  Carver cv(nullptr);
  for (int k = 0; k < 3; ++k) cv.take<double>(size_t(b.I[k]) * R);  // Q
  for (int k = 0; k < 3; ++k) cv.take<double>(size_t(R) * R);       // Rf
  cv.take<float>(t1);
  cv.take<float>(t2);
  cv.take<float>(t2);                 // Y
  cv.take<double>(size_t(R * R) * R);  // Q0
  cv.take<double>(size_t(R) * R);      // R0
  cv.take<double>(1);                  // xnorm2
  return cv.bytes();
}

int nt_needed(const cpqr_batch_item* items, int n) {
  int64_t need = 1;
  for (int b = 0; b < n; ++b) {
    need = std::max(need, std::max(items[b].I[0], std::max(items[b].I[1], items[b].I[2])));
    need = std::max<int64_t>(need, int64_t(items[b].R) * items[b].R);
  }
  return int(need);
}

int launch_batch(int nt, const Layout& L, int nsweeps, int do_init, int offset, hipStream_t s) {
  const dim3 grd(unsigned(L.n));
  if (nt == 256)
    hipLaunchKernelGGL(als_batch_kernel<256>, grd, dim3(256), 0, s, L.items, L.order, nsweeps, do_init, offset);
  else if (nt == 512)
    hipLaunchKernelGGL(als_batch_kernel<512>, grd, dim3(512), 0, s, L.items, L.order, nsweeps, do_init, offset);
  else
    hipLaunchKernelGGL(als_batch_kernel<1024>, grd, dim3(1024), 0, s, L.items, L.order, nsweeps, do_init, offset);
  return check_launch("als_batch_kernel");
}

// What cpqr_als_batch_prepare decided for one work buffer (host side).
struct BatchHeader {
  int n;
  int nt;      // workgroup size chosen
  int min_nt;  // smallest workgroup size that fits the batch
};
std::mutex g_batch_mu;
std::map<const void*, BatchHeader> g_batch;

struct GraphKey {
  const void* work;
  int nsweeps, init, offset, nt;
  bool operator<(const GraphKey& o) const {
    if (work != o.work) return work < o.work;
    if (nsweeps != o.nsweeps) return nsweeps < o.nsweeps;
    if (init != o.init) return init < o.init;
    if (offset != o.offset) return offset < o.offset;
    return nt < o.nt;
  }
};
std::map<GraphKey, hipGraphExec_t> g_graphs;
hipStream_t g_capture_stream = nullptr;

// autotune cache: key -> threads per tensor
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

std::string tune_path() {
  const char* p = getenv("CPQR_AUTOTUNE_CACHE");
  if (p && *p) return p;
  const char* h = getenv("HOME");
  return std::string(h ? h : "/tmp") + "/.cache/cpqr_autotune.txt";
}

void tune_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  FILE* f = fopen(tune_path().c_str(), "r");
  if (!f) return;
  char key[256];
  int v;
  while (fscanf(f, "%255s %d", key, &v) == 2) g_tune[key] = v;
  fclose(f);
}

void tune_store() {
  const std::string p = tune_path();
  const size_t slash = p.find_last_of('/');
  if (slash != std::string::npos) {
    const std::string dir = p.substr(0, slash);
    mkdir(dir.c_str(), 0755);  // best effort; fopen below reports nothing on failure
  }
  FILE* f = fopen(p.c_str(), "w");
  if (!f) return;
  for (auto& kv : g_tune) fprintf(f, "%s %d\n", kv.first.c_str(), kv.second);
  fclose(f);
}

std::string tune_key(const cpqr_batch_item* items, int n) {
  int64_t maxi = 0, tot = 0;
  int maxr = 0;
  for (int b = 0; b < n; ++b) {
    maxi = std::max(maxi, std::max(items[b].I[0], std::max(items[b].I[1], items[b].I[2])));
    maxr = std::max(maxr, items[b].R);
    tot += items[b].I[0] * items[b].I[1] * items[b].I[2];
  }
  int lg = 0;
  while ((int64_t(1) << lg) < tot) ++lg;
  hipDeviceProp_t prop;
  int dev = 0;
  std::string arch = "gfx";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  char buf[256];
  snprintf(buf, sizeof(buf), "%s|n%d|imax%lld|rmax%d|elems2^%d", arch.c_str(), n, (long long)((maxi + 31) / 32 * 32),
           maxr, lg);
  return buf;
}

}  // namespace
}  // namespace cpqr

using namespace cpqr;

extern "C" {

size_t cpqr_als_batch_work(const cpqr_batch_item* items, int nitems) {
  if (!items || nitems < 1) return 0;
  Carver cv(nullptr);
  cv.take<BItem>(nitems);
  cv.take<int>(nitems);
  for (int b = 0; b < nitems; ++b) {  // saved initial factors for autotuning
    cv.take<double>(size_t(items[b].I[1]) * items[b].R);
    cv.take<double>(size_t(items[b].I[2]) * items[b].R);
  }
  for (int b = 0; b < nitems; ++b) cv.take<char>(item_scratch(items[b]));
  return cv.bytes();
}

int cpqr_als_batch_prepare(const cpqr_batch_item* items, int nitems, int autotune, void* work,
                           size_t work_bytes, void* stream) {
  if (!items || nitems < 1) return fail(CPQR_ERR_ARG, "als_batch: no items");
  for (int b = 0; b < nitems; ++b) {
    const cpqr_batch_item& it = items[b];
    if (it.R < 1 || it.R > 16) return fail(CPQR_ERR_SHAPE, "als_batch: R must be in [1, 16]");
    for (int k = 0; k < 3; ++k) {
      if (it.I[k] < it.R || it.I[k] > UROWS)
        return fail(CPQR_ERR_SHAPE, "als_batch: mode sizes must be in [R, 256]");
      if (!it.A[k]) return fail(CPQR_ERR_ARG, "als_batch: NULL factor");
    }
    if (!it.X || !it.lambda) return fail(CPQR_ERR_ARG, "als_batch: NULL tensor or lambda");
  }
  CPQR_TRY(check_work(work, work_bytes, cpqr_als_batch_work(items, nitems)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver cv(work);
  BItem* items_dev = cv.take<BItem>(nitems);
  int* order_dev = cv.take<int>(nitems);
  std::vector<double*> saved(2 * nitems);
  for (int b = 0; b < nitems; ++b) {
    saved[2 * b] = cv.take<double>(size_t(items[b].I[1]) * items[b].R);
    saved[2 * b + 1] = cv.take<double>(size_t(items[b].I[2]) * items[b].R);
  }
  std::vector<BItem> h(nitems);
  for (int b = 0; b < nitems; ++b) {
    const cpqr_batch_item& it = items[b];
    Carver c2(cv.take<char>(item_scratch(it)));
    BItem& d = h[b];
    d = BItem{};
    for (int k = 0; k < 3; ++k) d.I[k] = it.I[k];
    d.R = it.R;
    d.X = it.X;
    for (int k = 0; k < 3; ++k) d.A[k] = it.A[k];
    d.lam = it.lambda;
    d.relerr = it.relerr;
    const int64_t R = it.R, imax = std::max(it.I[0], std::max(it.I[1], it.I[2]));
    for (int k = 0; k < 3; ++k) d.Q[k] = c2.take<double>(size_t(it.I[k]) * R);
    for (int k = 0; k < 3; ++k) d.Rf[k] = c2.take<double>(size_t(R) * R);
    d.T = c2.take<float>(std::max(it.I[0] * R * it.I[2], it.I[0] * it.I[1] * R));
    d.T2 = c2.take<float>(R * R * imax);
    d.Y = c2.take<float>(R * R * imax);
    d.Q0 = c2.take<double>(size_t(R * R) * R);
    d.R0 = c2.take<double>(size_t(R) * R);
    d.xnorm2 = c2.take<double>(1);
  }
  std::vector<int> order(nitems);
  for (int b = 0; b < nitems; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const auto w = [&](int t) { return items[t].I[0] * items[t].I[1] * items[t].I[2] * items[t].R; };
    return w(a) > w(b);
  });
  const int need = nt_needed(items, nitems);
  const int min_nt = need <= 256 ? 256 : (need <= 512 ? 512 : 1024);
  BatchHeader hdr{};
  hdr.n = nitems;
  hdr.min_nt = min_nt;
  hdr.nt = min_nt;
  CPQR_HIP(hipMemcpy(items_dev, h.data(), sizeof(BItem) * nitems, hipMemcpyHostToDevice));
  CPQR_HIP(hipMemcpy(order_dev, order.data(), sizeof(int) * nitems, hipMemcpyHostToDevice));
  for (int b = 0; b < nitems; ++b) {
    CPQR_HIP(hipMemcpyAsync(saved[2 * b], items[b].A[1], sizeof(double) * items[b].I[1] * items[b].R,
                            hipMemcpyDeviceToDevice, s));
    CPQR_HIP(hipMemcpyAsync(saved[2 * b + 1], items[b].A[2], sizeof(double) * items[b].I[2] * items[b].R,
                            hipMemcpyDeviceToDevice, s));
  }
  Layout L{items_dev, order_dev, nitems, nullptr};
  if (autotune) {
    const std::string key = tune_key(items, nitems);
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_load();
    auto found = g_tune.find(key);
    if (found != g_tune.end() && found->second >= min_nt) {
      hdr.nt = found->second;
    } else {
      // time one init + sweep per candidate, restoring the initial factors after each
      hipEvent_t e0, e1;
      CPQR_HIP(hipEventCreate(&e0));
      CPQR_HIP(hipEventCreate(&e1));
      float best = 1e30f;
      for (int nt : {256, 512, 1024}) {
        if (nt < min_nt) continue;
        CPQR_TRY(launch_batch(nt, L, 1, 1, 0, s));  // warm
        CPQR_HIP(hipEventRecord(e0, s));
        CPQR_TRY(launch_batch(nt, L, 1, 1, 0, s));
        CPQR_HIP(hipEventRecord(e1, s));
        CPQR_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        CPQR_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          hdr.nt = nt;
        }
        for (int b = 0; b < nitems; ++b) {
          CPQR_HIP(hipMemcpyAsync(items[b].A[1], saved[2 * b], sizeof(double) * items[b].I[1] * items[b].R,
                                  hipMemcpyDeviceToDevice, s));
          CPQR_HIP(hipMemcpyAsync(items[b].A[2], saved[2 * b + 1], sizeof(double) * items[b].I[2] * items[b].R,
                                  hipMemcpyDeviceToDevice, s));
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      g_tune[key] = hdr.nt;
      tune_store();
    }
  }
  CPQR_HIP(hipStreamSynchronize(s));
  {
    std::lock_guard<std::mutex> g(g_batch_mu);
    g_batch[work] = hdr;
    for (auto it = g_graphs.begin(); it != g_graphs.end();) {  // graphs of an older layout
      if (it->first.work == work) {
        (void)hipGraphExecDestroy(it->second);
        it = g_graphs.erase(it);
      } else {
        ++it;
      }
    }
  }
  return CPQR_OK;
}

static int batch_lookup(void* work, int threads, BatchHeader& hdr, int& nt) {
  if (!work) return fail(CPQR_ERR_WORKSPACE, "als_batch: work buffer is NULL");
  {
    std::lock_guard<std::mutex> g(g_batch_mu);
    auto f = g_batch.find(work);
    if (f == g_batch.end()) return fail(CPQR_ERR_WORKSPACE, "als_batch: work buffer not prepared");
    hdr = f->second;
  }
  nt = threads > 0 ? threads : hdr.nt;
  if (nt != 256 && nt != 512 && nt != 1024) return fail(CPQR_ERR_ARG, "als_batch: threads must be 256, 512 or 1024");
  if (nt < hdr.min_nt) return fail(CPQR_ERR_SHAPE, "als_batch: threads too few for the largest item");
  return CPQR_OK;
}

static Layout batch_layout(void* work, int n) {
  Carver cv(work);
  BItem* items_dev = cv.take<BItem>(n);
  int* order_dev = cv.take<int>(n);
  return Layout{items_dev, order_dev, n, nullptr};
}

int cpqr_als_batch_run(void* work, int nsweeps, int init, int sweep_offset, int threads, void* stream) {
  if (nsweeps < 0 || sweep_offset < 0) return fail(CPQR_ERR_ARG, "als_batch: negative sweep count");
  BatchHeader hdr;
  int nt;
  CPQR_TRY(batch_lookup(work, threads, hdr, nt));
  return launch_batch(nt, batch_layout(work, hdr.n), nsweeps, init ? 1 : 0, sweep_offset,
                      static_cast<hipStream_t>(stream));
}

int cpqr_als_batch_graph(void* work, int nsweeps, int init, int sweep_offset, int threads, void* stream) {
  if (nsweeps < 0 || sweep_offset < 0) return fail(CPQR_ERR_ARG, "als_batch: negative sweep count");
  BatchHeader hdr;
  int nt;
  CPQR_TRY(batch_lookup(work, threads, hdr, nt));
  const GraphKey key{work, nsweeps, init ? 1 : 0, sweep_offset, nt};
  hipGraphExec_t exec = nullptr;
  {
    std::lock_guard<std::mutex> g(g_batch_mu);
    auto f = g_graphs.find(key);
    if (f != g_graphs.end()) exec = f->second;
  }
  if (!exec) {
    if (!g_capture_stream) CPQR_HIP(hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking));
    CPQR_HIP(hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal));
    const int rc = launch_batch(nt, batch_layout(work, hdr.n), nsweeps, init ? 1 : 0, sweep_offset, g_capture_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(g_capture_stream, &graph);
    if (rc != CPQR_OK) return rc;
    if (e != hipSuccess) return fail(CPQR_ERR_HIP, std::string("als_batch: capture failed: ") + hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) return fail(CPQR_ERR_HIP, std::string("als_batch: instantiate failed: ") + hipGetErrorString(e2));
    std::lock_guard<std::mutex> g(g_batch_mu);
    g_graphs[key] = exec;
  }
  CPQR_HIP(hipGraphLaunch(exec, static_cast<hipStream_t>(stream)));
  return CPQR_OK;
}

int cpqr_als_batch_threads(void* work) {
  BatchHeader hdr;
  int nt;
  CPQR_TRY(batch_lookup(work, 0, hdr, nt));
  return nt;
}

}  // extern "C"
