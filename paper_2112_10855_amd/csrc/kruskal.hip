// Kruskal-form input tensors (section 3.3.2).  X = [[mu; V_1 .. V_N]] with S
// terms (V_k: I_k x S column-major, mu: S weights) is never formed by the
// method: the Multi-TTM of mode n is again a Kruskal tensor with factors
// B_k = Q_k^T V_k (R x S) and B_n = V_n, so
//   W_n = Y_(n) Q_0 = V_n diag(mu) [(B_{a_{N-1}} (.) .. (.) B_{a_1})^T Q_0].
// With Q_0 in the structured form (I (x) Q_2)(I (x) Q_3) .. Q_{N-1} of the
// Khatri-Rao QR chain, eq. (kr-id) turns the bracket into a chain over the
// terms: c_1 = B_{a_1}(:, s), c_j = Q_j^T (B_{a_j}(:, s) (x) c_{j-1}), and row s
// of the bracket is c_{N-1}^T; Q_0 (R^{N-1} x R) is never formed either.
// For Alg. 1, M_n = X_(n) Z_n = V_n diag(mu) (Hadamard product over k != n of
// V_k^T A_k), and ||X||^2 = mu^T (Hadamard product of V_k^T V_k) mu.
//
// Every kernel here is small next to a dense pass over a tensor: the cross
// products are I_k R S multiply-adds, the chain (N-2) R^3 per term, W and M
// I_n R S.  All sums run in a fixed order (bitwise reproducible).
//
// kr_full_* forms the dense tensor (for the direct error, section 3.3.1, and
// for tests): the modes are split in two groups, the Khatri-Rao rows of each
// group are formed (L = left rows scaled by mu, Rt = right rows), and
// X_(left x right) = L Rt^T is an LDS-tiled FP64 product.
#include "common.h"

namespace cpqr {
namespace {

constexpr int KB = 256;

// P = U^T V (R x S, column-major): P[r + R s] = sum_i U[i + ldu r] V[i + ldv s].
__global__ __launch_bounds__(KB) void kr_cross_kernel(const double* __restrict__ U, int64_t ldu,
                                                      const double* __restrict__ V, int64_t ldv, int64_t I, int R,
                                                      int S, double* __restrict__ P) {
  const int64_t e = int64_t(blockIdx.x) * KB + threadIdx.x;
  if (e >= int64_t(R) * S) return;
  const int r = int(e % R);
  const int64_t s = e / R;
  const double* u = U + ldu * r;
  const double* v = V + ldv * s;
  double acc = 0.0;
  for (int64_t i = 0; i < I; ++i) acc += u[i] * v[i];
  P[e] = acc;
}

struct ModePtrs {
  const double* P[CPQR_MAX_MODES];
  int count;
};

// The chain of eq. (kr-id) for one term s per workgroup: c <- P[0](:, s), then
// for each step j: x = P[j](:, s) (x) c (c's index fastest), c <- Q_j^T x.
// Writes M[s + S r] = c[r] (M is S x R).  One thread per output entry of a
// step, R^2 multiply-adds each in index order.
__global__ __launch_bounds__(64) void kr_chain_kernel(ModePtrs mp, const double* __restrict__ Qc, int R, int S,
                                                      double* __restrict__ M) {
  __shared__ double c[CPQR_MAX_RANK];
  __shared__ double x[CPQR_MAX_RANK * CPQR_MAX_RANK];
  const int s = blockIdx.x, t = threadIdx.x;
  const int R2 = R * R;
  if (t < R) c[t] = mp.P[0][t + int64_t(R) * s];
  __syncthreads();
  for (int j = 1; j < mp.count; ++j) {
    const double* b = mp.P[j] + int64_t(R) * s;
    for (int k = t; k < R2; k += 64) x[k] = b[k / R] * c[k % R];
    __syncthreads();
    double acc = 0.0;
    if (t < R) {
      const double* q = Qc + (int64_t(j - 1) * R + t) * R2;  // column t of Q_j (R^2 x R)
      for (int k = 0; k < R2; ++k) acc += q[k] * x[k];
    }
    __syncthreads();
    if (t < R) c[t] = acc;
    __syncthreads();
  }
  if (t < R) M[s + int64_t(S) * t] = c[t];
}

// H[s + S r] = product over the given P's of P[r + R s] (in the order given).
__global__ __launch_bounds__(KB) void kr_hadamard_kernel(ModePtrs mp, int R, int S, double* __restrict__ H) {
  const int64_t e = int64_t(blockIdx.x) * KB + threadIdx.x;
  if (e >= int64_t(R) * S) return;
  const int r = int(e % R);
  const int64_t s = e / R;
  double v = 1.0;
  for (int m = 0; m < mp.count; ++m) v *= mp.P[m][e];
  H[s + int64_t(S) * r] = v;
}

// W[i + I r] = sum_s (V[i + ldv s] mu[s]) M[s + S r]: V_n diag(mu) M.
__global__ __launch_bounds__(KB) void kr_w_kernel(const double* __restrict__ V, int64_t ldv, int64_t I, int S,
                                                  const double* __restrict__ mu, const double* __restrict__ M, int R,
                                                  double* __restrict__ W) {
  const int64_t e = int64_t(blockIdx.x) * KB + threadIdx.x;
  if (e >= I * R) return;
  const int64_t i = e % I;
  const int r = int(e / I);
  const double* m = M + int64_t(S) * r;
  double acc = 0.0;
  for (int s = 0; s < S; ++s) acc += (V[i + ldv * s] * mu[s]) * m[s];
  W[e] = acc;
}

struct KrFactors {
  const double* V[CPQR_MAX_MODES];
  int64_t I[CPQR_MAX_MODES];
  int N;
};

// Fixed-order workgroup sum of v (KB threads); the result is valid in thread 0.
__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = KB / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// Partial sums of mu_s mu_t prod_k (V_k^T V_k)(s, t) over pairs e = s + S t.
__global__ __launch_bounds__(KB) void kr_norm2_partial(KrFactors f, int S, const double* __restrict__ mu,
                                                       double* __restrict__ part) {
  __shared__ double red[KB];
  const int64_t e = int64_t(blockIdx.x) * KB + threadIdx.x;
  double g = 0.0;
  if (e < int64_t(S) * S) {
    const int s = int(e % S), t = int(e / S);
    g = mu[s] * mu[t];
    for (int k = 0; k < f.N; ++k) {
      const double* a = f.V[k] + f.I[k] * s;
      const double* b = f.V[k] + f.I[k] * t;
      double d = 0.0;
      for (int64_t i = 0; i < f.I[k]; ++i) d += a[i] * b[i];
      g *= d;
    }
  }
  const double tot = block_sum(g, red);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(KB) void kr_sum_kernel(const double* __restrict__ part, int64_t count,
                                                    double* __restrict__ out) {
  __shared__ double red[KB];
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += KB) v += part[i];
  const double tot = block_sum(v, red);
  if (threadIdx.x == 0) out[0] = tot;
}

// Khatri-Rao rows of a group of modes [lo, hi) (lowest mode fastest), scaled
// by mu when given: Z[row + rows s] = (mu_s) prod_k V_k(i_k, s).
__global__ __launch_bounds__(KB) void kr_rows_kernel(KrFactors f, int lo, int hi, int64_t rows, int S,
                                                     const double* __restrict__ mu, double* __restrict__ Z) {
  const int64_t e = int64_t(blockIdx.x) * KB + threadIdx.x;
  if (e >= rows * S) return;
  const int64_t row = e % rows;
  const int64_t s = e / rows;
  double v = mu ? mu[s] : 1.0;
  int64_t rem = row;
  for (int k = lo; k < hi; ++k) {
    const int64_t ik = rem % f.I[k];
    rem /= f.I[k];
    v *= f.V[k][ik + f.I[k] * s];
  }
  Z[e] = v;
}

// X[il + IL ir] = sum_s L[il + IL s] Rt[ir + IR s]: 64 x 64 tiles, 256 threads
// of 4 x 4 outputs, 16 terms of s per LDS stage.
template <class TX>
__global__ __launch_bounds__(KB) void kr_full_gemm(const double* __restrict__ L, int64_t IL,
                                                   const double* __restrict__ Rt, int64_t IR, int S,
                                                   TX* __restrict__ X) {
  constexpr int TM = 64, TK = 16;
  __shared__ double la[TK][TM + 1];
  __shared__ double rb[TK][TM + 1];
  const int t = threadIdx.x;
  const int tx = t % 16, ty = t / 16;
  const int64_t i0 = int64_t(blockIdx.x) * TM, j0 = int64_t(blockIdx.y) * TM;
  double acc[4][4] = {};
  for (int s0 = 0; s0 < S; s0 += TK) {
    for (int e = t; e < TM * TK; e += KB) {
      const int m = e % TM, k = e / TM;
      const int64_t gi = i0 + m, gj = j0 + m;
      const int sk = s0 + k;
      la[k][m] = (gi < IL && sk < S) ? L[gi + IL * sk] : 0.0;
      rb[k][m] = (gj < IR && sk < S) ? Rt[gj + IR * sk] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TK; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = la[k][tx * 4 + u];
        b[u] = rb[k][ty * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t gj = j0 + ty * 4 + v;
    if (gj >= IR) continue;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t gi = i0 + tx * 4 + u;
      if (gi < IL) X[gi + IL * gj] = TX(acc[u][v]);
    }
  }
}

KrFactors factors_of(int N, const int64_t* I, const double* const* V) {
  KrFactors f{};
  f.N = N;
  for (int k = 0; k < N; ++k) {
    f.V[k] = V[k];
    f.I[k] = I[k];
  }
  return f;
}

// Split of the modes for kr_full: the smallest h with prod_{k<h} I_k >= sqrt(total).
int full_split(int N, const int64_t* I) {
  double total = 1.0;
  for (int k = 0; k < N; ++k) total *= double(I[k]);
  double left = 1.0;
  for (int h = 1; h < N; ++h) {
    left *= double(I[h - 1]);
    if (left * left >= total) return h;
  }
  return N > 1 ? N - 1 : 1;
}

}  // namespace

int kr_cross_enqueue(int64_t I, int R, int S, const double* U, int64_t ldu, const double* V, int64_t ldv,
                     double* P, hipStream_t s) {
  const int64_t cnt = int64_t(R) * S;
  hipLaunchKernelGGL(kr_cross_kernel, dim3(unsigned(ceil_div(cnt, KB))), dim3(KB), 0, s, U, ldu, V, ldv, I, R, S,
                     P);
  return check_launch("kr_cross");
}

int kr_chain_enqueue(int nP, const double* const* P, const double* Qc, int R, int S, double* M, hipStream_t s) {
  ModePtrs mp{};
  mp.count = nP;
  for (int j = 0; j < nP; ++j) mp.P[j] = P[j];
  hipLaunchKernelGGL(kr_chain_kernel, dim3(unsigned(S)), dim3(64), 0, s, mp, Qc, R, S, M);
  return check_launch("kr_chain");
}

int kr_hadamard_enqueue(int nP, const double* const* P, int R, int S, double* H, hipStream_t s) {
  ModePtrs mp{};
  mp.count = nP;
  for (int j = 0; j < nP; ++j) mp.P[j] = P[j];
  const int64_t cnt = int64_t(R) * S;
  hipLaunchKernelGGL(kr_hadamard_kernel, dim3(unsigned(ceil_div(cnt, KB))), dim3(KB), 0, s, mp, R, S, H);
  return check_launch("kr_hadamard");
}

int kr_w_enqueue(int64_t I, int S, int R, const double* V, int64_t ldv, const double* mu, const double* M,
                 double* W, hipStream_t s) {
  const int64_t cnt = I * R;
  hipLaunchKernelGGL(kr_w_kernel, dim3(unsigned(ceil_div(cnt, KB))), dim3(KB), 0, s, V, ldv, I, S, mu, M, R, W);
  return check_launch("kr_w");
}

size_t kr_norm2_work(int S) { return sizeof(double) * size_t(ceil_div(int64_t(S) * S, KB)); }

int kr_norm2_enqueue(int N, const int64_t* I, int S, const double* mu, const double* const* V, double* out,
                     void* work, hipStream_t s) {
  const int64_t nb = ceil_div(int64_t(S) * S, KB);
  double* part = static_cast<double*>(work);
  hipLaunchKernelGGL(kr_norm2_partial, dim3(unsigned(nb)), dim3(KB), 0, s, factors_of(N, I, V), S, mu, part);
  CPQR_TRY(check_launch("kr_norm2_partial"));
  hipLaunchKernelGGL(kr_sum_kernel, dim3(1), dim3(KB), 0, s, part, nb, out);
  return check_launch("kr_sum");
}

int64_t kr_full_grid_y(int N, const int64_t* I) {
  const int h = full_split(N, I);
  int64_t IR = 1;
  for (int k = h; k < N; ++k) IR *= I[k];
  return ceil_div(IR, 64);
}

size_t kr_full_work(int N, const int64_t* I, int S) {
  const int h = full_split(N, I);
  int64_t IL = 1, IR = 1;
  for (int k = 0; k < N; ++k) (k < h ? IL : IR) *= I[k];
  Carver cv(nullptr);
  cv.take<double>(size_t(IL) * S);
  cv.take<double>(size_t(IR) * S);
  return cv.bytes();
}

int kr_full_enqueue(int N, const int64_t* I, int S, const double* mu, const double* const* V, int xdtype,
                    void* X, void* work, hipStream_t s) {
  const int h = full_split(N, I);
  int64_t IL = 1, IR = 1;
  for (int k = 0; k < N; ++k) (k < h ? IL : IR) *= I[k];
  Carver cv(work);
  double* L = cv.take<double>(size_t(IL) * S);
  double* Rt = cv.take<double>(size_t(IR) * S);
  const KrFactors f = factors_of(N, I, V);
  hipLaunchKernelGGL(kr_rows_kernel, dim3(unsigned(ceil_div(IL * S, KB))), dim3(KB), 0, s, f, 0, h, IL, S, mu, L);
  CPQR_TRY(check_launch("kr_rows"));
  hipLaunchKernelGGL(kr_rows_kernel, dim3(unsigned(ceil_div(IR * S, KB))), dim3(KB), 0, s, f, h, N, IR, S,
                     static_cast<const double*>(nullptr), Rt);
  CPQR_TRY(check_launch("kr_rows"));
  const dim3 grd(unsigned(ceil_div(IL, 64)), unsigned(ceil_div(IR, 64)));
  if (xdtype == CPQR_F64)
    hipLaunchKernelGGL(kr_full_gemm<double>, grd, dim3(KB), 0, s, L, IL, Rt, IR, S, static_cast<double*>(X));
  else
    hipLaunchKernelGGL(kr_full_gemm<float>, grd, dim3(KB), 0, s, L, IL, Rt, IR, S, static_cast<float*>(X));
  return check_launch("kr_full_gemm");
}

}  // namespace cpqr
