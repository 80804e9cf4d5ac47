// The small FP64 steps of a CP-ALS-QR mode update (paper Alg. 2, section 3.1)
// and the error forms of section 3.3.1:
//   apply_q0     W = Y_(n) Q_0                   (split over the long K index)
//   solve        Ahat R_0^T = W by substitution, or Ahat = W U S^+ V^T from a
//                one-sided Jacobi SVD of R_0 (CP-ALS-QR-SVD)
//   normalize    lambda_r = ||Ahat(:,r)||_2, A = Ahat / lambda
//   errors       efficient (from W_N, R_0, R_N, lambda) and direct (stream X)
// Everything is FP64; reductions are two-level and deterministic.

#include "common.h"

namespace cpqr {
namespace {

constexpr int BLK = 256;

template <class T>
__device__ inline T block_sum(T v, T* sh) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T t = 0;
  const int nw = blockDim.x / 64;
  for (int i = 0; i < nw; ++i) t += sh[i];
  return t;
}

// ------------------------------------------------------------ apply Q_0
// part[split][i + c*In] = sum over this split's rho of Y[i + rho*In] Q0[rho + c*K]
// One thread per (row i, column c): a block covers 256 / RM rows, so that
// even a few thousand rows spread over a few hundred workgroups.
template <class TY, int RM>
__global__ __launch_bounds__(BLK) void apply_q0_kernel(const TY* __restrict__ Y,
                                                       const double* __restrict__ Q0, double* part,
                                                       int64_t In, int64_t K, int R, int64_t kchunk) {
  constexpr int RPB = BLK / RM;
  __shared__ double q0s[64][RM + 1];
  const int c = threadIdx.x % RM, ri = threadIdx.x / RM;
  const int64_t i = int64_t(blockIdx.x) * RPB + ri;
  const int64_t k0 = int64_t(blockIdx.y) * kchunk;
  const int64_t k1 = min(K, k0 + kchunk);
  const bool live = i < In && c < R;
  double acc = 0.0;
  for (int64_t t0 = k0; t0 < k1; t0 += 64) {
    const int nt = int(min<int64_t>(64, k1 - t0));
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * RM; e += BLK) {
      const int rr = e % 64, cc = e / 64;
      q0s[rr][cc] = (rr < nt && cc < R) ? Q0[t0 + rr + int64_t(cc) * K] : 0.0;
    }
    __syncthreads();
    if (live) {
      const TY* y = Y + i + t0 * In;
#pragma unroll 8
      for (int rr = 0; rr < nt; ++rr) acc += double(y[rr * In]) * q0s[rr][c];
    }
  }
  if (live) part[int64_t(blockIdx.y) * In * R + i + int64_t(c) * In] = acc;
}

// The same product for a long K (many rows of Q_0 per row of W), as a tiled
// matrix product: a workgroup forms a 64 x RM tile of W over its split of K,
// each thread 2 rows x RM/8 columns; Y (widened to FP64) and Q_0 pass through
// LDS 32 rows of Q_0 at a time, the next 32 prefetched in registers.
template <class TY, int RM>
__global__ __launch_bounds__(BLK) void apply_q0_tile(const TY* __restrict__ Y, const double* __restrict__ Q0,
                                                     double* __restrict__ part, int64_t In, int64_t K, int R,
                                                     int64_t kchunk) {
  constexpr int KS = 32, TR = 64, CPT = RM / 8;
  static_assert(BLK == 256, "thread mapping");
  __shared__ double ys[KS][TR];
  __shared__ double qs[KS][RM + 1];
  const int t = threadIdx.x;
  const int64_t i0 = int64_t(blockIdx.x) * TR;
  const int64_t k0 = int64_t(blockIdx.y) * kchunk;
  const int64_t k1 = min(K, k0 + kchunk);
  const int rp = t / 8, cq = t % 8;      // W rows i0 + 2 rp, + 1; columns cq CPT ...
  const int lr = t % TR, lg = t / TR;    // Y loads: row lr, Q_0 rows 8 lg ... 8 lg + 7
  const int qk = t % KS, qc = t / KS;    // Q_0 loads: row qk, columns qc CPT ...
  double acc[2][CPT];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int u = 0; u < CPT; ++u) acc[r][u] = 0.0;
  TY yv[8];
  double qv[CPT];
  auto gload = [&](int64_t kb) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t k = kb + lg * 8 + u;
      yv[u] = (i0 + lr < In && k < k1) ? Y[i0 + lr + k * In] : TY(0);
    }
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int c = qc * CPT + u;
      const int64_t k = kb + qk;
      qv[u] = (c < R && k < k1) ? Q0[k + int64_t(c) * K] : 0.0;
    }
  };
  gload(k0);
  for (int64_t kb = k0; kb < k1; kb += KS) {
    __syncthreads();  // the previous rows are consumed
#pragma unroll
    for (int u = 0; u < 8; ++u) ys[lg * 8 + u][lr] = double(yv[u]);
#pragma unroll
    for (int u = 0; u < CPT; ++u) qs[qk][qc * CPT + u] = qv[u];
    __syncthreads();
    if (kb + KS < k1) gload(kb + KS);
#pragma unroll 8
    for (int k = 0; k < KS; ++k) {
      const double a0 = ys[k][2 * rp], a1 = ys[k][2 * rp + 1];
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const double b = qs[k][cq * CPT + u];
        acc[0][u] += a0 * b;
        acc[1][u] += a1 * b;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int64_t i = i0 + 2 * rp + r;
    if (i >= In) continue;
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int c = cq * CPT + u;
      if (c < R) part[int64_t(blockIdx.y) * In * R + i + int64_t(c) * In] = acc[r][u];
    }
  }
}

// The same long-K product on the FP64 matrix cores (v_mfma_f64_16x16x4f64):
// a workgroup of eight wavefronts forms 128 rows x 16 NB columns of one
// split's partial.  Wavefront w owns rows 16 w .. 16 w + 15 of the 128: its
// A operand is Y (widened to FP64), lane (l16, kq) holding row l16 of K-row
// kq of a step; the B operand is Q_0, 64 rows at a time in one of two LDS
// buffers.  The next block's Y (in registers) and Q_0 (in registers, then
// LDS) are loaded while the current block is multiplied, so each block waits
// for loads issued one block earlier.  The MFMA leaves row kq + 4 v of its
// 16 x 16 result in value v of lane (l16, kq).
typedef double doublex4 __attribute__((ext_vector_type(4)));
template <class TY, int NB>
__global__ __launch_bounds__(512) void apply_q0_mfma(const TY* __restrict__ Y, const double* __restrict__ Q0,
                                                     double* __restrict__ part, int64_t In, int64_t K, int R,
                                                     int64_t kchunk) {
  constexpr int RMP = 16 * NB, KB = 64, NT = 512, QPT = KB * RMP / NT;
  __shared__ double qs[2][KB][RMP];
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64, l16 = lane % 16, kq = lane / 16;
  const int64_t r0 = int64_t(blockIdx.x) * 128 + 16 * w;  // first row of the wavefront's block
  const int64_t i = r0 + l16;
  const bool irow = i < In;
  const int64_t k0 = int64_t(blockIdx.y) * kchunk, k1 = min(K, k0 + kchunk);
  doublex4 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = doublex4{0.0, 0.0, 0.0, 0.0};
  // rows past k1 (or past the block's end) read as zeros, without a memory request
  auto load_y = [&](TY(&dst)[KB / 4], int64_t kb) {
#pragma unroll
    for (int st = 0; st < KB / 4; ++st) {
      const int64_t k = kb + 4 * st + kq;
      dst[st] = (irow && k < k1) ? Y[i + k * In] : TY(0);
    }
  };
  auto load_q = [&](double(&dst)[QPT], int64_t kb) {
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
      const int e = tid + u * NT, kk = e % KB, c = e / KB;
      const int64_t k = kb + kk;
      dst[u] = (c < R && k < k1) ? Q0[k + int64_t(c) * K] : 0.0;
    }
  };
  auto store_q = [&](const double(&src)[QPT], int b) {
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
      const int e = tid + u * NT;
      qs[b][e % KB][e / KB] = src[u];
    }
  };
  auto mult = [&](const TY(&ya)[KB / 4], int b) {
#pragma unroll
    for (int st = 0; st < KB / 4; ++st) {
      const double a = double(ya[st]);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, qs[b][4 * st + kq][16 * nb + l16], acc[nb], 0, 0, 0);
    }
  };
  TY ya0[KB / 4], ya1[KB / 4];
  double qv[QPT];
  load_y(ya0, k0);
  load_q(qv, k0);
  store_q(qv, 0);
  __syncthreads();
  for (int64_t kb = k0; kb < k1; kb += 2 * KB) {
    // block kb (LDS buffer 0, ya0) is ready; fetch block kb + KB meanwhile
    load_y(ya1, kb + KB);
    load_q(qv, kb + KB);
    mult(ya0, 0);
    store_q(qv, 1);
    __syncthreads();
    if (kb + KB >= k1) break;  // uniform
    // block kb + KB (buffer 1, ya1) is ready; fetch block kb + 2 KB meanwhile
    load_y(ya0, kb + 2 * KB);
    load_q(qv, kb + 2 * KB);
    mult(ya1, 1);
    store_q(qv, 0);
    __syncthreads();
  }
  double* o = part + int64_t(blockIdx.y) * In * R;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int c = 16 * nb + l16;
    if (c >= R) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t ii = r0 + kq + 4 * v;
      if (ii < In) o[ii + int64_t(c) * In] = acc[nb][v];
    }
  }
}

// Kernel choice and split of the apply-Q_0 sum: the tiled product once K
// exceeds 1024, with about 1024 workgroups and at most 128 splits.
struct ApplyPlan {
  bool tiled;
  int64_t kchunk, splits;
};

__global__ void sum_parts(const double* __restrict__ part, int splits, int64_t count, double* dst) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= count) return;
  double a = part[e];
  for (int t = 1; t < splits; ++t) a += part[int64_t(t) * count + e];
  dst[e] = a;
}

// ------------------------------------------------------------ solves
// Back substitution per row: R0 ahat = w  <=>  ahat^T R0^T = w^T.
template <int RM>
__global__ __launch_bounds__(BLK) void solve_tri_kernel(const double* __restrict__ W,
                                                        const double* __restrict__ R0, double* A,
                                                        int64_t In, int R, int* status) {
  __shared__ double r0[RM][RM + 1];
  for (int e = threadIdx.x; e < R * R; e += BLK) r0[e % R][e / R] = R0[e];
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0 && status) {
    int bad = 0;
    for (int j = 0; j < R; ++j) {
      const double d = r0[j][j];
      if (d == 0.0 || !isfinite(d)) bad = 1;
    }
    if (bad) atomicOr(status, CPQR_STATUS_SINGULAR);
  }
  const int64_t i = int64_t(blockIdx.x) * BLK + threadIdx.x;
  if (i >= In) return;
  double a[RM];
#pragma unroll
  for (int c = 0; c < RM; ++c) a[c] = c < R ? W[i + c * In] : 0.0;
#pragma unroll
  for (int j = RM - 1; j >= 0; --j) {
    if (j >= R) continue;
    double v = a[j];
#pragma unroll
    for (int c = j + 1; c < RM; ++c)
      if (c < R) v -= r0[j][c] * a[c];
    a[j] = v / r0[j][j];
  }
  bool nonfinite = false;
#pragma unroll
  for (int c = 0; c < RM; ++c)
    if (c < R) {
      A[i + c * In] = a[c];
      nonfinite |= !isfinite(a[c]);
    }
  if (nonfinite && status) atomicOr(status, CPQR_STATUS_NONFINITE);
}

// The same solve when the apply-Q_0 product was split over K: one thread per
// (row, column) of W adds up that entry's partials (stride In R) and stores
// W; each row's back substitution then reads its W row from LDS, and the
// solved rows leave through LDS so that the stores of A stay coalesced.
template <int RM, int KG = 1>
__global__ __launch_bounds__(KG * BLK) void sum_solve_kernel(const double* __restrict__ part, int splits,
                                                             const double* __restrict__ R0, double* W,
                                                             double* A, int64_t In, int R, int* status) {
  constexpr int RPB = BLK / RM;
  __shared__ double r0[RM][RM + 1];
  __shared__ double ws[RM][RPB + 1];
  __shared__ double red[KG][RM][RPB + 1];
  for (int e = threadIdx.x; e < R * R; e += KG * BLK) r0[e % R][e / R] = R0[e];
  const int g = threadIdx.x / BLK, tl = threadIdx.x % BLK;  // KG groups of BLK threads
  const int ri = tl % RPB, c = tl / RPB;
  const int64_t i = int64_t(blockIdx.x) * RPB + ri;
  const bool live = i < In && c < R;
  const int64_t e = i + int64_t(c) * In;
  double w = 0.0;
  if (live) {  // group g adds partials g, g + KG, ...; one group adds them all in order
#pragma unroll 8
    for (int t = g; t < splits; t += KG) w += part[int64_t(t) * In * R + e];
  }
  red[g][c][ri] = w;
  __syncthreads();
  if (g == 0) {
    double sum = red[0][c][ri];
#pragma unroll
    for (int u = 1; u < KG; ++u) sum += red[u][c][ri];
    if (live) W[e] = sum;
    ws[c][ri] = sum;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0 && status) {
    int bad = 0;
    for (int j = 0; j < R; ++j) {
      const double d = r0[j][j];
      if (d == 0.0 || !isfinite(d)) bad = 1;
    }
    if (bad) atomicOr(status, CPQR_STATUS_SINGULAR);
  }
  if (threadIdx.x < RPB && i < In) {
    double a[RM];
#pragma unroll
    for (int k = 0; k < RM; ++k) a[k] = ws[k][ri];
#pragma unroll
    for (int j = RM - 1; j >= 0; --j) {
      if (j >= R) continue;
      double v = a[j];
#pragma unroll
      for (int k = j + 1; k < RM; ++k)
        if (k < R) v -= r0[j][k] * a[k];
      a[j] = v / r0[j][j];
    }
    bool nonfinite = false;
#pragma unroll
    for (int k = 0; k < RM; ++k) {
      ws[k][ri] = a[k];
      if (k < R) nonfinite |= !isfinite(a[k]);
    }
    if (nonfinite && status) atomicOr(status, CPQR_STATUS_NONFINITE);
  }
  __syncthreads();
  if (g == 0 && live) A[i + int64_t(c) * In] = ws[c][ri];
}

// Apply Q_0 and solve in one launch when the product is split over at most
// KG parts of K: group g of BLK threads forms the partial of rows
// [g kchunk, (g + 1) kchunk) of Q_0 (the split kernel's chunk, in the same
// order), the partials meet in LDS and are added in split order, so W and A
// are those of the split product followed by sum_solve_kernel.  The
// solve is sum_solve_kernel's: each row's back substitution in LDS.
template <class TY, int RM, int KG>
__global__ __launch_bounds__(KG * BLK) void apply_solve_kernel(const TY* __restrict__ Y,
                                                               const double* __restrict__ Q0,
                                                               const double* __restrict__ R0, double* W,
                                                               double* A, int64_t In, int64_t K, int R,
                                                               int64_t kchunk, int* status) {
  constexpr int RPB = BLK / RM, KC = 32;
  __shared__ double q0s[KG][KC][RM + 1];
  __shared__ double red[KG][RM][RPB + 1];
  __shared__ double r0[RM][RM + 1];
  __shared__ double ws[RM][RPB + 1];
  const int g = threadIdx.x / BLK, tl = threadIdx.x % BLK;
  const int ri = tl % RPB, c = tl / RPB;
  const int64_t i = int64_t(blockIdx.x) * RPB + ri;
  const bool live = i < In && c < R;
  const int64_t k0 = int64_t(g) * kchunk, k1 = min(K, k0 + kchunk);
  const int64_t nsteps = (kchunk + KC - 1) / KC;  // the same in every group
  double acc = 0.0;
  for (int64_t st = 0; st < nsteps; ++st) {
    const int64_t t0 = k0 + st * KC;
    const int nt = int(max<int64_t>(0, min<int64_t>(KC, k1 - t0)));
    __syncthreads();
    for (int e = tl; e < KC * RM; e += BLK) {
      const int rr = e % KC, cc = e / KC;
      q0s[g][rr][cc] = (rr < nt && cc < R) ? Q0[t0 + rr + int64_t(cc) * K] : 0.0;
    }
    __syncthreads();
    if (live) {
      const TY* y = Y + i + t0 * In;
#pragma unroll 8
      for (int rr = 0; rr < nt; ++rr) acc += double(y[rr * In]) * q0s[g][rr][c];
    }
  }
  red[g][c][ri] = acc;
  for (int e = threadIdx.x; e < R * R; e += KG * BLK) r0[e % R][e / R] = R0[e];
  __syncthreads();
  if (g == 0) {
    double w = 0.0;
#pragma unroll
    for (int t = 0; t < KG; ++t) w += red[t][c][ri];
    if (live) W[i + int64_t(c) * In] = w;
    ws[c][ri] = live ? w : 0.0;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0 && status) {
    int bad = 0;
    for (int j = 0; j < R; ++j) {
      const double d = r0[j][j];
      if (d == 0.0 || !isfinite(d)) bad = 1;
    }
    if (bad) atomicOr(status, CPQR_STATUS_SINGULAR);
  }
  if (threadIdx.x < RPB && i < In) {
    double a[RM];
#pragma unroll
    for (int k = 0; k < RM; ++k) a[k] = ws[k][ri];
#pragma unroll
    for (int j = RM - 1; j >= 0; --j) {
      if (j >= R) continue;
      double v = a[j];
#pragma unroll
      for (int k = j + 1; k < RM; ++k)
        if (k < R) v -= r0[j][k] * a[k];
      a[j] = v / r0[j][j];
    }
    bool nonfinite = false;
#pragma unroll
    for (int k = 0; k < RM; ++k) {
      ws[k][ri] = a[k];
      if (k < R) nonfinite |= !isfinite(a[k]);
    }
    if (nonfinite && status) atomicOr(status, CPQR_STATUS_NONFINITE);
  }
  __syncthreads();
  if (g == 0 && live) A[i + int64_t(c) * In] = ws[c][ri];
}

// One-sided Jacobi SVD of an R x R matrix B (R <= RM <= 32) in one wavefront,
// then M = U S^+ V^T = sum over kept j of (B v_j) v_j^T / sigma_j^2, with
// singular values <= rtol * sigma_max dropped (B = R_0: the transposed
// pseudo-inverse of R_0; B = S_n symmetric: pinv(S_n)).  The RM/2 column
// pairs of a round-robin round rotate at once, each on 64/(RM/2) lanes that
// hold its rows; a pair's three dot products are butterfly sums over those
// lanes, which leave the same bits on all of them, so every lane of a pair
// takes the same rotation.  Columns live in LDS between rounds.
template <int RM>
__global__ __launch_bounds__(64) void svd_pinv_kernel(const double* __restrict__ B, int R, double rtol,
                                                      double* M, int* kept_out, int* status) {
  constexpr int NP = RM / 2;
  constexpr int LPP = 64 / NP;
  constexpr int RPL = (RM + LPP - 1) / LPP;
  __shared__ double G[RM][RM + 1];  // columns of B V
  __shared__ double Vm[RM][RM + 1];
  __shared__ double sig[RM];
  const int lane = threadIdx.x;
  const int pr = lane / LPP, sub = lane % LPP;
  for (int e = lane; e < RM * RM; e += 64) {
    const int i = e % RM, j = e / RM;
    G[i][j] = (i < R && j < R) ? B[i + j * R] : 0.0;
    Vm[i][j] = (i == j && i < R) ? 1.0 : 0.0;
  }
  const int Rp = R + (R & 1);  // even number of players for the round robin
  const double eps = 2.220446049250313e-16;
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int round = 0; round < Rp - 1; ++round) {
      __syncthreads();
      int p = -1, q = -1;
      if (pr < Rp / 2) {
        auto pos = [&](int k) { return k == 0 ? 0 : ((k - 1 + round) % (Rp - 1)) + 1; };
        p = pos(pr);
        q = pos(Rp - 1 - pr);
        if (p > q) { const int t = p; p = q; q = t; }
      }
      const bool active = p >= 0 && q < R;
      double gp[RPL], gq[RPL];
      double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int row = sub + t * LPP;
        const bool ok = active && row < R;
        gp[t] = ok ? G[row][p] : 0.0;
        gq[t] = ok ? G[row][q] : 0.0;
        al += gp[t] * gp[t];
        be += gq[t] * gq[t];
        ga += gp[t] * gq[t];
      }
#pragma unroll
      for (int off = LPP / 2; off > 0; off >>= 1) {
        al += __shfl_xor(al, off, LPP);
        be += __shfl_xor(be, off, LPP);
        ga += __shfl_xor(ga, off, LPP);
      }
      if (active && fabs(ga) > eps * sqrt(al * be) && ga != 0.0) {
        const double zeta = (be - al) / (2.0 * ga);
        const double tn = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + tn * tn), sn = c * tn;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int row = sub + t * LPP;
          if (row < R) {
            G[row][p] = c * gp[t] - sn * gq[t];
            G[row][q] = sn * gp[t] + c * gq[t];
            const double vp = Vm[row][p], vq = Vm[row][q];
            Vm[row][p] = c * vp - sn * vq;
            Vm[row][q] = sn * vp + c * vq;
          }
        }
        rotated = true;
      }
    }
    __syncthreads();
    if (!__any(rotated)) break;
  }
  if (lane < RM) {
    double s2 = 0.0;
    for (int i = 0; i < R; ++i) s2 += G[i][lane] * G[i][lane];
    sig[lane] = lane < R ? sqrt(s2) : 0.0;
  }
  __syncthreads();
  double smax = 0.0;
  for (int j = 0; j < R; ++j) smax = fmax(smax, sig[j]);
  const double tau = rtol * smax;
  // U_j = G(:,j) / sigma_j
  for (int e = lane; e < R * R; e += 64) {
    const int a = e % R, b = e / R;
    double v = 0.0;
    for (int j = 0; j < R; ++j)
      if (sig[j] > tau && sig[j] > 0.0) v += G[a][j] * Vm[b][j] / (sig[j] * sig[j]);
    M[a + b * R] = v;
  }
  if (lane == 0) {
    int kept = 0;
    for (int j = 0; j < R; ++j) kept += (sig[j] > tau && sig[j] > 0.0) ? 1 : 0;
    *kept_out = kept;
    if (kept < R && status) atomicOr(status, CPQR_STATUS_TRUNCATED);
  }
}

// Ahat = W M (row by row)
template <int RM>
__global__ __launch_bounds__(BLK) void rowmul_kernel(const double* __restrict__ W,
                                                     const double* __restrict__ Mm, double* A,
                                                     int64_t In, int R, int* status) {
  __shared__ double m[RM][RM];
  for (int e = threadIdx.x; e < R * R; e += BLK) m[e % R][e / R] = Mm[e];
  __syncthreads();
  const int64_t i = int64_t(blockIdx.x) * BLK + threadIdx.x;
  if (i >= In) return;
  double w[RM];
#pragma unroll
  for (int c = 0; c < RM; ++c) w[c] = c < R ? W[i + c * In] : 0.0;
  bool nonfinite = false;
#pragma unroll
  for (int b = 0; b < RM; ++b) {
    if (b >= R) continue;
    double v = 0.0;
#pragma unroll
    for (int a = 0; a < RM; ++a)
      if (a < R) v += w[a] * m[a][b];
    A[i + b * In] = v;
    nonfinite |= !isfinite(v);
  }
  if (nonfinite && status) atomicOr(status, CPQR_STATUS_NONFINITE);
}

// lambda_c = ||A(:,c)||, A(:,c) /= lambda_c (one workgroup per column)
__global__ __launch_bounds__(BLK) void normalize_kernel(double* A, double* lambda, int64_t In,
                                                        int* status) {
  __shared__ double sh[BLK / 64];
  const int c = blockIdx.x;
  double* col = A + int64_t(c) * In;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < In; i += BLK) s += col[i] * col[i];
  const double nrm = sqrt(block_sum(s, sh));
  if (threadIdx.x == 0) {
    lambda[c] = nrm;
    if (nrm == 0.0 && status) atomicOr(status, CPQR_STATUS_ZERO_COLUMN);
  }
  if (nrm > 0.0) {
    const double inv = 1.0 / nrm;
    for (int64_t i = threadIdx.x; i < In; i += BLK) col[i] *= inv;
  }
}

// ------------------------------------------------------------ diagonal columns
// W[i + In r] = Y[i + In r dstep]: the columns of Y_(n) whose every
// Kronecker index equals r (dstep = 1 + R + .. + R^{N-2}).
template <class TY>
__global__ __launch_bounds__(BLK) void diag_cols_kernel(const TY* __restrict__ Y, int64_t In, int64_t dstep, int R,
                                                        double* __restrict__ W) {
  const int64_t e = int64_t(blockIdx.x) * BLK + threadIdx.x;
  if (e >= In * R) return;
  const int64_t i = e % In, r = e / In;
  W[e] = double(Y[i + In * r * dstep]);
}

// ------------------------------------------------------------ structured Q_0
// One step of forming Q_0 = (I kron Q_2) .. (I kron Q_{N-2}) Q_{N-1} from the
// right: out = (I_m kron Qj) G, i.e. out[k + R^2 s, c] = sum_j Qj[k, j] G[j + R s, c]
// (Qj R^2 x R, G (R m) x R, out (R^2 m) x R, all column-major); one thread per
// entry of out.
__global__ __launch_bounds__(BLK) void expand_q0_kernel(const double* __restrict__ Qj, const double* __restrict__ G,
                                                        int64_t m, int R, double* __restrict__ out) {
  const int64_t rows = int64_t(R) * R * m;
  const int64_t e = int64_t(blockIdx.x) * BLK + threadIdx.x;
  if (e >= rows * R) return;
  const int64_t row = e % rows;
  const int c = int(e / rows);
  const int64_t k = row % (int64_t(R) * R), s = row / (int64_t(R) * R);
  const double* g = G + int64_t(R) * s + int64_t(R) * m * c;
  double v = 0.0;
  for (int j = 0; j < R; ++j) v += Qj[k + int64_t(R) * R * j] * g[j];
  out[e] = v;
}

// ------------------------------------------------------------ errors
// relerr = sqrt(max(x2 - 2 ip + nn, 0) / x2) with
// ip = <W, Ahat R0^T>, Ahat = A diag(lambda), nn = <R0^T R0, diag(l) RN^T RN diag(l)>
template <int RM>
__global__ __launch_bounds__(BLK) void error_efficient_kernel(
    const double* __restrict__ W, const double* __restrict__ A, const double* __restrict__ lam,
    const double* __restrict__ R0, const double* __restrict__ RN, int64_t In, int R, double* __restrict__ part) {
  // one row per thread: block b sums rows 256 b ... of ip; block 0 also forms nn
  __shared__ double r0[RM][RM + 1];
  __shared__ double l[RM];
  __shared__ double sh[BLK / 64];
  for (int e = threadIdx.x; e < R * R; e += BLK) r0[e % R][e / R] = R0[e];
  for (int e = threadIdx.x; e < R; e += BLK) l[e] = lam[e];
  __syncthreads();
  double ip = 0.0;
  const int64_t i = int64_t(blockIdx.x) * BLK + threadIdx.x;
  if (i < In) {
    double ah[RM];
#pragma unroll
    for (int k = 0; k < RM; ++k) ah[k] = k < R ? A[i + k * In] * l[k] : 0.0;
#pragma unroll
    for (int c = 0; c < RM; ++c) {
      if (c >= R) continue;
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < RM; ++k)
        if (k >= c && k < R) v += ah[k] * r0[c][k];
      ip += W[i + c * In] * v;
    }
  }
  ip = block_sum(ip, sh);
  if (threadIdx.x == 0) part[1 + blockIdx.x] = ip;
  if (blockIdx.x != 0) return;
  double nn = 0.0;
  for (int e = threadIdx.x; e < R * R; e += BLK) {
    const int a = e % R, b = e / R;
    double g0 = 0.0, gn = 0.0;
    for (int k = 0; k < R; ++k) {
      g0 += r0[k][a] * r0[k][b];
      gn += RN[k + a * R] * RN[k + b * R];
    }
    nn += g0 * l[a] * l[b] * gn;
  }
  nn = block_sum(nn, sh);
  if (threadIdx.x == 0) part[0] = nn;
}

// sqrt(max(r2, 0) / x2); a NaN residual stays NaN (a non-finite model must
// not read as a perfect fit)
__device__ __forceinline__ double rel_from_r2(double r2, double x2) {
  return isnan(r2) ? r2 : sqrt((r2 > 0.0 ? r2 : 0.0) / x2);
}

// relerr from the partial sums (block order fixed): nb partial ip's after nn
__global__ void error_efficient_final(const double* __restrict__ part, int nb, const double* __restrict__ xnorm2,
                                      double* relerr) {
  double ip = 0.0;
  for (int b = 0; b < nb; ++b) ip += part[1 + b];
  const double x2 = *xnorm2;
  const double r2 = x2 - 2.0 * ip + part[0];
  *relerr = rel_from_r2(r2, x2);
}

__global__ void error_from_fit_kernel(const double* fit, double* relerr) {
  *relerr = rel_from_r2(fit[0], fit[1]);
}

__global__ void fill_kernel(double* p, int64_t count, double v) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < count) p[e] = v;
}

// partial sums of x^2 (grid-stride), then a one-block final sum
template <class TX>
__global__ __launch_bounds__(BLK) void norm2_partial(const TX* __restrict__ X, int64_t count,
                                                     double* part) {
  __shared__ double sh[BLK / 64];
  double s = 0.0;
  for (int64_t e = int64_t(blockIdx.x) * BLK + threadIdx.x; e < count; e += int64_t(gridDim.x) * BLK) {
    const double v = double(X[e]);
    s += v * v;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(BLK) void sum_final(const double* part, int n, int stride, double* out) {
  __shared__ double sh[BLK / 64];
  for (int c = 0; c < stride; ++c) {
    double s = 0.0;
    for (int e = threadIdx.x; e < n; e += BLK) s += part[int64_t(e) * stride + c];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[c] = s;
    __syncthreads();
  }
}

struct FactorPtrs {
  const double* A[CPQR_MAX_MODES];
  int64_t I[CPQR_MAX_MODES];
};

// Direct residual: X viewed as [I0, S]; workgroup = 256 rows x CS columns.
// The coefficients lambda_r prod_{k>0} A_k(i_k, r) of CS columns are built in
// LDS; each thread keeps its row of A_0 in registers.
constexpr int CS = 64;
template <class TX, int RM>
__global__ __launch_bounds__(BLK) void fit_direct_kernel(const TX* __restrict__ X, FactorPtrs f,
                                                         int N, const double* __restrict__ lam,
                                                         int R, int64_t I0, int64_t S,
                                                         double* part) {
  __shared__ double coef[CS][RM + 1];
  __shared__ double sh[BLK / 64];
  const int64_t i = int64_t(blockIdx.y) * BLK + threadIdx.x;
  const int64_t s0 = int64_t(blockIdx.x) * CS;
  const int ns = int(min<int64_t>(CS, S - s0));
  // every slot up to RM is written (zero beyond R): the row loop below runs
  // to RM, and 0 times stale LDS contents could be NaN
  for (int e = threadIdx.x; e < CS * RM; e += BLK) {
    const int sl = e % CS, r = e / CS;
    double v = 0.0;
    if (sl < ns && r < R) {
      v = lam[r];
      int64_t rest = s0 + sl;
      for (int k = 1; k < N; ++k) {
        const int64_t ik = rest % f.I[k];
        rest /= f.I[k];
        v *= f.A[k][ik + int64_t(r) * f.I[k]];
      }
    }
    coef[sl][r] = v;
  }
  __syncthreads();
  double d2 = 0.0, x2 = 0.0;
  if (i < I0) {
    double a[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) a[r] = r < R ? f.A[0][i + int64_t(r) * I0] : 0.0;
    for (int sl = 0; sl < ns; ++sl) {
      double mdl = 0.0;
#pragma unroll
      for (int r = 0; r < RM; ++r) mdl += a[r] * coef[sl][r];
      const double x = double(X[i + (s0 + sl) * I0]);
      const double d = x - mdl;
      d2 += d * d;
      x2 += x * x;
    }
  }
  d2 = block_sum(d2, sh);
  x2 = block_sum(x2, sh);
  if (threadIdx.x == 0) {
    const int64_t b = int64_t(blockIdx.y) * gridDim.x + blockIdx.x;  // < gridDim.x * gridDim.y
    part[2 * b] = d2;
    part[2 * b + 1] = x2;
  }
}

int64_t apply_splits(int64_t In, int64_t K, int R) {
  const int64_t rb = ceil_div(In, BLK / round_rank(R));
  int64_t sp = std::max<int64_t>(1, std::min<int64_t>(ceil_div(1024, rb), ceil_div(K, 64)));
  return std::min<int64_t>(sp, 512);
}

ApplyPlan apply_plan(int64_t In, int64_t K, int R) {
  ApplyPlan ap{};
  ap.tiled = K > 1024;
  const int64_t sp = ap.tiled ? std::max<int64_t>(1, std::min<int64_t>({ceil_div(1024, ceil_div(In, 64)), 128,
                                                                         ceil_div(K, 32)}))
                              : apply_splits(In, K, R);
  const int64_t q = ap.tiled ? 32 : 64;
  ap.kchunk = ceil_div(ceil_div(K, sp), q) * q;
  ap.splits = ceil_div(K, ap.kchunk);
  return ap;
}

// Launches the apply-Q_0 kernel of the plan; out holds one In x R block per split.
void launch_apply(const ApplyPlan& ap, int64_t In, int64_t K, int R, int ydtype, const void* Y, const double* Q0,
                  double* out, hipStream_t s) {
  const int RM = round_rank(R);
  if (ap.tiled && RM >= 16) {  // FP64 matrix cores, 128 rows per workgroup
    const dim3 grd(unsigned(ceil_div(In, 128)), unsigned(ap.splits));
#define APPLYM(TY, NBV)                                                                                     \
  hipLaunchKernelGGL((apply_q0_mfma<TY, NBV>), grd, dim3(512), 0, s, static_cast<const TY*>(Y), Q0, out, In, K, R, \
                     ap.kchunk)
    if (ydtype == CPQR_F64) {
      if (RM == 16) APPLYM(double, 1); else APPLYM(double, 2);
    } else {
      if (RM == 16) APPLYM(float, 1); else APPLYM(float, 2);
    }
#undef APPLYM
    return;
  }
  if (ap.tiled) {
    const dim3 grd(unsigned(ceil_div(In, 64)), unsigned(ap.splits));
#define APPLYT(TY, RMV)                                                                                    \
  hipLaunchKernelGGL((apply_q0_tile<TY, RMV>), grd, dim3(BLK), 0, s, static_cast<const TY*>(Y), Q0, out, In, K, \
                     R, ap.kchunk)
    if (ydtype == CPQR_F64) {
      if (RM == 8) APPLYT(double, 8); else if (RM == 16) APPLYT(double, 16); else APPLYT(double, 32);
    } else {
      if (RM == 8) APPLYT(float, 8); else if (RM == 16) APPLYT(float, 16); else APPLYT(float, 32);
    }
#undef APPLYT
    return;
  }
  const dim3 grd(unsigned(ceil_div(In, BLK / RM)), unsigned(ap.splits));
#define APPLY(TY, RMV)                                                                                     \
  hipLaunchKernelGGL((apply_q0_kernel<TY, RMV>), grd, dim3(BLK), 0, s, static_cast<const TY*>(Y), Q0, out, In, K, \
                     R, ap.kchunk)
  if (ydtype == CPQR_F64) {
    if (RM == 8) APPLY(double, 8); else if (RM == 16) APPLY(double, 16); else APPLY(double, 32);
  } else {
    if (RM == 8) APPLY(float, 8); else if (RM == 16) APPLY(float, 16); else APPLY(float, 32);
  }
#undef APPLY
}

constexpr int NORM_BLOCKS = 2048;

// ------------------------------------------------------------ Alg. 1 (normal equations)
// The value of v on lane j (j uniform across the wavefront).
__device__ inline double lane_value(double v, int j) {
  const long long b = __builtin_bit_cast(long long, v);
  const unsigned lo = __builtin_amdgcn_readlane(int(b), j);
  const unsigned hi = __builtin_amdgcn_readlane(int(b >> 32), j);
  return __builtin_bit_cast(double, (long long)((static_cast<unsigned long long>(hi) << 32) | lo));
}

// S_n = Hadamard product of the Gram matrices G_k = A_k^T A_k over k != n
// (section 2.3), multiplied in increasing k; for the Cholesky solve also the
// upper factor U of S_n = U^T U (right-looking, one column per step).  One
// workgroup; a non-positive or non-finite pivot sets CPQR_STATUS_SINGULAR.
__global__ __launch_bounds__(BLK) void ne_factor_kernel(const double* __restrict__ G, int N, int n, int R,
                                                        int chol, double* S, double* U, int* status) {
  __shared__ double s[32][33];
  __shared__ double u[32][33];
  __shared__ double sd[32];
  for (int e = threadIdx.x; e < R * R; e += BLK) {
    const int a = e % R, b = e / R;
    double v = 1.0;
    for (int k = 0; k < N; ++k)
      if (k != n) v *= G[int64_t(k) * R * R + e];
    s[a][b] = v;
    S[e] = v;
    if (a == b) sd[a] = v;
  }
  if (!chol) return;
  bool bad = false;
  for (int j = 0; j < R; ++j) {
    __syncthreads();
    const double piv = s[j][j];
    bad |= !(piv > 0.0) || !isfinite(piv);
    const double rj = sqrt(piv);
    if (threadIdx.x < R) {
      const int k = threadIdx.x;
      u[j][k] = k < j ? 0.0 : (k == j ? rj : s[j][k] / rj);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < R * R; e += BLK) {
      const int a = e % R, b = e / R;
      if (a > j && b >= a) s[a][b] -= u[j][a] * u[j][b];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < R * R; e += BLK) U[e] = u[e % R][e / R];
  if (!status) return;
  if (bad) {
    if (threadIdx.x == 0) atomicOr(status, CPQR_STATUS_SINGULAR);
    return;
  }
  if (threadIdx.x >= 64) return;
  // A lower bound on cond(S_n) by inverse iteration, in wavefront 0: for unit
  // x, ||S_n^-1 x|| <= 1 / lambda_min and max_j S_jj <= lambda_max.  Four
  // steps from the all-ones vector, each two substitutions with U done
  // column by column: lane i holds x_i and column and row i of U.
  const int lane = threadIdx.x;
  double ucol[32], urow[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    ucol[j] = (lane < R && j < R) ? u[j][lane] : 0.0;
    urow[j] = (lane < R && j < R) ? u[lane][j] : 0.0;
  }
  const double dinv = lane < R ? 1.0 / u[lane][lane] : 0.0;
  double smax = lane < R ? sd[lane] : 0.0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) smax = fmax(smax, __shfl_xor(smax, off, 64));
  double x = lane < R ? 1.0 / sqrt(double(R)) : 0.0, est = 0.0;
  for (int it = 0; it < 4; ++it) {
#pragma unroll
    for (int j = 0; j < 32; ++j) {  // U^T y = x
      if (j >= R) continue;
      const double yj = lane_value(x * dinv, j);
      if (lane == j) x = yj;
      else if (lane > j) x -= ucol[j] * yj;
    }
#pragma unroll
    for (int j = 31; j >= 0; --j) {  // U z = y
      if (j >= R) continue;
      const double zj = lane_value(x * dinv, j);
      if (lane == j) x = zj;
      else if (lane < j) x -= urow[j] * zj;
    }
    double n2 = x * x;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) n2 += __shfl_xor(n2, off, 64);
    const double nrm = sqrt(n2);
    est = fmax(est, smax * nrm);
    x /= nrm;
  }
  if (lane == 0 && est > 1e4) atomicOr(status, CPQR_STATUS_ILL_CONDITIONED);
}

// Row i of the MTTKRP M_n = X_(n) Z_n is read off Y_(n) = X_(n) (A_N kron ..
// kron A_1 without A_n): column r of Z_n is the Kronecker column whose every
// index is r, at position r (1 + R + .. + R^{N-2}) = r * dstep.  Then Ahat(i,:)
// solves Ahat S_n = M_n: S_n = U^T U by a forward and a back substitution
// (chol), or Ahat = M_n P with P = pinv(S_n).  One thread per row.
template <class TY, int RM>
__global__ __launch_bounds__(BLK) void ne_rows_kernel(const TY* __restrict__ Y, int64_t In, int64_t dstep,
                                                      const double* __restrict__ F, int chol, int R,
                                                      double* __restrict__ M, double* __restrict__ A,
                                                      int* status) {
  __shared__ double f[RM][RM + 1];
  for (int e = threadIdx.x; e < R * R; e += BLK) f[e % R][e / R] = F[e];
  __syncthreads();
  const int64_t i = int64_t(blockIdx.x) * BLK + threadIdx.x;
  if (i >= In) return;
  double m[RM], a[RM];
#pragma unroll
  for (int c = 0; c < RM; ++c) {
    m[c] = c < R ? double(Y[i + int64_t(c) * dstep * In]) : 0.0;
    if (c < R) M[i + int64_t(c) * In] = m[c];
  }
  if (chol) {
    // U^T y = m (forward), then U a = y (back)
#pragma unroll
    for (int j = 0; j < RM; ++j) {
      if (j >= R) continue;
      double v = m[j];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= f[k][j] * a[k];
      a[j] = v / f[j][j];
    }
#pragma unroll
    for (int j = RM - 1; j >= 0; --j) {
      if (j >= R) continue;
      double v = a[j];
#pragma unroll
      for (int k = j + 1; k < RM; ++k)
        if (k < R) v -= f[j][k] * a[k];
      a[j] = v / f[j][j];
    }
  } else {
#pragma unroll
    for (int b = 0; b < RM; ++b) {
      double v = 0.0;
#pragma unroll
      for (int c = 0; c < RM; ++c)
        if (c < R && b < R) v += m[c] * f[c][b];
      a[b] = v;
    }
  }
  bool nonfinite = false;
#pragma unroll
  for (int b = 0; b < RM; ++b) {
    if (b >= R) continue;
    A[i + int64_t(b) * In] = a[b];
    nonfinite |= !isfinite(a[b]);
  }
  if (nonfinite && status) atomicOr(status, CPQR_STATUS_NONFINITE);
}

// G = A^T A for an In x R column-major factor; one workgroup per entry, so
// the two halves of the symmetric matrix come out bit-identical.
__global__ __launch_bounds__(BLK) void gram_kernel(const double* __restrict__ A, int64_t In, int R, double* G) {
  __shared__ double sh[BLK / 64];
  const int a = blockIdx.x % R, b = blockIdx.x / R;
  const double* ca = A + int64_t(a) * In;
  const double* cb = A + int64_t(b) * In;
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < In; i += BLK) v += ca[i] * cb[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) G[blockIdx.x] = v;
}

// Alg. 1's efficient error: ip = <M_N, Ahat_N> = sum M(i,r) A(i,r) lambda_r,
// partial sums per 256 rows, then nn = <S_N, diag(lambda) G_N diag(lambda)>
// and relerr = sqrt(max(x2 - 2 ip + nn, 0) / x2) in one workgroup.
__global__ __launch_bounds__(BLK) void ne_err_partial(const double* __restrict__ M, const double* __restrict__ A,
                                                      const double* __restrict__ lam, int64_t In, int R,
                                                      double* part) {
  __shared__ double sh[BLK / 64];
  const int64_t i = int64_t(blockIdx.x) * BLK + threadIdx.x;
  double v = 0.0;
  if (i < In)
    for (int c = 0; c < R; ++c) v += M[i + int64_t(c) * In] * A[i + int64_t(c) * In] * lam[c];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ __launch_bounds__(BLK) void ne_err_final(const double* __restrict__ part, int nb,
                                                    const double* __restrict__ S, const double* __restrict__ GN,
                                                    const double* __restrict__ lam, int R,
                                                    const double* __restrict__ xnorm2, double* relerr) {
  __shared__ double sh[BLK / 64];
  double ip = 0.0, nn = 0.0;
  for (int b = threadIdx.x; b < nb; b += BLK) ip += part[b];
  for (int e = threadIdx.x; e < R * R; e += BLK) {
    const int a = e % R, b = e / R;
    nn += S[e] * (lam[a] * GN[e] * lam[b]);
  }
  ip = block_sum(ip, sh);
  __syncthreads();
  nn = block_sum(nn, sh);
  if (threadIdx.x == 0) {
    const double x2 = *xnorm2;
    *relerr = rel_from_r2(x2 - 2.0 * ip + nn, x2);
  }
}

int launch_svd_pinv(const double* B, int R, double rtol, double* M, int* kept, int* status, hipStream_t s) {
  const int RM = round_rank(R);
  if (RM == 8)
    hipLaunchKernelGGL(svd_pinv_kernel<8>, dim3(1), dim3(64), 0, s, B, R, rtol, M, kept, status);
  else if (RM == 16)
    hipLaunchKernelGGL(svd_pinv_kernel<16>, dim3(1), dim3(64), 0, s, B, R, rtol, M, kept, status);
  else
    hipLaunchKernelGGL(svd_pinv_kernel<32>, dim3(1), dim3(64), 0, s, B, R, rtol, M, kept, status);
  return check_launch("svd_pinv");
}

}  // namespace

size_t apply_q0_work(int64_t In, int64_t K, int R) {
  Carver cv(nullptr);
  cv.take<double>(size_t(apply_plan(In, K, R).splits) * In * R);
  return cv.bytes();
}

int apply_q0_enqueue(int64_t In, int64_t K, int R, int ydtype, const void* Y, const double* Q0,
                     double* W, void* work, hipStream_t s) {
  PhaseTimer pt(PH_APPLY_Q0, s);
  const ApplyPlan ap = apply_plan(In, K, R);
  Carver cv(work);
  double* part = cv.take<double>(size_t(ap.splits) * In * R);
  launch_apply(ap, In, K, R, ydtype, Y, Q0, ap.splits > 1 ? part : W, s);
  CPQR_TRY(check_launch("apply_q0"));
  if (ap.splits > 1) {
    const int64_t cnt = In * R;
    hipLaunchKernelGGL(sum_parts, dim3(unsigned(ceil_div(cnt, BLK))), dim3(BLK), 0, s, part,
                       int(ap.splits), cnt, W);
    CPQR_TRY(check_launch("apply_q0 sum"));
  }
  return CPQR_OK;
}

int apply_solve_enqueue(int64_t In, int64_t K, int R, int ydtype, const void* Y, const double* Q0,
                        const double* R0, int use_svd, double rtol, double* W, double* A, double* lambda,
                        int* status, void* work, hipStream_t s, bool normalize) {
  const ApplyPlan ap = apply_plan(In, K, R);
  const int64_t splits = ap.splits;
  if (use_svd || splits == 1) {
    CPQR_TRY(apply_q0_enqueue(In, K, R, ydtype, Y, Q0, W, work, s));
    return solve_enqueue(In, R, W, R0, use_svd, rtol, A, lambda, status, work, s, normalize);
  }
  const int RM = round_rank(R);
  if (!ap.tiled && splits <= 4) {  // product and solve in one launch
    PhaseTimer pt(PH_SOLVE, s);
    const dim3 grd(unsigned(ceil_div(In, BLK / RM)));
#define APSOLVE(TY, RMV)                                                                                   \
  hipLaunchKernelGGL((apply_solve_kernel<TY, RMV, 4>), grd, dim3(4 * BLK), 0, s, static_cast<const TY*>(Y), Q0, R0, \
                     W, A, In, K, R, ap.kchunk, status)
    if (ydtype == CPQR_F64) {
      if (RM == 8) APSOLVE(double, 8); else if (RM == 16) APSOLVE(double, 16); else APSOLVE(double, 32);
    } else {
      if (RM == 8) APSOLVE(float, 8); else if (RM == 16) APSOLVE(float, 16); else APSOLVE(float, 32);
    }
#undef APSOLVE
    CPQR_TRY(check_launch("apply_solve"));
    if (!normalize) return CPQR_OK;
    hipLaunchKernelGGL(normalize_kernel, dim3(R), dim3(BLK), 0, s, A, lambda, In, status);
    return check_launch("normalize");
  }
  // the solve adds up the partial W's itself (one kernel fewer)
  Carver cv(work);
  double* part = cv.take<double>(size_t(splits) * In * R);
  {
    PhaseTimer pt(PH_APPLY_Q0, s);
    launch_apply(ap, In, K, R, ydtype, Y, Q0, part, s);
    CPQR_TRY(check_launch("apply_q0"));
  }
  PhaseTimer pt(PH_SOLVE, s);
  const dim3 grd(unsigned(ceil_div(In, BLK / RM)));
  // many partials per entry (the tiled product over a long K): four groups add them
#define SUMSOLVE(RMV, KGV)                                                                                  \
  hipLaunchKernelGGL((sum_solve_kernel<RMV, KGV>), grd, dim3(KGV * BLK), 0, s, part, int(splits), R0, W, A, In, R, \
                     status)
  if (splits >= 8) {
    if (RM == 8) SUMSOLVE(8, 4); else if (RM == 16) SUMSOLVE(16, 4); else SUMSOLVE(32, 4);
  } else {
    if (RM == 8) SUMSOLVE(8, 1); else if (RM == 16) SUMSOLVE(16, 1); else SUMSOLVE(32, 1);
  }
#undef SUMSOLVE
  CPQR_TRY(check_launch("sum_solve"));
  if (!normalize) return CPQR_OK;
  hipLaunchKernelGGL(normalize_kernel, dim3(R), dim3(BLK), 0, s, A, lambda, In, status);
  return check_launch("normalize");
}

size_t solve_work(int64_t In, int R) {
  (void)In;
  Carver cv(nullptr);
  cv.take<double>(size_t(R) * R);
  cv.take<int>(4);
  return cv.bytes();
}

int solve_enqueue(int64_t In, int R, const double* W, const double* R0, int use_svd, double rtol,
                  double* A, double* lambda, int* status, void* work, hipStream_t s, bool normalize) {
  PhaseTimer pt(PH_SOLVE, s);
  Carver cv(work);
  double* M = cv.take<double>(size_t(R) * R);
  int* kept = cv.take<int>(4);
  const dim3 grd(unsigned(ceil_div(In, BLK)));
  const int RM = round_rank(R);
  if (!use_svd) {
    if (RM == 8)
      hipLaunchKernelGGL((solve_tri_kernel<8>), grd, dim3(BLK), 0, s, W, R0, A, In, R, status);
    else if (RM == 16)
      hipLaunchKernelGGL((solve_tri_kernel<16>), grd, dim3(BLK), 0, s, W, R0, A, In, R, status);
    else
      hipLaunchKernelGGL((solve_tri_kernel<32>), grd, dim3(BLK), 0, s, W, R0, A, In, R, status);
    CPQR_TRY(check_launch("solve_tri"));
  } else {
    if (rtol < 0) rtol = R * 2.220446049250313e-16;
    CPQR_TRY(launch_svd_pinv(R0, R, rtol, M, kept, status, s));
    if (RM == 8)
      hipLaunchKernelGGL((rowmul_kernel<8>), grd, dim3(BLK), 0, s, W, M, A, In, R, status);
    else if (RM == 16)
      hipLaunchKernelGGL((rowmul_kernel<16>), grd, dim3(BLK), 0, s, W, M, A, In, R, status);
    else
      hipLaunchKernelGGL((rowmul_kernel<32>), grd, dim3(BLK), 0, s, W, M, A, In, R, status);
    CPQR_TRY(check_launch("rowmul"));
  }
  if (!normalize) return CPQR_OK;
  hipLaunchKernelGGL(normalize_kernel, dim3(R), dim3(BLK), 0, s, A, lambda, In, status);
  return check_launch("normalize");
}

size_t norm2_work(int64_t count) {
  (void)count;
  Carver cv(nullptr);
  cv.take<double>(NORM_BLOCKS);
  return cv.bytes();
}

int norm2_enqueue(int64_t count, int xdtype, const void* X, double* out, void* work, hipStream_t s) {
  Carver cv(work);
  double* part = cv.take<double>(NORM_BLOCKS);
  const int nb = int(std::min<int64_t>(NORM_BLOCKS, std::max<int64_t>(1, ceil_div(count, BLK * 8))));
  if (xdtype == CPQR_F64)
    hipLaunchKernelGGL(norm2_partial<double>, dim3(nb), dim3(BLK), 0, s, static_cast<const double*>(X),
                       count, part);
  else
    hipLaunchKernelGGL(norm2_partial<float>, dim3(nb), dim3(BLK), 0, s, static_cast<const float*>(X),
                       count, part);
  CPQR_TRY(check_launch("norm2"));
  hipLaunchKernelGGL(sum_final, dim3(1), dim3(BLK), 0, s, part, nb, 1, out);
  return check_launch("norm2 final");
}

size_t error_efficient_work(int64_t In) { return size_t(1 + ceil_div(In, BLK)) * sizeof(double); }

int error_efficient_enqueue(int64_t In, int R, const double* W, const double* A,
                            const double* lambda, const double* R0, const double* RN,
                            const double* xnorm2, double* relerr, double* part, hipStream_t s) {
  PhaseTimer pt(PH_ERROR, s);
  const int RM = round_rank(R);
  const unsigned nb = unsigned(ceil_div(In, BLK));
  if (RM == 8)
    hipLaunchKernelGGL((error_efficient_kernel<8>), dim3(nb), dim3(BLK), 0, s, W, A, lambda, R0, RN, In, R, part);
  else if (RM == 16)
    hipLaunchKernelGGL((error_efficient_kernel<16>), dim3(nb), dim3(BLK), 0, s, W, A, lambda, R0, RN, In, R, part);
  else
    hipLaunchKernelGGL((error_efficient_kernel<32>), dim3(nb), dim3(BLK), 0, s, W, A, lambda, R0, RN, In, R, part);
  CPQR_TRY(check_launch("error_efficient"));
  hipLaunchKernelGGL(error_efficient_final, dim3(1), dim3(1), 0, s, part, int(nb), xnorm2, relerr);
  return check_launch("error_efficient_final");
}

// Q_0 = (Q_a kron I_R) Q_b for Q_a (R^2 x R) and Q_b (R^2 x R), column-major:
// Q_0(r + R j, c) = sum_t Q_a(j, t) Q_b(r + R t, c), r < R, j < R^2, c < R (the
// orthonormal factor of (Q_a T) (.) F = (Q_a kron I)(T (.) F), eq. (kr-id),
// once T (.) F = Q_b T_b).  One thread per entry of Q_0.
__global__ __launch_bounds__(BLK) void expand_kron_right_kernel(const double* __restrict__ Qa,
                                                                const double* __restrict__ Qb, int R,
                                                                double* __restrict__ Q0) {
  const int64_t R2 = int64_t(R) * R, R3 = R2 * R;
  const int64_t e = int64_t(blockIdx.x) * BLK + threadIdx.x;
  if (e >= R3 * R) return;
  const int64_t row = e % R3, c = e / R3;
  const int64_t r = row % R, j = row / R;
  double acc = 0.0;
  for (int t = 0; t < R; ++t) acc += Qa[j + R2 * t] * Qb[r + R * t + R2 * c];
  Q0[e] = acc;
}

int expand_kron_right_enqueue(int R, const double* Qa, const double* Qb, double* Q0, hipStream_t s) {
  const int64_t cnt = int64_t(R) * R * R * R;
  hipLaunchKernelGGL(expand_kron_right_kernel, dim3(unsigned(ceil_div(cnt, BLK))), dim3(BLK), 0, s, Qa, Qb, R, Q0);
  return check_launch("expand_kron_right");
}

int expand_q0_enqueue(int N, int R, const double* Qc, double* Q0, double* buf, hipStream_t s) {
  const size_t blk = size_t(R) * R * R;  // doubles per factor Q_j
  if (N == 3) {
    CPQR_HIP(hipMemcpyAsync(Q0, Qc, sizeof(double) * blk, hipMemcpyDeviceToDevice, s));
    return CPQR_OK;
  }
  // G = Q_{N-1}, then G <- (I kron Q_j) G for j = N-2 .. 2; the last step writes Q0
  const double* G = Qc + size_t(N - 3) * blk;
  int64_t m = R;
  for (int j = N - 2; j >= 2; --j) {
    double* out = j == 2 ? Q0 : buf + ((N - 2 - j) % 2) * (ipow(R, N - 1) * R);
    const int64_t cnt = int64_t(R) * R * m * R;
    hipLaunchKernelGGL(expand_q0_kernel, dim3(unsigned(ceil_div(cnt, BLK))), dim3(BLK), 0, s,
                       Qc + size_t(j - 2) * blk, G, m, R, out);
    CPQR_TRY(check_launch("expand_q0"));
    G = out;
    m *= R;
  }
  return CPQR_OK;
}

int diag_cols_enqueue(int64_t In, int N, int R, int ydtype, const void* Y, double* W, hipStream_t s) {
  int64_t dstep = 0, pw = 1;
  for (int k = 0; k + 1 < N; ++k) {
    dstep += pw;
    pw *= R;
  }
  const dim3 grd(unsigned(ceil_div(In * R, BLK)));
  if (ydtype == CPQR_F64)
    hipLaunchKernelGGL(diag_cols_kernel<double>, grd, dim3(BLK), 0, s, static_cast<const double*>(Y), In, dstep, R, W);
  else
    hipLaunchKernelGGL(diag_cols_kernel<float>, grd, dim3(BLK), 0, s, static_cast<const float*>(Y), In, dstep, R, W);
  return check_launch("diag_cols");
}

int error_from_fit_enqueue(const double* fit, double* relerr, hipStream_t s) {
  hipLaunchKernelGGL(error_from_fit_kernel, dim3(1), dim3(1), 0, s, fit, relerr);
  return check_launch("error_from_fit");
}

int fill_enqueue(double* p, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return CPQR_OK;
  hipLaunchKernelGGL(fill_kernel, dim3(unsigned(ceil_div(count, BLK))), dim3(BLK), 0, s, p, count, v);
  return check_launch("fill");
}

size_t fit_direct_work(int N, const int64_t* I, int R) {
  (void)R;
  int64_t S = 1;
  for (int k = 1; k < N; ++k) S *= I[k];
  const int64_t nb = ceil_div(I[0], BLK) * ceil_div(S, CS);
  Carver cv(nullptr);
  cv.take<double>(size_t(2 * nb));
  return cv.bytes();
}

int fit_direct_enqueue(int N, const int64_t* I, int xdtype, const void* X, int R,
                       const double* lambda, const double* const* A, double* out, void* work,
                       hipStream_t s) {
  PhaseTimer pt(PH_ERROR, s);
  FactorPtrs f{};
  int64_t S = 1;
  for (int k = 0; k < N; ++k) {
    f.A[k] = A[k];
    f.I[k] = I[k];
    if (k > 0) S *= I[k];
  }
  // column chunks on x (up to 2^31-1), row blocks on y (up to 65535)
  const int64_t gx = ceil_div(S, CS), gy = ceil_div(I[0], BLK);
  if (gx > 0x7fffffff || gy > 65535) return fail(CPQR_ERR_SHAPE, "fit_direct: tensor too large");
  Carver cv(work);
  double* part = cv.take<double>(size_t(2 * gx * gy));
  const dim3 grd{unsigned(gx), unsigned(gy)};
  const int RM = round_rank(R);
#define FIT(TX, RMV)                                                                                \
  hipLaunchKernelGGL((fit_direct_kernel<TX, RMV>), grd, dim3(BLK), 0, s, static_cast<const TX*>(X), f, N, \
                     lambda, R, I[0], S, part)
  if (xdtype == CPQR_F64) {
    if (RM == 8) FIT(double, 8); else if (RM == 16) FIT(double, 16); else FIT(double, 32);
  } else {
    if (RM == 8) FIT(float, 8); else if (RM == 16) FIT(float, 16); else FIT(float, 32);
  }
#undef FIT
  CPQR_TRY(check_launch("fit_direct"));
  hipLaunchKernelGGL(sum_final, dim3(1), dim3(BLK), 0, s, part, int(gx * gy), 2, out);
  return check_launch("fit_direct final");
}

// ------------------------------------------------------------ Alg. 1 host side
int gram_enqueue(int64_t In, int R, const double* A, double* G, hipStream_t s) {
  hipLaunchKernelGGL(gram_kernel, dim3(unsigned(R * R)), dim3(BLK), 0, s, A, In, R, G);
  return check_launch("gram");
}

size_t ne_update_work(int R) {
  Carver cv(nullptr);
  cv.take<int>(4);
  return cv.bytes();
}

namespace {
// The MTTKRP is column dstep * c of Y (dstep = 1 for a formed In x R matrix).
int ne_update_core(int64_t In, int N, int n, int R, int ydtype, const void* Y, int64_t dstep, double* G, int pinv,
                   double rtol, double* S, double* F, double* M, double* A, double* lambda, int* status,
                   void* work, hipStream_t s) {
  PhaseTimer pt(PH_SOLVE, s);
  Carver cv(work);
  int* kept = cv.take<int>(4);
  hipLaunchKernelGGL(ne_factor_kernel, dim3(1), dim3(BLK), 0, s, G, N, n, R, pinv ? 0 : 1, S, F, status);
  CPQR_TRY(check_launch("ne_factor"));
  if (pinv) {
    if (rtol < 0) rtol = R * 2.220446049250313e-16;
    // S_n is symmetric, so the transposed pseudo-inverse the kernel forms is pinv(S_n) itself
    CPQR_TRY(launch_svd_pinv(S, R, rtol, F, kept, status, s));
  }
  const dim3 grd(unsigned(ceil_div(In, BLK)));
  const int RM = round_rank(R);
#define ROWS(TY, RMV)                                                                                          \
  hipLaunchKernelGGL((ne_rows_kernel<TY, RMV>), grd, dim3(BLK), 0, s, static_cast<const TY*>(Y), In, dstep, F, \
                     pinv ? 0 : 1, R, M, A, status)
  if (ydtype == CPQR_F64) {
    if (RM == 8) ROWS(double, 8); else if (RM == 16) ROWS(double, 16); else ROWS(double, 32);
  } else {
    if (RM == 8) ROWS(float, 8); else if (RM == 16) ROWS(float, 16); else ROWS(float, 32);
  }
#undef ROWS
  CPQR_TRY(check_launch("ne_rows"));
  hipLaunchKernelGGL(normalize_kernel, dim3(R), dim3(BLK), 0, s, A, lambda, In, status);
  CPQR_TRY(check_launch("normalize"));
  return gram_enqueue(In, R, A, G + int64_t(n) * R * R, s);
}
}  // namespace

int ne_update_enqueue(int64_t In, int N, int n, int R, int ydtype, const void* Y, double* G, int pinv,
                      double rtol, double* S, double* F, double* M, double* A, double* lambda, int* status,
                      void* work, hipStream_t s) {
  // column r of M_n is the column of Y_(n) whose every Kronecker index is r:
  // r (1 + R + .. + R^{N-2})
  int64_t dstep = 0, pw = 1;
  for (int k = 0; k + 1 < N; ++k) {
    dstep += pw;
    pw *= R;
  }
  return ne_update_core(In, N, n, R, ydtype, Y, dstep, G, pinv, rtol, S, F, M, A, lambda, status, work, s);
}

int ne_update_from_m_enqueue(int64_t In, int N, int n, int R, const double* Mn, double* G, int pinv, double rtol,
                             double* S, double* F, double* M, double* A, double* lambda, int* status, void* work,
                             hipStream_t s) {
  return ne_update_core(In, N, n, R, CPQR_F64, Mn, 1, G, pinv, rtol, S, F, M, A, lambda, status, work, s);
}

size_t ne_error_work(int64_t In) { return size_t(ceil_div(In, BLK)) * sizeof(double); }

int ne_error_enqueue(int64_t In, int R, const double* M, const double* A, const double* lambda, const double* S,
                     const double* GN, const double* xnorm2, double* relerr, double* part, hipStream_t s) {
  PhaseTimer pt(PH_ERROR, s);
  const int nb = int(ceil_div(In, BLK));
  hipLaunchKernelGGL(ne_err_partial, dim3(unsigned(nb)), dim3(BLK), 0, s, M, A, lambda, In, R, part);
  CPQR_TRY(check_launch("ne_err_partial"));
  hipLaunchKernelGGL(ne_err_final, dim3(1), dim3(BLK), 0, s, part, nb, S, GN, lambda, R, xnorm2, relerr);
  return check_launch("ne_err_final");
}

}  // namespace cpqr
