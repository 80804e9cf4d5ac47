// Workgroup-level Householder QR building blocks (device code), shared by
// the tall-skinny QR kernels and the batched CP-ALS-QR kernel.  One
// workgroup of NT threads factorizes a block of at most NT rows, one row per
// thread, R <= RMAX columns in registers.  See tsqr.hip for the algorithm.
#pragma once

#include <hip/hip_runtime.h>

namespace cpqr {
namespace wgqr {

constexpr int WAVE = 64;

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// Sum over all threads of the workgroup of each x[i] (V a power of two <= 32).
// Result in res[0..V-1] (LDS), visible to every thread on return.
template <int V, int NW>
__device__ inline void block_sum_vec(double (&x)[V], double* red, double* res, int tid) {
  const int lane = tid % WAVE, w = tid / WAVE;
  constexpr int L = ilog2(V);
  int idx = 0;
#pragma unroll
  for (int l = 0; l < L; ++l) {
    const int mask = 32 >> l;
    const int half = V >> (l + 1);
    const bool hi = (lane & mask) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const double send = hi ? x[i] : x[half + i];
      const double got = __shfl_xor(send, mask, WAVE);
      x[i] = (hi ? x[half + i] : x[i]) + got;
    }
    idx += hi ? half : 0;
  }
#pragma unroll
  for (int mask = 32 >> L; mask >= 1; mask >>= 1) x[0] += __shfl_xor(x[0], mask, WAVE);
  if ((lane & ((64 >> L) - 1)) == 0) red[w * V + idx] = x[0];
  __syncthreads();
  if (tid < V) {
    double s = 0.0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) s += red[ww * V + tid];
    res[tid] = s;
  }
  __syncthreads();
}

// LDS workspace of one node.
template <int RMAX, int NT>
struct Shared {
  double red[(NT / WAVE) * RMAX];
  double res[RMAX];
  double alpha;
  double tau[RMAX];
  double G[RMAX][RMAX + 1];   // reflector Gram (strict upper part), later V1^T C
  double T[RMAX][RMAX + 1];   // compact WY factor
  double V1[RMAX][RMAX + 1];  // top R x R block of V
  double C[RMAX][RMAX + 1];   // input slice of the parent's Q
  double M[RMAX][RMAX + 1];   // T V1^T C
};

// Reflector component of row `row` for reflector c, from the factorized a[].
template <int RMAX>
__device__ inline double vcomp(const double (&a)[RMAX], int c, int row, int m) {
  return row == c ? 1.0 : ((row > c && row < m) ? a[c] : 0.0);
}

// Householder QR of the node block (row `tid` in a[], rows >= m are zero).
// On return rows < R hold R's rows (entries at c >= row), rows > c hold
// reflector c below the diagonal in a[c]; sh.tau and the strict upper part of
// sh.G are filled.
template <int RMAX, int NT>
__device__ void wg_factor(double (&a)[RMAX], int tid, int m, int R, Shared<RMAX, NT>& sh) {
  constexpr int NW = NT / WAVE;
  // The column loop stays rolled; a[j] is picked and replaced through compare
  // chains so the register array is only ever indexed by constants.
#pragma unroll 1
  for (int j = 0; j < R; ++j) {
    double aj = 0.0;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) aj = (c == j) ? a[c] : aj;
    if (tid == j) sh.alpha = aj;
    double x1[1] = {(tid > j && tid < m) ? aj * aj : 0.0};
    block_sum_vec<1, NW>(x1, sh.red, sh.res, tid);
    const double alpha = sh.alpha, sub2 = sh.res[0];
    double t = 0.0, beta = alpha, scal = 0.0;
    if (sub2 > 0.0) {
      const double nrm = sqrt(alpha * alpha + sub2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    const double v = (tid == j) ? 1.0 : ((tid > j && tid < m) ? aj * scal : 0.0);
    const double newj = (tid == j) ? beta : ((tid > j) ? v : aj);
#pragma unroll
    for (int c = 0; c < RMAX; ++c) a[c] = (c == j) ? newj : a[c];
    if (tid == 0) sh.tau[j] = t;
    double x[RMAX];
#pragma unroll
    for (int c = 0; c < RMAX; ++c)
      x[c] = (c < j) ? vcomp<RMAX>(a, c, tid, m) * v : ((c > j && c < R) ? v * a[c] : 0.0);
    block_sum_vec<RMAX, NW>(x, sh.red, sh.res, tid);
    const double tv = t * v;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) a[c] = (c > j && c < R) ? a[c] - tv * sh.res[c] : a[c];
    if (tid < j) sh.G[tid][j] = sh.res[tid];
  }
  __syncthreads();
}

// T of the compact WY form: T(j,j) = tau_j,
// T(0:j, j) = -tau_j T(0:j, 0:j) G(0:j, j).  One wavefront, lane = row of T.
template <int RMAX, int NT>
__device__ void wg_build_t(int tid, int R, Shared<RMAX, NT>& sh) {
  if (tid < WAVE) {
    for (int j = 0; j < R; ++j) {
      double v = 0.0;
      if (tid < j) {
        for (int k = tid; k < j; ++k) v += sh.T[tid][k] * sh.G[k][j];
        v *= -sh.tau[j];
      } else if (tid == j) {
        v = sh.tau[j];
      }
      if (tid < RMAX) sh.T[tid][j] = v;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  __syncthreads();
}

// Rows of this node's Q: q = [C; 0](row) - v(row) M with M = T V1^T C.
// Expects sh.T and sh.C filled; uses sh.V1, sh.G (as scratch) and sh.M.
template <int RMAX, int NT>
__device__ void wg_form_q(const double (&a)[RMAX], double (&q)[RMAX], int tid, int m, int R,
                          Shared<RMAX, NT>& sh) {
  if (tid < R) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c) sh.V1[tid][c] = (c < R) ? vcomp<RMAX>(a, c, tid, m) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < R * R; e += NT) {  // B = V1^T C
    const int k = e / R, c = e % R;
    double s = 0.0;
    for (int i = k; i < R; ++i) s += sh.V1[i][k] * sh.C[i][c];
    sh.G[k][c] = s;
  }
  __syncthreads();
  for (int e = tid; e < R * R; e += NT) {  // M = T B
    const int k = e / R, c = e % R;
    double s = 0.0;
    for (int i = k; i < R; ++i) s += sh.T[k][i] * sh.G[i][c];
    sh.M[k][c] = s;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < RMAX; ++c) q[c] = (tid < R && c < R) ? sh.C[tid][c] : 0.0;
#pragma unroll 1
  for (int k = 0; k < R; ++k) {
    double vk = 0.0;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) vk = (c == k) ? vcomp<RMAX>(a, c, tid, m) : vk;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) q[c] -= vk * sh.M[k][c];
  }
}

}  // namespace wgqr
}  // namespace cpqr
