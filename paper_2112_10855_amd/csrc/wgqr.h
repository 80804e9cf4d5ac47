// Workgroup-level Householder QR building blocks (device code) for the
// batched CP-ALS-QR kernel.  One workgroup of NT threads factorizes a block
// of at most NT rows, one row per thread, R <= RMAX columns in registers.
#pragma once

#include <hip/hip_runtime.h>

#include "wave.h"

namespace cpqr {
namespace wgqr {

using wave::ilog2;
constexpr int WAVE = 64;

// Sum over all threads of the workgroup of each x[i] (V a power of two <=
// 32): a reduce-scatter within each wave (DPP and lane swaps, no LDS), the
// wave partials through LDS.  Result in res[0..V-1] (LDS), visible to every
// thread on return.  The wave partials are added in wave order.
template <int V, int NW>
__device__ inline void block_sum_vec(double (&x)[V], double* red, double* res, int tid) {
  const int lane = tid % WAVE, w = tid / WAVE;
  const double s = wave::wave_sum<V>(x, lane);
  if ((lane & (WAVE / V - 1)) == 0) red[w * V + (lane >> (6 - ilog2(V)))] = s;
  __syncthreads();
  if (tid < V) {
    double t = 0.0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) t += red[ww * V + tid];
    res[tid] = t;
  }
  __syncthreads();
}

// The same sums returned in x[] of every thread after a single barrier: each
// thread adds the NW wave partials itself.  red holds two buffers of NW V
// doubles ([buf][i][wave]); consecutive calls must alternate buf, so that
// a call never overwrites partials a slower thread may still be reading
// (the barrier of the call in between orders the two).
template <int V, int NW>
__device__ inline void block_allsum(double (&x)[V], double* red, int buf, int tid) {
  const int lane = tid % WAVE, w = tid / WAVE;
  double* rb = red + buf * NW * V;
  const double s = wave::wave_sum<V>(x, lane);
  if ((lane & (WAVE / V - 1)) == 0) rb[(lane >> (6 - ilog2(V))) * NW + w] = s;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < V; ++i) {
    double t = 0.0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) t += rb[i * NW + ww];
    x[i] = t;
  }
}

// LDS workspace of one node.
template <int RMAX, int NT>
struct Shared {
  double red[2 * (NT / WAVE) * RMAX];
  double rowj[2][RMAX];       // row j of the block while column j is reduced
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
// sh.G are filled.  Column j takes one workgroup reduction: with the
// unscaled subcolumn a_(i>j, j) it sums, for every c, a_ij a_ic over the rows
// below j.  Entry j is the squared norm that fixes the reflector
// v = e_j + s a_(i>j, j) (s = 1 / (alpha - beta)); for c > j, row j of A plus
// s times entry c is v^T a_c, the coefficient of the rank-one update; for
// c < j, row j's v_c(j) plus s times entry c is v_c^T v, the reflector Gram
// entry that the compact WY factor needs.  Row j itself goes through LDS.
template <int RMAX, int NT>
__device__ void wg_factor(double (&a)[RMAX], int tid, int m, int R, Shared<RMAX, NT>& sh) {
  constexpr int NW = NT / WAVE;
  // The column loop stays rolled; a[j] is picked and replaced through compare
  // chains so the register array is only ever indexed by constants.
#pragma unroll 1
  for (int j = 0; j < R; ++j) {
    const int buf = j & 1;
    double aj = 0.0;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) aj = (c == j) ? a[c] : aj;
    if (tid == j) {
#pragma unroll
      for (int c = 0; c < RMAX; ++c) sh.rowj[buf][c] = a[c];
    }
    const bool below = tid > j && tid < m;
    double x[RMAX];
#pragma unroll
    for (int c = 0; c < RMAX; ++c) x[c] = (below && c < R) ? aj * a[c] : 0.0;
    block_allsum<RMAX, NW>(x, sh.red, buf, tid);
    double sub2 = 0.0;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) sub2 = (c == j) ? x[c] : sub2;
    const double alpha = sh.rowj[buf][j];
    double t = 0.0, beta = alpha, scal = 0.0;
    if (sub2 > 0.0) {
      const double nrm = sqrt(alpha * alpha + sub2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    const double v = (tid == j) ? 1.0 : (below ? aj * scal : 0.0);
    const double tv = t * v;
#pragma unroll
    for (int c = 0; c < RMAX; ++c)
      if (c > j && c < R) a[c] -= tv * (sh.rowj[buf][c] + scal * x[c]);
    const double newj = (tid == j) ? beta : ((tid > j) ? v : aj);
#pragma unroll
    for (int c = 0; c < RMAX; ++c) a[c] = (c == j) ? newj : a[c];
    if (tid == 0) sh.tau[j] = t;
    if (tid < j) {
      double xk = 0.0;
#pragma unroll
      for (int c = 0; c < RMAX; ++c) xk = (c == tid) ? x[c] : xk;
      sh.G[tid][j] = sh.rowj[buf][tid] + scal * xk;
    }
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
