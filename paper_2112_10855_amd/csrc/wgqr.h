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

// LDS workspace of one block of at most MROWS rows.
template <int RMAX, int NT, int MROWS>
struct Shared {
  double red[(NT / WAVE) * RMAX];
  double res[RMAX];
  double rowj[2][RMAX];       // row j of the block while column j is reduced
  double tau[RMAX];
  double G[RMAX][RMAX + 1];   // reflector Gram (strict upper part), later V1^T C
  double T[RMAX][RMAX + 1];   // compact WY factor
  double V1[RMAX][RMAX + 1];  // top R x R block of V
  double C[RMAX][RMAX + 1];   // input slice of the parent's Q
  double M[RMAX][RMAX + 1];   // T V1^T C
  double am[MROWS][RMAX + 1]; // the block, row i in am[i] (zero past column R)
};

// Householder QR of the block in sh.am (m rows, R columns; thread i owns row
// i).  On return rows < R hold R's rows (entries at c >= row), rows > c hold
// reflector c below the diagonal in column c (v_c = e_c + those entries);
// sh.tau and the strict upper part of sh.G are filled.  Column j takes one
// workgroup reduction: with the subcolumn a_(i>j, j) it sums, for every c,
// a_ij a_ic over the rows below j.  Entry j is the squared norm that fixes
// the reflector v = e_j + s a_(i>j, j) (s = 1 / (alpha - beta)); for c > j,
// row j of A plus s times entry c is v^T a_c, the coefficient of the rank-one
// update; for c < j, row j's v_c(j) plus s times entry c is v_c^T v, the
// reflector Gram entry that the compact WY factor needs.  The rows live in
// LDS, so the column index is a plain address: no compare chains over the
// registers of a row.
template <int RMAX, int NT, int MROWS>
__device__ void wg_factor(int tid, int m, int R, Shared<RMAX, NT, MROWS>& sh) {
  constexpr int NW = NT / WAVE;
  double* row = sh.am[tid < MROWS ? tid : 0];
  const bool has = tid < m;
#pragma unroll 1
  for (int j = 0; j < R; ++j) {
    const int buf = j & 1;
    if (tid == j) {
#pragma unroll
      for (int c = 0; c < RMAX; ++c) sh.rowj[buf][c] = row[c];
    }
    const bool below = has && tid > j;
    double aj = 0.0;
    double x[RMAX];
    if (below) {
      aj = row[j];
#pragma unroll
      for (int c = 0; c < RMAX; ++c) x[c] = aj * row[c];
    } else {
#pragma unroll
      for (int c = 0; c < RMAX; ++c) x[c] = 0.0;
    }
    block_sum_vec<RMAX, NW>(x, sh.red, sh.res, tid);
    const double sub2 = sh.res[j];
    const double alpha = sh.rowj[buf][j];
    double t = 0.0, beta = alpha, scal = 0.0;
    if (sub2 > 0.0) {
      const double nrm = sqrt(alpha * alpha + sub2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    if (has && tid >= j) {
      const double v = tid == j ? 1.0 : aj * scal;
      const double tv = t * v;
      for (int c = j + 1; c < R; ++c) row[c] -= tv * (sh.rowj[buf][c] + scal * sh.res[c]);
      row[j] = tid == j ? beta : v;
    }
    if (tid == 0) sh.tau[j] = t;
    if (tid < j) sh.G[tid][j] = sh.rowj[buf][tid] + scal * sh.res[tid];
  }
  __syncthreads();
}

// T of the compact WY form: T(j,j) = tau_j,
// T(0:j, j) = -tau_j T(0:j, 0:j) G(0:j, j).  One wavefront, lane = row of T.
template <int RMAX, int NT, int MROWS>
__device__ void wg_build_t(int tid, int R, Shared<RMAX, NT, MROWS>& sh) {
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

// Reflector c's component in row `row` of the factorized block.
template <int RMAX, int NT, int MROWS>
__device__ inline double vcomp(const Shared<RMAX, NT, MROWS>& sh, int c, int row, int m) {
  return row == c ? 1.0 : ((row > c && row < m) ? sh.am[row][c] : 0.0);
}

// Rows of the block's Q: q = [C; 0](row) - v(row) M with M = T V1^T C.
// Expects sh.T and sh.C filled; uses sh.V1, sh.G (as scratch) and sh.M.
template <int RMAX, int NT, int MROWS>
__device__ void wg_form_q(double (&q)[RMAX], int tid, int m, int R, Shared<RMAX, NT, MROWS>& sh) {
  if (tid < R) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c) sh.V1[tid][c] = (c < R) ? vcomp(sh, c, tid, m) : 0.0;
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
  if (tid < m) {
    const double* row = sh.am[tid];
#pragma unroll 1
    for (int k = 0; k < R; ++k) {
      const double vk = tid == k ? 1.0 : (tid > k ? row[k] : 0.0);
#pragma unroll
      for (int c = 0; c < RMAX; ++c) q[c] -= vk * sh.M[k][c];
    }
  }
}

}  // namespace wgqr
}  // namespace cpqr
