// Batched CP-ALS-QR (paper Alg. 2) for many small 3-way tensors in one
// persistent launch.
//
// Design.  One workgroup owns one tensor for the whole launch and runs every
// sweep of it: no workgroup ever waits on another, so the launch carries
// all sweeps of all tensors with workgroup barriers only.  Tensors are taken
// largest first.  A sweep (modes counted from 1 as in the paper):
//   Z = X x_3 Q_3^T                        streams X (and gives ||X||^2)
//   mode 1: Y_(1) = Z x_2 Q_2^T, W = Y Q_0, solve A R_0^T = W,
//           then normalize, factor QR of A_1, Khatri-Rao QR for mode 2
//   mode 2: Y_(2) = Z x_1 Q_1^T (new Q_1), W, solve, normalize, QRs
//   T = X x_2 Q_2^T (new Q_2)              streams X
//   mode 3: Y_(3) = T x_1 Q_1^T, W, solve, normalize, QRs, efficient error
// Z serves modes 1 and 2 (Q_3 does not change between them), so a sweep
// reads each tensor twice instead of three times: the reuse of partial TTMs
// across modes (dimension trees) that the paper names for Multi-TTM.  The
// results equal the per-mode Multi-TTMs up to FP32 rounding order.
//
// Arithmetic: contractions in FP32 on FP32 copies of Q_k (on the matrix
// cores, v_mfma_f32_16x16x4f32, 16 output columns >= R), everything else in
// FP64.  Limits: R <= 16, R <= I_k <= 256 (the factor QR keeps one row per
// thread).

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

constexpr int NT = 512;    // threads per workgroup (eight waves: two per SIMD, one workgroup per CU)
constexpr int NW = NT / WAVE;
constexpr int RB = 16;     // register width for rank-indexed rows (R <= 16)
constexpr int IMAX = 256;  // largest mode size

struct BItem {
  int64_t I[3];
  int R;
  int nB[3];     // row blocks per mode
  int rows[3];   // rows per block per mode
  const float* X;  // streamed copy: first mode padded to I0p (zeros), 16-byte aligned
  int64_t I0p;     // I[0] rounded up to a multiple of 4
  double* A[3];
  double* lam;
  double* relerr;
  double* Q[3];    // Q_k, column-major I_k x R (FP64)
  float* Qf[3];    // FP32 copy of Q_k, row-major I_k x RB, zero past R
  double* Rf[3];   // R_k, column-major R x R
  double* Q0b[3];  // Q_0 for mode n, row-major R^2 x R
  double* R0b[3];  // R_0 for mode n, column-major R x R
  float* Z;        // Z[i1 + I0p i2 + I0p I1 r3] (rows i1 >= I0 zero)
  float* T;        // T[i1 + I0p r2 + I0p R i3]
  float* Y;        // Y_(n) of the current mode (layout per mode, see task_y)
  double* lamp;    // [block][RB] column sums of squares of A rows per block
  double* ipp;     // [block] <W, A R_0^T> per block (mode 3)
  double* xnorm2;  // ||X||^2
};

static_assert(sizeof(BItem) % sizeof(int) == 0, "the kernel copies BItem into LDS word by word");

typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) const float gcfloat;
typedef __attribute__((address_space(1))) double gdouble;

// The kernel's view of a BItem: the same bytes, every pointer typed as
// global memory.  Generic (flat) accesses count on the LDS counter as well,
// so a flat access pending anywhere makes the compiler wait for all LDS and
// global traffic before the next LDS read; global pointers keep the two
// apart.
struct GItem {
  int64_t I[3];
  int R;
  int nB[3];
  int rows[3];
  gcfloat* X;
  int64_t I0p;
  gdouble* A[3];
  gdouble* lam;
  gdouble* relerr;
  gdouble* Q[3];
  gfloat* Qf[3];
  gdouble* Rf[3];
  gdouble* Q0b[3];
  gdouble* R0b[3];
  gfloat* Z;
  gfloat* T;
  gfloat* Y;
  gdouble* lamp;
  gdouble* ipp;
  gdouble* xnorm2;
};
static_assert(sizeof(GItem) == sizeof(BItem), "GItem mirrors BItem");
static_assert(offsetof(GItem, xnorm2) == offsetof(BItem, xnorm2), "GItem mirrors BItem");
static_assert(offsetof(GItem, Z) == offsetof(BItem, Z) && offsetof(GItem, X) == offsetof(BItem, X),
              "GItem mirrors BItem");

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
__device__ inline gcfloat* gview(const float* p) { return (gcfloat*)p; }
// Descriptor fields come from LDS, which the compiler does not know to be
// the same in every lane; these declare a value wave-uniform so that it
// stays in scalar registers (a buffer resource must).
__device__ inline uint32_t uni(uint32_t v) { return uint32_t(__builtin_amdgcn_readfirstlane(int(v))); }
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int64_t uni(int64_t v) {
  const uint64_t u = uint64_t(v);
  return int64_t((uint64_t(uni(uint32_t(u >> 32))) << 32) | uni(uint32_t(u)));
}
template <class T>
__device__ inline T* uni(T* p) {
  return reinterpret_cast<T*>(uni(int64_t(reinterpret_cast<uintptr_t>(p))));
}
__device__ inline gfloat* gview(float* p) { return (gfloat*)p; }

// About 103 KB (one workgroup per CU).
struct BShared {
  alignas(16) float us[IMAX * RB];  // contraction operand U (FP32, 16 columns; layout per use)
  Shared<RB, NT, IMAX> qr;
  double q0[RB * RB * RB];  // Q_0 of the current mode, row-major R^2 x R
  double r0[RB][RB + 1];
  double rn[RB][RB + 1];
  double lam[RB];
  double red[NW * RB];
  double res[RB];
};

// U rows [0, rows) into LDS (row-major, 16 floats a row, zero past R) and
// zero rows up to the next multiple of 4, so that a 4-step MFMA over the
// contraction index reads zeros past its end.
__device__ inline void stage_u(gcfloat* Qf, int rows, float* us, int tid) {
  const __attribute__((address_space(1))) floatx4* src = reinterpret_cast<const __attribute__((address_space(1))) floatx4*>(Qf);
  floatx4* dst = reinterpret_cast<floatx4*>(us);
  const int n = rows * (RB / 4), n4 = ((rows + 3) & ~3) * (RB / 4);
  for (int e = tid; e < n4; e += NT) dst[e] = e < n ? src[e] : floatx4{0.f, 0.f, 0.f, 0.f};
}

// U for stream_k: us4[(k / 4) * 64 + 4 c + k % 4] = U[k, c] (the four k of a
// lane's 16-byte run next to each other), zero for k >= rows up to the next
// multiple of 16.
__device__ inline void stage_u4(gcfloat* Qf, int rows, float* us4, int tid) {
  const int n16 = (rows + 15) & ~15;
  for (int e = tid; e < n16 * RB; e += NT) {
    const int j = e & 3, c = (e >> 2) & (RB - 1), k = 4 * (e >> 6) + j;
    us4[e] = k < rows ? Qf[k * RB + c] : 0.f;
  }
}

// ------------------------------------------------- streaming pass (AZ, AT)
// out[p + P r + P R s] = sum_k X[p + P k + P K s] U[k, r] for every row
// m = p + P s < M = P S of the [M, K] matrix (P a multiple of 4, X and out
// 16-byte aligned), U (K x R, rows zero from K to the next multiple of 4) in
// LDS.  Rows go on the M dimension of v_mfma_f32_16x16x4f32 in 64-row
// groups, dealt to the waves round robin; a wave works on MG of its groups
// at a time (a tile), in the same group order for every MG.  In step t, lane
// (l16, kq) loads the 16-byte run of rows 4 l16 .. 4 l16 + 3 of each group
// at k = 4 t + kq and feeds its four values to four MFMAs that share the B
// operand U[k, l16]; at the end the lane holds rows 16 kq + 4 v + j (v, j =
// 0..3) of each group, column l16.  Loads go through a buffer resource, so
// k >= K and rows past M read zeros from its range check, and run D steps
// ahead of the MFMAs within a tile.  A tile's results are stored after its
// last step: loads and stores in flight together would force the wait
// before every use down to zero, so each tile drains once instead.  The
// order of every sum is fixed by the layout alone (the sum of squares goes
// group by group in the wave's group order), so D and MG do not change the
// bits.  SQ: xx += the sum of x^2.
constexpr uint32_t OOB = 0x80000000u;  // a byte offset past any tensor here (at most 64 MB)

template <int D, int MG, bool SQ>
__device__ void stream_mfma(gcfloat* __restrict__ X, gfloat* __restrict__ out, uint32_t P, int K, uint32_t S,
                            int R, const float* us, double& xx, int tid) {
  X = uni(X);
  out = uni(out);
  P = uni(P);
  K = uni(K);
  S = uni(S);
  R = uni(R);
  const int lane = tid & (WAVE - 1), w = tid / WAVE, l16 = lane & 15, kq = lane >> 4;
  const uint32_t M = P * S;
  const int ngrp = int((M + 63) / 64);
  const int mygrp = ngrp > w ? (ngrp - w + NW - 1) / NW : 0;
  const int nks = (K + 3) >> 2;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)(const float*)X, short(0), int(M * uint32_t(K) * 4u), 0x00020000);
  const uint32_t step_bytes = P * 16u;
  gfloat* const og = out;
  // Drain every memory operation of the earlier phases (some are flat, which
  // count on both counters): with one pending here, the compiler could only
  // wait for zero outstanding loads at the top of every step group.
  __builtin_amdgcn_s_waitcnt(0);
  for (int t0 = 0; t0 < mygrp; t0 += MG) {
    uint32_t mg0[MG];  // first row of each group (M when the tile has no such group)
    uint32_t vo[MG];   // byte offset of the lane's run of each group at k = kq
#pragma unroll
    for (int g = 0; g < MG; ++g) {
      mg0[g] = t0 + g < mygrp ? uint32_t(w + NW * (t0 + g)) * 64u : M;
      const uint32_t m = mg0[g] + 4u * uint32_t(l16);
      const uint32_t s = m / P, p = m - s * P;
      vo[g] = m < M ? (p + P * (uint32_t(K) * s + uint32_t(kq))) * 4u : OOB;
    }
    auto load = [&](u32x4 (&dst)[MG], int st) {
      const bool kin = 4 * st + kq < K;
#pragma unroll
      for (int g = 0; g < MG; ++g)
        dst[g] = __builtin_amdgcn_raw_buffer_load_b128(rs, kin ? vo[g] : OOB, uint32_t(st) * step_bytes, 0);
    };
    floatx4 acc[MG][4];
    float sq[MG];
#pragma unroll
    for (int g = 0; g < MG; ++g) {
      sq[g] = 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[g][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    auto compute = [&](const u32x4 (&xu)[MG], int st) {
      const float bv = us[(4 * st + kq) * RB + l16];
#pragma unroll
      for (int g = 0; g < MG; ++g) {
        const floatx4 x = __builtin_bit_cast(floatx4, xu[g]);
        acc[g][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, bv, acc[g][0], 0, 0, 0);
        acc[g][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, bv, acc[g][1], 0, 0, 0);
        acc[g][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.z, bv, acc[g][2], 0, 0, 0);
        acc[g][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.w, bv, acc[g][3], 0, 0, 0);
        if (SQ) {
          sq[g] = fmaf(x.x, x.x, sq[g]);
          sq[g] = fmaf(x.y, x.y, sq[g]);
          sq[g] = fmaf(x.z, x.z, sq[g]);
          sq[g] = fmaf(x.w, x.w, sq[g]);
        }
      }
    };
    u32x4 xr[D][MG];
    // The loads leave in step order (no rescheduling across the barriers), so
    // that each wait in the loop is for the oldest loads only.
#pragma unroll
    for (int u = 0; u < D; ++u) {
      load(xr[u], u);
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int q = 0; q < nks; q += D) {
#pragma unroll
      for (int u = 0; u < D; ++u) {
        if (q + u < nks) compute(xr[u], q + u);
        load(xr[u], q + u + D);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (l16 < R) {
#pragma unroll
      for (int g = 0; g < MG; ++g)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const uint32_t m = mg0[g] + 16u * uint32_t(kq) + 4u * uint32_t(v);
          if (m < M) {
            const uint32_t s = m / P, p = m - s * P;
            *reinterpret_cast<__attribute__((address_space(1))) floatx4*>(og + p + size_t(P) * (size_t(l16) + size_t(R) * s)) =
                floatx4{acc[g][0][v], acc[g][1][v], acc[g][2][v], acc[g][3][v]};
          }
        }
    }
    if (SQ) {
#pragma unroll
      for (int g = 0; g < MG; ++g) xx += double(sq[g]);  // a missing group adds zero
    }
    // Let the stores finish before the next tile's loads go out, so that no
    // load waits behind a store of unknown order.
    __builtin_amdgcn_s_waitcnt(0);
  }
}

// ------------------------------------- contraction over the contiguous index
// out[p + P r + P R s] = sum_k X[k + L m] U[k, r] for the rows m = p + P s <
// M = P S (L a multiple of 4 and >= K, X 16-byte aligned), U in LDS as us4
// (zero for k >= K).  Tiles of 16 rows go on the M dimension of
// v_mfma_f32_16x16x4f32, MG tiles of a wave at a time (tiles dealt round
// robin).  In step t, lane (l16, kq) loads the 16-byte run k = 16 t + 4 kq
// .. + 3 of row l16 of each tile and feeds value j to MFMA j of the tile,
// whose k slots are 16 t + 4 kq + j; the four MFMAs of a tile add into the
// same accumulator.  Loads run D steps ahead within the MG tiles; runs past
// the row (k >= L) and rows past M read zeros (buffer range check).  The
// order of every sum is fixed by the layout, whatever D and MG.
template <int D, int MG>
__device__ void stream_k(gcfloat* __restrict__ X, gfloat* __restrict__ out, uint32_t L, int K, uint32_t P,
                         uint32_t S, int R, const float* us4, int tid) {
  X = uni(X);
  out = uni(out);
  L = uni(L);
  K = uni(K);
  P = uni(P);
  S = uni(S);
  R = uni(R);
  const int lane = tid & (WAVE - 1), w = tid / WAVE, l16 = lane & 15, kq = lane >> 4;
  const uint32_t M = P * S;
  const int ntile = int((M + 15) / 16);
  const int mytiles = ntile > w ? (ntile - w + NW - 1) / NW : 0;
  const int nks = (K + 15) >> 4;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)(const float*)X, short(0), int(M * L * 4u), 0x00020000);
  __builtin_amdgcn_s_waitcnt(0);  // as in stream_mfma
  for (int t0 = 0; t0 < mytiles; t0 += MG) {
    uint32_t m0[MG];  // first row of each tile (M when the wave has no such tile)
    uint32_t vo[MG];  // byte offset of the lane's run at k = 4 kq
#pragma unroll
    for (int g = 0; g < MG; ++g) {
      m0[g] = t0 + g < mytiles ? uint32_t(w + NW * (t0 + g)) * 16u : M;
      const uint32_t m = m0[g] + uint32_t(l16);
      vo[g] = m < M ? (m * L + 4u * uint32_t(kq)) * 4u : OOB;
    }
    auto load = [&](u32x4 (&dst)[MG], int st) {
      const bool kin = 16 * st + 4 * kq < int(L);
#pragma unroll
      for (int g = 0; g < MG; ++g)
        dst[g] = __builtin_amdgcn_raw_buffer_load_b128(rs, kin ? vo[g] : OOB, uint32_t(st) * 64u, 0);
    };
    floatx4 acc[MG];
#pragma unroll
    for (int g = 0; g < MG; ++g) acc[g] = floatx4{0.f, 0.f, 0.f, 0.f};
    auto compute = [&](const u32x4 (&xu)[MG], int st) {
      const floatx4 bv = *reinterpret_cast<const floatx4*>(us4 + ((4 * st + kq) * RB + l16) * 4);
#pragma unroll
      for (int g = 0; g < MG; ++g) {
        const floatx4 x = __builtin_bit_cast(floatx4, xu[g]);
        acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, bv.x, acc[g], 0, 0, 0);
        acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, bv.y, acc[g], 0, 0, 0);
        acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.z, bv.z, acc[g], 0, 0, 0);
        acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.w, bv.w, acc[g], 0, 0, 0);
      }
    };
    u32x4 xr[D][MG];
#pragma unroll
    for (int u = 0; u < D; ++u) {
      load(xr[u], u);
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int q = 0; q < nks; q += D) {
#pragma unroll
      for (int u = 0; u < D; ++u) {
        if (q + u < nks) compute(xr[u], q + u);
        load(xr[u], q + u + D);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (l16 < R) {
#pragma unroll
      for (int g = 0; g < MG; ++g)
#pragma unroll
        for (int v = 0; v < 4; ++v) {  // value v of the tile: row 4 kq + v, column l16
          const uint32_t m = m0[g] + 4u * uint32_t(kq) + uint32_t(v);
          if (m < M) {
            const uint32_t s = m / P, p = m - s * P;
            out[p + size_t(P) * (size_t(l16) + size_t(R) * s)] = acc[g][v];
          }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);  // as in stream_mfma
  }
}

__device__ inline void wg_sum16(double (&x)[RB], BShared& sh, int tid) {
  block_sum_vec<RB, NW>(x, sh.red, sh.res, tid);
}

__device__ inline double wg_sum1(double v, BShared& sh, int tid) {
  double x[1] = {v};
  block_sum_vec<1, NW>(x, sh.red, sh.res, tid);
  return sh.res[0];
}

// ------------------------------------------------------------- row steps
// Y_(n)(i, ru + R rt) = sum over the contracted index of U[., ru] times the
// source, U = Q_2 for mode 1 and Q_1 for modes 2 and 3 (new Q_1 for mode 2);
// ru, rt index the modes of Q_0's rows (ru fastest).  Y goes to global
// scratch at Y[i si + ru su + rt st]:
//   mode 1: from Z(i1, i2, r3), contract i2 (rows i1 of each r3 slab)
//   mode 2: from Z(i1, i2, r3), contract i1 (rows (i2, r3), i1 contiguous)
//   mode 3: from T(i1, r2, i3), contract i1 (rows (r2, i3), i1 contiguous)
struct YLayout {
  int64_t si, su, st;
};

__device__ inline YLayout y_layout(const GItem& it, int n) {
  const int64_t R = it.R, L0 = it.I0p, I1 = it.I[1];
  if (n == 0) return YLayout{1, L0, L0 * R};
  if (n == 1) return YLayout{1, I1, I1 * R};
  return YLayout{R * R, R, 1};
}

// Operands of mode n's row steps into LDS: U (in the layout its contraction
// reads), Q_0 (R^2 x R, FP64) and R_0.
__device__ __attribute__((always_inline)) void mode_begin(const GItem& it, int n, BShared& sh, int tid) {
  const int R = it.R;
  if (n == 0)
    stage_u(it.Qf[1], int(it.I[1]), sh.us, tid);
  else
    stage_u4(it.Qf[0], int(it.I[0]), sh.us, tid);
  gdouble* q0 = it.Q0b[n];
  for (int e = tid; e < R * R * R; e += NT) sh.q0[e] = q0[e];
  for (int e = tid; e < R * R; e += NT) sh.r0[e % R][e / R] = it.R0b[n][e];
  __syncthreads();
}

// Y_(n) of the whole mode into it.Y.
template <int D, int MG>
__device__ __attribute__((always_inline)) void task_y(const GItem& it, int n, BShared& sh, int tid) {
  const uint32_t L0 = uint32_t(it.I0p), I1 = uint32_t(it.I[1]), I2 = uint32_t(it.I[2]), R = uint32_t(it.R);
  double unused = 0.0;
  if (n == 0)       // out[i1 + L0 r2 + L0 R r3] = sum_i2 Z[i1 + L0 i2 + L0 I1 r3] Q_2[i2, r2]
    stream_mfma<D, MG, false>(it.Z, it.Y, L0, int(I1), R, int(R), sh.us, unused, tid);
  else if (n == 1)  // out[i2 + I1 r1 + I1 R r3] = sum_i1 Z[i1 + L0 (i2 + I1 r3)] Q_1[i1, r1]
    stream_k<D, MG>(it.Z, it.Y, L0, int(it.I[0]), I1, R, int(R), sh.us, tid);
  else              // out[r2 + R r1 + R^2 i3] = sum_i1 T[i1 + L0 (r2 + R i3)] Q_1[i1, r1]
    stream_k<D, MG>(it.T, it.Y, L0, int(it.I[0]), R, I2, int(R), sh.us, tid);
}

typedef double doublex4 __attribute__((ext_vector_type(4)));

// W = Y Q_0 for all rows of mode n on v_mfma_f64_16x16x4f64 (Y's FP32
// entries widened, FP64 products and sums), written into A[n] (column-major),
// which the substitution then overwrites row by row.  Tiles of 16 rows are
// dealt to the waves; step t takes Q_0 rows rho = 4 t + kq (lane (l16, kq)
// loads Y(row l16, rho) and Q_0(rho, l16), zero past R^2 and R), four steps
// of loads at a time.  The f64 MFMA returns row kq + 4 v of its tile in value
// v of lane (l16, kq).
__device__ __attribute__((always_inline)) void task_w(const GItem& it, int n, BShared& sh, int tid) {
  const int R = it.R;
  const int64_t In = it.I[n];
  const YLayout yl = y_layout(it, n);
  const int lane = tid & (WAVE - 1), w = tid / WAVE, l16 = lane & 15, kq = lane >> 4;
  const int K0 = R * R, nst = (K0 + 3) / 4;
  const int ntile = int((In + 15) / 16);
  gdouble* An = it.A[n];
  for (int t = w; t < ntile; t += NW) {
    const int64_t row = int64_t(t) * 16 + l16 < In ? int64_t(t) * 16 + l16 : In - 1;
    gcfloat* yr = it.Y + row * yl.si;
    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int st = 0; st < nst; st += 4) {
      float y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        int rho = 4 * (st + u) + kq;
        rho = rho < K0 ? rho : K0 - 1;
        const int rt = rho / R, ru = rho - rt * R;
        y[u] = yr[ru * yl.su + rt * yl.st];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int rho = 4 * (st + u) + kq;
        const double b = (rho < K0 && l16 < R) ? sh.q0[rho * R + l16] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(double(y[u]), b, acc, 0, 0, 0);
      }
    }
    if (l16 < R) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = int64_t(t) * 16 + kq + 4 * v;
        if (i < In) An[i + In * l16] = acc[v];
      }
    }
  }
}

// All rows of mode n, one per thread: the row of W from A[n], A R_0^T = W by
// substitution, then the column sums of squares of A (and for mode 3
// <W, A R_0^T>) as the single partial of slot 0.
__device__ __attribute__((always_inline)) void task_rows(const GItem& it, int n, BShared& sh, int tid) {
  const int R = it.R;
  const int64_t In = it.I[n];
  double w[RB];
#pragma unroll
  for (int c = 0; c < RB; ++c) w[c] = (tid < In && c < R) ? it.A[n][tid + In * c] : 0.0;
  double arow[RB], x[RB];
#pragma unroll
  for (int c = 0; c < RB; ++c) arow[c] = 0.0;
  double ip = 0.0;
  if (tid < In) {
#pragma unroll
    for (int j = RB - 1; j >= 0; --j) {
      if (j < R) {
        double v = w[j];
#pragma unroll
        for (int c = j + 1; c < RB; ++c)
          if (c < R) v -= sh.r0[j][c] * arow[c];
        arow[j] = v / sh.r0[j][j];
      }
    }
    gdouble* An = it.A[n] + tid;
#pragma unroll
    for (int c = 0; c < RB; ++c)
      if (c < R) An[int64_t(c) * In] = arow[c];
    if (n == 2) {
#pragma unroll
      for (int c = 0; c < RB; ++c) {
        if (c >= R) continue;
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < RB; ++k)
          if (k >= c && k < R) v += sh.r0[c][k] * arow[k];
        ip += w[c] * v;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < RB; ++c) x[c] = arow[c] * arow[c];
  wg_sum16(x, sh, tid);
  if (tid < RB) it.lamp[tid] = sh.res[tid];
  if (n == 2) {
    ip = wg_sum1(ip, sh, tid);
    if (tid == 0) it.ipp[0] = ip;
  }
}

// ------------------------------------------------------------ QR helper
// Householder QR of the rows a (row tid of thread tid, m rows; zero past
// column R and past row m), factorized in LDS.  Writes R (column-major R x R)
// to Rout and, if keep_rn, into sh.rn; Q as requested: column-major FP64
// (ld m), row-major FP32 padded to RB, row-major FP64 (ld R).
__device__ __attribute__((always_inline)) void qr_store(double (&a)[RB], int m, int R, BShared& sh, gdouble* Qcm, gfloat* Qf, gdouble* Qrm,
                         gdouble* Rout, bool keep_rn, int tid) {
  if (tid < IMAX) {
#pragma unroll
    for (int c = 0; c < RB; ++c) sh.qr.am[tid][c] = a[c];
  }
  wg_factor(tid, m, R, sh.qr);
  wg_build_t(tid, R, sh.qr);
  if (tid < R) {
#pragma unroll
    for (int c = 0; c < RB; ++c) {
      const double v = (c >= tid && c < R) ? sh.qr.am[tid][c] : 0.0;
      if (keep_rn) sh.rn[tid][c] = v;
      if (c < R) Rout[tid + c * R] = v;
    }
  }
  for (int e = tid; e < RB * RB; e += NT) sh.qr.C[e / RB][e % RB] = (e / RB == e % RB) ? 1.0 : 0.0;
  __syncthreads();
  double q[RB];
  wg_form_q(q, tid, m, R, sh.qr);
  if (tid < m) {
#pragma unroll
    for (int c = 0; c < RB; ++c) {
      if (Qcm && c < R) Qcm[tid + int64_t(c) * m] = q[c];
      if (Qrm && c < R) Qrm[tid * R + c] = q[c];
    }
    if (Qf) {
      __attribute__((address_space(1))) floatx4* dst = reinterpret_cast<__attribute__((address_space(1))) floatx4*>(Qf + tid * RB);
#pragma unroll
      for (int g = 0; g < RB / 4; ++g) {
        dst[g] = floatx4{4 * g < R ? float(q[4 * g]) : 0.f, 4 * g + 1 < R ? float(q[4 * g + 1]) : 0.f,
                         4 * g + 2 < R ? float(q[4 * g + 2]) : 0.f, 4 * g + 3 < R ? float(q[4 * g + 3]) : 0.f};
      }
    }
  }
  __syncthreads();
}

// QR of V_n = R_mb (.) R_ma (rows: index of ma fastest) into Q0b[n], R0b[n].
__device__ __attribute__((always_inline)) void krp_qr(const GItem& it, int n, BShared& sh, int tid) {
  const int R = it.R;
  const int ma = n == 0 ? 1 : 0, mb = n == 2 ? 1 : 2;
  const int K0 = R * R;
  double a[RB];
  const int da = tid % R, db = tid / R;
#pragma unroll
  for (int c = 0; c < RB; ++c)
    a[c] = (tid < K0 && c < R) ? it.Rf[ma][da + c * R] * it.Rf[mb][db + c * R] : 0.0;
  qr_store(a, K0, R, sh, nullptr, nullptr, it.Q0b[n], it.R0b[n], false, tid);
}

__device__ __attribute__((always_inline)) void task_init(const GItem& it, BShared& sh, int tid) {
  const int R = it.R;
  for (int k = 1; k < 3; ++k) {
    const int64_t Ik = it.I[k];
    double a[RB];
#pragma unroll
    for (int c = 0; c < RB; ++c) a[c] = (tid < Ik && c < R) ? it.A[k][tid + c * Ik] : 0.0;
    qr_store(a, int(Ik), R, sh, it.Q[k], it.Qf[k], nullptr, it.Rf[k], false, tid);
  }
  for (int c = tid; c < R; c += NT) it.lam[c] = 1.0;
  krp_qr(it, 0, sh, tid);
}

// Normalize A_n, factor QR of A_n, efficient error after mode 3, Khatri-Rao
// QR for the next mode.
__device__ __attribute__((always_inline)) void task_c(const GItem& it, int n, int sweep, int offset, BShared& sh, int tid) {
  const int R = it.R;
  const int64_t In = it.I[n];
  if (tid < RB) sh.lam[tid] = tid < R ? sqrt(it.lamp[tid]) : 0.0;
  __syncthreads();
  double a[RB];
#pragma unroll
  for (int c = 0; c < RB; ++c) {
    const double l = sh.lam[c];
    const double v = (tid < In && c < R) ? it.A[n][tid + c * In] : 0.0;
    a[c] = l > 0.0 ? v / l : 0.0;
  }
  if (tid < In) {
#pragma unroll
    for (int c = 0; c < RB; ++c)
      if (c < R) it.A[n][tid + c * In] = a[c];
  }
  for (int c = tid; c < R; c += NT) it.lam[c] = sh.lam[c];
  qr_store(a, int(In), R, sh, it.Q[n], it.Qf[n], nullptr, it.Rf[n], true, tid);
  if (n == 2) {  // ||X||^2 - 2 <W, A R_0^T> + <R_0^T R_0, L R_3^T R_3 L>   (section 3.3.1)
    for (int e = tid; e < R * R; e += NT) sh.r0[e % R][e / R] = it.R0b[2][e];
    double ip = 0.0, x2 = 0.0;
    if (tid == 0) {
      ip = it.ipp[0];
      x2 = *it.xnorm2;
    }
    __syncthreads();
    double nn = 0.0;
    for (int e = tid; e < R * R; e += NT) {
      const int p = e % R, q = e / R;
      double g0 = 0.0, gn = 0.0;
      for (int k = 0; k < R; ++k) {
        g0 += sh.r0[k][p] * sh.r0[k][q];
        gn += sh.rn[k][p] * sh.rn[k][q];
      }
      nn += g0 * sh.lam[p] * sh.lam[q] * gn;
    }
    ip = wg_sum1(ip, sh, tid);
    x2 = wg_sum1(x2, sh, tid);
    nn = wg_sum1(nn, sh, tid);
    if (tid == 0 && it.relerr) {
      const double r2 = x2 - 2.0 * ip + nn;
      it.relerr[offset + sweep] = isnan(r2) ? r2 : sqrt((r2 > 0.0 ? r2 : 0.0) / x2);  // NaN stays NaN
    }
    __syncthreads();
  }
  krp_qr(it, n == 2 ? 0 : n + 1, sh, tid);
}

// Streaming contraction over the whole tensor: Z = X x_3 Q_3^T (isz) or
// T = X x_2 Q_2^T.  Z also yields ||X||^2.
template <int D, int MG>
__device__ __attribute__((always_inline)) void task_a(const GItem& it, bool isz, BShared& sh, int tid) {
  const int k = isz ? 2 : 1;
  stage_u(it.Qf[k], int(it.I[k]), sh.us, tid);
  __syncthreads();
  const uint32_t L0 = uint32_t(it.I0p), I1 = uint32_t(it.I[1]), I2 = uint32_t(it.I[2]);
  double xx = 0.0;
  if (isz)
    stream_mfma<D, MG, true>(it.X, it.Z, L0 * I1, int(I2), 1u, it.R, sh.us, xx, tid);
  else
    stream_mfma<D, MG, false>(it.X, it.T, L0, int(I1), I2, it.R, sh.us, xx, tid);
  if (isz) {
    xx = wg_sum1(xx, sh, tid);
    if (tid == 0) *it.xnorm2 = xx;
  }
}

// One sweep schedule per tensor; the streaming passes keep D contraction
// steps of MG row groups in flight per lane.
template <int D, int MG>
__global__ __launch_bounds__(NT, 1) void als_batch_kernel(const BItem* __restrict__ items,
                                                          const int* __restrict__ order, int nsweeps, int do_init,
                                                          int offset) {
  __shared__ BShared sh;
  // The descriptor lives in LDS: its fields are read where they are used
  // instead of being held in registers for the whole launch.
  __shared__ GItem itl;
  const int tid = threadIdx.x;
  {
    const int* src = reinterpret_cast<const int*>(items + order[blockIdx.x]);
    int* dst = reinterpret_cast<int*>(&itl);
    for (int e = tid; e < int(sizeof(GItem) / sizeof(int)); e += NT) dst[e] = src[e];
  }
  __syncthreads();
  const GItem& it = itl;
  if (do_init) {
    task_init(it, sh, tid);
    __syncthreads();
  }
  for (int s = 0; s < nsweeps; ++s) {
    for (int n = 0; n < 3; ++n) {
      if (n == 0 || n == 2) {
        task_a<D, MG>(it, n == 0, sh, tid);
        __syncthreads();
      }
      mode_begin(it, n, sh, tid);
      task_y<D, MG>(it, n, sh, tid);
      __syncthreads();
      task_w(it, n, sh, tid);
      __syncthreads();
      task_rows(it, n, sh, tid);
      __syncthreads();
      task_c(it, n, s, offset, sh, tid);
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------ host side
// Streaming-pass shapes the autotuner chooses from: steps in flight (D) and
// 64-row groups per wave tile (MG).
constexpr int NVAR = 3;
constexpr int VAR_D[NVAR] = {8, 4, 16};
constexpr int VAR_MG[NVAR] = {2, 4, 1};

struct Config {
  int var;   // streaming-pass shape
  int rows;  // kept for the cache file format; the row steps take whole modes (0)
};


// The streaming passes read 16-byte runs along the first mode: a tensor is
// streamed in place when its first mode is a multiple of 4 and it is
// 16-byte aligned, else from a copy whose first mode is zero-padded.
bool needs_copy(const cpqr_batch_item& b) {
  return b.I[0] % 4 != 0 || reinterpret_cast<uintptr_t>(b.X) % 16 != 0;
}

size_t item_scratch(const cpqr_batch_item& b) {
  const int64_t R = b.R;
  const int64_t i0 = b.I[0], i1 = b.I[1], i2 = b.I[2];
  Carver cv(nullptr);
  for (int m = 0; m < 3; ++m) cv.take<double>(size_t(b.I[m]) * R);  // Q
  for (int m = 0; m < 3; ++m) cv.take<float>(size_t(b.I[m]) * RB);  // Qf
  for (int m = 0; m < 3; ++m) cv.take<double>(size_t(R) * R);       // Rf
  for (int m = 0; m < 3; ++m) cv.take<double>(size_t(R) * R * R);   // Q0b
  for (int m = 0; m < 3; ++m) cv.take<double>(size_t(R) * R);       // R0b
  const int64_t l0 = (i0 + 3) / 4 * 4;
  cv.take<float>(size_t(l0 * i1 * R));                             // Z
  cv.take<float>(size_t(l0 * R * i2));                             // T
  if (needs_copy(b)) cv.take<float>(size_t(l0 * i1 * i2));         // padded copy of X
  cv.take<float>(size_t(std::max(l0, std::max(i1, i2)) * R * R));  // Y
  cv.take<double>(size_t(RB));                                     // lamp
  cv.take<double>(1);                                              // ipp
  cv.take<double>(1);                                              // xnorm2
  return cv.bytes();
}

// What cpqr_als_batch_prepare decided for one work buffer (host side).
struct BatchState {
  int n = 0;
  Config cfg{};
  std::vector<BItem> h;  // host copy of the device descriptors
  BItem* items_dev = nullptr;
  int* order_dev = nullptr;
};

std::mutex g_batch_mu;
std::map<const void*, BatchState> g_batch;

int upload(BatchState& st, hipStream_t s) {
  for (auto& d : st.h) {
    for (int m = 0; m < 3; ++m) {
      d.rows[m] = int(d.I[m]);  // the row steps take a whole mode at once
      d.nB[m] = 1;
    }
  }
  CPQR_HIP(hipMemcpyAsync(st.items_dev, st.h.data(), sizeof(BItem) * st.n, hipMemcpyHostToDevice, s));
  CPQR_HIP(hipStreamSynchronize(s));  // the host copy may change after this call
  return CPQR_OK;
}

int launch_batch(const BatchState& st, int var, int nsweeps, int do_init, int offset, hipStream_t s) {
  const dim3 grd(unsigned(st.n)), blk(NT);
  switch (var) {
    case 0:
      hipLaunchKernelGGL((als_batch_kernel<VAR_D[0], VAR_MG[0]>), grd, blk, 0, s, st.items_dev, st.order_dev,
                         nsweeps, do_init, offset);
      break;
    case 1:
      hipLaunchKernelGGL((als_batch_kernel<VAR_D[1], VAR_MG[1]>), grd, blk, 0, s, st.items_dev, st.order_dev,
                         nsweeps, do_init, offset);
      break;
    default:
      hipLaunchKernelGGL((als_batch_kernel<VAR_D[2], VAR_MG[2]>), grd, blk, 0, s, st.items_dev, st.order_dev,
                         nsweeps, do_init, offset);
      break;
  }
  return check_launch("als_batch_kernel");
}

struct GraphKey {
  const void* work;
  int nsweeps, init, offset, var;
  bool operator<(const GraphKey& o) const {
    if (work != o.work) return work < o.work;
    if (nsweeps != o.nsweeps) return nsweeps < o.nsweeps;
    if (init != o.init) return init < o.init;
    if (offset != o.offset) return offset < o.offset;
    return var < o.var;
  }
};
std::map<GraphKey, hipGraphExec_t> g_graphs;
hipStream_t g_capture_stream = nullptr;

// ------------------------------------------------------------ autotune cache
std::mutex g_tune_mu;
std::map<std::string, Config> g_tune;
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
  Config c{};
  while (fscanf(f, "%255s %d %d", key, &c.var, &c.rows) == 3) g_tune[key] = c;
  fclose(f);
}

void tune_store() {
  const std::string p = tune_path();
  const size_t slash = p.find_last_of('/');
  if (slash != std::string::npos) mkdir(p.substr(0, slash).c_str(), 0755);  // best effort
  FILE* f = fopen(p.c_str(), "w");
  if (!f) return;
  for (auto& kv : g_tune) fprintf(f, "%s %d %d\n", kv.first.c_str(), kv.second.var, kv.second.rows);
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
  snprintf(buf, sizeof(buf), "batch4|%s|n%d|imax%lld|rmax%d|elems2^%d", arch.c_str(), n,
           (long long)((maxi + 31) / 32 * 32), maxr, lg);
  return buf;
}

int batch_lookup(void* work, int variant, BatchState*& st, int& var) {
  if (!work) return fail(CPQR_ERR_WORKSPACE, "als_batch: work buffer is NULL");
  std::lock_guard<std::mutex> g(g_batch_mu);
  auto f = g_batch.find(work);
  if (f == g_batch.end()) return fail(CPQR_ERR_WORKSPACE, "als_batch: work buffer not prepared");
  st = &f->second;
  if (variant < 0 || variant > NVAR) return fail(CPQR_ERR_ARG, "als_batch: variant must be 0 (tuned) or 1..3");
  var = variant > 0 ? variant - 1 : st->cfg.var;
  return CPQR_OK;
}

}  // namespace
}  // namespace cpqr

using namespace cpqr;

extern "C" {

size_t cpqr_als_batch_work(const cpqr_batch_item* items, int nitems) {
  if (!items || nitems < 1) return 0;
  for (int b = 0; b < nitems; ++b)
    if (items[b].R < 1 || items[b].R > RB || items[b].I[0] < 1 || items[b].I[1] < 1 || items[b].I[2] < 1) return 0;
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
    if (it.R < 1 || it.R > RB) return fail(CPQR_ERR_SHAPE, "als_batch: R must be in [1, 16]");
    for (int k = 0; k < 3; ++k) {
      if (it.I[k] < it.R || it.I[k] > IMAX) return fail(CPQR_ERR_SHAPE, "als_batch: mode sizes must be in [R, 256]");
      if (!it.A[k]) return fail(CPQR_ERR_ARG, "als_batch: NULL factor");
    }
    if (!it.X || !it.lambda) return fail(CPQR_ERR_ARG, "als_batch: NULL tensor or lambda");
    if (reinterpret_cast<uintptr_t>(it.X) % 4 != 0) return fail(CPQR_ERR_ARG, "als_batch: X must be 4-byte aligned");
  }
  CPQR_TRY(check_work(work, work_bytes, cpqr_als_batch_work(items, nitems)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  BatchState st;
  st.n = nitems;
  Carver cv(work);
  st.items_dev = cv.take<BItem>(nitems);
  st.order_dev = cv.take<int>(nitems);
  std::vector<double*> saved(2 * nitems);
  for (int b = 0; b < nitems; ++b) {
    saved[2 * b] = cv.take<double>(size_t(items[b].I[1]) * items[b].R);
    saved[2 * b + 1] = cv.take<double>(size_t(items[b].I[2]) * items[b].R);
  }
  st.h.resize(nitems);
  for (int b = 0; b < nitems; ++b) {
    const cpqr_batch_item& it = items[b];
    Carver c2(cv.take<char>(item_scratch(it)));
    BItem& d = st.h[b];
    d = BItem{};
    for (int k = 0; k < 3; ++k) d.I[k] = it.I[k];
    d.R = it.R;
    d.X = it.X;
    for (int k = 0; k < 3; ++k) d.A[k] = it.A[k];
    d.lam = it.lambda;
    d.relerr = it.relerr;
    const int64_t R = it.R;
    for (int k = 0; k < 3; ++k) d.Q[k] = c2.take<double>(size_t(it.I[k]) * R);
    for (int k = 0; k < 3; ++k) d.Qf[k] = c2.take<float>(size_t(it.I[k]) * RB);
    for (int k = 0; k < 3; ++k) d.Rf[k] = c2.take<double>(size_t(R) * R);
    for (int k = 0; k < 3; ++k) d.Q0b[k] = c2.take<double>(size_t(R) * R * R);
    for (int k = 0; k < 3; ++k) d.R0b[k] = c2.take<double>(size_t(R) * R);
    d.I0p = (it.I[0] + 3) / 4 * 4;
    d.Z = c2.take<float>(size_t(d.I0p * it.I[1] * R));
    d.T = c2.take<float>(size_t(d.I0p * R * it.I[2]));
    if (needs_copy(it)) {
      float* xp = c2.take<float>(size_t(d.I0p * it.I[1] * it.I[2]));
      CPQR_HIP(hipMemsetAsync(xp, 0, sizeof(float) * size_t(d.I0p * it.I[1] * it.I[2]), s));
      CPQR_HIP(hipMemcpy2DAsync(xp, sizeof(float) * size_t(d.I0p), it.X, sizeof(float) * size_t(it.I[0]),
                                sizeof(float) * size_t(it.I[0]), size_t(it.I[1] * it.I[2]), hipMemcpyDeviceToDevice, s));
      d.X = xp;
    }
    d.Y = c2.take<float>(size_t(std::max(d.I0p, std::max(it.I[1], it.I[2])) * R * R));
    d.lamp = c2.take<double>(size_t(RB));
    d.ipp = c2.take<double>(1);
    d.xnorm2 = c2.take<double>(1);
  }
  // larger tensors first (longest-processing-time order)
  std::vector<int> order(nitems);
  for (int b = 0; b < nitems; ++b) order[b] = b;
  const auto work_of = [&](int t) {
    return double(items[t].I[0]) * double(items[t].I[1]) * double(items[t].I[2]) * (2.0 + items[t].R);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work_of(a) > work_of(b); });
  CPQR_HIP(hipMemcpyAsync(st.order_dev, order.data(), sizeof(int) * nitems, hipMemcpyHostToDevice, s));
  for (int b = 0; b < nitems; ++b) {
    CPQR_HIP(hipMemcpyAsync(saved[2 * b], items[b].A[1], sizeof(double) * items[b].I[1] * items[b].R,
                            hipMemcpyDeviceToDevice, s));
    CPQR_HIP(hipMemcpyAsync(saved[2 * b + 1], items[b].A[2], sizeof(double) * items[b].I[2] * items[b].R,
                            hipMemcpyDeviceToDevice, s));
  }
  st.cfg = Config{1, 0};
  if (autotune) {
    const std::string key = tune_key(items, nitems);
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_load();
    auto found = g_tune.find(key);
    if (found != g_tune.end() && found->second.var >= 0 && found->second.var < NVAR &&
        found->second.rows == 0) {
      st.cfg = found->second;
    } else {
      // time one init + sweep per candidate, restoring the initial factors after each
      hipEvent_t e0, e1;
      CPQR_HIP(hipEventCreate(&e0));
      CPQR_HIP(hipEventCreate(&e1));
      float best = 1e30f;
      Config bestc = st.cfg;
      for (int var = 0; var < NVAR; ++var) {
        st.cfg = Config{var, 0};
        CPQR_TRY(upload(st, s));
        CPQR_TRY(launch_batch(st, var, 1, 1, 0, s));  // warm
        CPQR_HIP(hipEventRecord(e0, s));
        CPQR_TRY(launch_batch(st, var, 1, 1, 0, s));
        CPQR_HIP(hipEventRecord(e1, s));
        CPQR_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        CPQR_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          bestc = st.cfg;
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
      st.cfg = bestc;
      g_tune[key] = bestc;
      tune_store();
    }
  }
  CPQR_TRY(upload(st, s));
  {
    std::lock_guard<std::mutex> g(g_batch_mu);
    for (auto it = g_graphs.begin(); it != g_graphs.end();) {  // graphs of an older layout
      if (it->first.work == work) {
        (void)hipGraphExecDestroy(it->second);
        it = g_graphs.erase(it);
      } else {
        ++it;
      }
    }
    g_batch[work] = std::move(st);
  }
  return CPQR_OK;
}

int cpqr_als_batch_run(void* work, int nsweeps, int init, int sweep_offset, int variant, void* stream) {
  if (nsweeps < 0 || sweep_offset < 0) return fail(CPQR_ERR_ARG, "als_batch: negative sweep count");
  BatchState* st;
  int var;
  CPQR_TRY(batch_lookup(work, variant, st, var));
  return launch_batch(*st, var, nsweeps, init ? 1 : 0, sweep_offset, static_cast<hipStream_t>(stream));
}

int cpqr_als_batch_graph(void* work, int nsweeps, int init, int sweep_offset, int variant, void* stream) {
  if (nsweeps < 0 || sweep_offset < 0) return fail(CPQR_ERR_ARG, "als_batch: negative sweep count");
  BatchState* st;
  int var;
  CPQR_TRY(batch_lookup(work, variant, st, var));
  const GraphKey key{work, nsweeps, init ? 1 : 0, sweep_offset, var};
  hipGraphExec_t exec = nullptr;
  {
    std::lock_guard<std::mutex> g(g_batch_mu);
    auto f = g_graphs.find(key);
    if (f != g_graphs.end()) exec = f->second;
  }
  if (!exec) {
    if (!g_capture_stream) CPQR_HIP(hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking));
    CPQR_HIP(hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal));
    const int rc = launch_batch(*st, var, nsweeps, init ? 1 : 0, sweep_offset, g_capture_stream);
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

int cpqr_als_batch_config(void* work, int* cols_per_thread, int* unroll, int* rows) {
  BatchState* st;
  int var;
  CPQR_TRY(batch_lookup(work, 0, st, var));
  if (cols_per_thread) *cols_per_thread = 4 * VAR_MG[var];
  if (unroll) *unroll = VAR_D[var];
  if (rows) *rows = st->cfg.rows;
  return CPQR_OK;
}

}  // extern "C"
