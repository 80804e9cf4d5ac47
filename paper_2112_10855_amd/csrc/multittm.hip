// Multi-TTM Y = X x_k Q_k^T for all k != n (paper section 2.2, eq. multittm;
// Alg. 2), returned as the unfolding Y_(n).  This is the dominant cost of
// CP-ALS-QR (section 3.2): the first contraction streams the whole tensor,
// each later one works on a tensor R/I_k times smaller.
//
// Every contraction is "contract the middle index of a [P, K, S] array":
//     T'[p, r, s] = sum_i T[p, i, s] U[i, r],   U = Q_k (K x R),
// where P (S) is the product of the sizes of the modes before (after) the
// contracted mode in the current tensor, all column-major.  The output keeps
// the column-major layout with the contracted mode resized to R.
//
// Kernels (gfx950, wave64):
//  * ttm_mfma_m: P a multiple of 4.  Rows m = p + P s of the [M = P S, K]
//    matrix go on the MFMA M dimension.  Each lane loads a float4 of four
//    consecutive p (16 lanes cover 64 contiguous floats = 256 B per K index)
//    and feeds its four components to four v_mfma_f32_16x16x4f32 calls that
//    share the B operand (16 columns of U).  One wavefront owns 64 rows and
//    all R outputs; the K range can be split across workgroups (split-K) with
//    a deterministic reduction.
//  * ttm_mfma_k: P = 1 (contract the fastest mode), K a multiple of 4.  Each
//    lane loads a float4 of four consecutive i of one column s; U is stored
//    with four consecutive i interleaved so one float4 load feeds the four
//    MFMAs.  The output is R x S.
//  * ttm_valu: anything else, and the FP64 path: one thread per row m, all R
//    outputs in registers, FMA on the vector ALUs.
//  The last contraction lands in the tensor layout [P_n, I_n, S_n]; unless
//  n is the first mode a permute kernel writes the unfolding Y_(n).

#include <type_traits>
#include <hip/hip_ext.h>

#include <algorithm>

#include "common.h"

namespace cpqr {

// Launch with the dispatch's own start/stop events when they are set.
template <typename... Args, typename F = void (*)(Args...)>
void launch_ev(const KernelEvents& ke, F kernel, const dim3& grid, const dim3& block, size_t lds, hipStream_t st,
               Args... args) {
  if (ke.a)
    hipExtLaunchKernelGGL(kernel, grid, block, uint32_t(lds), st, ke.a, ke.b, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
}
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Tensor loads of the row-tiled kernels; NT marks them non-temporal.  A
// first contraction whose contracted-matrix rows are 128-byte multiples apart
// (P % 32 == 0) shares no cache line between row tiles and streams faster so
// (1000^3, mode-3 contraction: 0.70 -> 0.66 ms on MI355X); with unaligned
// rows (P = 1000) neighbouring tiles share lines and the hint costs 7 %.
template <bool NT>
__device__ __forceinline__ float4 ldx(const float* p) {
  if constexpr (NT) {
    const floatx4 v = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
  } else {
    return *reinterpret_cast<const float4*>(p);
  }
}

constexpr int WAVE = 64;
constexpr int TARGET_WAVES = 2048;  // wavefronts wanted when K is split (8 per CU)
constexpr int MIN_WAVES = 1024;     // below this many wavefronts, split K

// n floats (a multiple of 4, 16-byte aligned) from global memory into LDS
// by the NTH threads of a workgroup; every load of a batch is issued before
// the first LDS store, so the batch costs one round trip, not one per load.
template <int NTH>
__device__ __forceinline__ void stage_lds(const float* __restrict__ src, float* dst, int n, int tid) {
  constexpr int B = 8;
  const int n4 = n / 4;
  const float4* s4 = reinterpret_cast<const float4*>(src);
  float4* d4 = reinterpret_cast<float4*>(dst);
  for (int e0 = 0; e0 < n4; e0 += B * NTH) {
    float4 t[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int e = e0 + tid + i * NTH;
      t[i] = e < n4 ? s4[e] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int e = e0 + tid + i * NTH;
      if (e < n4) d4[e] = t[i];
    }
  }
}

// Steps of a row-tile kernel's load ring: three where the accumulators leave
// room (two 16-column blocks of one row group or fewer), else two; 0 (a
// plain pair of load buffers) for steps of more than four 16-byte loads per
// lane, whose ring would not fit four wavefronts per SIMD.
constexpr int ring_depth(int NB, int UN, int MG) { return UN * MG > 4 ? 0 : NB * MG <= 2 ? 3 : 2; }

// ------------------------------------------------------------ U preparation
// Row-major K x RP, zero padded: U[i*RP + r] = Q[i + r*ldq] (r < R).
template <class T>
__global__ void prep_u_rows(const double* __restrict__ Q, int64_t K, int64_t ldq, int R, int RP,
                            T* __restrict__ U) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= K * RP) return;
  const int64_t i = e / RP;
  const int r = int(e % RP);
  U[e] = r < R ? T(Q[i + r * ldq]) : T(0);
}

// Interleaved by four: U4[((i/4)*RP + r)*4 + i%4] = Q[i + r*ldq]; K % 4 == 0.
__global__ void prep_u_quads(const double* __restrict__ Q, int64_t K, int64_t ldq, int R, int RP,
                             float* __restrict__ U) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= K * RP) return;
  const int64_t q = e / (int64_t(RP) * 4);
  const int rem = int(e % (int64_t(RP) * 4));
  const int r = rem / 4, t = rem % 4;
  const int64_t i = q * 4 + t;
  U[e] = r < R ? float(Q[i + r * ldq]) : 0.0f;
}

// ------------------------------------------------------------ MFMA kernels
// Both MFMA kernels stage the contraction operand U in LDS, KC rows at a time
// (KC * RP floats <= 64 KB), shared by the NWV wavefronts of the workgroup.
// Inside a chunk the tensor loads are software pipelined with two register
// buffers (A, B): the loads of step t+1 are in flight while step t runs on the
// matrix cores.  Main-loop loads are unconditional (invalid rows and columns
// read a clamped in-bounds address and are never stored), so the compiler
// keeps them branch-free; the chunk tail is a separate masked step.
constexpr int LDS_FLOATS = 16384;  // 64 KB

// Output of the row-tiled kernels.  In the MFMA D layout, lane (l16, kq)
// holds for tile g the 16 consecutive rows m0 = mt + 64 g + 16 kq, ... of
// column l16 (row 4 v + j of the group in acc[g][j][v]).  When the 16 rows lie
// in one slab of P they are 64 contiguous bytes of the output, written as
// four float4 stores; otherwise (a slab boundary inside the group, the grid's
// end, or an output not 16-byte aligned) element by element.
template <int NB, int MG>
__device__ __forceinline__ void store_tiles(const floatx4 (&acc)[NB][MG][4], float* __restrict__ o, int64_t mt,
                                            int64_t M, int64_t P, int R, int l16, int kq) {
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int r = b * 16 + l16;
    if (r >= R) continue;
#pragma unroll
    for (int g = 0; g < MG; ++g) {
      const int64_t m0 = mt + 64 * g + 16 * kq;
      const int64_t p0 = m0 % P, s0 = m0 / P;
      float* d = o + p0 + r * P + s0 * P * R;
      if (m0 + 16 <= M && p0 + 16 <= P && (reinterpret_cast<uintptr_t>(d) & 15) == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          *reinterpret_cast<float4*>(d + 4 * q) =
              make_float4(acc[b][g][0][q], acc[b][g][1][q], acc[b][g][2][q], acc[b][g][3][q]);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t m = m0 + 4 * v + j;
            if (m < M) o[m % P + r * P + (m / P) * P * R] = acc[b][g][j][v];
          }
      }
    }
  }
}

// ---------------- P % 4 == 0: rows m = p + P s on the MFMA M dimension
// STREAM marks the instantiation used for a first contraction (it streams the
// whole tensor); it is the same code under its own symbol so that profiles and
// phase timers can single it out.
template <int NB, int UN, int MG, int NWV, bool STREAM, bool ONE, bool NT = false>
__global__ __launch_bounds__(NWV * 64) void ttm_mfma_m(const float* __restrict__ X,
                                                       const float* __restrict__ U,
                                                       float* __restrict__ out, int64_t P,
                                                       int64_t K, int64_t S, int R, int64_t kchunk,
                                                       int64_t split_stride) {
  constexpr int RP = 16 * NB;
  extern __shared__ float us[];
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int64_t M = P * S;
  const int64_t mt = (int64_t(blockIdx.x) * NWV + w) * 64 * MG;
  const bool active = mt < M;
  const int64_t kb0 = int64_t(blockIdx.y) * kchunk;
  const int64_t kb1 = min(K, kb0 + kchunk);
  const int l16 = lane % 16, kq = lane / 16;
  const float* base[MG];
#pragma unroll
  for (int g = 0; g < MG; ++g) {
    int64_t mrow = mt + 64 * g + 4 * l16;
    mrow = mrow < M ? mrow : M - 4;
    const int64_t p = mrow % P, s = mrow / P;
    base[g] = X + p + s * P * K + kq * P;
  }
  floatx4 acc[NB][MG][4];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int g = 0; g < MG; ++g)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[b][g][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  constexpr int STEP = 4 * UN;
  // rows [c0, c0 + cn) of U are in LDS (cn <= KC)
  auto chunk = [&](int64_t c0, int cn) {
    const int nfull = cn / STEP;
    const int last = nfull > 0 ? (nfull - 1) * STEP : 0;
    const float* bp[MG];
#pragma unroll
    for (int g = 0; g < MG; ++g) bp[g] = base[g] + c0 * P;
    auto load = [&](float4(&dst)[UN][MG], int t) {  // steps past the last full one re-read it
      const int i0 = min(t * STEP, last);
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int g = 0; g < MG; ++g)
          dst[u][g] = ldx<NT>(bp[g] + int64_t(i0 + 4 * u) * P);
    };
    auto compute = [&](const float4(&src)[UN][MG], int t) {
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const float bv = us[(t * STEP + 4 * u + kq) * RP + b * 16 + l16];
#pragma unroll
          for (int g = 0; g < MG; ++g) {
            acc[b][g][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(src[u][g].x, bv, acc[b][g][0], 0, 0, 0);
            acc[b][g][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(src[u][g].y, bv, acc[b][g][1], 0, 0, 0);
            acc[b][g][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(src[u][g].z, bv, acc[b][g][2], 0, 0, 0);
            acc[b][g][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(src[u][g].w, bv, acc[b][g][3], 0, 0, 0);
          }
        }
    };
    // A ring of D steps in flight (D > 0).  The loads leave in step order (no
    // rescheduling across the barriers) and are unconditional, so that the
    // wait before each step is for that step's loads only.
    constexpr int D = ring_depth(NB, UN, MG);
    if constexpr (D == 0) {
      float4 A[UN][MG], B[UN][MG];
      if (nfull > 0) {
        load(A, 0);
        for (int t = 0; t < nfull; t += 2) {
          load(B, t + 1);
          compute(A, t);
          load(A, t + 2);
          if (t + 1 < nfull) compute(B, t + 1);
        }
      }
    } else if (nfull > 0) {
      float4 xr[D][UN][MG];
#pragma unroll
      for (int u = 0; u < D; ++u) {
        load(xr[u], u);
        __builtin_amdgcn_sched_barrier(0);
      }
      for (int q = 0; q < nfull; q += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
          if (q + u < nfull) compute(xr[u], q + u);
          load(xr[u], q + u + D);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    for (int i = nfull * STEP; i < cn; i += 4) {  // chunk tail
      const int ii = i + kq;
      const bool ok = ii < cn;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const float bv = ok ? us[ii * RP + b * 16 + l16] : 0.f;
#pragma unroll
        for (int g = 0; g < MG; ++g) {
          const float4 xv = ok ? *reinterpret_cast<const float4*>(bp[g] + int64_t(i) * P)
                               : make_float4(0.f, 0.f, 0.f, 0.f);
          acc[b][g][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.x, bv, acc[b][g][0], 0, 0, 0);
          acc[b][g][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.y, bv, acc[b][g][1], 0, 0, 0);
          acc[b][g][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.z, bv, acc[b][g][2], 0, 0, 0);
          acc[b][g][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.w, bv, acc[b][g][3], 0, 0, 0);
        }
      }
    }
  };
  if constexpr (ONE) {  // the workgroup's K range fits in LDS: stage once, no chunk loop
    const int cn = int(kb1 > kb0 ? kb1 - kb0 : 0);
    const float* Uc = U + kb0 * RP;
    stage_lds<NWV * 64>(Uc, us, cn * RP, tid);
    __syncthreads();
    if (!active) return;
    chunk(kb0, cn);
  } else {
    constexpr int KC = (LDS_FLOATS / RP) / STEP * STEP;
    for (int64_t c0 = kb0; c0 < kb1; c0 += KC) {
      const int cn = int(min<int64_t>(kb1 - c0, KC));
      __syncthreads();
      const float* Uc = U + c0 * RP;
      stage_lds<NWV * 64>(Uc, us, cn * RP, tid);
      __syncthreads();
      if (active) chunk(c0, cn);
    }
    if (!active) return;
  }
  store_tiles<NB, MG>(acc, out + int64_t(blockIdx.y) * split_stride, mt, M, P, R, l16, kq);
}

// ---------------- FP64: the same row tiles on v_mfma_f64_16x16x4f64
// Each lane loads four consecutive doubles (rows 4 l16 .. 4 l16 + 3 of its
// 64-row group, two 16-byte loads) of K-row kq of a step and feeds them to
// four MFMAs sharing one B operand (16 columns of U, FP64 in LDS).  The f64
// MFMA returns row kq + 4 v of its 16 x 16 result in value v of lane
// (l16, kq), so the lane ends up with rows 16 v + 4 kq + j (j = MFMA index)
// of column l16: four runs of four consecutive rows.
typedef double doublex2 __attribute__((ext_vector_type(2)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ doublex2 ldx2(const double* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(reinterpret_cast<const doublex2*>(p));
  else
    return *reinterpret_cast<const doublex2*>(p);
}

constexpr int LDS_DOUBLES = 8192;  // 64 KB

// Four consecutive elements of X (FP64, or FP32 widened) as two pairs.
template <bool NT>
__device__ __forceinline__ void ldx4(const double* q, doublex2& a, doublex2& b) {
  a = ldx2<NT>(q);
  b = ldx2<NT>(q + 2);
}
template <bool NT>
__device__ __forceinline__ void ldx4(const float* q, doublex2& a, doublex2& b) {
  const float4 v = ldx<NT>(q);
  a = doublex2{double(v.x), double(v.y)};
  b = doublex2{double(v.z), double(v.w)};
}

// GENP: P need not be a multiple of 4 (the four rows of a lane may straddle
// slabs), so each of them is loaded by its own address; the four loads of a
// step cover the same lines as one vector load would.
template <int NB, int UN, int MG, int NWV, bool STREAM, bool NT, class TX = double, bool GENP = false>
__global__ __launch_bounds__(NWV * 64) void ttm_mfma_m_f64(const TX* __restrict__ X,
                                                           const double* __restrict__ U,
                                                           double* __restrict__ out, int64_t P, int64_t K,
                                                           int64_t S, int R, int64_t kchunk,
                                                           int64_t split_stride) {
  constexpr int RP = 16 * NB;
  extern __shared__ double usd[];
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int64_t M = P * S;
  const int64_t mt = (int64_t(blockIdx.x) * NWV + w) * 64 * MG;
  const bool active = mt < M;
  const int64_t kb0 = int64_t(blockIdx.y) * kchunk;
  const int64_t kb1 = min(K, kb0 + kchunk);
  const int l16 = lane % 16, kq = lane / 16;
  const TX* base[MG];
  const TX* rb[GENP ? MG : 1][4];  // GENP: the lane's four rows (clamped into the tensor)
#pragma unroll
  for (int g = 0; g < MG; ++g) {
    int64_t mrow = mt + 64 * g + 4 * l16;
    if (GENP) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t m = min(mrow + j, M - 1);
        rb[GENP ? g : 0][j] = X + m % P + (m / P) * P * K + kq * P;
      }
      base[g] = rb[GENP ? g : 0][0];
    } else {
      mrow = mrow < M ? mrow : M - 4;
      const int64_t p = mrow % P, s = mrow / P;
      base[g] = X + p + s * P * K + kq * P;
    }
  }
  // the four rows of group g at K row i: one vector load, or four
  auto ld4 = [&](int g, int64_t i, bool nt_ok, doublex2& lo, doublex2& hi) {
    if (GENP) {
      const int64_t o = i * P;
      lo = doublex2{double(rb[GENP ? g : 0][0][o]), double(rb[GENP ? g : 0][1][o])};
      hi = doublex2{double(rb[GENP ? g : 0][2][o]), double(rb[GENP ? g : 0][3][o])};
    } else if (nt_ok) {
      ldx4<NT>(base[g] + i * P, lo, hi);
    } else {
      ldx4<false>(base[g] + i * P, lo, hi);
    }
  };
  doublex4 acc[NB][MG][4];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int g = 0; g < MG; ++g)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[b][g][j] = doublex4{0.0, 0.0, 0.0, 0.0};

  constexpr int STEP = 4 * UN;
  auto chunk = [&](int64_t c0, int cn) {
    const int nfull = cn / STEP;
    const int last = nfull > 0 ? (nfull - 1) * STEP : 0;
    doublex2 A[UN][MG][2], B[UN][MG][2];
    auto load = [&](doublex2(&dst)[UN][MG][2], int t) {
      const int i0 = min(t * STEP, last);
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int g = 0; g < MG; ++g) ld4(g, c0 + i0 + 4 * u, true, dst[u][g][0], dst[u][g][1]);
    };
    auto compute = [&](const doublex2(&src)[UN][MG][2], int t) {
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const double bv = usd[(t * STEP + 4 * u + kq) * RP + b * 16 + l16];
#pragma unroll
          for (int g = 0; g < MG; ++g) {
            acc[b][g][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(src[u][g][0].x, bv, acc[b][g][0], 0, 0, 0);
            acc[b][g][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(src[u][g][0].y, bv, acc[b][g][1], 0, 0, 0);
            acc[b][g][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(src[u][g][1].x, bv, acc[b][g][2], 0, 0, 0);
            acc[b][g][3] = __builtin_amdgcn_mfma_f64_16x16x4f64(src[u][g][1].y, bv, acc[b][g][3], 0, 0, 0);
          }
        }
    };
    if (nfull > 0) {
      load(A, 0);
      for (int t = 0; t < nfull; t += 2) {
        load(B, t + 1);
        compute(A, t);
        load(A, t + 2);
        if (t + 1 < nfull) compute(B, t + 1);
      }
    }
    for (int i = nfull * STEP; i < cn; i += 4) {  // chunk tail
      const int ii = i + kq;
      const bool ok = ii < cn;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const double bv = ok ? usd[ii * RP + b * 16 + l16] : 0.0;
#pragma unroll
        for (int g = 0; g < MG; ++g) {
          doublex2 x0{0.0, 0.0}, x1{0.0, 0.0};
          if (ok) ld4(g, c0 + i, false, x0, x1);
          acc[b][g][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0.x, bv, acc[b][g][0], 0, 0, 0);
          acc[b][g][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0.y, bv, acc[b][g][1], 0, 0, 0);
          acc[b][g][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1.x, bv, acc[b][g][2], 0, 0, 0);
          acc[b][g][3] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1.y, bv, acc[b][g][3], 0, 0, 0);
        }
      }
    }
  };
  constexpr int KC = (LDS_DOUBLES / RP) / STEP * STEP;
  for (int64_t c0 = kb0; c0 < kb1; c0 += KC) {
    const int cn = int(min<int64_t>(kb1 - c0, KC));
    __syncthreads();
    const double* Uc = U + c0 * RP;
    stage_lds<NWV * 64>(reinterpret_cast<const float*>(Uc), reinterpret_cast<float*>(usd), 2 * cn * RP, tid);
    __syncthreads();
    if (active) chunk(c0, cn);
  }
  if (!active) return;
  double* o = out + int64_t(blockIdx.y) * split_stride;
  // lane (l16, kq) holds rows m0 + j (j = 0..3), m0 = mt + 64 g + 16 v + 4 kq,
  // of column r = 16 b + l16 in acc[b][g][j][v]
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int r = b * 16 + l16;
    if (r >= R) continue;
#pragma unroll
    for (int g = 0; g < MG; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m0 = mt + 64 * g + 16 * v + 4 * kq;
        const int64_t p0 = m0 % P, s0 = m0 / P;
        double* d = o + p0 + r * P + s0 * P * R;
        if (m0 + 4 <= M && p0 + 4 <= P && (reinterpret_cast<uintptr_t>(d) & 15) == 0) {
          *reinterpret_cast<doublex2*>(d) = doublex2{acc[b][g][0][v], acc[b][g][1][v]};
          *reinterpret_cast<doublex2*>(d + 2) = doublex2{acc[b][g][2][v], acc[b][g][3][v]};
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int64_t m = m0 + j;
            if (m < M) o[m % P + r * P + (m / P) * P * R] = acc[b][g][j][v];
          }
        }
      }
  }
}

// ---------------- first contraction of a middle mode with short slabs
// (P % 4 == 0, P % 32 != 0, P <= 64 MG NWV, R <= 16): one workgroup per slab
// s, i.e. per contiguous P x K block X[:, :, s].  Rows of that block are
// 4 P bytes apart, not a multiple of the 128-byte cache line, so row tiles
// of several wavefronts would share lines at their edges (and fetch them
// twice).  Here the workgroup copies KC whole rows of its block at a time
// (one contiguous stretch of memory; NRS stretches in flight, staged in
// registers) into LDS, then each wavefront runs the row-tiled MFMA steps on
// its 64 MG rows of the block from LDS.  U rows come with each stretch.
template <int MG, int NWV, int KC, int NRS, bool NT>
__global__ __launch_bounds__(NWV * 64) void ttm_slab_m(const float* __restrict__ X, const float* __restrict__ U,
                                                       float* __restrict__ out, int64_t P, int64_t K, int64_t S,
                                                       int R) {
  constexpr int NTH = NWV * 64, RP = 16;
  constexpr int LPT = (KC * 64 * MG * NWV / 4 + NTH - 1) / NTH;  // float4 loads per thread per stretch
  extern __shared__ float sm[];
  const int Pi = int(P);
  float* xb0 = sm;                        // [2][KC * P]
  float* ub0 = sm + 2 * KC * Pi;          // [2][KC * RP]
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int l16 = lane % 16, kq = lane / 16;
  const int64_t s = blockIdx.x;
  const float* Xs = X + s * P * K;
  const int nch = int((K + KC - 1) / KC);
  floatx4 acc[MG][4];
#pragma unroll
  for (int g = 0; g < MG; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[g][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  float4 rs[NRS][LPT];
  auto kcount = [&](int c) { return int(min<int64_t>(KC, K - int64_t(c) * KC)); };
  auto load = [&](float4(&r)[LPT], int c) {
    const float* src = Xs + int64_t(c) * KC * P;
    const int n4 = kcount(c) * Pi / 4;
#pragma unroll
    for (int i = 0; i < LPT; ++i) {
      const int e = tid + i * NTH;
      r[i] = e < n4 ? ldx<NT>(src + 4 * e) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto store = [&](const float4(&r)[LPT], int c) {
    float* xb = xb0 + (c & 1) * KC * Pi;
    float* ub = ub0 + (c & 1) * KC * RP;
    const int kc = kcount(c), n4 = kc * Pi / 4;
#pragma unroll
    for (int i = 0; i < LPT; ++i) {
      const int e = tid + i * NTH;
      if (e < n4) *reinterpret_cast<float4*>(xb + 4 * e) = r[i];
    }
    for (int e = tid; e < kc * RP; e += NTH) ub[e] = U[int64_t(c) * KC * RP + e];
  };
  const int prow = w * 64 * MG + 4 * l16;  // first of the lane's four rows in group 0
  auto compute = [&](int c) {
    const float* xb = xb0 + (c & 1) * KC * Pi;
    const float* ub = ub0 + (c & 1) * KC * RP;
    const int kc = kcount(c);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int k = kk + kq;
      const bool ok = k < kc;
      const float bv = ok ? ub[k * RP + l16] : 0.f;
#pragma unroll
      for (int g = 0; g < MG; ++g) {
        const int pr = prow + 64 * g;
        const float4 xv = (ok && pr < Pi) ? *reinterpret_cast<const float4*>(xb + k * Pi + pr)
                                          : make_float4(0.f, 0.f, 0.f, 0.f);
        acc[g][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.x, bv, acc[g][0], 0, 0, 0);
        acc[g][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.y, bv, acc[g][1], 0, 0, 0);
        acc[g][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.z, bv, acc[g][2], 0, 0, 0);
        acc[g][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.w, bv, acc[g][3], 0, 0, 0);
      }
    }
  };
  // register set j holds stretch c with c % NRS == j; at step c the set of
  // stretch c (already in LDS) takes the loads of stretch c + NRS, stretch c
  // is computed from LDS and stretch c + 1 goes to the other LDS buffer
#pragma unroll
  for (int j = 0; j < NRS; ++j)
    if (j < nch) load(rs[j], j);
  store(rs[0], 0);
  __syncthreads();
  for (int c0 = 0; c0 < nch; c0 += NRS) {
#pragma unroll
    for (int j = 0; j < NRS; ++j) {
      const int c = c0 + j;
      if (c < nch) {  // uniform over the workgroup
        if (c + NRS < nch) load(rs[j], c + NRS);
        compute(c);
        if (c + 1 < nch) store(rs[(j + 1) % NRS], c + 1);
        __syncthreads();
      }
    }
  }
  floatx4 acc1[1][MG][4];
#pragma unroll
  for (int g = 0; g < MG; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc1[0][g][j] = acc[g][j];
  // rows of this slab only: past P they would alias the next slab's rows
  store_tiles<1, MG>(acc1, out, s * P + w * 64 * MG, (s + 1) * P, P, R, l16, kq);
}

// ---------------- both leading modes of each slab in one pass (fused)
// out[r1 + R r2 + R^2 s] = sum_{i1, i2} X[i1, i2, s] U1[i1, r1] U2[i2, r2],
// i.e. the contraction of the middle mode of the [P = I_1, K = I_2, S]
// tensor followed by that of the first mode, for P <= 64 MG NWV, one
// workgroup per slab s.  The slab streams through LDS in stretches of KC of
// its K rows (KC P contiguous floats), together with the matching KC rows of
// U2, NRS stretches in flight in registers.  The loads are buffer loads with
// the slab (and U2) as their range: a lane past the stretch reads zeros
// without a memory request, so every load is unconditional and the waits
// before each LDS copy are for the oldest stretch only.  T1 = X(:, :, s) U2
// (P x R) is built in 16-row blocks (block j of 64-row group g holds rows
// 64 (MG slot + g) + 16 j + l16 in its A operand); blocks wholly past P are
// skipped, and the wavefront slot that holds the slab's partial group
// rotates with s so that the shortfall spreads over the SIMDs.  T1 stays in
// registers in the MFMA D layout: lane (l16, kq) holds
// T1(64 (MG slot + g) + 16 j + 4 kq + v, 16 b + l16) in acc[b][g][j][v].
// For fixed (g, j, v) those values are the B operand of a 16 x 16 x 4 MFMA
// whose K index kq runs over four rows of T1, so U1^T T1 needs no data
// movement: the A operand is U1(row, 16 b1 + l16).  Each wavefront sums its
// rows into an R x R partial, the partials are added in LDS in slot order,
// and the slab writes its R x R block.  The P x R x S intermediate never
// leaves the workgroup.
constexpr uint32_t OOB = 0x80000000u;  // a buffer offset past every range used here (< 2 GB)

// LDS strides of the fused slab kernel.  The four K rows that a wavefront
// reads at once (lane groups kq = 0..3) start 16 banks apart, so its 64
// lanes hit 64 distinct banks: X rows at a stride P' >= P with
// P' = 16 (mod 64), U2 rows at 48 floats for two 16-column blocks (16 for
// one).
__host__ __device__ constexpr int slab2_xstride(int P) { return P + ((16 - P) % 64 + 64) % 64; }
__host__ __device__ constexpr int slab2_ustride(int NB) { return NB == 1 ? 16 : 48; }
// Floats of one stretch buffer.  Every load of a stretch is stored (no
// branch around a store, so that no load sinks behind later ones): the
// loads past row KC hold zeros and land in rows KC and up.  The buffer also
// covers the reads of the rows past P of the last 64-row group (masked).
__host__ __device__ constexpr int slab2_xbuf(int P, int MG, int NWV, int KC) {
  const int ps = slab2_xstride(P), nf = 4 * ((KC * MG + 3) / 4) * NWV * 64;  // floats loaded per stretch
  const int a = (nf - 4) / P * ps + P, b = (KC - 1) * ps + 64 * MG * NWV;
  return ((a > b ? a : b) + 3) / 4 * 4;
}
__host__ __device__ constexpr int slab2_ubuf(int NB, int NWV, int KC) {
  const int nu = (KC * 16 * NB + NWV * 64 - 1) / (NWV * 64) * (NWV * 64);  // U2 values loaded per stretch
  return (nu + 16 * NB - 1) / (16 * NB) * slab2_ustride(NB);
}

template <int NB, int MG, int NWV, int KC, int NRS, bool NT>
__global__ __launch_bounds__(NWV * 64) __attribute__((amdgpu_waves_per_eu(NWV >= 8 && NB == 1 ? 4 : 1)))
void ttm_slab2_m(const float* __restrict__ X, const float* __restrict__ U2,
                                                        const float* __restrict__ U1, float* __restrict__ out,
                                                        int64_t P, int64_t K, int64_t S, int R) {
  constexpr int NTH = NWV * 64, RP = 16 * NB, PMAX = 64 * MG * NWV;
  constexpr int LPT = (KC * PMAX / 4 + NTH - 1) / NTH;  // X float4 loads per thread per stretch
  constexpr int UPT = (KC * RP + NTH - 1) / NTH;        // U2 loads per thread per stretch
  constexpr int RPS = slab2_ustride(NB), US = slab2_ubuf(NB, NWV, KC);
  extern __shared__ float sm[];
  const int Pi = int(P), Ki = int(K);
  const int PS = slab2_xstride(Pi), XS = slab2_xbuf(Pi, MG, NWV, KC);
  float* xb0 = sm;           // [2][XS], stretch row k at k PS
  float* ub0 = sm + 2 * XS;  // [2][US], U2 row k at k RPS
  float* red = sm;           // [NWV][RP * RP], after the stream (the stretch buffers are done)
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int l16 = lane % 16, kq = lane / 16;
  const int64_t s = blockIdx.x;
  const int slot = __builtin_amdgcn_readfirstlane(int((w + s) % NWV));  // uniform: skipped blocks branch on scalars
  const int nch = (Ki + KC - 1) / KC;
  const __amdgpu_buffer_rsrc_t rx =
      __builtin_amdgcn_make_buffer_rsrc((void*)(X + s * P * K), short(0), int(P * K * 4), 0x00020000);
  const __amdgpu_buffer_rsrc_t ru =
      __builtin_amdgcn_make_buffer_rsrc((void*)U2, short(0), int(K * RP * 4), 0x00020000);
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  u32x4 xr[NRS][LPT];
  unsigned int ur[NRS][UPT];
  auto load = [&](int q, int c) {  // stretch c into register set q (zeros past the slab)
    const bool in = c < nch;
    const int kc = in ? min(KC, Ki - c * KC) : 0;
    const int n4 = kc * Pi / 4, nu = kc * RP;
    const uint32_t sx = in ? uint32_t(c) * uint32_t(KC * Pi) * 4u : 0u;
    const uint32_t su = in ? uint32_t(c) * uint32_t(KC * RP) * 4u : 0u;
#pragma unroll
    for (int i = 0; i < LPT; ++i) {
      const int e = tid + i * NTH;
      xr[q][i] = __builtin_amdgcn_raw_buffer_load_b128(rx, e < n4 ? uint32_t(e) * 16u : OOB, sx, NT ? 2 : 0);
    }
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      const int e = tid + i * NTH;
      ur[q][i] = __builtin_amdgcn_raw_buffer_load_b32(ru, e < nu ? uint32_t(e) * 4u : OOB, su, 0);
    }
  };
  // LDS place of each of the thread's loads (the same in every stretch);
  // rows kc and up of a stretch receive zeros
  int xo[LPT], uo[UPT];
#pragma unroll
  for (int i = 0; i < LPT; ++i) {
    const int f = 4 * (tid + i * NTH), row = f / Pi;
    xo[i] = row * PS + (f - row * Pi);
  }
#pragma unroll
  for (int i = 0; i < UPT; ++i) {
    const int e = tid + i * NTH;
    uo[i] = (e / RP) * RPS + e % RP;
  }
  auto store = [&](int q, int c) {  // register set q into LDS buffer c & 1
    float* xb = xb0 + (c & 1) * XS;
    float* ub = ub0 + (c & 1) * US;
#pragma unroll
    for (int i = 0; i < LPT; ++i) *reinterpret_cast<u32x4*>(xb + xo[i]) = xr[q][i];
#pragma unroll
    for (int i = 0; i < UPT; ++i) ub[uo[i]] = __builtin_bit_cast(float, ur[q][i]);
  };
  int nblk[MG];  // 16-row blocks of each group that hold rows < P (uniform)
#pragma unroll
  for (int g = 0; g < MG; ++g) {
    const int r0 = 64 * (MG * slot + g);
    nblk[g] = r0 >= Pi ? 0 : min(4, (Pi - r0 + 15) / 16);
  }
  floatx4 acc[NB][MG][4];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int g = 0; g < MG; ++g)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[b][g][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  bool full = true;  // every row of the wavefront's groups is < P (uniform): no masks, no skips
#pragma unroll
  for (int g = 0; g < MG; ++g) full = full && 64 * (MG * slot + g) + 64 <= Pi;
  // FULL: no block to skip, straight-line MFMAs
  auto compute = [&](int c, auto full_tag) {
    constexpr bool FULL = decltype(full_tag)::value;
    const float* xb = xb0 + (c & 1) * XS;
    const float* ub = ub0 + (c & 1) * US;
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int k = kk + kq;  // rows past the stretch hold zeros
      float bv[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) bv[b] = ub[k * RPS + b * 16 + l16];
      float xv[MG][4];  // read for every block (in range of the buffer), used for the live ones
#pragma unroll
      for (int g = 0; g < MG; ++g)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = 64 * (MG * slot + g) + 16 * j + l16;
          const float x = xb[k * PS + row];
          xv[g][j] = (FULL || row < Pi) ? x : 0.f;
        }
#pragma unroll
      for (int g = 0; g < MG; ++g)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (FULL || j < nblk[g]) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
              acc[b][g][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[g][j], bv[b], acc[b][g][j], 0, 0, 0);
          }
    }
  };
  // The loads leave in stretch order (no rescheduling across the barriers).
  // The two forms of the loop differ only in the block guards.
  auto stream = [&](auto full_tag) {
    __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
    for (int q = 0; q < NRS; ++q) {
      load(q, q);
      __builtin_amdgcn_sched_barrier(0);
    }
    store(0, 0);
    __syncthreads();
    for (int c0 = 0; c0 < nch; c0 += NRS) {
#pragma unroll
      for (int q = 0; q < NRS; ++q) {
        const int c = c0 + q;
        load(q, c + NRS);  // register set q held stretch c, already in LDS
        __builtin_amdgcn_sched_barrier(0);
        if (c < nch) compute(c, full_tag);
        store((q + 1) % NRS, c + 1);
        __syncthreads();
      }
    }
  };
  if (full)
    stream(std::true_type{});
  else
    stream(std::false_type{});
  // U1^T T1 over this wavefront's rows (rows past P hold zeros in T1)
  floatx4 acc2[NB][NB];
#pragma unroll
  for (int b1 = 0; b1 < NB; ++b1)
#pragma unroll
    for (int b2 = 0; b2 < NB; ++b2) acc2[b1][b2] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int g = 0; g < MG; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < nblk[g]) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 64 * (MG * slot + g) + 16 * j + 4 * kq + v;
#pragma unroll
          for (int b1 = 0; b1 < NB; ++b1) {
            const float a = row < Pi ? U1[int64_t(row) * RP + b1 * 16 + l16] : 0.f;
#pragma unroll
            for (int b2 = 0; b2 < NB; ++b2)
              acc2[b1][b2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, acc[b2][g][j][v], acc2[b1][b2], 0, 0, 0);
          }
        }
      }
  // lane (l16, kq) holds partial(16 b1 + 4 kq + vv, 16 b2 + l16)
  float* rw = red + slot * RP * RP;
#pragma unroll
  for (int b1 = 0; b1 < NB; ++b1)
#pragma unroll
    for (int b2 = 0; b2 < NB; ++b2)
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) rw[(b1 * 16 + 4 * kq + vv) + RP * (b2 * 16 + l16)] = acc2[b1][b2][vv];
  __syncthreads();
  float* o = out + s * R * R;
  for (int e = tid; e < R * R; e += NTH) {
    const int r1 = e % R, r2 = e / R;
    float t = 0.f;
#pragma unroll
    for (int ww = 0; ww < NWV; ++ww) t += red[ww * RP * RP + r1 + RP * r2];
    o[e] = t;
  }
}

// LDS bytes of ttm_slab2_m: two stretch buffers of X and U2, or the
// wavefront partials, whichever is larger.
template <int NB, int MG, int NWV, int KC>
size_t slab2_lds(int P) {
  const int st = 2 * slab2_xbuf(P, MG, NWV, KC) + 2 * slab2_ubuf(NB, NWV, KC), rd = NWV * 16 * NB * 16 * NB;
  return size_t(st > rd ? st : rd) * sizeof(float);
}

// ---------------- P == 1: out[r + R*s] = sum_i U[i, r] X[i + K*s]
// U4 holds four consecutive i interleaved per r, so one float4 read feeds the
// four MFMAs of a step.  K % 4 == 0.
template <int NB, int UN, int NWV, bool STREAM>
__global__ __launch_bounds__(NWV * 64) void ttm_mfma_k(const float* __restrict__ X,
                                                       const float* __restrict__ U4,
                                                       float* __restrict__ out, int64_t K,
                                                       int64_t S, int R, int RP, int64_t kchunk,
                                                       int64_t split_stride) {
  extern __shared__ float4 us4[];
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int64_t st = (int64_t(blockIdx.x) * NWV + w) * 16;
  const bool active = st < S;
  const int64_t kb0 = int64_t(blockIdx.y) * kchunk;
  const int64_t kb1 = min(K, kb0 + kchunk);
  const int l16 = lane % 16, kq = lane / 16;
  int64_t scl = st + l16;
  scl = scl < S ? scl : S - 1;
  const float* col = X + scl * K + 4 * kq;
  floatx4 acc[NB][4];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[b][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  constexpr int STEP = 16 * UN;
  const int KC = (LDS_FLOATS / RP) / STEP * STEP;  // rows of U per chunk
  const float4* U4v = reinterpret_cast<const float4*>(U4);
  for (int64_t c0 = kb0; c0 < kb1; c0 += KC) {
    const int64_t c1 = min(kb1, c0 + KC);
    __syncthreads();
    for (int e = tid; e < (KC / 4) * RP; e += NWV * 64) {
      const int64_t q = c0 / 4 + e / RP;
      us4[e] = q * 4 < c1 ? U4v[q * RP + e % RP] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();
    if (!active) continue;
    const int64_t nfull = (c1 - c0) / STEP;
    const int64_t last = nfull > 0 ? c0 + (nfull - 1) * STEP : c0;
    float4 A[UN], B[UN];
    auto load = [&](float4(&dst)[UN], int64_t t) {
      const int64_t i0 = min(c0 + t * STEP, last);
#pragma unroll
      for (int u = 0; u < UN; ++u) dst[u] = *reinterpret_cast<const float4*>(col + i0 + 16 * u);
    };
    auto compute = [&](const float4(&src)[UN], int64_t t) {
#pragma unroll
      for (int u = 0; u < UN; ++u)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const float4 av = us4[((t * STEP + 16 * u) / 4 + kq) * RP + b * 16 + l16];
          acc[b][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, src[u].x, acc[b][0], 0, 0, 0);
          acc[b][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, src[u].y, acc[b][1], 0, 0, 0);
          acc[b][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, src[u].z, acc[b][2], 0, 0, 0);
          acc[b][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, src[u].w, acc[b][3], 0, 0, 0);
        }
    };
    if (nfull > 0) {
      load(A, 0);
      for (int64_t t = 0; t < nfull; t += 2) {
        load(B, t + 1);
        compute(A, t);
        load(A, t + 2);
        if (t + 1 < nfull) compute(B, t + 1);
      }
    }
    for (int64_t i = c0 + nfull * STEP; i < c1; i += 16) {  // chunk tail
      const int64_t ii = i + 4 * kq;
      const bool ok = ii < c1;  // c1 % 4 == 0: four valid together
      const float4 xv = ok ? *reinterpret_cast<const float4*>(col + i) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const float4 av = ok ? us4[((i - c0) / 4 + kq) * RP + b * 16 + l16] : make_float4(0.f, 0.f, 0.f, 0.f);
        acc[b][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, xv.x, acc[b][0], 0, 0, 0);
        acc[b][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, xv.y, acc[b][1], 0, 0, 0);
        acc[b][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, xv.z, acc[b][2], 0, 0, 0);
        acc[b][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, xv.w, acc[b][3], 0, 0, 0);
      }
    }
  }
  // The four MFMAs of one step cover different i, so their sums add up.
  const int64_t s = st + l16;
  if (!active || s >= S) return;
  float* o = out + int64_t(blockIdx.y) * split_stride;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const floatx4 t = acc[b][0] + acc[b][1] + acc[b][2] + acc[b][3];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = b * 16 + 4 * kq + v;
      if (r < R) o[r + int64_t(R) * s] = t[v];
    }
  }
}

// ------------------------------------------------------------ bfloat16 forms
// Operands are split as x = x_hi + x_lo with x_hi = bf16(x), x_lo = bf16(x -
// x_hi) (hardware round-to-nearest-even).  SPLIT = true keeps three products
// x_hi q_hi + x_hi q_lo + x_lo q_hi (the lo*lo term is dropped); SPLIT =
// false keeps x_hi q_hi only.  Products run on v_mfma_f32_16x16x16_bf16 with
// FP32 accumulation.  U's hi and lo halves are staged in LDS as quads of four
// consecutive K rows per column (8 bytes each), the operand layout of that
// instruction (lane l supplies k = 4*(l/16) .. +3).
typedef short shortx4 __attribute__((ext_vector_type(4)));

__device__ inline void split4(float a, float b, float c, float d, shortx4& hi, shortx4& lo) {
  const __bf16 ha = (__bf16)a, hb = (__bf16)b, hc = (__bf16)c, hd = (__bf16)d;
  const __bf16 la = (__bf16)(a - (float)ha), lb = (__bf16)(b - (float)hb);
  const __bf16 lc = (__bf16)(c - (float)hc), ld = (__bf16)(d - (float)hd);
  hi = shortx4{__builtin_bit_cast(short, ha), __builtin_bit_cast(short, hb), __builtin_bit_cast(short, hc),
               __builtin_bit_cast(short, hd)};
  lo = shortx4{__builtin_bit_cast(short, la), __builtin_bit_cast(short, lb), __builtin_bit_cast(short, lc),
               __builtin_bit_cast(short, ld)};
}

template <bool SPLIT>
__device__ inline floatx4 mfma_bf16(const shortx4& ah, const shortx4& al, const shortx4& bh,
                                    const shortx4& bl, floatx4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
  if (SPLIT) {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
  }
  return c;
}

// Stage rows [c0, c1) of U (row-major K x RP FP32) as bf16 quads:
// hiq/loq[q*RP + col] = 4 rows c0+4q..c0+4q+3 of column col.
__device__ inline void stage_u_bf16(const float* __restrict__ U, int64_t c0, int64_t c1, int KC, int RP,
                                    shortx4* hiq, shortx4* loq, int tid, int nthreads) {
  for (int e = tid; e < (KC / 4) * RP; e += nthreads) {
    const int64_t q = e / RP;
    const int col = e % RP;
    float v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t i = c0 + 4 * q + t;
      v[t] = i < c1 ? U[i * RP + col] : 0.f;
    }
    split4(v[0], v[1], v[2], v[3], hiq[e], loq[e]);
  }
}

// ---------------- P % 4 == 0 (rows on the MFMA M dimension)
// A step covers 16 K rows: lane kq loads rows 4kq..4kq+3 (four float4 of four
// consecutive p each); component j of the four loads forms the A operand of
// the MFMA for rows m = mt + 4*l16 + j.
template <bool SPLIT, int NB, int MG, int NWV, bool STREAM, bool NT = false>
__global__ __launch_bounds__(NWV * 64) void ttm_bf16_m(const float* __restrict__ X,
                                                       const float* __restrict__ U,
                                                       float* __restrict__ out, int64_t P,
                                                       int64_t K, int64_t S, int R, int RP,
                                                       int64_t kchunk, int64_t split_stride) {
  extern __shared__ shortx4 ubq[];
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int64_t M = P * S;
  const int64_t mt = (int64_t(blockIdx.x) * NWV + w) * 64 * MG;
  const bool active = mt < M;
  const int64_t kb0 = int64_t(blockIdx.y) * kchunk;
  const int64_t kb1 = min(K, kb0 + kchunk);
  const int l16 = lane % 16, kq = lane / 16;
  const float* base[MG];
#pragma unroll
  for (int g = 0; g < MG; ++g) {
    int64_t mrow = mt + 64 * g + 4 * l16;
    mrow = mrow < M ? mrow : M - 4;
    const int64_t p = mrow % P, s = mrow / P;
    base[g] = X + p + s * P * K + int64_t(4 * kq) * P;
  }
  floatx4 acc[NB][MG][4];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int g = 0; g < MG; ++g)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[b][g][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  constexpr int STEP = 16;
  const int KC = (LDS_FLOATS / RP) / STEP * STEP;  // hi + lo quads fill the budget
  shortx4* hiq = ubq;
  shortx4* loq = ubq + (KC / 4) * RP;
  for (int64_t c0 = kb0; c0 < kb1; c0 += KC) {
    const int64_t c1 = min(kb1, c0 + KC);
    __syncthreads();
    stage_u_bf16(U, c0, c1, KC, RP, hiq, loq, tid, NWV * 64);
    __syncthreads();
    if (!active) continue;
    const int64_t nfull = (c1 - c0) / STEP;
    const int64_t last = nfull > 0 ? c0 + (nfull - 1) * STEP : c0;
    float4 A[4][MG], B[4][MG];
    auto load = [&](float4(&dst)[4][MG], int64_t t) {
      const int64_t i0 = min(c0 + t * STEP, last);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int g = 0; g < MG; ++g) dst[r][g] = ldx<NT>(base[g] + (i0 + r) * P);
    };
    auto compute = [&](const float4(&src)[4][MG], int64_t qoff) {
#pragma unroll
      for (int g = 0; g < MG; ++g) {
        shortx4 ah[4], al[4];
        split4(src[0][g].x, src[1][g].x, src[2][g].x, src[3][g].x, ah[0], al[0]);
        split4(src[0][g].y, src[1][g].y, src[2][g].y, src[3][g].y, ah[1], al[1]);
        split4(src[0][g].z, src[1][g].z, src[2][g].z, src[3][g].z, ah[2], al[2]);
        split4(src[0][g].w, src[1][g].w, src[2][g].w, src[3][g].w, ah[3], al[3]);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const shortx4 bh = hiq[(qoff + kq) * RP + b * 16 + l16];
          const shortx4 bl = loq[(qoff + kq) * RP + b * 16 + l16];
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[b][g][j] = mfma_bf16<SPLIT>(ah[j], al[j], bh, bl, acc[b][g][j]);
        }
      }
    };
    if (nfull > 0) {
      load(A, 0);
      for (int64_t t = 0; t < nfull; t += 2) {
        load(B, t + 1);
        compute(A, t * (STEP / 4));
        load(A, t + 2);
        if (t + 1 < nfull) compute(B, (t + 1) * (STEP / 4));
      }
    }
    const int64_t ct = c0 + nfull * STEP;  // chunk tail (< 16 rows), masked by row
    if (ct < c1) {
      float4 T[4][MG];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool ok = ct + 4 * kq + r < c1;
#pragma unroll
        for (int g = 0; g < MG; ++g)
          T[r][g] = ok ? *reinterpret_cast<const float4*>(base[g] + (ct + r) * P) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
      compute(T, nfull * (STEP / 4));
    }
  }
  if (!active) return;
  store_tiles<NB, MG>(acc, out + int64_t(blockIdx.y) * split_stride, mt, M, P, R, l16, kq);
}

// ---------------- short slabs, bfloat16 forms: the whole-slab scheme of
// ttm_slab_m with 16-row stretches (one bf16 MFMA step each), split in
// registers as they leave LDS; slabs of at most SLAB_PMAX rows (static LDS).
constexpr int SLAB_PMAX = 1008;
template <bool SPLIT, int MG, int NWV, int NRS, bool NT>
__global__ __launch_bounds__(NWV * 64) void ttm_slab_bf16(const float* __restrict__ X, const float* __restrict__ U,
                                                          float* __restrict__ out, int64_t P, int64_t K, int64_t S,
                                                          int R) {
  constexpr int KC = 16, NTH = NWV * 64, RP = 16;
  constexpr int LPT = (KC * SLAB_PMAX / 4 + NTH - 1) / NTH;
  __shared__ float xs[2][KC * SLAB_PMAX];
  __shared__ shortx4 uh[2][(KC / 4) * RP], ul[2][(KC / 4) * RP];
  const int Pi = int(P);
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int l16 = lane % 16, kq = lane / 16;
  const int64_t s = blockIdx.x;
  const float* Xs = X + s * P * K;
  const int nch = int((K + KC - 1) / KC);
  floatx4 acc[1][MG][4];
#pragma unroll
  for (int g = 0; g < MG; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[0][g][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  float4 rs[NRS][LPT];
  auto kcount = [&](int c) { return int(min<int64_t>(KC, K - int64_t(c) * KC)); };
  auto load = [&](float4(&r)[LPT], int c) {
    const float* src = Xs + int64_t(c) * KC * P;
    const int n4 = kcount(c) * Pi / 4;
#pragma unroll
    for (int i = 0; i < LPT; ++i) {
      const int e = tid + i * NTH;
      r[i] = e < n4 ? ldx<NT>(src + 4 * e) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto store = [&](const float4(&r)[LPT], int c) {
    float* xb = xs[c & 1];
    const int kc = kcount(c), n4 = kc * Pi / 4;
#pragma unroll
    for (int i = 0; i < LPT; ++i) {
      const int e = tid + i * NTH;
      if (e < n4) *reinterpret_cast<float4*>(xb + 4 * e) = r[i];
    }
    stage_u_bf16(U, int64_t(c) * KC, int64_t(c) * KC + kc, KC, RP, uh[c & 1], ul[c & 1], tid, NTH);
  };
  const int prow = w * 64 * MG + 4 * l16;
  auto compute = [&](int c) {
    const float* xb = xs[c & 1];
    const int kc = kcount(c);
    const shortx4 bh = uh[c & 1][kq * RP + l16], bl = ul[c & 1][kq * RP + l16];
#pragma unroll
    for (int g = 0; g < MG; ++g) {
      const int pr = prow + 64 * g;
      float4 v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = 4 * kq + r;
        v[r] = (k < kc && pr < Pi) ? *reinterpret_cast<const float4*>(xb + k * Pi + pr)
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
      }
      shortx4 ah[4], al[4];
      split4(v[0].x, v[1].x, v[2].x, v[3].x, ah[0], al[0]);
      split4(v[0].y, v[1].y, v[2].y, v[3].y, ah[1], al[1]);
      split4(v[0].z, v[1].z, v[2].z, v[3].z, ah[2], al[2]);
      split4(v[0].w, v[1].w, v[2].w, v[3].w, ah[3], al[3]);
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[0][g][j] = mfma_bf16<SPLIT>(ah[j], al[j], bh, bl, acc[0][g][j]);
    }
  };
#pragma unroll
  for (int j = 0; j < NRS; ++j)
    if (j < nch) load(rs[j], j);
  store(rs[0], 0);
  __syncthreads();
  for (int c0 = 0; c0 < nch; c0 += NRS) {
#pragma unroll
    for (int j = 0; j < NRS; ++j) {
      const int c = c0 + j;
      if (c < nch) {  // uniform over the workgroup
        if (c + NRS < nch) load(rs[j], c + NRS);
        compute(c);
        if (c + 1 < nch) store(rs[(j + 1) % NRS], c + 1);
        __syncthreads();
      }
    }
  }
  store_tiles<1, MG>(acc, out, s * P + w * 64 * MG, (s + 1) * P, P, R, l16, kq);
}

// ---------------- P == 1 (columns on the MFMA N dimension)
// The float4 a lane loads from one column (rows 4kq..4kq+3 of the step) is the
// B operand of one MFMA; U quads are the A operand.  K % 4 == 0.
template <bool SPLIT, int NB, int UN, int NWV, bool STREAM>
__global__ __launch_bounds__(NWV * 64) void ttm_bf16_k(const float* __restrict__ X,
                                                       const float* __restrict__ U,
                                                       float* __restrict__ out, int64_t K,
                                                       int64_t S, int R, int RP, int64_t kchunk,
                                                       int64_t split_stride) {
  extern __shared__ shortx4 ubq[];
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  const int64_t st = (int64_t(blockIdx.x) * NWV + w) * 16;
  const bool active = st < S;
  const int64_t kb0 = int64_t(blockIdx.y) * kchunk;
  const int64_t kb1 = min(K, kb0 + kchunk);
  const int l16 = lane % 16, kq = lane / 16;
  int64_t scl = st + l16;
  scl = scl < S ? scl : S - 1;
  const float* col = X + scl * K + 4 * kq;
  floatx4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
  constexpr int STEP = 16 * UN;
  const int KC = (LDS_FLOATS / RP) / STEP * STEP;
  shortx4* hiq = ubq;
  shortx4* loq = ubq + (KC / 4) * RP;
  for (int64_t c0 = kb0; c0 < kb1; c0 += KC) {
    const int64_t c1 = min(kb1, c0 + KC);
    __syncthreads();
    stage_u_bf16(U, c0, c1, KC, RP, hiq, loq, tid, NWV * 64);
    __syncthreads();
    if (!active) continue;
    const int64_t nfull = (c1 - c0) / STEP;
    const int64_t last = nfull > 0 ? c0 + (nfull - 1) * STEP : c0;
    float4 A[UN], B[UN];
    auto load = [&](float4(&dst)[UN], int64_t t) {
      const int64_t i0 = min(c0 + t * STEP, last);
#pragma unroll
      for (int u = 0; u < UN; ++u) dst[u] = *reinterpret_cast<const float4*>(col + i0 + 16 * u);
    };
    auto compute = [&](const float4(&src)[UN], int64_t t) {
#pragma unroll
      for (int u = 0; u < UN; ++u) {
        shortx4 xh, xl;
        split4(src[u].x, src[u].y, src[u].z, src[u].w, xh, xl);
        const int64_t q = (t * STEP + 16 * u) / 4 + kq;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const shortx4 ah = hiq[q * RP + b * 16 + l16];
          const shortx4 al = loq[q * RP + b * 16 + l16];
          acc[b] = mfma_bf16<SPLIT>(ah, al, xh, xl, acc[b]);
        }
      }
    };
    if (nfull > 0) {
      load(A, 0);
      for (int64_t t = 0; t < nfull; t += 2) {
        load(B, t + 1);
        compute(A, t);
        load(A, t + 2);
        if (t + 1 < nfull) compute(B, t + 1);
      }
    }
    for (int64_t i = c0 + nfull * STEP; i < c1; i += 16) {  // chunk tail, c1 % 4 == 0
      const bool ok = i + 4 * kq < c1;
      const float4 xv = ok ? *reinterpret_cast<const float4*>(col + i) : make_float4(0.f, 0.f, 0.f, 0.f);
      shortx4 xh, xl;
      split4(xv.x, xv.y, xv.z, xv.w, xh, xl);
      const int64_t q = (i - c0) / 4 + kq;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const shortx4 ah = ok ? hiq[q * RP + b * 16 + l16] : shortx4{0, 0, 0, 0};
        const shortx4 al = ok ? loq[q * RP + b * 16 + l16] : shortx4{0, 0, 0, 0};
        acc[b] = mfma_bf16<SPLIT>(ah, al, xh, xl, acc[b]);
      }
    }
  }
  const int64_t s = st + l16;
  if (!active || s >= S) return;
  float* o = out + int64_t(blockIdx.y) * split_stride;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = b * 16 + 4 * kq + v;
      if (r < R) o[r + int64_t(R) * s] = acc[b][v];
    }
}

// ------------------------------------------------------------ VALU fallback
// MODE: 0 plain products in TA, 1 bfloat16 operands, 2 split bfloat16 (three
// products), the latter two in FP32 arithmetic.
template <int MODE>
__device__ inline float bf16_round(float v) { return (float)(__bf16)v; }

template <class TX, class TA, int RM, int MODE>
__global__ __launch_bounds__(256) void ttm_valu(const TX* __restrict__ X, const TA* __restrict__ U,
                                                TA* __restrict__ out, int64_t P, int64_t K,
                                                int64_t S, int R, int RP, int64_t kchunk,
                                                int64_t split_stride) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t M = P * S;
  if (m >= M) return;
  const int64_t k0 = int64_t(blockIdx.y) * kchunk;
  const int64_t k1 = min(K, k0 + kchunk);
  const int64_t p = m % P, s = m / P;
  const TX* base = X + p + s * P * K;
  TA acc[RM];
#pragma unroll
  for (int r = 0; r < RM; ++r) acc[r] = TA(0);
  for (int64_t i = k0; i < k1; ++i) {
    const TA x = TA(base[i * P]);
    const TA* u = U + i * RP;
    if (MODE == 0) {
#pragma unroll
      for (int r = 0; r < RM; ++r) acc[r] += x * u[r];
    } else {
      const float xh = bf16_round<MODE>(float(x));
      const float xl = bf16_round<MODE>(float(x) - xh);
#pragma unroll
      for (int r = 0; r < RM; ++r) {
        const float uh = bf16_round<MODE>(float(u[r]));
        const float ul = bf16_round<MODE>(float(u[r]) - uh);
        float v = xh * uh;
        if (MODE == 2) v += xh * ul + xl * uh;
        acc[r] += TA(v);
      }
    }
  }
  TA* o = out + int64_t(blockIdx.y) * split_stride;
#pragma unroll
  for (int r = 0; r < RM; ++r)
    if (r < R) o[p + r * P + s * P * R] = acc[r];
}

// ------------------------------------------------------------ reductions
template <class T>
__global__ void sum_splits(const T* __restrict__ part, int splits, int64_t count, T* __restrict__ dst) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= count) return;
  T acc = part[e];
  for (int t = 1; t < splits; ++t) acc += part[int64_t(t) * count + e];
  dst[e] = acc;
}

// Y_(n)[i + In*(p + Pn*s)] = T[p + Pn*i + Pn*In*s]: for each s the In x Pn
// block (p contiguous) is transposed, 32 x 32 tiles through LDS so that both
// the reads (along p) and the writes (along i) are coalesced.  One
// workgroup of 256 threads per tile, the tiles of all s in one flat grid.
constexpr int UT = 32;
template <class T>
__global__ __launch_bounds__(256) void unfold_copy(const T* __restrict__ src, int64_t Pn, int64_t In, int64_t Sn,
                                                   T* __restrict__ dst) {
  __shared__ T tile[UT][UT + 1];
  const int64_t tp = (Pn + UT - 1) / UT, ti = (In + UT - 1) / UT;
  const int64_t b = blockIdx.x;
  const int64_t s = b / (tp * ti), r = b % (tp * ti);
  const int64_t i0 = (r / tp) * UT, p0 = (r % tp) * UT;
  const int tx = threadIdx.x % UT, ty = threadIdx.x / UT;  // 32 x 8
  const T* S = src + Pn * In * s;
  T* Dd = dst + Pn * In * s;
#pragma unroll
  for (int k = 0; k < UT; k += 8) {
    const int64_t i = i0 + ty + k, p = p0 + tx;
    if (i < In && p < Pn) tile[ty + k][tx] = S[p + Pn * i];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < UT; k += 8) {
    const int64_t p = p0 + ty + k, i = i0 + tx;
    if (i < In && p < Pn) Dd[i + In * p] = tile[tx][ty + k];
  }
}

// ------------------------------------------------------------ planning
enum Kind { K_MFMA_M, K_MFMA_K, K_VALU };
// Smallest P that the FP64 row kernel takes when P is not a multiple of four.
// P = 1 (contracting the fastest mode) is taken too: a tile's 64 rows are one
// contiguous block of 64 K values that the K steps walk through, so its lines
// are reused from the caches (75^5 FP64, rank 4: 10.5 -> 8.7 ms per sweep
// against the vector-ALU kernel).
constexpr int64_t GENP_MIN_P = 1;

struct Step {
  int k;          // mode contracted
  int64_t P, K, S;
  Kind kind;
  int splits;
  int64_t kchunk;
  int64_t out_count;  // P * R * S
  int mg;             // row-tiled matrix-core kernels: 64 * mg rows per wavefront
};

struct Plan {
  int nsteps;
  Step st[CPQR_MAX_MODES];
  int64_t buf_count[2];  // elements of the two ping-pong buffers
  int64_t part_count;    // elements of the split-K partial buffer
  int64_t final_count;   // elements of Y
  int acc_bytes;
  int RP;
};

bool uses_mfma(int prec) { return prec != CPQR_PREC_F64; }
// every precision has the row-tiled kernels (FP64: ttm_mfma_m_f64); only
// the P = 1 form is FP32 / bfloat16 only
bool row_tiled(int) { return true; }
int valu_mode(int prec) { return prec == CPQR_PREC_BF16 ? 1 : (prec == CPQR_PREC_BF16X2 ? 2 : 0); }

// Contract the modes in cmask (bit k = mode k) of a tensor of sizes I.
Plan make_plan(int N, const int64_t* I, unsigned cmask, int R, int prec, bool x_aligned = true) {
  Plan pl{};
  pl.RP = ((R + 15) / 16) * 16;
  pl.acc_bytes = prec == CPQR_PREC_F64 ? 8 : 4;
  int order[CPQR_MAX_MODES];
  int no = 0;
  for (int k = 0; k < N; ++k)
    if (cmask >> k & 1u) order[no++] = k;
  std::stable_sort(order, order + no, [&](int a, int b) { return I[a] > I[b]; });
  // The first contraction streams the whole tensor.  Contracting the fastest
  // mode first (P = 1) has the least favourable access pattern for the matrix
  // cores, so when another contracted mode is at least half as large and its
  // index stride is small (rows at most 256 KB apart), start with the largest
  // such mode; the flop count of the first contraction is the same and the
  // later ones change by a factor of at most two.
  if (row_tiled(prec) && no > 1 && order[0] == 0) {
    for (int t = 1; t < no; ++t) {
      int64_t stride = 1;  // elements between consecutive indices of that mode
      for (int m = 0; m < order[t]; ++m) stride *= I[m];
      // large strides walk the tensor page by page: keep those for later
      // (FP64 also takes strides that are not multiples of four: its row
      // kernel has a form that loads rows one by one)
      const bool stride_ok = stride % 4 == 0 || (prec == CPQR_PREC_F64 && stride >= GENP_MIN_P);
      if (2 * I[order[t]] >= I[0] && stride_ok && stride <= 65536) {
        const int k = order[t];
        for (int u = t; u > 0; --u) order[u] = order[u - 1];
        order[0] = k;
        break;
      }
    }
  }
  int64_t D[CPQR_MAX_MODES];
  for (int k = 0; k < N; ++k) D[k] = I[k];
  pl.nsteps = no;
  for (int t = 0; t < no; ++t) {
    Step s{};
    s.k = order[t];
    s.P = 1;
    for (int m = 0; m < s.k; ++m) s.P *= D[m];
    s.K = D[s.k];
    s.S = 1;
    for (int m = s.k + 1; m < N; ++m) s.S *= D[m];
    s.out_count = s.P * R * s.S;
    int64_t units;  // independent work units without splitting K
    // float4 loads of the tensor need 16-byte alignment (carved buffers have it)
    const bool vec_ok = t > 0 || x_aligned;
    const bool genp = prec == CPQR_PREC_F64 && s.P % 4 != 0 && s.P >= GENP_MIN_P;
    if (row_tiled(prec) && ((vec_ok && s.P % 4 == 0) || genp)) {
      s.kind = K_MFMA_M;
      // wide row tiles; a step whose rows leave the GPU under-filled takes
      // 64-row tiles before it splits K (small operands: no streaming hints)
      // (two 16-column blocks, R > 16, halve the tile: at 4 x 64 rows the
      // FP32 kernel needs 202 VGPRs and one workgroup per CU)
      // (rows loaded one by one keep four more addresses per row group:
      // one group, so that two workgroups still fit on a CU)
      s.mg = genp ? 1 : (prec == CPQR_PREC_F32 ? 4 : 2) / (R > 16 ? 2 : 1);
      units = ceil_div(s.P * s.S, 64 * s.mg);
      if (units < MIN_WAVES) {
        s.mg = 1;
        units = ceil_div(s.P * s.S, 64);
      }
    } else if (uses_mfma(prec) && vec_ok && s.P == 1 && s.K % 4 == 0) {
      s.kind = K_MFMA_K;
      units = ceil_div(s.S, 16);
    } else {
      s.kind = K_VALU;
      units = ceil_div(s.P * s.S, 64);
    }
    // Split K only when the rows alone leave the GPU under-filled.
    const int64_t quantum = 16;
    int64_t splits = 1;
    // (K splits write P R S partial sums each; at most K / (4 R) of them keeps
    // that traffic under a quarter of the input's)
    if (units < MIN_WAVES)
      splits = std::min<int64_t>({ceil_div(TARGET_WAVES, units), std::max<int64_t>(1, s.K / quantum),
                                  std::max<int64_t>(1, s.K / (4 * R))});
    splits = std::max<int64_t>(1, std::min<int64_t>(splits, 64));
    s.kchunk = ceil_div(ceil_div(s.K, splits), quantum) * quantum;
    s.splits = int(ceil_div(s.K, s.kchunk));
    if (s.splits > 1) pl.part_count = std::max(pl.part_count, s.out_count * s.splits);
    D[s.k] = R;
    pl.st[t] = s;
    pl.buf_count[t % 2] = std::max(pl.buf_count[t % 2], s.out_count);
  }
  pl.final_count = 1;
  for (int k = 0; k < N; ++k) pl.final_count *= D[k];
  return pl;
}

unsigned all_but(int N, int n) { return ((1u << N) - 1u) & ~(1u << n); }

struct Bufs {
  void* U[CPQR_MAX_MODES];
  void* buf[2];
  void* part;
};

size_t carve(Carver& cv, const Plan& pl, int N, const int64_t* I, Bufs* b) {
  Bufs tmp{};
  for (int t = 0; t < pl.nsteps; ++t) {
    const int k = pl.st[t].k;
    tmp.U[k] = cv.take<char>(size_t(I[k] + 4) * pl.RP * pl.acc_bytes);
  }
  for (int j = 0; j < 2; ++j) tmp.buf[j] = cv.take<char>(size_t(pl.buf_count[j]) * pl.acc_bytes);
  tmp.part = cv.take<char>(size_t(pl.part_count) * pl.acc_bytes);
  if (b) *b = tmp;
  return cv.bytes();
}

template <class TA, int RM, int MODE>
int launch_valu(const void* src, int src_dtype, const TA* U, TA* dst, const Step& s, int R, int RP,
                hipStream_t st) {
  const dim3 grd(unsigned(ceil_div(s.P * s.S, 256)), unsigned(s.splits));
  if (src_dtype == CPQR_F64)
    hipLaunchKernelGGL((ttm_valu<double, TA, RM, MODE>), grd, dim3(256), 0, st,
                       static_cast<const double*>(src), U, dst, s.P, s.K, s.S, R, RP, s.kchunk,
                       s.out_count);
  else
    hipLaunchKernelGGL((ttm_valu<float, TA, RM, MODE>), grd, dim3(256), 0, st,
                       static_cast<const float*>(src), U, dst, s.P, s.K, s.S, R, RP, s.kchunk,
                       s.out_count);
  return check_launch("ttm_valu");
}

template <class TA, int MODE>
int launch_valu_r(const void* src, int src_dtype, const TA* U, TA* dst, const Step& s, int R,
                  int RP, hipStream_t st) {
  switch (round_rank(R)) {
    case 8: return launch_valu<TA, 8, MODE>(src, src_dtype, U, dst, s, R, RP, st);
    case 16: return launch_valu<TA, 16, MODE>(src, src_dtype, U, dst, s, R, RP, st);
    default: return launch_valu<TA, 32, MODE>(src, src_dtype, U, dst, s, R, RP, st);
  }
}

int launch_valu_f32(int prec, const void* src, int src_dtype, const float* U, float* dst, const Step& s,
                    int R, int RP, hipStream_t st) {
  switch (valu_mode(prec)) {
    case 1: return launch_valu_r<float, 1>(src, src_dtype, U, dst, s, R, RP, st);
    case 2: return launch_valu_r<float, 2>(src, src_dtype, U, dst, s, R, RP, st);
    default: return launch_valu_r<float, 0>(src, src_dtype, U, dst, s, R, RP, st);
  }
}

template <bool SPLIT, bool STREAM>
int launch_bf16_t(const float* src, const float* U, float* dst, const Step& s, int R, int RP, hipStream_t st,
                  const KernelEvents& ke) {
  const int NB = RP / 16;
  constexpr int NWV = 8;
  const size_t lds = LDS_FLOATS * sizeof(float);
  if (s.kind == K_MFMA_M) {
    const dim3 grd(unsigned(ceil_div(ceil_div(s.P * s.S, 64 * s.mg), NWV)), unsigned(s.splits));
    if (s.mg == 1) {
      // 64-row tiles: small operands, or two 16-column blocks streaming X
      const bool nt1 = STREAM && s.P % 32 == 0;
      if (NB == 1)
        launch_ev(ke, ttm_bf16_m<SPLIT, 1, 1, NWV, false>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                  s.P, s.K, s.S, R, RP, s.kchunk, s.out_count);
      else if (nt1)
        launch_ev(ke, ttm_bf16_m<SPLIT, 2, 1, NWV, STREAM, true>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                  s.P, s.K, s.S, R, RP, s.kchunk, s.out_count);
      else
        launch_ev(ke, ttm_bf16_m<SPLIT, 2, 1, NWV, STREAM>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                  s.P, s.K, s.S, R, RP, s.kchunk, s.out_count);
      return check_launch("ttm_bf16_m");
    }
    if (s.mg != 2 || NB != 1) return fail(CPQR_ERR_UNSUPPORTED, "ttm_bf16_m: unsupported row tile");
    // short slabs whose rows are not line multiples apart: whole-slab workgroups
    if (STREAM && NB == 1 && s.splits == 1 && s.P % 32 != 0 && s.P <= SLAB_PMAX && s.S >= 256) {
      const bool snt = (16 * s.P) % 32 == 0 && (s.P * s.K) % 32 == 0;  // stretches start on line boundaries
      if (snt)
        launch_ev(ke, ttm_slab_bf16<SPLIT, 2, 8, 2, true>, dim3(unsigned(s.S)), dim3(8 * 64), 0, st, src, U, dst,
                  s.P, s.K, s.S, R);
      else
        launch_ev(ke, ttm_slab_bf16<SPLIT, 2, 8, 2, false>, dim3(unsigned(s.S)), dim3(8 * 64), 0, st, src, U, dst,
                  s.P, s.K, s.S, R);
      return check_launch("ttm_slab_bf16");
    }
    const bool nt = STREAM && s.P % 32 == 0;  // see ldx
    if (nt)
      launch_ev(ke, ttm_bf16_m<SPLIT, 1, 2, NWV, STREAM, true>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                s.P, s.K, s.S, R, RP, s.kchunk, s.out_count);
    else
      launch_ev(ke, ttm_bf16_m<SPLIT, 1, 2, NWV, STREAM>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                s.P, s.K, s.S, R, RP, s.kchunk, s.out_count);
    return check_launch("ttm_bf16_m");
  }
  constexpr int UN = 2;
  const dim3 grd(unsigned(ceil_div(ceil_div(s.S, 16), NWV)), unsigned(s.splits));
  if (NB == 1)
    hipLaunchKernelGGL((ttm_bf16_k<SPLIT, 1, UN, NWV, STREAM>), grd, dim3(NWV * 64), lds, st, src, U, dst, s.K,
                       s.S, R, RP, s.kchunk, s.out_count);
  else
    hipLaunchKernelGGL((ttm_bf16_k<SPLIT, 2, UN, NWV, STREAM>), grd, dim3(NWV * 64), lds, st, src, U, dst, s.K,
                       s.S, R, RP, s.kchunk, s.out_count);
  return check_launch("ttm_bf16_k");
}

template <bool STREAM>
int launch_mfma_t(const float* src, const float* U, float* dst, const Step& s, int R, int RP,
                  hipStream_t st, const KernelEvents& ke) {
  const int NB = RP / 16;
  constexpr int NWV = 8;
  const size_t lds = LDS_FLOATS * sizeof(float);
  if (s.kind == K_MFMA_M) {
    constexpr int UN = 2, MG = 4;
    // an input well past the last-level cache (256 MB) streams like the
    // tensor itself: non-temporal row tiles (e.g. the 1 GB mode-3 result at
    // 200^4 rank 32 that the next contraction reads once)
    const bool cold = s.P * s.K * s.S * int64_t(sizeof(float)) > (int64_t(256) << 20);
    const dim3 grd(unsigned(ceil_div(ceil_div(s.P * s.S, 64 * s.mg), NWV)), unsigned(s.splits));
    const bool one = s.kchunk <= (LDS_FLOATS / RP) / (4 * UN) * (4 * UN);  // K range fits in LDS
    if (s.mg == 1) {
      if (NB == 1 && one)
        launch_ev(ke, ttm_mfma_m<1, UN, 1, NWV, false, true>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                  s.P, s.K, s.S, R, s.kchunk, s.out_count);
      else if (NB == 1)
        launch_ev(ke, ttm_mfma_m<1, UN, 1, NWV, false, false>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                  s.P, s.K, s.S, R, s.kchunk, s.out_count);
      else if (one)
        launch_ev(ke, ttm_mfma_m<2, UN, 1, NWV, false, true>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                  s.P, s.K, s.S, R, s.kchunk, s.out_count);
      else
        launch_ev(ke, ttm_mfma_m<2, UN, 1, NWV, false, false>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                  s.P, s.K, s.S, R, s.kchunk, s.out_count);
      return check_launch("ttm_mfma_m");
    }
    if (s.mg == 2 && NB == 2) {  // two 16-column blocks: 2 x 64-row tiles
      const bool nt2 = (STREAM || cold) && s.P % 32 == 0;
      if (one && nt2)
        launch_ev(ke, ttm_mfma_m<2, UN, 2, NWV, STREAM, true, true>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                  s.P, s.K, s.S, R, s.kchunk, s.out_count);
      else if (one)
        launch_ev(ke, ttm_mfma_m<2, UN, 2, NWV, STREAM, true>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                  s.P, s.K, s.S, R, s.kchunk, s.out_count);
      else
        launch_ev(ke, ttm_mfma_m<2, UN, 2, NWV, STREAM, false>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                  s.P, s.K, s.S, R, s.kchunk, s.out_count);
      return check_launch("ttm_mfma_m");
    }
    if (s.mg != MG || NB != 1) return fail(CPQR_ERR_UNSUPPORTED, "ttm_mfma_m: unsupported row tile");
    // short slabs whose rows are not line multiples apart: whole-slab workgroups
    constexpr int SKC = 8, SNWV = 8, SMG = 2, SNRS = 3;
    const size_t slab_lds = size_t(2) * SKC * (s.P + 16) * sizeof(float);
    if (STREAM && NB == 1 && s.splits == 1 && s.P % 32 != 0 && s.P <= 64 * SMG * SNWV && slab_lds <= lds &&
        s.S >= 256) {
      const bool snt = (SKC * s.P) % 32 == 0 && (s.P * s.K) % 32 == 0;  // stretches start on line boundaries
      if (snt)
        launch_ev(ke, ttm_slab_m<SMG, SNWV, SKC, SNRS, true>, dim3(unsigned(s.S)), dim3(SNWV * 64), slab_lds, st,
                  src, U, dst, s.P, s.K, s.S, R);
      else
        launch_ev(ke, ttm_slab_m<SMG, SNWV, SKC, SNRS, false>, dim3(unsigned(s.S)), dim3(SNWV * 64), slab_lds, st,
                  src, U, dst, s.P, s.K, s.S, R);
      return check_launch("ttm_slab_m");
    }
    const bool nt = (STREAM || cold) && s.P % 32 == 0;  // see ldx
    if (one && nt)
      launch_ev(ke, ttm_mfma_m<1, UN, MG, NWV, STREAM, true, true>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                s.P, s.K, s.S, R, s.kchunk, s.out_count);
    else if (one)
      launch_ev(ke, ttm_mfma_m<1, UN, MG, NWV, STREAM, true>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                s.P, s.K, s.S, R, s.kchunk, s.out_count);
    else
      launch_ev(ke, ttm_mfma_m<1, UN, MG, NWV, STREAM, false>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                s.P, s.K, s.S, R, s.kchunk, s.out_count);
    return check_launch("ttm_mfma_m");
  }
  constexpr int UN = 4;
  const dim3 grd(unsigned(ceil_div(ceil_div(s.S, 16), NWV)), unsigned(s.splits));
  if (NB == 1)
    hipLaunchKernelGGL((ttm_mfma_k<1, UN, NWV, STREAM>), grd, dim3(NWV * 64), lds, st, src, U, dst, s.K, s.S,
                       R, RP, s.kchunk, s.out_count);
  else
    hipLaunchKernelGGL((ttm_mfma_k<2, UN, NWV, STREAM>), grd, dim3(NWV * 64), lds, st, src, U, dst, s.K, s.S,
                       R, RP, s.kchunk, s.out_count);
  return check_launch("ttm_mfma_k");
}

// The fused leading-pair contraction applies to an FP32 first contraction of
// mode 2 over short slabs (P = I_1 <= 1024, P % 4 == 0, many slabs, no K
// split) directly followed by mode 1.
bool fused_pair(const Plan& pl, int prec, bool streams_tensor, bool x_aligned) {
  if (prec != CPQR_PREC_F32 || !streams_tensor || !x_aligned || pl.nsteps < 2) return false;
  const Step& a = pl.st[0];
  const Step& b = pl.st[1];
  // The slab and U_2 are the ranges of 32-bit buffer loads.
  return a.k == 1 && b.k == 0 && a.kind == K_MFMA_M && a.splits == 1 && a.P % 4 == 0 && a.P <= 1024 &&
         a.S >= 256 && a.P * a.K * 4 < (int64_t(1) << 31) && a.K * 32 * 4 < (int64_t(1) << 31);
}

// Slab stretch depth (rows of the slab staged per step) and stretches in
// flight for slabs of at most 256 rows; compile-time tuning parameters.
#ifndef CPQR_SLAB2_SMALL_KC
#define CPQR_SLAB2_SMALL_KC 8
#endif
#ifndef CPQR_SLAB2_SMALL_NRS
#define CPQR_SLAB2_SMALL_NRS 3
#endif

int launch_slab2(const float* X, const float* U2, const float* U1, float* dst, const Step& a, int R, int RP,
                 hipStream_t st, const KernelEvents& ke) {
  const int NB = RP / 16;
  const dim3 grd(unsigned(a.S));
  if (a.P <= 256) {
    constexpr int MG = 1, NWV = 4, KC = CPQR_SLAB2_SMALL_KC, NRS = CPQR_SLAB2_SMALL_NRS;
    const bool nt = (KC * a.P) % 32 == 0 && (a.P * a.K) % 32 == 0;  // stretches start on line boundaries
    const size_t lds = NB == 1 ? slab2_lds<1, MG, NWV, KC>(int(a.P)) : slab2_lds<2, MG, NWV, KC>(int(a.P));
    if (NB == 1 && nt)
      launch_ev(ke, ttm_slab2_m<1, MG, NWV, KC, NRS, true>, grd, dim3(NWV * 64), lds, st, X, U2, U1, dst, a.P, a.K,
                a.S, R);
    else if (NB == 1)
      launch_ev(ke, ttm_slab2_m<1, MG, NWV, KC, NRS, false>, grd, dim3(NWV * 64), lds, st, X, U2, U1, dst, a.P,
                a.K, a.S, R);
    else if (nt)
      launch_ev(ke, ttm_slab2_m<2, MG, NWV, KC, NRS, true>, grd, dim3(NWV * 64), lds, st, X, U2, U1, dst, a.P, a.K,
                a.S, R);
    else
      launch_ev(ke, ttm_slab2_m<2, MG, NWV, KC, NRS, false>, grd, dim3(NWV * 64), lds, st, X, U2, U1, dst, a.P,
                a.K, a.S, R);
  } else {
    constexpr int MG = 2, NWV = 8, KC = 8, NRS = 2;
    const bool nt = (KC * a.P) % 32 == 0 && (a.P * a.K) % 32 == 0;
    const size_t lds = NB == 1 ? slab2_lds<1, MG, NWV, KC>(int(a.P)) : slab2_lds<2, MG, NWV, KC>(int(a.P));
    if (NB == 1 && nt)
      launch_ev(ke, ttm_slab2_m<1, MG, NWV, KC, NRS, true>, grd, dim3(NWV * 64), lds, st, X, U2, U1, dst, a.P, a.K,
                a.S, R);
    else if (NB == 1)
      launch_ev(ke, ttm_slab2_m<1, MG, NWV, KC, NRS, false>, grd, dim3(NWV * 64), lds, st, X, U2, U1, dst, a.P,
                a.K, a.S, R);
    else if (nt)
      launch_ev(ke, ttm_slab2_m<2, MG, NWV, KC, NRS, true>, grd, dim3(NWV * 64), lds, st, X, U2, U1, dst, a.P, a.K,
                a.S, R);
    else
      launch_ev(ke, ttm_slab2_m<2, MG, NWV, KC, NRS, false>, grd, dim3(NWV * 64), lds, st, X, U2, U1, dst, a.P,
                a.K, a.S, R);
  }
  return check_launch("ttm_slab2_m");
}

template <bool STREAM, class TX>
int launch_mfma_f64_t(const TX* src, const double* U, double* dst, const Step& s, int R, int RP,
                      hipStream_t st, const KernelEvents& ke) {
  const int NB = RP / 16;
  // one step (four K rows) in flight per buffer: 122 VGPRs, two workgroups per CU
  constexpr int NWV = 8, UN = 1;
  const size_t lds = LDS_DOUBLES * sizeof(double);
  const dim3 grd(unsigned(ceil_div(ceil_div(s.P * s.S, 64 * s.mg), NWV)), unsigned(s.splits));
  const bool nt = STREAM && s.P % 16 == 0;  // rows 128-byte multiples apart: no line shared between tiles
  if (s.P % 4 != 0) {  // rows loaded one by one (a lane's four rows may straddle slabs)
    if (s.mg == 1 && NB == 1)
      launch_ev(ke, ttm_mfma_m_f64<1, UN, 1, NWV, STREAM, false, TX, true>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                s.P, s.K, s.S, R, s.kchunk, s.out_count);
    else if (s.mg == 1)
      launch_ev(ke, ttm_mfma_m_f64<2, UN, 1, NWV, STREAM, false, TX, true>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                s.P, s.K, s.S, R, s.kchunk, s.out_count);
    else if (s.mg == 2 && NB == 1)
      launch_ev(ke, ttm_mfma_m_f64<1, UN, 2, NWV, STREAM, false, TX, true>, grd, dim3(NWV * 64), lds, st, src, U, dst,
                s.P, s.K, s.S, R, s.kchunk, s.out_count);
    else
      return fail(CPQR_ERR_UNSUPPORTED, "ttm_mfma_m_f64: unsupported row tile");
    return check_launch("ttm_mfma_m_f64");
  }
  if (s.mg == 1) {  // 64-row tiles: small operands, or two 16-column blocks
    if (NB == 1)
      launch_ev(ke, ttm_mfma_m_f64<1, UN, 1, NWV, STREAM, false, TX>, grd, dim3(NWV * 64), lds, st, src, U, dst, s.P,
                s.K, s.S, R, s.kchunk, s.out_count);
    else if (nt)
      launch_ev(ke, ttm_mfma_m_f64<2, UN, 1, NWV, STREAM, true, TX>, grd, dim3(NWV * 64), lds, st, src, U, dst, s.P,
                s.K, s.S, R, s.kchunk, s.out_count);
    else
      launch_ev(ke, ttm_mfma_m_f64<2, UN, 1, NWV, STREAM, false, TX>, grd, dim3(NWV * 64), lds, st, src, U, dst, s.P,
                s.K, s.S, R, s.kchunk, s.out_count);
    return check_launch("ttm_mfma_m_f64");
  }
  if (s.mg != 2 || NB != 1) return fail(CPQR_ERR_UNSUPPORTED, "ttm_mfma_m_f64: unsupported row tile");
  if (nt)
    launch_ev(ke, ttm_mfma_m_f64<1, UN, 2, NWV, STREAM, true, TX>, grd, dim3(NWV * 64), lds, st, src, U, dst, s.P, s.K,
              s.S, R, s.kchunk, s.out_count);
  else
    launch_ev(ke, ttm_mfma_m_f64<1, UN, 2, NWV, STREAM, false, TX>, grd, dim3(NWV * 64), lds, st, src, U, dst, s.P, s.K,
              s.S, R, s.kchunk, s.out_count);
  return check_launch("ttm_mfma_m_f64");
}

template <class TX>
int launch_mfma_f64(bool first, const TX* src, const double* U, double* dst, const Step& s, int R, int RP,
                    hipStream_t st, const KernelEvents& ke) {
  return first ? launch_mfma_f64_t<true, TX>(src, U, dst, s, R, RP, st, ke)
               : launch_mfma_f64_t<false, TX>(src, U, dst, s, R, RP, st, ke);
}

int launch_mfma(int prec, bool first, const float* src, const float* U, float* dst, const Step& s, int R,
                int RP, hipStream_t st, const KernelEvents& ke) {
  if (prec == CPQR_PREC_BF16X2)
    return first ? launch_bf16_t<true, true>(src, U, dst, s, R, RP, st, ke)
                 : launch_bf16_t<true, false>(src, U, dst, s, R, RP, st, ke);
  if (prec == CPQR_PREC_BF16)
    return first ? launch_bf16_t<false, true>(src, U, dst, s, R, RP, st, ke)
                 : launch_bf16_t<false, false>(src, U, dst, s, R, RP, st, ke);
  return first ? launch_mfma_t<true>(src, U, dst, s, R, RP, st, ke)
               : launch_mfma_t<false>(src, U, dst, s, R, RP, st, ke);
}

}  // namespace

size_t multittm_general_work(int N, const int64_t* I, unsigned cmask, int R, int prec) {
  Plan pl = make_plan(N, I, cmask, R, prec);
  Carver cv(nullptr);
  return carve(cv, pl, N, I, nullptr);
}

int multittm_general_enqueue(int N, const int64_t* I, int xdtype, const void* X, unsigned cmask, int n_unfold,
                             int R, const double* const* Q, int prec, void* Y, void* work, hipStream_t st,
                             bool streams_tensor, const UCache* uc) {
  PhaseTimer whole(streams_tensor ? PH_MULTITTM : -1, st);
  const bool x_aligned = reinterpret_cast<uintptr_t>(X) % 16 == 0;
  const Plan pl = make_plan(N, I, cmask, R, prec, x_aligned);
  Bufs b;
  Carver cv(work);
  carve(cv, pl, N, I, &b);
  const int RP = pl.RP;
  const bool f64 = prec == CPQR_PREC_F64;
  const bool fused = fused_pair(pl, prec, streams_tensor, x_aligned);

  // operand preparation, skipped for operands the caller already holds
  // except those of the launch that streams the tensor: the short
  // preparation launches ahead of it let work on a second stream (the
  // sweep's Khatri-Rao QR) take compute units before the streaming kernel's
  // thousands of workgroups fill them (200^4 rank 32: without them the QR's
  // first level stretched over the whole 1.5 ms launch and its later levels
  // landed on the critical path, +60..130 us per sweep)
  const void* Uk[CPQR_MAX_MODES];
  for (int k = 0; k < N; ++k) Uk[k] = b.U[k];
  for (int t = 0; t < pl.nsteps; ++t) {
    const Step& s = pl.st[t];
    const int64_t cnt = s.K * RP;
    const dim3 grd(unsigned(ceil_div(cnt, 256)));
    const bool quads = !f64 && s.kind == K_MFMA_K && prec == CPQR_PREC_F32 && !(fused && t == 1);
    const bool streaming = streams_tensor && (t == 0 || (fused && t == 1));
    const float* pre = (uc && !f64 && uc->RP == RP && !streaming) ? (quads ? uc->quads[s.k] : uc->rows[s.k])
                                                                   : nullptr;
    if (pre) {
      Uk[s.k] = pre;
      continue;
    }
    if (f64)
      hipLaunchKernelGGL(prep_u_rows<double>, grd, dim3(256), 0, st, Q[s.k], s.K, s.K, R, RP,
                         static_cast<double*>(b.U[s.k]));
    else if (quads)
      hipLaunchKernelGGL(prep_u_quads, grd, dim3(256), 0, st, Q[s.k], s.K, s.K, R, RP,
                         static_cast<float*>(b.U[s.k]));
    else
      hipLaunchKernelGGL(prep_u_rows<float>, grd, dim3(256), 0, st, Q[s.k], s.K, s.K, R, RP,
                         static_cast<float*>(b.U[s.k]));
    CPQR_TRY(check_launch("prep_u"));
  }

  // the natural layout of the result is Y itself unless a later unfolding is asked for
  const bool direct = n_unfold <= 0;
  const void* cur = X;
  int cur_dtype = xdtype;
  int t0 = 0;
  if (fused) {  // steps 0 and 1 in one pass over X: the result of step 1
    void* dst = (pl.nsteps == 2 && direct) ? Y : b.buf[1];
    PhaseTimer ph_first(PH_TTM_FIRST, st);
    const KernelEvents ke = kernel_events(PH_TTM_STREAM_M, st);
    CPQR_TRY(launch_slab2(static_cast<const float*>(X), static_cast<const float*>(Uk[pl.st[0].k]),
                          static_cast<const float*>(Uk[pl.st[1].k]), static_cast<float*>(dst), pl.st[0], R, RP,
                          st, ke));
    kernel_events_done(ke);
    cur = dst;
    cur_dtype = CPQR_F32;
    t0 = 2;
  }
  for (int t = t0; t < pl.nsteps; ++t) {
    const Step& s = pl.st[t];
    const bool last = t + 1 == pl.nsteps;
    void* dst = (last && direct) ? Y : b.buf[t % 2];
    void* kout = s.splits > 1 ? b.part : dst;
    {
      const bool first = t == 0 && streams_tensor;
      PhaseTimer ph_first(first ? PH_TTM_FIRST : -1, st);
      if (f64 && s.kind == K_MFMA_M && (cur_dtype == CPQR_F64 || !first)) {
        // FP64 matrix cores; an FP32 operand that is not the streamed tensor
        // (the unfolded Y of the structured Q_0 application) is widened as it loads
        const KernelEvents ke = kernel_events(first ? PH_TTM_STREAM_M : -1, st);
        if (cur_dtype == CPQR_F64)
          CPQR_TRY(launch_mfma_f64(first, static_cast<const double*>(cur), static_cast<const double*>(Uk[s.k]),
                                   static_cast<double*>(kout), s, R, RP, st, ke));
        else
          CPQR_TRY(launch_mfma_f64(first, static_cast<const float*>(cur), static_cast<const double*>(Uk[s.k]),
                                   static_cast<double*>(kout), s, R, RP, st, ke));
        kernel_events_done(ke);
      } else if (f64) {
        CPQR_TRY((launch_valu_r<double, 0>(cur, cur_dtype, static_cast<const double*>(Uk[s.k]),
                                           static_cast<double*>(kout), s, R, RP, st)));
      } else if (s.kind == K_VALU) {
        CPQR_TRY(launch_valu_f32(prec, cur, cur_dtype, static_cast<const float*>(Uk[s.k]),
                                 static_cast<float*>(kout), s, R, RP, st));
      } else {
        const KernelEvents ke = kernel_events(first && s.kind == K_MFMA_M ? PH_TTM_STREAM_M : -1, st);
        CPQR_TRY(launch_mfma(prec, first, static_cast<const float*>(cur), static_cast<const float*>(Uk[s.k]),
                             static_cast<float*>(kout), s, R, RP, st, ke));
        kernel_events_done(ke);
      }
      if (s.splits > 1) {
        const dim3 grd(unsigned(ceil_div(s.out_count, 256)));
        if (f64)
          hipLaunchKernelGGL(sum_splits<double>, grd, dim3(256), 0, st,
                             static_cast<const double*>(b.part), s.splits, s.out_count,
                             static_cast<double*>(dst));
        else
          hipLaunchKernelGGL(sum_splits<float>, grd, dim3(256), 0, st,
                             static_cast<const float*>(b.part), s.splits, s.out_count,
                             static_cast<float*>(dst));
        CPQR_TRY(check_launch("sum_splits"));
      }
    }
    cur = dst;
    cur_dtype = f64 ? CPQR_F64 : CPQR_F32;
  }
  if (pl.nsteps == 0 && xdtype != (f64 ? CPQR_F64 : CPQR_F32))
    return fail(CPQR_ERR_UNSUPPORTED, "multittm: nothing to contract and the output type differs from the input");
  if (!direct || pl.nsteps == 0) {
    // Y_(n): result dims D (contracted modes have size R), unfolded along n
    int64_t D[CPQR_MAX_MODES];
    for (int k = 0; k < N; ++k) D[k] = (cmask >> k & 1u) ? R : I[k];
    const int n = n_unfold < 0 ? 0 : n_unfold;
    int64_t Pn = 1, Sn = 1;
    for (int m = 0; m < n; ++m) Pn *= D[m];
    for (int m = n + 1; m < N; ++m) Sn *= D[m];
    const int64_t tiles = ceil_div(Pn, UT) * ceil_div(D[n], UT) * Sn;
    const dim3 grd(static_cast<unsigned>(tiles));
    if (cur_dtype == CPQR_F64)
      hipLaunchKernelGGL(unfold_copy<double>, grd, dim3(256), 0, st, static_cast<const double*>(cur),
                         Pn, D[n], Sn, static_cast<double*>(Y));
    else
      hipLaunchKernelGGL(unfold_copy<float>, grd, dim3(256), 0, st, static_cast<const float*>(cur),
                         Pn, D[n], Sn, static_cast<float*>(Y));
    CPQR_TRY(check_launch("unfold_copy"));
  }
  return CPQR_OK;
}

size_t multittm_work(int N, const int64_t* I, int n, int R, int prec) {
  return multittm_general_work(N, I, all_but(N, n), R, prec);
}

int multittm_enqueue(int N, const int64_t* I, int xdtype, const void* X, int n, int R,
                     const double* const* Q, int prec, void* Y, void* work, hipStream_t st, const UCache* uc) {
  return multittm_general_enqueue(N, I, xdtype, X, all_but(N, n), n, R, Q, prec, Y, work, st, true, uc);
}

}  // namespace cpqr
