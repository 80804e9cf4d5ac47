// Learned initialization: tensor sketch, three-layer MLP (forward and
// backward), Kruskal-form loss gradient and Adam, for gfx950.
//
// Every contraction runs through one bfloat16 MFMA GEMM kernel
// (v_mfma_f32_16x16x16bf16_1k, FP32 accumulation):
//   C[m * ldc + n] = sum_k A(m, k) B(n, k)
// where each operand is either k-contiguous (A(m, k) = A[m * lda + k]) or
// m/n-contiguous (A(m, k) = A[k * lda + m]); tiles of 64 x 64 x 32 are staged
// through LDS in the MFMA operand order, and split-K writes per-split
// partial products that a reduction kernel sums in a fixed order (with the
// bias, ReLU, ReLU-derivative mask and bfloat16 conversion fused there).
// Weights and activations are bfloat16, gradients and optimizer state FP32.

#include <algorithm>
#include <cmath>

#include "common.h"

namespace cpqr {
namespace {

typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int GM = 64, GN = 64, GK = 32;  // GEMM tile
constexpr int GT = 256;                  // threads per GEMM workgroup
constexpr int LDK = GK + 8;              // LDS row pitch (bfloat16 elements)

__device__ inline unsigned short f2bf(float x) { return __builtin_bit_cast(unsigned short, (__bf16)x); }
__device__ inline float bf2f(unsigned short h) { return __uint_as_float(unsigned(h) << 16); }

// Load this thread's 8 elements of a 64 x 32 operand tile (rows r0.., k0..).
template <bool KC>
__device__ inline uint4 load_tile(const unsigned short* __restrict__ P, int64_t ld, int64_t r0, int64_t k0, int tid) {
  if (KC) {  // row = tid / 4, k = (tid % 4) * 8 .. +7
    const unsigned short* src = P + (r0 + tid / 4) * ld + k0 + (tid % 4) * 8;
    return *reinterpret_cast<const uint4*>(src);
  } else {   // k = tid / 8, rows (tid % 8) * 8 .. +7
    const unsigned short* src = P + (k0 + tid / 8) * ld + r0 + (tid % 8) * 8;
    return *reinterpret_cast<const uint4*>(src);
  }
}

template <bool KC>
__device__ inline void store_tile(unsigned short (*S)[LDK], uint4 v, int tid) {
  if (KC) {
    *reinterpret_cast<uint4*>(&S[tid / 4][(tid % 4) * 8]) = v;
  } else {
    const int k = tid / 8, r = (tid % 8) * 8;
    const unsigned short* e = reinterpret_cast<const unsigned short*>(&v);
#pragma unroll
    for (int j = 0; j < 8; ++j) S[r + j][k] = e[j];
  }
}

// grid: (N / 64, M / 64, batch * splits).  Split s of batch b covers
// k in [s * kchunk, min(K, (s + 1) * kchunk)) and writes C + (b * splits + s) * cstride.
template <bool AK, bool BK>
__global__ __launch_bounds__(GT) void gemm_bf16_kernel(const unsigned short* __restrict__ A, int64_t lda,
                                                       int64_t astride, const unsigned short* __restrict__ B,
                                                       int64_t ldb, int64_t bstride, float* __restrict__ C,
                                                       int64_t ldc, int64_t cstride, int64_t K, int64_t kchunk,
                                                       int splits) {
  __shared__ __attribute__((aligned(16))) unsigned short As[GM][LDK];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[GN][LDK];
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
  const int l16 = lane % 16, kq = lane / 16;
  const int wm = w / 2, wn = w % 2;
  const int bz = blockIdx.z / splits, sz = blockIdx.z % splits;
  const int64_t m0 = int64_t(blockIdx.y) * GM, n0 = int64_t(blockIdx.x) * GN;
  const int64_t kb = int64_t(sz) * kchunk, ke = std::min<int64_t>(K, kb + kchunk);
  A += bz * astride;
  B += bz * bstride;
  C += (int64_t(bz) * splits + sz) * cstride;
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  uint4 ra = uint4{0, 0, 0, 0}, rb = uint4{0, 0, 0, 0};
  if (kb < ke) {
    ra = load_tile<AK>(A, lda, m0, kb, tid);
    rb = load_tile<BK>(B, ldb, n0, kb, tid);
  }
  for (int64_t k0 = kb; k0 < ke; k0 += GK) {
    store_tile<AK>(As, ra, tid);
    store_tile<BK>(Bs, rb, tid);
    __syncthreads();
    if (k0 + GK < ke) {  // prefetch the next tile while this one is used
      ra = load_tile<AK>(A, lda, m0, k0 + GK, tid);
      rb = load_tile<BK>(B, ldb, n0, k0 + GK, tid);
    }
#pragma unroll
    for (int ks = 0; ks < GK; ks += 16) {
      shortx4 af[2], bfr[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        af[t] = *reinterpret_cast<const shortx4*>(&As[wm * 32 + t * 16 + l16][ks + 4 * kq]);
        bfr[t] = *reinterpret_cast<const shortx4*>(&Bs[wn * 32 + t * 16 + l16][ks + 4 * kq]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // lane holds rows 4 kq + v, column l16 of each 16 x 16 tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + wm * 32 + i * 16 + 4 * kq + v;
        const int64_t n = n0 + wn * 32 + j * 16 + l16;
        C[m * ldc + n] = acc[i][j][v];
      }
}

// out = sum over splits (+ bias[n]); act: 0 none, 1 ReLU; mask (bfloat16,
// nullable): multiply by (mask > 0).  Writes FP32 and/or bfloat16.
__global__ void reduce_epilogue_kernel(const float* __restrict__ part, int splits, int64_t M, int64_t N,
                                       const float* __restrict__ bias, int act,
                                       const unsigned short* __restrict__ mask, float* __restrict__ out,
                                       unsigned short* __restrict__ outb) {
  const int64_t total = M * N;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total; e += int64_t(gridDim.x) * blockDim.x) {
    float v = 0.f;
    for (int s = 0; s < splits; ++s) v += part[int64_t(s) * total + e];
    if (bias) v += bias[e % N];
    if (act == 1) v = v > 0.f ? v : 0.f;
    if (mask && !(bf2f(mask[e]) > 0.f)) v = 0.f;
    if (out) out[e] = v;
    if (outb) outb[e] = f2bf(v);
  }
}

// db[n] = sum_m D[m * N + n] (fixed order over m)
__global__ void colsum_kernel(const float* __restrict__ D, int64_t M, int64_t N, float* __restrict__ db) {
  const int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int64_t m = 0; m < M; ++m) s += D[m * N + n];
  db[n] = s;
}

__global__ void to_bf16_kernel(const float* __restrict__ x, int64_t n, const double* __restrict__ norm2,
                               unsigned short* __restrict__ y) {
  const float scale = norm2 ? float(sqrt(double(n) / (*norm2 > 0.0 ? *norm2 : 1.0))) : 1.f;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    y[e] = f2bf(x[e] * scale);
}

// Adam with bias correction (Kingma and Ba); optional bfloat16 copy of w.
__global__ void adam_kernel(int64_t n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, unsigned short* __restrict__ wb, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
    const float ge = g[e];
    const float me = b1 * m[e] + (1.f - b1) * ge;
    const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float we = w[e] - lr * (me / c1) / (sqrtf(ve / c2) + eps);
    w[e] = we;
    if (wb) wb[e] = f2bf(we);
  }
}

// Kruskal-form loss and gradient, one workgroup per sample (I_k <= 256,
// R, Rt <= 16).  y and target hold three column-major factor matrices one
// after the other (ranks R and Rt).  Gram matrices are accumulated in FP64.
constexpr int KT = 256, KRB = 16;

// kind 0: distance ||[[Ahat]] - [[A]]||^2 / ||[[A]]||^2;
// kind 1: cosine 1 - <[[Ahat]],[[A]]>^2 / (||[[Ahat]]||^2 ||[[A]]||^2).
__global__ __launch_bounds__(KT) void kruskal_grad_kernel(int64_t I0, int64_t I1, int64_t I2, int R, int Rt,
                                                          const float* __restrict__ y, int64_t ldy,
                                                          const float* __restrict__ tgt, int64_t ldt, int kind,
                                                          float* __restrict__ loss, float* __restrict__ dy,
                                                          unsigned short* __restrict__ dyb, float scale) {
  __shared__ float fa[256][KRB + 1];   // Ahat_k rows
  __shared__ float fb[256][KRB + 1];   // A_k rows
  __shared__ double gaa[3][KRB][KRB];  // Ahat^T Ahat
  __shared__ double gab[3][KRB][KRB];  // Ahat^T A
  __shared__ double gbb[3][KRB][KRB];  // A^T A
  __shared__ double red[KT];
  __shared__ double sc[3];             // ||[[A]]||^2, <[[Ahat]],[[A]]>, ||[[Ahat]]||^2
  const int tid = threadIdx.x;
  const int64_t b = blockIdx.x;
  const int64_t I[3] = {I0, I1, I2};
  const float* yb = y + b * ldy;
  const float* tb = tgt + b * ldt;
  int64_t oy = 0, ot = 0;
  for (int k = 0; k < 3; ++k) {
    for (int e = tid; e < I[k] * KRB; e += KT) {
      const int i = e / KRB, r = e % KRB;
      fa[i][r] = r < R ? yb[oy + i + r * I[k]] : 0.f;
      fb[i][r] = r < Rt ? tb[ot + i + r * I[k]] : 0.f;
    }
    __syncthreads();
    for (int e = tid; e < 3 * KRB * KRB; e += KT) {
      const int which = e / (KRB * KRB), r = (e / KRB) % KRB, s = e % KRB;
      double acc = 0.0;
      for (int64_t i = 0; i < I[k]; ++i) {
        const double u = which == 2 ? fb[i][r] : fa[i][r];
        const double v = which == 0 ? fa[i][s] : fb[i][s];
        acc += u * v;
      }
      if (which == 0) gaa[k][r][s] = acc;
      else if (which == 1) gab[k][r][s] = acc;
      else gbb[k][r][s] = acc;
    }
    __syncthreads();
    oy += I[k] * R;
    ot += I[k] * Rt;
  }
  // the three scalars
  for (int q = 0; q < 3; ++q) {
    double part = 0.0;
    for (int e = tid; e < KRB * KRB; e += KT) {
      const int r = e / KRB, s = e % KRB;
      double p = 1.0;
      for (int k = 0; k < 3; ++k) p *= q == 0 ? gbb[k][r][s] : (q == 1 ? gab[k][r][s] : gaa[k][r][s]);
      part += p;
    }
    red[tid] = part;
    __syncthreads();
    for (int h = KT / 2; h > 0; h /= 2) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) sc[q] = red[0];
    __syncthreads();
  }
  // dL/dAhat_k = ca Ahat_k G_k + cb A_k H_k^T
  const double t = sc[0], c = sc[1], a = sc[2];
  double ca, cb, lv;
  if (kind == 0) {
    lv = (a - 2.0 * c + t) / t;
    ca = 2.0 / t;
    cb = -2.0 / t;
  } else if (a > 0.0) {
    lv = 1.0 - c * c / (a * t);
    ca = 2.0 * c * c / (a * a * t);
    cb = -2.0 * c / (a * t);
  } else {  // zero prediction: the cosine is undefined; no gradient
    lv = 1.0;
    ca = cb = 0.0;
  }
  if (tid == 0 && loss) loss[b] = float(lv);
  oy = 0;
  ot = 0;
  for (int k = 0; k < 3; ++k) {
    for (int e = tid; e < I[k] * KRB; e += KT) {
      const int i = e / KRB, r = e % KRB;
      fa[i][r] = r < R ? yb[oy + i + r * I[k]] : 0.f;
      fb[i][r] = r < Rt ? tb[ot + i + r * I[k]] : 0.f;
    }
    __syncthreads();
    if (tid < I[k]) {
      for (int r = 0; r < R; ++r) {
        double ga = 0.0, gb = 0.0;
        for (int s = 0; s < R; ++s) {
          double G = 1.0;
          for (int j = 0; j < 3; ++j)
            if (j != k) G *= gaa[j][s][r];
          ga += fa[tid][s] * G;
        }
        for (int s = 0; s < Rt; ++s) {
          double H = 1.0;
          for (int j = 0; j < 3; ++j)
            if (j != k) H *= gab[j][r][s];
          gb += fb[tid][s] * H;
        }
        const float v = float(ca * ga + cb * gb) * scale;
        const int64_t idx = b * ldy + oy + tid + r * I[k];
        dy[idx] = v;
        if (dyb) dyb[idx] = f2bf(v);
      }
    }
    __syncthreads();
    oy += I[k] * R;
    ot += I[k] * Rt;
  }
}

int grid_for(int64_t n) { return int(std::min<int64_t>(ceil_div(n, 256), 8192)); }

}  // namespace

// C (+ batch/splits) = sum_k A(m, k) B(n, k); see the kernel comment.
int gemm_bf16_enqueue(bool ak, bool bk, int64_t M, int64_t N, int64_t K, const unsigned short* A, int64_t lda,
                      int64_t astride, const unsigned short* B, int64_t ldb, int64_t bstride, float* C, int64_t ldc,
                      int64_t cstride, int batch, int splits, hipStream_t s) {
  if (M % GM || N % GN || K % GK || lda % 8 || ldb % 8 || splits < 1 || batch < 1)
    return fail(CPQR_ERR_SHAPE, "gemm_bf16: M, N multiples of 64, K of 32, leading dimensions of 8");
  if ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) % 16)
    return fail(CPQR_ERR_ARG, "gemm_bf16: operands must be 16-byte aligned");
  const int64_t kchunk = ceil_div(ceil_div(K, splits), GK) * GK;
  const dim3 grd(unsigned(N / GN), unsigned(M / GM), unsigned(batch * splits));
  if (ak && bk)
    hipLaunchKernelGGL((gemm_bf16_kernel<true, true>), grd, dim3(GT), 0, s, A, lda, astride, B, ldb, bstride, C, ldc,
                       cstride, K, kchunk, splits);
  else if (ak)
    hipLaunchKernelGGL((gemm_bf16_kernel<true, false>), grd, dim3(GT), 0, s, A, lda, astride, B, ldb, bstride, C, ldc,
                       cstride, K, kchunk, splits);
  else if (bk)
    hipLaunchKernelGGL((gemm_bf16_kernel<false, true>), grd, dim3(GT), 0, s, A, lda, astride, B, ldb, bstride, C, ldc,
                       cstride, K, kchunk, splits);
  else
    hipLaunchKernelGGL((gemm_bf16_kernel<false, false>), grd, dim3(GT), 0, s, A, lda, astride, B, ldb, bstride, C,
                       ldc, cstride, K, kchunk, splits);
  return check_launch("gemm_bf16_kernel");
}

int reduce_epilogue_enqueue(const float* part, int splits, int64_t M, int64_t N, const float* bias, int act,
                            const unsigned short* mask, float* out, unsigned short* outb, hipStream_t s) {
  hipLaunchKernelGGL(reduce_epilogue_kernel, dim3(grid_for(M * N)), dim3(256), 0, s, part, splits, M, N, bias, act,
                     mask, out, outb);
  return check_launch("reduce_epilogue_kernel");
}

int to_bf16_enqueue(const float* x, int64_t n, const double* norm2, unsigned short* y, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, norm2, y);
  return check_launch("to_bf16_kernel");
}

}  // namespace cpqr

using namespace cpqr;

namespace {

// split count for a GEMM with few output tiles and a long K
int splits_for(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = (M / GM) * (N / GN);
  int s = 1;
  while (tiles * s < 1024 && K / (int64_t(s) * 2) >= 1024) s *= 2;
  return s;
}

// C = A B^T-style product followed by the epilogue.  Without an epilogue and
// with a single split the GEMM writes `out` directly; otherwise through
// `part` (size part_need).
bool gemm_direct(int64_t M, int64_t N, int64_t K, const float* bias, int act, const unsigned short* mask,
                 unsigned short* outb) {
  return splits_for(M, N, K) == 1 && !bias && act == 0 && !mask && !outb;
}

size_t part_need(int64_t M, int64_t N, int64_t K, const float* bias, int act, const unsigned short* mask,
                 unsigned short* outb) {
  return gemm_direct(M, N, K, bias, act, mask, outb) ? 0 : size_t(splits_for(M, N, K)) * M * N;
}

int gemm_out(bool ak, bool bk, int64_t M, int64_t N, int64_t K, const unsigned short* A, int64_t lda,
             const unsigned short* B, int64_t ldb, float* part, const float* bias, int act,
             const unsigned short* mask, float* out, unsigned short* outb, hipStream_t s) {
  const int sp = splits_for(M, N, K);
  if (gemm_direct(M, N, K, bias, act, mask, outb))
    return gemm_bf16_enqueue(ak, bk, M, N, K, A, lda, 0, B, ldb, 0, out, N, 0, 1, 1, s);
  CPQR_TRY(gemm_bf16_enqueue(ak, bk, M, N, K, A, lda, 0, B, ldb, 0, part, N, M * N, 1, sp, s));
  return reduce_epilogue_enqueue(part, sp, M, N, bias, act, mask, out, outb, s);
}

int check_mlp(const cpqr_mlp* net, int batch) {
  if (!net) return fail(CPQR_ERR_ARG, "mlp: NULL network");
  if (net->din < 64 || net->din % 64 || net->hidden < 64 || net->hidden % 64 || net->dout < 64 || net->dout % 64)
    return fail(CPQR_ERR_SHAPE, "mlp: layer widths must be positive multiples of 64");
  if (batch < 64 || batch % 64) return fail(CPQR_ERR_SHAPE, "mlp: batch must be a positive multiple of 64");
  for (int l = 0; l < 3; ++l)
    if (!net->W[l] || !net->b[l]) return fail(CPQR_ERR_ARG, "mlp: NULL weight or bias");
  return CPQR_OK;
}

size_t mlp_parts(const cpqr_mlp* net, int batch) {
  const int64_t B = batch, D = net->din, H = net->hidden, O = net->dout;
  const float* nb = reinterpret_cast<const float*>(16);  // any non-null bias
  unsigned short* ob = reinterpret_cast<unsigned short*>(16);
  size_t need = 0;
  need = std::max(need, part_need(B, H, D, nb, 1, nullptr, ob));   // forward layer 1
  need = std::max(need, part_need(B, H, H, nb, 1, nullptr, ob));   // forward layer 2
  need = std::max(need, part_need(B, O, H, nb, 0, nullptr, nullptr));  // forward layer 3
  need = std::max(need, part_need(O, H, B, nullptr, 0, nullptr, nullptr));  // dW3
  need = std::max(need, part_need(B, H, O, nullptr, 0, ob, ob));   // dh2
  need = std::max(need, part_need(H, H, B, nullptr, 0, nullptr, nullptr));  // dW2
  need = std::max(need, part_need(B, H, H, nullptr, 0, ob, ob));   // dh1
  need = std::max(need, part_need(H, D, B, nullptr, 0, nullptr, nullptr));  // dW1
  return need;
}

int colsum_enqueue(const float* D, int64_t M, int64_t N, float* db, hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel, dim3(unsigned(ceil_div(N, 256))), dim3(256), 0, s, D, M, N, db);
  return check_launch("colsum_kernel");
}

size_t sketch_work(const int64_t* I, const int* J) {
  Carver cv(nullptr);
  cv.take<unsigned short>(size_t(I[0] * I[1] * I[2]));  // X in bfloat16
  cv.take<float>(size_t(J[0] * I[1] * I[2]));           // T1
  cv.take<unsigned short>(size_t(J[0] * I[1] * I[2]));
  cv.take<float>(size_t(J[0] * J[1] * I[2]));           // T2
  cv.take<unsigned short>(size_t(J[0] * J[1] * I[2]));
  cv.take<double>(1);
  cv.take<char>(norm2_work(int64_t(J[0]) * J[1] * J[2]));
  return cv.bytes();
}

int check_sketch(const int64_t* I, const int* J) {
  if (!I || !J) return fail(CPQR_ERR_ARG, "sketch3: NULL sizes");
  for (int k = 0; k < 3; ++k)
    if (I[k] < 32 || I[k] % 32 || J[k] < 64 || J[k] % 64)
      return fail(CPQR_ERR_SHAPE, "sketch3: mode sizes must be multiples of 32, sketch sizes multiples of 64");
  if ((I[1] * I[2]) % 64 || I[2] % 64) return fail(CPQR_ERR_SHAPE, "sketch3: I2 I3 and I3 must be multiples of 64");
  return CPQR_OK;
}

}  // namespace

extern "C" {

size_t cpqr_mlp_work(const cpqr_mlp* net, int batch) {
  if (check_mlp(net, batch) != CPQR_OK) return 0;
  Carver cv(nullptr);
  cv.take<float>(std::max<size_t>(mlp_parts(net, batch), 1));
  cv.take<float>(size_t(batch) * net->hidden);           // dh (FP32)
  cv.take<unsigned short>(size_t(batch) * net->hidden);  // dh2 (bfloat16)
  cv.take<unsigned short>(size_t(batch) * net->hidden);  // dh1 (bfloat16)
  return cv.bytes();
}

int cpqr_mlp_forward(const cpqr_mlp* net, int batch, const uint16_t* x, uint16_t* h1, uint16_t* h2, float* y,
                     void* work, size_t work_bytes, void* stream) {
  CPQR_TRY(check_mlp(net, batch));
  if (!x || !h1 || !h2 || !y) return fail(CPQR_ERR_ARG, "mlp_forward: NULL buffer");
  CPQR_TRY(check_work(work, work_bytes, cpqr_mlp_work(net, batch)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver cv(work);
  float* part = cv.take<float>(std::max<size_t>(mlp_parts(net, batch), 1));
  const int64_t B = batch, D = net->din, H = net->hidden, O = net->dout;
  const auto* W1 = reinterpret_cast<const unsigned short*>(net->W[0]);
  const auto* W2 = reinterpret_cast<const unsigned short*>(net->W[1]);
  const auto* W3 = reinterpret_cast<const unsigned short*>(net->W[2]);
  const auto* xb = reinterpret_cast<const unsigned short*>(x);
  auto* h1b = reinterpret_cast<unsigned short*>(h1);
  auto* h2b = reinterpret_cast<unsigned short*>(h2);
  CPQR_TRY(gemm_out(true, true, B, H, D, xb, D, W1, D, part, net->b[0], 1, nullptr, nullptr, h1b, s));
  CPQR_TRY(gemm_out(true, true, B, H, H, h1b, H, W2, H, part, net->b[1], 1, nullptr, nullptr, h2b, s));
  return gemm_out(true, true, B, O, H, h2b, H, W3, H, part, net->b[2], 0, nullptr, y, nullptr, s);
}

int cpqr_mlp_backward(const cpqr_mlp* net, int batch, const uint16_t* x, const uint16_t* h1, const uint16_t* h2,
                      const float* dy, const uint16_t* dy_bf16, float* const* dW, float* const* db, void* work,
                      size_t work_bytes, void* stream) {
  CPQR_TRY(check_mlp(net, batch));
  if (!x || !h1 || !h2 || !dy || !dy_bf16 || !dW || !db) return fail(CPQR_ERR_ARG, "mlp_backward: NULL buffer");
  for (int l = 0; l < 3; ++l)
    if (!dW[l] || !db[l]) return fail(CPQR_ERR_ARG, "mlp_backward: NULL gradient");
  CPQR_TRY(check_work(work, work_bytes, cpqr_mlp_work(net, batch)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver cv(work);
  float* part = cv.take<float>(std::max<size_t>(mlp_parts(net, batch), 1));
  float* dh = cv.take<float>(size_t(batch) * net->hidden);
  unsigned short* dh2b = cv.take<unsigned short>(size_t(batch) * net->hidden);
  unsigned short* dh1b = cv.take<unsigned short>(size_t(batch) * net->hidden);
  const int64_t B = batch, D = net->din, H = net->hidden, O = net->dout;
  const auto* W2 = reinterpret_cast<const unsigned short*>(net->W[1]);
  const auto* W3 = reinterpret_cast<const unsigned short*>(net->W[2]);
  const auto* xb = reinterpret_cast<const unsigned short*>(x);
  const auto* h1b = reinterpret_cast<const unsigned short*>(h1);
  const auto* h2b = reinterpret_cast<const unsigned short*>(h2);
  const auto* dyb = reinterpret_cast<const unsigned short*>(dy_bf16);
  // output layer: dW3 = dy^T h2, db3 = column sums of dy
  CPQR_TRY(gemm_out(false, false, O, H, B, dyb, O, h2b, H, part, nullptr, 0, nullptr, dW[2], nullptr, s));
  CPQR_TRY(colsum_enqueue(dy, B, O, db[2], s));
  // dh2 = (dy W3) masked by h2 > 0
  CPQR_TRY(gemm_out(true, false, B, H, O, dyb, O, W3, H, part, nullptr, 0, h2b, dh, dh2b, s));
  CPQR_TRY(colsum_enqueue(dh, B, H, db[1], s));
  CPQR_TRY(gemm_out(false, false, H, H, B, dh2b, H, h1b, H, part, nullptr, 0, nullptr, dW[1], nullptr, s));
  // dh1 = (dh2 W2) masked by h1 > 0
  CPQR_TRY(gemm_out(true, false, B, H, H, dh2b, H, W2, H, part, nullptr, 0, h1b, dh, dh1b, s));
  CPQR_TRY(colsum_enqueue(dh, B, H, db[0], s));
  return gemm_out(false, false, H, D, B, dh1b, H, xb, D, part, nullptr, 0, nullptr, dW[0], nullptr, s);
}

int cpqr_kruskal_loss_grad(int batch, const int64_t* I, int R, int Rt, const float* y, int64_t ldy,
                           const float* target, int64_t ldt, int kind, float* loss, float* dy, uint16_t* dy_bf16,
                           float scale, void* stream) {
  if (batch < 1 || !I || !y || !target || !dy) return fail(CPQR_ERR_ARG, "kruskal_loss_grad: bad arguments");
  if (kind != CPQR_LOSS_DISTANCE && kind != CPQR_LOSS_COSINE) return fail(CPQR_ERR_ARG, "kruskal_loss_grad: unknown loss");
  if (R < 1 || R > KRB || Rt < 1 || Rt > KRB) return fail(CPQR_ERR_SHAPE, "kruskal_loss_grad: ranks must be in [1, 16]");
  for (int k = 0; k < 3; ++k)
    if (I[k] < 1 || I[k] > 256) return fail(CPQR_ERR_SHAPE, "kruskal_loss_grad: mode sizes must be in [1, 256]");
  if (ldy < (I[0] + I[1] + I[2]) * R || ldt < (I[0] + I[1] + I[2]) * Rt)
    return fail(CPQR_ERR_SHAPE, "kruskal_loss_grad: leading dimension too small");
  hipLaunchKernelGGL(kruskal_grad_kernel, dim3(unsigned(batch)), dim3(KT), 0, static_cast<hipStream_t>(stream), I[0],
                     I[1], I[2], R, Rt, y, ldy, target, ldt, kind, loss, dy, reinterpret_cast<unsigned short*>(dy_bf16),
                     scale);
  return check_launch("kruskal_grad_kernel");
}

int cpqr_adam(int64_t n, float* w, const float* g, float* m, float* v, uint16_t* w_bf16, int step, float lr,
              float beta1, float beta2, float eps, void* stream) {
  if (n < 1 || !w || !g || !m || !v || step < 1) return fail(CPQR_ERR_ARG, "adam: bad arguments");
  const float c1 = float(1.0 - std::pow(double(beta1), step)), c2 = float(1.0 - std::pow(double(beta2), step));
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), n, w, g, m, v,
                     reinterpret_cast<unsigned short*>(w_bf16), lr, beta1, beta2, eps, c1, c2);
  return check_launch("adam_kernel");
}

int cpqr_to_bf16(const float* x, int64_t n, uint16_t* y, void* stream) {
  if (!x || !y || n < 0) return fail(CPQR_ERR_ARG, "to_bf16: bad arguments");
  if (n == 0) return CPQR_OK;
  return to_bf16_enqueue(x, n, nullptr, reinterpret_cast<unsigned short*>(y), static_cast<hipStream_t>(stream));
}

size_t cpqr_sketch3_work(const int64_t* I, const int* J) {
  if (check_sketch(I, J) != CPQR_OK) return 0;
  return sketch_work(I, J);
}

int cpqr_sketch3(const int64_t* I, const float* X, const int* J, const uint16_t* const* S, float* xs,
                 uint16_t* xs_bf16, void* work, size_t work_bytes, void* stream) {
  CPQR_TRY(check_sketch(I, J));
  if (!X || !S || !S[0] || !S[1] || !S[2] || !xs) return fail(CPQR_ERR_ARG, "sketch3: NULL buffer");
  CPQR_TRY(check_work(work, work_bytes, sketch_work(I, J)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver cv(work);
  unsigned short* Xb = cv.take<unsigned short>(size_t(I[0] * I[1] * I[2]));
  float* T1 = cv.take<float>(size_t(J[0] * I[1] * I[2]));
  unsigned short* T1b = cv.take<unsigned short>(size_t(J[0] * I[1] * I[2]));
  float* T2 = cv.take<float>(size_t(J[0] * J[1] * I[2]));
  unsigned short* T2b = cv.take<unsigned short>(size_t(J[0] * J[1] * I[2]));
  double* nrm = cv.take<double>(1);
  void* nwork = cv.take<char>(norm2_work(int64_t(J[0]) * J[1] * J[2]));
  const auto* S1 = reinterpret_cast<const unsigned short*>(S[0]);
  const auto* S2 = reinterpret_cast<const unsigned short*>(S[1]);
  const auto* S3 = reinterpret_cast<const unsigned short*>(S[2]);
  const int64_t I0 = I[0], I1 = I[1], I2 = I[2], J0 = J[0], J1 = J[1], J2 = J[2];
  CPQR_TRY(to_bf16_enqueue(X, I0 * I1 * I2, nullptr, Xb, s));
  // T1[j1][i2 + I2 i3] = sum_i1 S1[j1][i1] X[i1 + I1 (i2 + I2 i3)]
  CPQR_TRY(gemm_bf16_enqueue(true, true, J0, I1 * I2, I0, S1, I0, 0, Xb, I0, 0, T1, I1 * I2, 0, 1, 1, s));
  CPQR_TRY(to_bf16_enqueue(T1, J0 * I1 * I2, nullptr, T1b, s));
  // per j1: T2[j1][j2][i3] = sum_i2 S2[j2][i2] T1[j1][i2 + I2 i3]
  CPQR_TRY(gemm_bf16_enqueue(true, true, J1, I2, I1, S2, I1, 0, T1b, I1, I1 * I2, T2, I2, J1 * I2, int(J0), 1, s));
  CPQR_TRY(to_bf16_enqueue(T2, J0 * J1 * I2, nullptr, T2b, s));
  // xs[j3][j1 J2 + j2] = sum_i3 S3[j3][i3] T2[j1][j2][i3]
  CPQR_TRY(gemm_bf16_enqueue(true, true, J2, J0 * J1, I2, S3, I2, 0, T2b, I2, 0, xs, J0 * J1, 0, 1, 1, s));
  if (xs_bf16) {
    CPQR_TRY(norm2_enqueue(J0 * J1 * J2, CPQR_F32, xs, nrm, nwork, s));
    CPQR_TRY(to_bf16_enqueue(xs, J0 * J1 * J2, nrm, reinterpret_cast<unsigned short*>(xs_bf16), s));
  }
  return CPQR_OK;
}

}  // extern "C"
