// Tall-skinny Householder QR for gfx950, used for the factor QRs A_k = Q_k R_k
// and for the QR of the Khatri-Rao product of triangular factors
// V_n = Q_0 R_0 (paper section 3.1, Alg. 2), both with the orthonormal
// factor formed explicitly.
//
// Design: a reduction tree whose every node is one workgroup.  A node holds
// up to 1024 rows (16 per lane); each of its wavefronts owns four columns of
// them, so the per-column work of the Householder sweep (the reflector's
// products with the trailing columns, their update) is split over the SIMDs
// and a column costs one barrier.  The owner of column J forms reflector J
// (one in-wave norm) and publishes it in LDS; every wavefront then takes the
// products v_J^T A(:, c) of its own columns in one batched in-wave
// reduction, updates the columns right of J and records the Gram entries
// v_c^T v_J (c < J) from which the compact WY factor T of
// H_0 ... H_{R-1} = I - V T V^T follows.  A leaf holds rows of the input;
// an inner node stacks the R factors of up to 1024 / R children (one level
// for up to 1024 rows, two up to 1024 * 1024 / R).  The up-sweep runs one
// launch per level; the root's R is the answer.  The down-sweep forms Q top
// down: each node applies its reflectors to [C; 0], C being its R x R slice
// of the parent's Q (the identity at the root), and hands R x R slices to
// its children.  Every step is a genuine Householder reflection of the real
// rows, so Q has orthonormal columns even when the input is rank deficient.

#include <algorithm>

#include "common.h"
#include "wave.h"

namespace cpqr {
namespace {

enum Src { SRC_MATRIX = 0, SRC_KRP = 1 };

struct KrpSrc {
  const double* Rk[CPQR_MAX_MODES];
  int nm;  // the N-1 modes k != n, ascending (lowest varies fastest)
  int64_t ldr;
};

// Balanced leaf partition: leaf b of nl covering `rows` rows.
__device__ __host__ inline void leaf_range(int64_t rows, int64_t nl, int64_t b, int64_t& start,
                                           int& m) {
  const int64_t base = rows / nl, rem = rows % nl;
  m = int(base + (b < rem ? 1 : 0));
  start = b * base + (b < rem ? b : rem);
}

// ------------------------------------------------------------ block nodes
// A node holds at most 64 P rows (P = 4 or 16 row slots per lane), row
// 64 p + lane in slot p of every lane; wavefront w of the node holds columns
// 4 w .. 4 w + 3.  Rows beyond the node's are zero and take part in every
// step, so the code has no row-count branches.
namespace bn {

constexpr int W = 64;   // lanes per wavefront
constexpr int CW = 4;   // columns per wavefront
constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// Workspace of the tree: per level l below the root, the reflectors V_l
// ([node][p][c][lane]) and the compact-WY factors T_l ([node][row][c]); per
// level l >= 1, S_l, which holds the R factors of level l-1 going up and
// their C blocks coming down ([child][row][c]).  A one-node tree needs none.
// Every piece is a multiple of 256 bytes, so the offsets are plain prefix
// sums (shared by the host's size query and the kernels).
struct NodeLevel {
  int nodes, prev;   // nodes here and at the level below (0 at the leaves)
  size_t v, t, s;    // offsets (doubles) of V_l, T_l, S_l
};

__host__ __device__ __forceinline__ NodeLevel level_of(int64_t rows, int R, int P, int RM, int l, size_t* total) {
  const int node = W * P, g = node / R;
  NodeLevel L{int((rows + node - 1) / node), 0, 0, 0, 0};
  size_t off = 0;
  for (int k = 0;; ++k) {
    if (k > 0) {
      L.prev = L.nodes;
      L.nodes = (L.nodes + g - 1) / g;
    }
    const bool root = L.nodes == 1;
    L.v = off;
    if (!root) off += size_t(L.nodes) * P * RM * W;
    L.t = off;
    if (!root) off += size_t(L.nodes) * RM * RM;
    L.s = off;
    if (k > 0) off += size_t(L.prev) * RM * RM;
    if (k == l || root) break;
  }
  if (total) *total = off;
  return L;
}

// Number of levels (the root level has one node).
__host__ __device__ __forceinline__ int level_count(int64_t rows, int R, int P) {
  const int node = W * P, g = node / R;
  int n = int((rows + node - 1) / node), nlev = 1;
  while (n > 1) {
    n = (n + g - 1) / g;
    ++nlev;
  }
  return nlev;
}

using namespace wave;

template <int RMAX, int P>
struct Shared {
  // the current reflector while factorizing (double buffered, [p][lane]),
  // then a chunk of QCHUNK slots of V while forming Q ([slot][c][lane])
  static constexpr int QCHUNK = P < 128 / RMAX ? P : 128 / RMAX;
  double buf[(2 * P > QCHUNK * RMAX ? 2 * P : QCHUNK * RMAX) * W];
  double G[RMAX][RMAX + 1];  // G(k, J) = v_k^T v_J, k < J
  double T[RMAX][RMAX + 1];
  double C[RMAX][RMAX + 1];
  double B[RMAX][RMAX + 1];  // V1^T C
  double M[RMAX][RMAX];      // T V1^T C
  double V1[RMAX][RMAX + 1]; // the top R x R block of V
  double tau[RMAX];
  double scal[RMAX];  // 1 / (alpha - beta) of each reflector (0 if none)
  double beta[RMAX];  // R(J, J)
};

// Component of reflector c in row `row` of the node from the stored entry ac
// of column c: v_c(row) = ac * sc below the diagonal, 1 on it, 0 above.
__device__ __forceinline__ double vcomp(double ac, double sc, int c, int row) {
  return row == c ? 1.0 : (row > c ? ac * sc : 0.0);
}

// Rows of a leaf (rows beyond it, and columns >= R, are zero).
template <int RMAX, int P, int SRC>
__device__ __forceinline__ void load_leaf(double (&a)[P][CW], int w, int lane, int64_t start, int m, int R,
                                          const double* A, int64_t lda, const KrpSrc& krp) {
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int r = p * W + lane;
    const int64_t g = start + r;
    if (SRC == SRC_MATRIX) {
#pragma unroll
      for (int j = 0; j < CW; ++j) {
        const int c = w * CW + j;
        a[p][j] = (r < m && c < R) ? A[g + c * lda] : 0.0;
      }
    } else {
      // base-R digits of the row index (lowest first) by a rounded
      // reciprocal: (d + 1/2) / R sits at least 1/(2R) away from an integer,
      // far more than the rounding error for d < 2^31
      const double inv = 1.0 / double(R);
      int digit[CPQR_MAX_MODES - 1];
      int d = int(g);
#pragma unroll
      for (int k = 0; k < CPQR_MAX_MODES - 1; ++k) {
        const int q = int((double(d) + 0.5) * inv);
        digit[k] = d - q * R;
        d = q;
      }
#pragma unroll
      for (int j = 0; j < CW; ++j) {
        const int c = w * CW + j;
        double v = (r < m && c < R) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < CPQR_MAX_MODES - 1; ++k)
          if (k < krp.nm && r < m && c < R) v *= krp.Rk[k][digit[k] + c * krp.ldr];
        a[p][j] = v;
      }
    }
  }
}

// Node rows of a stacked level: row i of child k's block at node row k R + i.
template <int RMAX, int P>
__device__ __forceinline__ void load_stack(double (&a)[P][CW], int w, int lane, int m, int R, const double* S,
                                           int64_t c0) {
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int r = p * W + lane;
    const int child = r / R, i = r % R;
#pragma unroll
    for (int j = 0; j < CW; ++j)
      a[p][j] = r < m ? S[((c0 + child) * RMAX + i) * RMAX + w * CW + j] : 0.0;
  }
}

// 1 / x from the hardware estimate and two Newton steps (a few ulp at most
// from the rounded quotient; x is never 0 here).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Reflector J from the wavefront's column slot JL (rows > J of it form x):
// H_J = I - tau v v^T with v(J) = 1, v(r > J) = x(r) scal, scal =
// 1 / (alpha - beta).  Writes v ([p][lane], zero above row J) to vb and
// tau, scal and beta to the shared arrays; the column itself keeps x (its
// reflector is x scal below the diagonal, R(J, J) is beta).
template <int RMAX, int P, int JL>
__device__ __forceinline__ void reflect(const double (&a)[P][CW], int J, int lane, double* vb,
                                        Shared<RMAX, P>& sh, double (&own_scal)[CW]) {
  constexpr int NA = P < 4 ? P : 4;  // independent partial sums
  double x[P], ss[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) ss[u] = 0.0;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    x[p] = (p > 0 || lane > J) ? a[p][JL] : 0.0;
    ss[p % NA] += x[p] * x[p];
  }
#pragma unroll
  for (int u = 1; u < NA; ++u) ss[0] += ss[u];
  const double sub2 = wave_allsum(ss[0], lane);
  const double alpha = rdlane(a[0][JL], J);
  double tau = 0.0, beta = alpha, scal = 0.0;
  if (sub2 > 0.0) {
    const double nrm = sqrt(alpha * alpha + sub2);
    beta = alpha >= 0.0 ? -nrm : nrm;
    tau = (beta - alpha) * recip(beta);
    scal = recip(alpha - beta);
  }
#pragma unroll
  for (int p = 0; p < P; ++p) vb[p * W + lane] = (p == 0 && lane == J) ? 1.0 : x[p] * scal;
  own_scal[JL] = scal;
  if (lane == 0) {
    sh.tau[J] = tau;
    sh.scal[J] = scal;
    sh.beta[J] = beta;
  }
}

// Compact WY factor T of columns [b, b + NC) from sh.tau and sh.G into
// sh.T: lane i < NC forms row b + i, T(i, J) = -tau_J sum_k T(i, k) G(k, J)
// (i < J), T(J, J) = tau_J, so the lanes need no exchange.  Zero beyond R.
template <int NC, int RMAX, int P>
__device__ __forceinline__ void t_block(int R, int b, int lane, Shared<RMAX, P>& sh) {
  double t[NC];
#pragma unroll
  for (int J = 0; J < NC; ++J) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < J; ++k) acc[k % 4] += t[k] * sh.G[b + k][b + J];
    const double tj = b + J < R ? sh.tau[b + J] : 0.0;
    t[J] = lane < J ? -tj * ((acc[0] + acc[1]) + (acc[2] + acc[3])) : (lane == J ? tj : 0.0);
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) sh.T[b + lane][b + c] = t[c];
}

// T of the whole node (all threads call it).  For RMAX >= 16 the columns
// split in halves, V = [V1 V2]: the product of the reflectors is
// (I - V1 T11 V1^T)(I - V2 T22 V2^T), so T = [T11, -T11 (V1^T V2) T22; 0,
// T22], where T11 and T22 follow the recurrence within their halves
// (wavefronts 0 and 1 at once) and V1^T V2 is the block G(0:H, H:RMAX).
// This halves the recurrence's dependent chain; V1^T V2 T22 goes to sh.B,
// which is free until Q is formed.
template <int RMAX, int P>
__device__ __forceinline__ void node_t(int R, int w, int lane, Shared<RMAX, P>& sh) {
  if constexpr (RMAX < 16) {
    if (w == 0 && lane < RMAX) t_block<RMAX>(R, 0, lane, sh);
  } else {
    constexpr int H = RMAX / 2;
    static_assert(RMAX / CW >= 2 && RMAX / CW * W >= H * H, "two wavefronts and H^2 threads");
    if (w < 2 && lane < H) t_block<H>(R, w * H, lane, sh);
    const int tid = w * W + lane;
    const int i = tid / H, c = tid % H;
    if (tid < H * H) sh.T[H + i][c] = 0.0;  // below the diagonal blocks
    __syncthreads();
    if (tid < H * H) {  // B = G(0:H, H:RMAX) T22 (T22 upper triangular)
      double acc = 0.0;
#pragma unroll 4
      for (int j = 0; j <= c; ++j) acc += sh.G[i][H + j] * sh.T[H + j][H + c];
      sh.B[i][c] = acc;
    }
    __syncthreads();
    if (tid < H * H) {  // T12 = -T11 B (T11 upper triangular)
      double acc = 0.0;
#pragma unroll 4
      for (int k = i; k < H; ++k) acc += sh.T[i][k] * sh.B[k][c];
      sh.T[i][H + c] = -acc;
    }
  }
}

// Householder QR of the node (rows beyond it zero).  On return the
// wavefront's column slots hold, for its columns c, R(r, c) in rows r < c
// and x_c below the diagonal (v_c = x_c scal_c there); sh.tau, sh.scal,
// sh.beta (R's diagonal), sh.G and sh.T (zero beyond R) are set and visible.
template <int RMAX, int P>
__device__ __forceinline__ void node_factor(double (&a)[P][CW], int R, int w, int lane,
                                            Shared<RMAX, P>& sh) {
  for (int e = threadIdx.x; e < RMAX * (RMAX + 1); e += RMAX / CW * W) (&sh.G[0][0])[e] = 0.0;
  double own_scal[CW] = {0.0, 0.0, 0.0, 0.0};
  for (int J = 0; J < R; ++J) {
    double* vb = sh.buf + (J & 1) * P * W;
    const int jl = J - w * CW;
    switch (jl) {  // the owner of column J forms the reflector
      case 0: reflect<RMAX, P, 0>(a, J, lane, vb, sh, own_scal); break;
      case 1: reflect<RMAX, P, 1>(a, J, lane, vb, sh, own_scal); break;
      case 2: reflect<RMAX, P, 2>(a, J, lane, vb, sh, own_scal); break;
      case 3: reflect<RMAX, P, 3>(a, J, lane, vb, sh, own_scal); break;
      default: break;
    }
    __syncthreads();
    double v[P];
#pragma unroll
    for (int p = 0; p < P; ++p) v[p] = vb[p * W + lane];
    const double tau = sh.tau[J];
    // s_j = v^T A(:, c) for the wavefront's columns c (v is zero above row J)
    double s[CW];
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int p = 0; p < P; ++p)
        acc += v[p] * a[p][j];
      s[j] = acc;
    }
    const double red = wave_sum<CW>(s, lane);
    double sj[CW];
#pragma unroll
    for (int j = 0; j < CW; ++j) sj[j] = rdlane(red, j << (6 - ilog2(CW)));
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      const int c = w * CW + j;
      if (c > J && c < R) {
        const double tw = tau * sj[j];
#pragma unroll
        for (int p = 0; p < P; ++p)
          a[p][j] -= tw * v[p];
      } else if (c < J && lane == 0) {
        sh.G[c][J] = own_scal[j] * sj[j];  // rows >= J of column c hold x_c there
      }
    }
  }
  __syncthreads();
  node_t<RMAX>(R, w, lane, sh);
  __syncthreads();
}

// Scale of the stored reflector entries of column c: scal_c straight after
// the factorization (SCALED), 1 for reflectors read back from memory.
template <bool SCALED, int RMAX, int P>
__device__ __forceinline__ double vscale(const Shared<RMAX, P>& sh, int c) {
  return SCALED ? sh.scal[c] : 1.0;
}

// The top R x R block of V into sh.V1 (zero beyond R).
template <bool SCALED, int RMAX, int P>
__device__ __forceinline__ void node_v1(const double (&a)[P][CW], int R, int w, int lane, Shared<RMAX, P>& sh) {
  if (lane < RMAX) {
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      const int c = w * CW + j;
      sh.V1[lane][c] = (lane < R && c < R) ? vcomp(a[0][j], vscale<SCALED>(sh, c), c, lane) : 0.0;
    }
  }
}

// Q rows of a node: [C; 0] - V M with M = T V1^T C (C in sh.C, T in sh.T,
// V1 in sh.V1, all visible; IDENT: C is the identity, so V1^T C is V1^T
// and is not formed).  The rows go to the output (leaf: Qout at `start`)
// or, as C blocks, to children c0 ... of the stacked level S.
// A leaf may also write FP32 copies of its Q rows: urows[i RMAX + c] and
// uquads[((i/4) RMAX + c) 4 + i%4] for global row i (zero for c >= R).
template <bool SCALED, int RMAX, bool IDENT = false, int P>
__device__ __forceinline__ void node_q(const double (&a)[P][CW], int R, int m, int w, int lane,
                                       Shared<RMAX, P>& sh, bool leaf, int64_t start, double* Qout, int64_t ldq,
                                       double* S, int64_t c0, float* urows = nullptr, float* uquads = nullptr) {
  constexpr int NT = RMAX / CW * W;
  const int tid = w * W + lane;
  if constexpr (!IDENT) {
    for (int e = tid; e < RMAX * RMAX; e += NT) {  // B = V1^T C
      const int k = e / RMAX, c = e % RMAX;
      double acc = 0.0;
#pragma unroll 8
      for (int i = 0; i < RMAX; ++i) acc += sh.V1[i][k] * sh.C[i][c];
      sh.B[k][c] = acc;
    }
    __syncthreads();
  }
  for (int e = tid; e < RMAX * RMAX; e += NT) {  // M = T B; with C = I, B(i, c) = V1(c, i)
    const int k = e / RMAX, c = e % RMAX;
    double acc = 0.0;
#pragma unroll 8
    for (int i = 0; i < RMAX; ++i) acc += sh.T[k][i] * (IDENT ? sh.V1[c][i] : sh.B[i][c]);
    sh.M[k][c] = acc;
  }
  __syncthreads();
  double sc[CW];
#pragma unroll
  for (int j = 0; j < CW; ++j) sc[j] = w * CW + j < R ? vscale<SCALED>(sh, w * CW + j) : 0.0;
  // QCHUNK slots at a time: every wavefront stages its columns of V for
  // those rows in LDS, then forms its columns of Q for them, k outermost so
  // that each row of M is read once per chunk.
  constexpr int QC = Shared<RMAX, P>::QCHUNK;
#pragma unroll
  for (int p0 = 0; p0 < P; p0 += QC) {
    if (p0 > 0) __syncthreads();  // the previous chunk has been read
#pragma unroll
    for (int u = 0; u < QC; ++u) {
#pragma unroll
      for (int j = 0; j < CW; ++j) {
        // rows of slots >= 1 lie below every diagonal (R <= 32 < 64); sc is 0 beyond R
        const int k = w * CW + j;
        sh.buf[(u * RMAX + k) * W + lane] =
            p0 + u > 0 ? a[p0 + u][j] * sc[j] : (k < R ? vcomp(a[0][j], sc[j], k, lane) : 0.0);
      }
    }
    __syncthreads();
    double q[QC][CW];
#pragma unroll
    for (int u = 0; u < QC; ++u) {
      const int r = (p0 + u) * W + lane;
#pragma unroll
      for (int j = 0; j < CW; ++j) q[u][j] = (p0 + u == 0 && r < RMAX) ? sh.C[r][w * CW + j] : 0.0;
    }
    // rows k >= R of M and of the staged V are zero: no branches on R
#pragma unroll 4
    for (int k = 0; k < RMAX; ++k) {
      double mk[CW];
#pragma unroll
      for (int j = 0; j < CW; ++j) mk[j] = sh.M[k][w * CW + j];
#pragma unroll
      for (int u = 0; u < QC; ++u) {
        const double vk = sh.buf[(u * RMAX + k) * W + lane];
#pragma unroll
        for (int j = 0; j < CW; ++j) q[u][j] -= vk * mk[j];
      }
    }
#pragma unroll
    for (int u = 0; u < QC; ++u) {
      const int r = (p0 + u) * W + lane;
      if (r < m) {
        if (leaf) {
#pragma unroll
          for (int j = 0; j < CW; ++j) {
            const int c = w * CW + j;
            if (c < R) Qout[start + r + c * ldq] = q[u][j];
          }
          const int64_t i = start + r;
          if (urows) {
#pragma unroll
            for (int j = 0; j < CW; ++j) {
              const int c = w * CW + j;
              urows[i * RMAX + c] = c < R ? float(q[u][j]) : 0.f;
            }
          }
          if (uquads) {
#pragma unroll
            for (int j = 0; j < CW; ++j) {
              const int c = w * CW + j;
              uquads[((i >> 2) * RMAX + c) * 4 + (i & 3)] = c < R ? float(q[u][j]) : 0.f;
            }
          }
        } else {
          const int child = r / R, i = r % R;
#pragma unroll
          for (int j = 0; j < CW; ++j) S[((c0 + child) * RMAX + i) * RMAX + w * CW + j] = q[u][j];
        }
      }
    }
  }
}

// Rows and first row of node `node` at level l.
__device__ __forceinline__ void node_rows(int64_t rows, int R, int P, int l, const NodeLevel& L, int node,
                                          int64_t& start, int64_t& c0, int& m) {
  start = 0;
  c0 = 0;
  if (l == 0) {
    leaf_range(rows, L.nodes, node, start, m);
  } else {
    const int g = W * P / R;
    c0 = int64_t(node) * g;
    m = int(min<int64_t>(g, L.prev - c0)) * R;
  }
}

// Up-sweep below the root, one launch per level, one workgroup per node:
// factorize the node, save its reflectors and T, pass its R up.
template <int RMAX, int P, int SRC>
__global__ __launch_bounds__(RMAX / CW * W) void bn_up(int64_t rows, int R, int l, const double* A, int64_t lda,
                                                       KrpSrc krp, double* work) {
  __shared__ Shared<RMAX, P> sh;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / W), lane = threadIdx.x % W, node = blockIdx.x;
  const NodeLevel L = level_of(rows, R, P, RMAX, l, nullptr);
  int64_t start, c0;
  int m;
  node_rows(rows, R, P, l, L, node, start, c0, m);
  double a[P][CW];
  if (l == 0)
    load_leaf<RMAX, P, SRC>(a, w, lane, start, m, R, A, lda, krp);
  else
    load_stack<RMAX, P>(a, w, lane, m, R, work + L.s, c0);
  node_factor<RMAX>(a, R, w, lane, sh);
  double* Tg = work + L.t + size_t(node) * RMAX * RMAX;
  for (int e = threadIdx.x; e < RMAX * RMAX; e += RMAX / CW * W) Tg[e] = sh.T[e / RMAX][e % RMAX];
  // reflector entries as v (scaled); rows on and above the diagonal as stored
  double* V = work + L.v + size_t(node) * P * RMAX * W;
  double sc[CW];
#pragma unroll
  for (int j = 0; j < CW; ++j) sc[j] = w * CW + j < R ? sh.scal[w * CW + j] : 0.0;
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int j = 0; j < CW; ++j) V[(p * RMAX + w * CW + j) * W + lane] = a[p][j] * sc[j];
  if (lane < RMAX) {
    double* Snext = work + level_of(rows, R, P, RMAX, l + 1, nullptr).s;
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      const int c = w * CW + j;
      Snext[(size_t(node) * RMAX + lane) * RMAX + c] =
          (lane < R && c < R && c >= lane) ? (c == lane ? sh.beta[c] : a[0][j]) : 0.0;
    }
  }
}

// The root (one workgroup): factorize, write R, and form the root's Q from
// C = I straight away: the output itself when the root is the only leaf,
// else the C blocks of its children.
//
// NORM (a single node of an input matrix only): the columns are first
// normalized, lambda_c = ||A(:, c)||_2 and A(:, c) /= lambda_c written back
// (a zero column stays zero, lambda_c = 0, CPQR_STATUS_ZERO_COLUMN), so the
// sweep's normalization and factor QR are one launch; a wavefront holds all
// rows of its columns, so the norms need no exchange between wavefronts.
template <int RMAX, int P, int SRC, bool NORM = false>
__global__ __launch_bounds__(RMAX / CW * W) void bn_root(int64_t rows, int R, const double* A, int64_t lda,
                                                         KrpSrc krp, double* Qout, int64_t ldq, double* Rout,
                                                         int64_t ldr, double* work, double* lambda = nullptr,
                                                         int* status = nullptr, float* urows = nullptr,
                                                         float* uquads = nullptr) {
  __shared__ Shared<RMAX, P> sh;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / W), lane = threadIdx.x % W;
  const int top = level_count(rows, R, P) - 1;
  const NodeLevel L = level_of(rows, R, P, RMAX, top, nullptr);
  int64_t start, c0;
  int m;
  node_rows(rows, R, P, top, L, 0, start, c0, m);
  double a[P][CW];
  if (top == 0)
    load_leaf<RMAX, P, SRC>(a, w, lane, start, m, R, A, lda, krp);
  else
    load_stack<RMAX, P>(a, w, lane, m, R, work + L.s, 0);
  if constexpr (NORM) {
    double ss[CW];
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int p = 0; p < P; ++p) acc += a[p][j] * a[p][j];
      ss[j] = acc;
    }
    const double red = wave_sum<CW>(ss, lane);
    double* Aw = const_cast<double*>(A);
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      const int c = w * CW + j;
      const double nrm = sqrt(rdlane(red, j << (6 - ilog2(CW))));
      if (lane == 0 && c < R) {
        lambda[c] = nrm;
        if (nrm == 0.0 && status) atomicOr(status, CPQR_STATUS_ZERO_COLUMN);
      }
      if (nrm > 0.0) {
        const double inv = 1.0 / nrm;
#pragma unroll
        for (int p = 0; p < P; ++p) a[p][j] *= inv;
      }
      if (c < R) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
          const int r = p * W + lane;
          if (r < m) Aw[start + r + c * lda] = a[p][j];
        }
      }
    }
  }
  node_factor<RMAX>(a, R, w, lane, sh);
  node_v1<true, RMAX>(a, R, w, lane, sh);
  if (lane < R) {
#pragma unroll
    for (int j = 0; j < CW; ++j) {
      const int c = w * CW + j;
      if (c < R) Rout[lane + c * ldr] = c > lane ? a[0][j] : (c == lane ? sh.beta[c] : 0.0);
    }
  }
  for (int e = threadIdx.x; e < RMAX * RMAX; e += RMAX / CW * W) {
    const int i = e / RMAX, c = e % RMAX;
    sh.C[i][c] = (i < R && i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  node_q<true, RMAX, true>(a, R, m, w, lane, sh, top == 0, start, Qout, ldq, work + L.s, 0, urows, uquads);
}

// Down-sweep below the root, one launch per level: each node applies its
// reflectors to its C block and writes its Q rows: the output, or its
// children's C blocks.
template <int RMAX, int P>
__global__ __launch_bounds__(RMAX / CW * W) void bn_down(int64_t rows, int R, int l, double* Qout, int64_t ldq,
                                                         double* work) {
  __shared__ Shared<RMAX, P> sh;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / W), lane = threadIdx.x % W, node = blockIdx.x;
  const NodeLevel L = level_of(rows, R, P, RMAX, l, nullptr);
  int64_t start, c0;
  int m;
  node_rows(rows, R, P, l, L, node, start, c0, m);
  const double* V = work + L.v + size_t(node) * P * RMAX * W;
  const double* T = work + L.t + size_t(node) * RMAX * RMAX;
  const double* Cin = work + level_of(rows, R, P, RMAX, l + 1, nullptr).s + size_t(node) * RMAX * RMAX;
  double a[P][CW];
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int j = 0; j < CW; ++j) a[p][j] = V[(p * RMAX + w * CW + j) * W + lane];
  for (int e = threadIdx.x; e < RMAX * RMAX; e += RMAX / CW * W) {
    const int i = e / RMAX, c = e % RMAX;
    sh.T[i][c] = T[e];
    sh.C[i][c] = (i < R && c < R) ? Cin[e] : 0.0;
  }
  node_v1<false, RMAX>(a, R, w, lane, sh);
  __syncthreads();
  node_q<false, RMAX>(a, R, m, w, lane, sh, l == 0, start, Qout, ldq, work + L.s, c0);
}

}  // namespace bn

// ------------------------------------------------------------ host side
// Row slots per lane: 4 (256-row nodes) when that takes a single node, else
// 16 (1024-row nodes, one level up to 1024 rows).
int bn_slots(int64_t rows) { return rows <= 4 * bn::W ? 4 : 16; }

size_t bn_work(int64_t rows, int R) {
  const int P = bn_slots(rows);
  size_t total = 0;
  bn::level_of(rows, R, P, round_rank(R), bn::level_count(rows, R, P) - 1, &total);
  return total * sizeof(double);
}

template <int RMAX, int P>
int bn_launch(int src, int64_t rows, int R, const double* A, int64_t lda, const KrpSrc& krp, double* Q,
              int64_t ldq, double* Rout, int64_t ldr_out, void* work, hipStream_t s, hipEvent_t r_ready) {
  double* w = static_cast<double*>(work);
  const int nlev = bn::level_count(rows, R, P);
  const dim3 blk(RMAX / bn::CW * bn::W);
  for (int l = 0; l + 1 < nlev; ++l) {
    const dim3 grd(unsigned(bn::level_of(rows, R, P, RMAX, l, nullptr).nodes));
    if (src == SRC_MATRIX)
      hipLaunchKernelGGL((bn::bn_up<RMAX, P, SRC_MATRIX>), grd, blk, 0, s, rows, R, l, A, lda, krp, w);
    else
      hipLaunchKernelGGL((bn::bn_up<RMAX, P, SRC_KRP>), grd, blk, 0, s, rows, R, l, A, lda, krp, w);
    CPQR_TRY(check_launch("bn_up"));
  }
  if (src == SRC_MATRIX)
    hipLaunchKernelGGL((bn::bn_root<RMAX, P, SRC_MATRIX>), dim3(1), blk, 0, s, rows, R, A, lda, krp, Q, ldq, Rout,
                       ldr_out, w);
  else
    hipLaunchKernelGGL((bn::bn_root<RMAX, P, SRC_KRP>), dim3(1), blk, 0, s, rows, R, A, lda, krp, Q, ldq, Rout,
                       ldr_out, w);
  CPQR_TRY(check_launch("bn_root"));
  if (r_ready) CPQR_HIP(hipEventRecord(r_ready, s));  // R is complete; Q may follow
  for (int l = nlev - 2; l >= 0; --l) {
    const dim3 grd(unsigned(bn::level_of(rows, R, P, RMAX, l, nullptr).nodes));
    hipLaunchKernelGGL((bn::bn_down<RMAX, P>), grd, blk, 0, s, rows, R, l, Q, ldq, w);
    CPQR_TRY(check_launch("bn_down"));
  }
  return CPQR_OK;
}

int tsqr_dispatch(int src, int64_t rows, int R, const double* A, int64_t lda, const KrpSrc& krp,
                  double* Q, int64_t ldq, double* Rout, int64_t ldr_out, void* work, hipStream_t s,
                  hipEvent_t r_ready = nullptr) {
  const bool small = bn_slots(rows) == 4;
  switch (round_rank(R)) {
    case 8:
      return small ? bn_launch<8, 4>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s, r_ready)
                   : bn_launch<8, 16>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s, r_ready);
    case 16:
      return small ? bn_launch<16, 4>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s, r_ready)
                   : bn_launch<16, 16>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s, r_ready);
    default:
      return small ? bn_launch<32, 4>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s, r_ready)
                   : bn_launch<32, 16>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s, r_ready);
  }
}

}  // namespace

size_t tsqr_work(int64_t rows, int R) { return bn_work(rows, R); }

int factor_qr_enqueue(int64_t I, int R, const double* A, int64_t lda, double* Q, int64_t ldq,
                      double* Rk, int64_t ldr, void* work, hipStream_t s, hipEvent_t r_ready) {
  PhaseTimer pt(PH_FACTOR_QR, s);
  KrpSrc none{};
  return tsqr_dispatch(SRC_MATRIX, I, R, A, lda, none, Q, ldq, Rk, ldr, work, s, r_ready);
}

bool norm_qr_fits(int64_t I, int R) {
  (void)R;
  return bn::level_count(I, R, bn_slots(I)) == 1;  // a single node holds all rows
}

int normalize_factor_qr_enqueue(int64_t I, int R, double* A, double* lambda, int* status, double* Q, double* Rk,
                                void* work, hipStream_t s, hipEvent_t r_ready, bool* fused, float* urows,
                                float* uquads, int RP) {
  *fused = false;
  if (!norm_qr_fits(I, R)) return CPQR_OK;
  if ((urows || uquads) && RP != round_rank(R)) return fail(CPQR_ERR_ARG, "factor QR: FP32 copies need RP = RMAX");
  if (uquads && I % 4 != 0) return fail(CPQR_ERR_ARG, "factor QR: the four-row layout needs I % 4 == 0");
  PhaseTimer pt(PH_FACTOR_QR, s);
  KrpSrc none{};
  const bool small = bn_slots(I) == 4;
#define NQR(RM, PP)                                                                                               \
  hipLaunchKernelGGL((bn::bn_root<RM, PP, SRC_MATRIX, true>), dim3(1), dim3(RM / bn::CW * bn::W), 0, s, I, R, A, I, \
                     none, Q, I, Rk, int64_t(R), static_cast<double*>(work), lambda, status, urows, uquads)
  switch (round_rank(R)) {
    case 8: if (small) NQR(8, 4); else NQR(8, 16); break;
    case 16: if (small) NQR(16, 4); else NQR(16, 16); break;
    default: if (small) NQR(32, 4); else NQR(32, 16); break;
  }
#undef NQR
  CPQR_TRY(check_launch("bn_root (normalizing)"));
  if (r_ready) CPQR_HIP(hipEventRecord(r_ready, s));
  *fused = true;
  return CPQR_OK;
}

int krp_qr_enqueue(int N, int n, int R, const double* const* Rk, int64_t ldr, double* Q0,
                   double* R0, void* work, hipStream_t s) {
  PhaseTimer pt(PH_Q0, s);
  KrpSrc krp{};
  krp.nm = 0;
  krp.ldr = ldr;
  for (int k = 0; k < N; ++k) {
    if (k == n) continue;
    krp.Rk[krp.nm++] = Rk[k];
  }
  const int64_t rows = ipow(R, N - 1);
  return tsqr_dispatch(SRC_KRP, rows, R, nullptr, 0, krp, Q0, rows, R0, R, work, s);
}

}  // namespace cpqr
