// Tall-skinny Householder QR for gfx950, used for the factor QRs A_k = Q_k R_k
// and for the QR of the Khatri-Rao product of triangular factors
// V_n = Q_0 R_0 (paper section 3.1, Alg. 2), both with the orthonormal
// factor formed explicitly.
//
// Design.  One workgroup of NT threads owns one block ("node") of at most NT
// rows; thread t holds row t of the block in registers (R <= 32 doubles).
// Column j of the Householder factorization needs two reductions over the
// rows: the norm of the sub-column, and one batched reduction that returns at
// once the trailing products w_c = v_j^T A(:,c) (c > j) and the reflector
// Gram entries G(i,j) = v_i^T v_j (i < j).  Reductions are reduce-scatter
// butterflies inside each wavefront followed by one LDS pass across
// wavefronts; their order is fixed, so results are bitwise reproducible.
// The orthonormal factor uses the compact WY form of the reflectors,
// H_0 ... H_{R-1} = I - V T V^T with T upper triangular built from G, so
// forming Q needs no further reductions: Q [C; 0] = [C; 0] - V (T V_1^T C),
// V_1 being the top R x R block of V.
//
// Blocks larger than one workgroup are combined in a tree: the triangular
// factors of up to NT/R children are stacked and factorized again, level by
// level, until one block remains (its R is the answer).  Q is formed top
// down: each node applies its reflectors to [C; 0], where C is the node's
// R x R slice of its parent's Q, and hands R x R slices to its children.
// Every step is a genuine Householder reflection of the real rows, so Q has
// orthonormal columns even when the input is rank deficient.

#include <algorithm>

#include "common.h"
#include "wgqr.h"

namespace cpqr {
namespace {

enum Src { SRC_MATRIX = 0, SRC_KRP = 1, SRC_STACK = 2 };

struct KrpSrc {
  const double* Rk[CPQR_MAX_MODES];
  int nm;  // the N-1 modes k != n, ascending (lowest varies fastest)
  int64_t ldr;
};

struct Level {
  int nt;             // rows per node (threads per workgroup)
  int64_t nodes;      // nodes at this level
  int64_t rows;       // leaf level: rows of the input
  int64_t prev_nodes; // internal levels: nodes of the level below
  int g;              // internal levels: children per node
  double* V;          // nodes x RMAX x nt reflectors (column c of node j at (j*RMAX + c)*nt)
  double* T;          // nodes x RMAX x RMAX compact-WY factors
  double* Rin;        // internal levels: prev_nodes blocks of RMAX x RMAX (stacked R's)
};

using namespace wgqr;

// Balanced leaf partition: leaf b of nl covering `rows` rows.
__device__ __host__ inline void leaf_range(int64_t rows, int64_t nl, int64_t b, int64_t& start,
                                           int& m) {
  const int64_t base = rows / nl, rem = rows % nl;
  m = int(base + (b < rem ? 1 : 0));
  start = b * base + (b < rem ? b : rem);
}

// Rows of the node's input block.
template <int RMAX, int SRC>
__device__ inline int load_rows(double (&a)[RMAX], const Level& L, int64_t node, int R, int tid,
                                const double* A, int64_t lda, const KrpSrc& krp, int64_t& start) {
  int m;
  if (SRC == SRC_STACK) {
    const int64_t c0 = node * L.g;
    const int64_t nch = min<int64_t>(L.g, L.prev_nodes - c0);
    m = int(nch) * R;
    start = 0;
    const int child = tid / R, i = tid % R;
#pragma unroll
    for (int c = 0; c < RMAX; ++c)
      a[c] = (tid < m && c < R) ? L.Rin[((c0 + child) * RMAX + c) * RMAX + i] : 0.0;
  } else {
    leaf_range(L.rows, L.nodes, node, start, m);
    const int64_t g = start + tid;
    if (SRC == SRC_MATRIX) {
#pragma unroll
      for (int c = 0; c < RMAX; ++c) a[c] = (tid < m && c < R) ? A[g + c * lda] : 0.0;
    } else {
      int digit[CPQR_MAX_MODES];
      int64_t d = g;
#pragma unroll
      for (int t = 0; t < CPQR_MAX_MODES; ++t) {
        digit[t] = int(d % R);
        d /= R;
      }
#pragma unroll
      for (int c = 0; c < RMAX; ++c) {
        double p = (tid < m && c < R) ? 1.0 : 0.0;
#pragma unroll
        for (int t = 0; t < CPQR_MAX_MODES; ++t)
          if (t < krp.nm && tid < m && c < R) p *= krp.Rk[t][digit[t] + c * krp.ldr];
        a[c] = p;
      }
    }
  }
  return m;
}

template <int RMAX>
__device__ inline void write_q(const double (&q)[RMAX], bool leaf, int64_t start, int m,
                               double* Qout, int64_t ldq, double* Cchild, int64_t node, int g,
                               int R, int tid) {
  if (tid >= m) return;
  if (leaf) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c)
      if (c < R) Qout[start + tid + c * ldq] = q[c];
  } else {
    const int64_t child = node * g + tid / R;
    const int i = tid % R;
#pragma unroll
    for (int c = 0; c < RMAX; ++c)
      if (c < R) Cchild[(child * RMAX + c) * RMAX + i] = q[c];
  }
}

// Up-sweep of one level (factorize, store reflectors and T, pass R up).  At
// the root (nodes == 1) also writes R to Rout and forms the root's Q from
// C = I.
template <int RMAX, int NT, int SRC>
__global__ __launch_bounds__(NT) void tsqr_up(Level L, int R, const double* A, int64_t lda,
                                              KrpSrc krp, double* Rnext, double* Rout,
                                              int64_t ldr_out, double* Qout, int64_t ldq,
                                              double* Cchild, int gchild) {
  __shared__ Shared<RMAX, NT> sh;
  const int tid = threadIdx.x;
  const int64_t node = blockIdx.x;
  double a[RMAX];
  int64_t start;
  const int m = load_rows<RMAX, SRC>(a, L, node, R, tid, A, lda, krp, start);
  wg_factor<RMAX, NT>(a, tid, m, R, sh);
  wg_build_t<RMAX, NT>(tid, R, sh);
  if (L.nodes > 1) {
    double* V = L.V + node * RMAX * NT;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) V[c * NT + tid] = a[c];
    for (int e = tid; e < RMAX * RMAX; e += NT)
      L.T[node * RMAX * RMAX + e] = (e / RMAX < R && e % RMAX < R) ? sh.T[e / RMAX][e % RMAX] : 0.0;
    if (tid < R) {
#pragma unroll
      for (int c = 0; c < RMAX; ++c) Rnext[(node * RMAX + c) * RMAX + tid] = (c >= tid) ? a[c] : 0.0;
    }
    return;
  }
  if (tid < R) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c)
      if (c < R) Rout[tid + c * ldr_out] = (c >= tid) ? a[c] : 0.0;
  }
  for (int e = tid; e < RMAX * RMAX; e += NT) sh.C[e / RMAX][e % RMAX] = (e / RMAX == e % RMAX) ? 1.0 : 0.0;
  __syncthreads();
  double q[RMAX];
  wg_form_q<RMAX, NT>(a, q, tid, m, R, sh);
  write_q<RMAX>(q, SRC != SRC_STACK, start, m, Qout, ldq, Cchild, node, gchild, R, tid);
}

// Down-sweep of one non-root level: form each node's Q from its C block.
template <int RMAX, int NT, bool LEAF>
__global__ __launch_bounds__(NT) void tsqr_down(Level L, int R, const double* Cin, double* Qout,
                                                int64_t ldq, double* Cchild, int gchild) {
  __shared__ Shared<RMAX, NT> sh;
  const int tid = threadIdx.x;
  const int64_t node = blockIdx.x;
  double a[RMAX], q[RMAX];
  const double* V = L.V + node * RMAX * NT;
#pragma unroll
  for (int c = 0; c < RMAX; ++c) a[c] = V[c * NT + tid];
  for (int e = tid; e < RMAX * RMAX; e += NT) {
    sh.T[e / RMAX][e % RMAX] = L.T[node * RMAX * RMAX + e];
    sh.C[e % RMAX][e / RMAX] = Cin[node * RMAX * RMAX + e];  // C blocks are column-major
  }
  int m;
  int64_t start = 0;
  if (LEAF) {
    leaf_range(L.rows, L.nodes, node, start, m);
  } else {
    const int64_t c0 = node * L.g;
    m = int(min<int64_t>(L.g, L.prev_nodes - c0)) * R;
  }
  __syncthreads();
  wg_form_q<RMAX, NT>(a, q, tid, m, R, sh);
  write_q<RMAX>(q, LEAF, start, m, Qout, ldq, Cchild, node, gchild, R, tid);
}

// ------------------------------------------------------------ one-workgroup wave tree
// For up to some thousands of rows the kernels above are bound by latency:
// each of the R columns costs two reductions across the whole workgroup, each
// with two workgroup barriers.  Here every node of the tree is one wavefront
// holding at most 64 P rows (P rows per lane, row 64 p + lane in slot p), and
// the whole tree runs inside one workgroup of a few wavefronts, level by
// level, with a workgroup barrier only between levels.
//
// Column j of a wavefront node costs one in-wave reduction.  With x the
// sub-column below the diagonal (rows r > j) it returns, in one batch of R
// sums, s_c = sum_r x(r) A(r, c) for every column c: s_j = ||x||^2 gives the
// reflector, s_c (c > j) the trailing products v_j^T A(:, c) = A(j, c) +
// s_c / (alpha - beta), and s_c (c < j) the reflector Gram entries
// v_c^T v_j = v_c(j) + s_c / (alpha - beta) for the compact WY factor T.
// Row j itself (alpha, A(j, c), v_c(j)) lives in lane j, slot 0 (R <= 32),
// and is broadcast from there.
namespace wt {

constexpr int W = 64;
constexpr int MAXLEV = 16;

// Workspace of the tree: per level l, the reflectors V_l ([node][p][c][lane]),
// the compact-WY factors T_l ([node][row][c]) and, for l >= 1, S_l, which
// holds the R factors of level l-1 going up and their C blocks coming down
// ([child][row][c]).  Every piece is a multiple of 256 bytes, so the offsets
// are plain prefix sums (shared by the host's size query and the kernel).
struct NodeLevel {
  int nodes, prev;        // nodes here and at the level below (0 at the leaves)
  size_t v, t, s;         // offsets (doubles) of V_l, T_l, S_l
};

__host__ __device__ __forceinline__ NodeLevel level_of(int64_t rows, int R, int P, int RM, int l, size_t* total) {
  const int g = W * P / R;
  NodeLevel L{int((rows + W * P - 1) / (W * P)), 0, 0, 0, 0};
  size_t off = 0;
  for (int k = 0;; ++k) {
    if (k > 0) {
      L.prev = L.nodes;
      L.nodes = (L.nodes + g - 1) / g;
    }
    L.v = off;
    off += size_t(L.nodes) * P * RM * W;
    L.t = off;
    off += size_t(L.nodes) * RM * RM;
    L.s = off;
    if (k > 0) off += size_t(L.prev) * RM * RM;
    if (k == l || L.nodes == 1) break;
  }
  if (total) *total = off;
  return L;
}

// Number of levels (the root level has one node).
__host__ __device__ __forceinline__ int level_count(int64_t rows, int R, int P) {
  const int g = W * P / R;
  int n = int((rows + W * P - 1) / (W * P)), nlev = 1;
  while (n > 1) {
    n = (n + g - 1) / g;
    ++nlev;
  }
  return nlev;
}

template <int RMAX>
struct Buf {
  double row[RMAX];           // row J of the node, broadcast during column J
  double sum[RMAX];           // the column's reduction results s_c
  double X[RMAX][RMAX + 1];
  double Y[RMAX][RMAX + 1];
  double Z[RMAX][RMAX];
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double rdlane(double x, int l) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
  const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(unsigned(b)), l));
  const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(unsigned(b >> 32)), l));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

__device__ __forceinline__ unsigned lo32(double x) {
  return unsigned(static_cast<unsigned long long>(__double_as_longlong(x)));
}
__device__ __forceinline__ unsigned hi32(double x) {
  return unsigned(static_cast<unsigned long long>(__double_as_longlong(x)) >> 32);
}
__device__ __forceinline__ double mkd(unsigned lo, unsigned hi) {
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// DPP lane moves within a row of 16 lanes: lanes of the enabled banks (groups
// of four lanes) take `src` from the lane CTRL names, the others keep `old`.
constexpr int DPP_XOR1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int DPP_MIRROR = 0x140;      // lane i of a row takes lane 15 - i
constexpr int DPP_HALF_MIRROR = 0x141; // lane i of a half row takes lane 7 - i
template <int CTRL, int BANKS>
__device__ __forceinline__ double dpp(double old, double src) {
  const unsigned lo = unsigned(__builtin_amdgcn_update_dpp(int(lo32(old)), int(lo32(src)), CTRL, 0xF, BANKS, false));
  const unsigned hi = unsigned(__builtin_amdgcn_update_dpp(int(hi32(old)), int(hi32(src)), CTRL, 0xF, BANKS, false));
  return mkd(lo, hi);
}

// Exchange across the halves of the wave (SPAN 32) or between neighbouring
// rows (SPAN 16).  The lanes with the SPAN bit clear get a from their partner
// lane (SPAN bit set) and keep their own a; the others get b from their
// partner and keep their own b; the two are summed.
template <int SPAN>
__device__ __forceinline__ double swap_sum(double a, double b) {
  if (SPAN == 32) {
    const auto l = __builtin_amdgcn_permlane32_swap(lo32(a), lo32(b), false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi32(a), hi32(b), false, false);
    return mkd(l[0], h[0]) + mkd(l[1], h[1]);
  } else {
    const auto l = __builtin_amdgcn_permlane16_swap(lo32(a), lo32(b), false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi32(a), hi32(b), false, false);
    return mkd(l[0], h[0]) + mkd(l[1], h[1]);
  }
}

// One level of the butterfly on lane bit B: the lanes with bit B clear keep
// (their a) + (partner's a), the others (their b) + (partner's b).  Bits 5
// and 4 use the permlane swaps, bits 3 and 2 the (half-)row mirrors, whose
// partner also differs in the lower bits; that is harmless because the lower
// bits are reduced afterwards.
template <int B>
__device__ __forceinline__ double bfly(double a, double b, int lane) {
  if (B == 5) return swap_sum<32>(a, b);
  if (B == 4) return swap_sum<16>(a, b);
  if (B == 3) return dpp<DPP_MIRROR, 0x3>(b, a) + dpp<DPP_MIRROR, 0xC>(a, b);
  if (B == 2) return dpp<DPP_HALF_MIRROR, 0x5>(b, a) + dpp<DPP_HALF_MIRROR, 0xA>(a, b);
  const bool hi = (lane >> B) & 1;
  const double send = hi ? a : b;
  return (hi ? b : a) + dpp<B == 1 ? DPP_XOR2 : DPP_XOR1, 0xF>(send, send);
}

// Sum over the 64 lanes of each x[i] (V a power of two <= 32): a
// reduce-scatter butterfly on lane bits 5, 4, ... splits the vector in half
// at each level, then the remaining lane bits are summed; sum i ends in the
// lanes whose bits 5 .. 6 - log2 V spell i, i.e. lanes (i << (6 - log2 V)) ..
// Returns the lane's sum, index lane >> (6 - log2 V).
template <int V, int LEV = 0>
__device__ __forceinline__ double wave_sum(double (&x)[V], int lane) {
  constexpr int L = ilog2(V);
  if constexpr (LEV < L) {
    constexpr int H = V >> (LEV + 1);
#pragma unroll
    for (int i = 0; i < H; ++i) x[i] = bfly<5 - LEV>(x[i], x[H + i], lane);
    return wave_sum<V, LEV + 1>(x, lane);
  } else if constexpr (LEV < 6) {
    x[0] = bfly<5 - LEV>(x[0], x[0], lane);
    return wave_sum<V, LEV + 1>(x, lane);
  } else {
    return x[0];
  }
}

// Column J of the wavefront Householder QR (J < R).  A template per column
// keeps every register-array index a compile-time constant.  alpha and s_J
// are read from their lanes directly; the other entries of row J and the
// other sums reach every lane through LDS while the reflector is formed.
template <int J, int RMAX, int P>
__device__ __forceinline__ void wave_column(double (&a)[P][RMAX], double (&t)[RMAX], int lane, int R,
                                            Buf<RMAX>& b) {
  constexpr int SH = 6 - ilog2(RMAX);
  if (lane == J) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c) b.row[c] = a[0][c];
  }
  double x[P], p[RMAX];
#pragma unroll
  for (int s = 0; s < P; ++s) x[s] = (s > 0 || lane > J) ? a[s][J] : 0.0;
#pragma unroll
  for (int c = 0; c < RMAX; ++c) {
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < P; ++s) acc += a[s][c] * x[s];
    p[c] = acc;
  }
  const double red = wave_sum<RMAX>(p, lane);
  if ((lane & ((1 << SH) - 1)) == 0) b.sum[lane >> SH] = red;
  const double alpha = rdlane(a[0][J], J), sub2 = rdlane(red, J << SH);
  wave_sync();
  double tau = 0.0, beta = alpha, scal = 0.0;
  if (sub2 > 0.0) {
    const double nrm = sqrt(alpha * alpha + sub2);
    beta = alpha >= 0.0 ? -nrm : nrm;
    tau = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
  double v[P];
#pragma unroll
  for (int s = 0; s < P; ++s) v[s] = (s == 0 && lane == J) ? 1.0 : x[s] * scal;
  // T(0:J, J) = -tau T(0:J, 0:J) G(0:J, J), G(k, J) = v_k^T v_J = v_k(J) + scal s_k
  double tg = 0.0;
#pragma unroll
  for (int k = 0; k < J; ++k) tg += t[k] * (b.row[k] + scal * b.sum[k]);
  t[J] = lane < J ? -tau * tg : (lane == J ? tau : 0.0);
  // trailing columns: A(:, c) -= tau v (v^T A(:, c)), v^T A(:, c) = A(J, c) + scal s_c
#pragma unroll
  for (int c = J + 1; c < RMAX; ++c) {
    if (c < R) {
      const double tw = tau * (b.row[c] + scal * b.sum[c]);
#pragma unroll
      for (int s = 0; s < P; ++s) a[s][c] -= tw * v[s];
    }
  }
  a[0][J] = lane == J ? beta : (lane > J ? v[0] : a[0][J]);
#pragma unroll
  for (int s = 1; s < P; ++s) a[s][J] = v[s];
  wave_sync();
}

template <int J, int RMAX, int P>
struct WaveColumns {
  static __device__ __forceinline__ void run(double (&a)[P][RMAX], double (&t)[RMAX], int lane, int R,
                                             Buf<RMAX>& b) {
    if (J >= R) return;
    wave_column<J, RMAX, P>(a, t, lane, R, b);
    WaveColumns<J + 1, RMAX, P>::run(a, t, lane, R, b);
  }
};
template <int RMAX, int P>
struct WaveColumns<RMAX, RMAX, P> {
  static __device__ __forceinline__ void run(double (&)[P][RMAX], double (&)[RMAX], int, int, Buf<RMAX>&) {}
};

// Householder QR of the node block (row 64 p + lane in a[p][.]; rows beyond
// the block and columns >= R are zero).  On return lanes < R of slot 0 hold
// R's rows (entries c >= lane), the rows below column c's diagonal hold
// reflector c's components (v_c(c) = 1 implicitly), and t[] holds row `lane`
// of T (lanes < R).
template <int RMAX, int P>
__device__ __forceinline__ void wave_factor(double (&a)[P][RMAX], double (&t)[RMAX], int lane, int R,
                                            Buf<RMAX>& b) {
#pragma unroll
  for (int c = 0; c < RMAX; ++c) t[c] = 0.0;
  WaveColumns<0, RMAX, P>::run(a, t, lane, R, b);
}

// Component of reflector c in row `row` of the node (from a[slot][c]).
__device__ __forceinline__ double vcomp(double ac, int c, int row) {
  return row == c ? 1.0 : (row > c ? ac : 0.0);
}

// Compact-WY product M = T V1^T C into b.Z, with C (R x R, zero beyond) in
// b.Z on entry; returns row `lane` of C (lanes < R, else zero) in crow[].
// Every R x R operand is zero-padded to RMAX, so the products run over fixed
// trip counts.
template <int RMAX, int P>
__device__ __forceinline__ void wave_m(const double (&a)[P][RMAX], const double (&t)[RMAX],
                                       double (&crow)[RMAX], int lane, int R, Buf<RMAX>& b) {
  constexpr int NE = (RMAX * RMAX + W - 1) / W;
  if (lane < RMAX) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
      b.X[lane][c] = (lane < R && c < R) ? vcomp(a[0][c], c, lane) : 0.0;
      b.Y[lane][c] = lane < R ? t[c] : 0.0;
    }
  }
  wave_sync();
  // lane's entries e = lane + 64 u: column c = lane % RMAX, rows k_u
  const int cc = lane % RMAX, k0 = lane / RMAX;
  constexpr int KS = W / RMAX < RMAX ? W / RMAX : RMAX;
  double e1[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) e1[u] = 0.0;
#pragma unroll 2
  for (int i = 0; i < RMAX; ++i) {  // B = V1^T C
    const double z = b.Z[i][cc];
#pragma unroll
    for (int u = 0; u < NE; ++u) e1[u] += b.X[i][(k0 + u * KS) % RMAX] * z;
  }
#pragma unroll
  for (int c = 0; c < RMAX; ++c) crow[c] = lane < RMAX ? b.Z[lane % RMAX][c] : 0.0;
  wave_sync();
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = lane + u * W;
    if (e < RMAX * RMAX) b.X[e / RMAX][e % RMAX] = e1[u];
  }
  wave_sync();
#pragma unroll
  for (int u = 0; u < NE; ++u) e1[u] = 0.0;
#pragma unroll 2
  for (int i = 0; i < RMAX; ++i) {  // M = T B
    const double x = b.X[i][cc];
#pragma unroll
    for (int u = 0; u < NE; ++u) e1[u] += b.Y[(k0 + u * KS) % RMAX][i] * x;
  }
  wave_sync();
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = lane + u * W;
    if (e < RMAX * RMAX) b.Z[e / RMAX][e % RMAX] = e1[u];
  }
  wave_sync();
}

// Row 64 s + lane of the node's Q: [C; 0](row) - v(row) M, M in b.Z.
template <int RMAX, int P>
__device__ __forceinline__ void wave_q_row(const double (&a)[P][RMAX], const double (&crow)[RMAX], int s,
                                  double (&q)[RMAX], int lane, int R, const Buf<RMAX>& b) {
  const int row = s * W + lane;
#pragma unroll
  for (int c = 0; c < RMAX; ++c) q[c] = s == 0 ? crow[c] : 0.0;
#pragma unroll 2
  for (int k = 0; k < RMAX; ++k) {
    double vk = 0.0;
#pragma unroll
    for (int kk = 0; kk < RMAX; ++kk) vk = (kk == k && k < R) ? vcomp(a[s][kk], kk, row) : vk;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) q[c] -= vk * b.Z[k][c];
  }
}

// Rows of a leaf (rows beyond it, and columns >= R, are zero).
template <int RMAX, int P, int SRC>
__device__ __forceinline__ void load_leaf(double (&a)[P][RMAX], int lane, int64_t start, int m, int R,
                                 const double* A, int64_t lda, const KrpSrc& krp) {
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int r = s * W + lane;
    const int64_t g = start + r;
    if (SRC == SRC_MATRIX) {
#pragma unroll
      for (int c = 0; c < RMAX; ++c) a[s][c] = (r < m && c < R) ? A[g + c * lda] : 0.0;
    } else {
      int digit[CPQR_MAX_MODES];
      int d = int(g);
#pragma unroll
      for (int k = 0; k < CPQR_MAX_MODES; ++k) {
        digit[k] = d % R;
        d /= R;
      }
#pragma unroll
      for (int c = 0; c < RMAX; ++c) {
        double p = (r < m && c < R) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < CPQR_MAX_MODES; ++k)
          if (k < krp.nm && r < m && c < R) p *= krp.Rk[k][digit[k] + c * krp.ldr];
        a[s][c] = p;
      }
    }
  }
}

// Node rows of a stacked level: row i of child k's block at node row k R + i.
template <int RMAX, int P>
__device__ __forceinline__ void load_stack(double (&a)[P][RMAX], int lane, int m, int R, const double* S,
                                  int64_t c0) {
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int r = s * W + lane;
    const int child = r / R, i = r % R;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) a[s][c] = r < m ? S[((c0 + child) * RMAX + i) * RMAX + c] : 0.0;
  }
}

// Writes the node's Q rows: to the output (leaf) or as the children's C blocks.
template <int RMAX, int P>
__device__ __forceinline__ void store_q(const double (&a)[P][RMAX], const double (&crow)[RMAX], int lane, int R,
                               int m, bool leaf, int64_t start, double* Qout, int64_t ldq, double* S,
                               int64_t c0, const Buf<RMAX>& b) {
#pragma unroll
  for (int s = 0; s < P; ++s) {
    double q[RMAX];
    wave_q_row<RMAX, P>(a, crow, s, q, lane, R, b);
    const int r = s * W + lane;
    if (r >= m) continue;
    if (leaf) {
#pragma unroll
      for (int c = 0; c < RMAX; ++c)
        if (c < R) Qout[start + r + c * ldq] = q[c];
    } else {
      const int child = r / R, i = r % R;
#pragma unroll
      for (int c = 0; c < RMAX; ++c) S[((c0 + child) * RMAX + i) * RMAX + c] = q[c];
    }
  }
}

// Up-sweep: factorize every node, save its reflectors and T, pass R up; the
// root's R is the answer.
template <int RMAX, int P, int NW, int SRC>
__global__ __launch_bounds__(NW * W) void wave_tree_up(int64_t rows, int R, const double* A, int64_t lda,
                                                      KrpSrc krp, double* Rout, int64_t ldr, double* work) {
  __shared__ Buf<RMAX> bufs[NW];
  const int lane = threadIdx.x % W, w = threadIdx.x / W;
  Buf<RMAX>& b = bufs[w];
  const int g = W * P / R;
  const int top = level_count(rows, R, P) - 1;
  double a[P][RMAX], t[RMAX];
#pragma unroll 1
  for (int l = 0; l <= top; ++l) {
    const NodeLevel L = level_of(rows, R, P, RMAX, l, nullptr);
    double* Snext = l < top ? work + level_of(rows, R, P, RMAX, l + 1, nullptr).s : nullptr;
#pragma unroll 1
    for (int node = w; node < L.nodes; node += NW) {
      if (l == 0) {
        int m;
        int64_t start;
        leaf_range(rows, L.nodes, node, start, m);
        load_leaf<RMAX, P, SRC>(a, lane, start, m, R, A, lda, krp);
      } else {
        const int64_t c0 = int64_t(node) * g;
        const int m = int(min<int64_t>(g, L.prev - c0)) * R;
        load_stack<RMAX, P>(a, lane, m, R, work + L.s, c0);
      }
      wave_factor<RMAX, P>(a, t, lane, R, b);
      double* V = work + L.v + int64_t(node) * P * RMAX * W;
#pragma unroll
      for (int s = 0; s < P; ++s)
#pragma unroll
        for (int c = 0; c < RMAX; ++c) V[(s * RMAX + c) * W + lane] = a[s][c];
      if (lane < R) {
        double* T = work + L.t + int64_t(node) * RMAX * RMAX;
#pragma unroll
        for (int c = 0; c < RMAX; ++c) {
          T[lane * RMAX + c] = t[c];
          const double r = c >= lane ? a[0][c] : 0.0;
          if (l < top)
            Snext[(int64_t(node) * RMAX + lane) * RMAX + c] = r;
          else if (c < R)
            Rout[lane + c * ldr] = r;
        }
      }
    }
    __syncthreads();
  }
}

// Down-sweep: each node applies its reflectors to its C block (the identity
// at the root) and writes its Q rows: the output, or its children's C blocks.
template <int RMAX, int P, int NW>
__global__ __launch_bounds__(NW * W) void wave_tree_down(int64_t rows, int R, double* Qout, int64_t ldq,
                                                        double* work) {
  __shared__ Buf<RMAX> bufs[NW];
  const int lane = threadIdx.x % W, w = threadIdx.x / W;
  Buf<RMAX>& b = bufs[w];
  const int g = W * P / R;
  const int top = level_count(rows, R, P) - 1;
  double a[P][RMAX], t[RMAX], crow[RMAX];
#pragma unroll 1
  for (int l = top; l >= 0; --l) {
    const NodeLevel L = level_of(rows, R, P, RMAX, l, nullptr);
    const double* Cin = l < top ? work + level_of(rows, R, P, RMAX, l + 1, nullptr).s : nullptr;
#pragma unroll 1
    for (int node = w; node < L.nodes; node += NW) {
      const double* V = work + L.v + int64_t(node) * P * RMAX * W;
      const double* T = work + L.t + int64_t(node) * RMAX * RMAX;
#pragma unroll
      for (int s = 0; s < P; ++s)
#pragma unroll
        for (int c = 0; c < RMAX; ++c) a[s][c] = V[(s * RMAX + c) * W + lane];
#pragma unroll
      for (int c = 0; c < RMAX; ++c) t[c] = lane < R ? T[lane * RMAX + c] : 0.0;
      for (int e = lane; e < RMAX * RMAX; e += W) {
        const int i = e / RMAX, c = e % RMAX;
        b.Z[i][c] = (i >= R || c >= R) ? 0.0
                    : (l < top ? Cin[int64_t(node) * RMAX * RMAX + e] : (i == c ? 1.0 : 0.0));
      }
      wave_sync();
      wave_m<RMAX, P>(a, t, crow, lane, R, b);
      int m;
      int64_t start = 0, c0 = 0;
      if (l == 0) {
        leaf_range(rows, L.nodes, node, start, m);
      } else {
        c0 = int64_t(node) * g;
        m = int(min<int64_t>(g, L.prev - c0)) * R;
      }
      store_q<RMAX, P>(a, crow, lane, R, m, l == 0, start, Qout, ldq, work + L.s, c0, b);
    }
    __syncthreads();
  }
}

}  // namespace wt

// ------------------------------------------------------------ host side
constexpr int ntmax_for(int RM) { return RM <= 16 ? 1024 : 512; }

int pick_nt(int64_t rows, int RM) {
  if (rows <= 64) return 64;
  if (rows <= 256) return 256;
  return ntmax_for(RM);
}

struct Tree {
  int nlev = 0;
  Level lev[40];
};

Tree make_tree(int64_t rows, int R, int RM) {
  Tree t;
  const int ntm = ntmax_for(RM);
  Level L{};
  L.nodes = rows <= ntm ? 1 : ceil_div(rows, ntm);
  L.rows = rows;
  L.nt = L.nodes == 1 ? pick_nt(rows, RM) : ntm;
  t.lev[t.nlev++] = L;
  while (t.lev[t.nlev - 1].nodes > 1) {
    const int64_t prev = t.lev[t.nlev - 1].nodes;
    Level U{};
    U.g = ntm / R;
    U.prev_nodes = prev;
    U.nodes = ceil_div(prev, U.g);
    const int64_t rows_here = std::min<int64_t>(U.g, prev) * R;
    U.nt = U.nodes == 1 ? pick_nt(rows_here, RM) : ntm;
    t.lev[t.nlev++] = U;
  }
  return t;
}

size_t carve_tree(Carver& cv, Tree& t, int RM) {
  for (int l = 0; l < t.nlev; ++l) {
    Level& L = t.lev[l];
    L.V = cv.take<double>(size_t(L.nodes) * RM * L.nt);
    L.T = cv.take<double>(size_t(L.nodes) * RM * RM);
    if (l > 0) L.Rin = cv.take<double>(size_t(L.prev_nodes) * RM * RM);
  }
  return cv.bytes();
}

template <int RMAX, int NT>
int launch_up(int src, const Level& L, int R, const double* A, int64_t lda, const KrpSrc& krp,
              double* Rnext, double* Rout, int64_t ldr_out, double* Q, int64_t ldq, double* Cchild,
              int gchild, hipStream_t s) {
  const dim3 grd(unsigned(L.nodes)), blk(NT);
  if (src == SRC_MATRIX)
    hipLaunchKernelGGL((tsqr_up<RMAX, NT, SRC_MATRIX>), grd, blk, 0, s, L, R, A, lda, krp, Rnext, Rout,
                       ldr_out, Q, ldq, Cchild, gchild);
  else if (src == SRC_KRP)
    hipLaunchKernelGGL((tsqr_up<RMAX, NT, SRC_KRP>), grd, blk, 0, s, L, R, A, lda, krp, Rnext, Rout,
                       ldr_out, Q, ldq, Cchild, gchild);
  else
    hipLaunchKernelGGL((tsqr_up<RMAX, NT, SRC_STACK>), grd, blk, 0, s, L, R, A, lda, krp, Rnext, Rout,
                       ldr_out, Q, ldq, Cchild, gchild);
  return check_launch("tsqr_up");
}

template <int RMAX, int NT>
int launch_down(bool leaf, const Level& L, int R, const double* Cin, double* Q, int64_t ldq,
                double* Cchild, int gchild, hipStream_t s) {
  const dim3 grd(unsigned(L.nodes)), blk(NT);
  if (leaf)
    hipLaunchKernelGGL((tsqr_down<RMAX, NT, true>), grd, blk, 0, s, L, R, Cin, Q, ldq, Cchild, gchild);
  else
    hipLaunchKernelGGL((tsqr_down<RMAX, NT, false>), grd, blk, 0, s, L, R, Cin, Q, ldq, Cchild, gchild);
  return check_launch("tsqr_down");
}

template <int RMAX>
int dispatch_up(int nt, int src, const Level& L, int R, const double* A, int64_t lda,
                const KrpSrc& krp, double* Rnext, double* Rout, int64_t ldr_out, double* Q,
                int64_t ldq, double* Cchild, int gchild, hipStream_t s) {
  constexpr int NTM = ntmax_for(RMAX);
  if (nt == 64)
    return launch_up<RMAX, 64>(src, L, R, A, lda, krp, Rnext, Rout, ldr_out, Q, ldq, Cchild, gchild, s);
  if (nt == 256)
    return launch_up<RMAX, 256>(src, L, R, A, lda, krp, Rnext, Rout, ldr_out, Q, ldq, Cchild, gchild, s);
  return launch_up<RMAX, NTM>(src, L, R, A, lda, krp, Rnext, Rout, ldr_out, Q, ldq, Cchild, gchild, s);
}

template <int RMAX>
int dispatch_down(int nt, bool leaf, const Level& L, int R, const double* Cin, double* Q,
                  int64_t ldq, double* Cchild, int gchild, hipStream_t s) {
  constexpr int NTM = ntmax_for(RMAX);
  if (nt == 64) return launch_down<RMAX, 64>(leaf, L, R, Cin, Q, ldq, Cchild, gchild, s);
  if (nt == 256) return launch_down<RMAX, 256>(leaf, L, R, Cin, Q, ldq, Cchild, gchild, s);
  return launch_down<RMAX, NTM>(leaf, L, R, Cin, Q, ldq, Cchild, gchild, s);
}

template <int RMAX>
int tsqr_run(int src, int64_t rows, int R, const double* A, int64_t lda, const KrpSrc& krp,
             double* Q, int64_t ldq, double* Rout, int64_t ldr_out, void* work, hipStream_t s) {
  Tree t = make_tree(rows, R, RMAX);
  Carver cv(work);
  carve_tree(cv, t, RMAX);
  for (int l = 0; l < t.nlev; ++l) {
    const Level& L = t.lev[l];
    double* Rnext = (l + 1 < t.nlev) ? t.lev[l + 1].Rin : nullptr;
    double* Cchild = l > 0 ? L.Rin : nullptr;
    const int gchild = l > 0 ? L.g : 0;
    CPQR_TRY(dispatch_up<RMAX>(L.nt, l == 0 ? src : SRC_STACK, L, R, A, lda, krp, Rnext, Rout,
                               ldr_out, Q, ldq, Cchild, gchild, s));
  }
  for (int l = t.nlev - 2; l >= 0; --l) {
    const Level& L = t.lev[l];
    const double* Cin = t.lev[l + 1].Rin;
    CPQR_TRY(dispatch_down<RMAX>(L.nt, l == 0, L, R, Cin, Q, ldq, l > 0 ? L.Rin : nullptr,
                                 l > 0 ? L.g : 0, s));
  }
  return CPQR_OK;
}

// One-workgroup wave tree: rows per lane P and wavefronts per workgroup NW
// for a problem, or P = 0 where the multi-workgroup tree is faster (measured
// on MI355X: the wave tree wins up to about 2k rows at R <= 16, up to about
// 6k rows at R <= 8, and only for a single node at R > 16).
struct WtShape {
  int P, NW;
};
WtShape wt_shape(int64_t rows, int R) {
  switch (round_rank(R)) {
    case 8:
      if (rows <= 128) return {2, 8};
      if (rows <= 256) return {4, 8};
      if (rows <= 1024) return {2, 8};
      return rows <= 6144 ? WtShape{4, 8} : WtShape{0, 0};
    case 16:
      if (rows <= 128) return {2, 4};
      if (rows <= 256) return {4, 4};
      return rows <= 2048 ? WtShape{2, 8} : WtShape{0, 0};
    default:
      return rows <= 64 ? WtShape{1, 4} : WtShape{0, 0};
  }
}

size_t wt_work(int64_t rows, int R, int P) {
  size_t total = 0;
  wt::level_of(rows, R, P, round_rank(R), wt::level_count(rows, R, P) - 1, &total);
  return total * sizeof(double);
}

template <int RMAX, int P, int NW>
int wt_launch(int src, int64_t rows, int R, const double* A, int64_t lda, const KrpSrc& krp, double* Q,
              int64_t ldq, double* Rout, int64_t ldr_out, void* work, hipStream_t s) {
  double* w = static_cast<double*>(work);
  const dim3 grd(1), blk(NW * wt::W);
  if (src == SRC_MATRIX)
    hipLaunchKernelGGL((wt::wave_tree_up<RMAX, P, NW, SRC_MATRIX>), grd, blk, 0, s, rows, R, A, lda, krp,
                       Rout, ldr_out, w);
  else
    hipLaunchKernelGGL((wt::wave_tree_up<RMAX, P, NW, SRC_KRP>), grd, blk, 0, s, rows, R, A, lda, krp,
                       Rout, ldr_out, w);
  CPQR_TRY(check_launch("wave_tree_up"));
  hipLaunchKernelGGL((wt::wave_tree_down<RMAX, P, NW>), grd, blk, 0, s, rows, R, Q, ldq, w);
  return check_launch("wave_tree_down");
}

int wt_run(const WtShape& sh, int src, int64_t rows, int R, const double* A, int64_t lda, const KrpSrc& krp,
           double* Q, int64_t ldq, double* Rout, int64_t ldr_out, void* work, hipStream_t s) {
  const int RM = round_rank(R);
  if (RM == 8 && sh.P == 2) return wt_launch<8, 2, 8>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
  if (RM == 8) return wt_launch<8, 4, 8>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
  if (RM == 16 && sh.NW == 8) return wt_launch<16, 2, 8>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
  if (RM == 16 && sh.P == 2) return wt_launch<16, 2, 4>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
  if (RM == 16) return wt_launch<16, 4, 4>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
  return wt_launch<32, 1, 4>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
}

int tsqr_dispatch(int src, int64_t rows, int R, const double* A, int64_t lda, const KrpSrc& krp,
                  double* Q, int64_t ldq, double* Rout, int64_t ldr_out, void* work, hipStream_t s) {
  const WtShape sh = wt_shape(rows, R);
  if (sh.P > 0) return wt_run(sh, src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
  switch (round_rank(R)) {
    case 8: return tsqr_run<8>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
    case 16: return tsqr_run<16>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
    default: return tsqr_run<32>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
  }
}

}  // namespace

size_t tsqr_work(int64_t rows, int R) {
  const int RM = round_rank(R);
  Carver cv(nullptr);
  const WtShape sh = wt_shape(rows, R);
  if (sh.P > 0) return wt_work(rows, R, sh.P);
  Tree t = make_tree(rows, R, RM);
  return carve_tree(cv, t, RM);
}

int factor_qr_enqueue(int64_t I, int R, const double* A, int64_t lda, double* Q, int64_t ldq,
                      double* Rk, int64_t ldr, void* work, hipStream_t s) {
  PhaseTimer pt(PH_FACTOR_QR, s);
  KrpSrc none{};
  return tsqr_dispatch(SRC_MATRIX, I, R, A, lda, none, Q, ldq, Rk, ldr, work, s);
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
