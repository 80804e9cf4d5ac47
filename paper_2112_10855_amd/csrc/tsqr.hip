// Tall-skinny Householder QR for gfx950, used for the factor QRs A_k = Q_k R_k
// and for the QR of the Khatri-Rao product of triangular factors
// V_n = Q_0 R_0 (paper section 3.1, Alg. 2), both with the orthonormal
// factor formed explicitly.
//
// Design: a reduction tree whose every node is one wavefront.  A leaf holds
// up to 64 P rows of the input (P rows per lane); an inner node stacks the R
// factors of up to 64 P / R children.  Each node is factorized by Householder
// reflections held in registers, one in-wave reduction per column, and keeps
// its reflectors in the compact WY form H_0 ... H_{R-1} = I - V T V^T.  The
// up-sweep runs one launch per level (one single-wavefront workgroup per
// node); the root's R is the answer.  The down-sweep forms Q top down: each
// node applies its reflectors to [C; 0], C being its R x R slice of the
// parent's Q (the identity at the root), and hands R x R slices to its
// children.  Every step is a genuine Householder reflection of the real
// rows, so Q has orthonormal columns even when the input is rank deficient.

#include <algorithm>

#include "common.h"

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

// ------------------------------------------------------------ wavefront nodes
// A node holds at most 64 P rows, row 64 p + lane in slot p of the lane.
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
constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

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
// keeps every register-array index a compile-time constant.  Row J and the
// sums are read from the lanes that hold them (readlane), so they arrive in
// scalar registers that every lane reads.
template <int J, int RMAX, int P>
__device__ __forceinline__ void wave_column(double (&a)[P][RMAX], double (&t)[RMAX], int lane, int R) {
  constexpr int SH = 6 - ilog2(RMAX);
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
  const double alpha = rdlane(a[0][J], J), sub2 = rdlane(red, J << SH);
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
  for (int k = 0; k < J; ++k) tg += t[k] * (rdlane(a[0][k], J) + scal * rdlane(red, k << SH));
  t[J] = lane < J ? -tau * tg : (lane == J ? tau : 0.0);
  // trailing columns: A(:, c) -= tau v (v^T A(:, c)), v^T A(:, c) = A(J, c) + scal s_c
#pragma unroll
  for (int c = J + 1; c < RMAX; ++c) {
    if (c < R) {
      const double tw = tau * (rdlane(a[0][c], J) + scal * rdlane(red, c << SH));
#pragma unroll
      for (int s = 0; s < P; ++s) a[s][c] -= tw * v[s];
    }
  }
  a[0][J] = lane == J ? beta : (lane > J ? v[0] : a[0][J]);
#pragma unroll
  for (int s = 1; s < P; ++s) a[s][J] = v[s];
}

template <int J, int RMAX, int P>
struct WaveColumns {
  static __device__ __forceinline__ void run(double (&a)[P][RMAX], double (&t)[RMAX], int lane, int R) {
    if (J >= R) return;
    wave_column<J, RMAX, P>(a, t, lane, R);
    WaveColumns<J + 1, RMAX, P>::run(a, t, lane, R);
  }
};
template <int RMAX, int P>
struct WaveColumns<RMAX, RMAX, P> {
  static __device__ __forceinline__ void run(double (&)[P][RMAX], double (&)[RMAX], int, int) {}
};

// Householder QR of the node block (row 64 p + lane in a[p][.]; rows beyond
// the block and columns >= R are zero).  On return lanes < R of slot 0 hold
// R's rows (entries c >= lane), the rows below column c's diagonal hold
// reflector c's components (v_c(c) = 1 implicitly), and t[] holds row `lane`
// of T (lanes < R).
template <int RMAX, int P>
__device__ __forceinline__ void wave_factor(double (&a)[P][RMAX], double (&t)[RMAX], int lane, int R) {
#pragma unroll
  for (int c = 0; c < RMAX; ++c) t[c] = 0.0;
  WaveColumns<0, RMAX, P>::run(a, t, lane, R);
}

// Component of reflector c in row `row` of the node (from a[slot][c]).
__device__ __forceinline__ double vcomp(double ac, int c, int row) {
  return row == c ? 1.0 : (row > c ? ac : 0.0);
}

// Compact-WY product M = T V1^T C into b.Z, with C (R x R, zero beyond) in
// b.Z on entry; returns row `lane` of C (lanes < R, else zero) in crow[].
// Every R x R operand is zero-padded to RMAX, so the products run over fixed
// trip counts.
template <int RMAX>
__device__ __forceinline__ void wave_m(const double* Vl, const double (&t)[RMAX], double (&crow)[RMAX],
                                       int lane, int R, Buf<RMAX>& b) {
  constexpr int NE = (RMAX * RMAX + W - 1) / W;
  if (lane < RMAX) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
      b.X[lane][c] = (lane < R && c < R) ? vcomp(Vl[c * W + lane], c, lane) : 0.0;
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

// Row 64 s + lane of the node's Q: [C; 0](row) - v(row) M, with M in b.Z
// and the node's reflectors in Vl ([p][c][lane]).
template <int RMAX>
__device__ __forceinline__ void wave_q_row(const double* Vl, const double (&crow)[RMAX], int s,
                                           double (&q)[RMAX], int lane, int R, const Buf<RMAX>& b) {
  const int row = s * W + lane;
#pragma unroll
  for (int c = 0; c < RMAX; ++c) q[c] = s == 0 ? crow[c] : 0.0;
#pragma unroll 4
  for (int k = 0; k < R; ++k) {
    const double vk = vcomp(Vl[(s * RMAX + k) * W + lane], k, row);
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
__device__ __forceinline__ void store_q(const double* Vl, const double (&crow)[RMAX], int lane, int R,
                               int m, bool leaf, int64_t start, double* Qout, int64_t ldq, double* S,
                               int64_t c0, const Buf<RMAX>& b) {
#pragma unroll
  for (int s = 0; s < P; ++s) {
    double q[RMAX];
    wave_q_row<RMAX>(Vl, crow, s, q, lane, R, b);
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

// Up-sweep below the root, one launch per level, one node per
// single-wavefront workgroup: factorize the node, save its reflectors and T,
// pass its R up.
template <int RMAX, int P, int SRC>
__global__ __launch_bounds__(W) void wave_tree_up(int64_t rows, int R, int l, const double* A, int64_t lda,
                                                  KrpSrc krp, double* work) {
  const int lane = threadIdx.x, node = blockIdx.x;
  const int g = W * P / R;
  const NodeLevel L = level_of(rows, R, P, RMAX, l, nullptr);
  double a[P][RMAX], t[RMAX];
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
  wave_factor<RMAX, P>(a, t, lane, R);
  double* V = work + L.v + int64_t(node) * P * RMAX * W;
#pragma unroll
  for (int s = 0; s < P; ++s)
#pragma unroll
    for (int c = 0; c < RMAX; ++c) V[(s * RMAX + c) * W + lane] = a[s][c];
  if (lane < R) {
    double* T = work + L.t + int64_t(node) * RMAX * RMAX;
    double* Snext = work + level_of(rows, R, P, RMAX, l + 1, nullptr).s;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
      T[lane * RMAX + c] = t[c];
      Snext[(int64_t(node) * RMAX + lane) * RMAX + c] = c >= lane ? a[0][c] : 0.0;
    }
  }
}

// The root (one workgroup): factorize, write R, and form the root's Q from
// C = I straight away: the output itself when the root is the only leaf,
// else the C blocks of its children.
template <int RMAX, int P, int SRC>
__global__ __launch_bounds__(W) void wave_tree_root(int64_t rows, int R, const double* A, int64_t lda,
                                                    KrpSrc krp, double* Qout, int64_t ldq, double* Rout,
                                                    int64_t ldr, double* work) {
  __shared__ Buf<RMAX> b;
  __shared__ double Vl[P * RMAX * W];
  const int lane = threadIdx.x;
  const int top = level_count(rows, R, P) - 1;
  const NodeLevel L = level_of(rows, R, P, RMAX, top, nullptr);
  double t[RMAX], crow[RMAX];
  int m;
  int64_t start = 0;
  {
    double a[P][RMAX];
    if (top == 0) {
      leaf_range(rows, 1, 0, start, m);
      load_leaf<RMAX, P, SRC>(a, lane, start, m, R, A, lda, krp);
    } else {
      m = L.prev * R;
      load_stack<RMAX, P>(a, lane, m, R, work + L.s, 0);
    }
    wave_factor<RMAX, P>(a, t, lane, R);
    if (lane < R) {
#pragma unroll
      for (int c = 0; c < RMAX; ++c)
        if (c < R) Rout[lane + c * ldr] = c >= lane ? a[0][c] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < P; ++s)
#pragma unroll
      for (int c = 0; c < RMAX; ++c) Vl[(s * RMAX + c) * W + lane] = a[s][c];
  }
  for (int e = lane; e < RMAX * RMAX; e += W) {
    const int i = e / RMAX, c = e % RMAX;
    b.Z[i][c] = (i < R && i == c) ? 1.0 : 0.0;
  }
  wave_sync();
  wave_m<RMAX>(Vl, t, crow, lane, R, b);
  store_q<RMAX, P>(Vl, crow, lane, R, m, top == 0, start, Qout, ldq, work + L.s, 0, b);
}

// Down-sweep below the root, one launch per level: each node applies its
// reflectors to its C block and writes its Q rows: the output, or its
// children's C blocks.
template <int RMAX, int P>
__global__ __launch_bounds__(W) void wave_tree_down(int64_t rows, int R, int l, double* Qout, int64_t ldq,
                                                    double* work) {
  __shared__ Buf<RMAX> b;
  __shared__ double Vl[P * RMAX * W];
  const int lane = threadIdx.x, node = blockIdx.x;
  const int g = W * P / R;
  const NodeLevel L = level_of(rows, R, P, RMAX, l, nullptr);
  const double* Cin = work + level_of(rows, R, P, RMAX, l + 1, nullptr).s;
  double t[RMAX], crow[RMAX];
  const double* V = work + L.v + int64_t(node) * P * RMAX * W;
  const double* T = work + L.t + int64_t(node) * RMAX * RMAX;
#pragma unroll 8
  for (int e = lane; e < P * RMAX * W; e += W) Vl[e] = V[e];
#pragma unroll
  for (int c = 0; c < RMAX; ++c) t[c] = lane < R ? T[lane * RMAX + c] : 0.0;
  for (int e = lane; e < RMAX * RMAX; e += W) {
    const int i = e / RMAX, c = e % RMAX;
    b.Z[i][c] = (i >= R || c >= R) ? 0.0 : Cin[int64_t(node) * RMAX * RMAX + e];
  }
  wave_sync();
  wave_m<RMAX>(Vl, t, crow, lane, R, b);
  int m;
  int64_t start = 0, c0 = 0;
  if (l == 0) {
    leaf_range(rows, L.nodes, node, start, m);
  } else {
    c0 = int64_t(node) * g;
    m = int(min<int64_t>(g, L.prev - c0)) * R;
  }
  store_q<RMAX, P>(Vl, crow, lane, R, m, l == 0, start, Qout, ldq, work + L.s, c0, b);
}

}  // namespace wt

// ------------------------------------------------------------ host side
// Rows per lane: 1 at R > 16 (registers); otherwise 2 or 4, whichever gives
// fewer levels, 2 on a tie (measured on MI355X: fewer, fatter levels win,
// and at equal depth the lighter nodes do).
int wt_rows_per_lane(int64_t rows, int R) {
  if (round_rank(R) > 16) return 1;
  return wt::level_count(rows, R, 4) < wt::level_count(rows, R, 2) ? 4 : 2;
}

size_t wt_work(int64_t rows, int R, int P) {
  size_t total = 0;
  wt::level_of(rows, R, P, round_rank(R), wt::level_count(rows, R, P) - 1, &total);
  return total * sizeof(double);
}

template <int RMAX, int P>
int wt_launch(int src, int64_t rows, int R, const double* A, int64_t lda, const KrpSrc& krp, double* Q,
              int64_t ldq, double* Rout, int64_t ldr_out, void* work, hipStream_t s, hipEvent_t r_ready) {
  double* w = static_cast<double*>(work);
  const int nlev = wt::level_count(rows, R, P);
  for (int l = 0; l + 1 < nlev; ++l) {
    const dim3 grd(unsigned(wt::level_of(rows, R, P, RMAX, l, nullptr).nodes)), blk(wt::W);
    if (src == SRC_MATRIX)
      hipLaunchKernelGGL((wt::wave_tree_up<RMAX, P, SRC_MATRIX>), grd, blk, 0, s, rows, R, l, A, lda, krp, w);
    else
      hipLaunchKernelGGL((wt::wave_tree_up<RMAX, P, SRC_KRP>), grd, blk, 0, s, rows, R, l, A, lda, krp, w);
    CPQR_TRY(check_launch("wave_tree_up"));
  }
  if (src == SRC_MATRIX)
    hipLaunchKernelGGL((wt::wave_tree_root<RMAX, P, SRC_MATRIX>), dim3(1), dim3(wt::W), 0, s, rows, R, A, lda,
                       krp, Q, ldq, Rout, ldr_out, w);
  else
    hipLaunchKernelGGL((wt::wave_tree_root<RMAX, P, SRC_KRP>), dim3(1), dim3(wt::W), 0, s, rows, R, A, lda,
                       krp, Q, ldq, Rout, ldr_out, w);
  CPQR_TRY(check_launch("wave_tree_root"));
  if (r_ready) CPQR_HIP(hipEventRecord(r_ready, s));  // R is complete; Q follows
  for (int l = nlev - 2; l >= 0; --l) {
    const dim3 grd(unsigned(wt::level_of(rows, R, P, RMAX, l, nullptr).nodes)), blk(wt::W);
    hipLaunchKernelGGL((wt::wave_tree_down<RMAX, P>), grd, blk, 0, s, rows, R, l, Q, ldq, w);
    CPQR_TRY(check_launch("wave_tree_down"));
  }
  return CPQR_OK;
}

int wt_run(int P, int src, int64_t rows, int R, const double* A, int64_t lda, const KrpSrc& krp, double* Q,
           int64_t ldq, double* Rout, int64_t ldr_out, void* work, hipStream_t s, hipEvent_t r_ready) {
  switch (round_rank(R)) {
    case 8:
      return P == 2 ? wt_launch<8, 2>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s, r_ready)
                    : wt_launch<8, 4>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s, r_ready);
    case 16:
      return P == 2 ? wt_launch<16, 2>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s, r_ready)
                    : wt_launch<16, 4>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s, r_ready);
    default:
      return wt_launch<32, 1>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s, r_ready);
  }
}

int tsqr_dispatch(int src, int64_t rows, int R, const double* A, int64_t lda, const KrpSrc& krp,
                  double* Q, int64_t ldq, double* Rout, int64_t ldr_out, void* work, hipStream_t s,
                  hipEvent_t r_ready = nullptr) {
  return wt_run(wt_rows_per_lane(rows, R), src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s, r_ready);
}

}  // namespace

size_t tsqr_work(int64_t rows, int R) { return wt_work(rows, R, wt_rows_per_lane(rows, R)); }

int factor_qr_enqueue(int64_t I, int R, const double* A, int64_t lda, double* Q, int64_t ldq,
                      double* Rk, int64_t ldr, void* work, hipStream_t s, hipEvent_t r_ready) {
  PhaseTimer pt(PH_FACTOR_QR, s);
  KrpSrc none{};
  return tsqr_dispatch(SRC_MATRIX, I, R, A, lda, none, Q, ldq, Rk, ldr, work, s, r_ready);
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
