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

int tsqr_dispatch(int src, int64_t rows, int R, const double* A, int64_t lda, const KrpSrc& krp,
                  double* Q, int64_t ldq, double* Rout, int64_t ldr_out, void* work, hipStream_t s) {
  switch (round_rank(R)) {
    case 8: return tsqr_run<8>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
    case 16: return tsqr_run<16>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
    default: return tsqr_run<32>(src, rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
  }
}

}  // namespace

size_t tsqr_work(int64_t rows, int R) {
  const int RM = round_rank(R);
  Tree t = make_tree(rows, R, RM);
  Carver cv(nullptr);
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
