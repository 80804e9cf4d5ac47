// Tall-skinny Householder QR for gfx950, used for the factor QRs A_k = Q_k R_k
// and for the QR of the Khatri-Rao product of triangular factors
// V_n = Q_0 R_0 (paper section 3.1, Alg. 2), both with the orthonormal
// factor formed explicitly.
//
// Design.  One wavefront (64 lanes) owns one block of at most 64 rows; lane
// l holds row l of the block in registers (R <= 32 doubles).  A block is
// factorized with Householder reflections whose column norms and
// reflector-times-matrix products are wavefront reductions, so no barrier is
// needed inside a block.  Blocks are combined in a tree: the triangular
// factors of up to 64/R children are stacked and factorized again, level by
// level, until one block remains (its R is the answer).  Q is then formed top
// down: each node applies its reflectors to [C; 0], where C is the node's
// R x R slice of its parent's Q, and hands R x R slices to its children.
// Every step is a genuine Householder reflection of the real rows (rows past
// a block's end are never touched), so Q has orthonormal columns even when
// the input is rank deficient.

#include "common.h"

namespace cpqr {
namespace {

constexpr int WAVE = 64;
constexpr int WPB = 4;  // wavefronts per workgroup; each owns one tree node

enum Src { SRC_MATRIX = 0, SRC_KRP = 1, SRC_STACK = 2 };

struct KrpSrc {
  const double* Rk[CPQR_MAX_MODES];
  int modes[CPQR_MAX_MODES];  // the N-1 modes k != n, ascending (lowest fastest)
  int nm;
  int64_t ldr;
};

struct Level {
  int64_t nodes;      // nodes at this level
  int64_t rows;       // leaves: rows of the input; else unused
  int64_t prev_nodes; // internal levels: nodes of the level below
  int g;              // internal levels: children per node
  double* V;          // nodes x RMAX x 64 (column c of node j at (j*RMAX + c)*64)
  double* tau;        // nodes x RMAX
  double* Rin;        // internal levels: prev_nodes blocks of RMAX x RMAX (stacked R's)
};

__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, WAVE);
  return x;
}

// Orders LDS writes by some lanes before reads by others within one
// wavefront.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Balanced leaf partition: leaf b of nl covering `rows` rows.
__device__ __host__ inline void leaf_range(int64_t rows, int64_t nl, int64_t b, int64_t& start,
                                           int& m) {
  int64_t base = rows / nl, rem = rows % nl;
  m = int(base + (b < rem ? 1 : 0));
  start = b * base + (b < rem ? b : rem);
}

// Householder QR of the wavefront's block (rows in a[], one per lane,
// lanes >= m hold zeros).  On return lanes < R hold R's rows (entries at
// c >= lane), lanes > j hold reflector j below the diagonal in a[j], and
// tau_s[j] holds the reflector scalars (H_j = I - tau_j v_j v_j^T, v_j(j)=1).
template <int RMAX>
__device__ void house_factor(double (&a)[RMAX], double* tau_s, int m, int R, int lane) {
#pragma unroll
  for (int j = 0; j < RMAX; ++j) {
    if (j < R) {
    const double aj = a[j];
    const double alpha = __shfl(aj, j, WAVE);
    const double below = (lane > j && lane < m) ? aj : 0.0;
    const double sub2 = wave_sum(below * below);
    double t = 0.0, beta = alpha, scal = 0.0;
    if (sub2 > 0.0) {
      const double nrm = sqrt(alpha * alpha + sub2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    const double v = (lane == j) ? 1.0 : ((lane > j && lane < m) ? aj * scal : 0.0);
    a[j] = (lane == j) ? beta : ((lane > j) ? v : aj);
    if (lane == 0) tau_s[j] = t;
    if (t != 0.0) {
#pragma unroll
      for (int c = j + 1; c < RMAX; ++c) {
        if (c < R) {
          const double w = wave_sum(v * a[c]);
          a[c] -= t * v * w;
        }
      }
    }
    }
  }
}

// q <- H_0 H_1 ... H_{R-1} q for the block's reflectors (held as in
// house_factor's output a[]).  q enters as [C; 0] and leaves as the block's
// rows of the orthonormal factor.
template <int RMAX>
__device__ void house_apply_q(const double (&a)[RMAX], const double* tau_s, double (&q)[RMAX],
                              int m, int R, int lane) {
#pragma unroll
  for (int j = RMAX - 1; j >= 0; --j) {
    const double t = j < R ? tau_s[j] : 0.0;
    if (t != 0.0) {
      const double v = (lane == j) ? 1.0 : ((lane > j && lane < m) ? a[j] : 0.0);
#pragma unroll
      for (int c = 0; c < RMAX; ++c) {
        if (c < R) {
          const double w = wave_sum(v * q[c]);
          q[c] -= t * v * w;
        }
      }
    }
  }
}

template <int RMAX>
__device__ inline void store_block(double* V, int64_t node, const double (&a)[RMAX], int lane) {
#pragma unroll
  for (int c = 0; c < RMAX; ++c) V[(node * RMAX + c) * WAVE + lane] = a[c];
}

template <int RMAX>
__device__ inline void load_block(const double* V, int64_t node, double (&a)[RMAX], int lane) {
#pragma unroll
  for (int c = 0; c < RMAX; ++c) a[c] = V[(node * RMAX + c) * WAVE + lane];
}

// Rows of the node's input block.
template <int RMAX, int SRC>
__device__ inline int load_rows(double (&a)[RMAX], const Level& L, int64_t node, int R, int lane,
                                const double* A, int64_t lda, const KrpSrc& krp,
                                int64_t& start) {
  int m;
  if (SRC == SRC_STACK) {
    const int64_t c0 = node * L.g;
    const int64_t nch = min<int64_t>(L.g, L.prev_nodes - c0);
    m = int(nch) * R;
    start = 0;
    const int child = lane / R, i = lane % R;
#pragma unroll
    for (int c = 0; c < RMAX; ++c)
      a[c] = (lane < m && c < R) ? L.Rin[((c0 + child) * RMAX + c) * RMAX + i] : 0.0;
  } else {
    leaf_range(L.rows, L.nodes, node, start, m);
    const int64_t g = start + lane;
    if (SRC == SRC_MATRIX) {
#pragma unroll
      for (int c = 0; c < RMAX; ++c) a[c] = (lane < m && c < R) ? A[g + c * lda] : 0.0;
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
        double p = (lane < m && c < R) ? 1.0 : 0.0;
#pragma unroll
        for (int t = 0; t < CPQR_MAX_MODES; ++t)
          if (t < krp.nm && lane < m && c < R) p *= krp.Rk[t][digit[t] + c * krp.ldr];
        a[c] = p;
      }
    }
  }
  return m;
}

// Write a formed Q block: to the output matrix (leaves) or as the R x R
// C blocks of the node's children (internal nodes).
template <int RMAX>
__device__ inline void write_q(const double (&q)[RMAX], bool leaf, int64_t start, int m,
                               double* Qout, int64_t ldq, double* Cchild, int64_t node, int g,
                               int R, int lane) {
  if (lane >= m) return;
  if (leaf) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c)
      if (c < R) Qout[start + lane + c * ldq] = q[c];
  } else {
    const int64_t child = node * g + lane / R;
    const int i = lane % R;
#pragma unroll
    for (int c = 0; c < RMAX; ++c)
      if (c < R) Cchild[(child * RMAX + c) * RMAX + i] = q[c];
  }
}

// Up-sweep of one level.  At the root (nodes == 1) also writes R to Rout and
// forms the root's Q from C = I.
template <int RMAX, int SRC>
__global__ __launch_bounds__(WAVE* WPB) void tsqr_up(Level L, int R, const double* A, int64_t lda,
                                                     KrpSrc krp, double* Rnext, double* Rout,
                                                     int64_t ldr_out, double* Qout, int64_t ldq,
                                                     double* Cchild, int gchild) {
  __shared__ double tau_s[WPB][RMAX];
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int64_t node = int64_t(blockIdx.x) * WPB + w;
  if (node >= L.nodes) return;
  double a[RMAX];
  int64_t start;
  const int m = load_rows<RMAX, SRC>(a, L, node, R, lane, A, lda, krp, start);
  house_factor<RMAX>(a, tau_s[w], m, R, lane);
  wave_sync();
  store_block<RMAX>(L.V, node, a, lane);
  if (lane < RMAX) L.tau[node * RMAX + lane] = lane < R ? tau_s[w][lane] : 0.0;
  if (L.nodes > 1) {
    if (lane < R) {
#pragma unroll
      for (int c = 0; c < RMAX; ++c) Rnext[(node * RMAX + c) * RMAX + lane] = (c >= lane) ? a[c] : 0.0;
    }
    return;
  }
  // root
  if (lane < R) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c)
      if (c < R) Rout[lane + c * ldr_out] = (c >= lane) ? a[c] : 0.0;
  }
  double q[RMAX];
#pragma unroll
  for (int c = 0; c < RMAX; ++c) q[c] = (lane < R && c == lane) ? 1.0 : 0.0;
  house_apply_q<RMAX>(a, tau_s[w], q, m, R, lane);
  write_q<RMAX>(q, SRC != SRC_STACK, start, m, Qout, ldq, Cchild, node, gchild, R, lane);
}

// Down-sweep of one non-root level: form each node's Q from its C block.
template <int RMAX, bool LEAF>
__global__ __launch_bounds__(WAVE* WPB) void tsqr_down(Level L, int R, const double* Cin,
                                                       double* Qout, int64_t ldq, double* Cchild,
                                                       int gchild) {
  __shared__ double tau_s[WPB][RMAX];
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int64_t node = int64_t(blockIdx.x) * WPB + w;
  if (node >= L.nodes) return;
  double a[RMAX], q[RMAX];
  load_block<RMAX>(L.V, node, a, lane);
  if (lane < RMAX) tau_s[w][lane] = L.tau[node * RMAX + lane];
  wave_sync();
  int m;
  int64_t start = 0;
  if (LEAF) {
    leaf_range(L.rows, L.nodes, node, start, m);
  } else {
    const int64_t c0 = node * L.g;
    m = int(min<int64_t>(L.g, L.prev_nodes - c0)) * R;
  }
#pragma unroll
  for (int c = 0; c < RMAX; ++c)
    q[c] = (lane < R && c < R) ? Cin[(node * RMAX + c) * RMAX + lane] : 0.0;
  house_apply_q<RMAX>(a, tau_s[w], q, m, R, lane);
  write_q<RMAX>(q, LEAF, start, m, Qout, ldq, Cchild, node, gchild, R, lane);
}

// Tree shape for `rows` input rows at rank R.
struct Tree {
  int nlev = 0;
  int64_t nodes[40];
  int g = 2;
};

Tree make_tree(int64_t rows, int R) {
  Tree t;
  t.g = std::max(2, WAVE / R);
  int64_t n = rows <= WAVE ? 1 : ceil_div(rows, WAVE);
  t.nodes[t.nlev++] = n;
  while (n > 1) {
    n = ceil_div(n, t.g);
    t.nodes[t.nlev++] = n;
  }
  return t;
}

size_t tsqr_carve(Carver& cv, const Tree& t, int RM, Level* lev) {
  for (int l = 0; l < t.nlev; ++l) {
    Level L{};
    L.nodes = t.nodes[l];
    L.V = cv.take<double>(size_t(L.nodes) * RM * WAVE);
    L.tau = cv.take<double>(size_t(L.nodes) * RM);
    if (l > 0) {
      L.prev_nodes = t.nodes[l - 1];
      L.g = t.g;
      L.Rin = cv.take<double>(size_t(L.prev_nodes) * RM * RM);
    }
    if (lev) lev[l] = L;
  }
  return cv.bytes();
}

template <int RMAX, int SRC>
int tsqr_run(int64_t rows, int R, const double* A, int64_t lda, const KrpSrc& krp, double* Q,
             int64_t ldq, double* Rout, int64_t ldr_out, void* work, hipStream_t s) {
  Tree t = make_tree(rows, R);
  Level lev[40];
  Carver cv(work);
  tsqr_carve(cv, t, RMAX, lev);
  lev[0].rows = rows;
  const dim3 blk(WAVE * WPB);
  // up-sweep
  for (int l = 0; l < t.nlev; ++l) {
    const dim3 grd(unsigned(ceil_div(lev[l].nodes, WPB)));
    double* Rnext = (l + 1 < t.nlev) ? lev[l + 1].Rin : nullptr;
    double* Cchild = l > 0 ? lev[l].Rin : nullptr;
    if (l == 0)
      hipLaunchKernelGGL((tsqr_up<RMAX, SRC>), grd, blk, 0, s, lev[l], R, A, lda, krp, Rnext, Rout,
                         ldr_out, Q, ldq, Cchild, t.g);
    else
      hipLaunchKernelGGL((tsqr_up<RMAX, SRC_STACK>), grd, blk, 0, s, lev[l], R, A, lda, krp, Rnext,
                         Rout, ldr_out, Q, ldq, Cchild, t.g);
    CPQR_TRY(check_launch("tsqr_up"));
  }
  // down-sweep below the root: level l reads its C blocks from level l+1's Rin
  for (int l = t.nlev - 2; l >= 0; --l) {
    const dim3 grd(unsigned(ceil_div(lev[l].nodes, WPB)));
    const double* Cin = lev[l + 1].Rin;
    if (l == 0)
      hipLaunchKernelGGL((tsqr_down<RMAX, true>), grd, blk, 0, s, lev[l], R, Cin, Q, ldq, nullptr, t.g);
    else
      hipLaunchKernelGGL((tsqr_down<RMAX, false>), grd, blk, 0, s, lev[l], R, Cin, Q, ldq,
                         lev[l].Rin, t.g);
    CPQR_TRY(check_launch("tsqr_down"));
  }
  return CPQR_OK;
}

template <int SRC>
int tsqr_dispatch(int64_t rows, int R, const double* A, int64_t lda, const KrpSrc& krp, double* Q,
                  int64_t ldq, double* Rout, int64_t ldr_out, void* work, hipStream_t s) {
  switch (round_rank(R)) {
    case 8: return tsqr_run<8, SRC>(rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
    case 16: return tsqr_run<16, SRC>(rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
    default: return tsqr_run<32, SRC>(rows, R, A, lda, krp, Q, ldq, Rout, ldr_out, work, s);
  }
}

}  // namespace

size_t tsqr_work(int64_t rows, int R) {
  Tree t = make_tree(rows, R);
  Carver cv(nullptr);
  return tsqr_carve(cv, t, round_rank(R), nullptr);
}

int factor_qr_enqueue(int64_t I, int R, const double* A, int64_t lda, double* Q, int64_t ldq,
                      double* Rk, int64_t ldr, void* work, hipStream_t s) {
  PhaseTimer pt(PH_FACTOR_QR, s);
  KrpSrc none{};
  return tsqr_dispatch<SRC_MATRIX>(I, R, A, lda, none, Q, ldq, Rk, ldr, work, s);
}

int krp_qr_enqueue(int N, int n, int R, const double* const* Rk, int64_t ldr, double* Q0,
                   double* R0, void* work, hipStream_t s) {
  PhaseTimer pt(PH_Q0, s);
  KrpSrc krp{};
  krp.nm = 0;
  krp.ldr = ldr;
  for (int k = 0; k < N; ++k) {
    if (k == n) continue;
    krp.Rk[krp.nm] = Rk[k];
    krp.modes[krp.nm] = k;
    ++krp.nm;
  }
  const int64_t rows = ipow(R, N - 1);
  return tsqr_dispatch<SRC_KRP>(rows, R, nullptr, 0, krp, Q0, rows, R0, R, work, s);
}

}  // namespace cpqr
