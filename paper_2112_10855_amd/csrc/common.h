// Internal helpers shared by the libcpqr sources: error reporting, HIP
// status checks, scratch carving, launch-shape helpers and the declarations
// of each translation unit's enqueue functions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/cpqr.h"

namespace cpqr {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define CPQR_HIP(expr)                                                               \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::cpqr::fail(CPQR_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CPQR_TRY(expr)              \
  do {                              \
    int rc_ = (expr);               \
    if (rc_ != CPQR_OK) return rc_; \
  } while (0)

// Launch status right after a kernel launch.
int check_launch(const char* what);

// ---------------------------------------------------------------- scratch
// Carves 256-byte aligned pieces from a caller buffer.  With base == nullptr
// it only measures.
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
  size_t bytes() const { return (used + 255) & ~size_t(255); }
};

int check_work(void* work, size_t have, size_t need);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int round_rank(int R) { return R <= 8 ? 8 : (R <= 16 ? 16 : 32); }
inline int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// ---------------------------------------------------------------- timing
enum Phase { PH_MULTITTM = 0, PH_TTM_FIRST = 1, PH_FACTOR_QR = 2, PH_Q0 = 3, PH_APPLY_Q0 = 4,
             PH_SOLVE = 5, PH_ERROR = 6, PH_TTM_STREAM_M = 7 };
// Events attached to one kernel dispatch (hipExtLaunchKernelGGL), so that
// timing a kernel adds no packets of its own to the stream; both null when
// the phase is not being timed.
struct KernelEvents {
  int phase = -1;
  hipEvent_t a = nullptr, b = nullptr;
};
KernelEvents kernel_events(int phase, hipStream_t s);
void kernel_events_done(const KernelEvents& ke);

// Scoped phase timer: records an event pair on `stream` when timing is on.
struct PhaseTimer {
  int phase;
  hipStream_t stream;
  hipEvent_t ev0 = nullptr;
  PhaseTimer(int ph, hipStream_t s);
  ~PhaseTimer();
};

// ---------------------------------------------------------------- pieces
// Each returns CPQR_OK or an error code; arguments are validated by callers.

// tsqr.hip
size_t tsqr_work(int64_t rows, int R);
int factor_qr_enqueue(int64_t I, int R, const double* A, int64_t lda, double* Q, int64_t ldq,
                      double* Rk, int64_t ldr, void* work, hipStream_t s,
                      hipEvent_t r_ready = nullptr);
int krp_qr_enqueue(int N, int n, int R, const double* const* Rk, int64_t ldr, double* Q0,
                   double* R0, void* work, hipStream_t s);
// Whether the factor QR of I x R takes a single workgroup (then the column
// normalization can be fused into it).
bool norm_qr_fits(int64_t I, int R);
// Column normalization (lambda, A scaled in place, zero-column status) and
// factor QR of A (leading dimensions I, I and R) in one launch; *fused is
// false (and nothing is enqueued) when norm_qr_fits(I, R) does not hold.
// urows / uquads (optional, round_rank(R) must equal the column padding RP):
// FP32 copies of Q in the layouts of the FP32 contraction kernels (see UCache).
int normalize_factor_qr_enqueue(int64_t I, int R, double* A, double* lambda, int* status, double* Q, double* Rk,
                                void* work, hipStream_t s, hipEvent_t r_ready, bool* fused,
                                float* urows = nullptr, float* uquads = nullptr, int RP = 0);

// multittm.hip
// FP32 contraction operands already prepared from the factor Q's: rows[k] is
// I_k x RP row-major, U[i RP + r] = Q_k(i, r); quads[k] interleaves four rows,
// U4[((i/4) RP + r) 4 + i%4] = Q_k(i, r); zero for r >= R.  A null entry is
// prepared from Q_k by the Multi-TTM itself.  Used by FP32 and bfloat16
// Multi-TTMs with padding RP only.
struct UCache {
  int RP = 0;
  const float* rows[CPQR_MAX_MODES] = {};
  const float* quads[CPQR_MAX_MODES] = {};
};
size_t multittm_work(int N, const int64_t* I, int n, int R, int prec);
// Contract the modes in cmask (bit k = mode k) of a tensor with sizes I (modes
// already contracted have size R and are left alone); write the result in its
// natural column-major layout (n_unfold < 0) or unfolded along n_unfold as
// Y_(n) (columns: lowest remaining mode fastest).  streams_tensor marks calls
// whose first contraction reads the input tensor (for the phase timers).
size_t multittm_general_work(int N, const int64_t* I, unsigned cmask, int R, int prec);
int multittm_general_enqueue(int N, const int64_t* I, int xdtype, const void* X, unsigned cmask, int n_unfold,
                             int R, const double* const* Q, int prec, void* Y, void* work, hipStream_t st,
                             bool streams_tensor, const UCache* uc = nullptr);
int multittm_enqueue(int N, const int64_t* I, int xdtype, const void* X, int n, int R,
                     const double* const* Q, int prec, void* Y, void* work, hipStream_t s,
                     const UCache* uc = nullptr);

// small.hip
size_t apply_q0_work(int64_t In, int64_t K, int R);
int apply_q0_enqueue(int64_t In, int64_t K, int R, int ydtype, const void* Y, const double* Q0,
                     double* W, void* work, hipStream_t s);
// W = Y_(n) Q_0, then A = W R0^-T with columns normalized into lambda; the
// triangular solve sums the split partials of W itself (work: apply_q0_work).
int apply_solve_enqueue(int64_t In, int64_t K, int R, int ydtype, const void* Y, const double* Q0,
                        const double* R0, int use_svd, double rtol, double* W, double* A, double* lambda,
                        int* status, void* work, hipStream_t s, bool normalize = true);
size_t solve_work(int64_t In, int R);
int solve_enqueue(int64_t In, int R, const double* W, const double* R0, int use_svd, double rtol,
                  double* A, double* lambda, int* status, void* work, hipStream_t s, bool normalize = true);
size_t fit_direct_work(int N, const int64_t* I, int R);
int fit_direct_enqueue(int N, const int64_t* I, int xdtype, const void* X, int R,
                       const double* lambda, const double* const* A, double* out, void* work,
                       hipStream_t s);
// ||X||^2 into out[0] (device double)
size_t norm2_work(int64_t count);
int norm2_enqueue(int64_t count, int xdtype, const void* X, double* out, void* work, hipStream_t s);
// efficient relative error into *relerr (device): section 3.3.1
// ip partial sums per 256 rows and nn go to part (error_efficient_work bytes).
size_t error_efficient_work(int64_t In);
int error_efficient_enqueue(int64_t In, int R, const double* W, const double* A,
                            const double* lambda, const double* R0, const double* RN,
                            const double* xnorm2, double* relerr, double* part, hipStream_t s);
// Q_0 (R^{N-1} x R) formed from the factors of the structured QR of V_n
// (Qc: Q_2 .. Q_{N-1}, each R^2 x R); buf holds 2 R^{N-1} R doubles (N >= 5)
int expand_q0_enqueue(int N, int R, const double* Qc, double* Q0, double* buf, hipStream_t s);
// Q_0 = (Q_a kron I_R) Q_b (both R^2 x R, column-major), Q_0 R^3 x R.
int expand_kron_right_enqueue(int R, const double* Qa, const double* Qb, double* Q0, hipStream_t s);
// W (In x R, FP64) = the columns of Y_(n) (In x R^{N-1}) whose every Kronecker
// index is r (the MTTKRP part of a Multi-TTM)
int diag_cols_enqueue(int64_t In, int N, int R, int ydtype, const void* Y, double* W, hipStream_t s);
// relerr = sqrt(max(out[0],0) / out[1]) from a fit_direct result
int error_from_fit_enqueue(const double* fit, double* relerr, hipStream_t s);
int fill_enqueue(double* p, int64_t count, double v, hipStream_t s);
// Alg. 1 (CP-ALS, normal equations): G = A^T A; one mode update from the
// unfolded Multi-TTM Y_(n) of the factors themselves (MTTKRP = its diagonal
// columns), the Gram matrices G (N blocks of R x R; block n is rewritten),
// S = their Hadamard product over k != n, F = its Cholesky factor or
// pseudo-inverse, M = the MTTKRP (In x R), A and lambda the new factor.
int gram_enqueue(int64_t In, int R, const double* A, double* G, hipStream_t s);
size_t ne_update_work(int R);
int ne_update_enqueue(int64_t In, int N, int n, int R, int ydtype, const void* Y, double* G, int pinv,
                      double rtol, double* S, double* F, double* M, double* A, double* lambda, int* status,
                      void* work, hipStream_t s);
size_t ne_error_work(int64_t In);
int ne_error_enqueue(int64_t In, int R, const double* M, const double* A, const double* lambda, const double* S,
                     const double* GN, const double* xnorm2, double* relerr, double* part, hipStream_t s);

// kruskal.hip: Kruskal-form input (section 3.3.2)
// P = U^T V (R x S) for U: I x R (ldu), V: I x S (ldv)
int kr_cross_enqueue(int64_t I, int R, int S, const double* U, int64_t ldu, const double* V, int64_t ldv,
                     double* P, hipStream_t s);
// M (S x R) = rows c_{nP-1}(s)^T of the chain c_1 = P[0](:, s),
// c_j = Q_j^T (P[j-1](:, s) (x) c_{j-1}); Qc as written by krp_chain_enqueue
int kr_chain_enqueue(int nP, const double* const* P, const double* Qc, int R, int S, double* M, hipStream_t s);
// H (S x R) = Hadamard product of the P's (each R x S), transposed
int kr_hadamard_enqueue(int nP, const double* const* P, int R, int S, double* H, hipStream_t s);
// W (I x R) = V diag(mu) M, V: I x S (ldv), M: S x R
int kr_w_enqueue(int64_t I, int S, int R, const double* V, int64_t ldv, const double* mu, const double* M,
                 double* W, hipStream_t s);
size_t kr_norm2_work(int S);
int kr_norm2_enqueue(int N, const int64_t* I, int S, const double* mu, const double* const* V, double* out,
                     void* work, hipStream_t s);
size_t kr_full_work(int N, const int64_t* I, int S);
// grid rows of the dense product (must stay <= 65535 for a launch)
int64_t kr_full_grid_y(int N, const int64_t* I);
int kr_full_enqueue(int N, const int64_t* I, int S, const double* mu, const double* const* V, int xdtype,
                    void* X, void* work, hipStream_t s);
// Alg. 1 update from a formed MTTKRP Mn (In x R, FP64)
int ne_update_from_m_enqueue(int64_t In, int N, int n, int R, const double* Mn, double* G, int pinv, double rtol,
                             double* S, double* F, double* M, double* A, double* lambda, int* status, void* work,
                             hipStream_t s);

}  // namespace cpqr
