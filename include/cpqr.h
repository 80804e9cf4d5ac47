/*
 * cpqr.h -- C ABI of libcpqr, the MI355X (gfx950) hot path of QR-based CP-ALS
 * (CP-ALS-QR and CP-ALS-QR-SVD) from Minster, Viviano, Liu and Ballard,
 * "CP Decomposition for Tensors via Alternating Least Squares with QR
 * Decomposition", arXiv:2112.10855.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named as device pointers are caller-owned device memory on the
 *    current HIP device.  The library never frees or keeps them.  Arrays of
 *    pointers (for example `const double* const* Q`) are HOST arrays whose
 *    elements are device pointers.
 *  - Matrices are column-major with the stated leading dimension.
 *  - A tensor X of sizes I[0..N-1] is stored column-major: mode 1 (I[0])
 *    varies fastest.  This is the layout of a contiguous torch tensor of
 *    shape (I[N-1], ..., I[0]).
 *  - The mode-n unfolding X_(n) (section 2.2) has I[n] rows; its columns
 *    are ordered with the lowest remaining mode fastest.  Y_(n) of the
 *    Multi-TTM has I[n] rows and R^(N-1) columns in that order, which is the
 *    row order of the Khatri-Rao product V_n of the triangular factors.
 *  - Modes are 0-based: paper mode n is `n-1` here.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call only enqueues work on it and returns; no call synchronizes
 *    the device or allocates device memory.
 *  - Scratch memory is caller-provided: each entry point that needs it
 *    takes (work, work_bytes) and has a *_work query returning the bytes it
 *    needs.  work must be 256-byte aligned; it may be NULL when the query
 *    returns 0.  Calls that share one work buffer must be ordered on one
 *    stream.
 *  - Return value: CPQR_OK or a negative CPQR_ERR_* code.  On error nothing
 *    has been enqueued and cpqr_last_error() gives a thread-local message.
 *  - Numerical conditions found on the device are OR-ed into an optional
 *    device int (`status`, may be NULL) as CPQR_STATUS_* bits.
 *
 * Limits: 2 <= N <= CPQR_MAX_MODES, 1 <= R <= CPQR_MAX_RANK, I[k] >= R for
 * every mode of a sweep on a dense tensor (sweeps on a Kruskal-form input and
 * cpqr_factor_qr accept smaller modes).
 */
#ifndef CPQR_H
#define CPQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPQR_MAX_MODES 10
#define CPQR_MAX_RANK 32
#define CPQR_MAX_KRUSKAL_TERMS 65536 /* terms S of a Kruskal-form input tensor */

/* return codes */
#define CPQR_OK 0
#define CPQR_ERR_ARG (-1)         /* null pointer, bad enum, bad count */
#define CPQR_ERR_SHAPE (-2)       /* sizes out of range or inconsistent */
#define CPQR_ERR_DTYPE (-3)       /* dtype / precision combination not offered */
#define CPQR_ERR_WORKSPACE (-4)   /* work buffer missing, small or misaligned */
#define CPQR_ERR_HIP (-5)         /* a HIP runtime call failed */
#define CPQR_ERR_UNSUPPORTED (-6) /* valid request this build does not implement */

/* element types */
#define CPQR_F32 0
#define CPQR_F64 1

/* arithmetic of the Multi-TTM contractions */
#define CPQR_PREC_F64 0    /* FP64 products and sums (X may be F32 or F64) */
#define CPQR_PREC_F32 1    /* FP32 MFMA products, FP32 sums (X must be F32) */
#define CPQR_PREC_BF16X2 2 /* split bfloat16 hi/lo, 3 MFMA products, FP32 sums */
#define CPQR_PREC_BF16 3   /* operands rounded to bfloat16, FP32 sums */

/* status bits OR-ed into the optional device status word */
#define CPQR_STATUS_SINGULAR 1   /* R_0 has a zero or non-finite diagonal (substitution) */
#define CPQR_STATUS_NONFINITE 2  /* a solved factor holds Inf/NaN */
#define CPQR_STATUS_TRUNCATED 4  /* the SVD solve dropped singular values */
#define CPQR_STATUS_ZERO_COLUMN 8 /* a solved factor column has zero norm */
#define CPQR_STATUS_ILL_CONDITIONED 16 /* CP-ALS (Cholesky): cond(S_n) is proven above 1e4 (so
                                          cond(Z_n) > 100): max_j S_jj ||S_n^-1 x|| > 1e4 for a unit x
                                          from four steps of inverse iteration */

/* error forms of section 3.3.1 */
#define CPQR_ERROR_EFFICIENT 0 /* from W_N, R_0, R_N and lambda; accurate to ~sqrt(eps) */
#define CPQR_ERROR_DIRECT 1    /* ||X - [[lambda; A]]|| streamed over X in FP64 */
#define CPQR_ERROR_NONE 2      /* skip the error */

/* Thread-local message for the last failed call on this thread. */
const char* cpqr_last_error(void);

/* ABI version (major*100 + minor). */
int cpqr_version(void);

/*
 * Compact QR of one factor matrix, A = Q R (Alg. 2, the factor QR before
 * the loop and after each mode update).  Householder reflections on the
 * GPU: one workgroup per block of up to 1024 rows, blocks combined in a
 * tall-skinny tree; Q formed explicitly.  Up to 1024 rows take one
 * workgroup and no work buffer.
 *   A   : device, I x R, column-major, lda >= I (read only)
 *   Q   : device, I x R, column-major, ldq >= I (written)
 *   Rk  : device, R x R upper triangular, column-major, ldr >= R (written,
 *         including the zeros below the diagonal)
 * Signs of the diagonal of Rk are not normalized.  I < R is allowed: the
 * result is the QR of A padded with R - I zero rows, so Q's columns I..R-1
 * and Rk's rows I..R-1 are zero (A = Q Rk still holds, and the nonzero
 * columns of Q are orthonormal); a sweep on a Kruskal input uses this for
 * modes smaller than the rank (the 10-way sine of sums, n = 8 < R = 10).
 */
size_t cpqr_factor_qr_work(int64_t I, int R);
int cpqr_factor_qr(int64_t I, int R, const double* A, int64_t lda, double* Q, int64_t ldq,
                   double* Rk, int64_t ldr, void* work, size_t work_bytes, void* stream);

/*
 * Khatri-Rao product of the triangular factors and its QR (section 3.1,
 * eq. Z_qr): V_n = R_N (.) ... (.) R_{n+1} (.) R_{n-1} (.) ... (.) R_1,
 * V_n = Q_0 R_0 with Q_0 explicit.  V_n is generated on the fly.
 *   Rk  : host array of N device pointers; Rk[k] is R x R column-major with
 *         leading dimension ldr; Rk[n] is not read
 *   Q0  : device, R^(N-1) x R, column-major, leading dimension R^(N-1)
 *   R0  : device, R x R upper triangular, column-major, leading dimension R
 */
size_t cpqr_krp_qr_work(int N, int R);
int cpqr_krp_qr(int N, int n, int R, const double* const* Rk, int64_t ldr, double* Q0, double* R0,
                void* work, size_t work_bytes, void* stream);

/*
 * Multi-TTM in every mode except n (section 2.2, eq. multittm; Alg. 2):
 * Y = X x_k Q_k^T for all k != n, returned as the unfolding Y_(n).
 *   I     : host array of N mode sizes
 *   X     : device tensor, column-major, element type xdtype
 *   Q     : host array of N device pointers; Q[k] is I[k] x R column-major
 *           FP64 with leading dimension I[k]; Q[n] is not read
 *   prec  : CPQR_PREC_*.  F32, BF16X2 and BF16 need xdtype == CPQR_F32.
 *   Y     : device, I[n] x R^(N-1) column-major (leading dimension I[n]);
 *           FP64 when prec == CPQR_PREC_F64, otherwise FP32
 * The contractions run largest mode first.  The first one streams X once.
 */
size_t cpqr_multittm_work(int N, const int64_t* I, int n, int R, int prec);
int cpqr_multittm(int N, const int64_t* I, int xdtype, const void* X, int n, int R,
                  const double* const* Q, int prec, void* Y, void* work, size_t work_bytes,
                  void* stream);

/*
 * The same Multi-TTM for callers that cannot allocate device memory or pass
 * a workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the scratch cpqr_multittm takes from `work` comes
 * instead from a static device array of CPQR_NOALLOC_SCRATCH_BYTES that the
 * library holds on every device it runs on until the process ends.  Same
 * arguments, kernels and results as cpqr_multittm.  A request whose
 * cpqr_multittm_work exceeds CPQR_NOALLOC_SCRATCH_BYTES is rejected with
 * CPQR_ERR_WORKSPACE before anything is enqueued.  The first call on a device
 * resolves the array's address there (may return CPQR_ERR_HIP).  Every call
 * on one device shares that array: calls that overlap in time on one device
 * (different streams, or host threads) race and must be ordered by the
 * caller.  No call allocates or frees device memory.
 */
#define CPQR_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int cpqr_multittm_noalloc(int N, const int64_t* I, int xdtype, const void* X, int n, int R,
                          const double* const* Q, int prec, void* Y, void* stream);

/*
 * Structured QR of V_n (section 3.3.3): the Khatri-Rao product of triangular
 * factors is factorized without forming it.  With a_1 < .. < a_{N-1} the
 * modes other than n, T_1 = R_{a_1} and, for j = 2..N-1, the QR
 * R_{a_j} (.) T_{j-1} = Q_j T_j of an R^2 x R Khatri-Rao product of two
 * triangular matrices, eq. (kr-id) gives
 *   V_n = (I kron Q_2)(I kron Q_3) .. (I kron Q_{N-2}) Q_{N-1} T_{N-1},
 * so R_0 = T_{N-1} and Q_0 = the product of the Kronecker-structured factors
 * (orthonormal columns), equal to the dense Q_0, R_0 up to column signs.
 * N - 2 QRs of R^2 x R rows replace one of R^{N-1} x R; Q_0 is never formed.
 * For N = 3 this is the QR of V_n itself.  Requires 3 <= N.
 *   Rk : host array of N device pointers to R x R factors (leading dimension
 *        ldr); Rk[n] is not read
 *   Qc : device, (N-2) blocks of R^2 x R column-major (Q_2 first)
 *   R0 : device, R x R upper triangular (leading dimension R)
 */
size_t cpqr_krp_qr_chain_work(int N, int R);
int cpqr_krp_qr_chain(int N, int n, int R, const double* const* Rk, int64_t ldr, double* Qc, double* R0,
                      void* work, size_t work_bytes, void* stream);

/*
 * Q_0 formed from the factors of cpqr_krp_qr_chain (section 3.3.3, eq. kr-id):
 * Q_0 = (I kron Q_2)(I kron Q_3) .. Q_{N-1}, built from the right, one
 * Kronecker step per factor (2 R^{N+1} flops in the last step).
 *   Qc : device, N - 2 blocks of R^2 x R column-major (as written by
 *        cpqr_krp_qr_chain)
 *   Q0 : device, R^{N-1} x R column-major (leading dimension R^{N-1}), written
 *   work : 2 R^N doubles for N >= 5, none below
 */
size_t cpqr_expand_q0_work(int N, int R);
int cpqr_expand_q0(int N, int R, const double* Qc, double* Q0, void* work, size_t work_bytes, void* stream);

/*
 * Randomized HOSVD start, the fallback of the learned initializer: for each
 * mode k >= k0, A[k] = the Q of the thin QR of W_k = X_(k) (Omega_N (.) ..
 * (.) Omega_{k+1} (.) Omega_{k-1} (.) .. (.) Omega_1), an orthonormal basis
 * of the range of X_(k) sampled by a Khatri-Rao test matrix (the leading-R
 * mode-k singular subspace when X_(k) has rank R).  W_k is the MTTKRP of
 * section 2.3, read off the Multi-TTM with U_j = Omega_j in precision prec.
 *   Omega : host array of N device I[j] x R column-major FP64 test factors
 *           (drawn by the caller, e.g. iid N(0, 1))
 *   A     : host array of N device I[k] x R column-major FP64 outputs
 *           (entries below k0 not read or written); I[k] >= R.
 */
size_t cpqr_hosvd_init_work(int N, const int64_t* I, int R, int prec);
int cpqr_hosvd_init(int N, const int64_t* I, int xdtype, const void* X, int R, const double* const* Omega, int prec,
                    int k0, double* const* A, void* work, size_t work_bytes, void* stream);

/*
 * Kruskal-form input X = [[mu; V_1 .. V_N]] (section 3.3.2).  mu: device, S
 * weights; V: host array of N device pointers to I[k] x S column-major FP64
 * factors (leading dimension I[k]); 1 <= S <= CPQR_MAX_KRUSKAL_TERMS.
 *
 * cpqr_kruskal_w: W = Y_(n) Q_0 for Y = X x_{k != n} Q_k^T, without forming Y
 * or Q_0: with B_k = Q_k^T V_k, W = V_n diag(mu) [(B_{a_{N-1}} (.) .. (.)
 * B_{a_1})^T Q_0], the bracket taken term by term through eq. (kr-id) on the
 * structured factors Qc of cpqr_krp_qr_chain (N >= 3): c_1 = B_{a_1}(:, s),
 * c_j = Q_j^T (B_{a_j}(:, s) (x) c_{j-1}), row s of the bracket = c_{N-1}^T.
 * Q: host array of device I[k] x R orthonormal factors (Q[n] not read);
 * W: device I[n] x R column-major FP64.  (N I R S + (N-2) R^3 S + I_n R S
 * multiply-adds.)
 */
size_t cpqr_kruskal_w_work(int N, int R, int S);
int cpqr_kruskal_w(int N, int n, int R, const int64_t* I, int S, const double* mu, const double* const* V,
                   const double* const* Q, const double* Qc, double* W, void* work, size_t work_bytes,
                   void* stream);

/* MTTKRP of a Kruskal input (section 3.3.2, Alg. 1): M = X_(n) Z_n =
 * V_n diag(mu) (Hadamard product over k != n of V_k^T A_k); A: host array of
 * device I[k] x R factors (A[n] not read); M: device I[n] x R FP64. */
size_t cpqr_kruskal_mttkrp_work(int N, int R, int S);
int cpqr_kruskal_mttkrp(int N, int n, int R, const int64_t* I, int S, const double* mu, const double* const* V,
                        const double* const* A, double* M, void* work, size_t work_bytes, void* stream);

/* ||X||^2 of a Kruskal input: mu^T (Hadamard product of V_k^T V_k) mu, into
 * out[0] (device double); fixed-order sums. */
size_t cpqr_kruskal_norm2_work(int S);
int cpqr_kruskal_norm2(int N, const int64_t* I, int S, const double* mu, const double* const* V, double* out,
                       void* work, size_t work_bytes, void* stream);

/* The dense tensor of a Kruskal input (eq. cp): X column-major (mode 1
 * fastest) in xdtype (CPQR_F64 or CPQR_F32, summed in FP64), as the product
 * of the scaled Khatri-Rao rows of the leading modes and those of the
 * trailing modes.  CPQR_ERR_SHAPE when the trailing modes hold more than
 * 65535 x 64 entries. */
size_t cpqr_kruskal_full_work(int N, const int64_t* I, int S);
int cpqr_kruskal_full(int N, const int64_t* I, int S, const double* mu, const double* const* V, int xdtype,
                      void* X, void* work, size_t work_bytes, void* stream);

/*
 * W = Y_(n) Q_0 with Q_0 in the structured form of cpqr_krp_qr_chain: step
 * j = 2..N-1 contracts the two fastest column digits of the current
 * I_n x (R^2 x R^{N-1-j}) array with Q_j (the first of them is the result of
 * the step before), FP64 results.  Y: device I_n x R^(N-1) column-major,
 * FP32 or FP64 (ydtype); W: device I_n x R column-major FP64.
 */
size_t cpqr_apply_q0_chain_work(int64_t In, int N, int R);
int cpqr_apply_q0_chain(int64_t In, int N, int R, int ydtype, const void* Y, const double* Qc, double* W,
                        void* work, size_t work_bytes, void* stream);

/*
 * Apply Q_0 (Alg. 2, eq. ls-qr-q0-step): W = Y_(n) Q_0 in FP64.
 *   Y   : device, In x K column-major (leading dimension In), ydtype F32/F64
 *   Q0  : device, K x R column-major (leading dimension K)
 *   W   : device, In x R column-major (leading dimension In)
 */
size_t cpqr_apply_q0_work(int64_t In, int64_t K, int R);
int cpqr_apply_q0(int64_t In, int64_t K, int R, int ydtype, const void* Y, const double* Q0,
                  double* W, void* work, size_t work_bytes, void* stream);

/*
 * Solve and normalize (Alg. 2, section 3.1): Ahat R_0^T = W by substitution
 * (use_svd == 0, CP-ALS-QR) or Ahat = W U S^+ V^T from the SVD R_0 = U S V^T
 * (use_svd != 0, CP-ALS-QR-SVD; singular values <= rtol * sigma_max are
 * dropped; rtol < 0 selects R * 2^-52).  Then lambda_r = ||Ahat(:,r)||_2 and
 * A = Ahat diag(lambda)^-1 (a zero column stays zero with lambda_r = 0).
 *   W      : device, In x R column-major (leading dimension In)
 *   R0     : device, R x R upper triangular (leading dimension R)
 *   A      : device, In x R column-major (leading dimension In), written
 *   lambda : device, R doubles, written
 *   status : device int or NULL; CPQR_STATUS_* bits OR-ed in
 */
size_t cpqr_solve_rsvd_work(int64_t In, int R);
int cpqr_solve_rsvd(int64_t In, int R, const double* W, const double* R0, int use_svd, double rtol,
                    double* A, double* lambda, int* status, void* work, size_t work_bytes,
                    void* stream);

/*
 * Direct residual of a Kruskal model (section 3.3.1, the accurate form):
 * out[0] = ||X - [[lambda; A_1..A_N]]||_F^2 and out[1] = ||X||_F^2, both
 * accumulated in FP64.  A is a host array of N device pointers to I[k] x R
 * column-major FP64 factors (leading dimension I[k]); out is device memory.
 */
size_t cpqr_fit_direct_work(int N, const int64_t* I, int R);
int cpqr_fit_direct(int N, const int64_t* I, int xdtype, const void* X, int R, const double* lambda,
                    const double* const* A, double* out, void* work, size_t work_bytes, void* stream);

/*
 * Whole sweeps of CP-ALS-QR / CP-ALS-QR-SVD (Alg. 2): for n = 1..N the
 * Khatri-Rao QR, Multi-TTM, Q_0 application, solve, normalization and
 * factor QR, then the relative error.  The ALS state lives in caller
 * memory described by cpqr_problem; the work buffer also keeps ||X||^2
 * between calls, so pass the same buffer to cpqr_als_init and every
 * cpqr_als_sweep of one problem.
 */
typedef struct cpqr_problem {
  int N;                          /* number of modes */
  int R;                          /* CP rank */
  int64_t I[CPQR_MAX_MODES];      /* mode sizes */
  int xdtype;                     /* CPQR_F32 or CPQR_F64 */
  const void* X;                  /* device tensor, column-major */
  double* A[CPQR_MAX_MODES];      /* device I[k] x R factors (normalized after each update) */
  double* Q[CPQR_MAX_MODES];      /* device I[k] x R orthonormal factors */
  double* Rf[CPQR_MAX_MODES];     /* device R x R triangular factors (leading dimension R) */
  double* lambda;                 /* device, R weights */
  int prec;                       /* CPQR_PREC_* of the Multi-TTM */
  int use_svd;                    /* CP-ALS-QR: 0 substitution, 1 SVD solve;
                                     CP-ALS (cpqr_als_ne_*): 0 Cholesky, 1 pseudo-inverse */
  double rtol;                    /* cutoff of the SVD or pseudo-inverse (negative: default) */
  int error_mode;                 /* CPQR_ERROR_* */
  int* status;                    /* device int or NULL */
  int dimtree;                    /* Multi-TTM reuse across modes: 0 off (one Multi-TTM of X
                                     per mode, as in Alg. 2), h in [1, N-1]: modes 1..h share
                                     X contracted over modes h+1..N and modes h+1..N share X
                                     contracted over modes 1..h (two passes over X per sweep),
                                     -1: the library picks h (off for N = 2) */
  int krp_chain;                  /* structured QR of V_n (cpqr_krp_qr_chain, Q_0 then formed
                                     from its factors) in place of the dense QR of the formed
                                     V_n: 1 on (N >= 3), 0 off, -1 the library picks (on for
                                     N >= 4 once V_n has more than 65536 rows) */
  int xS;                         /* 0: the input is the dense tensor X.  S > 0: the input is
                                     the Kruskal tensor [[xmu; xV[0], .., xV[N-1]]] of S terms
                                     (section 3.3.2): both algorithms work on its factors (the
                                     Multi-TTM and the MTTKRP are never formed densely; Alg. 2
                                     takes Q_0 in the structured form of cpqr_krp_qr_chain,
                                     whatever krp_chain says, and needs no R^{N-1} x R buffer),
                                     prec and dimtree are not used, and X may be NULL; when
                                     given (the same tensor, dense, e.g. from
                                     cpqr_kruskal_full) it is read only by the direct error */
  const double* xmu;              /* device, S weights of the Kruskal input (any sign) */
  const double* xV[CPQR_MAX_MODES]; /* device I[k] x S column-major factors of the Kruskal input
                                     (leading dimension I[k]) */
} cpqr_problem;

size_t cpqr_als_work(const cpqr_problem* p);

/* Alg. 2 set-up: compact QRs of the initial A[1..N-1] (A[0] is not read)
 * and ||X||^2 into the work buffer. */
int cpqr_als_init(const cpqr_problem* p, void* work, size_t work_bytes, void* stream);

/* nsweeps full sweeps; relerr (device, nsweeps doubles, or NULL) receives
 * the relative error after each sweep (NaN when error_mode is NONE). */
int cpqr_als_sweep(const cpqr_problem* p, int nsweeps, double* relerr, void* work, size_t work_bytes,
                   void* stream);

/*
 * nsweeps whole sweeps captured once into a HIP graph (the Alg. 2 or Alg. 1
 * loop body, algo 0 = cpqr_als_sweep, 1 = cpqr_als_ne_sweep, including the
 * side-stream fork and join) and replayed by cpqr_graph_launch on any
 * stream, one launch for all of them.  The graph keeps the device pointers of
 * *p, relerr (nsweeps doubles, written by every launch) and work: they must
 * stay valid and the problem unchanged while the graph is used; every launch
 * continues from the state the previous one left.  Capture runs nothing.
 * cpqr_graph_destroy releases it (NULL is accepted).
 */
typedef struct cpqr_graph_t* cpqr_graph;
int cpqr_als_graph_create(const cpqr_problem* p, int algo, int nsweeps, double* relerr, void* work,
                          size_t work_bytes, cpqr_graph* out);
int cpqr_graph_launch(cpqr_graph g, void* stream);
int cpqr_graph_destroy(cpqr_graph g);

/*
 * CP-ALS with the normal equations, the paper's comparison algorithm (Alg. 1,
 * section 2.3), on the same problem description and the same Multi-TTM:
 * the MTTKRP M_n = X_(n) Z_n is read off Y_(n) (the Multi-TTM with the
 * factors A_k themselves in place of Q_k), whose column r (1 + R + ... +
 * R^{N-2}) is column r of M_n.  S_n is the Hadamard product of the Gram
 * matrices A_k^T A_k over k != n, and Ahat_n S_n = M_n is solved by Cholesky
 * (use_svd = 0; a non-positive pivot sets CPQR_STATUS_SINGULAR, a proven
 * cond(S_n) > 1e4 sets CPQR_STATUS_ILL_CONDITIONED, the signal a hybrid
 * driver uses to switch to CP-ALS-QR) or with the
 * pseudo-inverse of S_n (use_svd = 1, CP-ALS-PINV: singular values of S_n at
 * or below rtol times the largest are dropped, rtol < 0 meaning R * 2^-52;
 * dropping sets CPQR_STATUS_TRUNCATED).  Columns are normalized into lambda.
 * The efficient error is ||X||^2 - 2 <M_N, Ahat_N> + <S_N, diag(lambda) G_N
 * diag(lambda)> (section 3.3.1).  Q and Rf are not used and may be NULL;
 * A[0..N-1] all hold the start on entry (A[0] enters only through its Gram
 * matrix, which the first update does not read).  prec, dimtree and
 * error_mode act as in cpqr_als_sweep.  The work buffer keeps ||X||^2 and
 * the N Gram matrices between calls: pass the same buffer to
 * cpqr_als_ne_init and every cpqr_als_ne_sweep of one problem.  Everything
 * runs on `stream`; the Gram matrices, S_n and its factor are FP64.
 */
size_t cpqr_als_ne_work(const cpqr_problem* p);
/* Gram matrices of the starting factors, lambda = 1 and ||X||^2. */
int cpqr_als_ne_init(const cpqr_problem* p, void* work, size_t work_bytes, void* stream);
/* nsweeps sweeps of Alg. 1; relerr as in cpqr_als_sweep. */
int cpqr_als_ne_sweep(const cpqr_problem* p, int nsweeps, double* relerr, void* work, size_t work_bytes,
                      void* stream);

/*
 * Batched CP-ALS-QR for many small 3-way FP32 tensors (Alg. 2 per tensor,
 * substitution solve, efficient error of section 3.3.1) in one persistent
 * launch: one workgroup runs every sweep of one tensor, tensors taken
 * largest first, no waits between workgroups.  The contraction X x_3 Q_3^T
 * is shared by the updates of modes 1 and 2 (reuse of partial TTMs across
 * modes), so a sweep reads each tensor twice.  Contractions in FP32 on the
 * matrix cores, all else FP64.  Limits: R <= 16, R <= I[k] <= 256; X
 * 4-byte aligned.
 *
 * Ownership: every pointer in an item is caller-owned device memory that
 * must stay valid while the prepared work buffer is used; A[0] is written
 * only.  relerr (nullable) must hold sweep_offset + nsweeps doubles.  The
 * streaming passes read 16-byte runs along the first mode: a tensor whose
 * I[0] is not a multiple of 4, or that is not 16-byte aligned, is streamed
 * from a copy in the work buffer with its first mode zero-padded, taken by
 * prepare; X must not change between prepare and the runs that use it.
 *
 * cpqr_als_batch_work returns the work-buffer size (0 for invalid items).
 * cpqr_als_batch_prepare writes the per-tensor descriptors into the work
 * buffer (synchronous: it returns after the stream has drained).  With
 * autotune != 0 it picks the streaming-pass shape (contraction steps in
 * flight and 64-row groups per wave tile: 8 x 2, 4 x 4 or 16 x 1) by timing
 * an init + one sweep of each candidate on the batch itself (the initial
 * factors are restored afterwards); choices are cached per (architecture,
 * batch shape) in the file named by CPQR_AUTOTUNE_CACHE (default
 * ~/.cache/cpqr_autotune.txt).
 * cpqr_als_batch_run enqueues nsweeps sweeps of every tensor (init != 0
 * first computes the QRs of A[1], A[2] and sets lambda = 1); relerr[b][s +
 * sweep_offset] receives the relative error of sweep s.  variant = 0 uses
 * the prepared streaming shape, 1..3 force one (all give identical results).
 * cpqr_als_batch_graph does the same through a hipGraph captured on first
 * use for these arguments and replayed afterwards.  Calls on one work
 * buffer must not overlap.
 */
typedef struct cpqr_batch_item {
  int64_t I[3];          /* mode sizes */
  int R;                 /* rank */
  const float* X;        /* device FP32 tensor, column-major */
  double* A[3];          /* device I[k] x R factors; A[1], A[2] hold the start on entry */
  double* lambda;        /* device, R weights */
  double* relerr;        /* device, one double per sweep, or NULL */
} cpqr_batch_item;

size_t cpqr_als_batch_work(const cpqr_batch_item* items, int nitems);
int cpqr_als_batch_prepare(const cpqr_batch_item* items, int nitems, int autotune, void* work,
                           size_t work_bytes, void* stream);
int cpqr_als_batch_run(void* work, int nsweeps, int init, int sweep_offset, int variant, void* stream);
int cpqr_als_batch_graph(void* work, int nsweeps, int init, int sweep_offset, int variant, void* stream);
/* the configuration chosen by prepare (any output may be NULL): tensor rows
 * a lane carries through the streaming pass (4 per 64-row group), contraction
 * steps in flight, and 0 for the row-block height (the row steps take a whole
 * mode at once) */
int cpqr_als_batch_config(void* work, int* cols_per_thread, int* unroll, int* rows);

/*
 * Learned initialization (the project's initializer for CP-ALS-QR; the paper
 * runs Alg. 2 from random starts).  A sketch of the tensor feeds a
 * three-layer MLP whose output holds initial factor matrices; the network
 * is trained on factors the method itself produced, with a loss that
 * compares Kruskal tensors through R x R Gram matrices (the identity behind
 * the efficient error of section 3.3.1).  bfloat16 values are passed as
 * uint16_t bit patterns (round to nearest even).  All pointers are device
 * memory owned by the caller; calls are asynchronous on `stream`.
 *
 * cpqr_sketch3: xs = X x_1 S[0] x_2 S[1] x_3 S[2] with X column-major
 * I[0] x I[1] x I[2] FP32 and S[k] row-major J[k] x I[k] bfloat16; xs (FP32)
 * is stored with the mode-2 index fastest, then mode 1, then mode 3:
 * xs[j2 + J[1] j1 + J[1] J[0] j3].  xs_bf16 (nullable) receives xs scaled to
 * unit root-mean-square entry, xs sqrt(J[0] J[1] J[2]) / ||xs||.
 * bfloat16 operands, FP32 accumulation.  I[k] multiples of 32, I[2] and
 * I[1] I[2] multiples of 64, J[k] multiples of 64.
 */
size_t cpqr_sketch3_work(const int64_t* I, const int* J);
int cpqr_sketch3(const int64_t* I, const float* X, const int* J, const uint16_t* const* S, float* xs,
                 uint16_t* xs_bf16, void* work, size_t work_bytes, void* stream);

/*
 * Three-layer MLP y = W3 relu(W2 relu(W1 x + b1) + b2) + b3 on a batch of
 * row vectors (x: batch x din, row-major bfloat16).  W[l] row-major
 * (out x in) bfloat16, b[l] FP32.  Widths and the batch are multiples of 64.
 * forward writes the activations h1, h2 (batch x hidden, bfloat16) and y
 * (batch x dout, FP32).  backward takes dL/dy (FP32 and its bfloat16 copy)
 * and writes FP32 gradients dW[l] (same layout as W[l]) and db[l]; every
 * sum has a fixed order.
 */
typedef struct cpqr_mlp {
  int din, hidden, dout;
  const uint16_t* W[3];
  const float* b[3];
} cpqr_mlp;

size_t cpqr_mlp_work(const cpqr_mlp* net, int batch);
int cpqr_mlp_forward(const cpqr_mlp* net, int batch, const uint16_t* x, uint16_t* h1, uint16_t* h2, float* y,
                     void* work, size_t work_bytes, void* stream);
int cpqr_mlp_backward(const cpqr_mlp* net, int batch, const uint16_t* x, const uint16_t* h1, const uint16_t* h2,
                      const float* dy, const uint16_t* dy_bf16, float* const* dW, float* const* db, void* work,
                      size_t work_bytes, void* stream);

/*
 * Per sample b, with Ahat the three column-major factor matrices (I[k] x R)
 * packed one after the other in row b of y (leading dimension ldy) and A
 * those of the target (rank Rt, leading dimension ldt):
 *   CPQR_LOSS_DISTANCE  L_b = ||[[Ahat]] - [[A]]||^2 / ||[[A]]||^2
 *   CPQR_LOSS_COSINE    L_b = 1 - <[[Ahat]],[[A]]>^2 / (||[[Ahat]]||^2 ||[[A]]||^2)
 * loss (nullable) receives L_b; dy receives scale * dL_b/dy (and its
 * bfloat16 copy if dy_bf16 != NULL).  I[k] <= 256, R, Rt <= 16.  Gram sums
 * in FP64.
 */
#define CPQR_LOSS_DISTANCE 0
#define CPQR_LOSS_COSINE 1
int cpqr_kruskal_loss_grad(int batch, const int64_t* I, int R, int Rt, const float* y, int64_t ldy,
                           const float* target, int64_t ldt, int kind, float* loss, float* dy, uint16_t* dy_bf16,
                           float scale, void* stream);

/* One Adam step (Kingma and Ba, with bias correction) at step >= 1 on n
 * FP32 parameters; w_bf16 (nullable) receives the updated weights. */
int cpqr_adam(int64_t n, float* w, const float* g, float* m, float* v, uint16_t* w_bf16, int step, float lr,
              float beta1, float beta2, float eps, void* stream);

/* y = bfloat16(x), round to nearest even. */
int cpqr_to_bf16(const float* x, int64_t n, uint16_t* y, void* stream);

/*
 * Phase timers (the per-iteration breakdown of the paper's performance
 * section): when enabled, eager calls record HIP events around each phase on
 * the launch stream.  cpqr_timing_read synchronizes those events and returns
 * accumulated milliseconds and launch counts per phase since the last reset.
 * Phases: 0 Multi-TTM, 1 first (tensor-streaming) contraction, 2 factor QR,
 * 3 computing Q_0, 4 applying Q_0, 5 solve + normalize, 6 error, 7 the
 * subset of phase 1 that runs the row-tiled matrix-core kernel.  Phase 7 is
 * timed by events attached to the kernel dispatch itself and adds no work
 * to the stream; the others record events between phases, which costs some
 * microseconds per event.  cpqr_timing_select limits recording to the
 * phases whose bit is set in mask (all phases after load).
 */
#define CPQR_NPHASES 8
int cpqr_timing_enable(int on);
int cpqr_timing_select(unsigned mask);
int cpqr_timing_reset(void);
int cpqr_timing_read(double* ms, int64_t* counts, int nphases);

#ifdef __cplusplus
}
#endif

#endif /* CPQR_H */
