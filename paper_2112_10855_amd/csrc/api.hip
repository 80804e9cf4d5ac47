// C ABI of libcpqr (include/cpqr.h): argument validation, scratch sizing,
// phase timers and the CP-ALS-QR sweep driver (paper Alg. 2).  Kernels live
// in tsqr.hip (QRs), multittm.hip (Multi-TTM) and small.hip (apply Q_0,
// solves, errors).

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace cpqr {

namespace {
thread_local std::string g_error;

struct TimingState {
  std::mutex mu;
  bool on = false;
  unsigned mask = ~0u;  // phases that record
  struct Pending {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double ms[CPQR_NPHASES] = {};
  int64_t count[CPQR_NPHASES] = {};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
TimingState& timing() {
  static TimingState t;
  return t;
}
}  // namespace

void set_error(const std::string& msg) { g_error = msg; }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CPQR_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return CPQR_OK;
}

int check_work(void* work, size_t have, size_t need) {
  if (need == 0) return CPQR_OK;
  if (!work) return fail(CPQR_ERR_WORKSPACE, "work buffer is NULL");
  if (reinterpret_cast<uintptr_t>(work) % 256 != 0)
    return fail(CPQR_ERR_WORKSPACE, "work buffer must be 256-byte aligned");
  if (have < need)
    return fail(CPQR_ERR_WORKSPACE, "work buffer too small: " + std::to_string(have) + " < " +
                                        std::to_string(need) + " bytes");
  return CPQR_OK;
}

KernelEvents kernel_events(int phase, hipStream_t s) {
  KernelEvents ke;
  if (phase < 0) return ke;
  TimingState& t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  if (!t.on || !((t.mask >> phase) & 1u)) return ke;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return ke;
  ke.a = t.get();
  ke.b = ke.a ? t.get() : nullptr;
  if (!ke.b) {
    if (ke.a) t.pool.push_back(ke.a);
    ke.a = nullptr;
    return ke;
  }
  ke.phase = phase;
  return ke;
}

void kernel_events_done(const KernelEvents& ke) {
  if (!ke.a) return;
  TimingState& t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  t.pending.push_back({ke.phase, ke.a, ke.b});
}

PhaseTimer::PhaseTimer(int ph, hipStream_t s) : phase(ph), stream(s) {
  if (ph < 0) return;
  TimingState& t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  if (!t.on || !((t.mask >> ph) & 1u)) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  ev0 = t.get();
  if (ev0 && hipEventRecord(ev0, s) != hipSuccess) ev0 = nullptr;
}

PhaseTimer::~PhaseTimer() {
  if (!ev0) return;
  TimingState& t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  hipEvent_t e1 = t.get();
  if (!e1 || hipEventRecord(e1, stream) != hipSuccess) return;
  t.pending.push_back({phase, ev0, e1});
}

}  // namespace cpqr

using namespace cpqr;

namespace {

int valid_dtype(int d) { return d == CPQR_F32 || d == CPQR_F64; }
int valid_prec(int p) { return p >= CPQR_PREC_F64 && p <= CPQR_PREC_BF16; }

int check_rank(int R) {
  if (R < 1 || R > CPQR_MAX_RANK)
    return fail(CPQR_ERR_SHAPE, "R must be in [1, " + std::to_string(CPQR_MAX_RANK) + "]");
  return CPQR_OK;
}

int check_modes(int N, const int64_t* I) {
  if (!I) return fail(CPQR_ERR_ARG, "mode sizes pointer is NULL");
  if (N < 2 || N > CPQR_MAX_MODES)
    return fail(CPQR_ERR_SHAPE, "N must be in [2, " + std::to_string(CPQR_MAX_MODES) + "]");
  for (int k = 0; k < N; ++k)
    if (I[k] < 1) return fail(CPQR_ERR_SHAPE, "mode size I[" + std::to_string(k) + "] < 1");
  return CPQR_OK;
}

int check_krp_rows(int N, int R) {
  double rows = std::pow(double(R), N - 1);
  if (rows > double(1LL << 31))
    return fail(CPQR_ERR_SHAPE, "R^(N-1) too large for the Khatri-Rao QR");
  return CPQR_OK;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// ------------------------------------------------------------ sweep scratch
struct AlsWs {
  double* xnorm2;
  double* Q0;
  double* Qc;  // factors of the structured QR of V_n (N - 2 blocks of R^2 x R)
  double* Qx;  // ping-pong buffers that expand them into Q0
  double* R0;
  void* Y;
  double* W;
  double* fit;
  double* relerr_tmp;
  void* sub;
  void* krp_sub;  // scratch of the Khatri-Rao QR, which runs beside the Multi-TTM
  void* Wt;       // X contracted over one half of the modes (dimension-tree reuse)
  double* err_part;  // partial sums of the efficient error (side stream)
  double* Tmid;      // the chain's last-but-one triangle, kept between the split chain's parts
  // FP32 contraction operands of each Q_k written by its normalizing factor
  // QR (rows and four-row layouts; null where not kept), padding urp (0: none)
  float* ur[CPQR_MAX_MODES];
  float* uq[CPQR_MAX_MODES];
  int urp;
};

// Split point of the dimension-tree reuse (0 = off).
int dt_split(const cpqr_problem* p) {
  if (p->dimtree == 0 || p->N < 3) return 0;
  if (p->dimtree > 0) return p->dimtree;
  return p->N == 3 ? 2 : p->N / 2;
}

unsigned range_mask(int lo, int hi) { return ((1u << hi) - 1u) & ~((1u << lo) - 1u); }

// Sizes of X contracted over the modes outside [lo, hi), and its element count.
int64_t half_dims(const cpqr_problem* p, int lo, int hi, int64_t* D) {
  int64_t c = 1;
  for (int k = 0; k < p->N; ++k) {
    D[k] = (k >= lo && k < hi) ? p->I[k] : p->R;
    c *= D[k];
  }
  return c;
}

size_t ttm_sub_bytes(const cpqr_problem* p) {
  const int N = p->N, R = p->R;
  size_t b = 0;
  const int h = dt_split(p);
  if (h > 0) {
    for (int half = 0; half < 2; ++half) {
      const int lo = half ? h : 0, hi = half ? N : h;
      int64_t D[CPQR_MAX_MODES];
      half_dims(p, lo, hi, D);
      b = std::max(b, multittm_general_work(N, p->I, ~range_mask(lo, hi) & range_mask(0, N), R, p->prec));
      for (int n = lo; n < hi; ++n)
        b = std::max(b, multittm_general_work(N, D, range_mask(lo, hi) & ~(1u << n), R, p->prec));
    }
  }
  int64_t count = 1;
  for (int k = 0; k < N; ++k) {
    count *= p->I[k];
    b = std::max(b, multittm_work(N, p->I, k, R, p->prec));
  }
  b = std::max(b, fit_direct_work(N, p->I, R));
  b = std::max(b, norm2_work(count));
  return b;
}

// ---------------------------------------------- structured QR of V_n
// V_n = R_{a_{N-1}} (.) ... (.) R_{a_1} (modes a_1 < a_2 < .. other than n,
// a_1's index fastest) is factorized without forming it, by eq. (kr-id):
// with T_1 = R_{a_1} and the QR R_{a_j} (.) T_{j-1} = Q_j T_j of an R^2 x R
// Khatri-Rao product of two triangular factors (j = 2..N-1),
//   R_{a_j} (.) (Q_{j-1} T_{j-1}) = (I_R kron Q_{j-1}) (R_{a_j} (.) T_{j-1}),
// so V_n = (I kron Q_2)(I kron Q_3) .. Q_{N-1} T_{N-1}: R_0 = T_{N-1} and Q_0 is
// the product of the Kronecker-structured factors, never formed.  N - 2 QRs
// of R^2 x R (4 R^4 flops each) replace one of R^{N-1} x R (4 R^{N+1}); for
// N = 3 it is the QR of V_n itself.  Qc holds Q_2 .. Q_{N-1} one after the
// other, each R^2 x R column-major.
size_t krp_chain_work(int R) {
  Carver cv(nullptr);
  for (int i = 0; i < 4; ++i) cv.take<double>(size_t(R) * R);
  cv.take<char>(tsqr_work(int64_t(R) * R, R));
  return cv.bytes();
}

// Steps [j0, j1) of the chain (1 <= j0 < j1 <= N - 1): step j factors
// R_{a_j} (.) T_{j-1} (T_0 = R_{a_0}; T_{j0-1} read from tkeep when j0 > 1).
// T_{j1-1} goes to tkeep when the chain goes on (j1 < N - 1), else to R0; so
// a chain can be split where its later factors are not final yet.
int krp_chain_steps(int N, int n, int R, const double* const* Rk, int64_t ldr, double* Qc, double* R0,
                    double* tkeep, int j0, int j1, void* work, hipStream_t s) {
  Carver cv(work);
  double* T[2] = {cv.take<double>(size_t(R) * R), cv.take<double>(size_t(R) * R)};
  double* F[2] = {cv.take<double>(size_t(R) * R), cv.take<double>(size_t(R) * R)};
  void* qw = cv.take<char>(tsqr_work(int64_t(R) * R, R));
  int a[CPQR_MAX_MODES], na = 0;
  for (int k = 0; k < N; ++k)
    if (k != n) a[na++] = k;
  // every factor of a step is read with leading dimension R
  auto packed = [&](const double* src, double* buf, const double** out) -> int {
    if (ldr == R) {
      *out = src;
      return CPQR_OK;
    }
    CPQR_HIP(hipMemcpy2DAsync(buf, sizeof(double) * R, src, sizeof(double) * ldr, sizeof(double) * R, R,
                              hipMemcpyDeviceToDevice, s));
    *out = buf;
    return CPQR_OK;
  };
  const double* t = tkeep;
  if (j0 == 1) CPQR_TRY(packed(Rk[a[0]], F[0], &t));
  for (int j = j0; j < j1; ++j) {
    const double* f = nullptr;
    CPQR_TRY(packed(Rk[a[j]], F[1], &f));
    double* tout = j == na - 1 ? R0 : (j == j1 - 1 ? tkeep : T[j % 2]);
    const double* fac[3] = {t, f, nullptr};  // R_{a_j} (.) T_{j-1}, T's index fastest
    CPQR_TRY(krp_qr_enqueue(3, 2, R, fac, R, Qc + size_t(j - 1) * R * R * R, tout, qw, s));
    t = tout;
  }
  return CPQR_OK;
}

int krp_chain_enqueue(int N, int n, int R, const double* const* Rk, int64_t ldr, double* Qc, double* R0,
                      void* work, hipStream_t s) {
  return krp_chain_steps(N, n, R, Rk, ldr, Qc, R0, nullptr, 1, N - 1, work, s);
}

// W = Y_(n) Q_0 with Q_0 = (I kron Q_2) .. Q_{N-1}: step j contracts the two
// fastest remaining column digits of Y (R^2 of them, the first being the
// output of step j - 1) with Q_j, a Multi-TTM step on the [I_n, R^2, R^{N-2-j}]
// view; FP64 results.
size_t apply_chain_work(int64_t In, int N, int R) {
  const int64_t rest = ipow(R, N - 3);
  const int64_t dims[3] = {In, int64_t(R) * R, rest};
  Carver cv(nullptr);
  if (N > 3)
    for (int i = 0; i < 2; ++i) cv.take<double>(size_t(In) * R * rest);
  cv.take<char>(multittm_general_work(3, dims, 2u, R, CPQR_PREC_F64));
  return cv.bytes();
}

int apply_chain_enqueue(int64_t In, int N, int R, int ydtype, const void* Y, const double* Qc, double* W,
                        void* work, hipStream_t s) {
  const int64_t rest = ipow(R, N - 3);
  Carver cv(work);
  double* buf[2] = {nullptr, nullptr};
  if (N > 3)
    for (int i = 0; i < 2; ++i) buf[i] = cv.take<double>(size_t(In) * R * rest);
  void* mw = cv.take<char>(0);
  const void* cur = Y;
  int cur_dt = ydtype;
  for (int j = 1; j <= N - 2; ++j) {
    const int64_t dims[3] = {In, int64_t(R) * R, ipow(R, N - 2 - j)};
    const double* Q[3] = {nullptr, Qc + size_t(j - 1) * R * R * R, nullptr};
    double* out = j == N - 2 ? W : buf[j % 2];
    CPQR_TRY(multittm_general_enqueue(3, dims, cur_dt, cur, 2u, -1, R, Q, CPQR_PREC_F64, out, mw, s, false));
    cur = out;
    cur_dt = CPQR_F64;
  }
  return CPQR_OK;
}

// The dense QR of the formed V_n overlaps the Multi-TTM on its own stream; it
// stays the default while V_n is short (R^{N-1} <= 65536 rows: at 32^3 rows it
// left the sweep about 2% faster than the structured form's longer chain of
// small launches) and the structured form takes over beyond.
bool use_chain(const cpqr_problem* p) {
  if (p->krp_chain > 0) return p->N >= 3;
  return p->krp_chain < 0 && p->N >= 4 && ipow(p->R, p->N - 1) > 65536;
}

size_t als_sub_bytes(const cpqr_problem* p) {
  const int N = p->N, R = p->R;
  const int64_t K = ipow(R, N - 1);
  size_t b = std::max(ttm_sub_bytes(p), tsqr_work(K, R));
  for (int k = 0; k < N; ++k) {
    b = std::max(b, tsqr_work(p->I[k], R));
    b = std::max(b, apply_q0_work(p->I[k], K, R));
    b = std::max(b, solve_work(p->I[k], R));
  }
  return b;
}

// Size of the dimension-tree intermediate (elements; 0 without the reuse).
int64_t dt_elems(const cpqr_problem* p) {
  const int N = p->N, h = dt_split(p);
  int64_t wt = 0;
  if (h > 0) {
    int64_t D[CPQR_MAX_MODES];
    if (h > 1) wt = std::max(wt, half_dims(p, 0, h, D));
    if (N - h > 1) wt = std::max(wt, half_dims(p, h, N, D));
  }
  return wt;
}

// ------------------------------------------------------------ Alg. 1 scratch
// The Gram matrices persist in the work buffer from cpqr_als_ne_init on.
struct NeWs {
  double* xnorm2;
  double* G;  // N blocks of R x R
  double* S;
  double* F;
  void* Y;
  double* M;
  double* relerr_tmp;
  void* sub;
  void* Wt;
  double* err_part;
};

size_t ne_carve(Carver& cv, const cpqr_problem* p, NeWs* ws) {
  const int N = p->N, R = p->R;
  const int64_t K = ipow(R, N - 1);
  int64_t imax = 0;
  for (int k = 0; k < N; ++k) imax = std::max(imax, p->I[k]);
  NeWs w{};
  w.xnorm2 = cv.take<double>(1);
  w.G = cv.take<double>(size_t(N) * R * R);
  w.S = cv.take<double>(size_t(R) * R);
  w.F = cv.take<double>(size_t(R) * R);
  w.Y = cv.take<double>(size_t(imax) * K);  // sized for FP64 Y
  w.M = cv.take<double>(size_t(imax) * R);
  w.relerr_tmp = cv.take<double>(1);
  w.sub = cv.take<char>(std::max(ttm_sub_bytes(p), ne_update_work(R)));
  w.Wt = cv.take<double>(size_t(dt_elems(p)));
  w.err_part = cv.take<double>(ne_error_work(p->I[N - 1]) / sizeof(double));
  if (ws) *ws = w;
  return cv.bytes();
}

// Y = X contracted with U_k^T over every mode but n, unfolded along n, with the
// dimension-tree reuse of the mode split h (shared by both algorithms).
int ttm_for_mode(const cpqr_problem* p, int h, int n, const double* const* U, void* Y, void* Wt, void* sub,
                 hipStream_t s, const UCache* uc) {
  const int N = p->N, R = p->R;
  const int ydt = p->prec == CPQR_PREC_F64 ? CPQR_F64 : CPQR_F32;
  const int lo = (h > 0 && n >= h) ? h : 0, hi = (h > 0 && n < h) ? h : N;
  if (h == 0 || hi - lo == 1)
    return multittm_enqueue(N, p->I, p->xdtype, p->X, n, R, U, p->prec, Y, sub, s, uc);
  // X contracted over the modes outside [lo, hi) once (when the first mode of
  // the half is updated; those factors do not change while the half is
  // updated), then the remaining modes of the half for each n
  if (n == lo)
    CPQR_TRY(multittm_general_enqueue(N, p->I, p->xdtype, p->X, ~range_mask(lo, hi) & range_mask(0, N), -1, R, U,
                                      p->prec, Wt, sub, s, true, uc));
  int64_t D[CPQR_MAX_MODES];
  half_dims(p, lo, hi, D);
  return multittm_general_enqueue(N, D, ydt, Wt, range_mask(lo, hi) & ~(1u << n), n, R, U, p->prec, Y, sub, s,
                                  false, uc);
}

size_t als_carve(Carver& cv, const cpqr_problem* p, AlsWs* ws) {
  const int N = p->N, R = p->R;
  const int64_t K = ipow(R, N - 1);
  int64_t imax = 0;
  for (int k = 0; k < N; ++k) imax = std::max(imax, p->I[k]);
  AlsWs w{};
  w.xnorm2 = cv.take<double>(1);
  w.Q0 = cv.take<double>(size_t(K) * R);
  // factors of the structured QR of V_n and the buffers that expand them into Q_0
  w.Qc = cv.take<double>(size_t(std::max(N - 2, 0)) * R * R * R);
  w.Qx = cv.take<double>(N >= 5 ? 2 * size_t(K) * R : 0);
  w.R0 = cv.take<double>(size_t(R) * R);
  w.Y = cv.take<double>(size_t(imax) * K);  // sized for FP64 Y
  w.W = cv.take<double>(size_t(imax) * R);
  w.fit = cv.take<double>(2);
  w.relerr_tmp = cv.take<double>(1);
  w.sub = cv.take<char>(als_sub_bytes(p));
  w.krp_sub = cv.take<char>(std::max(tsqr_work(K, R), krp_chain_work(R)));
  w.Wt = cv.take<double>(size_t(dt_elems(p)));  // sized for FP64
  w.err_part = cv.take<double>(error_efficient_work(p->I[N - 1]) / sizeof(double));
  w.Tmid = cv.take<double>(size_t(R) * R);
  // the FP32 operands need the factor QR's padded rank to equal the
  // contraction kernels' column padding (R > 8)
  const int rp = (R + 15) / 16 * 16;
  w.urp = p->prec != CPQR_PREC_F64 && round_rank(R) == rp ? rp : 0;
  for (int k = 0; k < N; ++k) {  // (take() returns null while only sizing: test the conditions, not pointers)
    const bool keep = w.urp && norm_qr_fits(p->I[k], R);
    w.ur[k] = keep ? cv.take<float>(size_t(p->I[k] + 4) * rp) : nullptr;
    w.uq[k] = keep && p->I[k] % 4 == 0 ? cv.take<float>(size_t(p->I[k] + 4) * rp) : nullptr;
  }
  if (ws) *ws = w;
  return cv.bytes();
}

// A second stream per device for the Khatri-Rao QR of a mode, which depends
// only on the R factors and so runs while the Multi-TTM streams the tensor
// (default priority, non-blocking), and two events that order it.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t ready = nullptr, done = nullptr;
};
std::mutex g_side_mu;
std::map<int, SideStream> g_side;

int side_stream(SideStream& out) {
  int dev = 0;
  CPQR_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_side_mu);
  SideStream& ss = g_side[dev];
  if (!ss.s) {
    CPQR_HIP(hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking));
    CPQR_HIP(hipEventCreateWithFlags(&ss.ready, hipEventDisableTiming));
    CPQR_HIP(hipEventCreateWithFlags(&ss.done, hipEventDisableTiming));
  }
  out = ss;
  return CPQR_OK;
}

bool kruskal_input(const cpqr_problem* p) { return p->xS > 0; }

int check_problem(const cpqr_problem* p, bool need_qr = true) {
  if (!p) return fail(CPQR_ERR_ARG, "problem is NULL");
  CPQR_TRY(check_modes(p->N, p->I));
  CPQR_TRY(check_rank(p->R));
  if (p->xS < 0 || p->xS > CPQR_MAX_KRUSKAL_TERMS)
    return fail(CPQR_ERR_SHAPE, "xS must be in [0, " + std::to_string(CPQR_MAX_KRUSKAL_TERMS) + "]");
  if (kruskal_input(p)) {
    if (!p->xmu) return fail(CPQR_ERR_ARG, "Kruskal input: xmu is NULL");
    for (int k = 0; k < p->N; ++k)
      if (!p->xV[k]) return fail(CPQR_ERR_ARG, "Kruskal input: xV[" + std::to_string(k) + "] is NULL");
    if (p->error_mode == CPQR_ERROR_DIRECT && !p->X)
      return fail(CPQR_ERR_ARG, "the direct error of a Kruskal input needs its dense tensor X");
    if (p->X && !valid_dtype(p->xdtype)) return fail(CPQR_ERR_DTYPE, "xdtype must be CPQR_F32 or CPQR_F64");
    if (p->error_mode < CPQR_ERROR_EFFICIENT || p->error_mode > CPQR_ERROR_NONE)
      return fail(CPQR_ERR_ARG, "unknown error_mode");
    if (!p->lambda) return fail(CPQR_ERR_ARG, "lambda is NULL");
    // modes smaller than the rank are allowed here: their factor QR is that of
    // the factor padded with zero rows (cpqr_factor_qr)
    for (int k = 0; k < p->N; ++k)
      if (!p->A[k] || (need_qr && (!p->Q[k] || !p->Rf[k])))
        return fail(CPQR_ERR_ARG, "A/Q/Rf pointer of mode " + std::to_string(k) + " is NULL");
    return CPQR_OK;
  }
  CPQR_TRY(check_krp_rows(p->N, p->R));
  if (!valid_dtype(p->xdtype)) return fail(CPQR_ERR_DTYPE, "xdtype must be CPQR_F32 or CPQR_F64");
  if (!valid_prec(p->prec)) return fail(CPQR_ERR_ARG, "unknown precision");
  if (p->prec != CPQR_PREC_F64 && p->xdtype != CPQR_F32)
    return fail(CPQR_ERR_DTYPE, "reduced-precision Multi-TTM needs an FP32 tensor");
  if (p->error_mode < CPQR_ERROR_EFFICIENT || p->error_mode > CPQR_ERROR_NONE)
    return fail(CPQR_ERR_ARG, "unknown error_mode");
  if (p->dimtree < -1 || (p->dimtree > 0 && p->dimtree >= p->N))
    return fail(CPQR_ERR_ARG, "dimtree must be -1, 0 or a split point in [1, N-1]");
  if (!p->X || !p->lambda) return fail(CPQR_ERR_ARG, "X or lambda is NULL");
  for (int k = 0; k < p->N; ++k) {
    if (!p->A[k] || (need_qr && (!p->Q[k] || !p->Rf[k])))
      return fail(CPQR_ERR_ARG, "A/Q/Rf pointer of mode " + std::to_string(k) + " is NULL");
    if (p->I[k] < p->R)
      return fail(CPQR_ERR_SHAPE, "mode " + std::to_string(k) + " is smaller than the rank");
  }
  return CPQR_OK;
}

int check_multittm_args(int N, const int64_t* I, int xdtype, const void* X, int n, int R,
                        const double* const* Q, int prec, void* Y) {
  CPQR_TRY(check_modes(N, I));
  CPQR_TRY(check_rank(R));
  if (n < 0 || n >= N) return fail(CPQR_ERR_ARG, "multittm: n out of range");
  if (!valid_dtype(xdtype)) return fail(CPQR_ERR_DTYPE, "multittm: xdtype must be CPQR_F32 or CPQR_F64");
  if (!valid_prec(prec)) return fail(CPQR_ERR_ARG, "multittm: unknown precision");
  if (prec != CPQR_PREC_F64 && xdtype != CPQR_F32)
    return fail(CPQR_ERR_DTYPE, "multittm: reduced-precision forms need an FP32 tensor");
  if (!X || !Y || !Q) return fail(CPQR_ERR_ARG, "multittm: NULL pointer");
  for (int k = 0; k < N; ++k)
    if (k != n && !Q[k]) return fail(CPQR_ERR_ARG, "multittm: Q[" + std::to_string(k) + "] is NULL");
  return check_krp_rows(N, R);
}

// Scratch of cpqr_multittm_noalloc: one copy per device, resolved there on the
// first call with that device current.  In host code `scratch` is a host-side
// stand-in for the symbol, never a device address: kernels get the address
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[CPQR_NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;

int noalloc_scratch(void** out) {
  int dev = 0;
  CPQR_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    CPQR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0)
      return fail(CPQR_ERR_HIP, "multittm_noalloc: the scratch array has no aligned device address");
    it = g_scratch_ptr.emplace(dev, p).first;
  }
  *out = it->second;
  return CPQR_OK;
}

}  // namespace

extern "C" {

const char* cpqr_last_error(void) { return g_error.c_str(); }

int cpqr_version(void) { return 100; }

size_t cpqr_factor_qr_work(int64_t I, int R) {
  if (I < 1 || R < 1 || R > CPQR_MAX_RANK) return 0;
  return tsqr_work(I, R);
}

int cpqr_factor_qr(int64_t I, int R, const double* A, int64_t lda, double* Q, int64_t ldq,
                   double* Rk, int64_t ldr, void* work, size_t work_bytes, void* stream) {
  CPQR_TRY(check_rank(R));
  if (I < 1) return fail(CPQR_ERR_SHAPE, "factor_qr needs I >= 1");
  if (!A || !Q || !Rk) return fail(CPQR_ERR_ARG, "factor_qr: NULL pointer");
  if (lda < I || ldq < I || ldr < R) return fail(CPQR_ERR_SHAPE, "factor_qr: leading dimension too small");
  CPQR_TRY(check_work(work, work_bytes, tsqr_work(I, R)));
  return factor_qr_enqueue(I, R, A, lda, Q, ldq, Rk, ldr, work, as_stream(stream));
}

size_t cpqr_krp_qr_work(int N, int R) {
  if (N < 2 || N > CPQR_MAX_MODES || R < 1 || R > CPQR_MAX_RANK) return 0;
  if (check_krp_rows(N, R) != CPQR_OK) return 0;
  return tsqr_work(ipow(R, N - 1), R);
}

int cpqr_krp_qr(int N, int n, int R, const double* const* Rk, int64_t ldr, double* Q0, double* R0,
                void* work, size_t work_bytes, void* stream) {
  if (N < 2 || N > CPQR_MAX_MODES) return fail(CPQR_ERR_SHAPE, "krp_qr: N out of range");
  if (n < 0 || n >= N) return fail(CPQR_ERR_ARG, "krp_qr: n out of range");
  CPQR_TRY(check_rank(R));
  CPQR_TRY(check_krp_rows(N, R));
  if (!Rk || !Q0 || !R0) return fail(CPQR_ERR_ARG, "krp_qr: NULL pointer");
  for (int k = 0; k < N; ++k)
    if (k != n && !Rk[k]) return fail(CPQR_ERR_ARG, "krp_qr: Rk[" + std::to_string(k) + "] is NULL");
  if (ldr < R) return fail(CPQR_ERR_SHAPE, "krp_qr: ldr < R");
  CPQR_TRY(check_work(work, work_bytes, tsqr_work(ipow(R, N - 1), R)));
  return krp_qr_enqueue(N, n, R, Rk, ldr, Q0, R0, work, as_stream(stream));
}

size_t cpqr_multittm_work(int N, const int64_t* I, int n, int R, int prec) {
  if (check_modes(N, I) != CPQR_OK || n < 0 || n >= N || R < 1 || R > CPQR_MAX_RANK) return 0;
  return multittm_work(N, I, n, R, prec);
}

int cpqr_multittm(int N, const int64_t* I, int xdtype, const void* X, int n, int R,
                  const double* const* Q, int prec, void* Y, void* work, size_t work_bytes,
                  void* stream) {
  CPQR_TRY(check_multittm_args(N, I, xdtype, X, n, R, Q, prec, Y));
  CPQR_TRY(check_work(work, work_bytes, multittm_work(N, I, n, R, prec)));
  return multittm_enqueue(N, I, xdtype, X, n, R, Q, prec, Y, work, as_stream(stream));
}

int cpqr_multittm_noalloc(int N, const int64_t* I, int xdtype, const void* X, int n, int R,
                          const double* const* Q, int prec, void* Y, void* stream) {
  CPQR_TRY(check_multittm_args(N, I, xdtype, X, n, R, Q, prec, Y));
  const size_t need = multittm_work(N, I, n, R, prec);
  if (need > CPQR_NOALLOC_SCRATCH_BYTES)
    return fail(CPQR_ERR_WORKSPACE, "multittm_noalloc: this Multi-TTM needs " + std::to_string(need) +
                                        " bytes of scratch, more than the " +
                                        std::to_string(CPQR_NOALLOC_SCRATCH_BYTES) +
                                        " of the static array; call cpqr_multittm with a workspace");
  void* scr = nullptr;
  CPQR_TRY(noalloc_scratch(&scr));
  return multittm_enqueue(N, I, xdtype, X, n, R, Q, prec, Y, scr, as_stream(stream));
}

size_t cpqr_krp_qr_chain_work(int N, int R) {
  if (N < 3 || N > CPQR_MAX_MODES || R < 1 || R > CPQR_MAX_RANK) return 0;
  return krp_chain_work(R);
}

int cpqr_krp_qr_chain(int N, int n, int R, const double* const* Rk, int64_t ldr, double* Qc, double* R0,
                      void* work, size_t work_bytes, void* stream) {
  if (N < 3 || N > CPQR_MAX_MODES) return fail(CPQR_ERR_SHAPE, "krp_qr_chain: N out of range (3..10)");
  if (n < 0 || n >= N) return fail(CPQR_ERR_ARG, "krp_qr_chain: n out of range");
  CPQR_TRY(check_rank(R));
  if (!Rk || !Qc || !R0) return fail(CPQR_ERR_ARG, "krp_qr_chain: NULL pointer");
  for (int k = 0; k < N; ++k)
    if (k != n && !Rk[k]) return fail(CPQR_ERR_ARG, "krp_qr_chain: Rk[" + std::to_string(k) + "] is NULL");
  if (ldr < R) return fail(CPQR_ERR_SHAPE, "krp_qr_chain: ldr < R");
  CPQR_TRY(check_work(work, work_bytes, krp_chain_work(R)));
  return krp_chain_enqueue(N, n, R, Rk, ldr, Qc, R0, work, as_stream(stream));
}

size_t cpqr_expand_q0_work(int N, int R) {
  if (N < 3 || N > CPQR_MAX_MODES || R < 1 || R > CPQR_MAX_RANK) return 0;
  return N >= 5 ? sizeof(double) * 2 * size_t(ipow(R, N)) : 0;
}

int cpqr_expand_q0(int N, int R, const double* Qc, double* Q0, void* work, size_t work_bytes, void* stream) {
  if (N < 3 || N > CPQR_MAX_MODES) return fail(CPQR_ERR_SHAPE, "expand_q0: N out of range (3..10)");
  CPQR_TRY(check_rank(R));
  CPQR_TRY(check_krp_rows(N, R));
  if (!Qc || !Q0) return fail(CPQR_ERR_ARG, "expand_q0: NULL pointer");
  CPQR_TRY(check_work(work, work_bytes, cpqr_expand_q0_work(N, R)));
  return expand_q0_enqueue(N, R, Qc, Q0, static_cast<double*>(work), as_stream(stream));
}

size_t hosvd_work(int N, const int64_t* I, int R, int prec) {
  const int64_t K = ipow(R, N - 1);
  int64_t imax = 0;
  size_t sub = 0;
  for (int k = 0; k < N; ++k) {
    imax = std::max(imax, I[k]);
    sub = std::max(sub, std::max(multittm_work(N, I, k, R, prec), tsqr_work(I[k], R)));
  }
  Carver cv(nullptr);
  cv.take<double>(size_t(imax) * K);  // Y_(k), sized for FP64
  cv.take<double>(size_t(imax) * R);  // W_k
  cv.take<double>(size_t(R) * R);     // R of the QR (not returned)
  cv.take<char>(sub);
  return cv.bytes();
}

size_t cpqr_hosvd_init_work(int N, const int64_t* I, int R, int prec) {
  if (check_modes(N, I) != CPQR_OK || R < 1 || R > CPQR_MAX_RANK || !valid_prec(prec)) return 0;
  if (check_krp_rows(N, R) != CPQR_OK) return 0;
  return hosvd_work(N, I, R, prec);
}

int cpqr_hosvd_init(int N, const int64_t* I, int xdtype, const void* X, int R, const double* const* Omega, int prec,
                    int k0, double* const* A, void* work, size_t work_bytes, void* stream) {
  if (!A || !Omega || !I) return fail(CPQR_ERR_ARG, "hosvd_init: NULL pointer array");
  CPQR_TRY(check_modes(N, I));
  if (k0 < 0 || k0 >= N) return fail(CPQR_ERR_ARG, "hosvd_init: k0 out of range");
  for (int k = k0; k < N; ++k)
    if (!A[k]) return fail(CPQR_ERR_ARG, "hosvd_init: A[" + std::to_string(k) + "] is NULL");
  // the Multi-TTM's own checks (its output is internal; A[k0] stands in for it)
  CPQR_TRY(check_multittm_args(N, I, xdtype, X, 0, R, Omega, prec, A[k0]));
  if (!Omega[0]) return fail(CPQR_ERR_ARG, "hosvd_init: Omega[0] is NULL");
  for (int k = k0; k < N; ++k)
    if (I[k] < R) return fail(CPQR_ERR_SHAPE, "hosvd_init: mode " + std::to_string(k) + " is smaller than R");
  CPQR_TRY(check_work(work, work_bytes, hosvd_work(N, I, R, prec)));
  hipStream_t s = as_stream(stream);
  const int64_t K = ipow(R, N - 1);
  int64_t imax = 0;
  for (int k = 0; k < N; ++k) imax = std::max(imax, I[k]);
  Carver cv(work);
  void* Y = cv.take<double>(size_t(imax) * K);
  double* W = cv.take<double>(size_t(imax) * R);
  double* Rk = cv.take<double>(size_t(R) * R);
  void* sub = cv.take<char>(0);
  const int ydt = prec == CPQR_PREC_F64 ? CPQR_F64 : CPQR_F32;
  for (int k = k0; k < N; ++k) {
    CPQR_TRY(multittm_enqueue(N, I, xdtype, X, k, R, Omega, prec, Y, sub, s));
    CPQR_TRY(diag_cols_enqueue(I[k], N, R, ydt, Y, W, s));
    CPQR_TRY(factor_qr_enqueue(I[k], R, W, I[k], A[k], I[k], Rk, R, sub, s));
  }
  return CPQR_OK;
}

int check_kruskal(int N, const int64_t* I, int S, const double* mu, const double* const* V) {
  CPQR_TRY(check_modes(N, I));
  if (S < 1 || S > CPQR_MAX_KRUSKAL_TERMS)
    return fail(CPQR_ERR_SHAPE, "S must be in [1, " + std::to_string(CPQR_MAX_KRUSKAL_TERMS) + "]");
  if (!mu || !V) return fail(CPQR_ERR_ARG, "Kruskal input: NULL pointer");
  for (int k = 0; k < N; ++k)
    if (!V[k]) return fail(CPQR_ERR_ARG, "Kruskal input: V[" + std::to_string(k) + "] is NULL");
  return CPQR_OK;
}

size_t cpqr_kruskal_w_work(int N, int R, int S) {
  if (N < 3 || N > CPQR_MAX_MODES || R < 1 || R > CPQR_MAX_RANK || S < 1 || S > CPQR_MAX_KRUSKAL_TERMS) return 0;
  Carver cv(nullptr);
  cv.take<double>(size_t(N) * R * S);
  cv.take<double>(size_t(S) * R);
  return cv.bytes();
}

int cpqr_kruskal_w(int N, int n, int R, const int64_t* I, int S, const double* mu, const double* const* V,
                   const double* const* Q, const double* Qc, double* W, void* work, size_t work_bytes,
                   void* stream) {
  CPQR_TRY(check_kruskal(N, I, S, mu, V));
  if (N < 3) return fail(CPQR_ERR_SHAPE, "kruskal_w: N must be at least 3 (Q_0 in structured form)");
  CPQR_TRY(check_rank(R));
  if (n < 0 || n >= N) return fail(CPQR_ERR_ARG, "kruskal_w: n out of range");
  if (!Q || !Qc || !W) return fail(CPQR_ERR_ARG, "kruskal_w: NULL pointer");
  for (int k = 0; k < N; ++k)
    if (k != n && !Q[k]) return fail(CPQR_ERR_ARG, "kruskal_w: Q[" + std::to_string(k) + "] is NULL");
  CPQR_TRY(check_work(work, work_bytes, cpqr_kruskal_w_work(N, R, S)));
  hipStream_t s = as_stream(stream);
  Carver cv(work);
  double* P = cv.take<double>(size_t(N) * R * S);
  double* M = cv.take<double>(size_t(S) * R);
  const double* Pa[CPQR_MAX_MODES];
  int na = 0;
  for (int k = 0; k < N; ++k) {
    if (k == n) continue;
    double* Pk = P + size_t(k) * R * S;
    CPQR_TRY(kr_cross_enqueue(I[k], R, S, Q[k], I[k], V[k], I[k], Pk, s));
    Pa[na++] = Pk;
  }
  CPQR_TRY(kr_chain_enqueue(na, Pa, Qc, R, S, M, s));
  return kr_w_enqueue(I[n], S, R, V[n], I[n], mu, M, W, s);
}

size_t cpqr_kruskal_mttkrp_work(int N, int R, int S) {
  if (N < 2 || N > CPQR_MAX_MODES || R < 1 || R > CPQR_MAX_RANK || S < 1 || S > CPQR_MAX_KRUSKAL_TERMS) return 0;
  Carver cv(nullptr);
  cv.take<double>(size_t(N) * R * S);
  cv.take<double>(size_t(S) * R);
  return cv.bytes();
}

int cpqr_kruskal_mttkrp(int N, int n, int R, const int64_t* I, int S, const double* mu, const double* const* V,
                        const double* const* A, double* M, void* work, size_t work_bytes, void* stream) {
  CPQR_TRY(check_kruskal(N, I, S, mu, V));
  CPQR_TRY(check_rank(R));
  if (n < 0 || n >= N) return fail(CPQR_ERR_ARG, "kruskal_mttkrp: n out of range");
  if (!A || !M) return fail(CPQR_ERR_ARG, "kruskal_mttkrp: NULL pointer");
  for (int k = 0; k < N; ++k)
    if (k != n && !A[k]) return fail(CPQR_ERR_ARG, "kruskal_mttkrp: A[" + std::to_string(k) + "] is NULL");
  CPQR_TRY(check_work(work, work_bytes, cpqr_kruskal_mttkrp_work(N, R, S)));
  hipStream_t s = as_stream(stream);
  Carver cv(work);
  double* P = cv.take<double>(size_t(N) * R * S);
  double* H = cv.take<double>(size_t(S) * R);
  const double* Pa[CPQR_MAX_MODES];
  int na = 0;
  for (int k = 0; k < N; ++k) {
    if (k == n) continue;
    double* Pk = P + size_t(k) * R * S;
    CPQR_TRY(kr_cross_enqueue(I[k], R, S, A[k], I[k], V[k], I[k], Pk, s));
    Pa[na++] = Pk;
  }
  CPQR_TRY(kr_hadamard_enqueue(na, Pa, R, S, H, s));
  return kr_w_enqueue(I[n], S, R, V[n], I[n], mu, H, M, s);
}

size_t cpqr_kruskal_norm2_work(int S) {
  if (S < 1 || S > CPQR_MAX_KRUSKAL_TERMS) return 0;
  return kr_norm2_work(S);
}

int cpqr_kruskal_norm2(int N, const int64_t* I, int S, const double* mu, const double* const* V, double* out,
                       void* work, size_t work_bytes, void* stream) {
  CPQR_TRY(check_kruskal(N, I, S, mu, V));
  if (!out) return fail(CPQR_ERR_ARG, "kruskal_norm2: out is NULL");
  CPQR_TRY(check_work(work, work_bytes, kr_norm2_work(S)));
  return kr_norm2_enqueue(N, I, S, mu, V, out, work, as_stream(stream));
}

size_t cpqr_kruskal_full_work(int N, const int64_t* I, int S) {
  if (!I || N < 2 || N > CPQR_MAX_MODES || S < 1 || S > CPQR_MAX_KRUSKAL_TERMS) return 0;
  for (int k = 0; k < N; ++k)
    if (I[k] < 1) return 0;
  return kr_full_work(N, I, S);
}

int cpqr_kruskal_full(int N, const int64_t* I, int S, const double* mu, const double* const* V, int xdtype,
                      void* X, void* work, size_t work_bytes, void* stream) {
  CPQR_TRY(check_kruskal(N, I, S, mu, V));
  if (!valid_dtype(xdtype)) return fail(CPQR_ERR_DTYPE, "kruskal_full: xdtype must be CPQR_F32 or CPQR_F64");
  if (!X) return fail(CPQR_ERR_ARG, "kruskal_full: X is NULL");
  if (kr_full_grid_y(N, I) > 65535)
    return fail(CPQR_ERR_SHAPE, "kruskal_full: the trailing modes hold more than 65535 x 64 entries");
  CPQR_TRY(check_work(work, work_bytes, kr_full_work(N, I, S)));
  return kr_full_enqueue(N, I, S, mu, V, xdtype, X, work, as_stream(stream));
}

size_t cpqr_apply_q0_chain_work(int64_t In, int N, int R) {
  if (In < 1 || N < 3 || N > CPQR_MAX_MODES || R < 1 || R > CPQR_MAX_RANK) return 0;
  return apply_chain_work(In, N, R);
}

int cpqr_apply_q0_chain(int64_t In, int N, int R, int ydtype, const void* Y, const double* Qc, double* W,
                        void* work, size_t work_bytes, void* stream) {
  if (N < 3 || N > CPQR_MAX_MODES) return fail(CPQR_ERR_SHAPE, "apply_q0_chain: N out of range (3..10)");
  CPQR_TRY(check_rank(R));
  if (In < 1) return fail(CPQR_ERR_SHAPE, "apply_q0_chain: In < 1");
  CPQR_TRY(check_krp_rows(N, R));
  if (!valid_dtype(ydtype)) return fail(CPQR_ERR_DTYPE, "apply_q0_chain: ydtype must be CPQR_F32 or CPQR_F64");
  if (!Y || !Qc || !W) return fail(CPQR_ERR_ARG, "apply_q0_chain: NULL pointer");
  CPQR_TRY(check_work(work, work_bytes, apply_chain_work(In, N, R)));
  return apply_chain_enqueue(In, N, R, ydtype, Y, Qc, W, work, as_stream(stream));
}

size_t cpqr_apply_q0_work(int64_t In, int64_t K, int R) {
  if (In < 1 || K < 1 || R < 1 || R > CPQR_MAX_RANK) return 0;
  return apply_q0_work(In, K, R);
}

int cpqr_apply_q0(int64_t In, int64_t K, int R, int ydtype, const void* Y, const double* Q0,
                  double* W, void* work, size_t work_bytes, void* stream) {
  CPQR_TRY(check_rank(R));
  if (In < 1 || K < R) return fail(CPQR_ERR_SHAPE, "apply_q0: need In >= 1 and K >= R");
  if (!valid_dtype(ydtype)) return fail(CPQR_ERR_DTYPE, "apply_q0: ydtype must be CPQR_F32 or CPQR_F64");
  if (!Y || !Q0 || !W) return fail(CPQR_ERR_ARG, "apply_q0: NULL pointer");
  CPQR_TRY(check_work(work, work_bytes, apply_q0_work(In, K, R)));
  return apply_q0_enqueue(In, K, R, ydtype, Y, Q0, W, work, as_stream(stream));
}

size_t cpqr_solve_rsvd_work(int64_t In, int R) {
  if (In < 1 || R < 1 || R > CPQR_MAX_RANK) return 0;
  return solve_work(In, R);
}

int cpqr_solve_rsvd(int64_t In, int R, const double* W, const double* R0, int use_svd, double rtol,
                    double* A, double* lambda, int* status, void* work, size_t work_bytes,
                    void* stream) {
  CPQR_TRY(check_rank(R));
  if (In < 1) return fail(CPQR_ERR_SHAPE, "solve_rsvd: In < 1");
  if (!W || !R0 || !A || !lambda) return fail(CPQR_ERR_ARG, "solve_rsvd: NULL pointer");
  if (std::isnan(rtol)) return fail(CPQR_ERR_ARG, "solve_rsvd: rtol is NaN");
  CPQR_TRY(check_work(work, work_bytes, solve_work(In, R)));
  return solve_enqueue(In, R, W, R0, use_svd, rtol, A, lambda, status, work, as_stream(stream));
}

size_t cpqr_fit_direct_work(int N, const int64_t* I, int R) {
  if (check_modes(N, I) != CPQR_OK || R < 1 || R > CPQR_MAX_RANK) return 0;
  return fit_direct_work(N, I, R);
}

int cpqr_fit_direct(int N, const int64_t* I, int xdtype, const void* X, int R, const double* lambda,
                    const double* const* A, double* out, void* work, size_t work_bytes, void* stream) {
  CPQR_TRY(check_modes(N, I));
  CPQR_TRY(check_rank(R));
  if (!valid_dtype(xdtype)) return fail(CPQR_ERR_DTYPE, "fit_direct: xdtype must be CPQR_F32 or CPQR_F64");
  if (!X || !lambda || !A || !out) return fail(CPQR_ERR_ARG, "fit_direct: NULL pointer");
  for (int k = 0; k < N; ++k)
    if (!A[k]) return fail(CPQR_ERR_ARG, "fit_direct: A[" + std::to_string(k) + "] is NULL");
  CPQR_TRY(check_work(work, work_bytes, fit_direct_work(N, I, R)));
  return fit_direct_enqueue(N, I, xdtype, X, R, lambda, A, out, work, as_stream(stream));
}

// ------------------------------------------------------------ Kruskal input
// Section 3.3.2: the sweeps of both algorithms on X = [[xmu; xV]] work on its
// factors.  P holds, per mode k, the R x S cross products with the factor
// the method contracts X with (Q_k^T V_k for Alg. 2, A_k^T V_k for Alg. 1);
// only P_n changes when mode n is updated.  Everything runs on the caller's
// stream (every step is small).
struct KrWs {
  double* xnorm2;
  double* G;  // Alg. 1: N blocks of R x R
  double* Sm;
  double* F;
  double* P;  // N blocks of R x S
  double* M;  // S x R: the chain's rows (Alg. 2) or the Hadamard product (Alg. 1)
  double* W;  // Imax x R: W_n (Alg. 2) or M_n (Alg. 1)
  double* Mn;  // Alg. 1: the MTTKRP as kept by the update (for the error)
  double* Qc;
  double* R0;
  double* fit;
  double* relerr_tmp;
  void* sub;
  double* err_part;
};

size_t kr_carve(Carver& cv, const cpqr_problem* p, bool ne, KrWs* ws) {
  const int N = p->N, R = p->R, S = p->xS;
  int64_t imax = 0;
  for (int k = 0; k < N; ++k) imax = std::max(imax, p->I[k]);
  KrWs w{};
  w.xnorm2 = cv.take<double>(1);
  w.G = cv.take<double>(ne ? size_t(N) * R * R : 0);
  w.Sm = cv.take<double>(ne ? size_t(R) * R : 0);
  w.F = cv.take<double>(ne ? size_t(R) * R : 0);
  w.P = cv.take<double>(size_t(N) * R * S);
  w.M = cv.take<double>(size_t(S) * R);
  w.W = cv.take<double>(size_t(imax) * R);
  w.Mn = cv.take<double>(ne ? size_t(imax) * R : 0);
  w.Qc = cv.take<double>(ne ? 0 : size_t(std::max(N - 2, 0)) * R * R * R);
  w.R0 = cv.take<double>(ne ? 0 : size_t(R) * R);
  w.fit = cv.take<double>(2);
  w.relerr_tmp = cv.take<double>(1);
  size_t sub = std::max(kr_norm2_work(S), ne ? ne_update_work(R) : krp_chain_work(R));
  for (int k = 0; k < N; ++k) {
    if (!ne) sub = std::max(sub, std::max(tsqr_work(p->I[k], R), solve_work(p->I[k], R)));
  }
  if (p->X) sub = std::max(sub, fit_direct_work(N, p->I, R));
  w.sub = cv.take<char>(sub);
  w.err_part = cv.take<double>(std::max(error_efficient_work(p->I[N - 1]), ne_error_work(p->I[N - 1])) /
                               sizeof(double));
  if (ws) *ws = w;
  return cv.bytes();
}

int kr_error_direct(const cpqr_problem* p, KrWs& w, double* out, hipStream_t s) {
  const double* Ap[CPQR_MAX_MODES];
  for (int k = 0; k < p->N; ++k) Ap[k] = p->A[k];
  CPQR_TRY(fit_direct_enqueue(p->N, p->I, p->xdtype, p->X, p->R, p->lambda, Ap, w.fit, w.sub, s));
  return error_from_fit_enqueue(w.fit, out, s);
}

int kr_als_init(const cpqr_problem* p, void* work, hipStream_t s) {
  KrWs w;
  Carver c2(work);
  kr_carve(c2, p, false, &w);
  const int N = p->N, R = p->R;
  for (int k = 1; k < N; ++k)
    CPQR_TRY(factor_qr_enqueue(p->I[k], R, p->A[k], p->I[k], p->Q[k], p->I[k], p->Rf[k], R, w.sub, s));
  CPQR_TRY(fill_enqueue(p->lambda, R, 1.0, s));
  return kr_norm2_enqueue(N, p->I, p->xS, p->xmu, p->xV, w.xnorm2, w.sub, s);
}

int kr_als_sweep(const cpqr_problem* p, int nsweeps, double* relerr, void* work, hipStream_t s) {
  KrWs w;
  Carver c2(work);
  kr_carve(c2, p, false, &w);
  const int N = p->N, R = p->R, S = p->xS;
  auto Pk = [&](int k) { return w.P + size_t(k) * R * S; };
  for (int k = 1; k < N; ++k)
    CPQR_TRY(kr_cross_enqueue(p->I[k], R, S, p->Q[k], p->I[k], p->xV[k], p->I[k], Pk(k), s));
  for (int sw = 0; sw < nsweeps; ++sw) {
    for (int n = 0; n < N; ++n) {
      const double* Pa[CPQR_MAX_MODES];
      int na = 0;
      for (int k = 0; k < N; ++k)
        if (k != n) Pa[na++] = Pk(k);
      {
        PhaseTimer pt(PH_Q0, s);
        if (N >= 3) {
          CPQR_TRY(krp_chain_enqueue(N, n, R, p->Rf, R, w.Qc, w.R0, w.sub, s));
        } else {  // V_n = R_{a_1} is already triangular: Q_0 = I, R_0 = R_{a_1}
          CPQR_HIP(hipMemcpyAsync(w.R0, p->Rf[1 - n], sizeof(double) * R * R, hipMemcpyDeviceToDevice, s));
        }
      }
      {
        PhaseTimer pt(PH_APPLY_Q0, s);
        CPQR_TRY(kr_chain_enqueue(na, Pa, w.Qc, R, S, w.M, s));
        CPQR_TRY(kr_w_enqueue(p->I[n], S, R, p->xV[n], p->I[n], p->xmu, w.M, w.W, s));
      }
      const bool fuse = norm_qr_fits(p->I[n], R);
      CPQR_TRY(solve_enqueue(p->I[n], R, w.W, w.R0, p->use_svd, p->rtol, p->A[n], p->lambda, p->status, w.sub,
                             s, !fuse));
      if (fuse) {
        bool done = false;
        CPQR_TRY(normalize_factor_qr_enqueue(p->I[n], R, p->A[n], p->lambda, p->status, p->Q[n], p->Rf[n], w.sub,
                                             s, nullptr, &done));
      } else {
        CPQR_TRY(factor_qr_enqueue(p->I[n], R, p->A[n], p->I[n], p->Q[n], p->I[n], p->Rf[n], R, w.sub, s));
      }
      CPQR_TRY(kr_cross_enqueue(p->I[n], R, S, p->Q[n], p->I[n], p->xV[n], p->I[n], Pk(n), s));
    }
    double* out = relerr ? relerr + sw : w.relerr_tmp;
    if (p->error_mode == CPQR_ERROR_EFFICIENT) {
      CPQR_TRY(error_efficient_enqueue(p->I[N - 1], R, w.W, p->A[N - 1], p->lambda, w.R0, p->Rf[N - 1], w.xnorm2,
                                       out, w.err_part, s));
    } else if (p->error_mode == CPQR_ERROR_DIRECT) {
      CPQR_TRY(kr_error_direct(p, w, out, s));
    } else {
      CPQR_TRY(fill_enqueue(out, 1, std::nan(""), s));
    }
  }
  return CPQR_OK;
}

int kr_ne_init(const cpqr_problem* p, void* work, hipStream_t s) {
  KrWs w;
  Carver c2(work);
  kr_carve(c2, p, true, &w);
  const int N = p->N, R = p->R;
  for (int k = 0; k < N; ++k) CPQR_TRY(gram_enqueue(p->I[k], R, p->A[k], w.G + int64_t(k) * R * R, s));
  CPQR_TRY(fill_enqueue(p->lambda, R, 1.0, s));
  return kr_norm2_enqueue(N, p->I, p->xS, p->xmu, p->xV, w.xnorm2, w.sub, s);
}

int kr_ne_sweep(const cpqr_problem* p, int nsweeps, double* relerr, void* work, hipStream_t s) {
  KrWs w;
  Carver c2(work);
  kr_carve(c2, p, true, &w);
  const int N = p->N, R = p->R, S = p->xS;
  auto Pk = [&](int k) { return w.P + size_t(k) * R * S; };
  for (int k = 0; k < N; ++k)
    CPQR_TRY(kr_cross_enqueue(p->I[k], R, S, p->A[k], p->I[k], p->xV[k], p->I[k], Pk(k), s));
  for (int sw = 0; sw < nsweeps; ++sw) {
    for (int n = 0; n < N; ++n) {
      const double* Pa[CPQR_MAX_MODES];
      int na = 0;
      for (int k = 0; k < N; ++k)
        if (k != n) Pa[na++] = Pk(k);
      {
        PhaseTimer pt(PH_MULTITTM, s);
        CPQR_TRY(kr_hadamard_enqueue(na, Pa, R, S, w.M, s));
        CPQR_TRY(kr_w_enqueue(p->I[n], S, R, p->xV[n], p->I[n], p->xmu, w.M, w.W, s));
      }
      CPQR_TRY(ne_update_from_m_enqueue(p->I[n], N, n, R, w.W, w.G, p->use_svd, p->rtol, w.Sm, w.F, w.Mn, p->A[n],
                                        p->lambda, p->status, w.sub, s));
      CPQR_TRY(kr_cross_enqueue(p->I[n], R, S, p->A[n], p->I[n], p->xV[n], p->I[n], Pk(n), s));
    }
    double* out = relerr ? relerr + sw : w.relerr_tmp;
    if (p->error_mode == CPQR_ERROR_EFFICIENT) {
      CPQR_TRY(ne_error_enqueue(p->I[N - 1], R, w.Mn, p->A[N - 1], p->lambda, w.Sm, w.G + int64_t(N - 1) * R * R,
                                w.xnorm2, out, w.err_part, s));
    } else if (p->error_mode == CPQR_ERROR_DIRECT) {
      CPQR_TRY(kr_error_direct(p, w, out, s));
    } else {
      CPQR_TRY(fill_enqueue(out, 1, std::nan(""), s));
    }
  }
  return CPQR_OK;
}

size_t cpqr_als_work(const cpqr_problem* p) {
  if (check_problem(p) != CPQR_OK) return 0;
  if (kruskal_input(p)) {
    Carver cv(nullptr);
    return kr_carve(cv, p, false, nullptr);
  }
  Carver cv(nullptr);
  return als_carve(cv, p, nullptr);
}

int cpqr_als_init(const cpqr_problem* p, void* work, size_t work_bytes, void* stream) {
  CPQR_TRY(check_problem(p));
  if (kruskal_input(p)) {
    Carver cv(nullptr);
    CPQR_TRY(check_work(work, work_bytes, kr_carve(cv, p, false, nullptr)));
    return kr_als_init(p, work, as_stream(stream));
  }
  Carver cv(nullptr);
  CPQR_TRY(check_work(work, work_bytes, als_carve(cv, p, nullptr)));
  AlsWs w;
  Carver c2(work);
  als_carve(c2, p, &w);
  hipStream_t s = as_stream(stream);
  const int N = p->N, R = p->R;
  for (int k = 1; k < N; ++k)
    CPQR_TRY(factor_qr_enqueue(p->I[k], R, p->A[k], p->I[k], p->Q[k], p->I[k], p->Rf[k], R, w.sub, s));
  CPQR_TRY(fill_enqueue(p->lambda, R, 1.0, s));
  int64_t count = 1;
  for (int k = 0; k < N; ++k) count *= p->I[k];
  return norm2_enqueue(count, p->xdtype, p->X, w.xnorm2, w.sub, s);
}

int cpqr_als_sweep(const cpqr_problem* p, int nsweeps, double* relerr, void* work, size_t work_bytes,
                   void* stream) {
  CPQR_TRY(check_problem(p));
  if (nsweeps < 0) return fail(CPQR_ERR_ARG, "nsweeps < 0");
  if (kruskal_input(p)) {
    Carver cv(nullptr);
    CPQR_TRY(check_work(work, work_bytes, kr_carve(cv, p, false, nullptr)));
    return kr_als_sweep(p, nsweeps, relerr, work, as_stream(stream));
  }
  Carver cv(nullptr);
  CPQR_TRY(check_work(work, work_bytes, als_carve(cv, p, nullptr)));
  AlsWs w;
  Carver c2(work);
  als_carve(c2, p, &w);
  if (c2.bytes() > work_bytes) return fail(CPQR_ERR_WORKSPACE, "als_sweep: workspace layout exceeds its size");
  hipStream_t s = as_stream(stream);
  const int N = p->N, R = p->R;
  const int64_t K = ipow(R, N - 1);
  const int ydt = p->prec == CPQR_PREC_F64 ? CPQR_F64 : CPQR_F32;
  SideStream side;
  CPQR_TRY(side_stream(side));
  const int h = dt_split(p);
  const bool chain = use_chain(p);
  bool r_marked = false;  // side.ready marks the last factor QR's R
  UCache uc;  // FP32 operands of the Q_k refreshed by this call's factor QRs
  uc.RP = w.urp;
  // With the dense Khatri-Rao QR (N >= 4), the last mode's V_N-1 is factored
  // as a chain (section 3.3.3 structure, older factors first): its steps up
  // to the newest factor R_{N-2} run beside the update of mode N-2, so that
  // after that mode's factor QR only one R^2 x R QR and the expansion of Q_0
  // remain before mode N-1 can apply Q_0.  For N = 4 mode 1 likewise: its
  // newest factor R_0 is the fastest index of V_1 = R_3 (.) R_2 (.) R_0, so
  // R_3 (.) R_2 = Q_a T_a is factored beside mode 0, and after R_0 only
  // T_a (.) R_0 = Q_b R_0' remains, Q_0 = (Q_a kron I) Q_b.
  const bool split = !chain && N >= 4;
  for (int sw = 0; sw < nsweeps; ++sw) {
    for (int n = 0; n < N; ++n) {
      // Khatri-Rao QR (reads R_k) on the side stream, Multi-TTM (reads Q_k)
      // on the caller's stream: the QR starts as soon as the previous factor
      // QR has its R (its Q is still being formed), the Multi-TTM after it.
      if (!r_marked) CPQR_HIP(hipEventRecord(side.ready, s));
      CPQR_HIP(hipStreamWaitEvent(side.s, side.ready, 0));
      if (chain) {  // structured QR, then Q_0 formed from its factors (both on the side stream)
        CPQR_TRY(krp_chain_enqueue(N, n, R, p->Rf, R, w.Qc, w.R0, w.krp_sub, side.s));
        CPQR_TRY(expand_q0_enqueue(N, R, w.Qc, w.Q0, w.Qx, side.s));
      } else if (split && n == N - 1) {  // the chain's last step, with the newest R, and Q_0
        CPQR_TRY(krp_chain_steps(N, n, R, p->Rf, R, w.Qc, w.R0, w.Tmid, N - 2, N - 1, w.krp_sub, side.s));
        CPQR_TRY(expand_q0_enqueue(N, R, w.Qc, w.Q0, w.Qx, side.s));
      } else if (split && N == 4 && n == 1) {  // (Q_a T_a) (.) R_0 = (Q_a kron I)(T_a (.) R_0)
        const double* fac[3] = {p->Rf[0], w.Tmid, nullptr};  // R_0's index fastest
        CPQR_TRY(krp_qr_enqueue(3, 2, R, fac, R, w.Qc + size_t(R) * R * R, w.R0, w.krp_sub, side.s));
        CPQR_TRY(expand_kron_right_enqueue(R, w.Qc, w.Qc + size_t(R) * R * R, w.Q0, side.s));
      } else {
        CPQR_TRY(krp_qr_enqueue(N, n, R, p->Rf, R, w.Q0, w.R0, w.krp_sub, side.s));
      }
      CPQR_HIP(hipEventRecord(side.done, side.s));
      if (split && n == N - 2)  // the last mode's chain up to its newest factor, off this mode's path
        CPQR_TRY(krp_chain_steps(N, N - 1, R, p->Rf, R, w.Qc, w.R0, w.Tmid, 1, N - 2, w.krp_sub, side.s));
      if (split && N == 4 && n == 0) {  // mode 1's V = R_3 (.) R_2 (.) R_0: the older part R_3 (.) R_2 = Q_a T_a
        const double* fac[3] = {p->Rf[2], p->Rf[3], nullptr};  // R_2's index fastest
        CPQR_TRY(krp_qr_enqueue(3, 2, R, fac, R, w.Qc, w.Tmid, w.krp_sub, side.s));
      }
      CPQR_TRY(ttm_for_mode(p, h, n, p->Q, w.Y, w.Wt, w.sub, s, &uc));
      CPQR_HIP(hipStreamWaitEvent(s, side.done, 0));
      // normalization and factor QR in one launch where one workgroup takes A_n
      const bool fuse = norm_qr_fits(p->I[n], R);
      CPQR_TRY(apply_solve_enqueue(p->I[n], K, R, ydt, w.Y, w.Q0, w.R0, p->use_svd, p->rtol, w.W, p->A[n],
                                   p->lambda, p->status, w.sub, s, !fuse));
      bool done = false;
      if (fuse) {
        CPQR_TRY(normalize_factor_qr_enqueue(p->I[n], R, p->A[n], p->lambda, p->status, p->Q[n], p->Rf[n], w.sub,
                                             s, side.ready, &done, w.ur[n], w.uq[n], w.urp));
      } else {
        CPQR_TRY(factor_qr_enqueue(p->I[n], R, p->A[n], p->I[n], p->Q[n], p->I[n], p->Rf[n], R, w.sub, s,
                                   side.ready));
      }
      uc.rows[n] = done ? w.ur[n] : nullptr;
      uc.quads[n] = done ? w.uq[n] : nullptr;
      r_marked = true;
    }
    double* out = relerr ? relerr + sw : w.relerr_tmp;
    if (p->error_mode == CPQR_ERROR_EFFICIENT) {
      // on the side stream, overlapping the next sweep's first Multi-TTM: the
      // next Khatri-Rao QR (which rewrites R_0) queues behind it there, and the
      // caller's stream waits for that QR before it rewrites W and lambda.  It
      // reads W, A_N, lambda and R_N, all complete once the last R is.
      CPQR_HIP(hipStreamWaitEvent(side.s, side.ready, 0));
      CPQR_TRY(error_efficient_enqueue(p->I[N - 1], R, w.W, p->A[N - 1], p->lambda, w.R0, p->Rf[N - 1],
                                       w.xnorm2, out, w.err_part, side.s));
      CPQR_HIP(hipEventRecord(side.done, side.s));
    } else if (p->error_mode == CPQR_ERROR_DIRECT) {
      const double* Ap[CPQR_MAX_MODES];
      for (int k = 0; k < N; ++k) Ap[k] = p->A[k];
      CPQR_TRY(fit_direct_enqueue(N, p->I, p->xdtype, p->X, R, p->lambda, Ap, w.fit, w.sub, s));
      CPQR_TRY(error_from_fit_enqueue(w.fit, out, s));
    } else {
      CPQR_TRY(fill_enqueue(out, 1, std::nan(""), s));
    }
  }
  // everything this call queued on the side stream completes before later
  // work on the caller's stream
  if (nsweeps > 0) CPQR_HIP(hipStreamWaitEvent(s, side.done, 0));
  return CPQR_OK;
}

size_t cpqr_als_ne_work(const cpqr_problem* p) {
  if (check_problem(p, false) != CPQR_OK) return 0;
  Carver cv(nullptr);
  return kruskal_input(p) ? kr_carve(cv, p, true, nullptr) : ne_carve(cv, p, nullptr);
}

int cpqr_als_ne_init(const cpqr_problem* p, void* work, size_t work_bytes, void* stream) {
  CPQR_TRY(check_problem(p, false));
  if (kruskal_input(p)) {
    Carver cv(nullptr);
    CPQR_TRY(check_work(work, work_bytes, kr_carve(cv, p, true, nullptr)));
    return kr_ne_init(p, work, as_stream(stream));
  }
  Carver cv(nullptr);
  CPQR_TRY(check_work(work, work_bytes, ne_carve(cv, p, nullptr)));
  NeWs w;
  Carver c2(work);
  ne_carve(c2, p, &w);
  hipStream_t s = as_stream(stream);
  const int N = p->N, R = p->R;
  for (int k = 0; k < N; ++k) CPQR_TRY(gram_enqueue(p->I[k], R, p->A[k], w.G + int64_t(k) * R * R, s));
  CPQR_TRY(fill_enqueue(p->lambda, R, 1.0, s));
  int64_t count = 1;
  for (int k = 0; k < N; ++k) count *= p->I[k];
  return norm2_enqueue(count, p->xdtype, p->X, w.xnorm2, w.sub, s);
}

int cpqr_als_ne_sweep(const cpqr_problem* p, int nsweeps, double* relerr, void* work, size_t work_bytes,
                      void* stream) {
  CPQR_TRY(check_problem(p, false));
  if (nsweeps < 0) return fail(CPQR_ERR_ARG, "nsweeps < 0");
  if (kruskal_input(p)) {
    Carver cv(nullptr);
    CPQR_TRY(check_work(work, work_bytes, kr_carve(cv, p, true, nullptr)));
    return kr_ne_sweep(p, nsweeps, relerr, work, as_stream(stream));
  }
  Carver cv(nullptr);
  CPQR_TRY(check_work(work, work_bytes, ne_carve(cv, p, nullptr)));
  NeWs w;
  Carver c2(work);
  ne_carve(c2, p, &w);
  hipStream_t s = as_stream(stream);
  const int N = p->N, R = p->R;
  const int ydt = p->prec == CPQR_PREC_F64 ? CPQR_F64 : CPQR_F32;
  const double* Ap[CPQR_MAX_MODES];
  for (int k = 0; k < N; ++k) Ap[k] = p->A[k];
  const int h = dt_split(p);
  for (int sw = 0; sw < nsweeps; ++sw) {
    for (int n = 0; n < N; ++n) {
      CPQR_TRY(ttm_for_mode(p, h, n, Ap, w.Y, w.Wt, w.sub, s, nullptr));
      CPQR_TRY(ne_update_enqueue(p->I[n], N, n, R, ydt, w.Y, w.G, p->use_svd, p->rtol, w.S, w.F, w.M, p->A[n],
                                 p->lambda, p->status, w.sub, s));
    }
    double* out = relerr ? relerr + sw : w.relerr_tmp;
    if (p->error_mode == CPQR_ERROR_EFFICIENT) {
      CPQR_TRY(ne_error_enqueue(p->I[N - 1], R, w.M, p->A[N - 1], p->lambda, w.S, w.G + int64_t(N - 1) * R * R,
                                w.xnorm2, out, w.err_part, s));
    } else if (p->error_mode == CPQR_ERROR_DIRECT) {
      CPQR_TRY(fit_direct_enqueue(N, p->I, p->xdtype, p->X, R, p->lambda, Ap, w.M, w.sub, s));
      CPQR_TRY(error_from_fit_enqueue(w.M, out, s));
    } else {
      CPQR_TRY(fill_enqueue(out, 1, std::nan(""), s));
    }
  }
  return CPQR_OK;
}

// ------------------------------------------------------------ HIP graphs
// Whole sweeps captured once into a HIP graph: one launch replays every
// kernel, copy and cross-stream dependency of the captured calls, without the
// host-side launch work and with the side-stream fork/join as graph edges.
struct cpqr_graph_t {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

int cpqr_als_graph_create(const cpqr_problem* p, int algo, int nsweeps, double* relerr, void* work,
                          size_t work_bytes, cpqr_graph* out) {
  if (!out) return fail(CPQR_ERR_ARG, "als_graph_create: out is NULL");
  *out = nullptr;
  if (algo != 0 && algo != 1) return fail(CPQR_ERR_ARG, "als_graph_create: algo must be 0 (Alg. 2) or 1 (Alg. 1)");
  if (nsweeps < 1) return fail(CPQR_ERR_ARG, "als_graph_create: nsweeps < 1");
  // the same checks as the sweep itself, before anything is captured
  CPQR_TRY(check_problem(p, algo == 0));
  {
    Carver cv(nullptr);
    const size_t need = kruskal_input(p) ? kr_carve(cv, p, algo == 1, nullptr)
                                         : (algo == 0 ? als_carve(cv, p, nullptr) : ne_carve(cv, p, nullptr));
    CPQR_TRY(check_work(work, work_bytes, need));
  }
  SideStream side;
  CPQR_TRY(side_stream(side));  // created outside the capture
  hipStream_t cap = nullptr;
  CPQR_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cap);
    return fail(CPQR_ERR_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  const int rc = algo == 0 ? cpqr_als_sweep(p, nsweeps, relerr, work, work_bytes, cap)
                           : cpqr_als_ne_sweep(p, nsweeps, relerr, work, work_bytes, cap);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(cap, &g);
  (void)hipStreamDestroy(cap);
  if (rc != CPQR_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(CPQR_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(CPQR_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  cpqr_graph h = new cpqr_graph_t;
  h->graph = g;
  h->exec = ex;
  *out = h;
  return CPQR_OK;
}

int cpqr_graph_launch(cpqr_graph g, void* stream) {
  if (!g || !g->exec) return fail(CPQR_ERR_ARG, "graph_launch: NULL graph");
  CPQR_HIP(hipGraphLaunch(g->exec, as_stream(stream)));
  return CPQR_OK;
}

int cpqr_graph_destroy(cpqr_graph g) {
  if (!g) return CPQR_OK;
  if (g->exec) CPQR_HIP(hipGraphExecDestroy(g->exec));
  if (g->graph) CPQR_HIP(hipGraphDestroy(g->graph));
  delete g;
  return CPQR_OK;
}

int cpqr_timing_enable(int on) {
  TimingState& t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  t.on = on != 0;
  return CPQR_OK;
}

int cpqr_timing_select(unsigned mask) {
  TimingState& t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  t.mask = mask;
  return CPQR_OK;
}

int cpqr_timing_reset(void) {
  TimingState& t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  for (auto& pe : t.pending) {
    (void)hipEventSynchronize(pe.b);
    t.pool.push_back(pe.a);
    t.pool.push_back(pe.b);
  }
  t.pending.clear();
  for (int i = 0; i < CPQR_NPHASES; ++i) {
    t.ms[i] = 0.0;
    t.count[i] = 0;
  }
  return CPQR_OK;
}

int cpqr_timing_read(double* ms, int64_t* counts, int nphases) {
  TimingState& t = timing();
  std::lock_guard<std::mutex> g(t.mu);
  for (auto& pe : t.pending) {
    CPQR_HIP(hipEventSynchronize(pe.b));
    float el = 0.f;
    CPQR_HIP(hipEventElapsedTime(&el, pe.a, pe.b));
    t.ms[pe.phase] += el;
    t.count[pe.phase] += 1;
    t.pool.push_back(pe.a);
    t.pool.push_back(pe.b);
  }
  t.pending.clear();
  for (int i = 0; i < nphases && i < CPQR_NPHASES; ++i) {
    if (ms) ms[i] = t.ms[i];
    if (counts) counts[i] = t.count[i];
  }
  return CPQR_OK;
}

}  // extern "C"
