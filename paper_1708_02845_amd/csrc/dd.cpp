// Host side of the C ABI declared in include/dd.h.
#include "dd.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "dd_internal.h"

namespace {

constexpr uint32_t kCtxMagic = 0xDD0C7A11u;
constexpr uint32_t kKernelMagic = 0xDD0E4E11u;
constexpr uint32_t kDead = 0xDEADDEADu;
constexpr double kU = 5.9604644775390625e-08;   // 2^-24, FP32 unit roundoff
constexpr int kMaxDegree = 64;
// a truncated handle takes the many-target pass from this many targets up
constexpr int32_t kCsrBatchMin = 8;
constexpr int32_t kMaxB = 16384;                // the target row must fit in LDS

thread_local std::string g_err;

dd_status fail(dd_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_OR(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(DD_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),      \
                  __FILE__, __LINE__);                                                    \
  } while (0)

// Device allocation owned by a handle.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);   // a destructor has no caller to report to
    p = nullptr;
    bytes = 0;
  }
  hipError_t alloc(size_t n) {
    release();
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// Stream-ordered scratch, freed on the same stream when it goes out of scope.
struct AsyncBuf {
  void* p = nullptr;
  hipStream_t s = nullptr;
  explicit AsyncBuf(hipStream_t st) : s(st) {}
  ~AsyncBuf() {
    if (p) (void)hipFreeAsync(p, s);   // stream-ordered after the launches that use it
  }
  hipError_t alloc(size_t n) { return hipMallocAsync(&p, n ? n : 1, s); }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Device scratch of one batch call: stream-ordered allocations freed on the
// same stream when the object goes out of scope, or, with a fixed buffer,
// consecutive 256-byte-aligned slices of it (the caller has checked the total
// against the buffer's size first).
class CallScratch {
 public:
  CallScratch(hipStream_t s, unsigned char* fixed) : s_(s), fixed_(fixed) {}
  ~CallScratch() {
    for (void* p : owned_) (void)hipFreeAsync(p, s_);
  }
  CallScratch(const CallScratch&) = delete;
  CallScratch& operator=(const CallScratch&) = delete;
  hipError_t get(size_t n, void** p) {
    if (fixed_) {
      if (used_ + align256(n) > dd::kFixedScratchBytes) return hipErrorOutOfMemory;
      *p = fixed_ + used_;
      used_ += align256(n);
      return hipSuccess;
    }
    const hipError_t e = hipMallocAsync(p, n ? n : 1, s_);
    if (e == hipSuccess) owned_.push_back(*p);
    return e;
  }

 private:
  hipStream_t s_;
  unsigned char* fixed_;
  size_t used_ = 0;
  std::vector<void*> owned_;
};

}  // namespace

struct dd_ctx {
  uint32_t magic = kCtxMagic;
  int device = 0;
  std::atomic<int> live_kernels{0};   // loads and frees may come from several threads
  void* scratch = nullptr;            // this device's fixed scratch (dd::fixed_scratch)
  double log2_ratio[2] = {0.0, 0.0};  // the device's hardware-log2 scan (check_log2_bound)
  int l1_ok = 0;                      // the scan passed
  int l1_on = 0;                      // level-1 re-decisions in KL walks
};

struct dd_kernel {
  uint32_t magic = kKernelMagic;
  dd_ctx* ctx = nullptr;
  int32_t N = 0, B_in = 0, B = 0;
  int64_t ld = 0;    // row stride of the streaming form (multiple of 4)
  int64_t lda = 0;   // row stride of the batched-KL operand (multiple of 64)
  int is_f64 = 0;
  int is_csr = 0;
  int gemm_form = DD_FORM_NONE;
  double tau = 0.0;
  int tau_relative = 1;
  // dense
  DevBuf P32, P64, H;
  std::vector<double> H_host;   // sum_b P_xb log P_xb per row (FP64)
  std::vector<double> W_host;   // row sums
  // batched-KL operand
  DevBuf L32, Lhi, Llo, Off;
  double omax = 0.0;   // max_x o_x (FP32 offsets as used)
  double lfloor = 0.0; // truncated handles: max_x (o_x - log phi_x) >= |l_xb| of the floored operand
  // truncated
  DevBuf start, len, col, val, val64, phi, lphi;
  DevBuf val16, rsc;   // FP16 form of the stored values and 2^-e_x per row
  int csr_values = DD_CSR_F32;
  double qmax = 0.0;   // max_x of the stored row sums
  int32_t max_len = 0; // most entries stored in one row
  int64_t nnz = 0;
  std::vector<double> Ht_host, Wt_host;   // per row over the stored entries
  double lphi_absmax = 0.0;               // max_x |log2 phi_x|
  // adjacency
  DevBuf adj;          // [N][adj_w] int32, -1 padded
  int32_t adj_w = 0;
  int has_adj = 0;
  // triangle mesh of the interior (triangle-based paths)
  DevBuf mesh_faces, mesh_xy, mesh_vf;
  int32_t mesh_F = 0, mesh_vf_w = 0;
  int has_mesh = 0;

  size_t footprint() const {
    return P32.bytes + P64.bytes + H.bytes + L32.bytes + Lhi.bytes + Llo.bytes + Off.bytes +
           start.bytes + len.bytes + col.bytes + val.bytes + val64.bytes + phi.bytes + lphi.bytes +
           val16.bytes + rsc.bytes +
           adj.bytes + mesh_faces.bytes + mesh_xy.bytes + mesh_vf.bytes;
  }
  dd::DenseView dense() const {
    return dd::DenseView{P32.as<const float>(), P64.as<const double>(), ld, N, B};
  }
  dd::CsrView csr() const {
    return dd::CsrView{start.as<const int64_t>(), len.as<const int32_t>(),
                       col.as<const uint16_t>(),  val.as<const float>(),
                       val64.as<const double>(),  phi.as<const double>(),
                       lphi.as<const double>(),   val16.as<const uint16_t>(),
                       rsc.as<const float>(),     N, B};
  }
};

namespace {

bool ctx_ok(const dd_ctx* c) { return c && c->magic == kCtxMagic; }
bool kernel_ok(const dd_kernel* k) { return k && k->magic == kKernelMagic && ctx_ok(k->ctx); }

dd_load_opts default_opts() {
  dd_load_opts o;
  o.gemm_form = DD_FORM_NONE;
  o.tau = 0.0;
  o.tau_relative = 1;
  o.validate = 1;
  o.csr_values = DD_CSR_F32;
  return o;
}

dd_status check_adjacency(int32_t N, const dd_adjacency* adj) {
  if (!adj) return DD_OK;
  if (adj->n != N) return fail(DD_EINVAL, "adjacency has n=%d, kernel has N=%d", adj->n, N);
  if (!adj->row_ptr || (!adj->col && adj->row_ptr[N] > 0))
    return fail(DD_EINVAL, "adjacency arrays are null");
  if (adj->row_ptr[0] != 0) return fail(DD_EINVAL, "adjacency row_ptr[0] != 0");
  for (int32_t v = 0; v < N; ++v) {
    const int64_t b = adj->row_ptr[v], e = adj->row_ptr[v + 1];
    if (e < b) return fail(DD_EINVAL, "adjacency row_ptr decreases at %d", v);
    if (e - b > kMaxDegree)
      return fail(DD_EINVAL, "vertex %d has %lld neighbours (max %d)", v, (long long)(e - b),
                  kMaxDegree);
    for (int64_t i = b; i < e; ++i) {
      const int32_t u = adj->col[i];
      if (u < 0 || u >= N) return fail(DD_EINVAL, "neighbour id %d of %d out of range", u, v);
      if (u == v) return fail(DD_EINVAL, "self loop at %d", v);
      if (i > b && adj->col[i - 1] >= u)
        return fail(DD_EINVAL, "neighbours of %d not strictly ascending", v);
    }
  }
  return DD_OK;
}

// The path kernel reads a vertex's neighbours as one padded row (fewer
// dependent loads per step than row_ptr + col).
dd_status upload_adjacency(dd_kernel* k, const dd_adjacency* adj) {
  if (!adj) return DD_OK;
  int32_t w = 1;
  for (int32_t v = 0; v < k->N; ++v)
    w = std::max<int32_t>(w, (int32_t)(adj->row_ptr[v + 1] - adj->row_ptr[v]));
  std::vector<int32_t> pad((size_t)k->N * (size_t)w, -1);
  for (int32_t v = 0; v < k->N; ++v)
    for (int64_t i = adj->row_ptr[v]; i < adj->row_ptr[v + 1]; ++i)
      pad[(size_t)v * w + (size_t)(i - adj->row_ptr[v])] = adj->col[i];
  HIP_OR(k->adj.alloc(sizeof(int32_t) * pad.size()));
  HIP_OR(hipMemcpy(k->adj.p, pad.data(), sizeof(int32_t) * pad.size(), hipMemcpyHostToDevice));
  k->adj_w = w;
  k->has_adj = 1;
  return DD_OK;
}

size_t dense_bytes(int64_t N, int64_t B, int is_f64, const dd_load_opts& o) {
  const int64_t ld = (B + 3) & ~int64_t(3);
  const int64_t lda = (B + 63) & ~int64_t(63);
  size_t b = (size_t)(N * ld * 4) + (size_t)N * 8;
  if (is_f64) b += (size_t)(N * B * 8);
  if (o.gemm_form == DD_FORM_F32 || o.gemm_form == DD_FORM_F16X3 || o.gemm_form == DD_FORM_BF16X3)
    b += (size_t)(dd::gemm_rows_padded(N) * lda * 4) + (size_t)N * 4;
  if (o.gemm_form == DD_FORM_F16) b += (size_t)(dd::gemm_rows_padded(N) * lda * 2) + (size_t)N * 4;
  return b;
}

dd_status check_free(size_t need) {
  size_t free_b = 0, total_b = 0;
  HIP_OR(hipMemGetInfo(&free_b, &total_b));
  if (need > free_b)
    return fail(DD_ENOMEM, "needs %zu bytes of device memory, %zu free", need, free_b);
  return DD_OK;
}

// Kinds a handle can evaluate: all four on a dense handle, TV and KL on a
// truncated one.
dd_status check_kind(const dd_kernel* k, int32_t kind) {
  if (kind == DD_TV || kind == DD_KL) return DD_OK;
  if (kind == DD_CHI2 || kind == DD_HELLINGER || (kind >= DD_KIND_POWER(1) && kind <= DD_KIND_POWER(16)) ||
      (kind >= DD_KIND_ALPHA_EIGHTHS(-7) && kind <= DD_KIND_ALPHA_EIGHTHS(7))) {
    if (k->is_csr) return fail(DD_EINVAL, "kind %d needs a dense handle", kind);
    return DD_OK;
  }
  return fail(DD_EINVAL, "unknown kind %d", kind);
}

// FP16 storage of a truncated handle's values (DD_CSR_F16): every stored
// value, target row included, moves by at most eps = 2^-11 + 2^-24 of itself
// (FP16 rounding of the FP32 value, itself within 2^-24 of an FP64 input).
//   TV: sum |q - p| moves by at most eps (Q_x + W_t) <= eps (Qmax + W_t).
//   KL: p (log p - log q) moves by at most eps p |log(p/q)| + 2.002 eps p, and
//       sum_{S_t} p |log(p/q)| <= d + 2 sum_{q > p} (q - p) <= d + 2 Qmax
//       (p log(q/p) <= q - p), so eps d + eps (2 Qmax + 2.002 W_t).
void add_f16_storage(const dd_kernel* k, int kind, double W, dd_error_bound& b) {
  if (k->csr_values != DD_CSR_F16) return;
  const double eps = std::ldexp(1.0, -11) + kU;
  if (kind == DD_TV) {
    b.abs += eps * (k->qmax + W);
  } else {
    b.rel += eps;
    b.abs += eps * (2.0 * k->qmax + 2.002 * W);
  }
}

// Error bound of a field, in the sense of include/dd.h.  u is the FP32 unit
// roundoff; hardware log2 is taken to be within 4u*|log2 y| + 4u of log2 y.
dd_error_bound field_bound(const dd_kernel* k, int kind, int32_t t) {
  dd_error_bound b;
  if (!k->is_csr) {
    const double H = std::fabs(k->H_host[t]);
    const double W = k->W_host[t];
    if (kind == DD_TV) {
      b.rel = 6.0 * kU;
      b.abs = (k->is_f64 ? 2.0 * kU * (1.0 + W) : 0.0) + 1e-300;
    } else if (kind == DD_CHI2) {
      // terms (q - p) * ((q - p) * fl(1/p)): 5u each, 4-term FP32 sums 2u,
      // output rounding u.  FP32 copies of FP64 rows move each term by at
      // most (2|q - p| u (q + p) + u (q - p)^2) / p; Cauchy-Schwarz with
      // sum (q + p)^2 / p = chi2 + 4 sum q bounds the sum by 3u chi2 + 4u.
      b.rel = 8.0 * kU + (k->is_f64 ? 3.0 * kU : 0.0);
      b.abs = (k->is_f64 ? 4.0 * kU : 0.0) + 1e-300;
    } else if (kind >= DD_KIND_POWER(1) && kind <= DD_KIND_POWER(16)) {
      // |d| (|d| r)^(k-1), r = fl(1/p): about 4u per factor, sums 2u, output u.
      // FP32 copies of FP64 rows move a term by at most k u (q + p) (|d|/p)^(k-1),
      // in sum k u (2 d_(k-1) + d_k) <= k u (3 d + 2 W) (Hoelder).
      const double kk = (double)(kind - DD_KIND_POWER(0));
      b.rel = (4.0 * kk + 3.0) * kU + (k->is_f64 ? 3.0 * kk * kU : 0.0);
      b.abs = (k->is_f64 ? 2.0 * kk * kU * W : 0.0) + 1e-300;
    } else if (kind >= DD_KIND_ALPHA_EIGHTHS(-7) && kind <= DD_KIND_ALPHA_EIGHTHS(7)) {
      // p (1 - z^j), z = (q fl(1/p))^(1/16) by four 1-ulp square roots, z^j by
      // squaring: (4j + 7)u relative on p z^j, whose sum is at most
      // (1 - s) W + s sum q <= W + 1 (weighted AM-GM), times 4/(1 - alpha^2).
      const int j = kind - DD_KIND_ALPHA_EIGHTHS(-8);
      const double al = (double)(kind - DD_KIND_ALPHA_EIGHTHS(0)) / 8.0;
      const double c = 4.0 / (1.0 - al * al);
      b.rel = 2.0 * kU;
      b.abs = c * ((4.0 * j + 7.0) * kU * (W + 1.0) + 3.0 * kU) +
              (k->is_f64 ? 2.0 * c * kU * (W + 1.0) : 0.0);
    } else if (kind == DD_HELLINGER) {
      // ((q - p) * rcp(sqrt q + sqrt p))^2 with 1-ulp hardware sqrt and rcp:
      // 15u per term, sums 2u, output u.  FP32 copies of FP64 rows move a
      // term by at most u |q - p|, in sum u (1 + W).
      b.rel = 18.0 * kU;
      b.abs = (k->is_f64 ? 2.0 * kU * (1.0 + W) : 0.0) + 1e-300;
    } else {
      b.rel = 11.0 * kU;
      b.abs = 18.0 * kU * H + 6.0 * kU * W + (k->is_f64 ? kU * (W + 2.0 * H) : 0.0);
    }
  } else {
    const double H = std::fabs(k->Ht_host[t]);
    const double W = k->Wt_host[t];
    if (kind == DD_TV) {
      b.rel = 6.0 * kU;
      b.abs = 4.0 * kU * W + 1e-300;
    } else {
      b.rel = 11.0 * kU;
      b.abs = 40.0 * kU * H + 12.0 * kU * W;
    }
    add_f16_storage(k, kind, W, b);
  }
  // FP64 accumulation over B terms: negligible next to the FP32 terms, kept
  // for completeness.
  b.rel += 1e-15 * (double)k->B;
  b.abs *= 2.0;   // safety factor on the analytic estimate
  b.rel *= 2.0;
  return b;
}

// Bound of a batched-KL field from the contraction.  Every l_xb = log P_xb - o_x
// is <= 0, so Lambda(x) = sum_b p_tb |l_xb| = -sum_b p_tb l_xb
// = d(x) - H_t + o_x W_t <= d(x) + |H_t| + max(0, max_x o_x) W_t (H_t <= 0, and
// o_x <= 0 whenever the row max is at most 1):
//   F32:   operand rounding u*Lambda, 64-term FP32 partial sums 33u*Lambda;
//   F16X3: hi+lo splits of l and q (2^-22 relative each), the dropped lo*lo
//          product (2^-22), 64-term partial sums over 12 accumulations
//          (30u), FP16 subnormal floors (2^-25 per entry, scaled by 1/s_t).
dd_error_bound gemm_bound(const dd_kernel* k, int32_t t) {
  if (k->is_csr) {
    // floored operand: every |l_xb| <= lfloor, and the truncated target row
    // sums to at most W_t, so the weight of the products is at most
    // W_t lfloor; the FP32 rounding of FP64 target values adds u per term
    const double c = k->gemm_form == DD_FORM_F32 ? 35.0 : 42.0;
    const double split = k->gemm_form == DD_FORM_BF16X3 ? 3.0 * std::ldexp(1.0, -16)
                         : k->gemm_form == DD_FORM_F16 ? std::ldexp(1.0, -10) + std::ldexp(1.0, -22)
                                                        : 0.0;
    const double W = k->W_host[t];
    dd_error_bound b;
    b.rel = 2.0 * ((c + 1.0) * kU + split);
    b.abs = 2.0 * (c * kU + split + (k->val64.p ? kU : 0.0)) * W * k->lfloor;
    if (k->gemm_form == DD_FORM_F16X3)
      b.abs += 2.0 * std::ldexp(1.0, -39) * (double)k->B * std::max(88.0, k->lfloor);
    if (k->gemm_form == DD_FORM_F16)
      b.abs += 2.0 * (std::ldexp(1.0, -25) * W +
                      std::ldexp(1.0, -38) * (double)k->B * std::max(88.0, k->lfloor));
    if (k->gemm_form == DD_FORM_BF16X3)
      b.abs += 2.0 * std::ldexp(1.0, -125) * (double)k->B * (104.0 + k->lfloor + W);
    return b;
  }
  const double H = std::fabs(k->H_host[t]);
  const double W = k->W_host[t];
  // BF16X3: hi+lo of l and of q each within 2^-16 relative, the dropped
  // lo*lo product 2^-16: 3 x 2^-16 relative per term on top of the
  // accumulation (F16X3's terms are 2^-22 and inside c).  F16: l and q*s_t
  // each rounded once to FP16, 2^-11 relative each, 2^-10 + 2^-22 per term.
  const double c = k->gemm_form == DD_FORM_F32 ? 35.0 : 42.0;
  const double split = k->gemm_form == DD_FORM_BF16X3 ? 3.0 * std::ldexp(1.0, -16)
                       : k->gemm_form == DD_FORM_F16  ? std::ldexp(1.0, -10) + std::ldexp(1.0, -22)
                                                      : 0.0;
  dd_error_bound b;
  b.rel = (c + 1.0) * kU + split;
  b.abs = (c * kU + split) * (H + std::max(0.0, k->omax) * W) +
          (k->is_f64 ? kU * (W + 2.0 * H) : 0.0);
  if (k->gemm_form == DD_FORM_F16X3) b.abs += std::ldexp(1.0, -39) * (double)k->B * 88.0;
  // F16: an l below the FP16 normal range is within 2^-25 (times q <= W_t in
  // sum), a q s_t below it within 2^-25 / s_t <= 2^-38 (times |l| <= 88 per entry)
  if (k->gemm_form == DD_FORM_F16)
    b.abs += std::ldexp(1.0, -25) * W + std::ldexp(1.0, -38) * (double)k->B * 88.0;
  // BF16 subnormal floors: a lo part below 2^-126 (if flushed) loses under
  // 2^-126 times the other operand (|l| <= 104 + max(0, o_max), q <= W_t) per
  // entry
  if (k->gemm_form == DD_FORM_BF16X3)
    b.abs += std::ldexp(1.0, -125) * (double)k->B * (104.0 + std::max(0.0, k->omax) + W);
  b.abs *= 2.0;
  b.rel *= 2.0;
  return b;
}

// Fixed-point shift of the many-target TV pass: values times 2^s with every
// sum of stored values (row sums, at most qmax) times 2^s below 2^32, plus one
// unit of rounding per entry; 0 keeps the FP32 path.
int tv_shift(const dd_kernel* k) {
  if (k->qmax <= 1.75) return 31;
  if (k->qmax <= 3.5) return 30;
  return 0;
}

// Bound of a truncated field from the many-target pass.  Per chunk of 32
// columns FP32 partial sums (31u of their magnitude), then FP64.
//   TV: d = W_t + Q_x - 2M, M = sum_{S_x} min(q, p~) <= W_t: 62u W_t in FP32;
//       in fixed point (values times 2^s) the longest row's entry count
//       times 2^-s (rounding only; the sums are exact).
//   KL: d = ln2 (Hb_t - log2(phi_x) W_t - S), S = sum_{S_x} p~ g with
//       g = hw_log2(q * fl(1/phi_x)): 2u relative in the argument (2.9u
//       absolute in g), hardware log2 4u|g| + 4u, product u, partial sums
//       31u; S <= |Hb_t| + max|log2 phi| W_t since d >= 0.
dd_error_bound csr_batch_bound(const dd_kernel* k, int kind, int32_t t) {
  dd_error_bound f16;
  f16.abs = f16.rel = 0.0;
  add_f16_storage(k, kind, k->Wt_host[t], f16);
  const double H = std::fabs(k->Ht_host[t]);
  const double W = k->Wt_host[t];
  const double ln2 = 0.69314718055994530942;
  dd_error_bound b;
  b.rel = kU;
  if (kind == DD_TV && tv_shift(k) > 0)
    // fixed point: min(fix q, fix p) = fix(min(q, p)) is within 2^-(s+1) of
    // min(q, p), the integer sums are exact, d = W_t + Q_x - 2M
    b.abs = std::ldexp((double)k->max_len, -tv_shift(k));
  else if (kind == DD_TV)
    b.abs = 62.0 * kU * W;
  else
    b.abs = ln2 * 6.9 * kU * W + 36.0 * kU * (H + ln2 * k->lphi_absmax * W);
  b.abs = 2.0 * (b.abs + f16.abs) + 1e-300;
  b.rel = 2.0 * (b.rel + f16.rel);
  return b;
}

// log2 of each row's floor, for the streaming kernel's missing-support term.
dd_status upload_log2_floor(dd_kernel* k, const std::vector<double>& phi) {
  std::vector<double> l(phi.size());
  k->lphi_absmax = 0.0;
  for (size_t i = 0; i < phi.size(); ++i) {
    l[i] = std::log2(phi[i]);
    k->lphi_absmax = std::max(k->lphi_absmax, std::fabs(l[i]));
  }
  HIP_OR(k->lphi.alloc(8 * l.size()));
  HIP_OR(hipMemcpy(k->lphi.p, l.data(), 8 * l.size(), hipMemcpyHostToDevice));
  return DD_OK;
}

// Shared tail of both load paths: truncate the dense view into CSR.
dd_status build_csr_from_dense(dd_kernel* k, dd::DenseView dv, const DevBuf& row_max) {
  const int32_t N = k->N;
  DevBuf thr, counts;
  HIP_OR(thr.alloc(sizeof(double) * (size_t)N));
  {
    std::vector<double> mx(N), th(N);
    HIP_OR(hipMemcpy(mx.data(), row_max.p, sizeof(double) * N, hipMemcpyDeviceToHost));
    for (int32_t x = 0; x < N; ++x) th[x] = k->tau_relative ? k->tau * mx[x] : k->tau;
    HIP_OR(hipMemcpy(thr.p, th.data(), sizeof(double) * N, hipMemcpyHostToDevice));
    if (dd_status s = upload_log2_floor(k, th)) return s;
  }
  HIP_OR(counts.alloc(sizeof(int32_t) * (size_t)N));
  HIP_OR(dd::launch_trunc_count(dv, thr.as<const double>(), counts.as<int32_t>(), nullptr));
  std::vector<int32_t> cnt(N);
  HIP_OR(hipMemcpy(cnt.data(), counts.p, sizeof(int32_t) * N, hipMemcpyDeviceToHost));
  std::vector<int64_t> st(N);
  int64_t pos = 0, nnz = 0;
  for (int32_t x = 0; x < N; ++x) {
    st[x] = pos;
    pos += (cnt[x] + 3) & ~3;
    nnz += cnt[x];
    if (cnt[x] == 0) return fail(DD_EINVAL, "row %d keeps no entry after truncation", x);
  }
  if (dd_status s = check_free((size_t)pos * (4 + 2 + (k->is_f64 ? 8 : 0)) + (size_t)N * 20))
    return s;
  HIP_OR(k->start.alloc(sizeof(int64_t) * N));
  HIP_OR(k->len.alloc(sizeof(int32_t) * N));
  HIP_OR(k->col.alloc(sizeof(uint16_t) * (size_t)pos));
  HIP_OR(k->val.alloc(sizeof(float) * (size_t)pos));
  if (k->is_f64) HIP_OR(k->val64.alloc(sizeof(double) * (size_t)pos));
  HIP_OR(hipMemset(k->col.p, 0, sizeof(uint16_t) * (size_t)pos));
  HIP_OR(hipMemset(k->val.p, 0, sizeof(float) * (size_t)pos));
  if (k->is_f64) HIP_OR(hipMemset(k->val64.p, 0, sizeof(double) * (size_t)pos));
  HIP_OR(hipMemcpy(k->start.p, st.data(), sizeof(int64_t) * N, hipMemcpyHostToDevice));
  HIP_OR(hipMemcpy(k->len.p, cnt.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice));
  HIP_OR(dd::launch_trunc_fill(dv, thr.as<const double>(), k->start.as<const int64_t>(),
                               k->col.as<uint16_t>(), k->val.as<float>(),
                               k->is_f64 ? k->val64.as<double>() : nullptr, nullptr));
  HIP_OR(hipDeviceSynchronize());
  k->phi.p = thr.p;
  k->phi.bytes = thr.bytes;
  thr.p = nullptr;
  thr.bytes = 0;
  k->nnz = nnz;
  k->is_csr = 1;
  return DD_OK;
}

// FP16 form of the stored values (DD_CSR_F16): row x scaled by 2^e_x with
// its max in [2^14, 2^15), so every kept value (>= phi_x >= 2^-28 max) is an
// FP16 normal number.  rowmax: the max stored value of each row.
dd_status build_csr_f16(dd_kernel* k, const std::vector<double>& rowmax,
                        const std::vector<double>& phi) {
  const int32_t N = k->N;
  std::vector<float> rs(N);
  for (int32_t x = 0; x < N; ++x) {
    if (!(rowmax[x] >= std::ldexp(1.0, -100)))
      return fail(DD_EINVAL, "FP16 values: row %d has max %g below 2^-100", x, rowmax[x]);
    if (!(phi[x] >= std::ldexp(rowmax[x], -28)))
      return fail(DD_EINVAL, "FP16 values: row %d keeps entries below 2^-28 of its max", x);
    int E = 0;
    (void)std::frexp(rowmax[x], &E);   // rowmax in [2^(E-1), 2^E)
    rs[x] = std::ldexp(1.0f, E - 15);  // 2^-e_x with e_x = 15 - E
  }
  const size_t pos = k->col.bytes / sizeof(uint16_t);
  HIP_OR(k->rsc.alloc(sizeof(float) * (size_t)N));
  HIP_OR(k->val16.alloc(sizeof(uint16_t) * pos));
  HIP_OR(hipMemcpy(k->rsc.p, rs.data(), sizeof(float) * (size_t)N, hipMemcpyHostToDevice));
  HIP_OR(hipMemset(k->val16.p, 0, sizeof(uint16_t) * pos));
  HIP_OR(dd::launch_csr_f16(k->start.as<const int64_t>(), k->len.as<const int32_t>(),
                            k->val.as<const float>(), k->rsc.as<const float>(), N,
                            k->val16.as<uint16_t>(), nullptr));
  HIP_OR(hipDeviceSynchronize());
  k->csr_values = DD_CSR_F16;
  return DD_OK;
}

// Per-row W and H over the stored entries of a CSR handle (host copies).
dd_status csr_row_constants(dd_kernel* k, std::vector<double>* rowmax) {
  const int32_t N = k->N;
  std::vector<int64_t> st(N);
  std::vector<int32_t> ln(N);
  HIP_OR(hipMemcpy(st.data(), k->start.p, sizeof(int64_t) * N, hipMemcpyDeviceToHost));
  HIP_OR(hipMemcpy(ln.data(), k->len.p, sizeof(int32_t) * N, hipMemcpyDeviceToHost));
  const size_t total = k->val.bytes / sizeof(float);
  std::vector<double> v(total);
  if (k->is_f64) {
    HIP_OR(hipMemcpy(v.data(), k->val64.p, sizeof(double) * total, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> f(total);
    HIP_OR(hipMemcpy(f.data(), k->val.p, sizeof(float) * total, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < total; ++i) v[i] = f[i];
  }
  k->Ht_host.assign(N, 0.0);
  k->Wt_host.assign(N, 0.0);
  k->qmax = 0.0;
  k->max_len = 0;
  if (rowmax) rowmax->assign(N, 0.0);
  for (int32_t x = 0; x < N; ++x) {
    k->max_len = std::max(k->max_len, ln[x]);
    double w = 0.0, h = 0.0, m = 0.0;
    for (int32_t i = 0; i < ln[x]; ++i) {
      const double p = v[st[x] + i];
      w += p;
      m = std::max(m, p);
      if (p > 0.0) h += p * std::log(p);
    }
    k->Wt_host[x] = w;
    k->Ht_host[x] = h;
    k->qmax = std::max(k->qmax, w);
    if (rowmax) (*rowmax)[x] = m;
  }
  return DD_OK;
}

dd_status finish_handle(dd_kernel* k, dd_ctx* ctx, dd_kernel** out) {
  ctx->live_kernels++;
  *out = k;
  return DD_OK;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

}  // namespace

// The batched-KL operand l_xb = log P_xb - o_x in the tiled layout of form
// `form`, from the dense rows still held by k; with `floor` (device [N]),
// l_xb = log max(P_xb, phi_x) - o_x, the floored kernel of a truncated handle.
dd_status build_gemm_operand(dd_kernel* k, int form, const double* floor) {
  const int32_t N = k->N;
  k->lda = ((int64_t)k->B + 63) & ~int64_t(63);
  DevBuf zeros;
  hipError_t e = zeros.alloc(4);
  if (!e) e = hipMemset(zeros.p, 0, 4);
  if (!e) e = k->Off.alloc(4 * (size_t)N);
  const size_t elems = (size_t)dd::gemm_rows_padded(N) * (size_t)k->lda;
  if (!e && form == DD_FORM_F32) {
    e = k->L32.alloc(4 * elems);
    if (!e) e = hipMemset(k->L32.p, 0, 4 * elems);
  }
  if (!e && form != DD_FORM_F32) {
    e = k->Lhi.alloc(2 * elems);
    if (!e) e = hipMemset(k->Lhi.p, 0, 2 * elems);
  }
  if (!e && (form == DD_FORM_F16X3 || form == DD_FORM_BF16X3)) {
    e = k->Llo.alloc(2 * elems);
    if (!e) e = hipMemset(k->Llo.p, 0, 2 * elems);
  }
  if (!e) e = dd::launch_log_forms(k->dense(), form, k->lda, k->L32.as<float>(),
                                   k->Lhi.as<uint16_t>(), k->Llo.as<uint16_t>(),
                                   k->Off.as<float>(), zeros.as<int32_t>(), floor, nullptr);
  if (!e) e = hipDeviceSynchronize();
  if (e) return fail(DD_EDEVICE, "log-kernel operand: %s", hipGetErrorString(e));
  int32_t nzero = 0;
  if (hipMemcpy(&nzero, zeros.p, 4, hipMemcpyDeviceToHost))
    return fail(DD_EDEVICE, "copy of the zero count failed");
  if (nzero > 0)
    return fail(DD_EINVAL,
                "%d rows hold a zero entry in a non-zero column: log P is not finite "
                "there, so the batched-KL operand cannot be built",
                nzero);
  // the largest row offset o_x (<= 0 for rows whose max is at most 1),
  // used by the error bound of the contraction
  std::vector<float> off(N);
  if (hipMemcpy(off.data(), k->Off.p, 4 * (size_t)N, hipMemcpyDeviceToHost))
    return fail(DD_EDEVICE, "copy of the row offsets failed");
  k->omax = -std::numeric_limits<double>::infinity();
  for (int32_t x = 0; x < N; ++x) k->omax = std::max(k->omax, (double)off[x]);
  if (floor) {
    std::vector<double> phi(N);
    if (hipMemcpy(phi.data(), floor, 8 * (size_t)N, hipMemcpyDeviceToHost))
      return fail(DD_EDEVICE, "copy of the floors failed");
    k->lfloor = 0.0;
    for (int32_t x = 0; x < N; ++x)
      k->lfloor = std::max(k->lfloor, (double)off[x] - std::log(phi[x]));
  }
  k->gemm_form = form;
  return DD_OK;
}

extern "C" {

const char* dd_last_error(void) { return g_err.c_str(); }

dd_status dd_create(int device, dd_ctx** out) {
  if (!out) return fail(DD_EINVAL, "out is null");
  int n = 0;
  HIP_OR(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(DD_EINVAL, "device %d of %d", device, n);
  HIP_OR(hipSetDevice(device));
  HIP_OR(dd::init_log_table());
  void* fixed = nullptr;
  HIP_OR(dd::fixed_scratch(device, &fixed));
  // the hardware log2 scan, once per device per process
  static std::mutex scan_mu;
  static std::unordered_map<int, std::pair<double, double>> scans;
  std::pair<double, double> r;
  {
    std::lock_guard<std::mutex> lk(scan_mu);
    auto it = scans.find(device);
    if (it == scans.end()) {
      double rr[2];
      HIP_OR(dd::check_log2_bound(rr));
      it = scans.emplace(device, std::make_pair(rr[0], rr[1])).first;
    }
    r = it->second;
  }
  dd_ctx* c = new (std::nothrow) dd_ctx;
  if (!c) return fail(DD_ENOMEM, "host allocation failed");
  c->device = device;
  c->scratch = fixed;
  c->log2_ratio[0] = r.first;
  c->log2_ratio[1] = r.second;
  c->l1_ok = r.first <= 1.0 ? 1 : 0;
  c->l1_on = c->l1_ok;
  *out = c;
  return DD_OK;
}

dd_status dd_destroy(dd_ctx* ctx) {
  if (!ctx_ok(ctx)) return fail(DD_ESTATE, "not a live context");
  if (ctx->live_kernels > 0)
    return fail(DD_ESTATE, "%d kernels still loaded in this context", ctx->live_kernels.load());
  ctx->magic = kDead;
  delete ctx;
  return DD_OK;
}

dd_status dd_path_level1(dd_ctx* ctx, int enable, int* enabled, double* ratios) {
  if (!ctx_ok(ctx)) return fail(DD_ESTATE, "not a live context");
  if (enable != -1 && enable != 0 && enable != 1)
    return fail(DD_EINVAL, "enable must be -1, 0 or 1, not %d", enable);
  if (enable == 1 && !ctx->l1_ok)
    return fail(DD_EINVAL, "the hardware log2 of device %d exceeds the level-1 bound (ratio %g)",
                ctx->device, ctx->log2_ratio[0]);
  if (enable >= 0) ctx->l1_on = enable;
  if (enabled) *enabled = ctx->l1_on;
  if (ratios) {
    ratios[0] = ctx->log2_ratio[0];
    ratios[1] = ctx->log2_ratio[1];
  }
  return DD_OK;
}

dd_status dd_dense_footprint(int32_t N, int32_t B, int32_t p_is_f64, const dd_load_opts* opts,
                             size_t* hbm_bytes) {
  if (N <= 0 || B <= 0 || !hbm_bytes) return fail(DD_EINVAL, "bad sizes or null output");
  const dd_load_opts o = opts ? *opts : default_opts();
  *hbm_bytes = dense_bytes(N, B, p_is_f64, o);
  return DD_OK;
}

dd_status dd_load_kernel_dense(dd_ctx* ctx, int32_t N, int32_t B, const void* P, int32_t p_is_f64,
                               int32_t p_on_device, const dd_adjacency* adj,
                               const dd_load_opts* opts, dd_kernel** out) {
  if (!ctx_ok(ctx)) return fail(DD_ESTATE, "not a live context");
  if (!out || !P) return fail(DD_EINVAL, "null argument");
  if (N <= 0 || B <= 0) return fail(DD_EINVAL, "N=%d B=%d must be positive", N, B);
  if (B > kMaxB) return fail(DD_EINVAL, "B=%d exceeds the supported %d columns", B, kMaxB);
  const dd_load_opts o = opts ? *opts : default_opts();
  if (o.gemm_form != DD_FORM_NONE && o.gemm_form != DD_FORM_F32 && o.gemm_form != DD_FORM_F16X3 &&
      o.gemm_form != DD_FORM_BF16X3 && o.gemm_form != DD_FORM_F16)
    return fail(DD_EINVAL, "unknown gemm_form %d", o.gemm_form);
  if (!(o.tau >= 0.0) || !std::isfinite(o.tau) || o.tau > 1.0)
    return fail(DD_EINVAL, "tau must be in [0, 1]");
  if (o.tau > 0.0 && o.gemm_form != DD_FORM_NONE && o.csr_values != DD_CSR_F32)
    return fail(DD_EINVAL, "the floored batched-KL operand needs FP32 stored values");
  if (o.csr_values != DD_CSR_F32 && o.csr_values != DD_CSR_F16)
    return fail(DD_EINVAL, "unknown csr_values %d", o.csr_values);
  if (dd_status s = check_adjacency(N, adj)) return s;
  HIP_OR(hipSetDevice(ctx->device));

  const size_t elt = p_is_f64 ? 8 : 4;
  const size_t raw_bytes = (size_t)N * (size_t)B * elt;
  if (dd_status s = check_free(dense_bytes(N, B, p_is_f64, o) + (p_on_device ? 0 : raw_bytes)))
    return s;

  dd_kernel* k = new (std::nothrow) dd_kernel;
  if (!k) return fail(DD_ENOMEM, "host allocation failed");
  k->ctx = ctx;
  k->N = N;
  k->B_in = B;
  k->is_f64 = p_is_f64 ? 1 : 0;
  k->tau = o.tau;
  k->tau_relative = o.tau_relative ? 1 : 0;

  auto bail = [&](dd_status s) {
    delete k;
    return s;
  };

  DevBuf raw_own;
  const void* raw = P;
  if (!p_on_device) {
    if (hipError_t e = raw_own.alloc(raw_bytes))
      return bail(fail(DD_EDEVICE, "hipMalloc(%zu): %s", raw_bytes, hipGetErrorString(e)));
    if (hipError_t e = hipMemcpy(raw_own.p, P, raw_bytes, hipMemcpyHostToDevice))
      return bail(fail(DD_EDEVICE, "upload: %s", hipGetErrorString(e)));
    raw = raw_own.p;
  }

  // row checks, row sums, row maxima, non-zero columns
  DevBuf rsum, rmax, bad, flags;
  {
    hipError_t e = rsum.alloc(8 * (size_t)N);
    if (!e) e = rmax.alloc(8 * (size_t)N);
    if (!e) e = bad.alloc(4);
    if (!e) e = flags.alloc(4 * (size_t)B);
    if (!e) e = hipMemset(bad.p, 0, 4);
    if (!e) e = hipMemset(flags.p, 0, 4 * (size_t)B);
    if (!e) e = dd::launch_row_stats(raw, k->is_f64, N, B, rsum.as<double>(), rmax.as<double>(),
                                     bad.as<int32_t>(), nullptr);
    if (!e) e = dd::launch_col_nonzero(raw, k->is_f64, N, B, flags.as<int32_t>(), nullptr);
    if (!e) e = hipDeviceSynchronize();
    if (e) return bail(fail(DD_EDEVICE, "row statistics: %s", hipGetErrorString(e)));
  }
  int32_t nbad = 0;
  std::vector<int32_t> fl(B);
  k->W_host.assign(N, 0.0);
  if (hipMemcpy(&nbad, bad.p, 4, hipMemcpyDeviceToHost) ||
      hipMemcpy(fl.data(), flags.p, 4 * (size_t)B, hipMemcpyDeviceToHost) ||
      hipMemcpy(k->W_host.data(), rsum.p, 8 * (size_t)N, hipMemcpyDeviceToHost))
    return bail(fail(DD_EDEVICE, "copy of row statistics failed"));
  if (nbad > 0)
    return bail(fail(DD_EINVAL,
                     "%d rows hold entries that are negative, not finite, or positive below "
                     "the FP32 normal range",
                     nbad));
  if (o.validate) {
    const double tol = k->is_f64 ? 1e-9 : 1e-5;
    for (int32_t x = 0; x < N; ++x)
      if (!(std::fabs(k->W_host[x] - 1.0) <= tol))
        return bail(fail(DD_EINVAL, "row %d sums to %.17g, not 1", x, k->W_host[x]));
  }
  std::vector<int32_t> kept;
  for (int32_t b = 0; b < B; ++b)
    if (fl[b]) kept.push_back(b);
  if (kept.empty()) return bail(fail(DD_EINVAL, "every column is zero"));
  k->B = (int32_t)kept.size();
  k->ld = ((int64_t)k->B + 3) & ~int64_t(3);

  // compact the kept columns into padded FP32 rows (+ FP64 master)
  {
    DevBuf kept_d;
    hipError_t e = kept_d.alloc(4 * kept.size());
    if (!e) e = hipMemcpy(kept_d.p, kept.data(), 4 * kept.size(), hipMemcpyHostToDevice);
    if (!e) e = k->P32.alloc(4 * (size_t)N * (size_t)k->ld);
    if (!e && k->is_f64) e = k->P64.alloc(8 * (size_t)N * (size_t)k->B);
    if (!e) e = dd::launch_gather_cols(raw, k->is_f64, N, B, kept_d.as<const int32_t>(), k->B,
                                       k->ld, k->P32.as<float>(),
                                       k->is_f64 ? k->P64.as<double>() : nullptr, nullptr);
    if (!e) e = hipDeviceSynchronize();
    if (e) return bail(fail(DD_EDEVICE, "column compaction: %s", hipGetErrorString(e)));
  }
  raw_own.release();

  if (o.tau > 0.0) {
    if (k->B > 65535) return bail(fail(DD_EINVAL, "CSR columns are 16-bit: B=%d", k->B));
    if (dd_status s = build_csr_from_dense(k, k->dense(), rmax)) return bail(s);
    std::vector<double> smax;
    if (dd_status s = csr_row_constants(k, &smax)) return bail(s);
    if (o.csr_values == DD_CSR_F16) {
      std::vector<double> phi(N);
      hipError_t e = hipMemcpy(phi.data(), k->phi.p, 8 * (size_t)N, hipMemcpyDeviceToHost);
      if (e) return bail(fail(DD_EDEVICE, "floor copy: %s", hipGetErrorString(e)));
      if (dd_status s = build_csr_f16(k, smax, phi)) return bail(s);
    }
    if (o.gemm_form != DD_FORM_NONE)
      if (dd_status s = build_gemm_operand(k, o.gemm_form, k->phi.as<const double>()))
        return bail(s);
    k->P32.release();
    k->P64.release();
  } else {
    hipError_t e = k->H.alloc(8 * (size_t)N);
    if (!e) e = dd::launch_row_entropy(k->dense(), k->H.as<double>(), nullptr);
    if (!e) e = hipDeviceSynchronize();
    k->H_host.assign(N, 0.0);
    if (!e) e = hipMemcpy(k->H_host.data(), k->H.p, 8 * (size_t)N, hipMemcpyDeviceToHost);
    if (e) return bail(fail(DD_EDEVICE, "row entropy: %s", hipGetErrorString(e)));
    if (o.gemm_form != DD_FORM_NONE)
      if (dd_status s = build_gemm_operand(k, o.gemm_form, nullptr)) return bail(s);
  }
  if (dd_status s = upload_adjacency(k, adj)) return bail(s);
  return finish_handle(k, ctx, out);
}

dd_status dd_load_kernel_csr(dd_ctx* ctx, int32_t N, int32_t B, const int64_t* row_ptr,
                             const int32_t* col, const void* val, int32_t val_is_f64,
                             const double* row_max, double tau, int32_t tau_relative,
                             const dd_adjacency* adj, const dd_load_opts* opts,
                             dd_kernel** out) {
  if (!ctx_ok(ctx)) return fail(DD_ESTATE, "not a live context");
  if (!out || !row_ptr || !col || !val || !row_max) return fail(DD_EINVAL, "null argument");
  if (N <= 0 || B <= 0) return fail(DD_EINVAL, "N=%d B=%d must be positive", N, B);
  if (B > kMaxB) return fail(DD_EINVAL, "B=%d exceeds the supported %d columns", B, kMaxB);
  if (!(tau > 0.0) || !(tau <= 1.0)) return fail(DD_EINVAL, "tau must be in (0, 1]");
  const dd_load_opts o = opts ? *opts : default_opts();
  if (o.gemm_form != DD_FORM_NONE)
    return fail(DD_EINVAL, "a CSR load has no dense rows to build the batched-KL operand from");
  if (o.csr_values != DD_CSR_F32 && o.csr_values != DD_CSR_F16)
    return fail(DD_EINVAL, "unknown csr_values %d", o.csr_values);
  if (dd_status s = check_adjacency(N, adj)) return s;
  if (row_ptr[0] != 0) return fail(DD_EINVAL, "row_ptr[0] != 0");
  std::vector<int64_t> st(N);
  std::vector<int32_t> ln(N);
  int64_t pos = 0;
  for (int32_t x = 0; x < N; ++x) {
    const int64_t b = row_ptr[x], e = row_ptr[x + 1];
    if (e <= b) return fail(DD_EINVAL, "row %d is empty or row_ptr decreases", x);
    if (!(row_max[x] > 0.0) || !std::isfinite(row_max[x]))
      return fail(DD_EINVAL, "row_max[%d] must be positive and finite", x);
    for (int64_t i = b; i < e; ++i) {
      const int32_t c = col[i];
      const double v = val_is_f64 ? static_cast<const double*>(val)[i]
                                  : (double)static_cast<const float*>(val)[i];
      if (c < 0 || c >= B) return fail(DD_EINVAL, "column %d of row %d out of range", c, x);
      if (i > b && col[i - 1] >= c)
        return fail(DD_EINVAL, "columns of row %d not strictly ascending", x);
      if (!(v > 0.0) || !std::isfinite(v) || v < 1.17549435e-38)
        return fail(DD_EINVAL, "stored value of row %d must be positive, finite, FP32-normal", x);
    }
    st[x] = pos;
    ln[x] = (int32_t)(e - b);
    pos += (ln[x] + 3) & ~3;
  }
  HIP_OR(hipSetDevice(ctx->device));
  if (dd_status s = check_free((size_t)pos * (6 + (val_is_f64 ? 8 : 0)) + (size_t)N * 20))
    return s;
  dd_kernel* k = new (std::nothrow) dd_kernel;
  if (!k) return fail(DD_ENOMEM, "host allocation failed");
  k->ctx = ctx;
  k->N = N;
  k->B_in = B;
  k->B = B;
  k->is_f64 = val_is_f64 ? 1 : 0;
  k->is_csr = 1;
  k->tau = tau;
  k->tau_relative = tau_relative ? 1 : 0;
  k->nnz = row_ptr[N];
  std::vector<uint16_t> colp((size_t)pos, 0);
  std::vector<float> valp((size_t)pos, 0.f);
  std::vector<double> val64p(val_is_f64 ? (size_t)pos : 0, 0.0);
  std::vector<double> phi(N), smax(N, 0.0);
  k->Ht_host.assign(N, 0.0);
  k->Wt_host.assign(N, 0.0);
  for (int32_t x = 0; x < N; ++x) {
    double w = 0.0, h = 0.0;
    for (int32_t i = 0; i < ln[x]; ++i) {
      const int64_t src = row_ptr[x] + i;
      const double v = val_is_f64 ? static_cast<const double*>(val)[src]
                                  : (double)static_cast<const float*>(val)[src];
      colp[st[x] + i] = (uint16_t)col[src];
      valp[st[x] + i] = (float)v;
      if (val_is_f64) val64p[st[x] + i] = v;
      w += v;
      h += v * std::log(v);
      smax[x] = std::max(smax[x], v);
    }
    k->Wt_host[x] = w;
    k->Ht_host[x] = h;
    k->qmax = std::max(k->qmax, w);
    k->max_len = std::max(k->max_len, ln[x]);
    phi[x] = tau_relative ? tau * row_max[x] : tau;
  }
  auto bail = [&](dd_status s) {
    delete k;
    return s;
  };
  hipError_t e = k->start.alloc(8 * (size_t)N);
  if (!e) e = k->len.alloc(4 * (size_t)N);
  if (!e) e = k->col.alloc(2 * (size_t)pos);
  if (!e) e = k->val.alloc(4 * (size_t)pos);
  if (!e && val_is_f64) e = k->val64.alloc(8 * (size_t)pos);
  if (!e) e = k->phi.alloc(8 * (size_t)N);
  if (!e) e = hipMemcpy(k->start.p, st.data(), 8 * (size_t)N, hipMemcpyHostToDevice);
  if (!e) e = hipMemcpy(k->len.p, ln.data(), 4 * (size_t)N, hipMemcpyHostToDevice);
  if (!e) e = hipMemcpy(k->col.p, colp.data(), 2 * (size_t)pos, hipMemcpyHostToDevice);
  if (!e) e = hipMemcpy(k->val.p, valp.data(), 4 * (size_t)pos, hipMemcpyHostToDevice);
  if (!e && val_is_f64) e = hipMemcpy(k->val64.p, val64p.data(), 8 * (size_t)pos, hipMemcpyHostToDevice);
  if (!e) e = hipMemcpy(k->phi.p, phi.data(), 8 * (size_t)N, hipMemcpyHostToDevice);
  if (e) return bail(fail(DD_EDEVICE, "CSR upload: %s", hipGetErrorString(e)));
  if (dd_status st = upload_log2_floor(k, phi)) return bail(st);
  if (o.csr_values == DD_CSR_F16)
    if (dd_status st = build_csr_f16(k, smax, phi)) return bail(st);
  if (dd_status s = upload_adjacency(k, adj)) return bail(s);
  return finish_handle(k, ctx, out);
}

dd_status dd_kernel_get_info(const dd_kernel* k, dd_kernel_info* info) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  if (!info) return fail(DD_EINVAL, "info is null");
  info->n = k->N;
  info->b_in = k->B_in;
  info->b = k->B;
  info->is_csr = k->is_csr;
  info->nnz = k->nnz;
  info->csr_values = k->csr_values;
  info->gemm_form = k->gemm_form;
  info->has_adjacency = k->has_adj;
  info->hbm_bytes = k->footprint();
  return DD_OK;
}

dd_status dd_distance_field(dd_kernel* k, int32_t target, int32_t kind, float* out_dev,
                            dd_error_bound* bound, void* stream) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  if (dd_status st = check_kind(k, kind)) return st;
  if (target < 0 || target >= k->N) return fail(DD_EINVAL, "target %d not in [0, %d)", target, k->N);
  if (!out_dev) return fail(DD_EINVAL, "out_dev is null");
  HIP_OR(hipSetDevice(k->ctx->device));
  if (k->is_csr)
    HIP_OR(dd::launch_csr_field(k->csr(), target, kind, out_dev, as_stream(stream)));
  else
    HIP_OR(dd::launch_dense_field(k->dense(), target, kind, out_dev, as_stream(stream)));
  if (bound) *bound = field_bound(k, kind, target);
  return DD_OK;
}

dd_status dd_distance_fields_tv_kl(dd_kernel* k, int32_t target, float* tv_dev, float* kl_dev,
                                   dd_error_bound* bounds, void* stream) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  if (target < 0 || target >= k->N) return fail(DD_EINVAL, "target %d not in [0, %d)", target, k->N);
  if (!tv_dev || !kl_dev) return fail(DD_EINVAL, "tv_dev or kl_dev is null");
  if (tv_dev == kl_dev) return fail(DD_EINVAL, "tv_dev and kl_dev are the same buffer");
  HIP_OR(hipSetDevice(k->ctx->device));
  if (k->is_csr)
    HIP_OR(dd::launch_csr_tv_kl(k->csr(), target, tv_dev, kl_dev, as_stream(stream)));
  else
    HIP_OR(dd::launch_dense_tv_kl(k->dense(), target, tv_dev, kl_dev, as_stream(stream)));
  if (bounds) {
    bounds[0] = field_bound(k, DD_TV, target);
    bounds[1] = field_bound(k, DD_KL, target);
  }
  return DD_OK;
}

namespace {

// Device scratch a batch call takes, in the order it takes it.
size_t batch_scratch_bytes(const dd_kernel* k, int32_t T, int32_t kind) {
  const int32_t tmax = std::min<int32_t>(T, dd::kMaxBatch);
  if (kind == DD_KL && k->gemm_form != DD_FORM_NONE) {
    dd::GemmView gv{nullptr, nullptr, nullptr, nullptr, k->lda, k->N, k->B, k->gemm_form};
    size_t n = align256(dd::batch_kl_workspace(gv, tmax));
    if (k->is_csr) {
      const size_t tpad = (size_t)((tmax + 63) / 64 * 64);
      n += align256(4 * tpad * (size_t)k->lda + (k->val64.p ? 8 * tpad * (size_t)k->B : 0));
    }
    return n;
  }
  if (k->is_csr && T >= kCsrBatchMin) return align256(dd::csr_batch_workspace(k->csr(), tmax));
  return 0;
}

dd_status batch_fields(dd_kernel* k, const int32_t* targets, int32_t T, int32_t kind,
                       float* out_dev, dd_error_bound* bounds, void* stream, bool fixed) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  if (dd_status st = check_kind(k, kind)) return st;
  if (T <= 0 || !targets || !out_dev) return fail(DD_EINVAL, "T=%d, targets or out_dev null", T);
  for (int32_t i = 0; i < T; ++i)
    if (targets[i] < 0 || targets[i] >= k->N)
      return fail(DD_EINVAL, "targets[%d]=%d not in [0, %d)", i, targets[i], k->N);
  if (fixed) {
    const size_t need = batch_scratch_bytes(k, T, kind);
    if (need > dd::kFixedScratchBytes)
      return fail(DD_EINVAL, "this call needs %zu bytes of scratch; the fixed buffer holds %zu",
                  need, dd::kFixedScratchBytes);
    if (!k->ctx->scratch) return fail(DD_ESTATE, "context has no fixed scratch");
  }
  HIP_OR(hipSetDevice(k->ctx->device));
  hipStream_t s = as_stream(stream);
  CallScratch scr(s, fixed ? static_cast<unsigned char*>(k->ctx->scratch) : nullptr);
  if (kind == DD_KL && k->gemm_form != DD_FORM_NONE) {
    dd::GemmView gv{k->L32.as<const float>(), k->Lhi.as<const uint16_t>(),
                    k->Llo.as<const uint16_t>(), k->Off.as<const float>(),
                    k->lda, k->N, k->B, k->gemm_form};
    // up to 256 targets per launch; each launch reads the log-kernel about once
    const int32_t tmax = std::min<int32_t>(T, dd::kMaxBatch);
    void* ws = nullptr;
    HIP_OR(scr.get(dd::batch_kl_workspace(gv, tmax), &ws));
    // a truncated handle: the truncated target rows are expanded to dense
    // rows first (FP32 [rows][lda], and FP64 [rows][B] from FP64 values);
    // the target preparation reads the first n rows of a group of n
    const int32_t tpad = (tmax + 63) / 64 * 64;
    const bool f64 = k->is_csr && k->val64.p;
    const size_t r32 = 4 * (size_t)tpad * (size_t)k->lda;
    void* rows = nullptr;
    if (k->is_csr) HIP_OR(scr.get(r32 + (f64 ? 8 * (size_t)tpad * (size_t)k->B : 0), &rows));
    for (int32_t g0 = 0; g0 < T; g0 += dd::kMaxBatch) {
      const int32_t n = std::min<int32_t>(dd::kMaxBatch, T - g0);
      dd::TargetList tl;
      std::memset(&tl, 0, sizeof tl);
      for (int32_t i = 0; i < n; ++i) tl.t[i] = targets[g0 + i];
      if (!k->is_csr) {
        HIP_OR(dd::launch_batch_kl(k->dense(), gv, tl, n, ws, out_dev + (int64_t)g0 * k->N, s));
        continue;
      }
      float* d32 = static_cast<float*>(rows);
      double* d64 = f64 ? reinterpret_cast<double*>(static_cast<unsigned char*>(rows) + r32)
                        : nullptr;
      const int32_t rows_n = (n + 63) / 64 * 64;   // <= tpad
      HIP_OR(dd::launch_csr_rows_dense(k->csr(), tl, n, rows_n, k->lda, d32, d64, s));
      dd::TargetList id;
      std::memset(&id, 0, sizeof id);
      for (int32_t i = 0; i < n; ++i) id.t[i] = i;
      const dd::DenseView dv{d32, d64, k->lda, rows_n, k->B};
      HIP_OR(dd::launch_batch_kl(dv, gv, id, n, ws, out_dev + (int64_t)g0 * k->N, s));
    }
    if (bounds)
      for (int32_t i = 0; i < T; ++i) bounds[i] = gemm_bound(k, targets[i]);
    return DD_OK;
  }
  if (k->is_csr && T >= kCsrBatchMin) {
    // one pass over the stored rows per group of up to 256 targets
    void* ws = nullptr;
    HIP_OR(scr.get(dd::csr_batch_workspace(k->csr(), std::min<int32_t>(T, dd::kMaxBatch)), &ws));
    for (int32_t g0 = 0; g0 < T; g0 += dd::kMaxBatch) {
      const int32_t n = std::min<int32_t>(dd::kMaxBatch, T - g0);
      dd::TargetList tl;
      std::memset(&tl, 0, sizeof tl);
      for (int32_t i = 0; i < n; ++i) tl.t[i] = targets[g0 + i];
      HIP_OR(dd::launch_csr_batch(k->csr(), tl, n, kind, tv_shift(k), ws,
                                  out_dev + (int64_t)g0 * k->N, s));
    }
    if (bounds)
      for (int32_t i = 0; i < T; ++i) bounds[i] = csr_batch_bound(k, kind, targets[i]);
    return DD_OK;
  }
  for (int32_t i = 0; i < T; ++i) {
    float* o = out_dev + (int64_t)i * k->N;
    if (k->is_csr)
      HIP_OR(dd::launch_csr_field(k->csr(), targets[i], kind, o, s));
    else
      HIP_OR(dd::launch_dense_field(k->dense(), targets[i], kind, o, s));
    if (bounds) bounds[i] = field_bound(k, kind, targets[i]);
  }
  return DD_OK;
}

}  // namespace

dd_status dd_batch_distance_fields(dd_kernel* k, const int32_t* targets, int32_t T, int32_t kind,
                                   float* out_dev, dd_error_bound* bounds, void* stream) {
  return batch_fields(k, targets, T, kind, out_dev, bounds, stream, false);
}

dd_status dd_batch_distance_fields_noalloc(dd_kernel* k, const int32_t* targets, int32_t T,
                                           int32_t kind, float* out_dev, dd_error_bound* bounds,
                                           void* stream) {
  static_assert(DD_NOALLOC_SCRATCH_BYTES == dd::kFixedScratchBytes,
                "the header states the fixed scratch size");
  return batch_fields(k, targets, T, kind, out_dev, bounds, stream, true);
}

namespace {

// Scratch of dd_trace_paths: [sources, targets, bounds when T is large]
// [FP64 target rows, their logs, constants].
struct PathScratch {
  bool inl;
  size_t n_small, o_row, total;
};

PathScratch path_scratch(const dd_kernel* k, int32_t T) {
  PathScratch l;
  l.inl = T <= dd::kInlinePaths;
  l.n_small = l.inl ? 0 : ((8 * (size_t)T + 15) & ~size_t(15)) + sizeof(dd::Bound) * T;
  l.o_row = align256(l.n_small);
  l.total = l.o_row + 16 * (size_t)T * (size_t)k->B + 32 * (size_t)T;
  return l;
}

}  // namespace

dd_status dd_kernel_footprint(const dd_kernel* k, size_t* hbm_bytes) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  if (!hbm_bytes) return fail(DD_EINVAL, "hbm_bytes is null");
  *hbm_bytes = k->footprint();
  return DD_OK;
}

dd_status dd_call_scratch_bytes(const dd_kernel* k, int32_t T, int32_t kind, size_t* fields_bytes,
                                size_t* paths_bytes) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  if (T <= 0) return fail(DD_EINVAL, "T=%d", T);
  if (dd_status st = check_kind(k, kind)) return st;
  if (fields_bytes) *fields_bytes = batch_scratch_bytes(k, T, kind);
  if (paths_bytes) *paths_bytes = k->has_adj ? path_scratch(k, T).total : 0;
  return DD_OK;
}

dd_status dd_trace_paths(dd_kernel* k, int32_t T, const int32_t* sources, const int32_t* targets,
                         int32_t kind, const float* fields_dev, const dd_error_bound* bounds,
                         int32_t max_steps, int32_t* path_dev, int32_t* len_dev,
                         int32_t* status_dev, int32_t* rechecks_dev, void* stream) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  if (!k->has_adj) return fail(DD_EINVAL, "kernel was loaded without adjacency");
  if (dd_status st = check_kind(k, kind)) return st;
  if (T <= 0 || !sources || !targets || !fields_dev || !bounds || !path_dev || !len_dev ||
      !status_dev)
    return fail(DD_EINVAL, "T=%d or a required pointer is null", T);
  if (max_steps < 0) return fail(DD_EINVAL, "max_steps=%d", max_steps);
  for (int32_t i = 0; i < T; ++i) {
    if (sources[i] < 0 || sources[i] >= k->N || targets[i] < 0 || targets[i] >= k->N)
      return fail(DD_EINVAL, "path %d: source %d / target %d not in [0, %d)", i, sources[i],
                  targets[i], k->N);
    if (!(bounds[i].abs >= 0.0) || !(bounds[i].rel >= 0.0))
      return fail(DD_EINVAL, "bound %d is negative or NaN", i);
  }
  HIP_OR(hipSetDevice(k->ctx->device));
  hipStream_t s = as_stream(stream);
  dd::PathArgs a;
  std::memset(&a, 0, sizeof a);
  a.adj = k->adj.as<const int32_t>();
  a.adj_w = k->adj_w;
  a.fields = fields_dev;
  a.path = path_dev;
  a.len = len_dev;
  a.status = status_dev;
  a.rechecks = rechecks_dev;
  a.T = T;
  a.max_steps = max_steps;
  a.kind = kind;
  a.is_csr = k->is_csr;
  a.l1 = k->ctx->l1_on && kind == DD_KL && !k->is_csr ? 1 : 0;
  const PathScratch lay = path_scratch(k, T);
  const bool inl = lay.inl;
  const size_t n_small = lay.n_small, o_row = lay.o_row;
  AsyncBuf ws(s);
  HIP_OR(ws.alloc(lay.total));
  unsigned char* base = ws.as<unsigned char>();
  std::vector<unsigned char> host;
  if (inl) {
    for (int32_t i = 0; i < T; ++i) {
      a.small.src[i] = sources[i];
      a.small.tgt[i] = targets[i];
      a.small.babs[i] = bounds[i].abs;
      a.small.brel[i] = bounds[i].rel;
    }
  } else {
    const size_t o_bnd = (8 * (size_t)T + 15) & ~size_t(15);
    host.resize(n_small);
    std::memcpy(host.data(), sources, 4 * (size_t)T);
    std::memcpy(host.data() + 4 * (size_t)T, targets, 4 * (size_t)T);
    for (int32_t i = 0; i < T; ++i) {
      dd::Bound b{bounds[i].abs, bounds[i].rel};
      std::memcpy(host.data() + o_bnd + sizeof(dd::Bound) * i, &b, sizeof b);
    }
    // pageable source: the copy is staged before hipMemcpyAsync returns
    HIP_OR(hipMemcpyAsync(base, host.data(), n_small, hipMemcpyHostToDevice, s));
    a.sources = reinterpret_cast<const int32_t*>(base);
    a.targets = reinterpret_cast<const int32_t*>(base + 4 * (size_t)T);
    a.bounds = reinterpret_cast<const dd::Bound*>(base + o_bnd);
  }
  {
    double* trow = reinterpret_cast<double*>(base + o_row);
    double* tlog = trow + (size_t)T * (size_t)k->B;
    double* tcon = tlog + (size_t)T * (size_t)k->B;
    HIP_OR(dd::launch_target_rows(k->dense(), k->csr(), a, trow, tlog, tcon, s));
    a.trow = trow;
    a.tlog = tlog;
    a.tconst = tcon;
  }
  HIP_OR(dd::launch_paths(k->dense(), k->csr(), a, s));
  return DD_OK;
}

dd_status dd_trace_paths_on_demand(dd_kernel* k, int32_t T, const int32_t* sources,
                                   const int32_t* targets, int32_t kind, double target_tau,
                                   int32_t target_tau_relative, int32_t max_steps,
                                   int32_t* path_dev, int32_t* len_dev, int32_t* status_dev,
                                   int32_t* evals_dev, void* stream) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  if (!k->has_adj) return fail(DD_EINVAL, "kernel was loaded without adjacency");
  if (dd_status st = check_kind(k, kind)) return st;
  if (T <= 0 || !sources || !targets || !path_dev || !len_dev || !status_dev)
    return fail(DD_EINVAL, "T=%d or a required pointer is null", T);
  if (max_steps < 0) return fail(DD_EINVAL, "max_steps=%d", max_steps);
  if (!(target_tau >= 0.0) || !std::isfinite(target_tau))
    return fail(DD_EINVAL, "target_tau=%g", target_tau);
  if (target_tau > 0.0 && (kind != DD_KL || k->is_csr))
    return fail(DD_EINVAL, "a target-row truncation needs DD_KL on a dense handle");
  for (int32_t i = 0; i < T; ++i)
    if (sources[i] < 0 || sources[i] >= k->N || targets[i] < 0 || targets[i] >= k->N)
      return fail(DD_EINVAL, "path %d: source %d / target %d not in [0, %d)", i, sources[i],
                  targets[i], k->N);
  HIP_OR(hipSetDevice(k->ctx->device));
  hipStream_t s = as_stream(stream);
  dd::PathArgs a;
  std::memset(&a, 0, sizeof a);
  a.adj = k->adj.as<const int32_t>();
  a.adj_w = k->adj_w;
  a.path = path_dev;
  a.len = len_dev;
  a.status = status_dev;
  a.rechecks = evals_dev;
  a.T = T;
  a.max_steps = max_steps;
  a.kind = kind;
  a.is_csr = k->is_csr;
  a.l1 = k->ctx->l1_on && kind == DD_KL && !k->is_csr ? 1 : 0;
  a.tgt_tau = target_tau;
  a.tgt_tau_relative = target_tau_relative ? 1 : 0;
  // scratch: [sources, targets when T is large] [FP64 target rows, logs, constants]
  const bool inl = T <= dd::kInlinePaths;
  const size_t n_small = inl ? 0 : 8 * (size_t)T;
  const size_t o_row = (n_small + 255) & ~size_t(255);
  const size_t n_row = 16 * (size_t)T * (size_t)k->B + 32 * (size_t)T;
  AsyncBuf ws(s);
  HIP_OR(ws.alloc(o_row + n_row));
  unsigned char* base = ws.as<unsigned char>();
  std::vector<int32_t> host;
  if (inl) {
    for (int32_t i = 0; i < T; ++i) {
      a.small.src[i] = sources[i];
      a.small.tgt[i] = targets[i];
    }
  } else {
    host.resize(2 * (size_t)T);
    std::memcpy(host.data(), sources, 4 * (size_t)T);
    std::memcpy(host.data() + T, targets, 4 * (size_t)T);
    // pageable source: the copy is staged before hipMemcpyAsync returns
    HIP_OR(hipMemcpyAsync(base, host.data(), n_small, hipMemcpyHostToDevice, s));
    a.sources = reinterpret_cast<const int32_t*>(base);
    a.targets = reinterpret_cast<const int32_t*>(base + 4 * (size_t)T);
  }
  double* trow = reinterpret_cast<double*>(base + o_row);
  double* tlog = trow + (size_t)T * (size_t)k->B;
  double* tcon = tlog + (size_t)T * (size_t)k->B;
  HIP_OR(dd::launch_target_rows(k->dense(), k->csr(), a, trow, tlog, tcon, s));
  a.trow = trow;
  a.tlog = tlog;
  a.tconst = tcon;
  HIP_OR(dd::launch_paths_on_demand(k->dense(), k->csr(), a, s));
  return DD_OK;
}

dd_status dd_support_kl_field(dd_kernel* k, int32_t target, double tau, int32_t tau_relative,
                              float* out_dev, dd_error_bound* bound, void* stream) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  if (k->is_csr) return fail(DD_EINVAL, "the target-support KL needs a dense handle");
  if (target < 0 || target >= k->N || !out_dev)
    return fail(DD_EINVAL, "target %d not in [0, %d) or out_dev null", target, k->N);
  if (!(tau >= 0.0) || !std::isfinite(tau) || (tau_relative && tau > 1.0))
    return fail(DD_EINVAL, "tau=%g", tau);
  HIP_OR(hipSetDevice(k->ctx->device));
  HIP_OR(dd::launch_support_kl_field(k->dense(), target, tau, tau_relative ? 1 : 0, out_dev,
                                     as_stream(stream)));
  // the terms are a subset of eq. (35)'s, so the dense KL bound holds
  if (bound) *bound = field_bound(k, DD_KL, target);
  return DD_OK;
}

dd_status dd_attach_mesh(dd_kernel* k, int32_t n_faces, const int32_t* faces, const double* xy) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  if (n_faces <= 0 || !faces || !xy) return fail(DD_EINVAL, "n_faces=%d or a null pointer", n_faces);
  const int32_t N = k->N;
  for (int64_t i = 0; i < 2 * (int64_t)N; ++i)
    if (!std::isfinite(xy[i])) return fail(DD_EINVAL, "xy[%lld] is not finite", (long long)i);
  std::vector<int32_t> rec((size_t)n_faces * 8, -1);
  std::unordered_map<uint64_t, std::pair<int32_t, int32_t>> edges;   // edge -> (face, k)
  edges.reserve((size_t)n_faces * 2);
  std::vector<int32_t> deg(N, 0);
  for (int32_t f = 0; f < n_faces; ++f) {
    int32_t v[3] = {faces[3 * (int64_t)f], faces[3 * (int64_t)f + 1], faces[3 * (int64_t)f + 2]};
    for (int j = 0; j < 3; ++j)
      if (v[j] < 0 || v[j] >= N) return fail(DD_EINVAL, "face %d: vertex %d not in [0, %d)", f, v[j], N);
    if (v[0] == v[1] || v[1] == v[2] || v[2] == v[0])
      return fail(DD_EINVAL, "face %d repeats a vertex", f);
    const double ax = xy[2 * v[1]] - xy[2 * v[0]], ay = xy[2 * v[1] + 1] - xy[2 * v[0] + 1];
    const double bx = xy[2 * v[2]] - xy[2 * v[0]], by = xy[2 * v[2] + 1] - xy[2 * v[0] + 1];
    const double area = ax * by - ay * bx;
    if (!(area != 0.0)) return fail(DD_EINVAL, "face %d has zero area", f);
    if (area < 0) std::swap(v[1], v[2]);
    for (int j = 0; j < 3; ++j) {
      rec[8 * (size_t)f + j] = v[j];
      ++deg[v[j]];
    }
  }
  for (int32_t f = 0; f < n_faces; ++f)
    for (int j = 0; j < 3; ++j) {
      const uint32_t a = (uint32_t)rec[8 * (size_t)f + j];
      const uint32_t b = (uint32_t)rec[8 * (size_t)f + (j + 1) % 3];
      const uint64_t key = ((uint64_t)std::min(a, b) << 32) | std::max(a, b);
      auto it = edges.find(key);
      if (it == edges.end()) {
        edges.emplace(key, std::make_pair(f, j));
      } else {
        const int32_t g = it->second.first, kg = it->second.second;
        if (g < 0 || rec[8 * (size_t)g + 3 + kg] >= 0)
          return fail(DD_EINVAL, "edge %u-%u is shared by more than two faces", a, b);
        rec[8 * (size_t)g + 3 + kg] = f;
        rec[8 * (size_t)f + 3 + j] = g;
      }
    }
  int32_t w = 1;
  for (int32_t v = 0; v < N; ++v) w = std::max(w, deg[v]);
  if (w > kMaxDegree) return fail(DD_EINVAL, "a vertex is in %d faces (limit %d)", w, kMaxDegree);
  std::vector<int32_t> vf((size_t)N * w, -1), fill(N, 0);
  for (int32_t f = 0; f < n_faces; ++f)   // ascending face index per vertex
    for (int j = 0; j < 3; ++j) {
      const int32_t v = rec[8 * (size_t)f + j];
      vf[(size_t)v * w + fill[v]++] = f;
    }
  HIP_OR(hipSetDevice(k->ctx->device));
  HIP_OR(k->mesh_faces.alloc(4 * rec.size()));
  HIP_OR(hipMemcpy(k->mesh_faces.p, rec.data(), 4 * rec.size(), hipMemcpyHostToDevice));
  HIP_OR(k->mesh_xy.alloc(16 * (size_t)N));
  HIP_OR(hipMemcpy(k->mesh_xy.p, xy, 16 * (size_t)N, hipMemcpyHostToDevice));
  HIP_OR(k->mesh_vf.alloc(4 * vf.size()));
  HIP_OR(hipMemcpy(k->mesh_vf.p, vf.data(), 4 * vf.size(), hipMemcpyHostToDevice));
  k->mesh_F = n_faces;
  k->mesh_vf_w = w;
  k->has_mesh = 1;
  return DD_OK;
}

}  // extern "C"

namespace {

dd_status triangle_paths(dd_kernel* k, int32_t T, const int32_t* sources, const int32_t* targets,
                         const float* fields_dev, const double* fields64_dev, int32_t max_steps,
                         double* points_dev, int32_t* where_dev, int32_t* len_dev,
                         int32_t* status_dev, void* stream) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  if (!k->has_mesh) return fail(DD_EINVAL, "no mesh attached (dd_attach_mesh)");
  if (!k->has_adj) return fail(DD_EINVAL, "kernel was loaded without adjacency");
  if (T <= 0 || !sources || !targets || (!fields_dev && !fields64_dev) || !points_dev ||
      !where_dev || !len_dev || !status_dev)
    return fail(DD_EINVAL, "T=%d or a required pointer is null", T);
  if (max_steps < 0) return fail(DD_EINVAL, "max_steps=%d", max_steps);
  for (int32_t i = 0; i < T; ++i)
    if (sources[i] < 0 || sources[i] >= k->N || targets[i] < 0 || targets[i] >= k->N)
      return fail(DD_EINVAL, "path %d: source %d / target %d not in [0, %d)", i, sources[i],
                  targets[i], k->N);
  HIP_OR(hipSetDevice(k->ctx->device));
  hipStream_t s = as_stream(stream);
  AsyncBuf ws(s);
  HIP_OR(ws.alloc(8 * (size_t)T));
  std::vector<int32_t> host(2 * (size_t)T);
  std::memcpy(host.data(), sources, 4 * (size_t)T);
  std::memcpy(host.data() + T, targets, 4 * (size_t)T);
  // pageable source: the copy is staged before hipMemcpyAsync returns
  HIP_OR(hipMemcpyAsync(ws.p, host.data(), 8 * (size_t)T, hipMemcpyHostToDevice, s));
  dd::TriArgs a;
  std::memset(&a, 0, sizeof a);
  a.faces = k->mesh_faces.as<const int32_t>();
  a.xy = k->mesh_xy.as<const double>();
  a.vfaces = k->mesh_vf.as<const int32_t>();
  a.vf_w = k->mesh_vf_w;
  a.adj = k->adj.as<const int32_t>();
  a.adj_w = k->adj_w;
  a.fields = fields_dev;
  a.fields64 = fields64_dev;
  a.sources = ws.as<const int32_t>();
  a.targets = ws.as<const int32_t>() + T;
  a.points = points_dev;
  a.where = where_dev;
  a.len = len_dev;
  a.status = status_dev;
  a.T = T;
  a.N = k->N;
  a.max_steps = max_steps;
  HIP_OR(dd::launch_triangle_paths(a, s));
  return DD_OK;
}

}  // namespace

extern "C" {

dd_status dd_trace_paths_triangles(dd_kernel* k, int32_t T, const int32_t* sources,
                                   const int32_t* targets, const float* fields_dev,
                                   int32_t max_steps, double* points_dev, int32_t* where_dev,
                                   int32_t* len_dev, int32_t* status_dev, void* stream) {
  if (!fields_dev) return fail(DD_EINVAL, "fields_dev is null");
  return triangle_paths(k, T, sources, targets, fields_dev, nullptr, max_steps, points_dev,
                        where_dev, len_dev, status_dev, stream);
}

dd_status dd_trace_paths_triangles_f64(dd_kernel* k, int32_t T, const int32_t* sources,
                                       const int32_t* targets, const double* fields_dev,
                                       int32_t max_steps, double* points_dev, int32_t* where_dev,
                                       int32_t* len_dev, int32_t* status_dev, void* stream) {
  if (!fields_dev) return fail(DD_EINVAL, "fields_dev is null");
  return triangle_paths(k, T, sources, targets, nullptr, fields_dev, max_steps, points_dev,
                        where_dev, len_dev, status_dev, stream);
}

dd_status dd_exact_distance_fields(dd_kernel* k, const int32_t* targets, int32_t T, int32_t kind,
                                   double* out_dev, void* stream) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  if (dd_status st = check_kind(k, kind)) return st;
  if (T <= 0 || !targets || !out_dev) return fail(DD_EINVAL, "T=%d, targets or out_dev null", T);
  if (T > 65535) return fail(DD_EINVAL, "T=%d above 65535 targets per call", T);
  for (int32_t i = 0; i < T; ++i)
    if (targets[i] < 0 || targets[i] >= k->N)
      return fail(DD_EINVAL, "targets[%d]=%d not in [0, %d)", i, targets[i], k->N);
  HIP_OR(hipSetDevice(k->ctx->device));
  hipStream_t s = as_stream(stream);
  dd::PathArgs a;
  std::memset(&a, 0, sizeof a);
  a.T = T;
  a.kind = kind;
  a.is_csr = k->is_csr;
  // scratch: [targets when T is large] [FP64 target rows, logs, constants]
  const bool inl = T <= dd::kInlinePaths;
  const size_t n_small = inl ? 0 : 4 * (size_t)T;
  const size_t o_row = align256(n_small);
  AsyncBuf ws(s);
  HIP_OR(ws.alloc(o_row + 16 * (size_t)T * (size_t)k->B + 32 * (size_t)T));
  unsigned char* base = ws.as<unsigned char>();
  if (inl) {
    for (int32_t i = 0; i < T; ++i) a.small.tgt[i] = targets[i];
  } else {
    // pageable source: the copy is staged before hipMemcpyAsync returns
    HIP_OR(hipMemcpyAsync(base, targets, n_small, hipMemcpyHostToDevice, s));
    a.targets = reinterpret_cast<const int32_t*>(base);
  }
  double* trow = reinterpret_cast<double*>(base + o_row);
  double* tlog = trow + (size_t)T * (size_t)k->B;
  double* tcon = tlog + (size_t)T * (size_t)k->B;
  HIP_OR(dd::launch_target_rows(k->dense(), k->csr(), a, trow, tlog, tcon, s));
  a.trow = trow;
  a.tlog = tlog;
  a.tconst = tcon;
  HIP_OR(dd::launch_exact_fields(k->dense(), k->csr(), a, k->N, out_dev, s));
  return DD_OK;
}

dd_status dd_local_minima(dd_kernel* k, int32_t T, const int32_t* targets, const float* fields_dev,
                          const dd_error_bound* bounds, uint8_t* class_dev, int32_t* counts_dev,
                          void* stream) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  if (!k->has_adj) return fail(DD_EINVAL, "kernel was loaded without adjacency");
  if (T <= 0 || !targets || !fields_dev || !bounds)
    return fail(DD_EINVAL, "T=%d or a required pointer is null", T);
  for (int32_t i = 0; i < T; ++i) {
    if (targets[i] < 0 || targets[i] >= k->N)
      return fail(DD_EINVAL, "targets[%d]=%d not in [0, %d)", i, targets[i], k->N);
    if (!(bounds[i].abs >= 0.0) || !(bounds[i].rel >= 0.0))
      return fail(DD_EINVAL, "bound %d is negative or NaN", i);
  }
  HIP_OR(hipSetDevice(k->ctx->device));
  hipStream_t s = as_stream(stream);
  dd::PathArgs a;
  std::memset(&a, 0, sizeof a);
  a.adj = k->adj.as<const int32_t>();
  a.adj_w = k->adj_w;
  a.fields = fields_dev;
  a.T = T;
  AsyncBuf ws(s);
  std::vector<unsigned char> host;
  if (T <= dd::kInlinePaths) {
    for (int32_t i = 0; i < T; ++i) {
      a.small.tgt[i] = targets[i];
      a.small.babs[i] = bounds[i].abs;
      a.small.brel[i] = bounds[i].rel;
    }
  } else {
    const size_t o_bnd = (4 * (size_t)T + 15) & ~size_t(15);
    host.resize(o_bnd + sizeof(dd::Bound) * T);
    std::memcpy(host.data(), targets, 4 * (size_t)T);
    for (int32_t i = 0; i < T; ++i) {
      dd::Bound b{bounds[i].abs, bounds[i].rel};
      std::memcpy(host.data() + o_bnd + sizeof(dd::Bound) * i, &b, sizeof b);
    }
    HIP_OR(ws.alloc(host.size()));
    HIP_OR(hipMemcpyAsync(ws.p, host.data(), host.size(), hipMemcpyHostToDevice, s));
    a.targets = ws.as<const int32_t>();
    a.bounds = reinterpret_cast<const dd::Bound*>(ws.as<unsigned char>() + o_bnd);
  }
  HIP_OR(dd::launch_local_minima(a, k->N, class_dev, counts_dev, s));
  return DD_OK;
}

dd_status dd_resolve_minima(dd_kernel* k, int32_t T, const int32_t* targets, int32_t kind,
                            uint8_t* class_dev, int32_t* counts_dev, void* stream) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  if (!k->has_adj) return fail(DD_EINVAL, "kernel was loaded without adjacency");
  if (dd_status st = check_kind(k, kind)) return st;
  if (T <= 0 || !targets || !class_dev)
    return fail(DD_EINVAL, "T=%d or a required pointer is null", T);
  for (int32_t i = 0; i < T; ++i)
    if (targets[i] < 0 || targets[i] >= k->N)
      return fail(DD_EINVAL, "targets[%d]=%d not in [0, %d)", i, targets[i], k->N);
  HIP_OR(hipSetDevice(k->ctx->device));
  hipStream_t s = as_stream(stream);
  dd::PathArgs a;
  std::memset(&a, 0, sizeof a);
  a.adj = k->adj.as<const int32_t>();
  a.adj_w = k->adj_w;
  a.T = T;
  a.kind = kind;
  a.is_csr = k->is_csr;
  // scratch: [targets when T is large] [FP64 target rows, logs, constants]
  const bool inl = T <= dd::kInlinePaths;
  const size_t n_tgt = inl ? 0 : (4 * (size_t)T + 255) & ~size_t(255);
  const size_t n_row = 16 * (size_t)T * (size_t)k->B + 32 * (size_t)T;
  AsyncBuf ws(s);
  HIP_OR(ws.alloc(n_tgt + n_row));
  unsigned char* base = ws.as<unsigned char>();
  if (inl) {
    for (int32_t i = 0; i < T; ++i) a.small.tgt[i] = targets[i];
  } else {
    // pageable source: the copy is staged before hipMemcpyAsync returns
    HIP_OR(hipMemcpyAsync(base, targets, 4 * (size_t)T, hipMemcpyHostToDevice, s));
    a.targets = reinterpret_cast<const int32_t*>(base);
  }
  double* trow = reinterpret_cast<double*>(base + n_tgt);
  double* tlog = trow + (size_t)T * (size_t)k->B;
  double* tcon = tlog + (size_t)T * (size_t)k->B;
  HIP_OR(dd::launch_target_rows(k->dense(), k->csr(), a, trow, tlog, tcon, s));
  a.trow = trow;
  a.tlog = tlog;
  a.tconst = tcon;
  HIP_OR(dd::launch_resolve_minima(k->dense(), k->csr(), a, k->N, class_dev, counts_dev, s));
  return DD_OK;
}

dd_status dd_plan_path(dd_kernel* k, int32_t source, int32_t target, int32_t kind,
                       int32_t max_steps, int32_t* path_host, int32_t* len, int32_t* status,
                       int32_t* rechecks, void* stream) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  if (!k->has_adj) return fail(DD_EINVAL, "kernel was loaded without adjacency");
  if (!path_host || !len || !status) return fail(DD_EINVAL, "null output");
  if (max_steps < 0) return fail(DD_EINVAL, "max_steps=%d", max_steps);
  if (source < 0 || source >= k->N || target < 0 || target >= k->N)
    return fail(DD_EINVAL, "source %d / target %d not in [0, %d)", source, target, k->N);
  if (dd_status st = check_kind(k, kind)) return st;
  HIP_OR(hipSetDevice(k->ctx->device));
  hipStream_t s = as_stream(stream);
  AsyncBuf field(s), pbuf(s);
  HIP_OR(field.alloc(4 * (size_t)k->N));
  HIP_OR(pbuf.alloc(4 * ((size_t)max_steps + 1 + 3)));
  dd_error_bound b;
  if (dd_status st = dd_distance_field(k, target, kind, field.as<float>(), &b, stream)) return st;
  int32_t* pd = pbuf.as<int32_t>();
  int32_t* tail = pd + max_steps + 1;
  if (dd_status st = dd_trace_paths(k, 1, &source, &target, kind, field.as<const float>(), &b,
                                    max_steps, pd, tail, tail + 1, tail + 2, stream))
    return st;
  int32_t info[3];
  HIP_OR(hipMemcpyAsync(path_host, pd, 4 * ((size_t)max_steps + 1), hipMemcpyDeviceToHost, s));
  HIP_OR(hipMemcpyAsync(info, tail, sizeof info, hipMemcpyDeviceToHost, s));
  HIP_OR(hipStreamSynchronize(s));
  *len = info[0];
  *status = info[1];
  if (rechecks) *rechecks = info[2];
  return DD_OK;
}

}  // extern "C"

namespace {

// Checks shared by the grid solves; counts the interior and boundary vertices.
dd_status check_grid(const dd_ctx* ctx, int32_t G, const uint8_t* node_type, const void* o32,
                     const void* o64, double tol, int32_t max_iter, int32_t batch,
                     int64_t& n_int, int64_t& n_bnd) {
  if (!ctx_ok(ctx)) return fail(DD_ESTATE, "not a live context");
  if (G < 3 || G > 46340) return fail(DD_EINVAL, "G=%d outside [3, 46340]", G);
  if (!node_type) return fail(DD_EINVAL, "node_type is null");
  if (!o32 && !o64) return fail(DD_EINVAL, "no output (both outputs null)");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(DD_EINVAL, "tol must be positive");
  if (max_iter < 1) return fail(DD_EINVAL, "max_iter must be >= 1");
  if (batch < 0 || batch % 64 != 0) return fail(DD_EINVAL, "batch %d is not a multiple of 64", batch);
  n_int = 0;
  n_bnd = 0;
  for (int64_t j = 0; j < G; ++j)
    for (int64_t i = 0; i < G; ++i) {
      const uint8_t t = node_type[j * G + i];
      if (t > 2) return fail(DD_EINVAL, "node_type %d at (%lld, %lld)", t, (long long)i, (long long)j);
      if (t == 2) ++n_bnd;
      if (t != 1) continue;
      ++n_int;
      if (i == 0 || j == 0 || i == G - 1 || j == G - 1)
        return fail(DD_EINVAL, "interior vertex (%lld, %lld) on the grid edge", (long long)i,
                    (long long)j);
      const int64_t g = j * G + i;
      if (!node_type[g - 1] || !node_type[g + 1] || !node_type[g - G] || !node_type[g + G])
        return fail(DD_EINVAL, "interior vertex (%lld, %lld) has a neighbour outside the domain",
                    (long long)i, (long long)j);
    }
  if (n_int == 0 || n_bnd == 0) return fail(DD_EINVAL, "no interior or no boundary vertex");
  return DD_OK;
}

// Columns per batch: the requested width, or the widest up to 1024 whose
// workspace takes at most 90% of free memory.
dd_status grid_batch(int32_t G, int32_t ncols, int32_t batch, int32_t& C) {
  size_t free_b = 0, total_b = 0;
  HIP_OR(hipMemGetInfo(&free_b, &total_b));
  C = batch;
  if (C == 0) {
    C = std::min<int32_t>(1024, (ncols + 63) / 64 * 64);
    while (C > 64 && dd::grid_poisson_workspace(G, C) > free_b / 10 * 9) C -= 64;
  }
  if (dd::grid_poisson_workspace(G, C) > free_b)
    return fail(DD_ENOMEM, "a batch of %d columns needs %zu bytes, %zu free", C,
                dd::grid_poisson_workspace(G, C), free_b);
  return DD_OK;
}

dd_status grid_result(hipError_t e, const dd::GridSolveStats& st, double tol,
                      dd_grid_solve_stats* stats) {
  if (e != hipSuccess) return fail(DD_EDEVICE, "grid solve: %s", hipGetErrorString(e));
  if (stats) {
    stats->iterations = st.iterations;
    stats->batches = st.batches;
    stats->levels = st.levels;
    stats->total_iterations = st.total_iterations;
    stats->max_rel_residual = st.max_rel_residual;
  }
  if (!st.converged)
    return fail(DD_ENOCONV, "relative residual %.3e above tol %.3e after %d iterations",
                st.max_rel_residual, tol, st.iterations);
  return DD_OK;
}

}  // namespace

extern "C" {

dd_status dd_grid_poisson_kernel(dd_ctx* ctx, int32_t G, const uint8_t* node_type,
                                 int32_t col_begin, int32_t ncols, float* P32, int64_t ld32,
                                 double* P64, int64_t ld64, double tol, int32_t max_iter,
                                 int32_t batch, dd_grid_solve_stats* stats, void* stream) {
  int64_t n_int = 0, n_bnd = 0;
  if (dd_status st = check_grid(ctx, G, node_type, P32, P64, tol, max_iter, batch, n_int, n_bnd))
    return st;
  if (col_begin < 0 || ncols < 1 || (int64_t)col_begin + ncols > n_bnd)
    return fail(DD_EINVAL, "columns [%d, %d + %d) outside the %lld boundary vertices", col_begin,
                col_begin, ncols, (long long)n_bnd);
  if (P32 && ld32 < ncols) return fail(DD_EINVAL, "ld32=%lld < ncols=%d", (long long)ld32, ncols);
  if (P64 && ld64 < ncols) return fail(DD_EINVAL, "ld64=%lld < ncols=%d", (long long)ld64, ncols);
  HIP_OR(hipSetDevice(ctx->device));
  int32_t C = 0;
  if (dd_status st = grid_batch(G, ncols, batch, C)) return st;
  dd::GridSolveStats st{};
  const hipError_t e = dd::grid_poisson(G, node_type, col_begin, ncols, C, tol, max_iter, P32,
                                        ld32, P64, ld64, &st, static_cast<hipStream_t>(stream));
  return grid_result(e, st, tol, stats);
}

dd_status dd_grid_green_function(dd_ctx* ctx, int32_t G, const uint8_t* node_type,
                                 const int32_t* poles, int32_t T, float* D32, int64_t ld32,
                                 double* D64, int64_t ld64, double tol, int32_t max_iter,
                                 int32_t batch, dd_grid_solve_stats* stats, void* stream) {
  int64_t n_int = 0, n_bnd = 0;
  if (dd_status st = check_grid(ctx, G, node_type, D32, D64, tol, max_iter, batch, n_int, n_bnd))
    return st;
  if (T < 1 || !poles) return fail(DD_EINVAL, "T=%d or poles null", T);
  for (int32_t i = 0; i < T; ++i)
    if (poles[i] < 0 || poles[i] >= n_int)
      return fail(DD_EINVAL, "poles[%d]=%d not in [0, %lld)", i, poles[i], (long long)n_int);
  if (D32 && ld32 < n_int) return fail(DD_EINVAL, "ld32=%lld < N=%lld", (long long)ld32, (long long)n_int);
  if (D64 && ld64 < n_int) return fail(DD_EINVAL, "ld64=%lld < N=%lld", (long long)ld64, (long long)n_int);
  HIP_OR(hipSetDevice(ctx->device));
  int32_t C = 0;
  if (dd_status st = grid_batch(G, T, batch, C)) return st;
  dd::GridSolveStats st{};
  const hipError_t e = dd::grid_green(G, node_type, poles, T, C, tol, max_iter, D32, ld32, D64,
                                      ld64, &st, static_cast<hipStream_t>(stream));
  return grid_result(e, st, tol, stats);
}

dd_status dd_free_kernel(dd_kernel* k) {
  if (!kernel_ok(k)) return fail(DD_ESTATE, "not a live kernel");
  // work in flight may still read the handle's memory: wait for it, then free
  hipError_t e = hipSetDevice(k->ctx->device);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  k->ctx->live_kernels--;
  k->magic = kDead;
  delete k;
  if (e != hipSuccess)
    return fail(DD_EDEVICE, "freed after a device error: %s", hipGetErrorString(e));
  return DD_OK;
}

}  // extern "C"
