// Edge-based steepest-descent paths (Section IV, "Gradient-descent path
// generation"): from the current vertex move to the neighbour with the
// smallest distance (ties: lowest id) while it is strictly below the current
// vertex; stop at the target, at a vertex with no strictly lower neighbour,
// or after max_steps moves.
//
// The walk is a chain of dependent steps, so its cost is latency per step.
// A step needs one round of independent loads: lane j reads the field value
// of the current vertex's j-th neighbour and (for rows of at most kPrefetchW
// slots) that neighbour's own adjacency row, so the row of whichever
// neighbour is chosen is already in registers for the next step; a scalar
// best/second-best selection follows.
//
// Each decision is checked against the field's stated error bound: when the
// best and the second-best neighbour (or the best neighbour and the current
// vertex) cannot be told apart within the bound, the distances of every
// neighbour that could be the minimum, and of the current vertex, are
// recomputed from the resident master rows and the decision is taken on
// those: for KL on dense rows first as level-1 values (FP32 hardware
// logarithms summed in FP64, with a stated bound), and in FP64 where those
// intervals still do not settle the step.
#include <cmath>
#include <cstring>
#include <type_traits>

#include "dd_internal.h"

namespace dd {

__device__ __forceinline__ double wsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ int path_source(const PathArgs& a, int i) {
  return a.sources ? a.sources[i] : a.small.src[i];
}
__device__ __forceinline__ int path_target(const PathArgs& a, int i) {
  return a.targets ? a.targets[i] : a.small.tgt[i];
}
__device__ __forceinline__ Bound path_bound(const PathArgs& a, int i) {
  if (a.bounds) return a.bounds[i];
  return Bound{a.small.babs[i], a.small.brel[i]};
}

// Target rows in FP64 (dense: the master row; truncated: the stored entries
// scattered into a dense row), their logarithms, and constants W = sum p,
// H = sum p ln p, |S| over the nonzero entries, sum p |ln p|.
__global__ __launch_bounds__(256) void target_rows_kernel(DenseView dv, CsrView cv, PathArgs a,
                                                          double* trow, double* tlog,
                                                          double* tconst) {
  const int t = path_target(a, blockIdx.x);
  const int B = a.is_csr ? cv.B : dv.B;
  double* out = trow + (int64_t)blockIdx.x * B;
  double* lout = tlog + (int64_t)blockIdx.x * B;
  __shared__ double red[4][8];
  __shared__ double thr_s;
  double w = 0.0, h = 0.0, c = 0.0, ha = 0.0;
  if (!a.is_csr) {
    // threshold of the target-row truncation (none when tgt_tau == 0)
    double thr = 0.0;
    if (a.tgt_tau > 0.0) {
      if (a.tgt_tau_relative) {
        double m = 0.0;
        for (int b = threadIdx.x; b < B; b += blockDim.x)
          m = fmax(m, dv.P64 ? dv.P64[(int64_t)t * dv.B + b] : (double)dv.P[(int64_t)t * dv.ld + b]);
        for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
        if ((threadIdx.x & 63) == 0) red[0][threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
          double M = 0.0;
          for (int i = 0; i < (int)(blockDim.x >> 6); ++i) M = fmax(M, red[0][i]);
          thr_s = a.tgt_tau * M;
        }
        __syncthreads();
        thr = thr_s;
      } else {
        thr = a.tgt_tau;
      }
    }
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
      double p = dv.P64 ? dv.P64[(int64_t)t * dv.B + b] : (double)dv.P[(int64_t)t * dv.ld + b];
      if (p < thr) p = 0.0;
      const double lp = p > 0.0 ? log(p) : 0.0;
      out[b] = p;
      lout[b] = lp;
      w += p;
      h += p * lp;
      ha += p * fabs(lp);
      c += p > 0.0 ? 1.0 : 0.0;
    }
  } else {
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
      out[b] = 0.0;
      lout[b] = 0.0;
    }
    __syncthreads();
    const int64_t s = cv.start[t];
    const int n = cv.len[t];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double p = cv.val64 ? cv.val64[s + i] : (double)cv.val[s + i];
      const double lp = log(p);
      out[cv.col[s + i]] = p;
      lout[cv.col[s + i]] = lp;
      w += p;
      h += p * lp;
      ha += p * fabs(lp);
      c += 1.0;
    }
  }
  w = wsum(w);
  h = wsum(h);
  ha = wsum(ha);
  c = wsum(c);
  __syncthreads();   // red[] may still be read by the threshold step
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wid] = w;
    red[1][wid] = h;
    red[2][wid] = c;
    red[3][wid] = ha;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double W = 0.0, H = 0.0, C = 0.0, HA = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      W += red[0][i];
      H += red[1][i];
      C += red[2][i];
      HA += red[3][i];
    }
    tconst[blockIdx.x * 4 + 0] = W;
    tconst[blockIdx.x * 4 + 1] = H;
    tconst[blockIdx.x * 4 + 2] = C;
    tconst[blockIdx.x * 4 + 3] = HA;
  }
}

// The KL terms are p (log p - log q); chi-squared (q - p)^2 / p (+inf for
// q > 0 on p = 0); Hellinger (q - p)^2 / (sqrt q + sqrt p)^2, the
// cancellation-free form of (sqrt q - sqrt p)^2.
// log c_i and 1/c_i for the centres c_i = 1 + (i + 1/2)/128 of the 128
// intervals of [1, 2), set by init_log_table (host logs, below 1 ulp).
__device__ double g_logtab[256];
// The kernels that evaluate FP64 rows copy the table into LDS first
// (stage_log_table): the terms' table reads are then LDS reads rather than
// gathers through the vector memory path.
__shared__ double s_logtab[256];

// Every thread of the block must call this before any use of log_pos.
__device__ __forceinline__ void stage_log_table() {
  for (int q = threadIdx.x; q < 256; q += blockDim.x) s_logtab[q] = g_logtab[q];
  __syncthreads();
}

// Natural log of a positive normal double: x = m 2^e with m in [1, 2) falls
// in interval i; with r = m/c_i - 1 (|r| < 2^-8), log x = e ln 2 + log c_i +
// log1p(r), and the series of log1p to r^7 leaves an error below 2^-67.  ln 2
// is split so that e * ln2_hi is exact (the published hi/lo pair of fdlibm's
// log: ln2_hi ends in 21 zero bits, and |e| < 2^11).  The error is within a few units of
// 1e-16 absolute (about 1 ulp where |log x| > 1).  A quarter of the FP64
// operations of the library log, which bounds the cost of the FP64
// re-decisions and on-demand rows for KL.
__device__ __forceinline__ double log_pos(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  // within 2^-8 of 1, r = x - 1 is exact and the table term is dropped, so a
  // result near 0 keeps its relative accuracy
  const bool near1 = fabs(x - 1.0) < 0.00390625;
  const double e = near1 ? 0.0 : (double)((int)((b >> 52) & 0x7ff) - 1023);
  const int i = (int)((b >> 45) & 127);
  const double m =
      __longlong_as_double((long long)((b & 0x000fffffffffffffull) | 0x3ff0000000000000ull));
  const double r = near1 ? x - 1.0 : fma(m, s_logtab[128 + i], -1.0);
  const double t = near1 ? 0.0 : s_logtab[i];
  double q = 1.0 / 7.0;
  q = fma(q, r, -1.0 / 6.0);
  q = fma(q, r, 1.0 / 5.0);
  q = fma(q, r, -0.25);
  q = fma(q, r, 1.0 / 3.0);
  q = fma(q, r, -0.5);
  q = fma(q, r, 1.0);
  const double ln2_hi = 6.93147180369123816490e-01, ln2_lo = 1.90821492927058770002e-10;
  return e * ln2_hi + (t + fma(e, ln2_lo, q * r));
}

hipError_t init_log_table() {
  double h[256];
  for (int i = 0; i < 128; ++i) {
    const double c = 1.0 + (i + 0.5) / 128.0;
    h[i] = std::log(c);
    h[128 + i] = 1.0 / c;
  }
  return hipMemcpyToSymbol(HIP_SYMBOL(g_logtab), h, sizeof h);
}

// ---- level-1 rows: FP32 logarithms with a verified bound ----
//
// The FP64 logarithm above costs a few dozen FP64 operations per entry, which
// makes a re-decision of a walk bound by the FP64 units of its compute unit.
// Most re-decisions are settled by values far less accurate than FP64 and far
// more accurate than the field: level-1 rows take log2 of each FP32 entry from
// the hardware's v_log_f32 (one transcendental instruction) and sum the KL
// terms in FP64.  The hardware log is trusted only within
//   |L(x) - log2 x| <= kL1Rel |log2 x| + kL1Abs  for every normal x in (0, 1],
// and the library checks that claim at start-up on every FP32 input in that
// range (log2_scan_kernel, against the FP64 log2); level-1 rows are used only
// on devices that pass.
constexpr double kL1Rel = 0x1p-22;
constexpr double kL1Abs = 0x1p-40;
constexpr double kLn2 = 0.6931471805599453;
constexpr double kInvLn2 = 1.4426950408889634;

// out[0] = max over x of |L(x) - log2 x| / (kL1Rel |log2 x| + kL1Abs),
// out[1] = max of |L(x) - log2 x| / |log2 x| over x != 1; a NaN ratio counts
// as +inf.  Inputs: the n FP32 values with bit patterns lo, lo + 1, ...
__global__ __launch_bounds__(256) void log2_scan_kernel(uint32_t lo, uint32_t n,
                                                        unsigned long long* out) {
  double m0 = 0.0, m1 = 0.0;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float x = __uint_as_float(lo + i);
    const double y = (double)__builtin_amdgcn_logf(x);
    const double r = log2((double)x);
    const double err = fabs(y - r);
    const double q0 = err / (kL1Rel * fabs(r) + kL1Abs);
    m0 = q0 == q0 ? fmax(m0, q0) : __builtin_inf();
    if (r != 0.0) {
      const double q1 = err / fabs(r);
      m1 = q1 == q1 ? fmax(m1, q1) : __builtin_inf();
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    m0 = fmax(m0, __shfl_xor(m0, off));
    m1 = fmax(m1, __shfl_xor(m1, off));
  }
  if ((threadIdx.x & 63) == 0) {
    // non-negative doubles order as their bit patterns
    atomicMax(&out[0], (unsigned long long)__double_as_longlong(m0));
    atomicMax(&out[1], (unsigned long long)__double_as_longlong(m1));
  }
}

hipError_t check_log2_bound(double ratio[2]) {
  unsigned long long* d = nullptr;
  hipError_t e = hipMalloc(&d, 16);
  if (e != hipSuccess) return e;
  e = hipMemset(d, 0, 16);
  // FLT_MIN = 0x00800000 up to 1.0f = 0x3f800000
  const uint32_t lo = 0x00800000u, n = 0x3f800000u - 0x00800000u + 1u;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(log2_scan_kernel, dim3(num_cus() * 8), dim3(256), 0, 0, lo, n, d);
    e = hipGetLastError();
  }
  unsigned long long h[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpy(h, d, 16, hipMemcpyDeviceToHost);
  const hipError_t f = hipFree(d);
  if (e == hipSuccess) e = f;
  for (int i = 0; i < 2; ++i) std::memcpy(&ratio[i], &h[i], 8);
  return e;
}

// KL of dense row x over columns [lo, hi) at level 1, one wave: returns
// sum_b p_b log2 q_b (log2 from v_log_f32 for normal FP32 q <= 1, else from
// log_pos) and sets s = sum_b p_b |log2 q_b|; terms with p_b = 0 are skipped.
// The target row p is read as FP32 from LDS (exact for an FP32 matrix); FP64
// rows and target values are rounded to FP32 first (within 2^-24 relative:
// within 2^-24 of log q per entry and 2^-24 of p, which l1_bound adds).
__device__ __forceinline__ void l1_term(float pf, float qf, double q, double& acc, double& s) {
  if (!(pf > 0.0f)) return;
  const double pb = (double)pf;
  double l2;
  if (qf >= 1.17549435e-38f && qf <= 1.0f)
    l2 = (double)__builtin_amdgcn_logf(qf);
  else
    l2 = q > 0.0 ? log_pos(q) * kInvLn2 : -__builtin_inf();
  acc += pb * l2;
  s += pb * fabs(l2);
}


// Terms per kind family F: 0 TV, 1 KL, 2 chi-squared, 3 Hellinger, 4 the
// power family |q - p|^k / p^(k-1) (k = param), 5 the alpha-divergence term
// p (1 - (q/p)^(param/16)) (its factor 4/(1 - alpha^2) is applied to the sum).
template <int F>
__device__ __forceinline__ double term64(double pb, double lpb, double q, int param) {
  const double df = q - pb;
  if (F == 0) return fabs(df);
  if (F == 1) return pb > 0.0 ? pb * (lpb - (q > 0.0 ? log_pos(q) : -__builtin_inf())) : 0.0;
  if (F == 5) return pb > 0.0 ? pb * (1.0 - pow(q / pb, (double)param / 16.0)) : 0.0;
  if (df == 0.0) return 0.0;
  if (F == 4) {
    if (!(pb > 0.0)) return param == 1 ? fabs(df) : __builtin_inf();
    const double r = fabs(df) / pb;
    double t = fabs(df);
    for (int j = 1; j < param; ++j) t *= r;
    return t;
  }
  if (F == 2) return pb > 0.0 ? df * df / pb : __builtin_inf();
  const double e = df / (sqrt(q) + sqrt(pb));
  return e * e;
}

// FP64 sum of the terms of dense row x over columns [lo, hi), one wave.  The row's entries are loaded kQ
// per lane at a time (indices clamped into the row, clamped slots not
// summed): one memory round trip per 64 * kQ entries.  The target row p and
// its logs lp are read from LDS when the block staged them there.  One
// instance per kind family keeps each instance's code small: the walk and the
// one instance a path uses stay in the instruction cache.
constexpr int kU = 8;
constexpr int kQ = 32;      // FP32 row entries in flight per lane
constexpr int kQ64 = 16;    // FP64 row entries in flight per lane
// Walks on dense rows of at least kSplitB columns split each FP64 re-decision
// row over kMaxParts waves of a kPathThreads block (below that a row is cheap,
// and the extra waves of the walk cost more than they save).
constexpr int kPathThreads = 512;
constexpr int kMaxParts = 4;
// adjacency rows up to this width travel with the neighbours' values (see paths_kernel)
constexpr int kPrefetchW = 8;
constexpr int kSplitB = 4096;
__host__ __device__ inline bool split_rows(int is_csr, int B) { return !is_csr && B >= kSplitB; }

template <int F>
__device__ __forceinline__ double exact_dense(const DenseView& dv, const double* p, const double* lp,
                                           int x, int param, int lo, int hi) {
  const int lane = threadIdx.x & 63;
  double acc = 0.0;
  // each lane sums its columns lo + lane, lo + lane + 64, ... in increasing
  // order whatever the batch width, so a row's value does not depend on kQ
  if (dv.P64) {
    const double* q64 = dv.P64 + (int64_t)x * dv.B;
    for (int b0 = lo + lane; b0 < hi; b0 += 64 * kQ64) {
      double q[kQ64];
#pragma unroll
      for (int u = 0; u < kQ64; ++u) q[u] = q64[b0 + 64 * u < hi ? b0 + 64 * u : lo];
#pragma unroll
      for (int u = 0; u < kQ64; ++u) {
        const int b = b0 + 64 * u;
        if (b < hi) acc += term64<F>(p[b], F == 1 ? lp[b] : 0.0, q[u], param);
      }
    }
  } else {
    // FP32 rows: the values stay FP32 in registers until their term
    const float* q32 = dv.P + (int64_t)x * dv.ld;
    for (int b0 = lo + lane; b0 < hi; b0 += 64 * kQ) {
      float q[kQ];
#pragma unroll
      for (int u = 0; u < kQ; ++u) q[u] = q32[b0 + 64 * u < hi ? b0 + 64 * u : lo];
#pragma unroll
      for (int u = 0; u < kQ; ++u) {
        const int b = b0 + 64 * u;
        if (b < hi) acc += term64<F>(p[b], F == 1 ? lp[b] : 0.0, (double)q[u], param);
      }
    }
  }
  return wsum(acc);
}

__device__ __forceinline__ double l1_dense(const DenseView& dv, const float* p, int x, int lo,
                                           int hi, double& sabs) {
  const int lane = threadIdx.x & 63;
  double acc = 0.0, s = 0.0;
  if (dv.P64) {
    const double* q64 = dv.P64 + (int64_t)x * dv.B;
    for (int b0 = lo + lane; b0 < hi; b0 += 64 * kQ64) {
      double q[kQ64];
#pragma unroll
      for (int u = 0; u < kQ64; ++u) q[u] = q64[b0 + 64 * u < hi ? b0 + 64 * u : lo];
#pragma unroll
      for (int u = 0; u < kQ64; ++u)
        if (b0 + 64 * u < hi) l1_term(p[b0 + 64 * u], (float)q[u], q[u], acc, s);
    }
  } else {
    const float* q32 = dv.P + (int64_t)x * dv.ld;
    for (int b0 = lo + lane; b0 < hi; b0 += 64 * kQ) {
      float q[kQ];
#pragma unroll
      for (int u = 0; u < kQ; ++u) q[u] = q32[b0 + 64 * u < hi ? b0 + 64 * u : lo];
#pragma unroll
      for (int u = 0; u < kQ; ++u)
        if (b0 + 64 * u < hi) l1_term(p[b0 + 64 * u], q[u], (double)q[u], acc, s);
    }
  }
  sabs = wsum(s);
  return wsum(acc);
}

// Level-1 KL of a dense row from its parts' sums A = sum p log2 q and
// S = sum p |log2 q| (natural-log value H - ln2 A), and the bound on its
// distance from the exact value and from the FP64 evaluation of the same row
// (so that intervals which settle a decision settle it for the FP64 values
// too).  Per entry the log is within kL1Rel |ln q| + ln2 kL1Abs (plus 2^-50
// |ln q| for the FP64 steps after it).  An FP64 matrix adds the FP32
// rounding of q (2^-24 of ln q, times p: 2^-23 W in all) and of p (2^-24
// relative: 2^-23 S), and target values below the FP32 range, which drop out
// (under 2^-120 per entry).  The sums of at most B/64 + 24 terms deep are
// within that many units of 2^-53 of the sums of magnitudes, counted twice
// (the FP64 evaluation has the same rounding); H, W and Habs = sum p |ln p|
// come from the target.
__device__ __forceinline__ double l1_bound(double S2, double W, double Habs, int B, bool p64) {
  const double S = kLn2 * S2;
  const double g = 2.0 * ((double)(B / 64) + 24.0) * 0x1p-53;
  return (kL1Rel + 0x1p-50 + (p64 ? 0x1p-23 : 0.0)) * (1.0 + 0x1p-20) * S +
         2.0 * kLn2 * kL1Abs * (1.0 + 0x1p-20) * W + g * (Habs + S) +
         (p64 ? 0x1p-23 * W + 0x1p-120 * (double)B : 0.0);
}

// FP64 distance of truncated row x (TV or KL of the truncated rows), one wave.
template <int F>
__device__ __forceinline__ double exact_csr(const CsrView& cv, const double* p, const double* lp,
                                         const double* tc, int x) {
  const int lane = threadIdx.x & 63;
  const int64_t s = cv.start[x];
  const int n = cv.len[x];
  double acc = 0.0, A = 0.0, E = 0.0, c = 0.0;
  for (int i0 = lane; i0 < n; i0 += 64 * kU) {
    double q[kU];
    int col[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t e = s + (i0 + 64 * u < n ? i0 + 64 * u : 0);
      q[u] = cv.val64 ? cv.val64[e] : (double)cv.val[e];
      col[u] = cv.col[e];
    }
    double pb[kU], lpb[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      pb[u] = p[col[u]];
      lpb[u] = lp[col[u]];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (i0 + 64 * u < n) {
        A += pb[u];
        acc += term64<F>(pb[u], lpb[u], q[u], 0);
        if (F == 1 && pb[u] > 0.0) E += pb[u] * lpb[u];
        c += pb[u] > 0.0 ? 1.0 : 0.0;
      }
    }
  }
  acc = wsum(acc);
  A = wsum(A);
  E = wsum(E);
  c = wsum(c);
  if (c == tc[2]) return acc;
  if (F == 0) return acc + (tc[0] - A);
  return acc + (tc[1] - E) - log(cv.phi[x]) * (tc[0] - A);
}

// Columns of part `part` of `parts` of a dense row: whole multiples of 64.
__device__ __forceinline__ void part_range(int B, int part, int parts, int& lo, int& hi) {
  const int chunk = (((B + parts - 1) / parts) + 63) & ~63;
  lo = min(B, part * chunk);
  hi = min(B, lo + chunk);
}

// Factor applied to the summed terms (the alpha family's 4/(1 - alpha^2)).
__device__ __forceinline__ double distance_scale(int kind) {
  if (kind > 200) {
    const double al = (double)(kind - 208) / 8.0;
    return 4.0 / (1.0 - al * al);
  }
  return 1.0;
}

// Kind family of a kind value: 0 TV, 1 KL, 2 chi-squared, 3 Hellinger, 4 the
// power family (100 + k), 5 the alpha family (200 + j); the kernels that
// evaluate FP64 rows are instantiated per family (launch_family), so each
// instance holds one family's terms inline.
__host__ __device__ inline int kind_family(int kind) {
  return kind > 200 ? 5 : (kind > 100 ? 4 : kind);
}

// Part `part` of `parts` of the FP64 distance of row x to the target, computed
// by one wave from the staged FP64 target row p, its logarithms lp and
// constants tc: the terms of a column range of a dense row (summed over the
// parts in order, then times distance_scale), or, on a truncated handle
// (parts = 1), the whole truncated distance.  F is the kind family of `kind`,
// the library's kind value (0..3, 100 + k, 200 + j); truncated handles carry
// TV and KL only.
template <int F>
__device__ __forceinline__ double exact_part(const DenseView& dv, const CsrView& cv, int is_csr,
                                             int kind, const double* p, const double* lp,
                                             const double* tc, int x, int part, int parts) {
  if constexpr (F <= 1)
    if (is_csr) return exact_csr<F>(cv, p, lp, tc, x);
  int lo, hi;
  part_range(dv.B, part, parts, lo, hi);
  const int param = F == 5 ? kind - 200 : (F == 4 ? kind - 100 : 0);
  return exact_dense<F>(dv, p, lp, x, param, lo, hi);
}

// FP64 distance of row x to the target, one wave.
template <int F>
__device__ __forceinline__ double exact_distance(const DenseView& dv, const CsrView& cv,
                                                 int is_csr, int kind, const double* p,
                                                 const double* lp, const double* tc, int x) {
  return exact_part<F>(dv, cv, is_csr, kind, p, lp, tc, x, 0, 1) * distance_scale(kind);
}

__device__ __forceinline__ double uniform(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Minimum of a 32-bit key over lanes [0, W) of the wave (W <= 64), uniform.
// Lanes at or above W must hold 0xffffffff.  Within each row of 16 lanes a
// butterfly of DPP moves (swap neighbours, swap pairs, mirror halves, mirror
// the row) leaves the row minimum in every lane; rows are then combined.
__device__ __forceinline__ uint32_t wave_min(uint32_t x, int W) {
  x = min(x, (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false));
  x = min(x, (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false));
  x = min(x, (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x141, 0xF, 0xF, false));
  x = min(x, (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x140, 0xF, 0xF, false));
  uint32_t m = (uint32_t)__builtin_amdgcn_readlane((int)x, 0);
  if (W > 16) m = min(m, (uint32_t)__builtin_amdgcn_readlane((int)x, 16));
  if (W > 32) {
    m = min(m, (uint32_t)__builtin_amdgcn_readlane((int)x, 32));
    m = min(m, (uint32_t)__builtin_amdgcn_readlane((int)x, 48));
  }
  return m;
}

// Order-preserving map of a float to an unsigned key (for any non-NaN value).
__device__ __forceinline__ uint32_t fkey(uint32_t b) {
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float unkey(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// One 256-thread block per path.  The walk itself is uniform: every wave
// takes the same decisions from the same loads; the four waves split the rows
// of an FP64 re-decision between them (one row per wave).  A step loads the
// padded neighbour row (ids and pre-gathered values), one slot per lane, then
// takes the best neighbour as a DPP minimum over order-preserving integer keys
// (ties: lowest id) and the set of neighbours that could still be the minimum
// as one ballot: a few dozen instructions between the loads of consecutive
// steps.
template <int F>
__global__ __launch_bounds__(kPathThreads) void paths_kernel(DenseView dv, CsrView cv,
                                                           PathArgs a) {
  // rows of the current and the previous FP64 re-decision (at most W + 1 <= 65),
  // and the parts of the rows being evaluated
  __shared__ int cur_x[65], prev_x[65];
  __shared__ double cur_d[65], prev_d[65], cur_e[65], prev_e[65];
  __shared__ double part_d[65 * kMaxParts], part_s[65 * kMaxParts];
  int prev_n = 0;
  // the walk is a chain of short dependent steps that shares its compute unit
  // with the field kernels of other streams: its waves issue first
  __builtin_amdgcn_s_setprio(3);
  stage_log_table();
  const int i = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int N = a.is_csr ? cv.N : dv.N;
  const int W = a.adj_w;
  const float* d = a.fields + (int64_t)i * N;
  const Bound bnd = path_bound(a, i);
  const double ea = uniform(bnd.abs), er = uniform(bnd.rel);
  const int Bt = a.is_csr ? cv.B : dv.B;
  // a long dense row of a re-decision is split over several waves; the split
  // depends only on B, so a row's FP64 value does not depend on which other
  // rows are evaluated with it
  const int parts = split_rows(a.is_csr, Bt) ? kMaxParts : 1;
  const double dscale = distance_scale(a.kind);
  const double* p = a.trow + (int64_t)i * Bt;
  const double* lpt = a.tlog + (int64_t)i * Bt;
  if (a.tgt_in_lds) {
    // FP64 target row and its logs in LDS for the row evaluations
    extern __shared__ double tsh[];
    for (int b = threadIdx.x; b < Bt; b += blockDim.x) {
      tsh[b] = p[b];
      tsh[Bt + b] = lpt[b];
    }
    __syncthreads();
    p = tsh;
    lpt = tsh + Bt;
  }
  // the FP32 target row of the level-1 rows, after the FP64 rows when those
  // are staged too
  const float* p32 = nullptr;
  if constexpr (F == 1) {
    if (a.l1) {
      extern __shared__ double tsh[];
      float* ps = reinterpret_cast<float*>(tsh + (a.tgt_in_lds ? 2 * Bt : 0));
      const double* pg = a.trow + (int64_t)i * Bt;
      for (int b = threadIdx.x; b < Bt; b += blockDim.x) ps[b] = (float)pg[b];
      __syncthreads();
      p32 = ps;
    }
  }
  const double* tc = a.tconst + (int64_t)i * 4;
  int32_t* path = a.path + (int64_t)i * (a.max_steps + 1);
  const int t = __builtin_amdgcn_readfirstlane(path_target(a, i));
  const int32_t* __restrict__ adj = a.adj;
  int v = path_source(a, i);
  float cur = d[v];   // FP32 field value at v
  int len = 1;
  int status = 0;
  int rechecks = 0;
  if (threadIdx.x == 0) path[0] = v;
  // lane j < W holds slot j of v's neighbour row; with W <= kPrefetchW every
  // neighbour's own row is loaded in the same round as the neighbours' values,
  // so the next vertex's row is in registers when the step is decided
  const bool pre = W <= kPrefetchW;
  int ul = lane < W ? adj[(int64_t)v * W + lane] : -1;
  for (;;) {
    // the walk state is wave-uniform; say so, so that its branches are scalar
    v = __builtin_amdgcn_readfirstlane(v);
    len = __builtin_amdgcn_readfirstlane(len);
    cur = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(cur)));
    if (v == t) {
      status = 0;
      break;
    }
    if (len - 1 >= a.max_steps) {
      status = 2;
      break;
    }
    // one round of independent loads: the neighbours' field values and, for
    // narrow rows, the neighbours' own rows
    float vl = __builtin_inff();
    int nrow[kPrefetchW];
#pragma unroll
    for (int q = 0; q < kPrefetchW; ++q) nrow[q] = -1;
    if (ul >= 0) {
      vl = d[ul];
      if (pre)
#pragma unroll
        for (int q = 0; q < kPrefetchW; ++q)
          if (q < W) nrow[q] = adj[(int64_t)ul * W + q];
    }
    const uint64_t live = __ballot(ul >= 0);
    if (live == 0) {
      status = 1;
      break;
    }
    // best neighbour: smallest key, ties to the lowest id
    const uint32_t kl = ul >= 0 ? fkey(__float_as_uint(vl)) : 0xffffffffu;
    const uint32_t k1 = wave_min(kl, W);
    const uint64_t eq = __ballot(kl == k1) & live;
    int L = (int)__builtin_ctzll(eq);
    int u1 = __builtin_amdgcn_readlane(ul, L);
    if (eq & (eq - 1)) {
      u1 = (int)wave_min(((eq >> lane) & 1) ? (uint32_t)ul : 0xffffffffu, W);
      L = (int)__builtin_ctzll(__ballot(ul == u1) & eq);
    }
    const double v1 = (double)unkey(k1);
    const double e1 = ea + er * fabs(v1);
    const double dvv = (double)cur;
    const double ev = ea + er * fabs(dvv);
    // neighbours that could be the minimum: all but those whose lower end
    // lies above the best's upper end (the test is monotone in the value)
    const double vj = (double)vl;
    const uint64_t cand = __ballot(ul >= 0 && !(vj - (ea + er * fabs(vj)) > v1 + e1));
    const bool certain = (cand & ~(1ull << L)) == 0;
    int next = u1;
    float nextv = unkey(k1);
    bool stuck;
    if (certain && v1 + e1 < dvv - ev) {
      stuck = false;
    } else if (certain && v1 - e1 >= dvv + ev) {
      stuck = true;
    } else {
      // Re-decision.  Rows: the current vertex, then every candidate
      // neighbour, each with a value and a bound (cur_e; 0 for an FP64 value,
      // negative while unknown).  KL walks on dense rows first take level-1
      // values (l1_dense); if their intervals settle the step it is the step
      // the FP64 values take, else the rows are computed in FP64 and the step
      // is decided on those (ties to the lowest id).  Wave (task % waves)
      // computes each part of a row; rows of the previous re-decision are
      // reused at the level they have.
      ++rechecks;
      const int nw = (int)(blockDim.x >> 6);
      int pos = 0;
      {
        uint64_t rest = cand | (1ull << L);
        for (;;) {
          int x = v;
          if (pos > 0) {
            if (rest == 0) break;
            x = __builtin_amdgcn_readlane(ul, (int)__builtin_ctzll(rest));
            rest &= rest - 1;
          }
          double dx = 0.0, ex = -1.0;
          for (int q = 0; q < prev_n; ++q)
            if (prev_x[q] == x) {
              dx = prev_d[q];
              ex = prev_e[q];
              break;
            }
          if (threadIdx.x == 0) {
            cur_x[pos] = x;
            cur_d[pos] = dx;
            cur_e[pos] = ex;
          }
          ++pos;
        }
      }
      __syncthreads();
      bool settled = false;
      int best_u = 0x7fffffff;
      if constexpr (F == 1) {
        if (a.l1) {
          int task = 0;
          for (int q = 0; q < pos; ++q) {
            if (cur_e[q] >= 0.0) continue;   // known
            const int x = cur_x[q];
            for (int part = 0; part < parts; ++part, ++task)
              if (task % nw == wave) {
                int lo, hi;
                part_range(Bt, part, parts, lo, hi);
                double sp;
                const double ap = l1_dense(dv, p32, x, lo, hi, sp);
                if (lane == 0) {
                  part_d[q * kMaxParts + part] = ap;
                  part_s[q * kMaxParts + part] = sp;
                }
              }
          }
          __syncthreads();
          if (threadIdx.x < pos && cur_e[threadIdx.x] < 0.0) {
            double A = 0.0, S = 0.0;
            for (int part = 0; part < parts; ++part) {
              A += part_d[threadIdx.x * kMaxParts + part];
              S += part_s[threadIdx.x * kMaxParts + part];
            }
            cur_d[threadIdx.x] = tc[1] - kLn2 * A;
            cur_e[threadIdx.x] = l1_bound(S, tc[0], tc[3], Bt, dv.P64 != nullptr);
          }
          __syncthreads();
          // the best row by value (ties: lowest id); settled when every other
          // candidate's interval lies above the best's, and the best's lies
          // wholly below the current vertex's (a move) or at or above it
          double best = __builtin_inf(), be = 0.0;
          for (int q = 1; q < pos; ++q) {
            const double dq = cur_d[q];
            const int xq = cur_x[q];
            if (dq < best || (dq == best && xq < best_u)) {
              best = dq;
              be = cur_e[q];
              best_u = xq;
            }
          }
          bool sep = true;
          for (int q = 1; q < pos; ++q)
            if (cur_x[q] != best_u && !(cur_d[q] - cur_e[q] > best + be)) sep = false;
          const double lo_v = cur_d[0] - cur_e[0], hi_v = cur_d[0] + cur_e[0];
          if (sep && best + be < lo_v) {
            settled = true;
            stuck = false;
          } else if (sep && best - be >= hi_v) {
            settled = true;
            stuck = true;
          }
        }
      }
      if (!settled) {
        int task = 0;
        for (int q = 0; q < pos; ++q) {
          if (cur_e[q] == 0.0) continue;   // FP64 value known
          const int x = cur_x[q];
          for (int part = 0; part < parts; ++part, ++task)
            if (task % nw == wave) {
              const double pd = exact_part<F>(dv, cv, a.is_csr, a.kind, p, lpt, tc, x, part, parts);
              if (lane == 0) part_d[q * kMaxParts + part] = pd;
            }
        }
        __syncthreads();
        // rows computed here: their parts summed in order
        if (threadIdx.x < pos && cur_e[threadIdx.x] != 0.0) {
          double dsum = 0.0;
          for (int part = 0; part < parts; ++part) dsum += part_d[threadIdx.x * kMaxParts + part];
          cur_d[threadIdx.x] = dsum * dscale;
          cur_e[threadIdx.x] = 0.0;
        }
        __syncthreads();
        double best = __builtin_inf();
        best_u = 0x7fffffff;
        for (int q = 1; q < pos; ++q) {
          const double dx = cur_d[q];
          const int cu = cur_x[q];
          if (dx < best || (dx == best && cu < best_u)) {
            best = dx;
            best_u = cu;
          }
        }
        stuck = !(best < cur_d[0]);
      }
      next = __builtin_amdgcn_readfirstlane(best_u);
      stuck = __builtin_amdgcn_readfirstlane(stuck ? 1 : 0) != 0;
      __syncthreads();   // everyone has read cur_* before it becomes prev_*
      if (threadIdx.x < pos) {
        prev_x[threadIdx.x] = cur_x[threadIdx.x];
        prev_d[threadIdx.x] = cur_d[threadIdx.x];
        prev_e[threadIdx.x] = cur_e[threadIdx.x];
      }
      prev_n = pos;   // uniform
      __syncthreads();
      if (!stuck) {
        const int ln = (int)__builtin_ctzll(__ballot(ul == next) & live);
        nextv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vl), ln));
      }
    }
    if (stuck) {
      status = 1;
      break;
    }
    cur = nextv;
    v = next;
    if (threadIdx.x == 0) path[len] = v;
    ++len;
    // the next vertex's neighbour row: from the lane that held it, or loaded
    if (pre) {
      const int ln = (int)__builtin_ctzll(__ballot(ul == next) & live);
      int nu = -1;
#pragma unroll
      for (int q = 0; q < kPrefetchW; ++q) {
        const int x = __builtin_amdgcn_readlane(nrow[q], ln);
        if (lane == q) nu = x;
      }
      ul = lane < W ? nu : -1;
    } else {
      ul = lane < W ? adj[(int64_t)v * W + lane] : -1;
    }
  }
  for (int k = len + threadIdx.x; k <= a.max_steps; k += blockDim.x) path[k] = -1;
  if (threadIdx.x == 0) {
    a.len[i] = len;
    a.status[i] = status;
    if (a.rechecks) a.rechecks[i] = rechecks;
  }
}

// On-demand walk (Section V: the CPU evaluates the distances only at the
// vertices the path needs).  No field is given: at each step the FP64
// distances of the current vertex's neighbours are computed from the resident
// rows, one row per wave, and the decision is taken on them directly, so the
// walk is the one the exact FP64 field gives.  Rows evaluated at the previous
// step (its neighbours and the vertex itself) are reused.  `rechecks`
// receives the number of rows evaluated.
template <int F>
__global__ __launch_bounds__(256) void paths_on_demand_kernel(DenseView dv, CsrView cv,
                                                              PathArgs a) {
  __shared__ int cur_x[66], prev_x[66];
  __shared__ double cur_d[66], prev_d[66], cur_e[66], prev_e[66], new_d[66], new_e[66];
  __shared__ double first_d;
  stage_log_table();
  const int i = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nw = (int)(blockDim.x >> 6);
  const int W = a.adj_w;
  const int Bt = a.is_csr ? cv.B : dv.B;
  const double* p = a.trow + (int64_t)i * Bt;
  const double* lpt = a.tlog + (int64_t)i * Bt;
  if (a.tgt_in_lds) {
    // FP64 target row and its logs in LDS for the row evaluations
    extern __shared__ double tsh[];
    for (int b = threadIdx.x; b < Bt; b += blockDim.x) {
      tsh[b] = p[b];
      tsh[Bt + b] = lpt[b];
    }
    __syncthreads();
    p = tsh;
    lpt = tsh + Bt;
  }
  // the FP32 target row of the level-1 rows, after the FP64 rows when those
  // are staged too
  const float* p32 = nullptr;
  if constexpr (F == 1) {
    if (a.l1) {
      extern __shared__ double tsh[];
      float* ps = reinterpret_cast<float*>(tsh + (a.tgt_in_lds ? 2 * Bt : 0));
      const double* pg = a.trow + (int64_t)i * Bt;
      for (int b = threadIdx.x; b < Bt; b += blockDim.x) ps[b] = (float)pg[b];
      __syncthreads();
      p32 = ps;
    }
  }
  const double* tc = a.tconst + (int64_t)i * 4;
  int32_t* path = a.path + (int64_t)i * (a.max_steps + 1);
  const int32_t* __restrict__ adj = a.adj;
  const int t = __builtin_amdgcn_readfirstlane(path_target(a, i));
  int v = __builtin_amdgcn_readfirstlane(path_source(a, i));
  if (wave == 0) {
    const double dx = exact_distance<F>(dv, cv, a.is_csr, a.kind, p, lpt, tc, v);
    if (lane == 0) first_d = dx;
  }
  __syncthreads();
  double dcur = uniform(first_d), ecur = 0.0;
  int evals = 1;
  int prev_n = 0;
  int len = 1;
  int status = 0;
  if (threadIdx.x == 0) path[0] = v;
  for (;;) {
    v = __builtin_amdgcn_readfirstlane(v);
    len = __builtin_amdgcn_readfirstlane(len);
    if (v == t) {
      status = 0;
      break;
    }
    if (len - 1 >= a.max_steps) {
      status = 2;
      break;
    }
    const int ul = lane < W ? adj[(int64_t)v * W + lane] : -1;
    const uint64_t live = __ballot(ul >= 0);
    if (live == 0) {
      status = 1;
      break;
    }
    // rows: the current vertex (position 0, known) and its neighbours, each
    // with a value and a bound (0 for an FP64 value, negative while unknown).
    // KL walks on dense rows take level-1 values first (l1_dense, l1_bound)
    // and compute rows in FP64 only when those intervals do not settle the
    // step, which is then the step of the FP64 values.
    uint64_t rest = live;
    int pos = 1;
    if (threadIdx.x == 0) {
      cur_x[0] = v;
      cur_d[0] = dcur;
      cur_e[0] = ecur;
    }
    while (rest) {
      const int x = __builtin_amdgcn_readlane(ul, (int)__builtin_ctzll(rest));
      rest &= rest - 1;
      double dx = 0.0, ex = -1.0;
      for (int q = 0; q < prev_n; ++q)
        if (prev_x[q] == x) {
          dx = prev_d[q];
          ex = prev_e[q];
        }
      if (ex < 0.0) ++evals;
      if (threadIdx.x == 0) {
        cur_x[pos] = x;
        cur_d[pos] = dx;
        cur_e[pos] = ex;
      }
      ++pos;
    }
    __syncthreads();
    bool settled = false, stop = false;
    int best_u = 0x7fffffff;
    double best = __builtin_inf(), best_e = 0.0;
    if constexpr (F == 1) {
      if (a.l1) {
        int task = 0;
        for (int q = 1; q < pos; ++q) {
          if (cur_e[q] >= 0.0) continue;   // known
          if (task++ % nw == wave) {
            double sp;
            const double ap = l1_dense(dv, p32, cur_x[q], 0, Bt, sp);
            if (lane == 0) {
              new_d[q] = tc[1] - kLn2 * ap;
              new_e[q] = l1_bound(sp, tc[0], tc[3], Bt, dv.P64 != nullptr);
            }
          }
        }
        __syncthreads();
        if (threadIdx.x < pos && cur_e[threadIdx.x] < 0.0) {
          cur_d[threadIdx.x] = new_d[threadIdx.x];
          cur_e[threadIdx.x] = new_e[threadIdx.x];
        }
        __syncthreads();
        for (int q = 1; q < pos; ++q) {
          const double dq = cur_d[q];
          const int xq = cur_x[q];
          if (dq < best || (dq == best && xq < best_u)) {
            best = dq;
            best_e = cur_e[q];
            best_u = xq;
          }
        }
        bool sep = true;
        for (int q = 1; q < pos; ++q)
          if (cur_x[q] != best_u && !(cur_d[q] - cur_e[q] > best + best_e)) sep = false;
        if (sep && best + best_e < cur_d[0] - cur_e[0]) {
          settled = true;
        } else if (sep && best - best_e >= cur_d[0] + cur_e[0]) {
          settled = true;
          stop = true;
        }
      }
    }
    if (!settled) {
      // FP64 values for every row that has none (the current vertex included)
      int task = 0;
      for (int q = 0; q < pos; ++q) {
        if (cur_e[q] == 0.0) continue;
        if (task++ % nw == wave) {
          const double dx = exact_distance<F>(dv, cv, a.is_csr, a.kind, p, lpt, tc, cur_x[q]);
          if (lane == 0) new_d[q] = dx;
        }
      }
      __syncthreads();
      if (threadIdx.x < pos && cur_e[threadIdx.x] != 0.0) {
        cur_d[threadIdx.x] = new_d[threadIdx.x];
        cur_e[threadIdx.x] = 0.0;
      }
      __syncthreads();
      best = __builtin_inf();
      best_u = 0x7fffffff;
      for (int q = 1; q < pos; ++q) {
        const double dx = cur_d[q];
        const int cu = cur_x[q];
        if (dx < best || (dx == best && cu < best_u)) {
          best = dx;
          best_u = cu;
        }
      }
      best_e = 0.0;
      stop = !(best < cur_d[0]);
    }
    best = uniform(best);
    best_e = uniform(best_e);
    best_u = __builtin_amdgcn_readfirstlane(best_u);
    stop = __builtin_amdgcn_readfirstlane(stop ? 1 : 0) != 0;
    __syncthreads();   // everyone has read cur_* before it becomes prev_*
    if (threadIdx.x < pos) {
      prev_x[threadIdx.x] = cur_x[threadIdx.x];
      prev_d[threadIdx.x] = cur_d[threadIdx.x];
      prev_e[threadIdx.x] = cur_e[threadIdx.x];
    }
    prev_n = pos;
    __syncthreads();
    if (stop) {
      status = 1;
      break;
    }
    v = best_u;
    dcur = best;
    ecur = best_e;
    if (threadIdx.x == 0) path[len] = v;
    ++len;
  }
  for (int k = len + threadIdx.x; k <= a.max_steps; k += blockDim.x) path[k] = -1;
  if (threadIdx.x == 0) {
    a.len[i] = len;
    a.status[i] = status;
    if (a.rechecks) a.rechecks[i] = evals;
  }
}

// One thread per (field, vertex).  Interval test against the field's bound:
// a neighbour is certainly lower when its upper end is below v's lower end,
// certainly not lower when its lower end is at or above v's upper end.
__global__ __launch_bounds__(256) void local_minima_kernel(PathArgs a, int32_t N, uint8_t* cls,
                                                           int32_t* counts) {
  const int64_t total = (int64_t)N * a.T;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / N);
    const int v = (int)(idx - (int64_t)i * N);
    const float* d = a.fields + (int64_t)i * N;
    const Bound bnd = path_bound(a, i);
    int c = 0;
    if (v != path_target(a, i)) {
      const double dv = (double)d[v];
      const double lo_v = dv - (bnd.abs + bnd.rel * fabs(dv));
      const double hi_v = dv + (bnd.abs + bnd.rel * fabs(dv));
      bool lower = false, unsure = false;
      for (int j = 0; j < a.adj_w; ++j) {
        const int u = a.adj[(int64_t)v * a.adj_w + j];
        if (u < 0) break;
        const double du = (double)d[u];
        const double e = bnd.abs + bnd.rel * fabs(du);
        if (du + e < lo_v) {
          lower = true;
          break;
        }
        if (du - e < hi_v) unsure = true;
      }
      c = lower ? 0 : (unsure ? 2 : 1);
    }
    if (cls) cls[idx] = (uint8_t)c;
    if (counts && c) atomicAdd(counts + 2 * i + (c - 1), 1);
  }
}

// Re-decision of the census in FP64: every vertex of class 2 (undecided) gets
// the FP64 distances of itself and its neighbours from the resident rows (one
// wave, rows in turn) and becomes 1 if no neighbour is strictly lower (the
// oracle's rule: min over neighbours >= d(v)), else 0.  A wave takes 64
// vertices at a time and works through the undecided ones among them.
template <int F>
__global__ __launch_bounds__(256) void resolve_minima_kernel(DenseView dv, CsrView cv, PathArgs a,
                                                             int32_t N, uint8_t* cls) {
  stage_log_table();
  const int lane = threadIdx.x & 63;
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t total = (int64_t)N * a.T;
  const int Bt = a.is_csr ? cv.B : dv.B;
  for (int64_t base = wid * 64; base < total; base += nw * 64) {
    const int64_t idx = base + lane;
    uint64_t m = __ballot(idx < total && cls[idx] == 2);
    while (m) {
      const int l = (int)__builtin_ctzll(m);
      m &= m - 1;
      const int64_t e = base + l;
      const int i = __builtin_amdgcn_readfirstlane((int)(e / N));
      const int v = __builtin_amdgcn_readfirstlane((int)(e - (int64_t)i * N));
      const double* p = a.trow + (int64_t)i * Bt;
      const double* lp = a.tlog + (int64_t)i * Bt;
      const double* tc = a.tconst + (int64_t)i * 4;
      const double d0 = exact_distance<F>(dv, cv, a.is_csr, a.kind, p, lp, tc, v);
      bool minimum = true;
      for (int j = 0; j < a.adj_w && minimum; ++j) {
        const int u = __builtin_amdgcn_readfirstlane(a.adj[(int64_t)v * a.adj_w + j]);
        if (u < 0) break;
        if (exact_distance<F>(dv, cv, a.is_csr, a.kind, p, lp, tc, u) < d0) minimum = false;
      }
      if (lane == 0) cls[e] = minimum ? 1 : 0;
    }
  }
}

// counts[i] = (minima, undecided) of field i from the classes.
__global__ __launch_bounds__(256) void count_classes_kernel(const uint8_t* cls, int32_t T,
                                                            int32_t N, int32_t* counts) {
  const int64_t total = (int64_t)N * T;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int c = cls[idx];
    if (c) atomicAdd(counts + 2 * (idx / N) + (c - 1), 1);
  }
}

// Clears the census counters with a kernel (not a memset node), so a caller
// may capture the call in a graph.
__global__ void zero_counts_kernel(int32_t* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

hipError_t launch_local_minima(PathArgs a, int32_t N, uint8_t* cls, int32_t* counts,
                               hipStream_t s) {
  if (counts) {
    hipLaunchKernelGGL(zero_counts_kernel, dim3(1), dim3(256), 0, s, counts, 2 * a.T);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t total = (int64_t)N * a.T;
  int64_t grid = (total + 255) / 256;
  const int64_t cap = (int64_t)num_cus() * 16;
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(local_minima_kernel, dim3((unsigned)grid), dim3(256), 0, s, a, N, cls,
                     counts);
  return hipGetLastError();
}

// fn(std::integral_constant<int, F>{}) for the kind family F of `kind`.
template <typename Fn>
static hipError_t by_family(int kind, Fn fn) {
  switch (kind_family(kind)) {
    case 0: return fn(std::integral_constant<int, 0>{});
    case 1: return fn(std::integral_constant<int, 1>{});
    case 2: return fn(std::integral_constant<int, 2>{});
    case 3: return fn(std::integral_constant<int, 3>{});
    case 4: return fn(std::integral_constant<int, 4>{});
    default: return fn(std::integral_constant<int, 5>{});
  }
}

hipError_t launch_resolve_minima(DenseView dv, CsrView cv, PathArgs a, int32_t N, uint8_t* cls,
                                 int32_t* counts, hipStream_t s) {
  const int64_t total = (int64_t)N * a.T;
  int64_t grid = (total + 255) / 256;
  const int64_t cap = (int64_t)num_cus() * 8;
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
  hipError_t e = by_family(a.kind, [&](auto f) {
    hipLaunchKernelGGL(resolve_minima_kernel<decltype(f)::value>, dim3((unsigned)grid), dim3(256),
                       0, s, dv, cv, a, N, cls);
    return hipGetLastError();
  });
  if (e != hipSuccess || !counts) return e;
  hipLaunchKernelGGL(zero_counts_kernel, dim3(1), dim3(256), 0, s, counts, 2 * a.T);
  hipLaunchKernelGGL(count_classes_kernel, dim3((unsigned)grid), dim3(256), 0, s, cls, a.T, N,
                     counts);
  return hipGetLastError();
}

// FP64 fields: every row x of every target by exact_distance (one wave per
// row), the evaluation the FP64 re-decisions use; the target's own entry is
// 0 by definition (d(t, t) = 0 for every kind).  Grid: (row groups of 4, T).
template <int F>
__global__ __launch_bounds__(256) void exact_fields_kernel(DenseView dv, CsrView cv, PathArgs a,
                                                           int32_t N, double* out) {
  stage_log_table();
  const int i = blockIdx.y;
  const int64_t x = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (x >= N) return;
  const int Bt = a.is_csr ? cv.B : dv.B;
  const int t = path_target(a, i);
  const double d = exact_distance<F>(dv, cv, a.is_csr, a.kind, a.trow + (int64_t)i * Bt,
                                  a.tlog + (int64_t)i * Bt, a.tconst + (int64_t)i * 4, (int)x);
  if ((threadIdx.x & 63) == 0) out[(int64_t)i * N + x] = x == t ? 0.0 : d;
}

hipError_t launch_exact_fields(DenseView dv, CsrView cv, PathArgs a, int32_t N, double* out,
                               hipStream_t s) {
  return by_family(a.kind, [&](auto f) {
    hipLaunchKernelGGL(exact_fields_kernel<decltype(f)::value>,
                       dim3((unsigned)((N + 3) / 4), (unsigned)a.T), dim3(256), 0, s, dv, cv, a, N,
                       out);
    return hipGetLastError();
  });
}

hipError_t launch_target_rows(DenseView dv, CsrView cv, PathArgs a, double* trow, double* tlog,
                              double* tconst, hipStream_t s) {
  hipLaunchKernelGGL(target_rows_kernel, dim3(a.T), dim3(256), 0, s, dv, cv, a, trow, tlog,
                     tconst);
  return hipGetLastError();
}

// Target rows of up to kLdsTargetMax entries are staged in LDS (16 bytes per
// entry: the row and its logs).  Longer rows are read from the target-row
// buffers in the same load rounds as the kernel rows: a walk block holding
// 130 KB of LDS (B = 8,146) leaves no room on its CU for the field kernels
// that run beside the walks, which then lose a quarter of the machine (the
// dense KL stream next to 64 walks at 1025²: 6.98 ms with the row in LDS,
// 5.79 ms without, against 5.1 ms alone; the walks 14.6 and 16.7 ms).
constexpr int kLdsTargetMax = 2048;

// Level-1 rows read an FP32 copy of the target row from LDS (4 bytes per
// entry); walks on longer rows use FP64 re-decisions only.
constexpr int kL1LdsMax = 16384;

template <typename K>
static hipError_t launch_with_target(K kern, int threads, DenseView dv, CsrView cv, PathArgs a,
                                     hipStream_t s) {
  const int B = a.is_csr ? cv.B : dv.B;
  a.tgt_in_lds = B <= kLdsTargetMax ? 1 : 0;
  if (a.is_csr || B > kL1LdsMax) a.l1 = 0;
  const size_t lds = (a.tgt_in_lds ? 16 * (size_t)B : 0) + (a.l1 ? 4 * (size_t)B : 0);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(a.T), dim3(threads), lds, s, dv, cv, a);
  return hipGetLastError();
}

hipError_t launch_paths(DenseView dv, CsrView cv, PathArgs a, hipStream_t s) {
  const int threads = split_rows(a.is_csr, a.is_csr ? cv.B : dv.B) ? kPathThreads : 256;
  return by_family(a.kind, [&](auto f) {
    return launch_with_target(paths_kernel<decltype(f)::value>, threads, dv, cv, a, s);
  });
}

hipError_t launch_paths_on_demand(DenseView dv, CsrView cv, PathArgs a, hipStream_t s) {
  return by_family(a.kind, [&](auto f) {
    return launch_with_target(paths_on_demand_kernel<decltype(f)::value>, 256, dv, cv, a, s);
  });
}

}  // namespace dd
