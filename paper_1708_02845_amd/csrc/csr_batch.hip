// Truncated (CSR) fields of many targets in one pass over the stored rows
// (Section V, "Precision": the truncated kernel; eqs. 34-35 on it).
//
// For target t with truncated row p~ (support S_t, W_t = sum p~, Hb_t =
// sum p~ log2 p~) and row x with stored entries q on S_x, floor phi_x and
// Q_x = sum_{S_x} q, the truncated fields rearrange to one product-like sum
// over the stored entries of x:
//   TV_tau(x, t) = sum_{S_x} |q - p~| + sum_{S_t \ S_x} p~
//                = W_t + Q_x - 2 sum_{S_x} min(q, p~)
//   KL_tau(x, t) / ln 2 = Hb_t - sum_{S_x} p~ log2 q - log2 phi_x (W_t - sum_{S_x} p~)
//                = Hb_t - log2(phi_x) W_t - sum_{S_x} p~ g,   g = log2(q / phi_x) >= 0
// since p~ is 0 outside S_t.  Each stored entry is read once per launch and
// costs two VALU operations (TV) or one FMA (KL) per target.  TV runs in
// unsigned fixed point (values times 2^s, rounded to nearest) when the stored
// row sums allow it: min commutes with the monotone rounding, the sums are
// exact integers (no FP64 carries), and two entries' minima and the
// accumulator combine in one v_add3_u32.
//
// Layout of the work: a wave owns R consecutive rows and all targets of the
// launch (TPL targets per lane, up to 256).  The target rows are a dense
// block tb[b][64*TPL] (zeros off the supports) streamed through LDS in chunks
// of kKC columns; for every chunk each row's entries in it (a contiguous run,
// columns ascending) are taken from a 64-entry register window, one entry at a
// time as wave-uniform values (v_readlane), and each lane reads its targets'
// weights for that column from LDS.  The next window of each row is loaded
// while the current one is consumed.  FP32 partial sums over one chunk are
// added into FP64 accumulators after every chunk.  Chunks in which none of a
// workgroup's rows has entries are not staged.
#include "dd_internal.h"

namespace dd {
namespace {

constexpr int kKC = 32;       // columns per LDS chunk
constexpr int kWaves = 8;     // waves per workgroup
constexpr int kEnd = 0x7fffffff;
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }

// Stored value of the FP16 form: FP16 bits times the row's 2^-e_x.
__device__ __forceinline__ float f16_value(uint16_t h, float rs) {
  return (float)__builtin_bit_cast(_Float16, h) * rs;
}

// Fixed-point value of q >= 0: q * 2^shift rounded to nearest (exact scaling).
__device__ __forceinline__ uint32_t fixq(float q, int shift) {
  return __float2uint_rn(ldexpf(q, shift));
}

__device__ __forceinline__ int rdlane(int v, int j) { return __builtin_amdgcn_readlane(v, j); }
__device__ __forceinline__ float rdlane(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

__global__ void clear_block_kernel(float4* __restrict__ p, int64_t n4) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// One workgroup per target slot: scatter the truncated target row into column
// `slot` of tb (as fixed-point bits when shift > 0) and reduce W_t and Hb_t in
// FP64 (the product p log2 p in FP32, as the single-target pass does).
__global__ __launch_bounds__(256) void csr_targets_kernel(CsrView v, TargetList tl, int32_t Tp,
                                                          int shift, float* __restrict__ tb,
                                                          double* __restrict__ wt,
                                                          double* __restrict__ hbt) {
  const int slot = blockIdx.x;
  const int32_t t = tl.t[slot];
  const int64_t s = v.start[t];
  const int n = v.len[t];
  const float rs = v.val16 ? v.rscale[t] : 1.f;
  double w = 0.0, hb = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int b = v.col[s + i];
    const float p = v.val16 ? f16_value(v.val16[s + i], rs) : v.val[s + i];
    tb[(int64_t)b * Tp + slot] = shift ? __uint_as_float(fixq(p, shift)) : p;
    w += (double)p;
    hb += (double)(p * hw_log2(p));
  }
  __shared__ double red[2][4];
  for (int off = 32; off > 0; off >>= 1) {
    w += __shfl_xor(w, off);
    hb += __shfl_xor(hb, off);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = w;
    red[1][threadIdx.x >> 6] = hb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      a += red[0][i];
      c += red[1][i];
    }
    wt[slot] = a;
    hbt[slot] = c;
  }
}

// A window is 64 consecutive entries of one row, starting at entry `base`:
// lane i holds entry base + i.  fetch_window issues the loads only (index
// clamped into the row, so every lane loads and no result is consumed yet);
// take_window turns the fetched column and value into the working form:
// column kEnd past the row's end, and q (TV) or g = log2(q / phi) (KL).
// With F16 the fetched value is the FP16 bits (carried in a float register)
// and q = FP16 value times the row's 2^-e_x.
// The loaders reject rows without entries; the rows past N of the last
// workgroup (n = 0) read entry 0 of the arrays and mark every lane past the end.
template <int F16>
__device__ __forceinline__ void fetch_window(const CsrView& v, int64_t s, int n, int base,
                                             int lane, int& rc, float& rq) {
  const int64_t i = n > 0 ? s + min(base + lane, n - 1) : 0;
  rc = v.col[i];
  rq = F16 ? __int_as_float((int)v.val16[i]) : v.val[i];
}

template <int KIND, int F16>
__device__ __forceinline__ void take_window(int n, int base, int lane, float rphi, float rs,
                                            int shift, int rc, float rq, int& col, float& val,
                                            double& qsum) {
  const bool ok = base + lane < n;
  col = ok ? rc : kEnd;
  if (F16) rq = f16_value((uint16_t)__float_as_int(rq), rs);
  if (KIND == 0 || KIND == 2) {
    val = KIND == 2 ? __uint_as_float(fixq(rq, shift)) : rq;
    qsum += ok ? (double)rq : 0.0;
  } else {
    val = hw_log2(rq * rphi);   // never read past the row's end
  }
}

// One stored entry (column c within the chunk, value g) for the lane's TPL targets.
template <int KIND, int TPL>
__device__ __forceinline__ void load_weights(const float* chunk, int c, int lane, float (&p)[TPL]) {
  const float* pw = chunk + c * (64 * TPL) + lane * TPL;
  if constexpr (TPL == 4) {
    const float4 q4 = *reinterpret_cast<const float4*>(pw);
    p[0] = q4.x;
    p[1] = q4.y;
    p[2] = q4.z;
    p[3] = q4.w;
  } else if constexpr (TPL == 2) {
    const float2 q2 = *reinterpret_cast<const float2*>(pw);
    p[0] = q2.x;
    p[1] = q2.y;
  } else {
    p[0] = pw[0];
  }
}

template <int KIND, int TPL>
__device__ __forceinline__ void accumulate(const float (&p)[TPL], float g, float (&a)[TPL]) {
#pragma unroll
  for (int i = 0; i < TPL; ++i) {
    if (KIND == 0)
      a[i] += fminf(p[i], g);
    else
      a[i] = fmaf(p[i], g, a[i]);
  }
}

template <int KIND, int TPL, int R, int F16>
__global__ __launch_bounds__(kWaves * 64) void csr_batch_kernel(CsrView v,
                                                               const float* __restrict__ tb,
                                                               const double* __restrict__ wt,
                                                               const double* __restrict__ hbt,
                                                                               TargetList tl, int32_t T,
                                                               int shift,
                                                               float* __restrict__ out) {
  constexpr int TP = 64 * TPL;                  // target slots of the block
  constexpr int NV4 = kKC * TP / 4 / (kWaves * 64);   // float4 per thread per chunk
  static_assert(NV4 >= 1 && NV4 * 4 * kWaves * 64 == kKC * TP, "chunk split");
  __shared__ f4 chunk4[kKC * TP / 4];
  const float* chunk = reinterpret_cast<const float*>(chunk4);

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t row0 = ((int64_t)blockIdx.x * kWaves + wave) * R;

  int64_t rs[R];
  int rn[R], wnext[R], j0[R], col[R], ncol[R];
  float val[R], nval[R], rphi[R], rsc[R];
  double qsum[R];
  float a32[R][TPL];
  double a64[R][TPL];
  uint32_t au[R][TPL];   // fixed-point TV sums
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t row = row0 + r;
    const bool ok = row < v.N;
    rs[r] = ok ? v.start[row] : 0;
    rn[r] = ok ? v.len[row] : 0;
    rphi[r] = ok && KIND == 1 ? (float)(1.0 / v.phi[row]) : 0.f;
    rsc[r] = ok && F16 ? v.rscale[row] : 1.f;
    qsum[r] = 0.0;
    j0[r] = 0;
    int rc;
    float rq;
    fetch_window<F16>(v, rs[r], rn[r], 0, lane, rc, rq);
    take_window<KIND, F16>(rn[r], 0, lane, rphi[r], rsc[r], shift, rc, rq, col[r], val[r],
                           qsum[r]);
    fetch_window<F16>(v, rs[r], rn[r], 64, lane, ncol[r], nval[r]);
    wnext[r] = 128;
#pragma unroll
    for (int i = 0; i < TPL; ++i) {
      a32[r][i] = 0.f;
      a64[r][i] = 0.0;
      au[r][i] = 0u;
    }
  }

  // Chunks that none of the workgroup's rows has an entry in are skipped:
  // after each chunk every wave posts the lowest column its rows still have to
  // consume, and the next chunk is the one holding the smallest of these.
  __shared__ int next_col[kWaves];
  const int nch = (v.B + kKC - 1) / kKC;
  const f4* tb4 = reinterpret_cast<const f4*>(tb);
  auto post_next = [&]() {
    int m = kEnd;
#pragma unroll
    for (int r = 0; r < R; ++r) m = min(m, j0[r] < 64 ? rdlane(col[r], j0[r]) : kEnd);
    if (lane == 0) next_col[wave] = m;
  };
  auto chunk_after = [&]() {
    int m = next_col[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) m = min(m, next_col[w]);
    return __builtin_amdgcn_readfirstlane(m / kKC);
  };
  f4 pre[NV4];
  post_next();
  __syncthreads();
  int ch = chunk_after();
  if (ch < nch) {
#pragma unroll
    for (int u = 0; u < NV4; ++u)
      pre[u] = tb4[(int64_t)ch * (kKC * TP / 4) + threadIdx.x + u * kWaves * 64];
  }
  while (ch < nch) {
#pragma unroll
    for (int u = 0; u < NV4; ++u) chunk4[threadIdx.x + u * kWaves * 64] = pre[u];
    __syncthreads();
    if (ch + 1 < nch) {   // the next chunk, in case it is needed
      const f4* src = tb4 + (int64_t)(ch + 1) * (kKC * TP / 4);
#pragma unroll
      for (int u = 0; u < NV4; ++u) pre[u] = src[threadIdx.x + u * kWaves * 64];
    }
    const int k0 = ch * kKC;
    const int kend = k0 + kKC;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int done = 0;
      while (true) {
        // columns ascend, so the window's entries below kend are a prefix
        const int j1 = (int)__popcll(__ballot(col[r] < kend));
        int j = j0[r];
        done += j1 - j;
        for (; j + 2 <= j1; j += 2) {
          const int c0 = rdlane(col[r], j) - k0;
          const int c1 = rdlane(col[r], j + 1) - k0;
          const float g0 = rdlane(val[r], j);
          const float g1 = rdlane(val[r], j + 1);
          float p0[TPL], p1[TPL];
          load_weights<KIND, TPL>(chunk, c0, lane, p0);
          load_weights<KIND, TPL>(chunk, c1, lane, p1);
          if constexpr (KIND == 2) {
            const uint32_t q0 = __float_as_uint(g0), q1 = __float_as_uint(g1);
#pragma unroll
            for (int i = 0; i < TPL; ++i)
              au[r][i] += min(q0, __float_as_uint(p0[i])) + min(q1, __float_as_uint(p1[i]));
          } else {
            accumulate<KIND, TPL>(p0, g0, a32[r]);
            accumulate<KIND, TPL>(p1, g1, a32[r]);
          }
        }
        if (j < j1) {
          const int c0 = rdlane(col[r], j) - k0;
          const float g0 = rdlane(val[r], j);
          float p0[TPL];
          load_weights<KIND, TPL>(chunk, c0, lane, p0);
          if constexpr (KIND == 2) {
            const uint32_t q0 = __float_as_uint(g0);
#pragma unroll
            for (int i = 0; i < TPL; ++i) au[r][i] += min(q0, __float_as_uint(p0[i]));
          } else {
            accumulate<KIND, TPL>(p0, g0, a32[r]);
          }
        }
        j0[r] = j1;
        // the whole window consumed and more entries left: move to the next
        if (j1 == 64 && wnext[r] - 64 < rn[r]) {
          take_window<KIND, F16>(rn[r], wnext[r] - 64, lane, rphi[r], rsc[r], shift, ncol[r],
                                 nval[r], col[r], val[r], qsum[r]);
          j0[r] = 0;
          fetch_window<F16>(v, rs[r], rn[r], wnext[r], lane, ncol[r], nval[r]);
          wnext[r] += 64;
          continue;
        }
        break;
      }
      if (KIND != 2 && done > 0) {
#pragma unroll
        for (int i = 0; i < TPL; ++i) {
          a64[r][i] += (double)a32[r][i];
          a32[r][i] = 0.f;
        }
      }
    }
    post_next();
    __syncthreads();   // the chunk is consumed and every wave's next column posted
    const int nxt = chunk_after();   // > ch: every entry below kend is consumed
    if (nxt < nch && nxt != ch + 1) {
#pragma unroll
      for (int u = 0; u < NV4; ++u)
        pre[u] = tb4[(int64_t)nxt * (kKC * TP / 4) + threadIdx.x + u * kWaves * 64];
    }
    ch = nxt;
  }

  double W[TPL], Hb[TPL];
#pragma unroll
  for (int i = 0; i < TPL; ++i) {
    const int slot = lane * TPL + i;
    W[i] = slot < T ? wt[slot] : 0.0;
    Hb[i] = slot < T ? hbt[slot] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t row = row0 + r;
    double Q = 0.0, lphi = 0.0;
    if (KIND == 0 || KIND == 2) {
      Q = qsum[r];
      for (int off = 32; off > 0; off >>= 1) Q += __shfl_xor(Q, off);
    }
    if (row >= v.N) continue;
    if (KIND == 1) lphi = v.lphi[row];
#pragma unroll
    for (int i = 0; i < TPL; ++i) {
      const int slot = lane * TPL + i;
      if (slot >= T) continue;
      double d;
      if (KIND == 0)
        d = W[i] + Q - 2.0 * a64[r][i];
      else if (KIND == 2)
        d = W[i] + Q - 2.0 * ldexp((double)au[r][i], -shift);
      else
        d = (Hb[i] - lphi * W[i] - a64[r][i]) * 0.69314718055994530942;
      out[(int64_t)slot * v.N + row] = row == tl.t[slot] ? 0.f : (float)d;
    }
  }
}

constexpr int rows_per_wave(int TPL) { return TPL == 4 ? 4 : 8; }

template <int KIND, int TPL>
hipError_t batch_launch(CsrView v, const float* tb, const double* wt, const double* hbt,
                        TargetList tl, int32_t T, int shift, float* out, hipStream_t s) {
  constexpr int R = rows_per_wave(TPL);
  const int64_t rows_per_block = (int64_t)kWaves * R;
  const int64_t grid = (v.N + rows_per_block - 1) / rows_per_block;
  if (v.val16)
    hipLaunchKernelGGL((csr_batch_kernel<KIND, TPL, R, 1>), dim3((unsigned)grid),
                       dim3(kWaves * 64), 0, s, v, tb, wt, hbt, tl, T, shift, out);
  else
    hipLaunchKernelGGL((csr_batch_kernel<KIND, TPL, R, 0>), dim3((unsigned)grid),
                       dim3(kWaves * 64), 0, s, v, tb, wt, hbt, tl, T, shift, out);
  return hipGetLastError();
}

int tpl_for(int32_t T) { return T <= 64 ? 1 : (T <= 128 ? 2 : 4); }

}  // namespace

size_t csr_batch_workspace(CsrView v, int32_t T) {
  const int64_t tp = 64 * tpl_for(T);
  const int64_t bpad = (v.B + kKC - 1) / kKC * kKC;
  return (size_t)(bpad * tp) * sizeof(float) + 2 * sizeof(double) * (size_t)kMaxBatch;
}

hipError_t launch_csr_batch(CsrView v, TargetList tl, int32_t T, int kind, int tv_shift, void* ws,
                            float* out, hipStream_t s) {
  if (T <= 0 || T > kMaxBatch) return hipErrorInvalidValue;
  const int tpl = tpl_for(T);
  const int64_t tp = 64 * tpl;
  const int64_t bpad = (v.B + kKC - 1) / kKC * kKC;
  float* tb = static_cast<float*>(ws);
  double* wt = reinterpret_cast<double*>(tb + bpad * tp);
  double* hbt = wt + kMaxBatch;
  const int64_t n4 = bpad * tp / 4;
  const int cgrid = (int)std::min<int64_t>((n4 + 255) / 256, 4096);
  hipLaunchKernelGGL(clear_block_kernel, dim3(cgrid), dim3(256), 0, s,
                     reinterpret_cast<float4*>(tb), n4);
  const int shift = kind == 0 ? tv_shift : 0;
  hipLaunchKernelGGL(csr_targets_kernel, dim3(T), dim3(256), 0, s, v, tl, (int32_t)tp, shift, tb,
                     wt, hbt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (kind == 0 && shift > 0) {
    if (tpl == 1) return batch_launch<2, 1>(v, tb, wt, hbt, tl, T, shift, out, s);
    if (tpl == 2) return batch_launch<2, 2>(v, tb, wt, hbt, tl, T, shift, out, s);
    return batch_launch<2, 4>(v, tb, wt, hbt, tl, T, shift, out, s);
  }
  if (kind == 0) {
    if (tpl == 1) return batch_launch<0, 1>(v, tb, wt, hbt, tl, T, 0, out, s);
    if (tpl == 2) return batch_launch<0, 2>(v, tb, wt, hbt, tl, T, 0, out, s);
    return batch_launch<0, 4>(v, tb, wt, hbt, tl, T, 0, out, s);
  }
  if (tpl == 1) return batch_launch<1, 1>(v, tb, wt, hbt, tl, T, 0, out, s);
  if (tpl == 2) return batch_launch<1, 2>(v, tb, wt, hbt, tl, T, 0, out, s);
  return batch_launch<1, 4>(v, tb, wt, hbt, tl, T, 0, out, s);
}

}  // namespace dd
