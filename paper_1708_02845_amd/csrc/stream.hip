// Streaming distance fields: one pass over the kernel rows for one target.
//
// TV (Section IV, eq. 34):  d(x) = sum_b |p_b - q_b|
// KL (Section IV, eq. 35):  d(x) = sum_b p_b log(p_b / q_b), p = target row
// chi-squared and squared Hellinger (f-divergences, Section VI):
//   d(x) = sum_b (q_b - p_b)^2 / p_b,   d(x) = sum_b (sqrt q_b - sqrt p_b)^2
// and the two families Section VI names: f(u) = |1 - u|^k for integer k, and
// the alpha-divergences f(u) = 4/(1 - alpha^2) (1 - u^((1+alpha)/2)).
//
// Mapping (gfx950): a group of LPR lanes (16, 32 or 64) owns one row x and
// sweeps it with 16-byte loads, UNROLL loads in flight per lane; the target
// row p (and log2 p for KL) sits in LDS, staged once per workgroup; the group
// then reduces its FP64 partial sums with cross-lane shuffles.  Workgroups
// stride over rows, so the grid is sized to the machine, not to N.
//
// KL evaluates each term as p_b * (log2 p_b - log2 q_b) with the hardware
// log2 (v_log_f32) applied to both operands, so the target's own row gives
// exactly 0; the ln 2 factor is applied once per row in FP64.  Four FP32
// terms are summed in FP32, then carried in FP64.
//
// KIND 7 computes the TV and the KL field of one target in one pass (the
// same terms and sums as KINDs 0 and 1, so the same values): a caller that
// wants both reads the rows once.
//
// chi-squared keeps 1/p_b in LDS (+inf where p_b = 0, so a row with mass
// outside the target's support gets +inf) and forms (q - p) * ((q - p) / p).
// Hellinger is evaluated as ((q - p) / (sqrt q + sqrt p))^2, which equals
// (sqrt q - sqrt p)^2 but has no cancellation: every term carries a small
// relative error, so the field has a relative error bound, also next to the
// target.  sqrt p sits in LDS beside p.
#include <algorithm>

#include "dd_internal.h"

namespace dd {

__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }

typedef float vf4 __attribute__((ext_vector_type(4)));

// 16-byte streaming load (non-temporal: the rows are read once per field).
__device__ __forceinline__ float4 ld_stream(const float4* p) {
  const vf4 v = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ float kl_term(float p, float lp, float q) {
  return p > 0.f ? p * (lp - hw_log2(q)) : 0.f;
}

// (q - p)^2 / p with r = 1/p (+inf for p = 0); 0 whenever q == p.
__device__ __forceinline__ float chi2_term(float p, float r, float q) {
  const float d = q - p;
  return d != 0.f ? d * (d * r) : 0.f;
}

// (sqrt q - sqrt p)^2 as ((q - p) / (sqrt q + sqrt p))^2 with the hardware
// square root and reciprocal (1 ulp each); 0 whenever q == p.
__device__ __forceinline__ float hel_term(float p, float sp, float q) {
  const float d = q - p;
  const float e = d * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(q) + sp);
  return d != 0.f ? e * e : 0.f;
}

// f(u) = |1 - u|^k, integer k >= 1: |q - p|^k / p^(k-1) as |d| (|d| / p)^(k-1)
// with r = 1/p (+inf for p = 0); 0 whenever q == p.
__device__ __forceinline__ float power_term(float p, float r, float q, int k) {
  const float d = fabsf(q - p);
  const float x = d * r;
  float t = d;
  for (int j = 1; j < k; ++j) t *= x;
  return d != 0.f ? t : 0.f;
}

// alpha-divergence with (1 + alpha)/2 = j/16: p (1 - (q/p)^(j/16)), the
// sixteenth root by four hardware square roots and the power by squaring;
// 0 when q == p (q * fl(1/p) need not be 1 there).  The factor
// 4/(1 - alpha^2) is applied per row.
__device__ __forceinline__ float alpha_term(float p, float r, float q, int j) {
  float z = q * r;
  z = __builtin_amdgcn_sqrtf(__builtin_amdgcn_sqrtf(__builtin_amdgcn_sqrtf(__builtin_amdgcn_sqrtf(z))));
  float pw = 1.f;
  for (int e = j; e; e >>= 1) {
    if (e & 1) pw *= z;
    z *= z;
  }
  return (p > 0.f && q != p) ? p * (1.f - pw) : 0.f;
}

// Second LDS array per kind: log2 p (KL), 1/p (chi-squared, power, alpha),
// sqrt p (Hellinger).
template <int KIND>
__device__ __forceinline__ float stage_aux(float p) {
  if (KIND == 1 || KIND == 7) return p > 0.f ? hw_log2(p) : 0.f;
  if (KIND == 2 || KIND == 4) return p > 0.f ? 1.0f / p : __builtin_inff();
  if (KIND == 5) return p > 0.f ? 1.0f / p : 0.f;
  return sqrtf(p);
}

template <int KIND>
__device__ __forceinline__ float term4(const float4& p, const float4& a, const float4& q,
                                       int param) {
  if (KIND == 0)
    return (fabsf(p.x - q.x) + fabsf(p.y - q.y)) + (fabsf(p.z - q.z) + fabsf(p.w - q.w));
  if (KIND == 1)
    return (kl_term(p.x, a.x, q.x) + kl_term(p.y, a.y, q.y)) +
           (kl_term(p.z, a.z, q.z) + kl_term(p.w, a.w, q.w));
  if (KIND == 2)
    return (chi2_term(p.x, a.x, q.x) + chi2_term(p.y, a.y, q.y)) +
           (chi2_term(p.z, a.z, q.z) + chi2_term(p.w, a.w, q.w));
  if (KIND == 4)
    return (power_term(p.x, a.x, q.x, param) + power_term(p.y, a.y, q.y, param)) +
           (power_term(p.z, a.z, q.z, param) + power_term(p.w, a.w, q.w, param));
  if (KIND == 5)
    return (alpha_term(p.x, a.x, q.x, param) + alpha_term(p.y, a.y, q.y, param)) +
           (alpha_term(p.z, a.z, q.z, param) + alpha_term(p.w, a.w, q.w, param));
  return (hel_term(p.x, a.x, q.x) + hel_term(p.y, a.y, q.y)) +
         (hel_term(p.z, a.z, q.z) + hel_term(p.w, a.w, q.w));
}

// Per-row factor of the FP64 sum: ln 2 for KL (log2 terms), 4/(1 - alpha^2)
// for the alpha-divergence, 1 otherwise.
template <int KIND>
__device__ __forceinline__ double row_factor(int param) {
  if (KIND == 1) return 0.69314718055994530942;
  if (KIND == 5) {
    const double al = (double)(param - 8) / 8.0;
    return 4.0 / (1.0 - al * al);
  }
  return 1.0;
}

template <int LPR, int KIND, int UNROLL>
__global__ __launch_bounds__(512) void dense_field_kernel(const float* __restrict__ P, int64_t ld,
                                                          int32_t N, int32_t target, int param,
                                                          float* __restrict__ out,
                                                          float* __restrict__ out2) {
  extern __shared__ float4 smem4[];
  const int nv = (int)(ld >> 2);
  float4* sp = smem4;
  float4* sl = smem4 + nv;
  const float4* trow = reinterpret_cast<const float4*>(P + (int64_t)target * ld);
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
    float4 p = trow[i];
    sp[i] = p;
    if (KIND != 0)
      sl[i] = make_float4(stage_aux<KIND>(p.x), stage_aux<KIND>(p.y), stage_aux<KIND>(p.z),
                          stage_aux<KIND>(p.w));
  }
  __syncthreads();

  const int lane = threadIdx.x & (LPR - 1);
  const int grp = threadIdx.x / LPR;
  const int gpb = blockDim.x / LPR;
  for (int64_t row = (int64_t)blockIdx.x * gpb + grp; row < N; row += (int64_t)gridDim.x * gpb) {
    const float4* q = reinterpret_cast<const float4*>(P + row * ld);
    double acc = 0.0, acc2 = 0.0;
    auto terms = [&](int i, const float4& qv) {
      const float4 p = sp[i];
      const float4 aux = KIND != 0 ? sl[i] : p;
      if (KIND == 7) {
        acc += (double)term4<0>(p, p, qv, param);
        acc2 += (double)term4<1>(p, aux, qv, param);
      } else {
        acc += (double)term4<KIND>(p, aux, qv, param);
      }
    };
    for (int base = lane; base < nv; base += LPR * UNROLL) {
      float4 v[UNROLL];
      if (__all(base + (UNROLL - 1) * LPR < nv)) {
        // every load of every lane inside its row: no masks
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) v[u] = ld_stream(q + base + u * LPR);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) terms(base + u * LPR, v[u]);
      } else {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const int i = base + u * LPR;
          v[u] = i < nv ? ld_stream(q + i) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const int i = base + u * LPR;
          if (i < nv) terms(i, v[u]);
        }
      }
    }
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) {
      acc += __shfl_xor(acc, off, LPR);
      if (KIND == 7) acc2 += __shfl_xor(acc2, off, LPR);
    }
    if (lane == 0) {
      out[row] = (float)(KIND == 1 || KIND == 5 ? acc * row_factor<KIND>(param) : acc);
      if (KIND == 7) out2[row] = (float)(acc2 * row_factor<1>(0));
    }
  }
}

// ---------------------------------------------------------------------------
// KL over the truncated support of the target row (the sparse KL of Section V,
// "Precision", with the rows of x kept exact):
//   d(x) = sum_{b in S_t} p_b log(p_b / q_b),  S_t = {b : p_b > 0, p_b >= thr},
// thr = tau * max_b p_b (row-relative) or tau.  The truncated target row and
// its log2 sit in LDS; a lane skips the 16-byte load of a row piece whose four
// target entries are all outside S_t, so the pass reads only the pieces of
// each row that meet the support (clustered along the boundary for the
// harmonic measure).  The support is decided on the FP64 master row when the
// handle has one, so it is the set the FP64 definition gives.
template <int LPR, int UNROLL>
__global__ __launch_bounds__(512) void support_kl_kernel(const float* __restrict__ P,
                                                         const double* __restrict__ P64,
                                                         int64_t ld, int32_t B, int32_t N,
                                                         int32_t target, double tau,
                                                         int tau_relative,
                                                         float* __restrict__ out) {
  extern __shared__ float4 smem4[];
  __shared__ double redm[8];
  const int nv = (int)(ld >> 2);
  float4* sp = smem4;
  float4* sl = smem4 + nv;
  const float* trow = P + (int64_t)target * ld;
  const double* trow64 = P64 ? P64 + (int64_t)target * B : nullptr;
  double thr = tau;
  if (tau_relative) {
    double m = 0.0;
    for (int b = threadIdx.x; b < B; b += blockDim.x)
      m = fmax(m, trow64 ? trow64[b] : (double)trow[b]);
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) redm[threadIdx.x >> 6] = m;
    __syncthreads();
    m = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) m = fmax(m, redm[i]);
    thr = tau * m;
  }
  float* spf = reinterpret_cast<float*>(sp);
  float* slf = reinterpret_cast<float*>(sl);
  for (int b = threadIdx.x; b < 4 * nv; b += blockDim.x) {
    float pv = b < B ? trow[b] : 0.f;
    const double pd = b < B ? (trow64 ? trow64[b] : (double)pv) : 0.0;
    if (!(pd > 0.0 && pd >= thr)) pv = 0.f;
    spf[b] = pv;
    slf[b] = pv > 0.f ? hw_log2(pv) : 0.f;
  }
  __syncthreads();

  const int lane = threadIdx.x & (LPR - 1);
  const int grp = threadIdx.x / LPR;
  const int gpb = blockDim.x / LPR;
  for (int64_t row = (int64_t)blockIdx.x * gpb + grp; row < N; row += (int64_t)gridDim.x * gpb) {
    const float4* q = reinterpret_cast<const float4*>(P + row * ld);
    double acc = 0.0;
    for (int base = lane; base < nv; base += LPR * UNROLL) {
      vf4 v[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const int i = base + u * LPR;
        const float4 pp = i < nv ? sp[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        const bool need = (pp.x + pp.y) + (pp.z + pp.w) > 0.f;
        v[u] = need ? __builtin_nontemporal_load(reinterpret_cast<const vf4*>(q + i))
                    : vf4{1.f, 1.f, 1.f, 1.f};
      }
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const int i = base + u * LPR;
        if (i < nv) {
          const float4 qv = make_float4(v[u].x, v[u].y, v[u].z, v[u].w);
          acc += (double)term4<1>(sp[i], sl[i], qv, 0);
        }
      }
    }
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LPR);
    if (lane == 0) out[row] = (float)(acc * 0.69314718055994530942);
  }
}

// ---------------------------------------------------------------------------
// Truncated (CSR) rows.  The truncated target row p~ is scattered into LDS as
// a dense vector of (p~, log2 p~) pairs (zeros where dropped).  For row x with
// stored support S_x:
//   TV_tau(x) = sum_{b in S_x} |q_b - p~_b| + sum_{b in S_t \ S_x} p~_b
//   KL_tau(x) = sum_{b in S_x} p~_b (log p~_b - log q_b)
//             + sum_{b in S_t \ S_x} p~_b (log p~_b - log phi_x)
// The S_t \ S_x sums are W_t - A_x and (Hb_t - E_x) - log2 phi_x (W_t - A_x),
// with A_x, E_x the sums of p~_b and p~_b log2 p~_b over S_x, all in FP64;
// when S_x covers S_t they are FP64 round-off (far inside the stated bound),
// and the target's own row is set to exactly 0.  Stored values are positive,
// so the KL terms need no zero guard.  With F16, the values come from the
// FP16 form (4 per 8 bytes), times the row's 2^-e_x.
__device__ __forceinline__ float f16_value(uint16_t h, float rs) {
  return (float)__builtin_bit_cast(_Float16, h) * rs;
}

template <int LPR, int KIND, int UNROLL, int F16>
__global__ __launch_bounds__(512) void csr_field_kernel(CsrView v, int32_t target,
                                                        float* __restrict__ out,
                                                        float* __restrict__ out2) {
  // LDS: the truncated target row as (p, log2 p) pairs, zeros where dropped
  extern __shared__ float2 smem2[];
  const int Bp = (v.B + 3) & ~3;
  float2* spl = smem2;
  __shared__ double red[2][8];
  for (int i = threadIdx.x; i < Bp; i += blockDim.x) spl[i] = make_float2(0.f, 0.f);
  __syncthreads();
  const int64_t ts = v.start[target];
  const int tl = v.len[target];
  const float trs = F16 ? v.rscale[target] : 1.f;
  double w = 0.0, hb = 0.0;
  for (int i = threadIdx.x; i < tl; i += blockDim.x) {
    const int b = v.col[ts + i];
    const float p = F16 ? f16_value(v.val16[ts + i], trs) : v.val[ts + i];
    const float l = hw_log2(p);
    spl[b] = make_float2(p, l);
    w += (double)p;
    hb += (double)(p * l);
  }
  for (int off = 32; off > 0; off >>= 1) {
    w += __shfl_xor(w, off);
    hb += __shfl_xor(hb, off);
  }
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wid] = w;
    red[1][wid] = hb;
  }
  __syncthreads();
  double Wt = 0.0, Hbt = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
    Wt += red[0][i];
    Hbt += red[1][i];
  }

  const int lane = threadIdx.x & (LPR - 1);
  const int grp = threadIdx.x / LPR;
  const int gpb = blockDim.x / LPR;
  for (int64_t row = (int64_t)blockIdx.x * gpb + grp; row < v.N; row += (int64_t)gridDim.x * gpb) {
    const int64_t s = v.start[row];
    const int n = v.len[row];
    const float4* val4 = reinterpret_cast<const float4*>(v.val + s);
    const ushort4* h4 = reinterpret_cast<const ushort4*>((F16 ? v.val16 : v.col) + s);
    const float rs = F16 ? v.rscale[row] : 1.f;
    const ushort4* col4 = reinterpret_cast<const ushort4*>(v.col + s);
    const int nv = (n + 3) >> 2;
    double acc = 0.0, acc2 = 0.0, A = 0.0, E = 0.0;
    // Loads are unconditional (index clamped into the row) and entries past
    // the row's end are masked arithmetically, so the loop has no divergent
    // branch that would make the loads wait.  Padding slots hold column 0.
    // Every load of an iteration is issued before any of its values is used
    // (the FP16 values are converted in the compute loop), and a group of
    // four entries wholly inside the row for every lane of the wave (all but
    // a row's last iteration) skips the masking.
    for (int base = lane; base < nv; base += LPR * UNROLL) {
      float4 q[UNROLL];
      ushort4 hq[UNROLL];
      ushort4 cb[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const int i = min(base + u * LPR, nv - 1);
        if (F16)
          hq[u] = h4[i];
        else
          q[u] = ld_stream(val4 + i);
        cb[u] = col4[i];
      }
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const int i = base + u * LPR;
        const int rem = i < nv ? n - 4 * i : 0;
        if (F16)
          q[u] = make_float4(f16_value(hq[u].x, rs), f16_value(hq[u].y, rs),
                             f16_value(hq[u].z, rs), f16_value(hq[u].w, rs));
        const float qv[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
        const int bv[4] = {cb[u].x, cb[u].y, cb[u].z, cb[u].w};
        float ts4 = 0.f, ks4 = 0.f, as4 = 0.f, es4 = 0.f;
        if (__all(rem >= 4)) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float2 pl = spl[bv[e]];
            as4 += pl.x;
            if (KIND != 1) ts4 += fabsf(qv[e] - pl.x);
            if (KIND != 0) {
              ks4 += pl.x * (pl.y - hw_log2(qv[e]));
              es4 += pl.x * pl.y;
            }
          }
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const bool ok = e < rem;
            const float2 pl = spl[bv[e]];
            const float p = ok ? pl.x : 0.f;
            as4 += p;
            if (KIND != 1) ts4 += fabsf((ok ? qv[e] : 0.f) - p);
            if (KIND != 0) {
              ks4 += p * (pl.y - hw_log2(ok ? qv[e] : 1.f));
              es4 += p * pl.y;
            }
          }
        }
        if (KIND != 1) acc += (double)ts4;
        if (KIND != 0) acc2 += (double)ks4;
        A += (double)as4;
        if (KIND != 0) E += (double)es4;
      }
    }
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) {
      if (KIND != 1) acc += __shfl_xor(acc, off, LPR);
      if (KIND != 0) {
        acc2 += __shfl_xor(acc2, off, LPR);
        E += __shfl_xor(E, off, LPR);
      }
      A += __shfl_xor(A, off, LPR);
    }
    if (lane == 0) {
      // KIND 0: TV into out; 1: KL into out; 2: TV into out and KL into out2
      const double tv = acc + (Wt - A);
      const double kl = (acc2 + (Hbt - E) - v.lphi[row] * (Wt - A)) * 0.69314718055994530942;
      if (KIND != 1) out[row] = row == target ? 0.f : (float)tv;
      if (KIND == 1) out[row] = row == target ? 0.f : (float)kl;
      if (KIND == 2) out2[row] = row == target ? 0.f : (float)kl;
    }
  }
}

int num_cus() {
  static int n = 0;
  if (n == 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (n <= 0) n = 256;
  }
  return n;
}

template <typename K>
static hipError_t allow_lds(K kern, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Large staged target rows limit the workgroups per CU (160 KB of LDS), so
// those launches use 512-thread workgroups: twice the waves share one copy.
static int block_threads(size_t lds) { return lds > 32 * 1024 ? 512 : 256; }

// Persistent grid: as many workgroups as the LDS allows, keeping four wave
// slots of each CU (of 32) free for concurrent work on other streams, such
// as a path walk beside a field: a workgroup that cannot start until another
// finishes would end the pass late.
static int grid_for(int64_t groups_needed, int gpb, int threads, size_t lds) {
  const int64_t need = (groups_needed + gpb - 1) / gpb;
  int per_cu = lds > 0 ? (int)((160 * 1024) / (lds + 1024)) : 8;
  per_cu = std::min(per_cu, (32 - 4) / (threads / 64));
  per_cu = std::max(1, std::min(per_cu, 8));
  const int64_t cap = (int64_t)num_cus() * per_cu;
  return (int)(need < cap ? (need > 0 ? need : 1) : cap);
}

template <int LPR, int KIND>
static hipError_t dense_launch(DenseView v, int32_t target, int param, float* out, hipStream_t s,
                               float* out2 = nullptr) {
  // TV and KL (apart or together): six 16-byte loads per lane in flight (a
  // 257^2 row in one round trip); the other kinds carry more per-entry state
  constexpr int UNROLL = KIND <= 1 || KIND == 7 ? 6 : 4;
  auto kern = dense_field_kernel<LPR, KIND, UNROLL>;
  const size_t lds = (size_t)v.ld * sizeof(float) * (KIND != 0 ? 2 : 1);
  hipError_t e = allow_lds(kern, lds);
  if (e != hipSuccess) return e;
  const int threads = block_threads(lds);
  const int grid = grid_for(v.N, threads / LPR, threads, lds);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, s, v.P, v.ld, v.N, target, param, out,
                     out2);
  return hipGetLastError();
}

template <int KIND>
static hipError_t dense_dispatch(DenseView v, int32_t target, int param, float* out,
                                 hipStream_t s, float* out2 = nullptr) {
  const int64_t nv = v.ld / 4;
  if (nv >= 256) return dense_launch<64, KIND>(v, target, param, out, s, out2);
  if (nv >= 128) return dense_launch<32, KIND>(v, target, param, out, s, out2);
  return dense_launch<16, KIND>(v, target, param, out, s, out2);
}

// kind: 0 TV, 1 KL, 2 chi-squared, 3 Hellinger, 100 + k power k (1..16),
// 200 + j alpha-divergence with (1 + alpha)/2 = j/16 (1..15)
hipError_t launch_dense_field(DenseView v, int32_t target, int kind, float* out, hipStream_t s) {
  if (kind > 100 && kind <= 116) return dense_dispatch<4>(v, target, kind - 100, out, s);
  if (kind > 200 && kind < 216) return dense_dispatch<5>(v, target, kind - 200, out, s);
  switch (kind) {
    case 0: return dense_dispatch<0>(v, target, 0, out, s);
    case 1: return dense_dispatch<1>(v, target, 0, out, s);
    case 2: return dense_dispatch<2>(v, target, 0, out, s);
    case 3: return dense_dispatch<3>(v, target, 0, out, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_dense_tv_kl(DenseView v, int32_t target, float* tv, float* kl, hipStream_t s) {
  return dense_dispatch<7>(v, target, 0, tv, s, kl);
}

template <int LPR>
static hipError_t support_launch(DenseView v, int32_t target, double tau, int tau_relative,
                                 float* out, hipStream_t s) {
  auto kern = support_kl_kernel<LPR, 4>;
  const size_t lds = (size_t)v.ld * sizeof(float) * 2;
  hipError_t e = allow_lds(kern, lds);
  if (e != hipSuccess) return e;
  const int threads = block_threads(lds);
  const int grid = grid_for(v.N, threads / LPR, threads, lds);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, s, v.P, v.P64, v.ld, v.B, v.N, target,
                     tau, tau_relative, out);
  return hipGetLastError();
}

hipError_t launch_support_kl_field(DenseView v, int32_t target, double tau, int tau_relative,
                                   float* out, hipStream_t s) {
  const int64_t nv = v.ld / 4;
  if (nv >= 256) return support_launch<64>(v, target, tau, tau_relative, out, s);
  if (nv >= 128) return support_launch<32>(v, target, tau, tau_relative, out, s);
  return support_launch<16>(v, target, tau, tau_relative, out, s);
}

template <int LPR, int KIND, int F16>
static hipError_t csr_launch(CsrView v, int32_t target, float* out, hipStream_t s,
                             float* out2 = nullptr) {
  auto kern = csr_field_kernel<LPR, KIND, 2, F16>;
  const size_t lds = (size_t)((v.B + 3) & ~3) * sizeof(float) * 2;
  hipError_t e = allow_lds(kern, lds);
  if (e != hipSuccess) return e;
  const int threads = block_threads(lds);
  const int grid = grid_for(v.N, threads / LPR, threads, lds);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, s, v, target, out, out2);
  return hipGetLastError();
}

hipError_t launch_csr_field(CsrView v, int32_t target, int kind, float* out, hipStream_t s) {
  // lanes per row from the mean stored row length
  if (v.val16) {
    if (kind == 0) return csr_launch<64, 0, 1>(v, target, out, s);
    return csr_launch<64, 1, 1>(v, target, out, s);
  }
  if (kind == 0) return csr_launch<64, 0, 0>(v, target, out, s);
  return csr_launch<64, 1, 0>(v, target, out, s);
}

hipError_t launch_csr_tv_kl(CsrView v, int32_t target, float* tv, float* kl, hipStream_t s) {
  if (v.val16) return csr_launch<64, 2, 1>(v, target, tv, s, kl);
  return csr_launch<64, 2, 0>(v, target, tv, s, kl);
}

}  // namespace dd
