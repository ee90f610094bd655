// Load-time conversion of a Poisson-kernel matrix into its resident forms:
// row checks and statistics, all-zero column detection, column compaction
// into padded FP32 rows (plus an FP64 master), per-row entropy, CSR
// truncation, and the log-kernel operand of the batched KL contraction.
#include <float.h>

#include "dd_internal.h"

namespace dd {

template <typename T>
__device__ __forceinline__ double ld_raw(const void* raw, int64_t i) {
  return (double)reinterpret_cast<const T*>(raw)[i];
}

__device__ __forceinline__ double raw_at(const void* raw, int is_f64, int64_t i) {
  return is_f64 ? ld_raw<double>(raw, i) : ld_raw<float>(raw, i);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// One wave per row: FP64 row sum and max; a row is bad if an entry is not
// finite, negative, or positive but below the FP32 normal range.
__global__ __launch_bounds__(256) void row_stats_kernel(const void* raw, int is_f64, int32_t N,
                                                        int32_t B, double* row_sum,
                                                        double* row_max, int32_t* bad_rows) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= N) return;
  double s = 0.0, m = 0.0;
  int bad = 0;
  for (int b = lane; b < B; b += 64) {
    const double v = raw_at(raw, is_f64, row * B + b);
    if (!(v >= 0.0) || !(v <= DBL_MAX) || (v > 0.0 && v < (double)FLT_MIN)) bad = 1;
    s += v;
    m = fmax(m, v);
  }
  s = wave_sum(s);
  m = wave_max(m);
  const unsigned long long any_bad = __ballot(bad);
  if (lane == 0) {
    row_sum[row] = s;
    row_max[row] = m;
    if (any_bad) atomicAdd(bad_rows, 1);
  }
}

__global__ __launch_bounds__(256) void col_nonzero_kernel(const void* raw, int is_f64, int32_t N,
                                                          int32_t B, int32_t* flags) {
  const int64_t rows_per_block = (N + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min((int64_t)N, r0 + rows_per_block);
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    int nz = 0;
    for (int64_t r = r0; r < r1 && !nz; ++r) nz = raw_at(raw, is_f64, r * B + b) != 0.0;
    if (nz) atomicOr(flags + b, 1);
  }
}

__global__ __launch_bounds__(256) void gather_cols_kernel(const void* raw, int is_f64, int32_t N,
                                                          int32_t B, const int32_t* kept,
                                                          int32_t Bk, int64_t ld, float* out32,
                                                          double* out64) {
  const int64_t total = (int64_t)N * ld;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / ld;
    const int j = (int)(i - r * ld);
    double v = 0.0;
    if (j < Bk) v = raw_at(raw, is_f64, r * B + kept[j]);
    out32[i] = (float)v;
    if (out64 && j < Bk) out64[r * Bk + j] = v;
  }
}

__device__ __forceinline__ double master_at(const DenseView& v, int64_t row, int b) {
  return v.P64 ? v.P64[row * v.B + b] : (double)v.P[row * v.ld + b];
}

// H[x] = sum_b P_xb log P_xb in FP64 from the master values.
__global__ __launch_bounds__(256) void row_entropy_kernel(DenseView v, double* H) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= v.N) return;
  double s = 0.0;
  for (int b = lane; b < v.B; b += 64) {
    const double p = master_at(v, row, b);
    if (p > 0.0) s += p * log(p);
  }
  s = wave_sum(s);
  if (lane == 0) H[row] = s;
}

__global__ __launch_bounds__(256) void trunc_count_kernel(DenseView v, const double* thr,
                                                          int32_t* counts) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= v.N) return;
  const double t = thr[row];
  int c = 0;
  for (int b = lane; b < v.B; b += 64) {
    const double p = master_at(v, row, b);
    c += (p > 0.0 && p >= t);
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if (lane == 0) counts[row] = c;
}

// Ballot compaction keeps the kept entries of each row in column order.
__global__ __launch_bounds__(256) void trunc_fill_kernel(DenseView v, const double* thr,
                                                         const int64_t* start, uint16_t* col,
                                                         float* val, double* val64) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= v.N) return;
  const double t = thr[row];
  int64_t pos = start[row];
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int b0 = 0; b0 < v.B; b0 += 64) {
    const int b = b0 + lane;
    double p = 0.0;
    if (b < v.B) p = master_at(v, row, b);
    const int keep = (b < v.B) && p > 0.0 && p >= t;
    const unsigned long long m = __ballot(keep);
    if (keep) {
      const int64_t o = pos + __popcll(m & below);
      col[o] = (uint16_t)b;
      val[o] = (float)p;
      if (val64) val64[o] = p;
    }
    pos += __popcll(m);
  }
}

// l_xb = log P_xb - o_x with o_x = log max_b P_xb (natural log, FP64 then
// rounded): FP32, an FP16 (form 1) or BF16 (form 2) hi + lo split, or the FP16
// hi part alone (form 3), written
// in the tiled layout
// of the contraction operand (padding rows are zeroed by the caller).
__global__ __launch_bounds__(256) void log_forms_kernel(DenseView v, int form, int64_t lda,
                                                        float* l32, uint16_t* lhi, uint16_t* llo,
                                                        float* offset, int32_t* zeros,
                                                        const double* floor) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= v.N) return;
  double m = 0.0;
  for (int b = lane; b < v.B; b += 64) m = fmax(m, master_at(v, row, b));
  m = wave_max(m);
  const double o = log(m);
  if (lane == 0) offset[row] = (float)o;
  const double of = (double)(float)o;   // the offset the epilogue will use
  int nz = 0;
  const int64_t R = gemm_row_tiles(v.N);
  const int64_t tile_base = (row / kGemmRows) * kGemmRows * kGemmK;
  const int xr = (int)(row % kGemmRows);
  const double fl = floor ? floor[row] : 0.0;   // > 0 when given
  for (int64_t b = lane; b < lda; b += 64) {
    const int64_t at = tile_base + (b / kGemmK) * R * kGemmRows * kGemmK +
                       gemm_tile_offset(form == 0, xr, (int)(b % kGemmK));
    double l = 0.0;
    if (b < v.B) {
      const double p = fmax(master_at(v, row, (int)b), fl);
      if (p > 0.0)
        l = log(p) - of;
      else
        nz = 1;   // log 0: this row cannot enter the contraction
    }
    if (form == 0) {
      l32[at] = (float)l;
    } else if (form == 2) {
      const __bf16 hi = (__bf16)(float)l;
      const __bf16 lo = (__bf16)(float)(l - (double)(float)hi);
      lhi[at] = __builtin_bit_cast(uint16_t, hi);
      llo[at] = __builtin_bit_cast(uint16_t, lo);
    } else {
      const _Float16 hi = (_Float16)l;
      const _Float16 lo = (_Float16)(l - (double)hi);
      lhi[at] = __builtin_bit_cast(uint16_t, hi);
      if (form == 1) llo[at] = __builtin_bit_cast(uint16_t, lo);
    }
  }
  if (__ballot(nz) != 0ull && lane == 0) atomicAdd(zeros, 1);
}

// One wave per row: val16 = FP16(val * 2^e_x), round to nearest even; the
// scaling is exact (a power of two, no overflow: the row max lands in
// [2^14, 2^15)).
__global__ __launch_bounds__(256) void csr_f16_kernel(const int64_t* start, const int32_t* len,
                                                      const float* val, const float* rscale,
                                                      int32_t N, uint16_t* val16) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= N) return;
  const int64_t s = start[row];
  const int n = len[row];
  const float sc = 1.0f / rscale[row];
  for (int i = lane; i < n; i += 64) {
    const _Float16 h = (_Float16)(val[s + i] * sc);
    val16[s + i] = __builtin_bit_cast(uint16_t, h);
  }
}

static int rows_grid(int64_t N) { return (int)((N + 3) / 4); }

hipError_t launch_row_stats(const void* raw, int is_f64, int32_t N, int32_t B, double* row_sum,
                            double* row_max, int32_t* bad_rows, hipStream_t s) {
  hipLaunchKernelGGL(row_stats_kernel, dim3(rows_grid(N)), dim3(256), 0, s, raw, is_f64, N, B,
                     row_sum, row_max, bad_rows);
  return hipGetLastError();
}

hipError_t launch_col_nonzero(const void* raw, int is_f64, int32_t N, int32_t B, int32_t* flags,
                              hipStream_t s) {
  int grid = num_cus() * 4;
  if (grid > N) grid = N > 0 ? N : 1;
  hipLaunchKernelGGL(col_nonzero_kernel, dim3(grid), dim3(256), 0, s, raw, is_f64, N, B, flags);
  return hipGetLastError();
}

hipError_t launch_gather_cols(const void* raw, int is_f64, int32_t N, int32_t B,
                              const int32_t* kept, int32_t Bk, int64_t ld, float* out32,
                              double* out64, hipStream_t s) {
  hipLaunchKernelGGL(gather_cols_kernel, dim3(num_cus() * 8), dim3(256), 0, s, raw, is_f64, N, B,
                     kept, Bk, ld, out32, out64);
  return hipGetLastError();
}

hipError_t launch_row_entropy(DenseView v, double* H, hipStream_t s) {
  hipLaunchKernelGGL(row_entropy_kernel, dim3(rows_grid(v.N)), dim3(256), 0, s, v, H);
  return hipGetLastError();
}

hipError_t launch_trunc_count(DenseView v, const double* thr, int32_t* counts, hipStream_t s) {
  hipLaunchKernelGGL(trunc_count_kernel, dim3(rows_grid(v.N)), dim3(256), 0, s, v, thr, counts);
  return hipGetLastError();
}

hipError_t launch_trunc_fill(DenseView v, const double* thr, const int64_t* start, uint16_t* col,
                             float* val, double* val64, hipStream_t s) {
  hipLaunchKernelGGL(trunc_fill_kernel, dim3(rows_grid(v.N)), dim3(256), 0, s, v, thr, start, col,
                     val, val64);
  return hipGetLastError();
}

hipError_t launch_csr_f16(const int64_t* start, const int32_t* len, const float* val,
                          const float* rscale, int32_t N, uint16_t* val16, hipStream_t s) {
  hipLaunchKernelGGL(csr_f16_kernel, dim3(rows_grid(N)), dim3(256), 0, s, start, len, val, rscale,
                     N, val16);
  return hipGetLastError();
}

hipError_t launch_log_forms(DenseView v, int form, int64_t lda, float* l32, uint16_t* lhi,
                            uint16_t* llo, float* offset, int32_t* zeros, const double* floor,
                            hipStream_t s) {
  hipLaunchKernelGGL(log_forms_kernel, dim3(rows_grid(v.N)), dim3(256), 0, s, v, form, lda, l32,
                     lhi, llo, offset, zeros, floor);
  return hipGetLastError();
}

// Row j of the dense target block: the truncated row of target tl.t[j] (its
// stored values, zero elsewhere) in FP32 [rows][ld] and, from the FP64
// values when the handle has them, FP64 [rows][B]; rows past T are zero.
// The contraction's target preparation reads rows j < T only.
__global__ __launch_bounds__(256) void csr_rows_dense_kernel(CsrView v, TargetList tl, int32_t T,
                                                             int64_t ld, float* out32,
                                                             double* out64) {
  const int j = blockIdx.x;
  float* o32 = out32 + (int64_t)j * ld;
  double* o64 = out64 ? out64 + (int64_t)j * v.B : nullptr;
  for (int64_t b = threadIdx.x; b < ld; b += blockDim.x) {
    o32[b] = 0.f;
    if (o64 && b < v.B) o64[b] = 0.0;
  }
  __syncthreads();
  if (j >= T) return;
  const int t = tl.t[j];
  const int64_t st = v.start[t];
  for (int i = threadIdx.x; i < v.len[t]; i += blockDim.x) {
    const int b = v.col[st + i];
    o32[b] = v.val[st + i];
    if (o64) o64[b] = v.val64[st + i];
  }
}

hipError_t launch_csr_rows_dense(CsrView v, TargetList tl, int32_t T, int32_t Tpad, int64_t ld,
                                 float* out32, double* out64, hipStream_t s) {
  hipLaunchKernelGGL(csr_rows_dense_kernel, dim3(Tpad), dim3(256), 0, s, v, tl, T, ld, out32,
                     out64);
  return hipGetLastError();
}

}  // namespace dd
