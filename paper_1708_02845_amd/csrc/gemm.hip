// Batched KL as one contraction (Section IV, eq. 35 expanded):
//
//   d(x, t) = sum_b p_tb log(p_tb / P_xb) = H_t - o_x W_t - S_xt,
//   S_xt    = sum_b l_xb p_tb,   l_xb = log P_xb - o_x,   o_x = log max_b P_xb,
//   H_t     = sum_b p_tb log p_tb,   W_t = sum_b p_tb,
//
// with S = l * P_T^T an (N x B) by (B x T) product on MFMA.  The log-kernel l
// (built once at load) is the A operand; the target rows are the B operand,
// staged per K-chunk in LDS and shared by the four waves of a workgroup.  A
// workgroup owns 128 rows and one group of up to 64 targets; each wave owns
// 32 rows and all columns of the group (32 per column tile).
//
// Up to 256 targets run in one launch as groups of 64.  The workgroups of
// one row block (one per group) are given consecutive positions in the
// dispatch order of one XCD: work-groups are handed to the eight XCDs round
// robin, so block b runs on XCD b mod 8, and the decode below places row block
// rb's groups at consecutive b with the same b mod 8.  They start together and
// read the same A chunks at about the same time, so the A operand comes from
// HBM about once and from that XCD's L2 for the other groups.
//
// Forms:
//   F32    l and p in FP32, v_mfma_f32_32x32x2_f32.
//   F16X3  l = l_hi + l_lo and p*s_t = q_hi + q_lo in FP16 (s_t a power of two
//          putting max q at 2^13..2^14), three products l_hi q_hi + l_hi q_lo
//          + l_lo q_hi on v_mfma_f32_32x32x16_f16, divided by s_t at the end.
//   BF16X3 the same split in BF16 (no scale: BF16 has the FP32 range) on
//          v_mfma_f32_32x32x16_bf16; 8 + 8 significant bits per operand.
//   F16    the hi parts only: l_hi q_hi on v_mfma_f32_32x32x16_f16, half the
//          operand bytes of F16X3, 11 significant bits per operand.
//
// Both forms carry the FP32 accumulators into FP64 after every K-chunk of 64,
// so the FP32 accumulation error is that of 64-term partial sums; H_t, W_t and
// the final combination are FP64.
//
// The operand is stored in 128-row x 64-column blocks, chunk-major (see
// dd_internal.h), so a workgroup's K-chunk is one 16 KB (FP16) or 32 KB (FP32)
// block, a wave's loads cover 4-8 KB contiguously, and the workgroups running
// together read adjacent blocks.  The order
// of K inside a chunk is a free choice, as long as both operands use the same
// one: lane half h of a wave reads the contiguous K range [32h, 32h+32) of
// its row in the chunk.
#include <math.h>

#include "dd_internal.h"

namespace dd {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bhalf8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
// Register arrays use native vector types: arrays of HIP's struct vector
// types are not promoted to registers and end up in scratch memory.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int KC = kGemmK;       // K per chunk
constexpr int GW = 4;            // waves per workgroup
constexpr int GROWS = 32 * GW;   // rows per workgroup
static_assert(GROWS == kGemmRows, "a workgroup owns one row tile of the operand");

struct BatchOperand {
  float* b32;        // [Tpad][lda] FP32 targets (F32)
  uint16_t* bhi;     // [Tpad][lda] FP16 / BF16 bits (F16X3 / BF16X3)
  uint16_t* blo;
  double* H;         // [Tpad]
  double* W;         // [Tpad]
  double* inv_s;     // [Tpad] 1/s_t
};

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Target operands by form: FP32 (0), or hi + lo halves (1, 2; form 3 uses hi).
static BatchOperand carve(GemmView gv, int Tpad, void* ws) {
  unsigned char* p = static_cast<unsigned char*>(ws);
  BatchOperand o{};
  size_t off = 0;
  if (gv.form == 0) {
    o.b32 = reinterpret_cast<float*>(p + off);
    off = align256(off + 4 * (size_t)Tpad * gv.lda);
  } else {
    o.bhi = reinterpret_cast<uint16_t*>(p + off);
    off = align256(off + 2 * (size_t)Tpad * gv.lda);
    o.blo = reinterpret_cast<uint16_t*>(p + off);
    off = align256(off + 2 * (size_t)Tpad * gv.lda);
  }
  o.H = reinterpret_cast<double*>(p + off);
  o.W = o.H + Tpad;
  o.inv_s = o.W + Tpad;
  return o;
}

constexpr int kXcds = 8;   // MI355X: 8 XCDs, work-groups dispatched round robin

static int padded_targets(int32_t T) { return T <= 32 ? 32 : (T + 63) / 64 * 64; }

// Row block and target group of this workgroup (see the header comment).
__device__ __forceinline__ void block_tile(int groups, int& rb, int& g) {
  const int b = (int)blockIdx.x;
  const int j = b / kXcds;
  rb = (j / groups) * kXcds + b % kXcds;
  g = j % groups;
}

size_t batch_kl_workspace(GemmView gv, int32_t T) {
  const int Tpad = padded_targets(T);
  size_t off = gv.form == 0 ? align256(4 * (size_t)Tpad * gv.lda)
                            : 2 * align256(2 * (size_t)Tpad * gv.lda);
  return off + 3 * 8 * (size_t)Tpad;
}

// One block per padded target slot: FP64 H_t, W_t, the scale, and the B operand.
__global__ __launch_bounds__(256) void batch_target_prep(DenseView dv, GemmView gv, TargetList tl,
                                                         int32_t T, BatchOperand o) {
  const int j = blockIdx.x;
  const bool real = j < T;
  const int t = real ? tl.t[j] : 0;
  __shared__ double red[3][4];
  __shared__ double bcast[2];
  double w = 0.0, h = 0.0, m = 0.0;
  if (real) {
    for (int b = threadIdx.x; b < dv.B; b += blockDim.x) {
      const double p = dv.P64 ? dv.P64[(int64_t)t * dv.B + b] : (double)dv.P[(int64_t)t * dv.ld + b];
      w += p;
      if (p > 0.0) h += p * log(p);
      m = fmax(m, p);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    w += __shfl_xor(w, off);
    h += __shfl_xor(h, off);
    m = fmax(m, __shfl_xor(m, off));
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = w;
    red[1][threadIdx.x >> 6] = h;
    red[2][threadIdx.x >> 6] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double W = 0.0, H = 0.0, M = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      W += red[0][i];
      H += red[1][i];
      M = fmax(M, red[2][i]);
    }
    double s = 1.0;
    if ((gv.form == 1 || gv.form == 3) && M > 0.0) {
      int e = 0;
      frexp(M, &e);          // M in [2^(e-1), 2^e)
      s = ldexp(1.0, 14 - e);
    }
    o.H[j] = H;
    o.W[j] = W;
    o.inv_s[j] = 1.0 / s;
    bcast[0] = s;
  }
  __syncthreads();
  const float s = (float)bcast[0];
  for (int64_t k = threadIdx.x; k < gv.lda; k += blockDim.x) {
    float p = 0.f;
    if (real && k < dv.B)
      p = dv.P64 ? (float)dv.P64[(int64_t)t * dv.B + k] : dv.P[(int64_t)t * dv.ld + k];
    if (gv.form == 0) {
      o.b32[(int64_t)j * gv.lda + k] = p;
    } else if (gv.form == 2) {
      const __bf16 qh = (__bf16)p;
      const __bf16 ql = (__bf16)(p - (float)qh);
      o.bhi[(int64_t)j * gv.lda + k] = __builtin_bit_cast(uint16_t, qh);
      o.blo[(int64_t)j * gv.lda + k] = __builtin_bit_cast(uint16_t, ql);
    } else {
      const float q = p * s;                    // exact: s is a power of two
      const _Float16 qh = (_Float16)q;
      const _Float16 ql = (_Float16)(q - (float)qh);
      o.bhi[(int64_t)j * gv.lda + k] = __builtin_bit_cast(uint16_t, qh);
      if (gv.form == 1) o.blo[(int64_t)j * gv.lda + k] = __builtin_bit_cast(uint16_t, ql);
    }
  }
}

// Epilogue shared by both forms: d = H_t - o_x W_t - S_xt / s_t (FP64),
// rounded to FP32.  Each 32x32 column tile of a wave is transposed through
// LDS (stride 33 floats) so that one store instruction writes two full
// 128-byte row segments of two target fields.  `stage` is 4 x 32 x 33 floats.
template <int NT>
__device__ __forceinline__ void write_fields(const GemmView& gv, const BatchOperand& o, int32_t T,
                                             int tbase, int64_t row0, int lane,
                                             const double (&accd)[NT][16], float* stage,
                                             float* out) {
  const int r = lane & 31, h = lane >> 5;
  float* tile = stage + (threadIdx.x >> 6) * (32 * 33);
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const int t = tbase + n * 32 + r;
    const bool tv = t < T;
    const double H = tv ? o.H[t] : 0.0, W = tv ? o.W[t] : 0.0, is = tv ? o.inv_s[t] : 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int xl = 8 * (i >> 2) + 4 * h + (i & 3);
      const int64_t x = row0 + xl;
      float d = 0.f;
      if (tv && x < gv.N) d = (float)(H - (double)gv.offset[x] * W - accd[n][i] * is);
      tile[r * 33 + xl] = d;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int tl = 2 * q + h;
      const int tt = tbase + n * 32 + tl;
      const int64_t x = row0 + r;
      if (tt < T && x < gv.N) out[(int64_t)tt * gv.N + x] = tile[tl * 33 + r];
    }
    __syncthreads();
  }
}

// The three products of one K step of 16 (FP16 or BF16 operands).
template <bool BF>
__device__ __forceinline__ floatx16 split3(u32x4 ah, u32x4 al, u32x4 bh, u32x4 bl, floatx16 c) {
  if constexpr (BF) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bhalf8, ah),
                                                __builtin_bit_cast(bhalf8, bh), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bhalf8, ah),
                                                __builtin_bit_cast(bhalf8, bl), c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bhalf8, al),
                                                   __builtin_bit_cast(bhalf8, bh), c, 0, 0, 0);
  } else {
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, ah),
                                               __builtin_bit_cast(half8, bh), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, ah),
                                               __builtin_bit_cast(half8, bl), c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, al),
                                                  __builtin_bit_cast(half8, bh), c, 0, 0, 0);
  }
}

// HI: the F16 form, hi parts only (one product per K step; the lo loads and
// their registers drop out).  ST: the A operand is read with non-temporal
// loads, for launches of one target group, where no other workgroup reads the
// same A tile (with several groups the tile's co-running readers share it
// through L2, which non-temporal loads would give up).
template <int NT, bool BF, bool HI = false, bool ST = false>
__device__ __forceinline__ void gemm_split_body(GemmView gv, BatchOperand o, int32_t T,
                                                int32_t groups, float* __restrict__ out) {
  int rb, grp;
  block_tile(groups, rb, grp);
  if ((int64_t)rb * GROWS >= gv.N) return;   // padding of the grid to whole XCD rounds
  const int tbase = grp * 64;
  // target tiles (hi, lo) in one LDS buffer, reused by the epilogue as a
  // 4 x 32 x 33-float stage
  constexpr int TILE_BYTES = 2 * NT * 32 * (KC + 8) * 2;
  constexpr int STAGE_BYTES = 4 * 32 * 33 * 4;
  __shared__ __attribute__((aligned(16)))
      unsigned char lds[TILE_BYTES > STAGE_BYTES ? TILE_BYTES : STAGE_BYTES];
  _Float16 (*sbh)[KC + 8] = reinterpret_cast<_Float16 (*)[KC + 8]>(lds);
  _Float16 (*sbl)[KC + 8] = sbh + NT * 32;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
  const int64_t row0 = (int64_t)rb * GROWS + wv * 32;
  const int nchunks = (int)(gv.lda / KC);
  // tiled operand: this workgroup's chunk c is one contiguous block of
  // GROWS x KC, the blocks of one chunk index adjacent across row tiles;
  // rows past N are zero in memory
  const int64_t tile0 = (int64_t)rb * (GROWS * KC);
  const int64_t cstride = gemm_row_tiles(gv.N) * (GROWS * KC);
  const uint16_t* bhp = o.bhi + (int64_t)tbase * gv.lda;
  const uint16_t* blp = HI ? nullptr : o.blo + (int64_t)tbase * gv.lda;
  // load q of this lane: row r, columns h*32 + q*8 .. + 8 of the tile (one
  // contiguous kilobyte per wave and load)
  const int64_t lane_off = (int64_t)(wv * 4 * 64 + lane) * 8;
  constexpr int SEGS = NT * 32 * 8;          // 16-byte segments per chunk per array
  constexpr int SPT = SEGS / 256;            // per thread
  // every thread stages whole segments unconditionally: a guarded, partly
  // assigned staging array is placed in scratch memory by the compiler
  static_assert(SEGS % 256 == 0, "B segments must divide evenly over the workgroup");

  // Software pipeline.  The A fragment of chunk c is loaded three chunks
  // ahead into one of three register sets (c mod 3) that the MFMAs of chunk c
  // read directly; the next load into a set is issued after the MFMAs that
  // read it.  The B segments of chunk c are loaded two chunks ahead into one
  // of two staging sets (c mod 2) and written to LDS at the top of chunk c.
  // Every chunk issues, in this order, B(c+2) after its LDS write and A(c+3)
  // after its MFMAs, so at the top of chunk c the loads still in flight are
  // A(c+1), B(c+1) and A(c+2): waiting for B(c) (and, being older, A(c))
  // leaves two chunks of A, 64 KB per workgroup, in flight while chunk c
  // computes.  All loads are unconditional (chunk indices clamped to the last
  // chunk, whose re-reads hit the cache), the loop is unrolled six chunks
  // deep so that every set is a fixed register range, and the prologue issues
  // the loads in the loop's order: the compiler's count of loads in flight is
  // the same on every path into a chunk.  Chunks past the end only load.
  u32x4 s0h[4], s0l[4], s1h[4], s1l[4], s2h[4], s2l[4];
  u32x4 t0h[SPT], t0l[SPT], t1h[SPT], t1l[SPT];
  const int last = nchunks - 1;
  // addresses as a wave-uniform base plus a 32-bit lane offset, so the loads
  // take the scalar-base form and keep few vector registers for addresses
  const uint16_t* abh = gv.lhi + tile0;
  const uint16_t* abl = HI ? nullptr : gv.llo + tile0;
  const int a_lane = (int)lane_off;
  int b_lane[SPT];
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int sg = threadIdx.x + q * 256;
    b_lane[q] = (sg >> 3) * (int)gv.lda + (sg & 7) * 8;
  }
  auto load_a = [&](int c, u32x4 (&dh)[4], u32x4 (&dl)[4]) {
    const uint16_t* bh_ = abh + (int64_t)c * cstride;
    const uint16_t* bl_ = HI ? nullptr : abl + (int64_t)c * cstride;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if constexpr (ST) {
        dh[q] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(bh_ + (a_lane + q * 512)));
        if constexpr (!HI)
          dl[q] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(bl_ + (a_lane + q * 512)));
      } else {
        dh[q] = *reinterpret_cast<const u32x4*>(bh_ + (a_lane + q * 512));
        if constexpr (!HI) dl[q] = *reinterpret_cast<const u32x4*>(bl_ + (a_lane + q * 512));
      }
    }
  };
  auto load_b = [&](int c, u32x4 (&dh)[SPT], u32x4 (&dl)[SPT]) {
    const uint16_t* bh_ = bhp + (int64_t)c * KC;
    const uint16_t* bl_ = HI ? nullptr : blp + (int64_t)c * KC;
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      dh[q] = *reinterpret_cast<const u32x4*>(bh_ + b_lane[q]);
      if constexpr (!HI) dl[q] = *reinterpret_cast<const u32x4*>(bl_ + b_lane[q]);
    }
  };
  load_a(0, s0h, s0l);
  load_b(0, t0h, t0l);
  load_a(min(1, last), s1h, s1l);
  load_b(min(1, last), t1h, t1l);
  load_a(min(2, last), s2h, s2l);
  floatx16 acc[NT];
  double accd[NT][16];
#pragma unroll
  for (int n = 0; n < NT; ++n)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      acc[n][i] = 0.f;
      accd[n][i] = 0.0;
    }

  auto step = [&](int c, u32x4 (&sh)[4], u32x4 (&sl)[4], u32x4 (&th)[SPT], u32x4 (&tl)[SPT]) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int sg = threadIdx.x + q * 256;
      *reinterpret_cast<u32x4*>(&sbh[sg >> 3][(sg & 7) * 8]) = th[q];
      if constexpr (!HI) *reinterpret_cast<u32x4*>(&sbl[sg >> 3][(sg & 7) * 8]) = tl[q];
    }
    __syncthreads();
    load_b(min(c + 2, last), th, tl);
    if (c < nchunks) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int n = 0; n < NT; ++n) {
          const u32x4 b_h = *reinterpret_cast<const u32x4*>(&sbh[n * 32 + r][h * 32 + j * 8]);
          if constexpr (HI) {
            acc[n] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, sh[j]),
                                                            __builtin_bit_cast(half8, b_h),
                                                            acc[n], 0, 0, 0);
          } else {
            const u32x4 b_l =
                *reinterpret_cast<const u32x4*>(&sbl[n * 32 + r][h * 32 + j * 8]);
            acc[n] = split3<BF>(sh[j], sl[j], b_h, b_l, acc[n]);
          }
        }
        // keep the B fragments of one K step live at a time (register budget)
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int n = 0; n < NT; ++n)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          accd[n][i] += (double)acc[n][i];
          acc[n][i] = 0.f;
        }
    }
    load_a(min(c + 3, last), sh, sl);
  };
  for (int c = 0; c < nchunks; c += 6) {
    step(c, s0h, s0l, t0h, t0l);
    step(c + 1, s1h, s1l, t1h, t1l);
    step(c + 2, s2h, s2l, t0h, t0l);
    step(c + 3, s0h, s0l, t1h, t1l);
    step(c + 4, s1h, s1l, t0h, t0l);
    step(c + 5, s2h, s2l, t1h, t1l);
  }
  __syncthreads();   // every wave is done with the staged target tiles
  write_fields<NT>(gv, o, T, tbase, row0, lane, accd, reinterpret_cast<float*>(lds), out);
}

template <int NT, bool ST>
__global__ __launch_bounds__(256, 2) void kl_gemm_f16x3(GemmView gv, BatchOperand o, int32_t T,
                                                     int32_t groups, float* __restrict__ out) {
  gemm_split_body<NT, false, false, ST>(gv, o, T, groups, out);
}

template <int NT, bool ST>
__global__ __launch_bounds__(256, 2) void kl_gemm_bf16x3(GemmView gv, BatchOperand o, int32_t T,
                                                      int32_t groups, float* __restrict__ out) {
  gemm_split_body<NT, true, false, ST>(gv, o, T, groups, out);
}

template <int NT, bool ST>
__global__ __launch_bounds__(256, 2) void kl_gemm_f16(GemmView gv, BatchOperand o, int32_t T,
                                                   int32_t groups, float* __restrict__ out) {
  gemm_split_body<NT, false, true, ST>(gv, o, T, groups, out);
}

template <int NT>
__global__ __launch_bounds__(256) void kl_gemm_f32(GemmView gv, BatchOperand o, int32_t T,
                                                   int32_t groups, float* __restrict__ out) {
  int rb, grp;
  block_tile(groups, rb, grp);
  if ((int64_t)rb * GROWS >= gv.N) return;   // padding of the grid to whole XCD rounds
  const int tbase = grp * 64;
  // target tile, reused by the epilogue as a 4 x 32 x 33-float stage
  // (at least 64 rows of 68 floats = 17,408 bytes >= 16,896)
  __shared__ __attribute__((aligned(16))) float sb[(NT == 1 ? 2 : NT) * 32][KC + 4];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
  const int64_t row0 = (int64_t)rb * GROWS + wv * 32;
  const int nchunks = (int)(gv.lda / KC);
  const int64_t tile0 = (int64_t)rb * (GROWS * KC);
  const int64_t cstride = gemm_row_tiles(gv.N) * (GROWS * KC);
  // load q of this lane: row r, columns h*32 + q*4 .. + 4 of the tile
  const float* ap = gv.l32 + tile0 + (int64_t)(wv * 8 * 64 + lane) * 4;
  const float* bp = o.b32 + (int64_t)tbase * gv.lda;
  constexpr int SEGS = NT * 32 * 16;          // 16-byte segments per chunk
  constexpr int SPT = SEGS / 256;
  static_assert(SEGS % 256 == 0, "B segments must divide evenly over the workgroup");

  // A fragments are staged as in kl_gemm_f16x3: loaded into na, copied into a.
  f32x4 a[8], na[8], bq[SPT];
#pragma unroll
  for (int q = 0; q < 8; ++q) na[q] = *reinterpret_cast<const f32x4*>(ap + q * 256);
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int sg = threadIdx.x + q * 256;
    bq[q] = *reinterpret_cast<const f32x4*>(bp + (int64_t)(sg >> 4) * gv.lda + (sg & 15) * 4);
  }
  floatx16 acc[NT];
  double accd[NT][16];
#pragma unroll
  for (int n = 0; n < NT; ++n)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      acc[n][i] = 0.f;
      accd[n][i] = 0.0;
    }

  for (int c = 0; c < nchunks; ++c) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int sg = threadIdx.x + q * 256;
      *reinterpret_cast<f32x4*>(&sb[sg >> 4][(sg & 15) * 4]) = bq[q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = na[q];
    __syncthreads();
    if (c + 1 < nchunks) {
      const int64_t ko = (int64_t)(c + 1) * KC;
      const int64_t ao = (int64_t)(c + 1) * cstride;
#pragma unroll
      for (int q = 0; q < 8; ++q) na[q] = *reinterpret_cast<const f32x4*>(ap + ao + q * 256);
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        const int sg = threadIdx.x + q * 256;
        bq[q] = *reinterpret_cast<const f32x4*>(bp + (int64_t)(sg >> 4) * gv.lda + ko +
                                                 (sg & 15) * 4);
      }
    }
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const float av[4] = {a[jj].x, a[jj].y, a[jj].z, a[jj].w};
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const f32x4 b4 = *reinterpret_cast<const f32x4*>(&sb[n * 32 + r][h * 32 + jj * 4]);
        const float bv[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
          acc[n] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[e], bv[e], acc[n], 0, 0, 0);
      }
    }
#pragma unroll
    for (int n = 0; n < NT; ++n)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        accd[n][i] += (double)acc[n][i];
        acc[n][i] = 0.f;
      }
  }
  __syncthreads();
  write_fields<NT>(gv, o, T, tbase, row0, lane, accd, &sb[0][0], out);
}

hipError_t launch_batch_kl(DenseView dv, GemmView gv, TargetList tl, int32_t T, void* ws,
                           float* out, hipStream_t s) {
  if (T <= 0 || T > kMaxBatch || gv.lda % KC != 0) return hipErrorInvalidValue;
  const int Tpad = padded_targets(T);
  const BatchOperand o = carve(gv, Tpad, ws);
  hipLaunchKernelGGL(batch_target_prep, dim3(Tpad), dim3(256), 0, s, dv, gv, tl, T, o);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int groups = Tpad <= 32 ? 1 : Tpad / 64;
  const int64_t rblocks = (gv.N + GROWS - 1) / GROWS;
  const int64_t rpad = (rblocks + kXcds - 1) / kXcds * kXcds;
  const dim3 grid((unsigned)(rpad * groups));
  if (gv.form == 0) {
    if (Tpad == 32)
      hipLaunchKernelGGL(kl_gemm_f32<1>, grid, dim3(256), 0, s, gv, o, T, groups, out);
    else
      hipLaunchKernelGGL(kl_gemm_f32<2>, grid, dim3(256), 0, s, gv, o, T, groups, out);
  } else if (gv.form == 2) {
    if (Tpad == 32)
      hipLaunchKernelGGL((kl_gemm_bf16x3<1, true>), grid, dim3(256), 0, s, gv, o, T, groups, out);
    else if (groups == 1)
      hipLaunchKernelGGL((kl_gemm_bf16x3<2, true>), grid, dim3(256), 0, s, gv, o, T, groups, out);
    else
      hipLaunchKernelGGL((kl_gemm_bf16x3<2, false>), grid, dim3(256), 0, s, gv, o, T, groups, out);
  } else if (gv.form == 3) {
    if (Tpad == 32)
      hipLaunchKernelGGL((kl_gemm_f16<1, true>), grid, dim3(256), 0, s, gv, o, T, groups, out);
    else if (groups == 1)
      hipLaunchKernelGGL((kl_gemm_f16<2, true>), grid, dim3(256), 0, s, gv, o, T, groups, out);
    else
      hipLaunchKernelGGL((kl_gemm_f16<2, false>), grid, dim3(256), 0, s, gv, o, T, groups, out);
  } else {
    if (Tpad == 32)
      hipLaunchKernelGGL((kl_gemm_f16x3<1, true>), grid, dim3(256), 0, s, gv, o, T, groups, out);
    else if (groups == 1)
      hipLaunchKernelGGL((kl_gemm_f16x3<2, true>), grid, dim3(256), 0, s, gv, o, T, groups, out);
    else
      hipLaunchKernelGGL((kl_gemm_f16x3<2, false>), grid, dim3(256), 0, s, gv, o, T, groups, out);
  }
  return hipGetLastError();
}

}  // namespace dd
