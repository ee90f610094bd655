// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dd {

constexpr int kWave = 64;

// Dense resident form: FP32 rows of the kept columns, row stride `ld`
// (a multiple of 4 floats, zero padded), plus an optional FP64 master when
// the matrix was loaded in FP64.
struct DenseView {
  const float* P;      // [N][ld]
  const double* P64;   // [N][B] or nullptr (then P is the master)
  int64_t ld;
  int32_t N, B;
};

// Truncated resident form.  Row x occupies [start[x], start[x] + len[x]) of
// col/val; start[x] is a multiple of 4.  Padding slots hold col 0, val 0.
struct CsrView {
  const int64_t* start;  // [N]
  const int32_t* len;    // [N]
  const uint16_t* col;   // [nnz_padded]
  const float* val;      // [nnz_padded]
  const double* val64;   // [nnz_padded] or nullptr
  const double* phi;     // [N] floor of each row (the truncation threshold)
  const double* lphi;    // [N] log2 of the floor
  const uint16_t* val16; // [nnz_padded] FP16 bits of val * 2^e_x, or nullptr
  const float* rscale;   // [N] 2^-e_x (with val16)
  int32_t N, B;
};

struct Bound {
  double abs, rel;
};

// ---- load-time conversion (convert.hip) ----
hipError_t launch_row_stats(const void* raw, int is_f64, int32_t N, int32_t B, double* row_sum,
                            double* row_max, int32_t* bad_rows, hipStream_t s);
hipError_t launch_col_nonzero(const void* raw, int is_f64, int32_t N, int32_t B, int32_t* flags,
                              hipStream_t s);
hipError_t launch_gather_cols(const void* raw, int is_f64, int32_t N, int32_t B,
                              const int32_t* kept, int32_t Bk, int64_t ld, float* out32,
                              double* out64, hipStream_t s);
hipError_t launch_row_entropy(DenseView v, double* H, hipStream_t s);
hipError_t launch_trunc_count(DenseView v, const double* thr, int32_t* counts, hipStream_t s);
hipError_t launch_trunc_fill(DenseView v, const double* thr, const int64_t* start, uint16_t* col,
                             float* val, double* val64, hipStream_t s);
// FP16 copy of the stored values, row x scaled by 2^e_x (rscale[x] = 2^-e_x).
hipError_t launch_csr_f16(const int64_t* start, const int32_t* len, const float* val,
                          const float* rscale, int32_t N, uint16_t* val16, hipStream_t s);
// floor: nullable per-row floor phi_x; with it l = log max(P_xb, phi_x) - o_x.
hipError_t launch_log_forms(DenseView v, int form, int64_t lda, float* l32, uint16_t* lhi,
                            uint16_t* llo, float* offset, int32_t* zeros, const double* floor,
                            hipStream_t s);

// ---- streaming fields (stream.hip) ----
hipError_t launch_dense_field(DenseView v, int32_t target, int kind, float* out, hipStream_t s);
hipError_t launch_csr_field(CsrView v, int32_t target, int kind, float* out, hipStream_t s);
// TV and KL of one target in one pass over the rows (the same values as two
// single-kind launches)
hipError_t launch_dense_tv_kl(DenseView v, int32_t target, float* tv, float* kl, hipStream_t s);
hipError_t launch_csr_tv_kl(CsrView v, int32_t target, float* tv, float* kl, hipStream_t s);

// ---- batched KL contraction (gemm.hip) ----
// The log-kernel operand is stored in tiles of kGemmRows rows by kGemmK
// columns, chunk-major: with R = rows padded / kGemmRows, the tile of element
// (x, b) starts at
//   ((b / kGemmK) * R + x / kGemmRows) * kGemmRows * kGemmK,
// so one workgroup's chunk is one contiguous block, and the workgroups that
// run together (consecutive row tiles, all at about the same chunk) read one
// contiguous window of memory rather than blocks a fixed stride apart, which
// would load the same memory channels.  Inside a tile the elements are in the
// order the contraction's waves load them (gemm_tile_offset): a wave owns 32
// rows, lane r + 32 h holds row r, columns h*32 + q*V .. + V for its load q
// (V = 8 FP16 values or 4 FP32 values: 16 bytes), and load q of a wave reads
// one contiguous kilobyte.  Rows are padded to a multiple of kGemmRows and
// columns to lda; padding holds zeros.
constexpr int kGemmRows = 128;
constexpr int kGemmK = 64;
__host__ __device__ inline int64_t gemm_tile_offset(int form_f32, int xr, int k) {
  const int w = xr >> 5, r = xr & 31, h = k >> 5, lane = h * 32 + r;
  if (form_f32) return ((int64_t)(w * 8 + ((k & 31) >> 2)) * 64 + lane) * 4 + (k & 3);
  return ((int64_t)(w * 4 + ((k & 31) >> 3)) * 64 + lane) * 8 + (k & 7);
}
struct GemmView {
  const float* l32;      // tiled log P - o_x  (form F32)
  const uint16_t* lhi;   // tiled FP16 bits    (form F16X3)
  const uint16_t* llo;
  const float* offset;   // [N] o_x = log max_b P_xb
  int64_t lda;           // a multiple of kGemmK
  int32_t N, B, form;
};
inline int64_t gemm_rows_padded(int64_t N) { return (N + kGemmRows - 1) / kGemmRows * kGemmRows; }
__host__ __device__ inline int64_t gemm_row_tiles(int64_t N) { return (N + kGemmRows - 1) / kGemmRows; }
constexpr int kMaxBatch = 256;  // targets per contraction launch (groups of 64 per workgroup)
struct TargetList {
  int32_t t[kMaxBatch];
};
size_t batch_kl_workspace(GemmView gv, int32_t T);
// Dense rows of the truncated target rows (see convert.hip), one block per row.
hipError_t launch_csr_rows_dense(CsrView v, TargetList tl, int32_t T, int32_t Tpad, int64_t ld,
                                 float* out32, double* out64, hipStream_t s);

// ---- Poisson kernel of a grid domain (poisson.hip) ----
struct GridSolveStats {
  int32_t iterations, batches, levels, total_iterations;
  int32_t converged;   // every column reached rr <= tol^2 bb
  double max_rel_residual;
};
int32_t grid_levels(int32_t G);
size_t grid_poisson_workspace(int32_t G, int32_t C);
// Columns [col_begin, col_begin + ncols) of P_IB, C columns per batch (a
// multiple of 64); node_type as in dd_grid_poisson_kernel, already validated.
hipError_t grid_poisson(int32_t G, const uint8_t* node_type, int32_t col_begin, int32_t ncols,
                        int32_t C, double tol, int32_t max_iter, float* P32, int64_t ld32,
                        double* P64, int64_t ld64, GridSolveStats* st, hipStream_t s);
// Dirichlet Green's functions D_Ip = (-L_II)^{-1} e_p of the same operator for
// the interior vertices p = poles[c] (interior-local ids, validated), written
// one per output row: D32[c][ld32], D64[c][ld64] over the interior rows.
hipError_t grid_green(int32_t G, const uint8_t* node_type, const int32_t* poles, int32_t ncols,
                      int32_t C, double tol, int32_t max_iter, float* D32, int64_t ld32,
                      double* D64, int64_t ld64, GridSolveStats* st, hipStream_t s);

// Truncated fields of many targets in one pass over the stored rows
// (csr_batch.hip).  Up to kMaxBatch targets per launch; ws holds
// csr_batch_workspace(v, T) bytes.
size_t csr_batch_workspace(CsrView v, int32_t T);
// TV runs in fixed point with values times 2^tv_shift when tv_shift > 0 (the
// caller picks it so that row sums times 2^tv_shift stay below 2^32).
hipError_t launch_csr_batch(CsrView v, TargetList tl, int32_t T, int kind, int tv_shift, void* ws,
                            float* out, hipStream_t s);
hipError_t launch_batch_kl(DenseView dv, GemmView gv, TargetList tl, int32_t T, void* ws,
                           float* out, hipStream_t s);

// ---- paths (path.hip) ----
// Up to kInlinePaths paths carry their sources, targets and bounds in the
// kernel arguments (no host-to-device copy per call).
constexpr int kInlinePaths = 16;
struct PathSmall {
  int32_t src[kInlinePaths];
  int32_t tgt[kInlinePaths];
  double babs[kInlinePaths];
  double brel[kInlinePaths];
};
struct PathArgs {
  const int32_t* adj;       // [N][adj_w] neighbour ids, -1 padded
  int32_t adj_w;
  const float* fields;      // [T][N]
  const Bound* bounds;      // [T] device, or nullptr when inline
  const int32_t* sources;   // [T] device, or nullptr when inline
  const int32_t* targets;   // [T] device, or nullptr when inline
  PathSmall small;
  const double* trow;       // [T][B] FP64 target rows (truncated rows for CSR handles)
  const double* tlog;       // [T][B] log of trow (0 where trow is 0)
  const double* tconst;     // [T][4]: W_t, H_t (natural log), |S_t|, sum p |ln p|
  int32_t* path;            // [T][max_steps+1]
  int32_t* len;             // [T]
  int32_t* status;          // [T]
  int32_t* rechecks;        // [T] or nullptr (on-demand walk: rows evaluated)
  int32_t T, max_steps, kind, is_csr;
  // truncation of the target row before the sums (0: none); thr = tau * max
  // of the row when tau_relative, else tau
  double tgt_tau;
  int32_t tgt_tau_relative;
  int32_t tgt_in_lds;       // set by the launcher: trow/tlog staged in LDS
  int32_t l1;               // KL walks on dense rows: level-1 rows first (see path.hip)
};
hipError_t launch_target_rows(DenseView dv, CsrView cv, PathArgs a, double* trow, double* tlog,
                              double* tconst, hipStream_t s);
hipError_t launch_paths(DenseView dv, CsrView cv, PathArgs a, hipStream_t s);
// walk that evaluates FP64 distances on demand (no field): uses adj, sources,
// targets, trow/tlog/tconst, path/len/status, rechecks (= rows evaluated)
hipError_t launch_paths_on_demand(DenseView dv, CsrView cv, PathArgs a, hipStream_t s);
// FP64 fields of T targets into out[T][N] (uses T, targets, kind, is_csr,
// trow/tlog/tconst of PathArgs)
hipError_t launch_exact_fields(DenseView dv, CsrView cv, PathArgs a, int32_t N, double* out,
                               hipStream_t s);
// KL over the truncated support of the target row, one streaming pass
hipError_t launch_support_kl_field(DenseView v, int32_t target, double tau, int tau_relative,
                                   float* out, hipStream_t s);
// local-minimum census (path.hip): uses adj, adj_w, fields, T, targets/bounds
// (inline or device) of PathArgs
hipError_t launch_local_minima(PathArgs a, int32_t N, uint8_t* cls, int32_t* counts,
                               hipStream_t s);
// FP64 re-decision of the undecided census entries (uses adj, adj_w, T,
// targets, kind, is_csr, trow/tlog/tconst of PathArgs); counts recomputed
hipError_t launch_resolve_minima(DenseView dv, CsrView cv, PathArgs a, int32_t N, uint8_t* cls,
                                 int32_t* counts, hipStream_t s);

// Triangle-based paths (tri.hip).
struct TriArgs {
  const int32_t* faces;     // [F][8]: v0 v1 v2 counter-clockwise, then the face across
                            // edge (v_k, v_k+1) for k = 0..2 (-1: none), 2 unused
  const double* xy;         // [N][2]
  const int32_t* vfaces;    // [N][vf_w] incident faces ascending, -1 padded
  int32_t vf_w;
  const int32_t* adj;       // [N][adj_w] neighbour ids, -1 padded
  int32_t adj_w;
  const float* fields;      // [T][N] FP32, or
  const double* fields64;   // [T][N] FP64 (exactly one of the two is set)
  const int32_t* sources;   // device [T]
  const int32_t* targets;   // device [T]
  double* points;           // [T][max_steps+1][2]
  int32_t* where;           // [T][max_steps+1][2]
  int32_t* len;             // [T]
  int32_t* status;          // [T]
  int32_t T, N, max_steps;
};
hipError_t launch_triangle_paths(TriArgs a, hipStream_t s);

// Device table of the FP64 log used by the path kernels; once per device.
hipError_t init_log_table();
// Exhaustive check of the FP32 hardware log2 against the bound the level-1
// rows assume (path.hip); ratio[0] <= 1 means the bound holds on this device.
hipError_t check_log2_bound(double ratio[2]);

// Fixed per-GPU scratch of the allocation-free batch entry point
// (scratch.hip): its size, and its device address on `device` (which must be
// current), looked up once per device.
constexpr size_t kFixedScratchBytes = size_t(48) << 20;
hipError_t fixed_scratch(int device, void** out);

int num_cus();

}  // namespace dd
