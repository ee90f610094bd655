// Discrete Poisson kernel of a grid domain on the device (Section IV, eqs.
// 32-33): column b of P_IB is the discrete harmonic function on the interior
// vertices whose boundary values are the indicator of boundary vertex b.  On
// the right-triangle grid the cotangent Laplacian is the five-point stencil,
// so every column solves
//     4 u_v - sum_{interior n ~ v} u_n = #{boundary n ~ v : n = b}
// over the interior vertices v.  The paper pre-factorises L_II (sparse
// Cholesky) and back-substitutes per column; a sparse factorisation is a
// poor fit for a GPU, so this file solves all columns of a batch at once by
// conjugate gradients preconditioned with one geometric multigrid V-cycle:
//
// * Every level is the full G_l x G_l vertex grid, one FP64 value per vertex
//   and column, columns contiguous ([G_l^2][C]): a wave holds 64 columns of
//   one vertex, so every load and store is one 512-byte segment and every
//   branch on the vertex type is wave-uniform.  Values at vertices that are
//   not unknowns are kept at zero, so a stencil reads its four neighbours
//   without masks.
// * Level l+1 has G_{l+1} = floor(G_l / 2) + 1 vertices per side; coarse
//   vertex I is an unknown when fine vertex 2I is inside the fine grid and an
//   unknown there.  The fine grid's edge holds no unknown, so neither does
//   the coarse grid's (for odd G_l the edge maps to the edge; for even G_l
//   the coarse edge lies past the fine grid), and every stencil, restriction
//   and prolongation index of an unknown stays inside its grid.  The coarse
//   operator is the same unscaled five-point stencil, restriction is the
//   transpose of bilinear prolongation (weights 1, 1/2, 1/4), which matches
//   it to the Galerkin operator for smooth errors.
// * Smoothing is damped Jacobi (omega = 0.8, one sweep before and one after
//   the coarse correction); the coarsest level runs a fixed number of sweeps
//   from zero.  Each piece is symmetric, so the V-cycle is a symmetric
//   positive definite preconditioner.
// * A level costs two passes: the pre-smoothed residual is formed inside the
//   restriction, and prolongation is fused with the post-smoothing sweep.
// * Per-column scalars (alpha, beta, residual norms) stay on the device; dot
//   products reduce in a fixed order, so results do not depend on timing.
//   A column stops updating at its first iterate with ||r||^2 <= tol^2 ||b||^2
//   (a device flag), so its result does not depend on the other columns of
//   its batch either: the batch runs until all its columns have stopped.
// * Work-groups take row ranges that are contiguous per XCD (work-groups go
//   to the 8 XCDs round robin), so the ranges an XCD runs together are
//   adjacent and a vertex's neighbours one grid row up and down were fetched
//   shortly before by the same XCD.  Part of them are fetched again (from the
//   memory-side cache): the stencil kernels are bound by load latency, and a
//   column-walking variant that removed those fetches ran slower.
#include <math.h>

#include <vector>

#include "dd_internal.h"

namespace dd {
namespace {

constexpr int kRowsPerWave = 128;                // vertices per wave
constexpr int kWaves = 4;
constexpr int kRowsPerBlock = kWaves * kRowsPerWave;
constexpr double kW = 0.2;                       // omega / diagonal = 0.8 / 4
constexpr int kCoarseSweeps = 20;
constexpr int kCheckEvery = 4;                   // iterations between convergence checks
constexpr int kXcd = 8;

__host__ __device__ inline int64_t row_blocks(int64_t nodes) {
  return (nodes + kRowsPerBlock - 1) / kRowsPerBlock;
}

// Row block and column group of this work-group; false for grid padding.
__device__ __forceinline__ bool block_of(int64_t nodes, int groups, int64_t& rb, int& grp) {
  const int64_t nrb = row_blocks(nodes);
  const int64_t rpx = (nrb + kXcd - 1) / kXcd;
  const int64_t b = blockIdx.x, k = b / kXcd;
  grp = (int)(k / rpx);
  rb = (b % kXcd) * rpx + k % rpx;
  return grp < groups && rb < nrb;
}

inline unsigned grid_size(int64_t nodes, int groups) {
  const int64_t nrb = row_blocks(nodes);
  return (unsigned)(kXcd * ((nrb + kXcd - 1) / kXcd) * groups);
}

// Sum of the four waves' per-column partials into part[rb][c].
__device__ __forceinline__ void block_partial(double v, double* part, int64_t rb, int64_t C,
                                              int64_t c) {
  __shared__ double red[kWaves][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  red[wv][lane] = v;
  __syncthreads();
  if (wv == 0) part[rb * C + c] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

__global__ __launch_bounds__(256) void pk_fill(double* a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0.0;
}

// Right-hand sides of a batch: column c has a 1 at every interior neighbour
// of boundary vertex bnd[c] (r is zero on entry).
__global__ void pk_rhs(double* r, const uint8_t* act, int32_t G, int64_t C, const int32_t* bnd,
                       int32_t ncols) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  const int b = bnd[c], i = b % G, j = b / G;
  const int di[4] = {1, -1, 0, 0}, dj[4] = {0, 0, 1, -1};
  for (int d = 0; d < 4; ++d) {
    const int ni = i + di[d], nj = j + dj[d];
    if (ni < 0 || nj < 0 || ni >= G || nj >= G) continue;
    const int64_t n = (int64_t)nj * G + ni;
    if (act[n]) r[n * C + c] = 1.0;
  }
}

// Right-hand sides of a batch of Green's functions: column c is the unit
// vector of interior vertex src[c] (global grid id; r is zero on entry).
__global__ void pk_rhs_point(double* r, int64_t C, const int32_t* src, int32_t ncols) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  r[(int64_t)src[c] * C + c] = 1.0;
}

// part = per-block partials of sum_v a_v b_v per column.
__global__ __launch_bounds__(256) void pk_dot(const double* a, const double* b, const uint8_t* act,
                                              int32_t G, int64_t C, int groups, double* part) {
  const int64_t nodes = (int64_t)G * G;
  int64_t rb;
  int grp;
  if (!block_of(nodes, groups, rb, grp)) return;
  const int64_t c = grp * 64 + (threadIdx.x & 63);
  const int64_t g0 = rb * kRowsPerBlock + (threadIdx.x >> 6) * kRowsPerWave;
  double acc = 0.0;
  for (int k = 0; k < kRowsPerWave; ++k) {
    const int64_t g = g0 + k;
    if (g >= nodes) break;
    if (act[g]) acc += a[g * C + c] * b[g * C + c];
  }
  block_partial(acc, part, rb, C, c);
}

// q = A p and the partials of p.q.
__global__ __launch_bounds__(256) void pk_matvec(const double* __restrict__ p,
                                                 double* __restrict__ q, const uint8_t* act,
                                                 int32_t G, int64_t C, int groups, double* part) {
  const int64_t nodes = (int64_t)G * G;
  int64_t rb;
  int grp;
  if (!block_of(nodes, groups, rb, grp)) return;
  const int64_t c = grp * 64 + (threadIdx.x & 63);
  const int64_t g0 = rb * kRowsPerBlock + (threadIdx.x >> 6) * kRowsPerWave;
  const int64_t up = (int64_t)G * C;
  double acc = 0.0;
#pragma unroll 4
  for (int k = 0; k < kRowsPerWave; ++k) {
    const int64_t g = g0 + k;
    if (g >= nodes) break;
    const int64_t o = g * C + c;
    double v = 0.0;
    if (act[g]) {
      const double pc = p[o];
      v = 4.0 * pc - ((p[o - C] + p[o + C]) + (p[o - up] + p[o + up]));
      acc += pc * v;
    }
    q[o] = v;
  }
  block_partial(acc, part, rb, C, c);
}

// alpha = rz / pq per column (0 once the column has stopped), kept in
// alpha_out for the step x += alpha p, which the next direction update makes
// while it reads p anyway; r -= alpha q; partials of r.r.
__global__ __launch_bounds__(256) void pk_update(double* __restrict__ r,
                                                 const double* __restrict__ q, const double* rz,
                                                 const double* pq, const double* done,
                                                 double* alpha_out, const uint8_t* act, int32_t G,
                                                 int64_t C, int groups, double* part) {
  const int64_t nodes = (int64_t)G * G;
  int64_t rb;
  int grp;
  if (!block_of(nodes, groups, rb, grp)) return;
  const int64_t c = grp * 64 + (threadIdx.x & 63);
  const double a = done[c] == 0.0 && pq[c] > 0.0 ? rz[c] / pq[c] : 0.0;
  if (rb == 0 && threadIdx.x < 64) alpha_out[c] = a;   // one writer per column
  const int64_t g0 = rb * kRowsPerBlock + (threadIdx.x >> 6) * kRowsPerWave;
  double acc = 0.0;
#pragma unroll 4
  for (int k = 0; k < kRowsPerWave; ++k) {
    const int64_t g = g0 + k;
    if (g >= nodes) break;
    if (!act[g]) continue;
    const int64_t o = g * C + c;
    const double rn = r[o] - a * q[o];
    r[o] = rn;
    acc += rn * rn;
  }
  block_partial(acc, part, rb, C, c);
}

// p = z (first) or z + beta p, beta = rz_new / rz_old per column; before p
// is replaced, the previous step's x += alpha p.
__global__ __launch_bounds__(256) void pk_direction(double* __restrict__ p,
                                                    const double* __restrict__ z,
                                                    double* __restrict__ x, const double* alpha,
                                                    const double* rz_new, const double* rz_old,
                                                    int first, const uint8_t* act, int32_t G,
                                                    int64_t C, int groups) {
  const int64_t nodes = (int64_t)G * G;
  int64_t rb;
  int grp;
  if (!block_of(nodes, groups, rb, grp)) return;
  const int64_t c = grp * 64 + (threadIdx.x & 63);
  const double beta = first ? 0.0 : (rz_old[c] > 0.0 ? rz_new[c] / rz_old[c] : 0.0);
  const double a = first ? 0.0 : alpha[c];
  const int64_t g0 = rb * kRowsPerBlock + (threadIdx.x >> 6) * kRowsPerWave;
#pragma unroll 4
  for (int k = 0; k < kRowsPerWave; ++k) {
    const int64_t g = g0 + k;
    if (g >= nodes) break;
    const int64_t o = g * C + c;
    if (!act[g]) {
      p[o] = 0.0;
      continue;
    }
    if (first) {
      p[o] = z[o];
    } else {
      const double po = p[o];
      x[o] += a * po;
      p[o] = z[o] + beta * po;
    }
  }
}

// The last step x += alpha p (at exit, with no direction update after it).
__global__ __launch_bounds__(256) void pk_axpy(double* __restrict__ x,
                                               const double* __restrict__ p, const double* alpha,
                                               const uint8_t* act, int32_t G, int64_t C,
                                               int groups) {
  const int64_t nodes = (int64_t)G * G;
  int64_t rb;
  int grp;
  if (!block_of(nodes, groups, rb, grp)) return;
  const int64_t c = grp * 64 + (threadIdx.x & 63);
  const double a = alpha[c];
  const int64_t g0 = rb * kRowsPerBlock + (threadIdx.x >> 6) * kRowsPerWave;
  for (int k = 0; k < kRowsPerWave; ++k) {
    const int64_t g = g0 + k;
    if (g >= nodes) break;
    if (act[g]) x[g * C + c] += a * p[g * C + c];
  }
}

// Restriction of the pre-smoothed residual: with e = W r (one damped Jacobi
// sweep from zero) the residual is t = r - A e; rc[I] = sum of the bilinear
// weights times t over the 3 x 3 fine vertices around 2I.  A wave walks
// consecutive coarse vertices of a row, so the fine column 2I + 1 of one is
// the column 2I' - 1 of the next: its three t values are carried over.
__global__ __launch_bounds__(256) void pk_down(const double* __restrict__ r, const uint8_t* act,
                                               int32_t G, double* __restrict__ rc,
                                               const uint8_t* actc, int32_t Gc, int64_t C,
                                               int groups) {
  const int64_t nodes = (int64_t)Gc * Gc;
  int64_t rb;
  int grp;
  if (!block_of(nodes, groups, rb, grp)) return;
  const int64_t c = grp * 64 + (threadIdx.x & 63);
  const int64_t g0 = rb * kRowsPerBlock + (threadIdx.x >> 6) * kRowsPerWave;
  const int64_t up = (int64_t)G * C;
  // t at a fine vertex n around an unknown centre.  n may lie on the grid's
  // edge (then it is not an unknown), where a neighbour can be past the
  // grid: a vertex that is not an unknown reads itself in place of its
  // neighbours, so every load is in the grid and none needs a branch (the
  // vertex type only selects)
  auto t_at = [&](int64_t n) -> double {
    const bool a = act[n];
    const int64_t o = n * C + c;
    const int64_t dh = a ? C : 0, dv = a ? up : 0;
    const double rn = r[o];
    const double t = rn - kW * (4.0 * rn - ((r[o - dh] + r[o + dh]) + (r[o - dv] + r[o + dv])));
    return a ? t : 0.0;
  };
  double l0 = 0.0, l1 = 0.0, l2 = 0.0;   // t at column 2I - 1, rows 2J - 1, 2J, 2J + 1
  bool carried = false;                  // l* hold the previous vertex's column 2I + 1
  int64_t I = g0 % Gc, J = g0 / Gc;      // coordinates of gc, carried along
  for (int k = 0; k < kRowsPerWave; ++k, I = I + 1 == Gc ? 0 : I + 1, J += I == 0) {
    const int64_t gc = g0 + k;
    if (gc >= nodes) break;
    double v = 0.0;
    if (actc[gc]) {
      const int64_t g = 2 * J * G + 2 * I;
      if (!carried) {
        l0 = t_at(g - 1 - G);
        l1 = t_at(g - 1);
        l2 = t_at(g - 1 + G);
      }
      const double m0 = t_at(g - G), m1 = t_at(g), m2 = t_at(g + G);
      const double r0 = t_at(g + 1 - G), r1 = t_at(g + 1), r2 = t_at(g + 1 + G);
      v = (m1 + 0.5 * ((m0 + m2) + (l1 + r1))) + 0.25 * ((l0 + l2) + (r0 + r2));
      l0 = r0;
      l1 = r1;
      l2 = r2;
      carried = true;
    } else {
      carried = false;
    }
    rc[gc * C + c] = v;
  }
}

// Bilinear prolongation of the coarse correction ec at fine vertex (i, j).
__device__ __forceinline__ double prolong(const double* __restrict__ ec, int32_t Gc, int64_t C,
                                          int64_t c, int32_t i, int32_t j) {
  const int64_t i0 = i >> 1, j0 = j >> 1;
  const int64_t a = (j0 * Gc + i0) * C + c;
  const bool oi = i & 1, oj = j & 1;
  if (!oi && !oj) return ec[a];
  if (!oj) return 0.5 * (ec[a] + ec[a + C]);
  const int64_t rowc = (int64_t)Gc * C;
  if (!oi) return 0.5 * (ec[a] + ec[a + rowc]);
  return 0.25 * ((ec[a] + ec[a + C]) + (ec[a + rowc] + ec[a + rowc + C]));
}

// Coarse correction and post-smoothing of one level: with the corrected
// e = W r + P ec at the unknowns (zero elsewhere),
//   out = e + W (r - A e);
// with `part`, also the partials of r.out (the preconditioned inner product).
__global__ __launch_bounds__(256) void pk_up(const double* __restrict__ r, const uint8_t* act,
                                             int32_t G, const double* __restrict__ ec, int32_t Gc,
                                             double* __restrict__ out, int64_t C, int groups,
                                             double* part) {
  const int64_t nodes = (int64_t)G * G;
  int64_t rb;
  int grp;
  if (!block_of(nodes, groups, rb, grp)) return;
  const int64_t c = grp * 64 + (threadIdx.x & 63);
  const int64_t g0 = rb * kRowsPerBlock + (threadIdx.x >> 6) * kRowsPerWave;
  // e at vertex n = (i, j); coordinates are carried along, not divided out.
  // The loads need no guard: r[n] is in the grid, and the prolongation of
  // any fine vertex reads coarse vertices (i+1)/2 <= Gc - 1, (j+1)/2 <= Gc - 1
  // (the vertex type only selects)
  auto e_at = [&](int64_t n, int32_t i, int32_t j) -> double {
    const double e = kW * r[n * C + c] + prolong(ec, Gc, C, c, i, j);
    return act[n] ? e : 0.0;
  };
  // a window of e along the wave's vertices: e(g - 1), e(g), e(g + 1) (the
  // vertices g +- 1 of an unknown g are its left and right neighbours)
  double acc = 0.0;
  double e_m = 0.0, e_c = 0.0;
  int32_t gi = 0, gj = 0;   // coordinates of g
  if (g0 < nodes) {
    gi = (int32_t)(g0 % G);
    gj = (int32_t)(g0 / G);
    // g0 - 1 is never an unknown when g0 starts a grid row (an edge vertex)
    e_m = gi > 0 ? e_at(g0 - 1, gi - 1, gj) : 0.0;
    e_c = e_at(g0, gi, gj);
  }
  for (int k = 0; k < kRowsPerWave; ++k) {
    const int64_t g = g0 + k;
    if (g >= nodes) break;
    const bool wrap = gi + 1 == G;
    const int32_t ni = wrap ? 0 : gi + 1, nj = wrap ? gj + 1 : gj;
    const double e_p = g + 1 < nodes ? e_at(g + 1, ni, nj) : 0.0;
    double v = 0.0;
    if (act[g]) {
      const double rg = r[g * C + c];
      const double s = (e_m + e_p) + (e_at(g - G, gi, gj - 1) + e_at(g + G, gi, gj + 1));
      v = e_c + kW * (rg - (4.0 * e_c - s));
      acc += rg * v;
    }
    out[g * C + c] = v;
    e_m = e_c;
    e_c = e_p;
    gi = ni;
    gj = nj;
  }
  if (part) block_partial(acc, part, rb, C, c);
}

// Damped Jacobi on the coarsest level: out = W r (first) or
// e + W (r - A e).
__global__ __launch_bounds__(256) void pk_jacobi(const double* __restrict__ r,
                                                 const double* __restrict__ e,
                                                 double* __restrict__ out, int first,
                                                 const uint8_t* act, int32_t G, int64_t C,
                                                 int groups, double* part) {
  const int64_t nodes = (int64_t)G * G;
  int64_t rb;
  int grp;
  if (!block_of(nodes, groups, rb, grp)) return;
  const int64_t c = grp * 64 + (threadIdx.x & 63);
  const int64_t g0 = rb * kRowsPerBlock + (threadIdx.x >> 6) * kRowsPerWave;
  const int64_t up = (int64_t)G * C;
  double acc = 0.0;
  for (int k = 0; k < kRowsPerWave; ++k) {
    const int64_t g = g0 + k;
    if (g >= nodes) break;
    const int64_t o = g * C + c;
    double v = 0.0;
    if (act[g]) {
      const double rg = r[o];
      if (first) {
        v = kW * rg;
      } else {
        const double eg = e[o];
        v = eg + kW * (rg - (4.0 * eg - ((e[o - C] + e[o + C]) + (e[o - up] + e[o + up]))));
      }
      acc += rg * v;
    }
    out[o] = v;
  }
  if (part) block_partial(acc, part, rb, C, c);
}

// done[c] = 1 from the first residual with rr <= tol2 * bb on (tol2 = tol^2,
// the same product the host tests).
__global__ void pk_converged(const double* rr, const double* bb, double tol2, double* done,
                             int64_t C) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c < C && rr[c] <= tol2 * bb[c]) done[c] = 1.0;
}

// out[c] = sum over row blocks of part[rb][c], in a fixed order: wave w of
// 16 sums the blocks w, w+16, ...; the 16 sums are added in wave order.
__global__ __launch_bounds__(1024) void pk_dot_final(const double* part, int64_t nrb, int64_t C,
                                                     double* out) {
  __shared__ double red[16][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t c = blockIdx.x * 64 + lane;
  double s = 0.0;
  for (int64_t b = wv; b < nrb; b += 16) s += part[b * C + c];
  red[wv][lane] = s;
  __syncthreads();
  if (wv == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w][lane];
    out[c] = t;
  }
}

// Rows of P from the solution: P[iloc[g]][c] = max(x, 0) (the exact solution
// is >= 0; this clears round-off below zero).
__global__ __launch_bounds__(256) void pk_write(const double* __restrict__ x, const uint8_t* act,
                                                const int32_t* iloc, int32_t G, int64_t C,
                                                int groups, int32_t ncols, float* P32,
                                                int64_t ld32, double* P64, int64_t ld64,
                                                int trans) {
  const int64_t nodes = (int64_t)G * G;
  int64_t rb;
  int grp;
  if (!block_of(nodes, groups, rb, grp)) return;
  const int64_t c = grp * 64 + (threadIdx.x & 63);
  const int64_t g0 = rb * kRowsPerBlock + (threadIdx.x >> 6) * kRowsPerWave;
  for (int k = 0; k < kRowsPerWave; ++k) {
    const int64_t g = g0 + k;
    if (g >= nodes) break;
    if (!act[g] || c >= ncols) continue;
    const double v = fmax(x[g * C + c], 0.0);
    const int64_t row = iloc[g];
    if (trans) {   // column c is output row c (one field per pole)
      if (P32) P32[c * ld32 + row] = (float)v;
      if (P64) P64[c * ld64 + row] = v;
    } else {
      if (P32) P32[row * ld32 + c] = (float)v;
      if (P64) P64[row * ld64 + c] = v;
    }
  }
}

struct Buf {
  void* p = nullptr;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t n) { return hipMalloc(&p, n ? n : 1); }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

#define PK_OR(expr)                      \
  do {                                   \
    hipError_t e_ = (expr);              \
    if (e_ != hipSuccess) return e_;     \
  } while (0)

}  // namespace

int32_t grid_levels(int32_t G) {
  int32_t n = 1;
  while (G / 2 + 1 >= 5) {
    G = G / 2 + 1;
    ++n;
  }
  return n;
}

size_t grid_poisson_workspace(int32_t G, int32_t C) {
  const int32_t L = grid_levels(G);
  size_t bytes = 0;
  int64_t Gl = G;
  for (int32_t l = 0; l < L; ++l) {
    const int64_t nodes = Gl * Gl;
    const int arrays = l == 0 ? 5 : (l == L - 1 ? 3 : 2);
    bytes += (size_t)arrays * nodes * C * 8 + (size_t)nodes;
    Gl = Gl / 2 + 1;
  }
  bytes += (size_t)row_blocks((int64_t)G * G) * C * 8 + 7 * (size_t)C * 8;
  bytes += (size_t)G * G * 4 + (size_t)C * 4;
  return bytes;
}

// The two column families share the solver: boundary indicators (P_IB, row-
// major output) or unit vectors of interior vertices (Green's functions,
// one output row per column).
static hipError_t grid_solve(int32_t G, const uint8_t* node_type, bool green,
                             const int32_t* poles, int32_t col_begin, int32_t ncols, int32_t C,
                             double tol, int32_t max_iter, float* P32, int64_t ld32, double* P64,
                             int64_t ld64, GridSolveStats* st, hipStream_t s) {
  const int32_t L = grid_levels(G);
  const int64_t nodes = (int64_t)G * G;
  const int groups = C / 64;
  // host: level masks, interior row index, boundary vertex list
  std::vector<std::vector<uint8_t>> act(L);
  std::vector<int32_t> Gs(L);
  act[0].resize(nodes);
  std::vector<int32_t> iloc(nodes, -1), bnd, ints;
  int32_t n_int = 0;
  for (int64_t g = 0; g < nodes; ++g) {
    act[0][g] = node_type[g] == 1;
    if (node_type[g] == 1) {
      iloc[g] = n_int++;
      ints.push_back((int32_t)g);
    }
    if (node_type[g] == 2) bnd.push_back((int32_t)g);
  }
  // global ids of the batch's sources: boundary vertices, or the poles
  std::vector<int32_t> src;
  if (green)
    for (int32_t c = 0; c < ncols; ++c) src.push_back(ints[poles[c]]);
  else
    src.assign(bnd.begin() + col_begin, bnd.begin() + col_begin + ncols);
  Gs[0] = G;
  for (int32_t l = 1; l < L; ++l) {
    const int32_t Gf = Gs[l - 1], Gc = Gf / 2 + 1;
    Gs[l] = Gc;
    act[l].assign((size_t)Gc * Gc, 0);
    for (int32_t J = 0; 2 * J < Gf; ++J)
      for (int32_t I = 0; 2 * I < Gf; ++I)
        act[l][(size_t)J * Gc + I] = act[l - 1][(size_t)(2 * J) * Gf + 2 * I];
  }
  // device buffers
  std::vector<Buf> dact(L), dr(L), de(L);
  Buf x, p, q, z, tco, part, sc, dil, dbnd;
  for (int32_t l = 0; l < L; ++l) {
    const size_t n = (size_t)Gs[l] * Gs[l];
    PK_OR(dact[l].alloc(n));
    PK_OR(hipMemcpyAsync(dact[l].p, act[l].data(), n, hipMemcpyHostToDevice, s));
    if (l > 0) {
      PK_OR(dr[l].alloc(n * C * 8));
      PK_OR(de[l].alloc(n * C * 8));
    }
  }
  const size_t v0 = (size_t)nodes * C * 8;
  PK_OR(dr[0].alloc(v0));
  PK_OR(x.alloc(v0));
  PK_OR(p.alloc(v0));
  PK_OR(q.alloc(v0));
  PK_OR(z.alloc(v0));
  if (L > 1) PK_OR(tco.alloc((size_t)Gs[L - 1] * Gs[L - 1] * C * 8));
  const int64_t nrb0 = row_blocks(nodes);
  PK_OR(part.alloc((size_t)nrb0 * C * 8));
  PK_OR(sc.alloc(7 * (size_t)C * 8));
  PK_OR(dil.alloc((size_t)nodes * 4));
  PK_OR(dbnd.alloc((size_t)C * 4));
  PK_OR(hipMemcpyAsync(dil.p, iloc.data(), (size_t)nodes * 4, hipMemcpyHostToDevice, s));
  double* rz = sc.as<double>();
  double* rzn = rz + C;
  double* pq = rz + 2 * C;
  double* rr = rz + 3 * C;
  double* bb = rz + 4 * C;
  double* done = rz + 5 * C;
  double* alpha = rz + 6 * C;
  const double tol2 = tol * tol;

  auto fill = [&](void* a, size_t n) {
    hipLaunchKernelGGL(pk_fill, dim3(2048), dim3(256), 0, s, static_cast<double*>(a), (int64_t)n);
  };
  auto dot_final = [&](int64_t nrb, double* out) {
    hipLaunchKernelGGL(pk_dot_final, dim3(groups), dim3(1024), 0, s, part.as<double>(), nrb,
                       (int64_t)C, out);
  };
  const uint8_t* a0 = dact[0].as<uint8_t>();
  const unsigned g0 = grid_size(nodes, groups);
  // z = M r and rz_out = r.z
  auto precondition = [&](double* rz_out) {
    if (L == 1) {
      // one level: the Jacobi sweeps of the coarsest level on the grid
      // itself, ping-ponging through q (free until the next product); the
      // start is chosen so that the last sweep lands in z
      double* bufs[2] = {z.as<double>(), q.as<double>()};
      int cur = kCoarseSweeps % 2 == 0 ? 0 : 1;
      hipLaunchKernelGGL(pk_jacobi, dim3(g0), dim3(256), 0, s, dr[0].as<double>(), nullptr,
                         bufs[cur], 1, a0, G, (int64_t)C, groups,
                         kCoarseSweeps == 0 ? part.as<double>() : nullptr);
      for (int k = 1; k <= kCoarseSweeps; ++k) {
        hipLaunchKernelGGL(pk_jacobi, dim3(g0), dim3(256), 0, s, dr[0].as<double>(), bufs[cur],
                           bufs[1 - cur], 0, a0, G, (int64_t)C, groups,
                           k == kCoarseSweeps ? part.as<double>() : nullptr);
        cur = 1 - cur;
      }
      dot_final(nrb0, rz_out);
      return;
    }
    for (int32_t l = 0; l + 1 < L; ++l) {
      const int64_t nc = (int64_t)Gs[l + 1] * Gs[l + 1];
      hipLaunchKernelGGL(pk_down, dim3(grid_size(nc, groups)), dim3(256), 0, s,
                         dr[l].as<double>(), dact[l].as<uint8_t>(), Gs[l], dr[l + 1].as<double>(),
                         dact[l + 1].as<uint8_t>(), Gs[l + 1], (int64_t)C, groups);
    }
    {
      const int32_t l = L - 1;
      const int64_t nc = (int64_t)Gs[l] * Gs[l];
      double* bufs[2] = {de[l].as<double>(), tco.as<double>()};
      int cur = kCoarseSweeps % 2 == 0 ? 0 : 1;   // the last sweep lands in de[l]
      const unsigned gc = grid_size(nc, groups);
      hipLaunchKernelGGL(pk_jacobi, dim3(gc), dim3(256), 0, s, dr[l].as<double>(), nullptr,
                         bufs[cur], 1, dact[l].as<uint8_t>(), Gs[l], (int64_t)C, groups, nullptr);
      for (int k = 1; k <= kCoarseSweeps; ++k) {
        hipLaunchKernelGGL(pk_jacobi, dim3(gc), dim3(256), 0, s, dr[l].as<double>(), bufs[cur],
                           bufs[1 - cur], 0, dact[l].as<uint8_t>(), Gs[l], (int64_t)C, groups,
                           nullptr);
        cur = 1 - cur;
      }
    }
    for (int32_t l = L - 2; l >= 0; --l) {
      const int64_t nf = (int64_t)Gs[l] * Gs[l];
      double* out = l == 0 ? z.as<double>() : de[l].as<double>();
      hipLaunchKernelGGL(pk_up, dim3(grid_size(nf, groups)), dim3(256), 0, s, dr[l].as<double>(),
                         dact[l].as<uint8_t>(), Gs[l], de[l + 1].as<double>(), Gs[l + 1], out,
                         (int64_t)C, groups, l == 0 ? part.as<double>() : nullptr);
    }
    dot_final(nrb0, rz_out);
  };

  st->levels = L;
  st->batches = 0;
  st->iterations = 0;
  st->total_iterations = 0;
  st->converged = 1;
  st->max_rel_residual = 0.0;
  std::vector<double> h_rr(C), h_bb(C);
  for (int32_t c0 = 0; c0 < ncols; c0 += C) {
    const int32_t nb = ncols - c0 < C ? ncols - c0 : C;
    PK_OR(hipMemcpyAsync(dbnd.p, src.data() + c0, (size_t)nb * 4, hipMemcpyHostToDevice, s));
    fill(dr[0].p, (size_t)nodes * C);
    fill(x.p, (size_t)nodes * C);
    fill(done, (size_t)C);
    if (green)
      hipLaunchKernelGGL(pk_rhs_point, dim3((nb + 63) / 64), dim3(64), 0, s, dr[0].as<double>(),
                         (int64_t)C, dbnd.as<int32_t>(), nb);
    else
      hipLaunchKernelGGL(pk_rhs, dim3((nb + 63) / 64), dim3(64), 0, s, dr[0].as<double>(), a0, G,
                         (int64_t)C, dbnd.as<int32_t>(), nb);
    hipLaunchKernelGGL(pk_dot, dim3(g0), dim3(256), 0, s, dr[0].as<double>(), dr[0].as<double>(),
                       a0, G, (int64_t)C, groups, part.as<double>());
    dot_final(nrb0, bb);
    PK_OR(hipGetLastError());
    PK_OR(hipMemcpyAsync(h_bb.data(), bb, (size_t)C * 8, hipMemcpyDeviceToHost, s));
    precondition(rz);
    hipLaunchKernelGGL(pk_direction, dim3(g0), dim3(256), 0, s, p.as<double>(), z.as<double>(),
                       x.as<double>(), alpha, rz, rz, 1, a0, G, (int64_t)C, groups);
    PK_OR(hipGetLastError());
    int32_t it = 0;
    double res = 0.0;
    bool all = false;
    for (;;) {
      ++it;
      hipLaunchKernelGGL(pk_matvec, dim3(g0), dim3(256), 0, s, p.as<double>(), q.as<double>(), a0,
                         G, (int64_t)C, groups, part.as<double>());
      dot_final(nrb0, pq);
      hipLaunchKernelGGL(pk_update, dim3(g0), dim3(256), 0, s, dr[0].as<double>(),
                         q.as<double>(), rz, pq, done, alpha, a0, G, (int64_t)C, groups,
                         part.as<double>());
      dot_final(nrb0, rr);
      hipLaunchKernelGGL(pk_converged, dim3((C + 255) / 256), dim3(256), 0, s, rr, bb, tol2, done,
                         (int64_t)C);
      PK_OR(hipGetLastError());
      if (it % kCheckEvery == 0 || it >= max_iter) {
        PK_OR(hipMemcpyAsync(h_rr.data(), rr, (size_t)C * 8, hipMemcpyDeviceToHost, s));
        PK_OR(hipStreamSynchronize(s));
        res = 0.0;
        all = true;
        for (int32_t c = 0; c < nb; ++c) {
          if (h_bb[c] > 0.0) res = fmax(res, sqrt(h_rr[c] / h_bb[c]));
          all = all && h_rr[c] <= tol2 * h_bb[c];
        }
        if (all || it >= max_iter) break;
      }
      precondition(rzn);
      hipLaunchKernelGGL(pk_direction, dim3(g0), dim3(256), 0, s, p.as<double>(), z.as<double>(),
                         x.as<double>(), alpha, rzn, rz, 0, a0, G, (int64_t)C, groups);
      PK_OR(hipGetLastError());
      double* t = rz;
      rz = rzn;
      rzn = t;
    }
    hipLaunchKernelGGL(pk_axpy, dim3(g0), dim3(256), 0, s, x.as<double>(), p.as<double>(), alpha,
                       a0, G, (int64_t)C, groups);
    float* o32 = P32 ? (green ? P32 + (int64_t)c0 * ld32 : P32 + c0) : nullptr;
    double* o64 = P64 ? (green ? P64 + (int64_t)c0 * ld64 : P64 + c0) : nullptr;
    hipLaunchKernelGGL(pk_write, dim3(g0), dim3(256), 0, s, x.as<double>(), a0, dil.as<int32_t>(),
                       G, (int64_t)C, groups, nb, o32, ld32, o64, ld64, green ? 1 : 0);
    PK_OR(hipGetLastError());
    st->batches += 1;
    if (!all) st->converged = 0;
    st->total_iterations += it;
    st->iterations = it > st->iterations ? it : st->iterations;
    st->max_rel_residual = fmax(st->max_rel_residual, res);
  }
  PK_OR(hipStreamSynchronize(s));   // the buffers are freed on return
  return hipSuccess;
}

hipError_t grid_poisson(int32_t G, const uint8_t* node_type, int32_t col_begin, int32_t ncols,
                        int32_t C, double tol, int32_t max_iter, float* P32, int64_t ld32,
                        double* P64, int64_t ld64, GridSolveStats* st, hipStream_t s) {
  return grid_solve(G, node_type, false, nullptr, col_begin, ncols, C, tol, max_iter, P32, ld32,
                    P64, ld64, st, s);
}

hipError_t grid_green(int32_t G, const uint8_t* node_type, const int32_t* poles, int32_t ncols,
                      int32_t C, double tol, int32_t max_iter, float* D32, int64_t ld32,
                      double* D64, int64_t ld64, GridSolveStats* st, hipStream_t s) {
  return grid_solve(G, node_type, true, poles, 0, ncols, C, tol, max_iter, D32, ld32, D64, ld64,
                    st, s);
}

}  // namespace dd
