// Edge-based steepest-descent paths (Section IV, "Gradient-descent path
// generation"): from the current vertex move to the neighbour with the
// smallest distance (ties: lowest id) while it is strictly below the current
// vertex; stop at the target, at a vertex with no strictly lower neighbour,
// or after max_steps moves.
//
// The walk is a chain of dependent steps, so its cost is memory latency per
// step.  A parallel gather first lays out, for every vertex, the field values
// of its neighbour slots next to each other (nv[v][j] = d(adj[v][j])); a step
// then needs one round of independent loads (ids and values of the current
// vertex's row) before the cross-lane argmin.  One wavefront per path.
//
// Each decision is checked against the field's stated error bound: when two
// neighbours (or the best neighbour and the current vertex) cannot be told
// apart within the bound, their distances are recomputed in FP64 from the
// resident master rows and the decision is taken on those.
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

// Truncated target rows in FP64 (stored entries scattered into a dense row)
// and constants W = sum p, H = sum p ln p, |S| over the stored entries.
__global__ __launch_bounds__(256) void target_rows_kernel(CsrView cv, PathArgs a, double* trow,
                                                          double* tconst) {
  const int t = path_target(a, blockIdx.x);
  const int B = cv.B;
  double* out = trow + (int64_t)blockIdx.x * B;
  __shared__ double red[3][8];
  for (int b = threadIdx.x; b < B; b += blockDim.x) out[b] = 0.0;
  __syncthreads();
  const int64_t s = cv.start[t];
  const int n = cv.len[t];
  double w = 0.0, h = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double p = cv.val64 ? cv.val64[s + i] : (double)cv.val[s + i];
    out[cv.col[s + i]] = p;
    w += p;
    h += p * log(p);
    c += 1.0;
  }
  w = wsum(w);
  h = wsum(h);
  c = wsum(c);
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wid] = w;
    red[1][wid] = h;
    red[2][wid] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double W = 0.0, H = 0.0, C = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      W += red[0][i];
      H += red[1][i];
      C += red[2][i];
    }
    tconst[blockIdx.x * 4 + 0] = W;
    tconst[blockIdx.x * 4 + 1] = H;
    tconst[blockIdx.x * 4 + 2] = C;
    tconst[blockIdx.x * 4 + 3] = 0.0;
  }
}

__global__ __launch_bounds__(256) void neighbor_values_kernel(PathArgs a, int32_t N, float* nv) {
  const int64_t per = (int64_t)N * a.adj_w;
  const int64_t total = per * a.T;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / per;
    const int32_t u = a.adj[idx - i * per];
    nv[idx] = u >= 0 ? a.fields[i * N + u] : __builtin_inff();
  }
}

// FP64 distance of row x to the target (whole wave cooperates).  Dense
// handles read the target row from the master; truncated handles use the
// staged FP64 target row and its constants.
__device__ double exact_distance(const DenseView& dv, const CsrView& cv, int is_csr, int kind,
                                 int t, const double* p, const double* tc, int x) {
  const int lane = threadIdx.x & 63;
  if (!is_csr) {
    double acc = 0.0;
    for (int b = lane; b < dv.B; b += 64) {
      double q, pb;
      if (dv.P64) {
        q = dv.P64[(int64_t)x * dv.B + b];
        pb = dv.P64[(int64_t)t * dv.B + b];
      } else {
        q = (double)dv.P[(int64_t)x * dv.ld + b];
        pb = (double)dv.P[(int64_t)t * dv.ld + b];
      }
      if (kind == 0) {
        acc += fabs(pb - q);
      } else if (pb > 0.0) {
        acc += pb * log(pb / q);
      }
    }
    return wsum(acc);
  }
  const int64_t s = cv.start[x];
  const int n = cv.len[x];
  double acc = 0.0, A = 0.0, E = 0.0, c = 0.0;
  for (int i = lane; i < n; i += 64) {
    const double q = cv.val64 ? cv.val64[s + i] : (double)cv.val[s + i];
    const double pb = p[cv.col[s + i]];
    A += pb;
    if (kind == 0) {
      acc += fabs(q - pb);
    } else if (pb > 0.0) {
      acc += pb * log(pb / q);
      E += pb * log(pb);
    }
    c += pb > 0.0 ? 1.0 : 0.0;
  }
  acc = wsum(acc);
  A = wsum(A);
  E = wsum(E);
  c = wsum(c);
  if (c == tc[2]) return acc;
  if (kind == 0) return acc + (tc[0] - A);
  return acc + (tc[1] - E) - log(cv.phi[x]) * (tc[0] - A);
}

__global__ __launch_bounds__(64) void paths_kernel(DenseView dv, CsrView cv, PathArgs a) {
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const int N = a.is_csr ? cv.N : dv.N;
  const int W = a.adj_w;
  const float* d = a.fields + (int64_t)i * N;
  const float* nvi = a.nv + (int64_t)i * N * W;
  const Bound bnd = path_bound(a, i);
  const double ea = bnd.abs, er = bnd.rel;
  const double* p = a.is_csr ? a.trow + (int64_t)i * cv.B : nullptr;
  const double* tc = a.is_csr ? a.tconst + (int64_t)i * 4 : nullptr;
  int32_t* path = a.path + (int64_t)i * (a.max_steps + 1);
  const int t = path_target(a, i);
  int v = path_source(a, i);
  float cur = d[v];   // FP32 field value at v
  int len = 1;
  int status = 0;
  int rechecks = 0;
  if (lane == 0) path[0] = v;
  for (;;) {
    if (v == t) {
      status = 0;
      break;
    }
    if (len - 1 >= a.max_steps) {
      status = 2;
      break;
    }
    // one round of independent loads: neighbour ids and their field values
    int u = -1;
    float val = __builtin_inff();
    if (lane < W) {
      u = a.adj[(int64_t)v * W + lane];
      val = nvi[(int64_t)v * W + lane];
    }
    const bool valid = u >= 0;
    if (__ballot(valid) == 0ull) {
      status = 1;
      break;
    }
    const double e = valid ? ea + er * fabs((double)val) : 0.0;
    const double hi = valid ? (double)val + e : __builtin_inf();
    const double lo = valid ? (double)val - e : __builtin_inf();
    // lexicographic argmin of (val, u) and the smallest upper end
    float bv = val;
    int bu = valid ? u : 0x7fffffff;
    double mh = hi;
    for (int off = 32; off > 0; off >>= 1) {
      const float ov = __shfl_xor(bv, off);
      const int ou = __shfl_xor(bu, off);
      if (ov < bv || (ov == bv && ou < bu)) {
        bv = ov;
        bu = ou;
      }
      mh = fmin(mh, __shfl_xor(mh, off));
    }
    const bool cand = valid && lo <= mh;
    const unsigned long long cm = __ballot(cand);
    const int nc = __popcll(cm);
    const double dvv = (double)cur;
    const double evv = ea + er * fabs(dvv);
    const double eb = ea + er * fabs((double)bv);
    int next = bu;
    bool stuck;
    if (nc == 1 && ((double)bv + eb < dvv - evv)) {
      stuck = false;
    } else if (nc == 1 && ((double)bv - eb >= dvv + evv)) {
      stuck = true;
    } else {
      ++rechecks;
      const double dxv = exact_distance(dv, cv, a.is_csr, a.kind, t, p, tc, v);
      double best = __builtin_inf();
      int best_u = 0x7fffffff;
      unsigned long long m = cm;
      while (m) {
        const int l = __ffsll((long long)m) - 1;
        m &= m - 1;
        const int cu = __shfl(u, l);
        const double dx = exact_distance(dv, cv, a.is_csr, a.kind, t, p, tc, cu);
        if (dx < best || (dx == best && cu < best_u)) {
          best = dx;
          best_u = cu;
        }
      }
      next = best_u;
      stuck = !(best < dxv);
    }
    if (stuck) {
      status = 1;
      break;
    }
    const unsigned long long at = __ballot(valid && u == next);
    cur = __shfl(val, __ffsll((long long)at) - 1);
    v = next;
    if (lane == 0) path[len] = v;
    ++len;
  }
  for (int k = len + lane; k <= a.max_steps; k += 64) path[k] = -1;
  if (lane == 0) {
    a.len[i] = len;
    a.status[i] = status;
    if (a.rechecks) a.rechecks[i] = rechecks;
  }
}

hipError_t launch_target_rows(CsrView cv, PathArgs a, double* trow, double* tconst,
                              hipStream_t s) {
  hipLaunchKernelGGL(target_rows_kernel, dim3(a.T), dim3(256), 0, s, cv, a, trow, tconst);
  return hipGetLastError();
}

hipError_t launch_neighbor_values(PathArgs a, int32_t N, float* nv, hipStream_t s) {
  const int64_t total = (int64_t)N * a.adj_w * a.T;
  int64_t grid = (total + 255) / 256;
  const int64_t cap = (int64_t)num_cus() * 8;
  if (grid > cap) grid = cap;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(neighbor_values_kernel, dim3((unsigned)grid), dim3(256), 0, s, a, N, nv);
  return hipGetLastError();
}

hipError_t launch_paths(DenseView dv, CsrView cv, PathArgs a, hipStream_t s) {
  hipLaunchKernelGGL(paths_kernel, dim3(a.T), dim3(64), 0, s, dv, cv, a);
  return hipGetLastError();
}

}  // namespace dd
