// Triangle-based gradient-descent paths (Section IV, "Gradient-descent path
// generation", the second method; Fig. 2).
//
// The distance is linear on each triangle, so a triangle has one gradient g.
// From the source vertex the descent direction -g of an incident triangle that
// points into it is followed to the far edge; the path then enters the
// neighbouring triangle and follows its descent direction, and so on.
// Choices where the paper is silent:
//   * at a vertex: among incident triangles whose -g points strictly into
//     them, the largest |g| (ties: lowest triangle index); with none, the
//     incident edge with the largest decrease per unit length (ties: lowest
//     id) to its other end; with no decreasing edge the path is stuck; both
//     maxima are taken on squares, which order the same;
//   * on an edge: when the far triangle is missing or its -g does not point
//     into it, slide along the edge to the endpoint with the lower value
//     (ties: lowest id);
//   * an exit within a parameter distance kEps of a corner is that corner;
//   * an edge incident on the target, or the target itself, ends the path at
//     the target.
// Only triangles with three interior vertices are walkable.
//
// One wave per path.  The state is wave-uniform; at a vertex the incident
// triangles (one per lane) are evaluated in parallel.  Geometry is FP64 on
// the given field (an FP32 field upcast, or an FP64 field, on which every
// decision is the one the exact field takes up to the rounding of its sums),
// with contraction into FMA turned off so that every product and sum is
// rounded as written.
#include <math.h>

#include "dd_internal.h"

namespace dd {

namespace {

constexpr double kEps = 1e-9;

struct V2 {
  double x, y;
};

#pragma clang fp contract(off)

__device__ __forceinline__ double cross(V2 u, V2 v) { return u.x * v.y - u.y * v.x; }
__device__ __forceinline__ V2 sub(V2 a, V2 b) { return V2{a.x - b.x, a.y - b.y}; }

__device__ __forceinline__ V2 load_xy(const double* xy, int v) {
  return V2{xy[2 * (int64_t)v], xy[2 * (int64_t)v + 1]};
}

// Descent direction -g of the linear interpolant on triangle (i, j, k).
__device__ __forceinline__ V2 descent(V2 pi, V2 pj, V2 pk, double di, double dj, double dk) {
  const V2 e1 = sub(pj, pi), e2 = sub(pk, pi);
  const double a = dj - di, b = dk - di;
  const double det = cross(e1, e2);
  const V2 g{(a * e2.y - b * e1.y) / det, (b * e1.x - a * e2.x) / det};
  return V2{-g.x, -g.y};
}

// Parameter s of x + lam w = p + s (q - p); false when w is parallel to pq.
__device__ __forceinline__ bool segment_param(V2 x, V2 w, V2 p, V2 q, double& s) {
  const V2 r = sub(q, p);
  const double den = cross(w, r);
  if (den == 0.0) return false;
  s = cross(sub(p, x), w) / den;
  return true;
}

__device__ __forceinline__ double uni(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double lane_d(double x, int j) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, j);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), j);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

#pragma clang fp contract(on)

}  // namespace

#pragma clang fp contract(off)

template <typename F>
__global__ __launch_bounds__(64) void triangle_paths_kernel(TriArgs a, const F* fields) {
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const int N = a.N;
  const F* d = fields + (int64_t)i * N;
  double* pts = a.points + (int64_t)i * (a.max_steps + 1) * 2;
  int32_t* wh = a.where + (int64_t)i * (a.max_steps + 1) * 2;
  const int t = __builtin_amdgcn_readfirstlane(a.targets[i]);
  int v = __builtin_amdgcn_readfirstlane(a.sources[i]);
  // state: on a vertex (v), or inside edge (p, q) at point X, leaving face ff
  bool at_vertex = true;
  int p = -1, q = -1, ff = -1;
  V2 X = load_xy(a.xy, v);
  int len = 0;
  int status = 0;

  auto emit_vertex = [&](int u) {
    const V2 pu = load_xy(a.xy, u);
    if (lane == 0) {
      pts[2 * len] = pu.x;
      pts[2 * len + 1] = pu.y;
      wh[2 * len] = u;
      wh[2 * len + 1] = -1;
    }
    ++len;
    at_vertex = true;
    v = u;
    X = pu;
  };
  // point at parameter s on edge (e0, e1), leaving face from
  auto go_edge = [&](int e0, int e1, double s, int from) {
    if (s <= kEps) {
      emit_vertex(e0);
    } else if (s >= 1.0 - kEps) {
      emit_vertex(e1);
    } else if (e0 == t || e1 == t) {
      emit_vertex(t);
    } else {
      const V2 p0 = load_xy(a.xy, e0), p1 = load_xy(a.xy, e1);
      const V2 x{p0.x + s * (p1.x - p0.x), p0.y + s * (p1.y - p0.y)};
      if (lane == 0) {
        pts[2 * len] = x.x;
        pts[2 * len + 1] = x.y;
        wh[2 * len] = min(e0, e1);
        wh[2 * len + 1] = max(e0, e1);
      }
      ++len;
      at_vertex = false;
      p = e0;
      q = e1;
      ff = from;
      X = x;
    }
  };
  auto lower_end = [&](int e0, int e1) {
    const double d0 = (double)d[e0], d1 = (double)d[e1];
    return (d0 < d1 || (d0 == d1 && e0 < e1)) ? e0 : e1;
  };

  emit_vertex(v);
  for (;;) {
    v = __builtin_amdgcn_readfirstlane(v);
    len = __builtin_amdgcn_readfirstlane(len);
    if (at_vertex && v == t) {
      status = 0;
      break;
    }
    if (len - 1 >= a.max_steps) {
      status = 2;
      break;
    }
    if (at_vertex) {
      const V2 pv = load_xy(a.xy, v);
      const double dv = (double)d[v];
      // incident triangles, one per lane, in increasing index
      const int f = lane < a.vf_w ? a.vfaces[(int64_t)v * a.vf_w + lane] : -1;
      bool enters = false;
      double nrm = -1.0, sx = 0.0;
      int fa = -1, fb = -1;
      if (f >= 0) {
        const int4 rec = *reinterpret_cast<const int4*>(a.faces + 8 * (int64_t)f);
        const int r = rec.x == v ? 0 : (rec.y == v ? 1 : 2);
        const int c0 = r == 0 ? rec.y : (r == 1 ? rec.z : rec.x);
        const int c1 = r == 0 ? rec.z : (r == 1 ? rec.x : rec.y);
        const V2 pa = load_xy(a.xy, c0), pb = load_xy(a.xy, c1);
        const V2 P0 = load_xy(a.xy, rec.x), P1 = load_xy(a.xy, rec.y), P2 = load_xy(a.xy, rec.z);
        const V2 w = descent(P0, P1, P2, (double)d[rec.x], (double)d[rec.y], (double)d[rec.z]);
        if (cross(sub(pa, pv), w) > 0.0 && cross(w, sub(pb, pv)) > 0.0) {
          enters = true;
          nrm = w.x * w.x + w.y * w.y;   // |g|^2 orders as |g|
          double s = 0.0;
          segment_param(pv, w, pa, pb, s);
          sx = fmin(fmax(s, 0.0), 1.0);
          fa = c0;
          fb = c1;
        }
      }
      const uint64_t ent = __ballot(enters);
      if (ent) {
        int bj = -1;
        double bn = -1.0;
        for (uint64_t m = ent; m; m &= m - 1) {
          const int j = (int)__builtin_ctzll(m);
          const double nj = lane_d(nrm, j);
          if (nj > bn) {
            bn = nj;
            bj = j;
          }
        }
        const int e0 = __builtin_amdgcn_readlane(fa, bj), e1 = __builtin_amdgcn_readlane(fb, bj);
        const int bf = __builtin_amdgcn_readlane(f, bj);
        go_edge(e0, e1, lane_d(sx, bj), bf);
        continue;
      }
      // no triangle: the steepest decreasing incident edge
      const int u = lane < a.adj_w ? a.adj[(int64_t)v * a.adj_w + lane] : -1;
      double slope = -1.0;
      if (u >= 0) {
        const double du = (double)d[u];
        if (du < dv) {
          const V2 e = sub(load_xy(a.xy, u), pv);
          const double dd = dv - du;
          slope = dd * dd / (e.x * e.x + e.y * e.y);   // squared slope: same order
        }
      }
      const uint64_t dec = __ballot(slope > 0.0);
      if (!dec) {
        status = 1;
        break;
      }
      int bu = -1;
      double bs = 0.0;
      for (uint64_t m = dec; m; m &= m - 1) {
        const int j = (int)__builtin_ctzll(m);
        const double sj = lane_d(slope, j);
        const int uj = __builtin_amdgcn_readlane(u, j);
        if (sj > bs || (sj == bs && uj < bu)) {
          bs = sj;
          bu = uj;
        }
      }
      emit_vertex(bu);
      continue;
    }
    // inside edge (p, q), leaving face ff: the triangle on the far side
    const int4 rf = *reinterpret_cast<const int4*>(a.faces + 8 * (int64_t)ff);
    const int2 rn = *reinterpret_cast<const int2*>(a.faces + 8 * (int64_t)ff + 4);
    // neighbour across edge k of ff is (k == 0: rf.w, 1: rn.x, 2: rn.y)
    const int k0 = (rf.x == p || rf.x == q) + 0;
    const int k1 = (rf.y == p || rf.y == q);
    const int k2 = (rf.z == p || rf.z == q);
    const int ek = (k0 && k1) ? 0 : ((k1 && k2) ? 1 : 2);
    const int g = __builtin_amdgcn_readfirstlane(ek == 0 ? rf.w : (ek == 1 ? rn.x : rn.y));
    if (g < 0) {
      emit_vertex(lower_end(p, q));
      continue;
    }
    const int4 rg = *reinterpret_cast<const int4*>(a.faces + 8 * (int64_t)g);
    const int c = (rg.x != p && rg.x != q) ? rg.x : ((rg.y != p && rg.y != q) ? rg.y : rg.z);
    const V2 P0 = load_xy(a.xy, rg.x), P1 = load_xy(a.xy, rg.y), P2 = load_xy(a.xy, rg.z);
    V2 w = descent(P0, P1, P2, (double)d[rg.x], (double)d[rg.y], (double)d[rg.z]);
    w = V2{uni(w.x), uni(w.y)};
    const V2 pp = load_xy(a.xy, p), pq = load_xy(a.xy, q), pc = load_xy(a.xy, c);
    const double side_c = cross(sub(pq, pp), sub(pc, pp));
    if (!(cross(sub(pq, pp), w) * side_c > 0.0)) {
      emit_vertex(lower_end(p, q));
      continue;
    }
    const double turn = cross(sub(pc, X), w);
    if (turn == 0.0) {
      emit_vertex(c);
      continue;
    }
    const bool via_q = (turn < 0.0) == (side_c > 0.0);
    const int e0 = via_q ? q : p;
    double s = 0.0;
    if (!segment_param(X, w, via_q ? pq : pp, pc, s)) {
      emit_vertex(c);
      continue;
    }
    go_edge(e0, c, fmin(fmax(s, 0.0), 1.0), g);
  }
  for (int k = len + lane; k <= a.max_steps; k += 64) {
    pts[2 * k] = 0.0;
    pts[2 * k + 1] = 0.0;
    wh[2 * k] = -1;
    wh[2 * k + 1] = -1;
  }
  if (lane == 0) {
    a.len[i] = len;
    a.status[i] = status;
  }
}

#pragma clang fp contract(on)

hipError_t launch_triangle_paths(TriArgs a, hipStream_t s) {
  if (a.fields64)
    hipLaunchKernelGGL(triangle_paths_kernel<double>, dim3(a.T), dim3(64), 0, s, a, a.fields64);
  else
    hipLaunchKernelGGL(triangle_paths_kernel<float>, dim3(a.T), dim3(64), 0, s, a, a.fields);
  return hipGetLastError();
}

}  // namespace dd
