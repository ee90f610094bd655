"""Triangle-based gradient-descent paths (Section IV, "Gradient-descent path
generation", the second method; Fig. 2).

Test infrastructure: plain FP64 Python, written from the paper's description;
it shares nothing with the library.

The distance is linear on each triangle (it interpolates the three vertex
values), so every triangle has one gradient g.  From the source vertex the
descent direction -g of an incident triangle that points into that triangle
is followed across it; at the far edge the path enters the neighbouring
triangle and follows that triangle's descent direction, and so on.  Readings
where the paper is silent (listed with the others in the design notes):

* at a vertex, among the incident triangles whose descent direction points
  strictly into the triangle, the one with the largest |g| is followed (ties:
  lowest triangle index; |g| is compared through |g|^2).  With none, the path
  moves along the incident edge with the largest decrease per unit length
  (compared through its square) to its other end (ties: lowest vertex id), and
  stops (STUCK) when no incident edge decreases;
* on an edge, when the triangle on the far side does not exist or its descent
  direction does not point into it, the path slides along the edge to the
  endpoint with the lower value (ties: lowest id);
* an exit within a parameter distance EPS of a triangle corner is that corner;
* reaching an edge incident on the target, or the target itself, ends the path
  at the target (REACHED); MAX_STEPS after ``max_steps`` points.

Only triangles with three interior vertices (vertices that carry a distance
value) take part.  Triangles are oriented counter-clockwise here.

A path is a list of points and, for each point, where it lies: (v, -1) for
vertex v, (a, b) with a < b for a point inside edge ab.
"""

import numpy as np

REACHED, STUCK, MAX_STEPS = 0, 1, 2
EPS = 1e-9


def cross(u, v):
    return u[0] * v[1] - u[1] * v[0]


class Mesh:
    """Interior-only triangulation: faces [F, 3] of vertex ids, xy [N, 2]."""

    def __init__(self, faces, xy):
        self.xy = np.asarray(xy, dtype=np.float64)
        faces = np.asarray(faces, dtype=np.int64).copy()
        for f in range(len(faces)):
            a, b, c = faces[f]
            if cross(self.xy[b] - self.xy[a], self.xy[c] - self.xy[a]) < 0:
                faces[f, 1], faces[f, 2] = c, b
        self.faces = faces
        self.edge_faces = {}
        self.vertex_faces = [[] for _ in range(len(self.xy))]
        for f, (a, b, c) in enumerate(faces):
            for p, q in ((a, b), (b, c), (c, a)):
                self.edge_faces.setdefault((min(p, q), max(p, q)), []).append(f)
            for v in (a, b, c):
                self.vertex_faces[v].append(f)

    def other_face(self, p, q, f):
        for g in self.edge_faces[(min(p, q), max(p, q))]:
            if g != f:
                return g
        return -1

    def gradient(self, f, d):
        i, j, k = self.faces[f]
        e1 = self.xy[j] - self.xy[i]
        e2 = self.xy[k] - self.xy[i]
        dj = d[j] - d[i]
        dk = d[k] - d[i]
        det = cross(e1, e2)
        return np.array([(dj * e2[1] - dk * e1[1]) / det, (dk * e1[0] - dj * e2[0]) / det])


def segment_hit(x, w, p, q):
    """(lam, s) with x + lam w = p + s (q - p), or None if parallel."""
    r = q - p
    den = cross(w, r)
    if den == 0.0:
        return None
    return cross(p - x, r) / den, cross(p - x, w) / den


def triangle_path(mesh, d, adj_ptr, adj_idx, source, target, max_steps):
    """(points [k, 2], where [(a, b)], status) of the triangle-based walk on d."""
    d = np.asarray(d, dtype=np.float64)
    xy = mesh.xy
    pts = [xy[source].copy()]
    where = [(int(source), -1)]
    state = ("v", int(source))

    def push_vertex(v):
        pts.append(xy[v].copy())
        where.append((int(v), -1))
        return ("v", int(v))

    def lower_end(a, b):
        if d[a] < d[b] or (d[a] == d[b] and a < b):
            return a
        return b

    def go_edge(p, q, s, f_from):
        """Point at parameter s on edge pq, leaving face f_from."""
        if s <= EPS:
            return push_vertex(p)
        if s >= 1.0 - EPS:
            return push_vertex(q)
        if p == target or q == target:
            return push_vertex(target)
        pts.append(xy[p] + s * (xy[q] - xy[p]))
        where.append((int(min(p, q)), int(max(p, q))))
        return ("e", int(p), int(q), f_from)

    while True:
        if state[0] == "v" and state[1] == target:
            return np.array(pts), where, REACHED
        if len(pts) - 1 >= max_steps:
            return np.array(pts), where, MAX_STEPS
        if state[0] == "v":
            v = state[1]
            best, best_norm = -1, -1.0
            for f in sorted(mesh.vertex_faces[v]):
                fa = list(mesh.faces[f])
                r = fa.index(v)
                a, b = fa[(r + 1) % 3], fa[(r + 2) % 3]
                w = -mesh.gradient(f, d)
                if cross(xy[a] - xy[v], w) > 0 and cross(w, xy[b] - xy[v]) > 0:
                    n = w[0] * w[0] + w[1] * w[1]      # |g|^2 orders as |g|
                    if n > best_norm:
                        best, best_norm = f, n
            if best >= 0:
                fa = list(mesh.faces[best])
                r = fa.index(v)
                a, b = fa[(r + 1) % 3], fa[(r + 2) % 3]
                w = -mesh.gradient(best, d)
                hit = segment_hit(xy[v], w, xy[a], xy[b])
                s = min(max(hit[1], 0.0), 1.0)
                state = go_edge(a, b, s, best)
                continue
            # edge fallback: steepest decreasing incident edge
            bu, bslope = -1, 0.0
            for u in adj_idx[adj_ptr[v]:adj_ptr[v + 1]]:
                u = int(u)
                if not d[u] < d[v]:
                    continue
                e = xy[u] - xy[v]
                dd = d[v] - d[u]
                slope = dd * dd / (e[0] * e[0] + e[1] * e[1])   # squared: same order
                if slope > bslope or (slope == bslope and bu >= 0 and u < bu):
                    bu, bslope = u, slope
            if bu < 0:
                return np.array(pts), where, STUCK
            state = push_vertex(bu)
            continue
        # on edge pq, arriving from face f_from
        _, p, q, f_from = state
        g = mesh.other_face(p, q, f_from)
        x = pts[-1]
        if g < 0:
            state = push_vertex(lower_end(p, q))
            continue
        fa = list(mesh.faces[g])
        c = [v for v in fa if v != p and v != q][0]
        w = -mesh.gradient(g, d)
        side_c = cross(xy[q] - xy[p], xy[c] - xy[p])
        if not cross(xy[q] - xy[p], w) * side_c > 0:
            state = push_vertex(lower_end(p, q))
            continue
        # exit through (p, c) or (c, q): decided by the side of c the ray passes
        turn = cross(xy[c] - x, w)
        if turn == 0.0:
            state = push_vertex(c)
            continue
        # with pq oriented so that c is on the left, a clockwise turn from
        # x->c exits through the edge at q's end
        left = side_c > 0
        via_q = (turn < 0) == left
        e0, e1 = (q, c) if via_q else (p, c)
        hit = segment_hit(x, w, xy[e0], xy[e1])
        if hit is None:
            state = push_vertex(c)
            continue
        s = min(max(hit[1], 0.0), 1.0)
        state = go_edge(e0, e1, s, g)
