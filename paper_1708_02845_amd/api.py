"""Python face of libdd: argument marshalling over the C ABI.

PyTorch supplies device memory (output tensors) and streams; every step of the
computation runs in the library's HIP kernels.  There is no CPU fallback: the
calls raise if the library is missing or the device is unavailable.
"""

import ctypes as C

import numpy as np

from . import _lib as L

KINDS = {"tv": L.DD_TV, "kl": L.DD_KL, "chi2": L.DD_CHI2, "hellinger": L.DD_HELLINGER}
KINDS.update({v: v for v in list(KINDS.values())})
FORMS = {None: L.DD_FORM_NONE, "none": L.DD_FORM_NONE, "f32": L.DD_FORM_F32,
         "f16x3": L.DD_FORM_F16X3, "bf16x3": L.DD_FORM_BF16X3, "f16": L.DD_FORM_F16}
CSR_VALUES = {"f32": L.DD_CSR_F32, "f16": L.DD_CSR_F16}
PATH_STATUS = {L.DD_PATH_REACHED: "reached", L.DD_PATH_STUCK: "stuck",
               L.DD_PATH_MAX_STEPS: "max_steps"}


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _kind(kind):
    """Kind value of a name ("tv", "kl", "chi2", "hellinger"), a family tuple
    ("power", k) with integer 1 <= k <= 16 or ("alpha", a) with a = m/8,
    |m| <= 7, or a kind value."""
    if isinstance(kind, tuple) and len(kind) == 2:
        fam, val = kind
        if fam == "power" and float(val).is_integer() and 1 <= int(val) <= 16:
            return 100 + int(val)
        if fam == "alpha" and float(val * 8).is_integer() and -7 <= int(val * 8) <= 7:
            return 208 + int(val * 8)
        raise ValueError(f"unsupported family member {kind!r}")
    try:
        return KINDS[kind.lower() if isinstance(kind, str) else kind]
    except (KeyError, TypeError):
        if isinstance(kind, int) and not isinstance(kind, bool):
            return kind      # a kind value; the library validates it
        raise ValueError(f"unknown kind {kind!r}") from None


def _adjacency(adj, n):
    """(struct, keep-alive arrays) from an (row_ptr, col) pair or None."""
    if adj is None:
        return None, ()
    ptr = np.ascontiguousarray(adj[0], dtype=np.int64)
    col = np.ascontiguousarray(adj[1], dtype=np.int32)
    s = L.dd_adjacency(int(n), ptr.ctypes.data_as(C.POINTER(C.c_int64)),
                       col.ctypes.data_as(C.POINTER(C.c_int32)))
    return s, (ptr, col)


def bound_tuple(b):
    return (b.abs, b.rel)


class Context:
    """A library context bound to one HIP device."""

    def __init__(self, device=0):
        self._lib = L.load()
        self.device = int(device)
        h = C.c_void_p()
        L.check(self._lib.dd_create(self.device, C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            L.check(self._lib.dd_destroy(self._h))
            self._h = None

    def path_level1(self, enable=None):
        """(enabled, (ratio to the assumed bound, max relative error)) of the
        level-1 re-decisions of KL walks; ``enable`` True/False switches them."""
        on = C.c_int()
        r = (C.c_double * 2)()
        L.check(self._lib.dd_path_level1(self._h, -1 if enable is None else int(bool(enable)),
                                         C.byref(on), r))
        return bool(on.value), (r[0], r[1])

    def grid_poisson_kernel(self, node_type, cols=None, tol=1e-12, max_iter=1000, batch=0,
                            dtype="f32", out=None, stream=None):
        """Poisson kernel P_IB of a grid domain, computed on the device.

        node_type: [G, G] or [G*G] uint8 (0 outside, 1 interior, 2 boundary;
        vertex (i, j) at j*G + i).  cols: (begin, count) of the boundary
        columns to compute (all by default).  dtype "f32" or "f64".  out:
        optional device tensor [N, >= count] of that dtype.  Returns
        (P tensor [N, count] view, stats dict)."""
        torch = _torch()
        nt = np.ascontiguousarray(np.asarray(node_type, dtype=np.uint8).reshape(-1))
        G = int(round(len(nt) ** 0.5))
        if G * G != len(nt):
            raise ValueError("node_type is not a square grid")
        N = int((nt == 1).sum())
        K = int((nt == 2).sum())
        begin, count = (0, K) if cols is None else (int(cols[0]), int(cols[1]))
        tdt = {"f32": torch.float32, "f64": torch.float64}[dtype]
        if out is None:
            out = torch.empty((N, max(count, 1)), dtype=tdt, device=f"cuda:{self.device}")
        if out.dtype != tdt or out.dim() != 2 or out.shape[0] != N or out.stride(1) != 1:
            raise ValueError("out must be a row-major [N, >= count] tensor of the dtype")
        st = L.dd_grid_solve_stats()
        ptr = C.c_void_p(out.data_ptr())
        ld = out.stride(0)
        L.check(self._lib.dd_grid_poisson_kernel(
            self._h, G, nt.ctypes.data_as(C.c_void_p), begin, count,
            ptr if dtype == "f32" else None, ld if dtype == "f32" else 0,
            ptr if dtype == "f64" else None, ld if dtype == "f64" else 0,
            float(tol), int(max_iter), int(batch), C.byref(st), _stream_handle(stream)))
        stats = {"iterations": st.iterations, "batches": st.batches, "levels": st.levels,
                 "total_iterations": st.total_iterations,
                 "max_rel_residual": st.max_rel_residual}
        return out[:, :count], stats


    def grid_green_function(self, node_type, poles, tol=1e-12, max_iter=1000, batch=0,
                            dtype="f32", out=None, stream=None):
        """Dirichlet Green's functions D_Ip = (-L_II)^{-1} e_p of a grid domain for
        the interior vertices p in ``poles``, computed on the device.  Returns
        (D tensor [T, N] of the dtype, one field per pole, stats dict)."""
        torch = _torch()
        nt = np.ascontiguousarray(np.asarray(node_type, dtype=np.uint8).reshape(-1))
        G = int(round(len(nt) ** 0.5))
        if G * G != len(nt):
            raise ValueError("node_type is not a square grid")
        N = int((nt == 1).sum())
        pl = np.ascontiguousarray(poles, dtype=np.int32)
        T = len(pl)
        tdt = {"f32": torch.float32, "f64": torch.float64}[dtype]
        if out is None:
            out = torch.empty((T, N), dtype=tdt, device=f"cuda:{self.device}")
        if out.dtype != tdt or out.dim() != 2 or out.shape[0] != T or out.shape[1] < N \
                or out.stride(1) != 1:
            raise ValueError("out must be a row-major [T, >= N] tensor of the dtype")
        st = L.dd_grid_solve_stats()
        ptr = C.c_void_p(out.data_ptr())
        ld = out.stride(0)
        L.check(self._lib.dd_grid_green_function(
            self._h, G, nt.ctypes.data_as(C.c_void_p), C.c_void_p(pl.ctypes.data), T,
            ptr if dtype == "f32" else None, ld if dtype == "f32" else 0,
            ptr if dtype == "f64" else None, ld if dtype == "f64" else 0,
            float(tol), int(max_iter), int(batch), C.byref(st), _stream_handle(stream)))
        stats = {"iterations": st.iterations, "batches": st.batches, "levels": st.levels,
                 "total_iterations": st.total_iterations,
                 "max_rel_residual": st.max_rel_residual}
        return out[:, :N], stats


class Kernel:
    """A resident Poisson-kernel matrix (dense or truncated) on the device."""

    def __init__(self, ctx, handle):
        self.ctx = ctx
        self._lib = ctx._lib
        self._h = handle
        info = L.dd_kernel_info()
        L.check(self._lib.dd_kernel_get_info(self._h, C.byref(info)))
        self.N, self.B_in, self.B = info.n, info.b_in, info.b
        self.is_csr = bool(info.is_csr)
        self.nnz = info.nnz
        self.gemm_form = info.gemm_form
        self.has_adjacency = bool(info.has_adjacency)
        self.hbm_bytes = info.hbm_bytes
        self.csr_values = {0: "f32", 1: "f16"}[info.csr_values] if self.is_csr else None

    # ---- loading ----
    @classmethod
    def load_dense(cls, ctx, P, adjacency=None, gemm_form=None, tau=0.0, tau_relative=True,
                   validate=True, csr_values="f32"):
        """Load an N x B matrix given as a numpy array or a torch tensor (any device).
        With tau > 0 the handle keeps the truncation, its values read as FP32 or,
        with csr_values="f16", as FP16 scaled per row.  gemm_form ("f32", "f16x3",
        "bf16x3", "f16") builds the batched-KL contraction operand; with tau > 0 it is
        the floored log-kernel, and KL_tau of many targets runs as one
        contraction (FP32 values only)."""
        torch = _torch()
        keep = []
        if isinstance(P, np.ndarray):
            arr = np.ascontiguousarray(P)
            if arr.dtype not in (np.float32, np.float64):
                raise TypeError("P must be float32 or float64")
            ptr, on_dev, f64 = arr.ctypes.data, 0, int(arr.dtype == np.float64)
            keep.append(arr)
            N, B = arr.shape
        else:
            t = P.contiguous()
            if t.dtype not in (torch.float32, torch.float64):
                raise TypeError("P must be float32 or float64")
            ptr, on_dev, f64 = t.data_ptr(), int(t.is_cuda), int(t.dtype == torch.float64)
            keep.append(t)
            N, B = t.shape
        adj, adj_keep = _adjacency(adjacency, N)
        opts = L.dd_load_opts(FORMS[gemm_form], float(tau), int(bool(tau_relative)),
                              int(bool(validate)), CSR_VALUES[csr_values])
        h = C.c_void_p()
        L.check(ctx._lib.dd_load_kernel_dense(ctx.handle, int(N), int(B), C.c_void_p(ptr), f64,
                                              on_dev, C.byref(adj) if adj else None,
                                              C.byref(opts), C.byref(h)))
        del keep, adj_keep
        return cls(ctx, h)

    @classmethod
    def load_csr(cls, ctx, N, B, row_ptr, col, val, row_max, tau, tau_relative=True,
                 adjacency=None, csr_values="f32"):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        vl = np.ascontiguousarray(val)
        if vl.dtype not in (np.float32, np.float64):
            vl = vl.astype(np.float64)
        rm = np.ascontiguousarray(row_max, dtype=np.float64)
        adj, adj_keep = _adjacency(adjacency, N)
        h = C.c_void_p()
        opts = L.dd_load_opts(L.DD_FORM_NONE, 0.0, 1, 1, CSR_VALUES[csr_values])
        L.check(ctx._lib.dd_load_kernel_csr(
            ctx.handle, int(N), int(B), C.c_void_p(rp.ctypes.data), C.c_void_p(cl.ctypes.data),
            C.c_void_p(vl.ctypes.data), int(vl.dtype == np.float64), C.c_void_p(rm.ctypes.data),
            float(tau), int(bool(tau_relative)), C.byref(adj) if adj else None, C.byref(opts),
            C.byref(h)))
        del adj_keep
        return cls(ctx, h)

    @staticmethod
    def dense_footprint(N, B, f64=False, gemm_form=None):
        lib = L.load()
        opts = L.dd_load_opts(FORMS[gemm_form], 0.0, 1, 1, 0)
        out = C.c_size_t()
        L.check(lib.dd_dense_footprint(int(N), int(B), int(bool(f64)), C.byref(opts), C.byref(out)))
        return out.value

    def footprint(self):
        """Device bytes resident in the handle."""
        out = C.c_size_t()
        L.check(self._lib.dd_kernel_footprint(self._h, C.byref(out)))
        return out.value

    def call_scratch(self, T, kind="kl"):
        """(batch_fields scratch bytes, trace_paths scratch bytes) of calls with T
        targets / paths: device memory a launch allocates beyond its outputs."""
        fb, pb = C.c_size_t(), C.c_size_t()
        L.check(self._lib.dd_call_scratch_bytes(self._h, int(T), _kind(kind), C.byref(fb),
                                                C.byref(pb)))
        return fb.value, pb.value

    def free(self):
        if self._h:
            L.check(self._lib.dd_free_kernel(self._h))
            self._h = None

    @property
    def handle(self):
        return self._h

    # ---- fields ----
    def _out(self, shape, out):
        torch = _torch()
        if out is None:
            return torch.empty(shape, dtype=torch.float32, device=f"cuda:{self.ctx.device}")
        if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous() \
                or out.numel() < int(np.prod(shape)):
            raise ValueError("out must be a contiguous float32 CUDA tensor of the right size")
        return out

    def field(self, target, kind, out=None, stream=None):
        """(field tensor [N], (abs, rel) error bound) for one target."""
        out = self._out((self.N,), out)
        b = L.dd_error_bound()
        L.check(self._lib.dd_distance_field(self._h, int(target), _kind(kind),
                                            C.c_void_p(out.data_ptr()), C.byref(b),
                                            _stream_handle(stream)))
        return out, bound_tuple(b)

    def fields_tv_kl(self, target, out=None, stream=None):
        """(fields [2, N]: TV then KL, [(abs, rel) of TV, of KL]) of one target
        from one pass over the rows."""
        out = self._out((2, self.N), out)
        b = (L.dd_error_bound * 2)()
        L.check(self._lib.dd_distance_fields_tv_kl(
            self._h, int(target), C.c_void_p(out[0].data_ptr()), C.c_void_p(out[1].data_ptr()), b,
            _stream_handle(stream)))
        return out, [bound_tuple(b[0]), bound_tuple(b[1])]

    def batch_fields(self, targets, kind, out=None, stream=None):
        """(fields [T, N], list of (abs, rel) bounds) for T targets: KL through the
        contraction when the handle has an operand, the pass over the stored rows
        on a truncated handle from 8 targets, else one streaming pass each."""
        return self._batch(self._lib.dd_batch_distance_fields, targets, kind, out, stream)

    def batch_fields_noalloc(self, targets, kind, out=None, stream=None):
        """batch_fields with the library's fixed per-GPU scratch instead of
        per-call device allocations (pass ``out`` to allocate nothing at all).
        Calls on one GPU must not overlap."""
        return self._batch(self._lib.dd_batch_distance_fields_noalloc, targets, kind, out, stream)

    def _batch(self, fn, targets, kind, out, stream):
        t = np.ascontiguousarray(targets, dtype=np.int32)
        T = len(t)
        out = self._out((T, self.N), out)
        bounds = (L.dd_error_bound * max(T, 1))()
        L.check(fn(self._h, C.c_void_p(t.ctypes.data), int(T), _kind(kind),
                   C.c_void_p(out.data_ptr()), bounds, _stream_handle(stream)))
        return out, [bound_tuple(bounds[i]) for i in range(T)]

    # ---- paths ----
    def trace_paths(self, sources, targets, kind, fields, bounds, max_steps, stream=None):
        """Device tensors (paths [T, max_steps+1], len [T], status [T], rechecks [T])."""
        torch = _torch()
        s = np.ascontiguousarray(sources, dtype=np.int32)
        t = np.ascontiguousarray(targets, dtype=np.int32)
        T = len(s)
        dev = f"cuda:{self.ctx.device}"
        paths = torch.empty((T, max_steps + 1), dtype=torch.int32, device=dev)
        info = torch.empty((3, T), dtype=torch.int32, device=dev)
        b = (L.dd_error_bound * T)(*[L.dd_error_bound(a, r) for a, r in bounds])
        if not fields.is_contiguous() or fields.dtype != torch.float32:
            raise ValueError("fields must be contiguous float32")
        L.check(self._lib.dd_trace_paths(self._h, int(T), C.c_void_p(s.ctypes.data),
                                         C.c_void_p(t.ctypes.data), _kind(kind),
                                         C.c_void_p(fields.data_ptr()), b, int(max_steps),
                                         C.c_void_p(paths.data_ptr()),
                                         C.c_void_p(info[0].data_ptr()),
                                         C.c_void_p(info[1].data_ptr()),
                                         C.c_void_p(info[2].data_ptr()), _stream_handle(stream)))
        return paths, info[0], info[1], info[2]

    def trace_paths_on_demand(self, sources, targets, kind, max_steps, target_tau=0.0,
                              target_tau_relative=True, stream=None):
        """Device tensors (paths [T, max_steps+1], len [T], status [T], evaluations [T])
        of walks that evaluate FP64 distances only where the path needs them."""
        torch = _torch()
        s = np.ascontiguousarray(sources, dtype=np.int32)
        t = np.ascontiguousarray(targets, dtype=np.int32)
        T = len(s)
        dev = f"cuda:{self.ctx.device}"
        paths = torch.empty((T, max_steps + 1), dtype=torch.int32, device=dev)
        info = torch.empty((3, T), dtype=torch.int32, device=dev)
        L.check(self._lib.dd_trace_paths_on_demand(
            self._h, int(T), C.c_void_p(s.ctypes.data), C.c_void_p(t.ctypes.data), _kind(kind),
            float(target_tau), int(bool(target_tau_relative)), int(max_steps),
            C.c_void_p(paths.data_ptr()), C.c_void_p(info[0].data_ptr()),
            C.c_void_p(info[1].data_ptr()), C.c_void_p(info[2].data_ptr()),
            _stream_handle(stream)))
        return paths, info[0], info[1], info[2]

    def support_kl_field(self, target, tau, relative=True, out=None, stream=None):
        """(field [N], bound) of KL summed over the truncated target support."""
        out = self._out((self.N,), out)
        b = L.dd_error_bound()
        L.check(self._lib.dd_support_kl_field(self._h, int(target), float(tau), int(bool(relative)),
                                              C.c_void_p(out.data_ptr()), C.byref(b),
                                              _stream_handle(stream)))
        return out, bound_tuple(b)

    def attach_mesh(self, faces, xy):
        """Triangle mesh of the interior: faces [F, 3] interior-local ids, xy [N, 2]."""
        f = np.ascontiguousarray(faces, dtype=np.int32)
        c = np.ascontiguousarray(xy, dtype=np.float64)
        if f.ndim != 2 or f.shape[1] != 3 or c.shape != (self.N, 2):
            raise ValueError("faces must be [F, 3] and xy [N, 2]")
        L.check(self._lib.dd_attach_mesh(self._h, int(f.shape[0]), C.c_void_p(f.ctypes.data),
                                         C.c_void_p(c.ctypes.data)))

    def exact_fields(self, targets, kind, out=None, stream=None):
        """FP64 fields [T, N] of T targets, every term and sum in FP64."""
        torch = _torch()
        t = np.ascontiguousarray(targets, dtype=np.int32)
        T = len(t)
        if out is None:
            out = torch.empty((T, self.N), dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        if out.dtype != torch.float64 or not out.is_contiguous() or out.numel() < T * self.N:
            raise ValueError("out must be a contiguous float64 tensor of T x N")
        L.check(self._lib.dd_exact_distance_fields(self._h, C.c_void_p(t.ctypes.data), int(T),
                                                   _kind(kind), C.c_void_p(out.data_ptr()),
                                                   _stream_handle(stream)))
        return out

    def trace_paths_triangles(self, sources, targets, fields, max_steps, stream=None):
        """Device tensors (points [T, max_steps+1, 2] f64, where [T, max_steps+1, 2] i32,
        len [T], status [T]) of triangle-based paths on the given fields (FP32, or
        FP64 fields from exact_fields)."""
        torch = _torch()
        s = np.ascontiguousarray(sources, dtype=np.int32)
        t = np.ascontiguousarray(targets, dtype=np.int32)
        T = len(s)
        dev = f"cuda:{self.ctx.device}"
        if not fields.is_contiguous() or fields.dtype not in (torch.float32, torch.float64):
            raise ValueError("fields must be contiguous float32 or float64")
        fn = (self._lib.dd_trace_paths_triangles if fields.dtype == torch.float32
              else self._lib.dd_trace_paths_triangles_f64)
        pts = torch.empty((T, max_steps + 1, 2), dtype=torch.float64, device=dev)
        wh = torch.empty((T, max_steps + 1, 2), dtype=torch.int32, device=dev)
        info = torch.empty((2, T), dtype=torch.int32, device=dev)
        L.check(fn(
            self._h, int(T), C.c_void_p(s.ctypes.data), C.c_void_p(t.ctypes.data),
            C.c_void_p(fields.data_ptr()), int(max_steps), C.c_void_p(pts.data_ptr()),
            C.c_void_p(wh.data_ptr()), C.c_void_p(info[0].data_ptr()),
            C.c_void_p(info[1].data_ptr()), _stream_handle(stream)))
        return pts, wh, info[0], info[1]

    def local_minima(self, targets, fields, bounds, stream=None):
        """Device tensors (classes uint8 [T, N], counts int32 [T, 2]) of the
        local-minimum census: 0 not a minimum, 1 certain minimum, 2 undecided."""
        torch = _torch()
        t = np.ascontiguousarray(targets, dtype=np.int32)
        T = len(t)
        dev = f"cuda:{self.ctx.device}"
        if not fields.is_contiguous() or fields.dtype != torch.float32:
            raise ValueError("fields must be contiguous float32")
        cls = torch.empty((T, self.N), dtype=torch.uint8, device=dev)
        counts = torch.empty((T, 2), dtype=torch.int32, device=dev)
        b = (L.dd_error_bound * T)(*[L.dd_error_bound(a, r) for a, r in bounds])
        L.check(self._lib.dd_local_minima(self._h, int(T), C.c_void_p(t.ctypes.data),
                                          C.c_void_p(fields.data_ptr()), b,
                                          C.c_void_p(cls.data_ptr()), C.c_void_p(counts.data_ptr()),
                                          _stream_handle(stream)))
        return cls, counts

    def resolve_minima(self, targets, kind, classes, counts=None, stream=None):
        """Re-decide the undecided entries (class 2) of a census in FP64, in place;
        counts ([T, 2] int32 device tensor, optional) recomputed."""
        torch = _torch()
        t = np.ascontiguousarray(targets, dtype=np.int32)
        if not classes.is_contiguous() or classes.dtype != torch.uint8:
            raise ValueError("classes must be a contiguous uint8 tensor")
        L.check(self._lib.dd_resolve_minima(
            self._h, int(len(t)), C.c_void_p(t.ctypes.data), _kind(kind),
            C.c_void_p(classes.data_ptr()),
            C.c_void_p(counts.data_ptr()) if counts is not None else None,
            _stream_handle(stream)))
        return classes, counts

    def plan_path(self, source, target, kind, max_steps=4000, stream=None):
        """(vertex list, status name, FP64 re-decisions) for one query; synchronous."""
        buf = (C.c_int32 * (max_steps + 1))()
        n, st, rc = C.c_int32(), C.c_int32(), C.c_int32()
        L.check(self._lib.dd_plan_path(self._h, int(source), int(target), _kind(kind),
                                       int(max_steps), buf, C.byref(n), C.byref(st), C.byref(rc),
                                       _stream_handle(stream)))
        return list(buf[:n.value]), PATH_STATUS[st.value], rc.value
