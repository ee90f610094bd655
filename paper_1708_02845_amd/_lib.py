"""ctypes declarations of libdd.so (the C ABI in include/dd.h)."""

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdd.so")

DD_OK, DD_EINVAL, DD_ENOMEM, DD_EDEVICE, DD_ESTATE, DD_ENOCONV = range(6)
DD_TV, DD_KL, DD_CHI2, DD_HELLINGER = 0, 1, 2, 3
DD_FORM_NONE, DD_FORM_F32, DD_FORM_F16X3, DD_FORM_BF16X3, DD_FORM_F16 = -1, 0, 1, 2, 3
DD_CSR_F32, DD_CSR_F16 = 0, 1
DD_PATH_REACHED, DD_PATH_STUCK, DD_PATH_MAX_STEPS = 0, 1, 2
DD_NOALLOC_SCRATCH_BYTES = 48 << 20

STATUS_NAMES = {0: "DD_OK", 1: "DD_EINVAL", 2: "DD_ENOMEM", 3: "DD_EDEVICE", 4: "DD_ESTATE",
                5: "DD_ENOCONV"}


class DDError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class dd_adjacency(C.Structure):
    _fields_ = [("n", C.c_int32), ("row_ptr", C.POINTER(C.c_int64)), ("col", C.POINTER(C.c_int32))]


class dd_load_opts(C.Structure):
    _fields_ = [("gemm_form", C.c_int32), ("tau", C.c_double), ("tau_relative", C.c_int32),
                ("validate", C.c_int32), ("csr_values", C.c_int32)]


class dd_error_bound(C.Structure):
    _fields_ = [("abs", C.c_double), ("rel", C.c_double)]


class dd_grid_solve_stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("batches", C.c_int32), ("levels", C.c_int32),
                ("total_iterations", C.c_int32), ("max_rel_residual", C.c_double)]


class dd_kernel_info(C.Structure):
    _fields_ = [("n", C.c_int32), ("b_in", C.c_int32), ("b", C.c_int32), ("is_csr", C.c_int32),
                ("nnz", C.c_int64), ("gemm_form", C.c_int32), ("has_adjacency", C.c_int32),
                ("hbm_bytes", C.c_size_t), ("csr_values", C.c_int32)]


EXPORTS = {
    # name: (restype, argtypes)
    "dd_create": (C.c_int, [C.c_int, C.POINTER(C.c_void_p)]),
    "dd_destroy": (C.c_int, [C.c_void_p]),
    "dd_path_level1": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int),
                                 C.POINTER(C.c_double)]),
    "dd_load_kernel_dense": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                                       C.c_int32, C.POINTER(dd_adjacency), C.POINTER(dd_load_opts),
                                       C.POINTER(C.c_void_p)]),
    "dd_load_kernel_csr": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_int32, C.c_void_p, C.c_double, C.c_int32,
                                     C.POINTER(dd_adjacency), C.POINTER(dd_load_opts),
                                     C.POINTER(C.c_void_p)]),
    "dd_kernel_get_info": (C.c_int, [C.c_void_p, C.POINTER(dd_kernel_info)]),
    "dd_dense_footprint": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(dd_load_opts),
                                     C.POINTER(C.c_size_t)]),
    "dd_distance_field": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                    C.POINTER(dd_error_bound), C.c_void_p]),
    "dd_distance_fields_tv_kl": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                           C.POINTER(dd_error_bound), C.c_void_p]),
    "dd_batch_distance_fields": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                           C.POINTER(dd_error_bound), C.c_void_p]),
    "dd_trace_paths": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                 C.c_void_p, C.POINTER(dd_error_bound), C.c_int32, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dd_resolve_minima": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                    C.c_void_p, C.c_void_p]),
    "dd_plan_path": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                               C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                               C.c_void_p]),
    "dd_local_minima": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                  C.POINTER(dd_error_bound), C.c_void_p, C.c_void_p, C.c_void_p]),
    "dd_trace_paths_on_demand": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                           C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p]),
    "dd_support_kl_field": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_int32, C.c_void_p,
                                      C.POINTER(dd_error_bound), C.c_void_p]),
    "dd_attach_mesh": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "dd_trace_paths_triangles": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_void_p, C.c_void_p]),
    "dd_grid_poisson_kernel": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32,
                                         C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                         C.c_double, C.c_int32, C.c_int32,
                                         C.POINTER(dd_grid_solve_stats), C.c_void_p]),
    "dd_batch_distance_fields_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                                   C.c_void_p, C.POINTER(dd_error_bound),
                                                   C.c_void_p]),
    "dd_kernel_footprint": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "dd_call_scratch_bytes": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32,
                                        C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "dd_grid_green_function": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                         C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                         C.c_double, C.c_int32, C.c_int32,
                                         C.POINTER(dd_grid_solve_stats), C.c_void_p]),
    "dd_trace_paths_triangles_f64": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                               C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                               C.c_void_p, C.c_void_p, C.c_void_p]),
    "dd_exact_distance_fields": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                           C.c_void_p, C.c_void_p]),
    "dd_free_kernel": (C.c_int, [C.c_void_p]),
    "dd_last_error": (C.c_char_p, []),
}

_lib = None


def load():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1708_02845_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status):
    if status != DD_OK:
        raise DDError(status, load().dd_last_error().decode(errors="replace"))
