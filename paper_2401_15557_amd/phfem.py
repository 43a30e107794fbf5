"""Thin ctypes binding of libphfem.so (the C ABI declared in include/phfem.h).

Every ``phf_*`` function here marshals its arguments and calls the C entry
point of the same name; all computation runs in the HIP library. Device
buffers are torch tensors on a ROCm device (torch is used for memory and
streams only). A missing or unloadable library raises ``PhfLibraryError``:
there is no fallback path.

Small conveniences on top (``Context``, ``Mesh``, ``alloc_system``) only
allocate tensors and forward to the same calls.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libphfem.so")

PHF_OK, PHF_EINVAL, PHF_EORIENT, PHF_EMESH = 0, -1, -2, -3
PHF_EBOUNDARY, PHF_ENOMEM, PHF_ENOCONV, PHF_EHIP, PHF_ESTATE = -4, -5, -6, -7, -8
PHF_ETIMEDOUT = -9
PHF_REQ_ELLIPTIC, PHF_REQ_CN = 0, 1
PHF_HOST, PHF_DEVICE = 0, 1

PHF_FN_ZERO, PHF_FN_CONST, PHF_FN_SIN_COS, PHF_FN_SIN_SIN = 0, 1, 2, 3
PHF_FN_GRAD_SIN_COS, PHF_FN_GRAD_SIN_SIN = 4, 5
PHF_FN_PAPER_U, PHF_FN_PAPER_F, PHF_FN_PAPER_FLUX = 6, 7, 8
PHF_FN_EDGE_ARRAY = 100
PHF_SOLVER_NULLSPACE_CG = 0
PHF_SOLVER_NULLSPACE_BICGSTAB = 1
PHF_PRECOND_JACOBI, PHF_PRECOND_MULTIGRID = 0, 1
PHF_MG_SMOOTH_DEFAULT, PHF_MG_SMOOTH_JACOBI, PHF_MG_SMOOTH_CHEBYSHEV = 0, 1, 2

EXPORTED = (
    "phf_create", "phf_destroy", "phf_set_stream", "phf_synchronize", "phf_mem_stats",
    "phf_release_cache", "phf_status_str", "phf_last_error", "phf_version",
    "phf_trace_enable", "phf_trace_filter", "phf_trace_reset", "phf_trace_query",
    "phf_trace_dump", "phf_trace_samples",
    "phf_mesh_create", "phf_mesh_destroy", "phf_mesh_refine", "phf_mesh_geometry",
    "phf_mesh_get_info", "phf_mesh_topology", "phf_mesh_pattern",
    "phf_assemble", "phf_spmv", "phf_solve",
    "phf_cn_create", "phf_cn_set_state", "phf_cn_run", "phf_cn_get_state", "phf_cn_destroy",
    "phf_cn_batch_create", "phf_cn_batch_run", "phf_cn_batch_destroy",
    "phf_error_norms", "phf_error_norms_noalloc",
    "phf_batch_create", "phf_batch_destroy", "phf_batch_assemble", "phf_batch_tune",
    "phf_batch_get_config", "phf_batch_set_config",
    "phf_server_create", "phf_server_destroy", "phf_server_submit", "phf_server_wait",
    "phf_server_query",
)


class PhfLibraryError(ImportError):
    """libphfem.so is missing or cannot be loaded."""


class PhfError(RuntimeError):
    def __init__(self, code, fn, msg):
        super().__init__(f"{fn} failed with {code} ({_status(code)}): {msg}")
        self.code = code


# ---- ABI structures (layout mirrors include/phfem.h) -----------------------

class phf_mesh_info(ctypes.Structure):
    _fields_ = [("nC", ctypes.c_int32), ("nE", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("N", ctypes.c_int32), ("L", ctypes.c_int32), ("nD", ctypes.c_int32),
                ("nN", ctypes.c_int32), ("n_interior", ctypes.c_int32),
                ("n_free", ctypes.c_int32), ("nnz_K", ctypes.c_int64),
                ("nnz_C", ctypes.c_int64), ("nnz_saddle", ctypes.c_int64),
                ("nnz_reduced", ctypes.c_int64), ("device_bytes", ctypes.c_int64)]


class phf_coeffs(ctypes.Structure):
    _fields_ = [("A", ctypes.c_double * 4), ("p", ctypes.c_double * 2),
                ("delta", ctypes.c_double), ("a_T", ctypes.c_void_p)]


class phf_fn(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("c", ctypes.c_double * 4), ("edge_values", ctypes.c_void_p)]


class phf_data(ctypes.Structure):
    _fields_ = [("f", phf_fn), ("g", phf_fn), ("uD", phf_fn), ("t", ctypes.c_double)]


class phf_system(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("K", "M", "D", "C", "F", "bD", "S")]


class phf_solver_opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("check_every", ctypes.c_int32),
                ("saddle_residual", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("mg_sweeps", ctypes.c_int32), ("mg_omega", ctypes.c_double),
                ("mg_smoother", ctypes.c_int32), ("reserved_", ctypes.c_int32),
                ("mg_range", ctypes.c_double), ("saddle_rtol", ctypes.c_double)]


class phf_solve_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("saddle_rel_residual", ctypes.c_double)]


class phf_cn_opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("iters_per_step", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("mg_sweeps", ctypes.c_int32), ("mg_omega", ctypes.c_double),
                ("mg_smoother", ctypes.c_int32), ("reserved_", ctypes.c_int32),
                ("mg_range", ctypes.c_double)]


PHF_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
PHF_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class phf_allocator(ctypes.Structure):
    _fields_ = [("alloc", PHF_ALLOC_FN), ("free", PHF_FREE_FN), ("user", ctypes.c_void_p)]


class phf_batch_config(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("ms", ctypes.c_double), ("lanes", ctypes.c_int32), ("direct", ctypes.c_int32),
                ("gather", ctypes.c_int32), ("reserved_", ctypes.c_int32)]


class phf_server_opts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("reserved_", ctypes.c_int32),
                ("memory_bytes", ctypes.c_int64)]


class phf_request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("xy", ctypes.c_void_p), ("elem", ctypes.c_void_p), ("dir", ctypes.c_void_p),
                ("neu", ctypes.c_void_p), ("nC", ctypes.c_int32), ("nE", ctypes.c_int32),
                ("nD", ctypes.c_int32), ("nN", ctypes.c_int32), ("coeffs", phf_coeffs),
                ("data", phf_data), ("u0", phf_fn), ("exact", phf_fn), ("rtol", ctypes.c_double),
                ("k", ctypes.c_double), ("steps", ctypes.c_int32), ("want_norms", ctypes.c_int32),
                ("U_out", ctypes.c_void_p)]


class phf_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("nE", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("h1", ctypes.c_double), ("l2", ctypes.c_double),
                ("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double)]


class phf_server_stats(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("running", ctypes.c_int32),
                ("peak_running", ctypes.c_int32), ("queued", ctypes.c_int32),
                ("completed", ctypes.c_int64), ("budget_bytes", ctypes.c_double),
                ("reserved_bytes", ctypes.c_double), ("peak_reserved_bytes", ctypes.c_double)]


_lib = None
_VP, _I32, _I64, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_SIGS = {
    "phf_create": [ctypes.POINTER(_VP), ctypes.c_int, _VP, ctypes.POINTER(phf_allocator)],
    "phf_destroy": [_VP],
    "phf_set_stream": [_VP, _VP],
    "phf_synchronize": [_VP],
    "phf_mem_stats": [_VP, ctypes.POINTER(_I64), ctypes.POINTER(_I64)],
    "phf_release_cache": [_VP],
    "phf_status_str": [ctypes.c_int],
    "phf_last_error": [_VP],
    "phf_version": [],
    "phf_trace_enable": [_VP, ctypes.c_int],
    "phf_trace_filter": [_VP, ctypes.c_char_p],
    "phf_trace_reset": [_VP],
    "phf_trace_query": [_VP, ctypes.c_char_p, ctypes.POINTER(_I64), ctypes.POINTER(_D)],
    "phf_trace_dump": [_VP, ctypes.c_char_p, ctypes.c_size_t],
    "phf_trace_samples": [_VP, ctypes.c_char_p, ctypes.POINTER(ctypes.c_float), ctypes.c_int64,
                          ctypes.POINTER(ctypes.c_int64)],
    "phf_mesh_create": [_VP, _VP, _I32, _VP, _I32, _VP, _I32, _VP, _I32, ctypes.c_int,
                        ctypes.POINTER(_VP)],
    "phf_mesh_destroy": [_VP],
    "phf_mesh_refine": [_VP, ctypes.POINTER(_VP)],
    "phf_mesh_geometry": [_VP, _VP, _VP, _VP, _VP, ctypes.c_int],
    "phf_mesh_get_info": [_VP, ctypes.POINTER(phf_mesh_info)],
    "phf_mesh_topology": [_VP] + [_VP] * 9 + [ctypes.c_int],
    "phf_mesh_pattern": [_VP] + [_VP] * 6 + [ctypes.c_int],
    "phf_assemble": [_VP, ctypes.POINTER(phf_coeffs), ctypes.POINTER(phf_data),
                     ctypes.POINTER(phf_system)],
    "phf_spmv": [_VP, _I32, _VP, _VP, _VP, _D, _VP, _D, _VP],
    "phf_solve": [_VP, ctypes.POINTER(phf_coeffs), ctypes.POINTER(phf_system),
                  ctypes.POINTER(phf_solver_opts), _VP, _VP, ctypes.POINTER(phf_solve_stats)],
    "phf_cn_create": [_VP, ctypes.POINTER(phf_coeffs), _D, ctypes.POINTER(phf_cn_opts),
                      ctypes.POINTER(_VP)],
    "phf_cn_set_state": [_VP, _VP, _VP, _D],
    "phf_cn_run": [_VP, ctypes.POINTER(phf_data), _I32, _I32, ctypes.POINTER(phf_solve_stats)],
    "phf_cn_get_state": [_VP, _VP, _VP, ctypes.POINTER(_D)],
    "phf_cn_destroy": [_VP],
    "phf_cn_batch_create": [ctypes.POINTER(_VP), _I32, ctypes.POINTER(_VP)],
    "phf_cn_batch_run": [_VP, ctypes.POINTER(phf_data), _I32, ctypes.POINTER(phf_solve_stats)],
    "phf_cn_batch_destroy": [_VP],
    "phf_error_norms": [_VP, _VP, ctypes.POINTER(phf_fn), _D, ctypes.POINTER(_D),
                        ctypes.POINTER(_D)],
    "phf_error_norms_noalloc": [_VP, _VP, ctypes.POINTER(phf_fn), _D, _VP],
    "phf_batch_create": [_VP, ctypes.POINTER(_VP), _I32, ctypes.POINTER(_VP)],
    "phf_batch_destroy": [_VP],
    "phf_batch_assemble": [_VP, ctypes.POINTER(phf_coeffs), ctypes.POINTER(phf_data),
                           ctypes.POINTER(phf_system)],
    "phf_batch_tune": [_VP, ctypes.POINTER(phf_coeffs), ctypes.POINTER(phf_data),
                       ctypes.POINTER(phf_system), _I32, ctypes.POINTER(phf_batch_config), _I32,
                       ctypes.POINTER(_I32)],
    "phf_batch_get_config": [_VP, ctypes.POINTER(phf_batch_config)],
    "phf_batch_set_config": [_VP, ctypes.POINTER(phf_batch_config)],
    "phf_server_create": [ctypes.c_int, ctypes.POINTER(phf_server_opts), ctypes.POINTER(_VP)],
    "phf_server_destroy": [_VP],
    "phf_server_submit": [_VP, ctypes.POINTER(phf_request), ctypes.POINTER(_I64)],
    "phf_server_wait": [_VP, _I64, _D, ctypes.POINTER(phf_result)],
    "phf_server_query": [_VP, ctypes.POINTER(phf_server_stats)],
}


def load(path=None):
    """Loads libphfem.so (once). Raises PhfLibraryError if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise PhfLibraryError(f"{p} not found: build it with `python -m paper_2401_15557_amd.build`")
    try:
        lib = ctypes.CDLL(p)
    except OSError as e:
        raise PhfLibraryError(f"cannot load {p}: {e}") from e
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name in ("phf_status_str", "phf_last_error",
                                                 "phf_version") else ctypes.c_int
    _lib = lib
    return lib


def _status(code):
    try:
        return load().phf_status_str(code).decode()
    except Exception:
        return str(code)


def _ptr(x):
    """Raw address of a tensor / numpy array / int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "ctypes"):
        return x.ctypes.data
    raise TypeError(type(x))


def _call(name, ctx, *args):
    rc = getattr(load(), name)(*args)
    if rc < 0:
        msg = load().phf_last_error(ctx).decode() if ctx else ""
        raise PhfError(rc, name, msg)
    return rc


# ---- C entry points (same names) -------------------------------------------

def phf_version():
    return load().phf_version().decode()


def phf_status_str(code):
    return load().phf_status_str(code).decode()


def make_allocator(alloc_fn, free_fn):
    """A phf_allocator calling two Python functions: alloc_fn(nbytes) -> device
    address (0 or an exception: failure) and free_fn(address). The returned
    structure keeps the C callbacks alive; keep it as long as the context."""
    def _alloc(nbytes, user):
        try:
            return int(alloc_fn(int(nbytes))) or None
        except Exception:
            return None

    def _free(ptr, user):
        try:
            free_fn(int(ptr))
        except Exception:
            pass

    a = phf_allocator(PHF_ALLOC_FN(_alloc), PHF_FREE_FN(_free), None)
    a._keep = (_alloc, _free)
    return a


def torch_allocator(device, stream):
    """phf_allocator backed by torch's caching allocator on ``stream``, so that
    torch owns every device byte of the context."""
    import torch
    return make_allocator(lambda n: torch.cuda.caching_allocator_alloc(n, device, stream),
                          torch.cuda.caching_allocator_delete)


def phf_create(device=0, stream=None, allocator=None):
    """allocator: a phf_allocator (make_allocator / torch_allocator) or None
    (the library's hipMalloc)."""
    h = _VP()
    _call("phf_create", None, ctypes.byref(h), int(device), _ptr(stream),
          ctypes.byref(allocator) if allocator is not None else None)
    return h.value


def phf_destroy(ctx):
    _call("phf_destroy", None, ctx)


def phf_set_stream(ctx, stream):
    _call("phf_set_stream", ctx, ctx, _ptr(stream))


def phf_synchronize(ctx):
    _call("phf_synchronize", ctx, ctx)


def phf_mem_stats(ctx):
    """(live_bytes, cached_bytes) of the context's device memory pool."""
    live, cached = _I64(), _I64()
    _call("phf_mem_stats", ctx, ctx, ctypes.byref(live), ctypes.byref(cached))
    return live.value, cached.value


def phf_release_cache(ctx):
    _call("phf_release_cache", ctx, ctx)


def phf_last_error(ctx):
    return load().phf_last_error(ctx).decode()


def phf_trace_enable(ctx, on=True):
    _call("phf_trace_enable", ctx, ctx, 1 if on else 0)


def phf_trace_filter(ctx, kernel=None):
    """Trace only launches named ``kernel`` (None: every launch)."""
    _call("phf_trace_filter", ctx, ctx, kernel.encode() if kernel else None)


def phf_trace_reset(ctx):
    _call("phf_trace_reset", ctx, ctx)


def phf_trace_query(ctx, kernel=None):
    c, ms = _I64(), _D()
    _call("phf_trace_query", ctx, ctx, kernel.encode() if kernel else None, ctypes.byref(c),
          ctypes.byref(ms))
    return c.value, ms.value


def phf_trace_samples(ctx, kernel):
    """Per-launch milliseconds of the traced launches named ``kernel``."""
    n = _I64()
    _call("phf_trace_samples", ctx, ctx, kernel.encode(), None, 0, ctypes.byref(n))
    buf = (ctypes.c_float * max(n.value, 1))()
    _call("phf_trace_samples", ctx, ctx, kernel.encode(), buf, n.value, ctypes.byref(n))
    return [float(buf[i]) for i in range(n.value)]


def phf_trace_dump(ctx):
    buf = ctypes.create_string_buffer(1 << 16)
    _call("phf_trace_dump", ctx, ctx, buf, len(buf))
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out


def phf_mesh_create(ctx, xy, elem, dirichlet, neumann, memspace=PHF_HOST):
    """xy (nC,2) float64, elem (nE,3) int32, dirichlet/neumann (n,2) int32,
    numpy arrays (memspace=PHF_HOST) or device tensors (PHF_DEVICE)."""
    h = _VP()
    _call("phf_mesh_create", ctx, ctx, _ptr(xy), int(xy.shape[0]), _ptr(elem),
          int(elem.shape[0]), _ptr(dirichlet) if len(dirichlet) else None, int(len(dirichlet)),
          _ptr(neumann) if len(neumann) else None, int(len(neumann)), int(memspace),
          ctypes.byref(h))
    return h.value


def phf_mesh_destroy(mesh):
    _call("phf_mesh_destroy", None, mesh)


def phf_mesh_refine(mesh):
    """Red-refined device mesh (Listing 4 numbering); keeps a reference to mesh."""
    h = _VP()
    _call("phf_mesh_refine", None, mesh, ctypes.byref(h))
    return h.value


def phf_mesh_geometry(mesh, xy=None, elem=None, dirichlet=None, neumann=None,
                      memspace=PHF_DEVICE):
    _call("phf_mesh_geometry", None, mesh, _ptr(xy), _ptr(elem), _ptr(dirichlet), _ptr(neumann),
          int(memspace))


def phf_mesh_get_info(mesh):
    info = phf_mesh_info()
    _call("phf_mesh_get_info", None, mesh, ctypes.byref(info))
    return info


def phf_mesh_topology(mesh, edge_nodes=None, edge_elems=None, elem_edges=None, led=None,
                      ledTN=None, edge_type=None, edge_row=None, dir_edges=None, neu_edges=None,
                      memspace=PHF_DEVICE):
    _call("phf_mesh_topology", None, mesh, *(_ptr(a) for a in (
        edge_nodes, edge_elems, elem_edges, led, ledTN, edge_type, edge_row, dir_edges,
        neu_edges)), int(memspace))


def phf_mesh_pattern(mesh, K_rowptr=None, K_col=None, C_rowptr=None, C_col=None, S_rowptr=None,
                     S_col=None, memspace=PHF_DEVICE):
    _call("phf_mesh_pattern", None, mesh, *(_ptr(a) for a in (
        K_rowptr, K_col, C_rowptr, C_col, S_rowptr, S_col)), int(memspace))


def make_coeffs(A=(1.0, 0.0, 0.0, 1.0), p=(0.0, 0.0), delta=0.0, a_T=None):
    c = phf_coeffs()
    for q in range(4):
        c.A[q] = float(A[q])
    c.p[0], c.p[1] = float(p[0]), float(p[1])
    c.delta = float(delta)
    c.a_T = _ptr(a_T)
    c._keep = a_T
    return c


def make_fn(kind=PHF_FN_ZERO, *c, edge_values=None):
    f = phf_fn()
    f.kind = int(kind)
    for q, v in enumerate(c[:4]):
        f.c[q] = float(v)
    if edge_values is not None:
        f.kind = PHF_FN_EDGE_ARRAY
        f.edge_values = _ptr(edge_values)
    return f


def make_data(f=None, g=None, uD=None, t=0.0):
    d = phf_data()
    d.f = f if f is not None else make_fn()
    d.g = g if g is not None else make_fn()
    d.uD = uD if uD is not None else make_fn()
    d.t = float(t)
    return d


def phf_assemble(mesh, coeffs, data, system):
    _call("phf_assemble", None, mesh, ctypes.byref(coeffs), ctypes.byref(data),
          ctypes.byref(system))


def phf_spmv(ctx, nrows, rowptr, col, val, alpha, x, beta, y):
    _call("phf_spmv", ctx, ctx, int(nrows), _ptr(rowptr), _ptr(col), _ptr(val), float(alpha),
          _ptr(x), float(beta), _ptr(y))


def phf_solve(mesh, coeffs, system, U, Lam=None, rtol=1e-10, max_iter=20000, check_every=0,
              saddle_residual=False, raise_on_noconv=True, precond=PHF_PRECOND_JACOBI,
              mg_sweeps=0, mg_omega=0.0, method=PHF_SOLVER_NULLSPACE_CG,
              mg_smoother=PHF_MG_SMOOTH_DEFAULT, mg_range=0.0, saddle_rtol=0.0):
    o = phf_solver_opts(int(method), int(max_iter), float(rtol), int(check_every),
                        1 if saddle_residual else 0, int(precond), int(mg_sweeps),
                        float(mg_omega), int(mg_smoother), 0, float(mg_range),
                        float(saddle_rtol))
    st = phf_solve_stats()
    rc = load().phf_solve(mesh, ctypes.byref(coeffs), ctypes.byref(system), ctypes.byref(o),
                          _ptr(U), _ptr(Lam), ctypes.byref(st))
    if rc < 0 and (rc != PHF_ENOCONV or raise_on_noconv):
        raise PhfError(rc, "phf_solve", "")
    return st


def phf_error_norms(mesh, U, u, t=0.0):
    """(broken H1 seminorm, L2 norm) of u - U_h; u is a phf_fn."""
    h1, l2 = _D(), _D()
    rc = load().phf_error_norms(mesh, _ptr(U), ctypes.byref(u), float(t), ctypes.byref(h1),
                                ctypes.byref(l2))
    if rc < 0:
        raise PhfError(rc, "phf_error_norms", "")
    return h1.value, l2.value


def phf_error_norms_noalloc(mesh, U, u, t, norms):
    """(H1, L2) of u - U_h into the device array norms (2 doubles), without
    allocating or waiting."""
    rc = load().phf_error_norms_noalloc(mesh, _ptr(U), ctypes.byref(u), float(t), _ptr(norms))
    if rc < 0:
        raise PhfError(rc, "phf_error_norms_noalloc", "")


def _struct_array(typ, items):
    arr = (typ * len(items))()
    for i, it in enumerate(items):
        ctypes.memmove(ctypes.byref(arr, i * ctypes.sizeof(typ)), ctypes.byref(it),
                       ctypes.sizeof(typ))
    return arr


def phf_batch_create(ctx, meshes):
    """meshes: phf_mesh handles of one context."""
    arr = (_VP * len(meshes))(*meshes)
    out = _VP()
    _call("phf_batch_create", ctx, ctx, arr, len(meshes), ctypes.byref(out))
    return out.value


def phf_batch_destroy(batch):
    rc = load().phf_batch_destroy(batch)
    if rc < 0:
        raise PhfError(rc, "phf_batch_destroy", "")


def phf_batch_assemble(batch, coeffs, data, systems):
    """Lists of phf_coeffs, phf_data and phf_system, one per mesh."""
    rc = load().phf_batch_assemble(batch, _struct_array(phf_coeffs, coeffs),
                                   _struct_array(phf_data, data),
                                   _struct_array(phf_system, systems))
    if rc < 0:
        raise PhfError(rc, "phf_batch_assemble", "")


def phf_batch_tune(batch, coeffs, data, systems, reps=5):
    """Times every launch shape; returns [(tile, blocks_per_cu, lanes, direct,
    gather, ms)] and keeps the fastest as the batch's configuration."""
    res = (phf_batch_config * 32)()
    n = _I32()
    rc = load().phf_batch_tune(batch, _struct_array(phf_coeffs, coeffs),
                               _struct_array(phf_data, data), _struct_array(phf_system, systems),
                               int(reps), res, 32, ctypes.byref(n))
    if rc < 0:
        raise PhfError(rc, "phf_batch_tune", "")
    return [(res[i].tile, res[i].blocks_per_cu, res[i].lanes, res[i].direct, res[i].gather,
             res[i].ms) for i in range(n.value)]


def phf_batch_get_config(batch):
    """(tile, blocks_per_cu, lanes, direct, gather) of the batch's launch shape."""
    c = phf_batch_config()
    rc = load().phf_batch_get_config(batch, ctypes.byref(c))
    if rc < 0:
        raise PhfError(rc, "phf_batch_get_config", "")
    return c.tile, c.blocks_per_cu, c.lanes, c.direct, c.gather


def phf_batch_set_config(batch, tile, blocks_per_cu=0, lanes=1, direct=0, gather=0):
    c = phf_batch_config(int(tile), int(blocks_per_cu), 0.0, int(lanes), int(direct),
                         int(gather), 0)
    rc = load().phf_batch_set_config(batch, ctypes.byref(c))
    if rc < 0:
        raise PhfError(rc, "phf_batch_set_config", "")


def _check(rc, name):
    if rc < 0:
        raise PhfError(rc, name, "")


def phf_server_create(device=0, slots=4, memory_bytes=0):
    out = _VP()
    _check(load().phf_server_create(int(device), ctypes.byref(phf_server_opts(int(slots), 0,
                                                                               int(memory_bytes))),
                                    ctypes.byref(out)), "phf_server_create")
    return out.value


def phf_server_destroy(server):
    _check(load().phf_server_destroy(server), "phf_server_destroy")


def make_request(kind, mesh, refine=0, coeffs=None, data=None, u0=None, exact=None, rtol=1e-10,
                 k=0.0, steps=0, want_norms=False, U_out=None):
    """A phf_request for a meshgen.Mesh base mesh (host arrays are copied by
    phf_server_submit, so they only need to live until it returns)."""
    import numpy as np
    r = phf_request()
    r.kind, r.refine = int(kind), int(refine)
    xy = np.ascontiguousarray(mesh.coords, np.float64)
    el = np.ascontiguousarray(mesh.elements, np.int32)
    di = np.ascontiguousarray(mesh.dirichlet, np.int32).reshape(-1, 2)
    ne = np.ascontiguousarray(mesh.neumann, np.int32).reshape(-1, 2)
    r.xy, r.elem = xy.ctypes.data, el.ctypes.data
    r.dir = di.ctypes.data if len(di) else None
    r.neu = ne.ctypes.data if len(ne) else None
    r.nC, r.nE, r.nD, r.nN = len(xy), len(el), len(di), len(ne)
    r.coeffs = coeffs if coeffs is not None else make_coeffs()
    r.data = data if data is not None else make_data()
    r.u0 = u0 if u0 is not None else make_fn()
    r.exact = exact if exact is not None else make_fn()
    r.rtol, r.k, r.steps = float(rtol), float(k), int(steps)
    r.want_norms = 1 if want_norms else 0
    r.U_out = U_out.ctypes.data if U_out is not None else None
    r._keep = (xy, el, di, ne, U_out)
    return r


def phf_server_submit(server, req):
    i = _I64()
    _check(load().phf_server_submit(server, ctypes.byref(req), ctypes.byref(i)),
           "phf_server_submit")
    return i.value


def phf_server_wait(server, rid, timeout_ms=-1.0):
    """The phf_result of request rid, or None on PHF_ETIMEDOUT."""
    res = phf_result()
    rc = load().phf_server_wait(server, int(rid), float(timeout_ms), ctypes.byref(res))
    if rc == PHF_ETIMEDOUT:
        return None
    _check(rc, "phf_server_wait")
    return res


def phf_server_query(server):
    st = phf_server_stats()
    _check(load().phf_server_query(server, ctypes.byref(st)), "phf_server_query")
    return st


def phf_cn_create(mesh, coeffs, k, rtol=1e-10, max_iter=5000, iters_per_step=8,
                  precond=PHF_PRECOND_JACOBI, mg_sweeps=0, mg_omega=0.0,
                  mg_smoother=PHF_MG_SMOOTH_DEFAULT, mg_range=0.0):
    h = _VP()
    o = phf_cn_opts(float(rtol), int(max_iter), int(iters_per_step), int(precond),
                    int(mg_sweeps), float(mg_omega), int(mg_smoother), 0, float(mg_range))
    _call("phf_cn_create", None, mesh, ctypes.byref(coeffs), float(k), ctypes.byref(o),
          ctypes.byref(h))
    return h.value


def phf_cn_set_state(cn, U, Lam, t):
    _call("phf_cn_set_state", None, cn, _ptr(U), _ptr(Lam), float(t))


def phf_cn_run(cn, data, nsteps, use_graph=False, raise_on_noconv=True):
    st = phf_solve_stats()
    rc = load().phf_cn_run(cn, ctypes.byref(data), int(nsteps), 1 if use_graph else 0,
                           ctypes.byref(st))
    if rc < 0 and (rc != PHF_ENOCONV or raise_on_noconv):
        raise PhfError(rc, "phf_cn_run", "")
    return st


def phf_cn_get_state(cn, U=None, Lam=None):
    t = _D()
    _call("phf_cn_get_state", None, cn, _ptr(U), _ptr(Lam), ctypes.byref(t))
    return t.value


def phf_cn_destroy(cn):
    _call("phf_cn_destroy", None, cn)


def phf_cn_batch_create(steppers):
    """A batch of Crank-Nicolson steppers (handles) of one context."""
    arr = (_VP * len(steppers))(*steppers)
    out = _VP()
    _check(load().phf_cn_batch_create(arr, len(steppers), ctypes.byref(out)),
           "phf_cn_batch_create")
    return out.value


def phf_cn_batch_run(batch, data, nsteps, raise_on_noconv=True):
    """Advances every stepper of the batch nsteps steps; data: one phf_data
    per stepper. Returns the per-stepper phf_solve_stats."""
    st = (phf_solve_stats * len(data))()
    rc = load().phf_cn_batch_run(batch, _struct_array(phf_data, data), int(nsteps), st)
    if rc < 0 and (rc != PHF_ENOCONV or raise_on_noconv):
        raise PhfError(rc, "phf_cn_batch_run", "")
    return [st[i] for i in range(len(data))]


def phf_cn_batch_destroy(batch):
    _check(load().phf_cn_batch_destroy(batch), "phf_cn_batch_destroy")


# ---- conveniences: tensor allocation around the calls above ----------------

class Context:
    """A phf context on ``device`` bound to torch's current stream. Its device
    memory comes from torch's caching allocator unless ``allocator`` is
    given (a phf_allocator, or False for the library's own hipMalloc)."""

    def __init__(self, device=0, stream=None, allocator=None):
        import torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        if allocator is None:
            allocator = torch_allocator(self.device, stream)
        self.allocator = allocator or None
        self.handle = phf_create(device, stream.cuda_stream, self.allocator)
        self._meshes = []  # weak references, in creation order

    def close(self):
        """Destroys the context after the meshes made through it (newest
        first, so refinements go before their parents)."""
        if self.handle:
            for ref in reversed(self._meshes):
                mesh = ref()
                if mesh is not None:
                    mesh.close()
            self._meshes = []
            phf_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    """Device mesh built from a meshgen.Mesh (host arrays), or by refinement."""

    def __init__(self, ctx: Context, m=None, handle=None, parent=None):
        import weakref
        self.ctx = ctx
        if handle is None:
            handle = phf_mesh_create(ctx.handle, m.coords, m.elements, m.dirichlet, m.neumann,
                                     PHF_HOST)
        self.handle = handle
        self.parent = parent  # a refinement keeps its parent alive
        ctx._meshes.append(weakref.ref(self))
        self.info = phf_mesh_get_info(self.handle)

    def refine(self):
        """One device red refinement; the result keeps this mesh alive."""
        return Mesh(self.ctx, handle=phf_mesh_refine(self.handle), parent=self)

    def close(self):
        if self.handle:
            phf_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def geometry(self):
        """(xy, elements, dirichlet, neumann) copied to host numpy arrays."""
        import numpy as np
        i = self.info
        xy = np.empty((i.nC, 2)); el = np.empty((i.nE, 3), np.int32)
        d = np.empty((i.nD, 2), np.int32); n = np.empty((i.nN, 2), np.int32)
        phf_mesh_geometry(self.handle, xy, el, d, n, PHF_HOST)
        return xy, el, d, n

    def topology(self):
        """Topology tables as host numpy arrays."""
        import numpy as np
        i = self.info
        out = dict(edge_nodes=np.empty((i.n_edges, 2), np.int32),
                   edge_elems=np.empty((i.n_edges, 2), np.int32),
                   elem_edges=np.empty((i.nE, 3), np.int32), led=np.empty(i.n_edges, np.int8),
                   ledTN=np.empty(i.n_edges, np.int8), edge_type=np.empty(i.n_edges, np.int8),
                   edge_row=np.empty(i.n_edges, np.int32), dir_edges=np.empty(i.nD, np.int32),
                   neu_edges=np.empty(i.nN, np.int32))
        phf_mesh_topology(self.handle, memspace=PHF_HOST, **out)
        return out

    def patterns(self):
        import numpy as np
        i = self.info
        out = dict(K_rowptr=np.empty(i.N + 1, np.int32), K_col=np.empty(i.nnz_K, np.int32),
                   C_rowptr=np.empty(i.L + 1, np.int32), C_col=np.empty(i.nnz_C, np.int32),
                   S_rowptr=np.empty(i.N + i.L + 1, np.int32),
                   S_col=np.empty(i.nnz_saddle, np.int32))
        phf_mesh_pattern(self.handle, memspace=PHF_HOST, **out)
        return out


def alloc_system(mesh: Mesh, with_D=False, with_S=False, fill=None):
    """Device output tensors sized from the mesh info, and the phf_system.
    fill: a value written into every output first (tests pass NaN, so that
    an entry the library does not write cannot pass a comparison)."""
    return alloc_system_for(mesh.info, mesh.ctx.device, with_D, with_S, fill)


def alloc_system_for(i, dev, with_D=False, with_S=False, fill=None):
    """As alloc_system, from a phf_mesh_info and a torch device."""
    import torch

    def buf(n):
        if fill is None:
            return torch.empty(n, dtype=torch.float64, device=dev)
        return torch.full((n,), float(fill), dtype=torch.float64, device=dev)

    t = dict(K=buf(i.nnz_K), M=buf(i.nnz_K), C=buf(max(i.nnz_C, 1)), F=buf(i.N),
             bD=buf(max(i.L, 1)))
    if with_D:
        t["D"] = buf(i.nnz_K)
    if with_S:
        t["S"] = buf(i.nnz_saddle)
    s = phf_system()
    for k, v in t.items():
        setattr(s, k, v.data_ptr())
    s._keep = t
    return s, t
