"""ctypes binding of libhhg.so: the C ABI declared in include/hhg.h.

Argument marshalling only: every computation runs in the HIP library.  Device
buffers are torch tensors (or raw integer pointers); streams default to the
current torch stream.  Every call raises HHGError on a non-zero status.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhhg.so")

HHG_OK, HHG_EINVAL, HHG_ENOMEM, HHG_EHIP, HHG_ENOTCONV = 0, -1, -2, -3, -4
HHG_F64, HHG_F32, HHG_BF16 = 0, 1, 2
HHG_OP_LAPLACE, HHG_OP_DIFFUSION, HHG_OP_MASS = 0, 1, 2
HHG_SMOOTH_GS, HHG_SMOOTH_NET = 0, 1
HHG_FEAT_F64, HHG_FEAT_MP, HHG_FEAT_VARK, HHG_FEAT_NET, HHG_FEAT_STOKES, HHG_FEAT_P2 = 1, 2, 4, 8, 16, 32
HHG_MODE_PLAIN_FP64, HHG_MODE_MP_IR, HHG_MODE_LEARNED = 0, 1, 2

_c = ctypes
_vp = _c.c_void_p
_i32 = _c.c_int32
_i64 = _c.c_int64


class hhg_solve_opts(_c.Structure):
    _fields_ = [("mode", _i32), ("op", _i32), ("rtol", _c.c_double), ("max_iters", _i32),
                ("nu1", _i32), ("nu2", _i32), ("res_history", _c.POINTER(_c.c_double)),
                ("history_capacity", _i32)]


class hhg_solve_stats(_c.Structure):
    _fields_ = [("iters", _i32), ("converged", _i32), ("smoother_used", _i32),
                ("fallback", _i32), ("res0", _c.c_double), ("rel_res", _c.c_double),
                ("ms", _c.c_double)]


class hhg_stokes_opts(_c.Structure):
    _fields_ = [("precision", _i32), ("rtol", _c.c_double), ("max_iters", _i32), ("nu1", _i32),
                ("nu2", _i32), ("res_history", _c.POINTER(_c.c_double)), ("history_capacity", _i32)]


class hhg_stokes_stats(_c.Structure):
    _fields_ = [("iters", _i32), ("converged", _i32), ("res0", _c.c_double), ("rel_res", _c.c_double),
                ("ms", _c.c_double)]


class hhg_energy_opts(_c.Structure):
    _fields_ = [("stokes", hhg_stokes_opts), ("Ra", _c.c_double), ("dt", _c.c_double),
                ("steps", _i32), ("stokes_every", _i32)]


class hhg_energy_stats(_c.Structure):
    _fields_ = [("steps", _i32), ("stokes_solves", _i32), ("minres_iters", _i64),
                ("worst_rel_res", _c.c_double), ("ms", _c.c_double)]



class hhg_p2_opts(_c.Structure):
    _fields_ = [("level", _i32), ("rtol", _c.c_double), ("max_iters", _i32), ("nu1", _i32), ("nu2", _i32),
                ("vnu1", _i32), ("vnu2", _i32), ("omega", _c.c_double),
                ("res_history", _c.POINTER(_c.c_double)), ("history_capacity", _i32)]


class hhg_p2_stats(_c.Structure):
    _fields_ = [("iters", _i32), ("converged", _i32), ("res0", _c.c_double), ("rel_res", _c.c_double),
                ("ms", _c.c_double)]

# name -> (restype, argtypes); restype int unless stated
_SIGS = {
    "hhg_last_error": (_c.c_char_p, []),
    "hhg_setup_mesh": (_c.c_int, [_vp, _i32, _vp, _i32, _i32, _i32, _c.POINTER(_vp)]),
    "hhg_destroy_mesh": (None, [_vp]),
    "hhg_workspace_bytes": (_c.c_int, [_vp, _c.c_uint32, _c.POINTER(_c.c_size_t)]),
    "hhg_bind_workspace": (_c.c_int, [_vp, _c.c_uint32, _vp, _c.c_size_t, _vp]),
    "hhg_field_elems": (_c.c_int, [_vp, _i32, _c.POINTER(_i64)]),
    "hhg_n_dofs": (_c.c_int, [_vp, _i32, _c.POINTER(_i64), _c.POINTER(_i64)]),
    "hhg_coords": (_c.c_int, [_vp, _i32, _vp]),
    "hhg_from_canonical": (_c.c_int, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "hhg_to_canonical": (_c.c_int, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "hhg_set_coefficient": (_c.c_int, [_vp, _vp, _vp]),
    "hhg_apply": (_c.c_int, [_vp, _i32, _i32, _i32, _vp, _vp, _vp]),
    "hhg_residual": (_c.c_int, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "hhg_smooth": (_c.c_int, [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _i32, _i32, _vp]),
    "hhg_vcycle": (_c.c_int, [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _i32, _i32, _vp]),
    "hhg_solve": (_c.c_int, [_vp, _c.POINTER(hhg_solve_opts), _vp, _vp,
                             _c.POINTER(hhg_solve_stats), _vp]),
    "hhg_jacobi": (_c.c_int, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp]),
    "hhg_dot": (_c.c_int, [_vp, _i32, _i32, _vp, _vp, _vp, _vp]),
    "hhg_axpby": (_c.c_int, [_vp, _i32, _i32, _c.c_double, _vp, _c.c_double, _vp, _vp, _vp]),
    "hhg_convert": (_c.c_int, [_vp, _i32, _i32, _vp, _i32, _vp, _vp]),
    "hhg_restrict": (_c.c_int, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "hhg_prolong_add": (_c.c_int, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "hhg_net_set_weights": (_c.c_int, [_vp, _vp, _i32, _vp]),
    "hhg_net_get_weights": (_c.c_int, [_vp, _vp, _i32, _vp]),
    "hhg_net_set_options": (_c.c_int, [_vp, _i32, _i32]),
    "hhg_net_forward": (_c.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "hhg_net_backward": (_c.c_int, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "hhg_net_adam_step": (_c.c_int, [_vp, _vp, _c.c_float, _i32, _vp]),
    "hhg_dot_noalloc": (_c.c_int, [_vp, _i32, _i32, _vp, _vp, _vp, _vp]),
    "hhg_set_face_coefficient": (_c.c_int, [_vp, _vp, _vp]),
    "hhg_stokes_setup": (_c.c_int, [_vp, _vp, _c.c_double, _vp]),
    "hhg_stokes_apply": (_c.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "hhg_stokes_residual": (_c.c_int, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "hhg_stokes_precond": (_c.c_int, [_vp, _i32, _vp, _vp, _i32, _i32, _vp]),
    "hhg_stokes_dot": (_c.c_int, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "hhg_stokes_solve": (_c.c_int, [_vp, _c.POINTER(hhg_stokes_opts), _vp, _vp,
                                    _c.POINTER(hhg_stokes_stats), _vp]),
    "hhg_timing_enable": (_c.c_int, [_vp, _i32]),
    "hhg_timing_read": (_c.c_int, [_vp, _c.POINTER(_i64), _c.POINTER(_c.c_double), _i32]),
    "hhg_ghost_table": (_c.c_int, [_vp, _i32, _c.POINTER(_i64), _vp, _vp]),
    "hhg_cell_coords": (_c.c_int, [_vp, _i32, _vp]),
    "hhg_cells_from_canonical": (_c.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "hhg_cells_to_canonical": (_c.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "hhg_transport_step": (_c.c_int, [_vp, _i32, _vp, _vp, _vp, _c.c_double, _vp]),
    "hhg_buoyancy": (_c.c_int, [_vp, _i32, _vp, _c.c_double, _vp, _vp]),
    "hhg_energy_run": (_c.c_int, [_vp, _c.POINTER(hhg_energy_opts), _vp, _vp,
                                  _c.POINTER(hhg_energy_stats), _vp]),
    "hhg_p2_setup": (_c.c_int, [_vp, _vp]),
    "hhg_p2_apply": (_c.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "hhg_p2_residual": (_c.c_int, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "hhg_p2_jacobi": (_c.c_int, [_vp, _i32, _c.c_double, _vp, _vp, _vp, _vp]),
    "hhg_p2_solve": (_c.c_int, [_vp, _c.POINTER(hhg_p2_opts), _vp, _vp, _c.POINTER(hhg_p2_stats), _vp]),
}

_lib = None


def lib():
    """Load libhhg.so (fails loudly if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhhg.so is not built; run `python -m paper_1805_10167_amd.build`")
        # torch first: its HIP runtime then satisfies the library's dependency,
        # so both share one runtime (loaded the other way round, torch would
        # bring a second copy, and the library's copy would see no device)
        import torch  # noqa: F401
        L = _c.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class HHGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("HHG error %d: %s" % (code, msg))
        self.code = code


def _check(rc):
    if rc != HHG_OK:
        raise HHGError(rc, lib().hhg_last_error().decode())
    return rc


def _ptr(x):
    """Device/host pointer of a torch tensor, numpy array, int or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------- raw calls

def hhg_last_error():
    return lib().hhg_last_error().decode()


def hhg_setup_mesh(vxy, tri, max_level, coarse_level):
    vxy = np.ascontiguousarray(vxy, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    h = _vp()
    _check(lib().hhg_setup_mesh(vxy.ctypes.data, len(vxy), tri.ctypes.data, len(tri),
                                max_level, coarse_level, _c.byref(h)))
    return h.value


def hhg_destroy_mesh(h):
    lib().hhg_destroy_mesh(h)


def hhg_workspace_bytes(h, features):
    n = _c.c_size_t()
    _check(lib().hhg_workspace_bytes(h, features, _c.byref(n)))
    return n.value


def hhg_bind_workspace(h, features, ws, nbytes=None, stream=None):
    if nbytes is None:
        nbytes = ws.numel() * ws.element_size()
    _check(lib().hhg_bind_workspace(h, features, _ptr(ws), nbytes, _stream(stream)))


def hhg_field_elems(h, level):
    n = _i64()
    _check(lib().hhg_field_elems(h, level, _c.byref(n)))
    return n.value


def hhg_n_dofs(h, level):
    a, b = _i64(), _i64()
    _check(lib().hhg_n_dofs(h, level, _c.byref(a), _c.byref(b)))
    return a.value, b.value


def hhg_coords(h, level):
    _, n_all = hhg_n_dofs(h, level)
    xy = np.empty((n_all, 2), dtype=np.float64)
    _check(lib().hhg_coords(h, level, xy.ctypes.data))
    return xy


def hhg_from_canonical(h, level, dtype, canon, field, stream=None):
    _check(lib().hhg_from_canonical(h, level, dtype, _ptr(canon), _ptr(field), _stream(stream)))


def hhg_to_canonical(h, level, dtype, field, canon, stream=None):
    _check(lib().hhg_to_canonical(h, level, dtype, _ptr(field), _ptr(canon), _stream(stream)))


def hhg_set_coefficient(h, k_canon, stream=None):
    _check(lib().hhg_set_coefficient(h, _ptr(k_canon), _stream(stream)))


def hhg_dot_noalloc(h, level, dtype, x, y, out, stream=None):
    _check(lib().hhg_dot_noalloc(h, level, dtype, _ptr(x), _ptr(y), _ptr(out), _stream(stream)))


def hhg_set_face_coefficient(h, coef, stream=None):
    c = np.ascontiguousarray(coef, dtype=np.float64)
    _check(lib().hhg_set_face_coefficient(h, c.ctypes.data, _stream(stream)))


def hhg_stokes_setup(h, viscosity, delta, stream=None):
    c = np.ascontiguousarray(viscosity, dtype=np.float64)
    _check(lib().hhg_stokes_setup(h, c.ctypes.data, float(delta), _stream(stream)))


def hhg_stokes_apply(h, level, x, y, stream=None):
    _check(lib().hhg_stokes_apply(h, level, _ptr(x), _ptr(y), _stream(stream)))


def hhg_stokes_residual(h, level, x, b, r, stream=None):
    _check(lib().hhg_stokes_residual(h, level, _ptr(x), _ptr(b), _ptr(r), _stream(stream)))


def hhg_stokes_precond(h, precision, r, z, nu1, nu2, stream=None):
    _check(lib().hhg_stokes_precond(h, precision, _ptr(r), _ptr(z), nu1, nu2, _stream(stream)))


def hhg_stokes_dot(h, level, a, b, out, stream=None):
    _check(lib().hhg_stokes_dot(h, level, _ptr(a), _ptr(b), _ptr(out), _stream(stream)))


def hhg_stokes_solve(h, x, b, precision=HHG_F64, rtol=1e-8, max_iters=500, nu1=2, nu2=2,
                     history=True, stream=None):
    """Returns (status, stats dict, history of the preconditioned residual
    norm)."""
    hist = np.zeros(max_iters + 1) if history else None
    o = hhg_stokes_opts(precision, rtol, max_iters, nu1, nu2,
                        hist.ctypes.data_as(_c.POINTER(_c.c_double)) if history else None,
                        len(hist) if history else 0)
    st = hhg_stokes_stats()
    rc = lib().hhg_stokes_solve(h, _c.byref(o), _ptr(x), _ptr(b), _c.byref(st), _stream(stream))
    if rc not in (HHG_OK, HHG_ENOTCONV):
        _check(rc)
    stats = {k: getattr(st, k) for k, _ in hhg_stokes_stats._fields_}
    hl = list(hist[:st.iters + 1]) if history else []
    return rc, stats, hl


def hhg_ghost_table(h, level):
    """(dst, src): field offsets of every copy slot and of the value it copies."""
    n = _i64()
    _check(lib().hhg_ghost_table(h, level, _c.byref(n), None, None))
    dst = np.zeros(n.value, dtype=np.int64)
    src = np.zeros(n.value, dtype=np.int64)
    _check(lib().hhg_ghost_table(h, level, _c.byref(n), dst.ctypes.data, src.ctypes.data))
    return dst, src


def hhg_cell_coords(h, level, n_faces):
    """Cell centroids in canonical cell order, numpy [n_faces (n-1)^2, 2]."""
    n = 2 ** level + 1
    xy = np.zeros((n_faces * (n - 1) ** 2, 2))
    _check(lib().hhg_cell_coords(h, level, xy.ctypes.data))
    return xy


def hhg_cells_from_canonical(h, level, canon, cells, stream=None):
    _check(lib().hhg_cells_from_canonical(h, level, _ptr(canon), _ptr(cells), _stream(stream)))


def hhg_cells_to_canonical(h, level, cells, canon, stream=None):
    _check(lib().hhg_cells_to_canonical(h, level, _ptr(cells), _ptr(canon), _stream(stream)))


def hhg_transport_step(h, level, x, T_in, T_out, dt, stream=None):
    _check(lib().hhg_transport_step(h, level, _ptr(x), _ptr(T_in), _ptr(T_out), float(dt),
                                    _stream(stream)))


def hhg_buoyancy(h, level, T, Ra, b, stream=None):
    _check(lib().hhg_buoyancy(h, level, _ptr(T), float(Ra), _ptr(b), _stream(stream)))


def hhg_energy_run(h, x, T, Ra, dt, steps, stokes_every=3, precision=HHG_F64, rtol=1e-8,
                   max_iters=2000, nu1=2, nu2=2, stream=None):
    """Returns (status, stats dict)."""
    so = hhg_stokes_opts(precision, rtol, max_iters, nu1, nu2, None, 0)
    o = hhg_energy_opts(so, float(Ra), float(dt), steps, stokes_every)
    st = hhg_energy_stats()
    rc = lib().hhg_energy_run(h, _c.byref(o), _ptr(x), _ptr(T), _c.byref(st), _stream(stream))
    if rc not in (HHG_OK, HHG_ENOTCONV):
        _check(rc)
    return rc, {k: getattr(st, k) for k, _ in hhg_energy_stats._fields_}


def hhg_p2_setup(h, stream=None):
    _check(lib().hhg_p2_setup(h, _stream(stream)))


def hhg_p2_apply(h, level, x, y, stream=None):
    _check(lib().hhg_p2_apply(h, level, _ptr(x), _ptr(y), _stream(stream)))


def hhg_p2_residual(h, level, x, f, r, stream=None):
    _check(lib().hhg_p2_residual(h, level, _ptr(x), _ptr(f), _ptr(r), _stream(stream)))


def hhg_p2_jacobi(h, level, omega, x, f, y, stream=None):
    _check(lib().hhg_p2_jacobi(h, level, float(omega), _ptr(x), _ptr(f), _ptr(y), _stream(stream)))


def hhg_p2_solve(h, level, x, f, rtol=1e-8, max_iters=100, nu1=3, nu2=3, vnu1=2, vnu2=2, omega=0.7,
                 history=True, stream=None):
    """Returns (status, stats dict, residual history list)."""
    hist = np.zeros(max_iters + 1) if history else None
    o = hhg_p2_opts(level, rtol, max_iters, nu1, nu2, vnu1, vnu2, omega,
                    hist.ctypes.data_as(_c.POINTER(_c.c_double)) if history else None,
                    len(hist) if history else 0)
    st = hhg_p2_stats()
    rc = lib().hhg_p2_solve(h, _c.byref(o), _ptr(x), _ptr(f), _c.byref(st), _stream(stream))
    if rc not in (HHG_OK, HHG_ENOTCONV):
        _check(rc)
    stats = {k: getattr(st, k) for k, _ in hhg_p2_stats._fields_}
    hl = list(hist[:st.iters + 1]) if history else []
    return rc, stats, hl


def hhg_apply(h, level, op, dtype, x, y, stream=None):
    _check(lib().hhg_apply(h, level, op, dtype, _ptr(x), _ptr(y), _stream(stream)))


def hhg_residual(h, level, op, dtype, u, f, r, norm=None, stream=None):
    _check(lib().hhg_residual(h, level, op, dtype, _ptr(u), _ptr(f), _ptr(r), _ptr(norm),
                              _stream(stream)))


def hhg_smooth(h, level, op, smoother, dtype, u, f, sweeps=1, backward=0, stream=None):
    _check(lib().hhg_smooth(h, level, op, smoother, dtype, _ptr(u), _ptr(f), sweeps,
                            int(backward), _stream(stream)))


def hhg_vcycle(h, level, op, smoother, dtype, u, f, nu1, nu2, stream=None):
    _check(lib().hhg_vcycle(h, level, op, smoother, dtype, _ptr(u), _ptr(f), nu1, nu2,
                            _stream(stream)))


def hhg_solve(h, u, f, mode=HHG_MODE_PLAIN_FP64, op=HHG_OP_LAPLACE, rtol=1e-8, max_iters=100,
              nu1=3, nu2=3, history=True, stream=None):
    """Returns (status, stats dict, residual history list)."""
    hist = np.zeros(max_iters + 1) if history else None
    o = hhg_solve_opts(mode, op, rtol, max_iters, nu1, nu2,
                       hist.ctypes.data_as(_c.POINTER(_c.c_double)) if history else None,
                       len(hist) if history else 0)
    st = hhg_solve_stats()
    rc = lib().hhg_solve(h, _c.byref(o), _ptr(u), _ptr(f), _c.byref(st), _stream(stream))
    if rc not in (HHG_OK, HHG_ENOTCONV):
        _check(rc)
    stats = {k: getattr(st, k) for k, _ in hhg_solve_stats._fields_}
    hl = list(hist[:st.iters + 1]) if history else []
    return rc, stats, hl


def hhg_jacobi(h, level, op, dtype, u, f, rho, stream=None):
    _check(lib().hhg_jacobi(h, level, op, dtype, _ptr(u), _ptr(f), _ptr(rho), _stream(stream)))


def hhg_dot(h, level, dtype, x, y, out, stream=None):
    _check(lib().hhg_dot(h, level, dtype, _ptr(x), _ptr(y), _ptr(out), _stream(stream)))


def hhg_axpby(h, level, dtype, alpha, x, beta, y, z, stream=None):
    _check(lib().hhg_axpby(h, level, dtype, alpha, _ptr(x), beta, _ptr(y), _ptr(z),
                           _stream(stream)))


def hhg_restrict(h, level, dtype, r, fc, stream=None):
    _check(lib().hhg_restrict(h, level, dtype, _ptr(r), _ptr(fc), _stream(stream)))


def hhg_prolong_add(h, level, dtype, uc, u, stream=None):
    _check(lib().hhg_prolong_add(h, level, dtype, _ptr(uc), _ptr(u), _stream(stream)))


def hhg_convert(h, level, src_dtype, src, dst_dtype, dst, stream=None):
    _check(lib().hhg_convert(h, level, src_dtype, _ptr(src), dst_dtype, _ptr(dst), _stream(stream)))


def hhg_net_set_weights(h, w, stream=None):
    w = np.ascontiguousarray(w, dtype=np.float32)
    _check(lib().hhg_net_set_weights(h, w.ctypes.data, len(w), _stream(stream)))


def hhg_net_get_weights(h, stream=None):
    w = np.zeros(224, dtype=np.float32)
    _check(lib().hhg_net_get_weights(h, w.ctypes.data, len(w), _stream(stream)))
    return w


def hhg_net_set_options(h, precision=HHG_BF16, accepted=0):
    _check(lib().hhg_net_set_options(h, precision, int(accepted)))


def hhg_net_forward(h, level, rho, out, stream=None):
    _check(lib().hhg_net_forward(h, level, _ptr(rho), _ptr(out), _stream(stream)))


def hhg_net_backward(h, level, rho, g, dW, stream=None):
    _check(lib().hhg_net_backward(h, level, _ptr(rho), _ptr(g), _ptr(dW), _stream(stream)))


def hhg_net_adam_step(h, grad, lr, step, stream=None):
    _check(lib().hhg_net_adam_step(h, _ptr(grad), lr, step, _stream(stream)))


def hhg_timing_enable(h, enable):
    _check(lib().hhg_timing_enable(h, int(enable)))


def hhg_timing_read(h, reset=True):
    n, ms = _i64(), _c.c_double()
    _check(lib().hhg_timing_read(h, _c.byref(n), _c.byref(ms), int(reset)))
    return n.value, ms.value
