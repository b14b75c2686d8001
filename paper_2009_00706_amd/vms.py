"""ctypes binding of libvms (argument marshalling only).

Every entry point of ``include/vms.h`` has a function of the same name here.
Device buffers are torch tensors on a ROCm device (PyTorch provides device
memory and the stream); all computation runs in the HIP library. Loading
fails loudly if ``libvms.so`` has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvms.so")

VMS_OK, VMS_EINVAL, VMS_EMESH, VMS_EHIP, VMS_ENOMEM, VMS_EOVERFLOW, VMS_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6)
VMS_FP64, VMS_MIXED_BF16, VMS_MIXED_FP16 = 0, 1, 2
VMS_INOUT_EXACT, VMS_INOUT_LEARNED, VMS_INOUT_NORMAL = 0, 1, 2
VMS_SCATTER_RECORDS, VMS_SCATTER_ATOMIC = 0, 1
VMS_RELABEL = 1
VMS_KSP_BCGS, VMS_KSP_GMRES = 0, 1
VMS_SOLVE_DIRICHLET = 1
VMS_EXPORT_SURFGP = 8
VMS_EXPORT_NODE_ROW_PTR, VMS_EXPORT_NODE_COL = 9, 10
(VMS_EXPORT_NODE_XYZ, VMS_EXPORT_ROW_PTR, VMS_EXPORT_COL_IDX, VMS_EXPORT_MARKERS,
 VMS_EXPORT_VERTEX_LAB, VMS_EXPORT_SUBGP, VMS_EXPORT_MASTERS) = range(1, 8)

EXPORTED = ["vms_create", "vms_sizes", "vms_export", "vms_assemble", "vms_apply",
            "vms_apply_jacobian", "vms_spmv", "vms_solve", "vms_dirichlet_nodes", "vms_dirichlet_in_nodes",
            "vms_set_weak_bc", "vms_element_weights",
            "inout_classify",
            "inout_prepare", "inout_classify_prepared", "inout_release", "vms_stats",
            "inout_classify_static", "inout_static_last_error", "inout_reserve",
            "vms_set_inout", "vms_relabel_stats", "vms_batch_set_order",
            "vms_q2_create", "vms_q2_sizes", "vms_q2_export", "vms_q2_assemble", "vms_q2_last_error",
            "vms_q2_last_timing",
            "vms_q2_destroy",
            "vms_mesh_create", "vms_mesh_sizes", "vms_mesh_export", "vms_mesh_destroy",
            "vms_set_timing", "vms_last_timing", "vms_set_overlap", "vms_set_scatter", "vms_components", "vms_surface_components", "vms_mlp_create", "vms_mlp_get_params",
            "vms_mlp_set_margin", "vms_mlp_set_margin_grid", "vms_mlp_grad", "vms_mlp_train", "vms_mlp_adam_step",
            "vms_mlp_predict", "vms_mlp_last_error", "vms_mlp_destroy", "vms_sdf_sample",
            "vms_batch_create", "vms_batch_set_config", "vms_batch_get_config",
            "vms_batch_use_graph", "vms_batch_assemble", "vms_batch_autotune", "vms_batch_last_timing",
            "vms_batch_destroy", "vms_last_error", "vms_destroy"]


class VmsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libvms error {code}: {msg}")
        self.code = code


class Octree(C.Structure):
    _fields_ = [("n_oct", C.c_int64), ("ax", C.c_void_p), ("ay", C.c_void_p), ("az", C.c_void_p),
                ("level", C.c_void_p), ("max_level", C.c_int32), ("pad", C.c_int32),
                ("origin", C.c_double * 3), ("root_len", C.c_double)]


class Surface(C.Structure):
    _fields_ = [("n_vert", C.c_int32), ("n_tri", C.c_int32), ("verts", C.c_void_p),
                ("tri", C.c_void_p), ("body_id", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("rho", C.c_double), ("mu", C.c_double), ("dt", C.c_double),
                ("theta", C.c_double), ("c_t", C.c_double), ("c_i", C.c_double),
                ("quad_depth", C.c_int32), ("precision", C.c_uint32),
                ("inout_mode", C.c_uint32), ("learned_min_bt", C.c_int32)]


class Fields(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("ux", "uy", "uz", "p", "ux0", "uy0", "uz0")]


_lib = None


def lib():
    """Load libvms.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2009_00706_amd/build.py")
        L = C.CDLL(LIB_PATH)
        p, i64, i32, u32 = C.c_void_p, C.c_int64, C.c_int32, C.c_uint32
        L.vms_create.argtypes = [C.POINTER(p), C.POINTER(Octree), C.POINTER(Surface),
                                 C.POINTER(Params), p]
        L.vms_sizes.argtypes = [p, p, p, p, p]
        L.vms_export.argtypes = [p, u32, p]
        L.vms_assemble.argtypes = [p, C.POINTER(Fields), p, p, u32]
        L.vms_apply.argtypes = [p, C.POINTER(Fields), p, p]
        L.vms_apply_jacobian.argtypes = [p, C.POINTER(Fields), p, p]
        L.vms_spmv.argtypes = [p, p, p, p]
        L.vms_dirichlet_nodes.argtypes = [p, C.POINTER(C.c_int64), p]
        L.vms_dirichlet_in_nodes.argtypes = [p, p, p]
        L.vms_solve.argtypes = [p, p, C.POINTER(Fields), p, p, C.c_int, C.c_int, C.c_int, C.c_double,
                                C.c_uint32, C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.vms_set_weak_bc.argtypes = [p, C.c_int, C.c_double, p]
        L.vms_element_weights.argtypes = [p, C.c_double, p]
        L.inout_classify.argtypes = [C.POINTER(Surface), p, p, p, i64, p, u32, p, p]
        L.inout_prepare.argtypes = [C.POINTER(Surface), p, C.POINTER(p)]
        L.inout_classify_prepared.argtypes = [p, p, p, p, i64, p, u32, p]
        L.inout_release.argtypes = [p]
        L.inout_release.restype = None
        L.vms_q2_create.argtypes = [C.POINTER(p), C.POINTER(Octree), C.POINTER(Params), p]
        L.vms_q2_create.restype = C.c_int
        L.vms_q2_sizes.argtypes = [p, p, p, p]
        L.vms_q2_sizes.restype = C.c_int
        L.vms_q2_export.argtypes = [p, u32, p]
        L.vms_q2_export.restype = C.c_int
        L.vms_q2_assemble.argtypes = [p, C.POINTER(Fields), p, p]
        L.vms_q2_assemble.restype = C.c_int
        L.vms_q2_last_timing.argtypes = [p, p]
        L.vms_q2_last_timing.restype = C.c_int
        L.vms_q2_last_error.argtypes = [p]
        L.vms_q2_last_error.restype = C.c_char_p
        L.vms_q2_destroy.argtypes = [p]
        L.vms_q2_destroy.restype = None
        L.vms_set_inout.argtypes = [p, u32, p, i32]
        L.vms_set_inout.restype = C.c_int
        L.vms_relabel_stats.argtypes = [p, p]
        L.vms_relabel_stats.restype = C.c_int
        L.vms_set_overlap.argtypes = [p, C.c_int]
        L.vms_set_overlap.restype = C.c_int
        L.vms_set_scatter.argtypes = [p, u32]
        L.vms_set_scatter.restype = C.c_int
        L.vms_components.argtypes = [p, p, p]
        L.vms_components.restype = C.c_int
        L.vms_surface_components.argtypes = [C.POINTER(Surface), p, p]
        L.vms_surface_components.restype = C.c_int
        L.inout_reserve.argtypes = [p, i64]
        L.inout_reserve.restype = C.c_int
        L.inout_classify_static.argtypes = [C.POINTER(Surface), p, p, p, i64, p, p]
        L.inout_classify_static.restype = C.c_int
        L.inout_static_last_error.argtypes = []
        L.inout_static_last_error.restype = C.c_char_p
        L.vms_stats.argtypes = [p, p]
        L.vms_mesh_create.argtypes = [C.POINTER(p), C.POINTER(Octree), p]
        L.vms_mesh_sizes.argtypes = [p, p, p, p]
        L.vms_mesh_export.argtypes = [p, u32, p]
        L.vms_mesh_destroy.argtypes = [p]
        L.vms_mesh_destroy.restype = None
        L.vms_mlp_create.argtypes = [C.POINTER(p), p, p, p, p, C.c_float, p]
        L.vms_mlp_get_params.argtypes = [p, p]
        L.vms_mlp_set_margin.argtypes = [p, C.c_float]
        L.vms_mlp_set_margin_grid.argtypes = [p, C.c_int, C.c_int, C.c_int, p]
        L.vms_mlp_grad.argtypes = [p, p, p, p, p, i64, p, p]
        L.vms_mlp_train.argtypes = [p, p, p, p, p, i64, C.c_int, C.c_int, C.c_float, p]
        L.vms_mlp_adam_step.argtypes = [p, p, C.c_float]
        L.vms_mlp_predict.argtypes = [p, p, p, p, i64, p]
        L.vms_mlp_last_error.argtypes = []
        L.vms_mlp_last_error.restype = C.c_char_p
        L.vms_mlp_destroy.argtypes = [p]
        L.vms_mlp_destroy.restype = None
        L.vms_sdf_sample.argtypes = [p, p, p, p, i64, C.c_double, p]
        L.vms_batch_create.argtypes = [C.POINTER(p), p, C.c_int, p]
        L.vms_batch_set_config.argtypes = [p, C.c_int, C.c_int]
        L.vms_batch_get_config.argtypes = [p, p, p, p]
        L.vms_batch_set_order.argtypes = [p, C.c_int]
        L.vms_batch_set_order.restype = C.c_int
        L.vms_batch_use_graph.argtypes = [p, C.c_int]
        L.vms_batch_assemble.argtypes = [p, p, p, p]
        L.vms_batch_autotune.argtypes = [p, p, p, p, p]
        L.vms_batch_last_timing.argtypes = [p, p]
        L.vms_batch_destroy.argtypes = [p]
        L.vms_batch_destroy.restype = None
        L.vms_set_timing.argtypes = [p, C.c_int]
        L.vms_last_timing.argtypes = [p, p]
        L.vms_last_error.argtypes = [p]
        L.vms_last_error.restype = C.c_char_p
        L.vms_destroy.argtypes = [p]
        L.vms_destroy.restype = None
        for n in ("vms_create", "vms_sizes", "vms_export", "vms_assemble", "vms_apply",
                  "inout_classify", "inout_prepare", "inout_classify_prepared", "vms_stats",
                  "vms_mesh_create", "vms_mesh_sizes", "vms_mesh_export", "vms_set_timing",
                  "vms_last_timing", "vms_mlp_create", "vms_mlp_get_params", "vms_mlp_set_margin",
                  "vms_mlp_set_margin_grid",
                  "vms_mlp_grad", "vms_mlp_train", "vms_mlp_adam_step", "vms_mlp_predict",
                  "vms_sdf_sample", "vms_batch_create", "vms_batch_set_config",
                  "vms_batch_get_config", "vms_batch_use_graph", "vms_batch_assemble",
                  "vms_batch_autotune", "vms_batch_last_timing"):
            getattr(L, n).restype = C.c_int
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != VMS_OK:
        raise VmsError(rc, lib().vms_last_error(ctx).decode())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def make_surface(verts, tris, body_id=None):
    v = _np(verts, np.float64).reshape(-1, 3)
    t = _np(tris, np.int32).reshape(-1, 3)
    b = None if body_id is None else _np(body_id, np.int32).reshape(-1)
    s = Surface(v.shape[0], t.shape[0], v.ctypes.data, t.ctypes.data, None if b is None else b.ctypes.data)
    s._keep = (v, t, b)
    return s


def make_params(rho=1.0, mu=0.01, dt=0.01, theta=0.5, c_t=4.0, c_i=36.0, quad_depth=3,
                precision=VMS_FP64, inout_mode=VMS_INOUT_EXACT, learned_min_bt=0):
    return Params(rho, mu, dt, theta, c_t, c_i, quad_depth, precision, inout_mode, learned_min_bt)


# ---------------------------------------------------------------------------
# entry points (same names as the C-ABI)
# ---------------------------------------------------------------------------


def vms_create(tree, surf=None, params=None, stream=None):
    """tree: object with ax, ay, az, level, max_level, origin, root_len (host arrays);
    surf: object with verts (n,3), tris (m,3) or None. Returns the context handle."""
    o = _octree(tree)
    s = make_surface(surf.verts, surf.tris, getattr(surf, "body_id", None)) if surf is not None else None
    prm = params if params is not None else make_params()
    h = C.c_void_p()
    rc = lib().vms_create(C.byref(h), C.byref(o), C.byref(s) if s is not None else None,
                          C.byref(prm), _stream(stream))
    _check(rc, None)
    return h


def _octree(tree):
    ax, ay, az = (_np(a, np.int32) for a in (tree.ax, tree.ay, tree.az))
    lv = _np(tree.level, np.uint8)
    o = Octree(ax.shape[0], ax.ctypes.data, ay.ctypes.data, az.ctypes.data, lv.ctypes.data,
               int(tree.max_level), 0, (C.c_double * 3)(*tree.origin), float(tree.root_len))
    o._keep = (ax, ay, az, lv)
    return o


def vms_mesh_create(tree, markers=None):
    o = _octree(tree)
    mk = _np(markers, np.uint8) if markers is not None else None
    h = C.c_void_p()
    _check(lib().vms_mesh_create(C.byref(h), C.byref(o), mk.ctypes.data if mk is not None else None),
           None)
    return h


def vms_mesh_sizes(h):
    v = (C.c_int64 * 3)()
    _check(lib().vms_mesh_sizes(h, C.byref(v, 0), C.byref(v, 8), C.byref(v, 16)), None)
    return {"n_nodes": v[0], "nnz": v[1], "n_hanging": v[2]}


def vms_mesh_export(h, what, n_oct=None):
    sz = vms_mesh_sizes(h)
    shapes = {VMS_EXPORT_NODE_XYZ: ((3, sz["n_nodes"]), np.int32),
              VMS_EXPORT_ROW_PTR: ((4 * sz["n_nodes"] + 1,), np.int64),
              VMS_EXPORT_COL_IDX: ((sz["nnz"],), np.int32),
              VMS_EXPORT_MASTERS: ((n_oct, 8), np.int32)}
    shp, dt = shapes[what]
    out = np.zeros(shp, dt)
    _check(lib().vms_mesh_export(h, what, out.ctypes.data), None)
    return out


def vms_mesh_destroy(h):
    lib().vms_mesh_destroy(h)


def vms_sizes(ctx):
    v = (C.c_int64 * 4)()
    _check(lib().vms_sizes(ctx, C.byref(v, 0), C.byref(v, 8), C.byref(v, 16), C.byref(v, 24)), ctx)
    return {"n_nodes": v[0], "n_rows": v[1], "nnz": v[2], "n_subgp": v[3]}


def vms_stats(ctx):
    v = (C.c_int64 * 7)()
    _check(lib().vms_stats(ctx, v), ctx)
    return {"n_out": v[0], "n_intercepted": v[1], "n_labelled": v[2], "n_degenerate": v[3],
            "n_hanging": v[4], "n_subgp": v[5], "n_surfgp": v[6]}


def _q2_check(rc, q):
    if rc != VMS_OK:
        raise VmsError(rc, lib().vms_q2_last_error(q).decode())


def vms_q2_create(tree, params=None, stream=None):
    """Triquadratic elements of a uniform octree (no body); returns the handle."""
    o = _octree(tree)
    prm = params if params is not None else make_params()
    h = C.c_void_p()
    _q2_check(lib().vms_q2_create(C.byref(h), C.byref(o), C.byref(prm), _stream(stream)), None)
    return h


def vms_q2_sizes(q):
    v = [C.c_int64() for _ in range(3)]
    _q2_check(lib().vms_q2_sizes(q, *(C.byref(x) for x in v)), q)
    return {"n_nodes": v[0].value, "n_rows": v[1].value, "nnz": v[2].value}


def vms_q2_export(q, what):
    sz = vms_q2_sizes(q)
    if what == VMS_EXPORT_NODE_XYZ:
        out = np.zeros((3, sz["n_nodes"]), np.int32)
    elif what == VMS_EXPORT_ROW_PTR:
        out = np.zeros(sz["n_rows"] + 1, np.int64)
    elif what == VMS_EXPORT_COL_IDX:
        out = np.zeros(sz["nnz"], np.int32)
    else:
        raise ValueError("unknown selector")
    _q2_check(lib().vms_q2_export(q, what, out.ctypes.data), q)
    return out


def vms_q2_assemble(q, fields, vals, resid=None):
    fs = _fields(fields)
    _q2_check(lib().vms_q2_assemble(q, C.byref(fs), _ptr(vals), _ptr(resid) if resid is not None else None), q)


def vms_q2_last_timing(q):
    v = (C.c_float * 2)()
    _q2_check(lib().vms_q2_last_timing(q, v), q)
    return list(v)


def vms_q2_destroy(q):
    lib().vms_q2_destroy(q)


def vms_set_inout(ctx, mode, mlp=None, min_bt=0):
    """In-out test of the sub-cell quadrature on relabel: exact, or the learned
    filter (a vms_mlp handle) on elements with at least min_bt background triangles."""
    m = C.c_void_p(mlp.value if isinstance(mlp, C.c_void_p) else mlp) if mlp else None
    _check(lib().vms_set_inout(ctx, int(mode), m, int(min_bt)), ctx)


def vms_relabel_stats(ctx):
    v = (C.c_int64 * 2)()
    _check(lib().vms_relabel_stats(ctx, v), ctx)
    return {"candidates": v[0], "exact_in_last_relabel": v[1]}


def vms_element_weights(ctx, n_oct, ts_over_tv):
    """Per-element weights of eq. (Wpart) (host array of n_oct doubles)."""
    w = np.zeros(n_oct, np.float64)
    _check(lib().vms_element_weights(ctx, float(ts_over_tv), w.ctypes.data), ctx)
    return w


def vms_set_weak_bc(ctx, enable=True, c_b=4.0, g=(0.0, 0.0, 0.0)):
    """Weak (Nitsche) boundary terms on the immersed surface (see include/vms.h)."""
    gg = (C.c_double * 3)(*[float(x) for x in g])
    _check(lib().vms_set_weak_bc(ctx, int(bool(enable)), float(c_b), gg), ctx)


def vms_export(ctx, what, n_oct=None):
    sz = vms_sizes(ctx)
    if what == VMS_EXPORT_NODE_XYZ:
        out = np.zeros((3, sz["n_nodes"]), np.int32)
    elif what == VMS_EXPORT_ROW_PTR:
        out = np.zeros(sz["n_rows"] + 1, np.int64)
    elif what == VMS_EXPORT_COL_IDX:
        out = np.zeros(sz["nnz"], np.int32)
    elif what == VMS_EXPORT_NODE_ROW_PTR:
        out = np.zeros(sz["n_nodes"] + 1, np.int64)
    elif what == VMS_EXPORT_NODE_COL:
        out = np.zeros(sz["nnz"] // 16, np.int32)
    elif what == VMS_EXPORT_MARKERS:
        out = np.zeros(n_oct, np.uint8)
    elif what == VMS_EXPORT_VERTEX_LAB:
        out = np.zeros((n_oct, 8), np.uint8)
    elif what == VMS_EXPORT_MASTERS:
        out = np.zeros((n_oct, 8), np.int32)
    elif what == VMS_EXPORT_SURFGP:
        n = vms_stats(ctx)["n_surfgp"]
        raw = np.zeros(n * 64 + 8, np.uint8)
        _check(lib().vms_export(ctx, what, raw.ctypes.data), ctx)
        return {"el": raw[:8 * n].view(np.int64).copy(),
                "xi": raw[8 * n:32 * n].view(np.float64).reshape(n, 3).copy(),
                "w": raw[32 * n:40 * n].view(np.float64).copy(),
                "n": raw[40 * n:64 * n].view(np.float64).reshape(n, 3).copy()}
    elif what == VMS_EXPORT_SUBGP:
        n = sz["n_subgp"]
        raw = np.zeros(n * 37 + 8, np.uint8)
        _check(lib().vms_export(ctx, what, raw.ctypes.data), ctx)
        return {"el": raw[:8 * n].view(np.int64).copy(),
                "key": raw[8 * n:12 * n].view(np.int32).copy(),
                "lvl": raw[12 * n:13 * n].copy(),
                "xyz": raw[13 * n:37 * n].view(np.float64).reshape(n, 3).copy()}
    else:
        raise ValueError(what)
    _check(lib().vms_export(ctx, what, out.ctypes.data), ctx)
    return out


def _fields(f):
    return Fields(*[f[k].data_ptr() for k in ("ux", "uy", "uz", "p", "ux0", "uy0", "uz0")])


def vms_assemble(ctx, fields, csr_vals, resid=None, flags=0):
    """fields: dict of 7 float64 device tensors; csr_vals: device tensor (nnz)."""
    fs = _fields(fields)
    _check(lib().vms_assemble(ctx, C.byref(fs), _ptr(csr_vals), _ptr(resid), flags), ctx)


def vms_apply(ctx, fields, resid, want_norm=False):
    fs = _fields(fields)
    nrm = C.c_double(0.0)
    _check(lib().vms_apply(ctx, C.byref(fs), _ptr(resid), C.byref(nrm) if want_norm else None), ctx)
    return nrm.value if want_norm else None


def vms_apply_jacobian(ctx, fields, x, y):
    """y = J(fields) x, matrix-free (device tensors of n_rows doubles)."""
    fs = _fields(fields)
    _check(lib().vms_apply_jacobian(ctx, C.byref(fs), _ptr(x), _ptr(y)), ctx)


def vms_spmv(ctx, vals, x, y):
    """y = A x with the context's CSR pattern and values vals (device tensors)."""
    _check(lib().vms_spmv(ctx, _ptr(vals), _ptr(x), _ptr(y)), ctx)


def vms_dirichlet_nodes(ctx):
    """Sorted ids of the CG nodes of IN elements (int32 numpy array)."""
    n = C.c_int64(0)
    _check(lib().vms_dirichlet_nodes(ctx, C.byref(n), None), ctx)
    out = np.zeros(n.value, np.int32)
    _check(lib().vms_dirichlet_nodes(ctx, C.byref(n), out.ctypes.data_as(C.c_void_p)), ctx)
    return out


def vms_dirichlet_in_nodes(ctx, vals, resid=None):
    """Identity rows (and zero residual entries) at the CG nodes of IN elements."""
    _check(lib().vms_dirichlet_in_nodes(ctx, _ptr(vals), _ptr(resid)), ctx)


def vms_solve(ctx, vals, b, x, fields=None, method=VMS_KSP_BCGS, restart=30, max_iter=1000, rtol=1e-6,
              flags=0):
    """Krylov solve of A x = b (device tensors of n_rows doubles; x: initial
    guess in, iterate out); A is the assembled matrix with values vals, or the
    matrix-free Jacobian action at fields. Returns (steps, true relative residual)."""
    it, rr = C.c_int(0), C.c_double(0.0)
    fs = C.byref(_fields(fields)) if fields is not None else None
    _check(lib().vms_solve(ctx, _ptr(vals), fs, _ptr(b), _ptr(x), int(method), int(restart), int(max_iter),
                           float(rtol), int(flags), C.byref(it), C.byref(rr)), ctx)
    return it.value, rr.value


def inout_classify(surf, px, py, pz, labels, mode=VMS_INOUT_EXACT, mlp=None, stream=None):
    s = make_surface(surf.verts, surf.tris)
    rc = lib().inout_classify(C.byref(s), _ptr(px), _ptr(py), _ptr(pz), px.numel(), _ptr(labels),
                              mode, C.c_void_p(mlp) if mlp else None, _stream(stream))
    _check(rc, None)


def inout_classify_static(surf, px, py, pz, labels, stream=None):
    """Exact labels with the surface staged in the library's static device
    array (no device allocation)."""
    s = make_surface(surf.verts, surf.tris)
    rc = lib().inout_classify_static(C.byref(s), _ptr(px), _ptr(py), _ptr(pz), px.numel(), _ptr(labels),
                                     _stream(stream))
    if rc != VMS_OK:
        raise VmsError(rc, lib().inout_static_last_error().decode())


def inout_prepare(surf, stream=None):
    s = make_surface(surf.verts, surf.tris)
    h = C.c_void_p()
    _check(lib().inout_prepare(C.byref(s), _stream(stream), C.byref(h)), None)
    return h


def inout_classify_prepared(h, px, py, pz, labels, mode=VMS_INOUT_EXACT, mlp=None):
    rc = lib().inout_classify_prepared(h, _ptr(px), _ptr(py), _ptr(pz), px.numel(), _ptr(labels),
                                       mode, C.c_void_p(mlp) if mlp else None)
    _check(rc, None)


def inout_reserve(h, n):
    _check(lib().inout_reserve(h, int(n)), None)


def inout_release(h):
    lib().inout_release(h)


def vms_set_overlap(ctx, on=True):
    """Overlapped (default) or in-order schedule of the matrix assembly (same outputs)."""
    _check(lib().vms_set_overlap(ctx, 1 if on else 0), ctx)


def vms_components(ctx):
    """(n_comp, convex flags) of the context's surface bodies."""
    n = C.c_int32(0)
    _check(lib().vms_components(ctx, C.byref(n), None), ctx)
    cv = np.zeros(max(n.value, 1), np.uint8)
    _check(lib().vms_components(ctx, C.byref(n), cv.ctypes.data), ctx)
    return n.value, cv[:n.value].astype(bool)


def vms_surface_components(surf):
    """Body index of every triangle (body_id groups or connected pieces), host only."""
    s = make_surface(surf.verts, surf.tris, getattr(surf, "body_id", None))
    comp = np.zeros(s.n_tri, np.int32)
    n = C.c_int32(0)
    _check(lib().vms_surface_components(C.byref(s), comp.ctypes.data, C.byref(n)), None)
    return comp, n.value


def vms_set_scatter(ctx, mode):
    """VMS_SCATTER_RECORDS (fixed summation order, default) or VMS_SCATTER_ATOMIC."""
    _check(lib().vms_set_scatter(ctx, int(mode)), ctx)


def vms_set_timing(ctx, on=True):
    _check(lib().vms_set_timing(ctx, 1 if on else 0), ctx)


def vms_last_timing(ctx):
    """ms of the last call: relabel, argument set-up (empty), OUT-element kernel, INTERCEPTED kernel,
    CSR summation (with identity rows). After an overlapped assembly the first and fourth ran on the
    second stream beside the fifth, which spans from the end of the OUT kernel to the end of the call."""
    v = (C.c_float * 5)()
    _check(lib().vms_last_timing(ctx, v), ctx)
    return list(v)


def _mcheck(rc):
    if rc != VMS_OK:
        raise VmsError(rc, lib().vms_mlp_last_error().decode())


def vms_mlp_create(lo, hi, theta, B, trunc, stream=None):
    lo = _np(lo, np.float64); hi = _np(hi, np.float64)
    th = _np(theta, np.float32); Bm = _np(B, np.float32)
    h = C.c_void_p()
    _mcheck(lib().vms_mlp_create(C.byref(h), lo.ctypes.data, hi.ctypes.data, th.ctypes.data,
                                 Bm.ctypes.data, float(trunc), _stream(stream)))
    return h


def vms_mlp_get_params(h):
    out = np.zeros(12545, np.float32)
    _mcheck(lib().vms_mlp_get_params(h, out.ctypes.data))
    return out


def vms_mlp_set_margin(h, m):
    _mcheck(lib().vms_mlp_set_margin(h, float(m)))


def vms_mlp_set_margin_grid(h, margins):
    """margins: host array (nz, ny, nx) of per-cell margins, or None to remove."""
    if margins is None:
        _mcheck(lib().vms_mlp_set_margin_grid(h, 0, 0, 0, None))
        return
    m = np.ascontiguousarray(margins, np.float32)
    nz, ny, nx = m.shape
    _mcheck(lib().vms_mlp_set_margin_grid(h, nx, ny, nz, m.ctypes.data))


def vms_mlp_grad(h, px, py, pz, sdf, grad=None):
    loss = C.c_double(0)
    _mcheck(lib().vms_mlp_grad(h, _ptr(px), _ptr(py), _ptr(pz), _ptr(sdf), px.numel(), _ptr(grad),
                               C.byref(loss)))
    return loss.value


def vms_mlp_train(h, px, py, pz, sdf, steps, batch, lr):
    loss = C.c_double(0)
    _mcheck(lib().vms_mlp_train(h, _ptr(px), _ptr(py), _ptr(pz), _ptr(sdf), px.numel(), int(steps),
                                int(batch), float(lr), C.byref(loss)))
    return loss.value


def vms_mlp_adam_step(h, grad, lr):
    _mcheck(lib().vms_mlp_adam_step(h, _ptr(grad), float(lr)))


def vms_mlp_predict(h, px, py, pz, pred):
    _mcheck(lib().vms_mlp_predict(h, _ptr(px), _ptr(py), _ptr(pz), px.numel(), _ptr(pred)))


def vms_mlp_destroy(h):
    lib().vms_mlp_destroy(h)


def vms_sdf_sample(h, px, py, pz, trunc, sdf):
    _check(lib().vms_sdf_sample(h, _ptr(px), _ptr(py), _ptr(pz), px.numel(), float(trunc), _ptr(sdf)),
           None)


def vms_batch_create(ctxs, stream=None):
    arr = (C.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    h = C.c_void_p()
    _check(lib().vms_batch_create(C.byref(h), arr, len(ctxs), _stream(stream)), None)
    h._keep = arr
    return h


def vms_batch_set_config(b, tile, groups_per_cu):
    _check(lib().vms_batch_set_config(b, int(tile), int(groups_per_cu)), None)


def vms_batch_get_config(b):
    t, g, n = C.c_int(), C.c_int(), C.c_int64()
    _check(lib().vms_batch_get_config(b, C.byref(t), C.byref(g), C.byref(n)), None)
    return {"tile": t.value, "groups_per_cu": g.value, "n_units": n.value}


def vms_batch_set_order(b, by_weight=True):
    _check(lib().vms_batch_set_order(b, 1 if by_weight else 0), None)


def vms_batch_use_graph(b, on=True):
    _check(lib().vms_batch_use_graph(b, 1 if on else 0), None)


def _batch_arrays(fields, vals, resid):
    fa = (Fields * len(fields))(*[_fields(f) for f in fields])
    va = (C.c_void_p * len(vals))(*[v.data_ptr() for v in vals])
    ra = (C.c_void_p * len(vals))(*[(r.data_ptr() if r is not None else None) for r in resid]) \
        if resid is not None else None
    return fa, va, ra


def vms_batch_assemble(b, fields, vals, resid=None):
    fa, va, ra = _batch_arrays(fields, vals, resid)
    _check(lib().vms_batch_assemble(b, fa, va, ra), None)


def vms_batch_autotune(b, fields, vals, resid=None):
    fa, va, ra = _batch_arrays(fields, vals, resid)
    ms = C.c_float(0)
    _check(lib().vms_batch_autotune(b, fa, va, ra, C.byref(ms)), None)
    return ms.value


def vms_batch_last_timing(b):
    """ms of the last eager batched call: empty interval, persistent kernel, record summations."""
    ms = (C.c_float * 3)()
    _check(lib().vms_batch_last_timing(b, ms), None)
    return list(ms)


def vms_batch_destroy(b):
    lib().vms_batch_destroy(b)


def vms_last_error(ctx=None):
    return lib().vms_last_error(ctx).decode()


def vms_destroy(ctx):
    lib().vms_destroy(ctx)


# ---------------------------------------------------------------------------
# convenience wrapper used by tests and the benchmark
# ---------------------------------------------------------------------------


class Assembler:
    """One context plus its device outputs; fields are given as host arrays."""

    def __init__(self, tree, surf=None, params=None, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.params = params if params is not None else make_params()
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.ctx = vms_create(tree, surf, self.params, self.stream.cuda_stream)
        self.sizes = vms_sizes(self.ctx)
        self.n_oct = tree.ax.shape[0]
        fp64 = self.params.precision == VMS_FP64
        self.vals = torch.zeros(self.sizes["nnz"], dtype=torch.float64 if fp64 else torch.float32,
                                device=self.device)
        self.resid = torch.zeros(self.sizes["n_rows"], dtype=torch.float64, device=self.device)
        self.fields = None

    def set_fields(self, f):
        t = self.torch
        self.fields = {k: t.as_tensor(np.ascontiguousarray(f[k], np.float64), device=self.device)
                       for k in ("ux", "uy", "uz", "p", "ux0", "uy0", "uz0")}

    def assemble(self, flags=0, resid=True):
        vms_assemble(self.ctx, self.fields, self.vals, self.resid if resid else None, flags)

    def apply(self, want_norm=False):
        return vms_apply(self.ctx, self.fields, self.resid, want_norm)

    def jacobian_action(self, x, y=None):
        """y = J x without the matrix (x: device float64 tensor of n_rows)."""
        if y is None:
            y = self.torch.empty_like(x)
        vms_apply_jacobian(self.ctx, self.fields, x, y)
        return y

    def set_weak_bc(self, enable=True, c_b=4.0, g=(0.0, 0.0, 0.0)):
        vms_set_weak_bc(self.ctx, enable, c_b, g)

    def spmv(self, x, y=None):
        """y = A x with the values of the last assemble."""
        if y is None:
            y = self.torch.empty_like(x)
        vms_spmv(self.ctx, self.vals, x, y)
        return y

    def apply_dirichlet(self, resid=True):
        """Dirichlet rows at the CG nodes of IN elements in the current values
        (and residual)."""
        vms_dirichlet_in_nodes(self.ctx, self.vals, self.resid if resid else None)

    def solve(self, b, x=None, matrix_free=False, method=VMS_KSP_BCGS, restart=30, max_iter=1000,
              rtol=1e-6, dirichlet=True):
        """Solve J x = b with the last assembled values (preconditioner, and the
        operator unless matrix_free; dirichlet: the values carry the Dirichlet
        rows of apply_dirichlet, which the matrix-free operator then copies);
        returns (x, steps, true relative residual)."""
        if x is None:
            x = self.torch.zeros_like(b)
        it, rr = vms_solve(self.ctx, self.vals, b, x, self.fields if matrix_free else None, method,
                           restart, max_iter, rtol, VMS_SOLVE_DIRICHLET if dirichlet else 0)
        return x, it, rr

    def export(self, what):
        return vms_export(self.ctx, what, self.n_oct)

    def close(self):
        if self.ctx:
            vms_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
