"""ctypes binding of libfmbem.so (argument marshalling only).

Every computation runs in the HIP library; this module only checks tensor
dtypes, shapes, devices and contiguity, and passes raw pointers and the
current torch stream.  If the library has not been built the import fails
loudly: there is no fallback.
"""

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmbem.so")

FMB_OK, FMB_EINVAL, FMB_ENOMEM, FMB_EDEVICE, FMB_ENOCONV, FMB_EBREAKDOWN, FMB_ENONFINITE, FMB_ENOTIMPL = range(8)
# largest target count of bem_field_noalloc (FMB_FIELD_NOALLOC_MAX_TARGETS in the header)
FIELD_NOALLOC_MAX = 65536
FMB_FP64, FMB_FP32 = 0, 1
CORR = {"none": 0, "mean": 1, "linear": 2}


class FmbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("fmbem error %d: %s" % (code, msg))
        self.code = code


class PlanOpts(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("precision", ctypes.c_int32), ("nrhs_max", ctypes.c_int32),
                ("corr_mode", ctypes.c_int32), ("point_tri", ctypes.c_void_p), ("tri_vertices", ctypes.c_void_p),
                ("ntri", ctypes.c_int64), ("leaf_target", ctypes.c_int32), ("translate_mode", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("tol", ctypes.c_double), ("far_cutoff", ctypes.c_double)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("order", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("nrhs_max", ctypes.c_int32), ("n", ctypes.c_int64), ("nbox", ctypes.c_int64 * 16),
                ("m2l_pairs", ctypes.c_int64 * 16), ("p2p_pairs", ctypes.c_int64),
                ("corr_blocks", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("order_level", ctypes.c_int32 * 16), ("far_lmin", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class GmresOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int32), ("maxit", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("x0_given", ctypes.c_int32), ("mixed", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("inner_maxit", ctypes.c_int32), ("serial", ctypes.c_int32),
                ("adjoint", ctypes.c_int32), ("inner_reorth", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class GmresInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("refinements", ctypes.c_int32), ("matvecs64", ctypes.c_int32),
                ("matvecs32", ctypes.c_int32), ("fp64_fallback", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("residual", ctypes.c_double), ("history", ctypes.c_double * 256)]


EXPORTS = [
    "fmb_plan_opts_default", "fmm_plan", "fmm_matvec", "fmm_matvec_adjoint", "fmm_plan_info",
    "fmm_plan_export_tree", "fmm_plan_destroy", "fmm_plan_profile", "fmm_plan_profile_read", "fmb_gmres_opts_default", "bem_problem_create", "bem_problem_create_multi", "bem_problem_create_ibc", "bem_problem_use_graphs", "bem_apply", "bem_apply32", "bem_apply_adjoint",
    "bem_precond_apply", "bem_rhs_planewave", "bem_field", "bem_field_noalloc", "bem_field_fmm", "bem_far_field_adjoint", "bem_shape_pairs", "bem_self_blocks", "gmres_solve", "gmres_solve_group", "bem_problem_destroy", "fmb_last_error",
]

_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfmbem.so is not built (run __graft_entry__.build() or "
                          "python -m paper_1211_7177_amd.build); no fallback exists")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.fmb_last_error.restype = ctypes.c_char_p
    lib.fmb_last_error.argtypes = []
    sig = {
        "fmb_plan_opts_default": [vp],
        "fmm_plan": [vp, vp, vp, i64, f64, f64, i32, vp, vp, vp],
        "fmm_matvec": [vp, vp, vp, vp, i32, vp],
        "fmm_matvec_adjoint": [vp, vp, vp, vp, i32, vp],
        "fmm_plan_info": [vp, vp],
        "fmm_plan_export_tree": [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp],
        "fmm_plan_destroy": [vp],
        "fmm_plan_profile": [vp, i32],
        "fmm_plan_profile_read": [vp, vp, vp, i32],
        "fmb_gmres_opts_default": [vp],
        "bem_problem_create": [vp, vp, vp, vp, vp, vp, vp, vp],
        "bem_problem_create_ibc": [vp, vp, vp, vp, vp],
        "bem_problem_create_multi": [vp, vp, i32, vp, vp, vp, vp, vp, vp, vp],
        "bem_problem_use_graphs": [vp, i32],
        "bem_apply_adjoint": [vp, vp, vp, i32, vp],
        "bem_apply": [vp, vp, vp, i32, vp],
        "bem_apply32": [vp, vp, vp, i32, vp],
        "bem_precond_apply": [vp, vp, vp, i32, vp],
        "bem_rhs_planewave": [vp, vp, vp, vp, i32, vp],
        "gmres_solve": [vp, vp, vp, i32, vp, vp, vp],
        "gmres_solve_group": [vp, i32, vp, vp, vp, vp, vp, vp],
        "bem_field": [vp, vp, i32, vp, ctypes.c_int64, i32, i32, vp, vp],
        "bem_field_noalloc": [vp, vp, i32, vp, ctypes.c_int64, i32, i32, vp, vp],
        "bem_field_fmm": [vp, vp, i32, vp, ctypes.c_int64, i32, i32, vp, vp],
        "bem_far_field_adjoint": [vp, vp, i32, vp, ctypes.c_int64, vp, vp],
        "bem_shape_pairs": [vp, vp, vp, vp, i64, f64, f64, vp, vp, vp, vp, vp, vp, vp],
        "bem_self_blocks": [vp, vp, vp, vp, i64, i64, i32, f64, f64, vp, vp, vp],
        "bem_problem_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = args
    _lib = lib
    return lib


def check(code):
    if code != FMB_OK:
        raise FmbError(code, load().fmb_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _dev(t, dtype, shape_tail, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if tuple(t.shape[-len(shape_tail):]) != tuple(shape_tail):
        raise ValueError("%s has shape %s, expected [..., %s]" % (name, tuple(t.shape), shape_tail))
    return ctypes.c_void_p(t.data_ptr())


def shape_pairs(points, normals, weights, point_tri, k, lam, a, b):
    """(ds, dn, dw): derivatives of B = sum conj(lam) . PS_k(a, b) with respect to
    the node positions, normals and weights (`bem_shape_pairs`).  points,
    normals f64 [n, 3], weights f64 [n], point_tri i32 [n], lam, a, b c128
    [n, 3], all on the GPU; returns c128 [n, 3], [n, 3], [n]."""
    lib = load()
    n = points.shape[0]
    args = [_dev(points, torch.float64, (n, 3), "points"), _dev(normals, torch.float64, (n, 3), "normals"),
            _dev(weights, torch.float64, (n,), "weights"), _dev(point_tri, torch.int32, (n,), "point_tri")]
    args += [_dev(t, torch.complex128, (n, 3), nm) for t, nm in ((lam, "lam"), (a, "a"), (b, "b"))]
    ds = torch.empty((n, 3), dtype=torch.complex128, device=points.device)
    dn = torch.empty_like(ds)
    dw = torch.empty((n,), dtype=torch.complex128, device=points.device)
    k = complex(k)
    check(lib.bem_shape_pairs(*args[:4], n, k.real, k.imag, *args[4:], ctypes.c_void_p(ds.data_ptr()),
                              ctypes.c_void_p(dn.data_ptr()), ctypes.c_void_p(dw.data_ptr()), _stream()))
    return ds, dn, dw


def self_blocks(points, normals, point_tri, tri_vertices, k, mode="linear", device="cuda"):
    """(dV c128 [n, m, 3], dG c128 [n, m]) on the GPU: the self-triangle blocks of
    the given geometry (`bem_self_blocks`; host inputs, m = n / ntri)."""
    lib = load()
    pts = _host(points, np.float64)
    nrm = _host(normals, np.float64)
    pt = _host(point_tri, np.int32)
    tv = _host(tri_vertices, np.float64)
    n, ntri = pts.shape[0], tv.shape[0]
    m = n // ntri
    dv = torch.empty((n, m, 3), dtype=torch.complex128, device=device)
    dg = torch.empty((n, m), dtype=torch.complex128, device=device)
    k = complex(k)
    check(lib.bem_self_blocks(pts.ctypes.data, nrm.ctypes.data, pt.ctypes.data, tv.ctypes.data, n, ntri,
                              CORR[mode] if isinstance(mode, str) else int(mode), k.real, k.imag,
                              ctypes.c_void_p(dv.data_ptr()), ctypes.c_void_p(dg.data_ptr()), _stream()))
    return dv, dg


class Plan:
    """One wavenumber's FMM operator (`fmm_plan`)."""

    def __init__(self, points, normals, weights, k, order, depth=0, precision="fp64", nrhs_max=1,
                 corr="linear", point_tri=None, tri_vertices=None, leaf_target=32, translate="fp32", tol=0.0,
                 far_cutoff=0.0):
        lib = load()
        self._lib = lib
        pts = _host(points, np.float64)
        nrm = _host(normals, np.float64)
        w = _host(weights, np.float64)
        n = pts.shape[0]
        opts = PlanOpts()
        check(lib.fmb_plan_opts_default(ctypes.byref(opts)))
        opts.depth = int(depth)
        opts.precision = FMB_FP64 if precision == "fp64" else FMB_FP32
        opts.nrhs_max = int(nrhs_max)
        opts.corr_mode = CORR[corr] if isinstance(corr, str) else int(corr)
        opts.leaf_target = int(leaf_target)
        opts.translate_mode = {"fp32": 1, "bf16x3": 2}[translate]
        opts.tol = float(tol)
        opts.far_cutoff = float(far_cutoff)
        keep = []
        if point_tri is not None:
            pt = _host(point_tri, np.int32)
            keep.append(pt)
            opts.point_tri = pt.ctypes.data
            ntri = int(pt.max()) + 1
            if tri_vertices is not None:
                tv = _host(tri_vertices, np.float64)
                keep.append(tv)
                opts.tri_vertices = tv.ctypes.data
                ntri = tv.shape[0]
            opts.ntri = ntri
        k = complex(k)
        h = ctypes.c_void_p()
        check(lib.fmm_plan(pts.ctypes.data, nrm.ctypes.data, w.ctypes.data, n, k.real, k.imag, int(order),
                           ctypes.byref(opts), _stream(), ctypes.byref(h)))
        self.h = h
        self.n = n
        self.k = k
        self.precision = precision
        self.cdtype = torch.complex128 if precision == "fp64" else torch.complex64
        self.nrhs_max = int(nrhs_max)

    def matvec(self, a, b, out=None):
        """y = Op_k(a, b); a, b complex [nrhs, n, 3] or [n, 3] on the GPU."""
        squeeze = a.dim() == 2
        if squeeze:
            a = a.unsqueeze(0)
            b = b.unsqueeze(0)
        nrhs = a.shape[0]
        pa = _dev(a, self.cdtype, (self.n, 3), "a")
        pb = _dev(b, self.cdtype, (self.n, 3), "b")
        if out is None:
            out = torch.empty_like(a)
        py = _dev(out, self.cdtype, (self.n, 3), "y")
        check(self._lib.fmm_matvec(self.h, pa, pb, py, nrhs, _stream()))
        return out[0] if squeeze else out

    def matvec_adjoint(self, y):
        """(a_bar, b_bar) = Op_k^H y; y complex [nrhs, n, 3] or [n, 3] on the GPU."""
        squeeze = y.dim() == 2
        if squeeze:
            y = y.unsqueeze(0)
        py = _dev(y, self.cdtype, (self.n, 3), "y")
        a = torch.empty_like(y)
        b = torch.empty_like(y)
        check(self._lib.fmm_matvec_adjoint(self.h, py, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                           y.shape[0], _stream()))
        return (a[0], b[0]) if squeeze else (a, b)

    def info(self):
        inf = PlanInfo()
        check(self._lib.fmm_plan_info(self.h, ctypes.byref(inf)))
        d = inf.depth
        return {"depth": d, "order": inf.order, "n": inf.n, "nbox": list(inf.nbox[:d + 1]),
                "m2l_pairs": list(inf.m2l_pairs[:d + 1]), "p2p_pairs": inf.p2p_pairs,
                "corr_blocks": inf.corr_blocks, "device_bytes": inf.device_bytes,
                "order_level": list(inf.order_level[:d + 1]), "far_lmin": inf.far_lmin}

    def export_tree(self, level):
        inf = self.info()
        B = inf["nbox"][level]
        codes = np.zeros(self.n, np.uint64)
        perm = np.zeros(self.n, np.int32)
        keys = np.zeros(B, np.uint64)
        parent = np.zeros(B, np.int32)
        start = np.zeros(B + 1, np.int32)
        nbr = np.zeros((B, 27), np.int32)
        ff_ofs = np.zeros(B + 1, np.int32)
        check(self._lib.fmm_plan_export_tree(self.h, level, codes.ctypes.data, perm.ctypes.data, keys.ctypes.data,
                                             parent.ctypes.data, start.ctypes.data, nbr.ctypes.data,
                                             ff_ofs.ctypes.data, None))
        ff_idx = np.zeros(max(1, int(ff_ofs[-1])), np.int32)
        check(self._lib.fmm_plan_export_tree(self.h, level, None, None, None, None, None, None, None,
                                             ff_idx.ctypes.data))
        return {"codes": codes, "perm": perm, "keys": keys, "parent": parent, "start": start, "nbr": nbr,
                "ff_ofs": ff_ofs, "ff_idx": ff_idx[:int(ff_ofs[-1])]}

    STAGES = ("gather", "p2m", "m2m", "m2l", "l2l", "l2p", "p2p", "corr", "scatter", "sums", "m2l_fine")

    def profile(self, enable=True, stages=None):
        """Time stages with HIP events on later matvecs: all of them, or only
        the names in stages (a subset of STAGES); enable=False stops timing."""
        if not enable:
            mask = 0
        elif stages is None:
            mask = (1 << len(self.STAGES)) - 1
        else:
            mask = sum(1 << self.STAGES.index(s) for s in stages)
        check(self._lib.fmm_plan_profile(self.h, mask))

    def profile_read(self, reset=True):
        ms = np.zeros(len(self.STAGES))
        cnt = np.zeros(len(self.STAGES), np.int64)
        check(self._lib.fmm_plan_profile_read(self.h, ms.ctypes.data, cnt.ctypes.data, 1 if reset else 0))
        return {s: (float(ms[i]), int(cnt[i])) for i, s in enumerate(self.STAGES)}

    def close(self):
        if getattr(self, "h", None):
            self._lib.fmm_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
