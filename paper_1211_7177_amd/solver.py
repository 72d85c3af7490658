"""Binding of the BEM system and fGMRES entry points (marshalling only)."""

import ctypes

import numpy as np
import torch

from . import _abi
from ._abi import Plan, check, _stream


def _opts(lib, tol, restart, maxit, precond, mixed, inner_tol, inner_maxit, serial, adjoint=False,
          inner_reorth=False):
    opts = _abi.GmresOpts()
    check(lib.fmb_gmres_opts_default(ctypes.byref(opts)))
    opts.tol = tol
    opts.restart = restart
    opts.maxit = maxit
    # precond: False (none), True or "block" (exact 6x6 block inverse), "gmres" (the paper's inner
    # GMRES of at most 10 steps on the same blocks)
    opts.precond = 2 if precond == "gmres" else (1 if precond else 0)
    opts.mixed = 2 if mixed == "nested" else (1 if mixed else 0)
    opts.inner_tol = inner_tol
    opts.inner_maxit = inner_maxit
    opts.serial = 1 if serial else 0
    opts.adjoint = 1 if adjoint else 0
    opts.inner_reorth = 1 if inner_reorth else 0
    return opts


def _info_dict(info, code):
    return {"iterations": info.iterations, "refinements": info.refinements, "matvecs64": info.matvecs64,
            "matvecs32": info.matvecs32, "fp64_fallback": bool(info.fp64_fallback), "residual": info.residual,
            "code": code,
            "history": list(info.history[:min(256, max(info.iterations, info.refinements + 1))])}


def solve_group(problems, rhs_list, tol=1e-6, restart=100, maxit=1000, precond=True, mixed=False, inner_tol=1e-3,
                inner_maxit=300, raise_on_noconv=True, serial=False):
    """Solve several independent problems (meshes of any sizes) in one
    `gmres_solve_group` call; rhs_list[i] is complex128 [nrhs_i, n_i, 6] on the
    GPU.  Returns the solutions and one info dict per problem."""
    if len(problems) != len(rhs_list) or not problems:
        raise ValueError("one right-hand side tensor per problem")
    lib = _abi.load()
    opts = _opts(lib, tol, restart, maxit, precond, mixed, inner_tol, inner_maxit, serial)
    opts.x0_given = 0
    cnt = len(problems)
    xs, ptr_r, nrs = [], [], []
    for pb, rhs in zip(problems, rhs_list):
        pr, nr = pb._v(rhs, "rhs")
        ptr_r.append(pr.value)
        nrs.append(nr)
        xs.append(torch.zeros_like(rhs if rhs.dim() == 3 else rhs.unsqueeze(0)))
    hs = (ctypes.c_void_p * cnt)(*[pb.h.value for pb in problems])
    rp = (ctypes.c_void_p * cnt)(*ptr_r)
    xp = (ctypes.c_void_p * cnt)(*[x.data_ptr() for x in xs])
    nv = (ctypes.c_int32 * cnt)(*nrs)
    infos = (_abi.GmresInfo * cnt)()
    code = lib.gmres_solve_group(hs, cnt, rp, xp, nv, ctypes.byref(opts), infos, _stream())
    if code != _abi.FMB_OK and (code != _abi.FMB_ENOCONV or raise_on_noconv):
        check(code)
    return xs, [_info_dict(infos[i], code) for i in range(cnt)]


class BemProblem:
    """One scatterer in vacuum: plans at k0 and k1 = k0 sqrt(eps mu) over the same nodes.

    `bem_problem_create` wires the plans into the 6N system and builds the
    A_self block preconditioner; solves run through `gmres_solve`.
    """

    def __init__(self, nodes, k0, eps, mu=1.0, order=16, depth=0, nrhs_max=1, order32=None,
                 corr="linear", leaf_target=32, translate32="fp32", tol=0.0, tol32=0.0):
        """order / order32 = 0 choose an order per level for tol / tol32 (fmm_plan with
        order <= 0); order32 None builds no FP32 plans."""
        lib = _abi.load()
        self._lib = lib
        self.k0 = complex(k0)
        self.eps = complex(eps)
        self.mu = complex(mu)
        self.k1 = self.k0 * np.sqrt(self.eps * self.mu)
        kw = dict(point_tri=nodes["point_tri"], tri_vertices=nodes["tri_vertices"], nrhs_max=nrhs_max,
                  corr=corr, depth=depth, leaf_target=leaf_target)
        pts, nrm, w = nodes["points"], nodes["normals"], nodes["weights"]
        self.p0 = Plan(pts, nrm, w, self.k0, order, tol=tol, **kw)
        kw["depth"] = self.p0.info()["depth"]
        self.p1 = Plan(pts, nrm, w, self.k1, order, tol=tol, **kw)
        self.p0_32 = self.p1_32 = None
        if order32 is not None:
            self.p0_32 = Plan(pts, nrm, w, self.k0, order32, precision="fp32", translate=translate32, tol=tol32, **kw)
            self.p1_32 = Plan(pts, nrm, w, self.k1, order32, precision="fp32", translate=translate32, tol=tol32, **kw)
        self.n = pts.shape[0]
        self.nrhs_max = nrhs_max
        eps_a = np.array([self.eps.real, self.eps.imag])
        mu_a = np.array([self.mu.real, self.mu.imag])
        h = ctypes.c_void_p()
        check(lib.bem_problem_create(self.p0.h, self.p1.h, self.p0_32.h if self.p0_32 else None,
                                     self.p1_32.h if self.p1_32 else None, eps_a.ctypes.data, mu_a.ctypes.data,
                                     _stream(), ctypes.byref(h)))
        self.h = h

    nu = 6                      # unknowns per node

    def _v(self, t, name):
        if t.dim() == 2:
            t = t.unsqueeze(0)
        return _abi._dev(t, torch.complex128, (self.n, self.nu), name), t.shape[0]

    def use_graphs(self, enable=True):
        """Replay the two FMM products of each application from a captured HIP
        graph (the default) or launch them one by one."""
        check(self._lib.bem_problem_use_graphs(self.h, 1 if enable else 0))

    def apply(self, x):
        """A x, x complex128 [nrhs, n, 6] (or [n, 6]) on the GPU."""
        out = torch.empty_like(x)
        px, nr = self._v(x, "x")
        check(self._lib.bem_apply(self.h, px, ctypes.c_void_p(out.data_ptr()), nr, _stream()))
        return out

    def apply32(self, x, out=None):
        """A x with the FP32 plans (the inner solves' operator), x complex64 [nrhs, n, nu] on the GPU."""
        if x.dim() == 2:
            x = x.unsqueeze(0)
        px = _abi._dev(x, torch.complex64, (self.n, self.nu), "x")
        out = torch.empty_like(x) if out is None else out
        _abi._dev(out, torch.complex64, (self.n, self.nu), "out")
        check(self._lib.bem_apply32(self.h, px, ctypes.c_void_p(out.data_ptr()), x.shape[0], _stream()))
        return out

    def apply_adjoint(self, v):
        """A^H v, v complex128 [nrhs, n, 6] (or [n, 6]) on the GPU."""
        out = torch.empty_like(v)
        pv, nr = self._v(v, "v")
        check(self._lib.bem_apply_adjoint(self.h, pv, ctypes.c_void_p(out.data_ptr()), nr, _stream()))
        return out

    def field(self, x, points, region="host", far=False, curl=False, method="direct", order=16):
        """Fields from the solution x [nrhs, n, nu]: the scattered field at host
        points (region "host"), the interior field ("interior"), with far=True
        the far-field amplitude F at unit directions, or with curl=True the curl
        of the scattered field at host points.  points: host array [nt, 3].
        method "fmm" evaluates the first two by a fast multipole product of the
        given order over nodes and targets (for many targets).
        Returns complex128 [nrhs, nt, 3] on the GPU."""
        px, nr = self._v(x, "x")
        pts = np.ascontiguousarray(np.atleast_2d(points), dtype=np.float64)
        nt = pts.shape[0]
        out = torch.empty((nr, nt, 3), dtype=torch.complex128, device="cuda")
        reg = {"host": 0, "interior": 1}[region]
        if method == "fmm":
            if far or curl:
                raise ValueError("the FMM evaluation serves the near field and the interior field")
            check(self._lib.bem_field_fmm(self.h, px, nr, pts.ctypes.data, nt, reg, int(order),
                                          ctypes.c_void_p(out.data_ptr()), _stream()))
            return out
        if method != "direct":
            raise ValueError("method must be 'direct' or 'fmm'")
        if far and curl:
            raise ValueError("far and curl are exclusive")
        kind = 1 if far else (2 if curl else 0)
        check(self._lib.bem_field(self.h, px, nr, pts.ctypes.data, nt, reg, kind,
                                  ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def far_field_adjoint(self, G, dirs):
        """x_bar = L^H G for far-field samples G [nrhs, nd, 3] at unit directions
        dirs [nd, 3], L the map x -> F of field(..., far=True).  Returns
        complex128 [nrhs, n, nu] on the GPU."""
        G = G.contiguous()
        if G.dtype != torch.complex128 or not G.is_cuda or G.dim() != 3:
            raise ValueError("G must be a complex128 CUDA tensor [nrhs, nd, 3]")
        d = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
        nr, nd = G.shape[0], G.shape[1]
        if d.shape != (nd, 3):
            raise ValueError("dirs must be [nd, 3] matching G")
        out = torch.empty((nr, self.n, self.nu), dtype=torch.complex128, device="cuda")
        check(self._lib.bem_far_field_adjoint(self.h, ctypes.c_void_p(G.data_ptr()), nr, d.ctypes.data, nd,
                                              ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    def precond(self, v):
        out = torch.empty_like(v)
        pv, nr = self._v(v, "v")
        check(self._lib.bem_precond_apply(self.h, pv, ctypes.c_void_p(out.data_ptr()), nr, _stream()))
        return out

    def rhs_planewave(self, dirs, pols):
        d = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
        p = np.ascontiguousarray(np.atleast_2d(pols), dtype=np.complex128)
        nr = d.shape[0]
        out = torch.empty((nr, self.n, self.nu), dtype=torch.complex128, device="cuda")
        check(self._lib.bem_rhs_planewave(self.h, d.ctypes.data, p.ctypes.data, ctypes.c_void_p(out.data_ptr()),
                                          nr, _stream()))
        return out

    def solve(self, rhs, tol=1e-6, restart=100, maxit=1000, precond=True, mixed=False, inner_tol=1e-3,
              inner_maxit=300, x0=None, raise_on_noconv=True, serial=False, adjoint=False, inner_reorth=False):
        """Solve A x = rhs (or A^H x = rhs with adjoint=True) with fGMRES.
        mixed: False (FP64), True (FP32 inner solves inside FP64 refinement) or
        "nested" (FP64 fGMRES preconditioned by one FP32 fGMRES cycle per step)."""
        opts = _opts(self._lib, tol, restart, maxit, precond, mixed, inner_tol, inner_maxit, serial, adjoint,
                     inner_reorth)
        x = torch.zeros_like(rhs) if x0 is None else x0.clone()
        opts.x0_given = 0 if x0 is None else 1
        info = _abi.GmresInfo()
        pr, nr = self._v(rhs, "rhs")
        code = self._lib.gmres_solve(self.h, pr, ctypes.c_void_p(x.data_ptr()), nr, ctypes.byref(opts),
                                     ctypes.byref(info), _stream())
        res = _info_dict(info, code)
        if code != _abi.FMB_OK and (code != _abi.FMB_ENOCONV or raise_on_noconv):
            check(code)
        return x, res

    def close(self):
        if getattr(self, "h", None):
            self._lib.bem_problem_destroy(self.h)
            self.h = None
        for p in (self.p0, self.p1, self.p0_32, self.p1_32):
            if p is not None:
                p.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class IbcProblem(BemProblem):
    """A good conductor under the impedance boundary condition (eqs. 2.24-2.25):
    three unknowns per node (Phi = E_0), one plan at k0, surface impedance Z
    relative to vacuum.  Vectors are complex128 [nrhs, n, 3]; `apply`,
    `apply_adjoint`, `precond`, `rhs_planewave` and `solve` work as for
    BemProblem."""

    nu = 3

    def __init__(self, nodes, k0, Z, order=16, depth=0, nrhs_max=1, order32=None, corr="linear", leaf_target=32,
                 translate32="fp32", tol=0.0, tol32=0.0):
        lib = _abi.load()
        self._lib = lib
        self.k0 = complex(k0)
        self.Z = complex(Z)
        kw = dict(point_tri=nodes["point_tri"], tri_vertices=nodes["tri_vertices"], nrhs_max=nrhs_max,
                  corr=corr, depth=depth, leaf_target=leaf_target)
        pts, nrm, w = nodes["points"], nodes["normals"], nodes["weights"]
        self.p0 = Plan(pts, nrm, w, self.k0, order, tol=tol, **kw)
        kw["depth"] = self.p0.info()["depth"]
        self.p1 = self.p1_32 = None
        self.p0_32 = None
        if order32 is not None:
            self.p0_32 = Plan(pts, nrm, w, self.k0, order32, precision="fp32", translate=translate32, tol=tol32, **kw)
        self.n = pts.shape[0]
        self.nrhs_max = nrhs_max
        z = np.array([self.Z.real, self.Z.imag])
        h = ctypes.c_void_p()
        check(lib.bem_problem_create_ibc(self.p0.h, self.p0_32.h if self.p0_32 else None, z.ctypes.data, _stream(),
                                         ctypes.byref(h)))
        self.h = h


def _nodes_of(nodes, mask):
    """The nodes with mask set, in their global order, as a node set of its own
    (triangles renumbered in order)."""
    idx = np.nonzero(mask)[0]
    tri = nodes["point_tri"][idx]
    uniq, inv = np.unique(tri, return_inverse=True)
    return {"points": np.ascontiguousarray(nodes["points"][idx]), "normals": np.ascontiguousarray(nodes["normals"][idx]),
            "weights": np.ascontiguousarray(nodes["weights"][idx]), "point_tri": inv.astype(np.int32),
            "tri_vertices": np.ascontiguousarray(nodes["tri_vertices"][uniq])}


class MultiBemProblem(BemProblem):
    """J dielectric scatterers in vacuum: region[alpha] in 0..J-1 names the
    scatterer of node alpha; eps, mu list the scatterers' constants.  The host
    plan covers every node, plan j the nodes of scatterer j (built here from
    the node subset).  Vectors are complex128 [nrhs, n, 6]."""

    def __init__(self, nodes, region, k0, eps, mu=None, order=16, depth=0, depths=None, nrhs_max=1, order32=None,
                 corr="linear", leaf_target=32, translate32="fp32"):
        lib = _abi.load()
        self._lib = lib
        region = np.ascontiguousarray(region, dtype=np.int32)
        J = int(region.max()) + 1
        self.k0 = complex(k0)
        self.eps = [complex(e) for e in eps]
        self.mu = [complex(m) for m in (mu if mu is not None else [1.0] * J)]
        self.kj = [self.k0 * np.sqrt(e * m) for e, m in zip(self.eps, self.mu)]
        kw = dict(nrhs_max=nrhs_max, corr=corr, leaf_target=leaf_target)
        self.p0 = Plan(nodes["points"], nodes["normals"], nodes["weights"], self.k0, order, depth=depth,
                       point_tri=nodes["point_tri"], tri_vertices=nodes["tri_vertices"], **kw)
        self.p0_32 = None
        if order32:
            self.p0_32 = Plan(nodes["points"], nodes["normals"], nodes["weights"], self.k0, order32,
                              depth=self.p0.info()["depth"], precision="fp32", translate=translate32,
                              point_tri=nodes["point_tri"], tri_vertices=nodes["tri_vertices"], **kw)
        self.pj, self.pj_32 = [], []
        for j in range(J):
            sub = _nodes_of(nodes, region == j)
            dj = depths[j] if depths is not None else 0
            P = Plan(sub["points"], sub["normals"], sub["weights"], self.kj[j], order, depth=dj,
                     point_tri=sub["point_tri"], tri_vertices=sub["tri_vertices"], **kw)
            self.pj.append(P)
            if order32:
                self.pj_32.append(Plan(sub["points"], sub["normals"], sub["weights"], self.kj[j], order32,
                                       depth=P.info()["depth"], precision="fp32", translate=translate32,
                                       point_tri=sub["point_tri"], tri_vertices=sub["tri_vertices"], **kw))
        self.p1 = self.pj[0]
        self.p1_32 = self.pj_32[0] if self.pj_32 else None
        self.n = nodes["points"].shape[0]
        self.nrhs_max = nrhs_max
        hs = (ctypes.c_void_p * J)(*[P.h.value for P in self.pj])
        hs32 = (ctypes.c_void_p * J)(*[P.h.value for P in self.pj_32]) if self.pj_32 else None
        e = np.array([[z.real, z.imag] for z in self.eps]).ravel()
        m = np.array([[z.real, z.imag] for z in self.mu]).ravel()
        h = ctypes.c_void_p()
        check(lib.bem_problem_create_multi(self.p0.h, hs, J, region.ctypes.data, e.ctypes.data, m.ctypes.data,
                                           self.p0_32.h if self.p0_32 else None, hs32, _stream(), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self._lib.bem_problem_destroy(self.h)
            self.h = None
        for p in [self.p0, self.p0_32] + list(self.pj) + list(self.pj_32):
            if p is not None:
                p.close()
        self.pj, self.pj_32 = [], []
        self.p0 = self.p0_32 = self.p1 = self.p1_32 = None
