"""MI355X-native short-range TreePM gravity step (Ishiyama, Nitadori & Makino, SC12).

A thin binding of ``libsrf.so`` (declared in ``include/srf.h``): argument
marshalling only -- every step of the path runs in the library's HIP
kernels.  Tensors are torch CUDA (HIP) tensors; work is ordered on torch's
current stream.  The library must be built (``python
paper_1211_4406_amd/build.py``); importing this module without it raises.

    tree  = tree_build(x, m, params)          # a1-a5
    lists = make_lists(tree, params)          # a6
    a     = short_range_force(tree, lists, params)            # a7-a8
    gx, gm = short_range_adjoint(tree, lists, params, w)      # a9
    phi   = short_range_potential(tree, lists, params)        # potential of the split
    a     = ShortRange.apply(x, m, params)    # autograd: backward rebuilds the lists
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

__all__ = [
    "Params", "Tree", "Lists", "SrfError", "FP32_REL", "FP64", "MAC_CENTRE", "MAC_COM", "lib", "lib_path", "tree_build",
    "tree_refit", "make_lists",
    "short_range_force", "short_range_adjoint", "short_range_adjoint_noalloc", "short_range_potential", "short_range_quadrupole", "ShortRange", "short_range", "pm_force", "kick", "drift",
    "TreePMIntegrator", "set_kernel_timing", "last_kernel_ms",
]

FP32_REL = 0
FP64 = 1
MAC_CENTRE = 0   # opening distance to the cell's geometric centre
MAC_COM = 1      # ... to its centre of mass

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsrf.so")


class SrfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"srf error {status}: {msg}")
        self.status = status


class _CParams(C.Structure):
    _fields_ = [("G", C.c_double), ("r_cut", C.c_double), ("eps", C.c_double), ("theta", C.c_double),
                ("n_group", C.c_int32), ("n_leaf", C.c_int32), ("precision", C.c_int32), ("compensated", C.c_int32),
                ("mac", C.c_int32)]


@dataclass(frozen=True)
class Params:
    """Parameters of one short-range evaluation (box side 1, periodic)."""
    G: float = 1.0
    r_cut: float = 0.1
    eps: float = 1e-3
    theta: float = 0.5
    n_group: int = 64
    n_leaf: int = 16
    precision: int = FP32_REL
    compensated: int = 0
    mac: int = MAC_CENTRE

    def c(self) -> _CParams:
        return _CParams(float(self.G), float(self.r_cut), float(self.eps), float(self.theta), int(self.n_group),
                        int(self.n_leaf), int(self.precision), int(self.compensated), int(self.mac))

    @staticmethod
    def of(p, precision: int | None = None, compensated: int | None = None) -> "Params":
        """Convert any object with G, r_cut, eps, theta, n_group, n_leaf."""
        prec = getattr(p, "precision", FP32_REL) if precision is None else precision
        comp = getattr(p, "compensated", 0) if compensated is None else compensated
        return Params(p.G, p.r_cut, p.eps, p.theta, p.n_group, p.n_leaf, prec, comp, getattr(p, "mac", MAC_CENTRE))


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded libsrf.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with `python paper_1211_4406_amd/build.py` "
                           "(there is no fallback implementation)")
    L = C.CDLL(_LIB_PATH)
    vp, i64, i32, pp = C.c_void_p, C.c_int64, C.c_int32, C.POINTER(_CParams)
    L.srf_tree_build.argtypes = [i64, vp, vp, vp, i64, vp, i64, pp, vp, C.POINTER(vp)]
    L.srf_tree_refit.argtypes = [vp, vp, vp, vp, i64, vp, i64, vp]
    L.srf_make_lists.argtypes = [vp, pp, vp, C.POINTER(vp)]
    L.srf_short_range_force.argtypes = [vp, vp, pp, vp, vp, vp, i64, vp]
    L.srf_short_range_adjoint.argtypes = [vp, vp, pp, vp, vp, vp, i64, vp, vp, vp, i64, vp, i64, vp]
    L.srf_short_range_adjoint_noalloc.argtypes = [vp, vp, pp, vp, vp, vp, i64, vp, vp, vp, i64, vp, i64, vp]
    L.srf_tree_free.argtypes = [vp]
    L.srf_tree_free.restype = None
    L.srf_lists_free.argtypes = [vp]
    L.srf_lists_free.restype = None
    L.srf_release_cache.argtypes = []
    L.srf_release_cache.restype = None
    L.srf_strerror.argtypes = [C.c_int]
    L.srf_strerror.restype = C.c_char_p
    L.srf_last_error.argtypes = []
    L.srf_last_error.restype = C.c_char_p
    L.srf_tree_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i32)]
    L.srf_tree_export.argtypes = [vp] + [vp] * 10
    L.srf_moments_export.argtypes = [vp] + [vp] * 4
    L.srf_sorted_export.argtypes = [vp] + [vp] * 4
    L.srf_cell_boxes_export.argtypes = [vp, vp, vp]
    L.srf_lists_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    L.srf_lists_export.argtypes = [vp] * 5
    L.srf_short_range_potential.argtypes = [vp, vp, pp, vp, i64, vp]
    L.srf_short_range_quadrupole.argtypes = [vp, vp, pp, vp, vp, vp, i64, vp]
    L.srf_pm_force.argtypes = [vp, C.c_double, C.c_double, C.c_int32, vp, vp, vp, i64, vp]
    L.srf_kick.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp, i64, C.c_double, vp]
    L.srf_drift.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp, i64, C.c_double, vp]
    L.srf_set_kernel_timing.argtypes = [C.c_int]
    L.srf_last_kernel_ms.argtypes = [C.c_char_p, C.POINTER(C.c_double)]
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise SrfError(status, lib().srf_last_error().decode())


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _hptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _cols(x: torch.Tensor):
    """Column pointers and element stride of an [N,3] float64 CUDA tensor
    (any layout whose rows have a constant stride and unit column stride)."""
    if x.dtype != torch.float64 or not x.is_cuda or x.dim() != 2 or x.shape[1] != 3:
        raise ValueError("positions must be a float64 CUDA tensor of shape [N, 3]")
    # the library reads rows at a positive element stride with unit column
    # stride; anything else (a transposed view, or an expanded gradient whose
    # rows share memory, stride 0) is copied first
    if x.stride(1) != 1 or x.stride(0) < 1:
        x = x.contiguous()
    base = x.data_ptr()
    return x, [C.c_void_p(base), C.c_void_p(base + 8), C.c_void_p(base + 16)], x.stride(0)


class Tree:
    """Handle of a built tree (owns library device memory)."""

    def __init__(self, handle, params: Params, n: int):
        self._h = handle
        self.params = params
        self.n = n

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _lib is not None:
            _lib.srf_tree_free(h)

    @property
    def handle(self):
        return self._h

    def info(self):
        n, nn, ng, ml = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib().srf_tree_info(self._h, C.byref(n), C.byref(nn), C.byref(ng), C.byref(ml)))
        return dict(n=n.value, n_nodes=nn.value, n_groups=ng.value, max_level=ml.value)

    def export(self):
        """Host copies: keys, perm, cells (preorder), groups and boxes."""
        inf = self.info()
        n, nn, ng = inf["n"], inf["n_nodes"], inf["n_groups"]
        out = dict(keys=np.empty(n, np.uint64), perm=np.empty(n, np.int64), level=np.empty(nn, np.int32),
                   prefix=np.empty(nn, np.uint64), first=np.empty(nn, np.int64), count=np.empty(nn, np.int64),
                   gfirst=np.empty(ng, np.int64), gcount=np.empty(ng, np.int64), lo=np.empty((ng, 3)),
                   hi=np.empty((ng, 3)))
        _check(lib().srf_tree_export(self._h, *(_hptr(out[k]) for k in
                                                ("keys", "perm", "level", "prefix", "first", "count", "gfirst",
                                                 "gcount", "lo", "hi"))))
        return out

    def moments(self):
        nn = self.info()["n_nodes"]
        M, X, Y, Z = (np.empty(nn) for _ in range(4))
        _check(lib().srf_moments_export(self._h, _hptr(M), _hptr(X), _hptr(Y), _hptr(Z)))
        return M, np.stack([X, Y, Z], axis=1)

    def cell_boxes(self):
        """Boxes (lo, hi) [n_nodes, 3] of the cells of a refitted tree."""
        nn = self.info()["n_nodes"]
        lo, hi = np.empty((nn, 3)), np.empty((nn, 3))
        _check(lib().srf_cell_boxes_export(self._h, _hptr(lo), _hptr(hi)))
        return lo, hi

    def sorted_particles(self):
        x, y, z, m = (np.empty(self.n) for _ in range(4))
        _check(lib().srf_sorted_export(self._h, _hptr(x), _hptr(y), _hptr(z), _hptr(m)))
        return np.stack([x, y, z], axis=1), m


class Lists:
    """Handle of built interaction lists."""

    def __init__(self, handle, tree: Tree, params: Params):
        self._h = handle
        self.tree = tree          # keeps the tree alive
        self.params = params

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _lib is not None:
            _lib.srf_lists_free(h)

    @property
    def handle(self):
        return self._h

    def info(self):
        a, b, c, d = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().srf_lists_info(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return dict(n_groups=a.value, n_particle_entries=b.value, n_node_entries=c.value, interactions=d.value)

    def export(self):
        inf = self.info()
        ng = inf["n_groups"]
        poff = np.empty(ng + 1, np.int64)
        noff = np.empty(ng + 1, np.int64)
        pidx = np.empty(inf["n_particle_entries"], np.int64)
        nidx = np.empty(inf["n_node_entries"], np.int64)
        _check(lib().srf_lists_export(self._h, _hptr(poff), _hptr(pidx), _hptr(noff), _hptr(nidx)))
        return dict(poff=poff, pidx=pidx, noff=noff, nidx=nidx)


def tree_build(x: torch.Tensor, m: torch.Tensor, params: Params) -> Tree:
    """a1-a5 on an [N,3] float64 position tensor and an [N] float64 mass tensor."""
    x, cols, ps = _cols(x)
    if m.dtype != torch.float64 or not m.is_cuda or m.dim() != 1 or m.shape[0] != x.shape[0]:
        raise ValueError("masses must be a float64 CUDA tensor of shape [N]")
    if x.device != m.device:
        raise ValueError("positions and masses must be on the same device")
    cp = params.c()
    h = C.c_void_p()
    _check(lib().srf_tree_build(C.c_int64(x.shape[0]), *cols, C.c_int64(ps), _dptr(m), C.c_int64(m.stride(0)),
                                C.byref(cp), _stream(), C.byref(h)))
    return Tree(h, params, int(x.shape[0]))


def tree_refit(tree: Tree, x: torch.Tensor, m: torch.Tensor | None = None) -> Tree:
    """Reuse ``tree`` at new positions x [N,3] (and masses m [N], or the
    tree's if None): sort order, cells and groups kept, moments and boxes
    recomputed.  Lists of the old positions are refused afterwards."""
    x, cols, ps = _cols(x)
    if x.shape[0] != tree.n:
        raise ValueError("x must hold the tree's n particles")
    mp, ms = None, 1
    if m is not None:
        if m.dtype != torch.float64 or not m.is_cuda or m.dim() != 1 or m.shape[0] != tree.n:
            raise ValueError("masses must be a float64 CUDA tensor of shape [N]")
        mp, ms = _dptr(m), m.stride(0)
    _check(lib().srf_tree_refit(tree.handle, *cols, C.c_int64(ps), mp, C.c_int64(ms), _stream()))
    return tree


def make_lists(tree: Tree, params: Params) -> Lists:
    cp = params.c()
    h = C.c_void_p()
    _check(lib().srf_make_lists(tree.handle, C.byref(cp), _stream(), C.byref(h)))
    return Lists(h, tree, params)


def short_range_force(tree: Tree, lists: Lists, params: Params, out: torch.Tensor | None = None,
                      device=None, quadrupole: bool = False) -> torch.Tensor:
    """a7-a8: [N,3] float64 accelerations in input order; with
    ``quadrupole`` the cells' quadrupole terms are added (no adjoint)."""
    if out is None:
        out = torch.empty((tree.n, 3), dtype=torch.float64, device=device or torch.device("cuda"))
    out_, cols, os_ = _cols(out)
    if out_.data_ptr() != out.data_ptr():
        raise ValueError("out must have unit column stride")
    cp = params.c()
    _check(lib().srf_short_range_force(tree.handle, lists.handle, C.byref(cp), *cols, C.c_int64(os_), _stream()))
    if quadrupole:
        short_range_quadrupole(tree, lists, params, out)
    return out


def short_range_quadrupole(tree: Tree, lists: Lists, params: Params, out: torch.Tensor) -> torch.Tensor:
    """Adds the cells' quadrupole terms to the [N,3] float64 accelerations
    ``out`` (input order) in place."""
    out_, cols, os_ = _cols(out)
    if out_.data_ptr() != out.data_ptr():
        raise ValueError("out must have unit column stride")
    cp = params.c()
    _check(lib().srf_short_range_quadrupole(tree.handle, lists.handle, C.byref(cp), *cols, C.c_int64(os_),
                                            _stream()))
    return out


def short_range_adjoint(tree: Tree, lists: Lists, params: Params, w: torch.Tensor, device=None):
    """a9: (dL/dx [N,3], dL/dm [N]) for L = sum_i w_i . a_i."""
    w, wcols, ws = _cols(w)
    gx = torch.empty((tree.n, 3), dtype=torch.float64, device=w.device)
    gm = torch.empty((tree.n,), dtype=torch.float64, device=w.device)
    _, gcols, gs = _cols(gx)
    cp = params.c()
    _check(lib().srf_short_range_adjoint(tree.handle, lists.handle, C.byref(cp), *wcols, C.c_int64(ws), *gcols,
                                         C.c_int64(gs), _dptr(gm), C.c_int64(1), _stream()))
    return gx, gm


def short_range_adjoint_noalloc(tree: Tree, lists: Lists, params: Params, w: torch.Tensor, gx: torch.Tensor,
                                gm: torch.Tensor) -> None:
    """a9 into caller-provided outputs gx [N,3] and gm [N] (float64, device),
    with the library's static device workspace: no device allocation."""
    w, wcols, ws = _cols(w)
    gx_, gcols, gs = _cols(gx)
    if gx_.data_ptr() != gx.data_ptr():
        raise ValueError("gx must have unit column stride")
    if gm.dtype != torch.float64 or gm.dim() != 1 or gm.shape[0] != tree.n or not gm.is_cuda:
        raise ValueError("gm must be a float64 CUDA vector of length n")
    cp = params.c()
    _check(lib().srf_short_range_adjoint_noalloc(tree.handle, lists.handle, C.byref(cp), *wcols, C.c_int64(ws),
                                                 *gcols, C.c_int64(gs), _dptr(gm), C.c_int64(gm.stride(0)),
                                                 _stream()))


def short_range_potential(tree: Tree, lists: Lists, params: Params, out: torch.Tensor | None = None,
                          device=None) -> torch.Tensor:
    """[N] float64 short-range potentials in input order over the same lists
    as the force (own entry left out)."""
    if out is None:
        out = torch.empty((tree.n,), dtype=torch.float64, device=device or torch.device("cuda"))
    if out.dtype != torch.float64 or out.dim() != 1 or out.shape[0] != tree.n or not out.is_cuda:
        raise ValueError("out must be a float64 CUDA vector of length n")
    cp = params.c()
    _check(lib().srf_short_range_potential(tree.handle, lists.handle, C.byref(cp), _dptr(out),
                                           C.c_int64(out.stride(0)), _stream()))
    return out


def pm_force(tree: Tree, G: float, r_cut: float, n_mesh: int, out: torch.Tensor | None = None,
             device=None) -> torch.Tensor:
    """Long-range (PM) accelerations [N,3] float64 of the tree's particles,
    in input order, on an n_mesh^3 mesh with the S2 split of radius r_cut/2."""
    if out is None:
        out = torch.empty((tree.n, 3), dtype=torch.float64, device=device or torch.device("cuda"))
    out_, cols, os_ = _cols(out)
    if out_.data_ptr() != out.data_ptr():
        raise ValueError("out must have unit column stride")
    _check(lib().srf_pm_force(tree.handle, C.c_double(G), C.c_double(r_cut), C.c_int32(n_mesh), *cols,
                              C.c_int64(os_), _stream()))
    return out


def kick(v: torch.Tensor, a: torch.Tensor, dt: float) -> None:
    """v += dt a, in place ([N,3] float64 device tensors)."""
    v_, vcols, vs = _cols(v)
    if v_.data_ptr() != v.data_ptr():
        raise ValueError("v must have unit column stride")
    _, acols, as_ = _cols(a)
    _check(lib().srf_kick(C.c_int64(v.shape[0]), *vcols, C.c_int64(vs), *acols, C.c_int64(as_), C.c_double(dt),
                          _stream()))


def drift(x: torch.Tensor, v: torch.Tensor, dt: float) -> None:
    """x += dt v, wrapped into [0,1), in place ([N,3] float64 device tensors)."""
    x_, xcols, xs = _cols(x)
    if x_.data_ptr() != x.data_ptr():
        raise ValueError("x must have unit column stride")
    _, vcols, vs = _cols(v)
    _check(lib().srf_drift(C.c_int64(x.shape[0]), *xcols, C.c_int64(xs), *vcols, C.c_int64(vs), C.c_double(dt),
                           _stream()))


class TreePMIntegrator:
    """Multiple-stepsize (impulse) integrator of the TreePM force (Sec. 3:
    one step is one PM cycle and two PP cycles).  A step of length dt is

        kick(PM, dt/2); 2 x [kick(PP, dt/4); drift(dt/2); PP at new x; kick(PP, dt/4)]; PM at new x; kick(PM, dt/2)

    which evaluates PM once and PP twice per step; the PM of the new
    positions uses the tree of the last PP evaluation, and the accelerations
    of the step's end start the next.  With ``reuse_tree`` the second PP
    cycle refits the first one's tree to the drifted positions instead of
    building a new one (lists are always rebuilt); the step is then
    time-symmetric only up to the tree's truncation error (exactly so at
    theta = 0, where the lists hold every pair within r_cut either way).
    x, v are [N,3] float64 device tensors updated in place; m is [N]."""

    def __init__(self, params: Params, n_mesh: int, pm_r_cut: float | None = None, reuse_tree: bool = True):
        self.params = params
        self.n_mesh = int(n_mesh)
        self.pm_r_cut = params.r_cut if pm_r_cut is None else pm_r_cut
        self.reuse_tree = bool(reuse_tree)
        self.a_pp = None
        self.a_pm = None

    def _pp(self, x, m, tree=None):
        if tree is None:
            tree = tree_build(x, m, self.params)
        else:
            tree_refit(tree, x)
        lists = make_lists(tree, self.params)
        return tree, short_range_force(tree, lists, self.params, device=x.device)

    def step(self, x: torch.Tensor, v: torch.Tensor, m: torch.Tensor, dt: float) -> None:
        if self.a_pp is None or self.a_pm is None:
            tree, self.a_pp = self._pp(x, m)
            self.a_pm = pm_force(tree, self.params.G, self.pm_r_cut, self.n_mesh, device=x.device)
        kick(v, self.a_pm, 0.5 * dt)
        tree = None
        for _ in range(2):
            kick(v, self.a_pp, 0.25 * dt)
            drift(x, v, 0.5 * dt)
            tree, self.a_pp = self._pp(x, m, tree if self.reuse_tree else None)
            kick(v, self.a_pp, 0.25 * dt)
        self.a_pm = pm_force(tree, self.params.G, self.pm_r_cut, self.n_mesh, device=x.device)
        kick(v, self.a_pm, 0.5 * dt)

    def reset(self) -> None:
        """Forget the cached accelerations (call after changing x or m outside step)."""
        self.a_pp = None
        self.a_pm = None


class ShortRange(torch.autograd.Function):
    """a = short-range accelerations of (x, m); backward recomputes the tree
    and lists from the saved inputs and runs the hand-written adjoint."""

    @staticmethod
    def forward(ctx, x, m, params):
        tree = tree_build(x, m, params)
        lists = make_lists(tree, params)
        a = short_range_force(tree, lists, params, device=x.device)
        ctx.save_for_backward(x, m)
        ctx.params = params
        return a

    @staticmethod
    def backward(ctx, w):
        x, m = ctx.saved_tensors
        p = ctx.params
        tree = tree_build(x, m, p)
        lists = make_lists(tree, p)
        gx, gm = short_range_adjoint(tree, lists, p, w.to(torch.float64))
        return gx, gm, None


def short_range(x: torch.Tensor, m: torch.Tensor, params: Params) -> torch.Tensor:
    return ShortRange.apply(x, m, params)


def set_kernel_timing(enable: bool):
    _check(lib().srf_set_kernel_timing(1 if enable else 0))


def last_kernel_ms(which: str) -> float:
    v = C.c_double()
    _check(lib().srf_last_kernel_ms(which.encode(), C.byref(v)))
    return v.value


# Fail loudly at import if the HIP library is absent.
lib()
