"""FP64 CPU oracle of the short-range TreePM step -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library: the arithmetic lives in ``srf_oracle.c`` (plain C, FP64, built with
no FMA contraction) and this module only marshals numpy arrays to it and
strings the steps together in the paper's order.

Steps (Ishiyama, Nitadori & Makino, SC12):
  a1 wrap + Morton key       (tree of Sec. 1 over the periodic box)
  a2 sort by (key, index)
  a3 octree                  (Barnes-Hut cells, Sec. 1 / Fig. 1)
  a4 monopole moments
  a5 particle groups         (Barnes' modified algorithm, Sec. 2)
  a6 interaction lists       (opening angle theta + cutoff pruning, Fig. 2)
  a7 same-list force         (Sec. 2 force sum with eq. (cutoff))
  a8 unpermute
  a9 adjoint of L = sum_i w_i . a_i with the structure held fixed.
Accuracy variants over the same lists: the short-range potential and the
quadrupole term of the cells (second moments about the centre of mass).
Plus the plain definition: brute-force minimum-image sums (O(N^2) and a
cell list) and their gradient.  The long-range (PM) half of the force split
and the Ewald sum that checks PP + PM live in ``oracle.pm`` (numpy, FP64).

Parity pins (tests/test_oracle_*.py): g against the S2-S2 cloud integral
that defines it; brute force against O(N^2), momentum, translation and the
two-body closed form; tree at theta = 0 against brute force; list coverage
by brute force; adjoint against central differences, translation
invariance and the brute-force closed form.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "srf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_d = C.c_double
_i64 = C.c_int64
_p = C.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle library in place (gcc, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        L.or_gcut.restype = _d
        L.or_gcut.argtypes = [_d]
        L.or_gcut_deriv.restype = _d
        L.or_gcut_deriv.argtypes = [_d]
        L.or_wrap.restype = _d
        L.or_wrap.argtypes = [_d]
        L.or_morton3.restype = C.c_uint64
        L.or_morton3.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32]
        L.or_tree_count.restype = _i64
        L.or_groups.restype = _i64
        L.or_bf_pair_count.restype = _i64
        L.or_bf_cells.restype = C.c_int
        L.or_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().or_num_threads())


# ---------------------------------------------------------------- kernels
def gcut(xi):
    """g_P3M(xi) (Sec. 2, eq. cutoff), vectorised; also its derivative."""
    xi = _f64(np.atleast_1d(xi))
    g = np.empty_like(xi)
    dg = np.empty_like(xi)
    lib().or_gcut_vec(_i64(xi.size), _ptr(xi), _ptr(g), _ptr(dg))
    return g, dg


def gcut_printed(xi):
    """g_P3M exactly as printed (zeta branch form), for transcription pins."""
    xi = _f64(np.atleast_1d(xi))
    g = np.empty_like(xi)
    lib().or_gcut_printed_vec(_i64(xi.size), _ptr(xi), _ptr(g))
    return g


def gcut_deriv2(xi):
    """d^2 g / d xi^2 (quadrupole term of a cell)."""
    xi = _f64(np.atleast_1d(xi))
    out = np.empty_like(xi)
    lib().or_gcut_deriv2_vec(_i64(xi.size), _ptr(xi), _ptr(out))
    return out


def quad_term(d, S, r_cut, eps):
    """1/2 S_ab d_a d_b F(d) of one unit-weighted second-moment tensor
    S = (xx, yy, zz, xy, xz, yz) at offset d (source minus target)."""
    S = _f64(S)
    out = np.empty(3)
    lib().or_quad_term(_d(d[0]), _d(d[1]), _d(d[2]), _ptr(S), _d(r_cut), _d(eps), _ptr(out))
    return out


def second_moments(tree: "Tree", ux, uy, uz, m, X):
    """Second moments S [nn, 6] = (xx, yy, zz, xy, xz, yz) of every cell
    about its centre of mass X [nn, 3] (sorted-order inputs)."""
    nn = tree.size
    S = np.empty((nn, 6))
    X0, X1, X2 = (np.ascontiguousarray(X[:, k]) for k in range(3))
    lib().or_second_moments(_i64(nn), _ptr(tree.level), _ptr(tree.prefix), _ptr(tree.first), _ptr(tree.count),
                            _ptr(_f64(ux)), _ptr(_f64(uy)),
                            _ptr(_f64(uz)), _ptr(_f64(m)), _ptr(X0), _ptr(X1), _ptr(X2), _ptr(S))
    return S


def qcut(xi):
    """Potential factor q of the split (short-range potential -G m q(xi) / r)."""
    xi = _f64(xi)
    q = np.empty_like(xi)
    lib().or_qcut_vec(_i64(xi.size), _ptr(xi), _ptr(q))
    return q


def brute_force_potential(x, y, z, m, G, r_cut, eps):
    """Short-range potential by O(N^2) minimum-image summation (j != i)."""
    x, y, z, m = map(_f64, (x, y, z, m))
    phi = np.empty(x.size)
    lib().or_bf_potential_n2(_i64(x.size), _ptr(x), _ptr(y), _ptr(z), _ptr(m), _d(G), _d(r_cut), _d(eps),
                             _ptr(phi))
    return phi


def pair_force(d, r_cut, eps):
    """F(d) = d (|d|^2+eps^2)^(-3/2) g(2|d|/r_cut) [|d| < r_cut] for one offset."""
    out = np.empty(3)
    lib().or_pair_force(_d(d[0]), _d(d[1]), _d(d[2]), _d(r_cut), _d(eps), _ptr(out))
    return out


def pair_jac(d, w, r_cut, eps):
    """J(d) w, J = dF/dd."""
    w = _f64(w)
    out = np.empty(3)
    lib().or_pair_jac(_d(d[0]), _d(d[1]), _d(d[2]), _d(r_cut), _d(eps), _ptr(w), _ptr(out))
    return out


# ------------------------------------------------------------- brute force
def brute_force(x, y, z, m, G, r_cut, eps, method="cells"):
    """Exact short-range accelerations (minimum image, all pairs within r_cut)."""
    x, y, z, m = map(_f64, (x, y, z, m))
    n = x.size
    ax, ay, az = np.empty(n), np.empty(n), np.empty(n)
    fn = lib().or_bf_cells if method == "cells" else lib().or_bf_n2
    fn(_i64(n), _ptr(x), _ptr(y), _ptr(z), _ptr(m), _d(G), _d(r_cut), _d(eps), _ptr(ax), _ptr(ay), _ptr(az))
    return np.stack([ax, ay, az], axis=1)


def brute_force_sel(x, y, z, m, G, r_cut, eps, sel, count_pairs=False):
    """Exact short-range accelerations of the particles sel (input indices);
    with ``count_pairs`` also the number of pairs within r_cut summed."""
    x, y, z, m = map(_f64, (x, y, z, m))
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    ax, ay, az = np.empty(sel.size), np.empty(sel.size), np.empty(sel.size)
    npairs = np.zeros(1, np.int64)
    lib().or_bf_cells_sel(_i64(x.size), _ptr(x), _ptr(y), _ptr(z), _ptr(m), _d(G), _d(r_cut), _d(eps),
                          _ptr(sel), _i64(sel.size), _ptr(ax), _ptr(ay), _ptr(az), _ptr(npairs))
    a = np.stack([ax, ay, az], axis=1)
    return (a, int(npairs[0])) if count_pairs else a


def pair_count(x, y, z, r_cut) -> int:
    x, y, z = map(_f64, (x, y, z))
    return int(lib().or_bf_pair_count(_i64(x.size), _ptr(x), _ptr(y), _ptr(z), _d(r_cut)))


def brute_force_adjoint(x, y, z, m, w, G, r_cut, eps):
    """Gradient of L = sum w_i . a_i for the exact sum: (dL/dx [N,3], dL/dm [N])."""
    x, y, z, m = map(_f64, (x, y, z, m))
    w = _f64(w)
    n = x.size
    wx, wy, wz = (np.ascontiguousarray(w[:, k]) for k in range(3))
    gx, gy, gz, gm = (np.empty(n) for _ in range(4))
    lib().or_bf_adjoint(_i64(n), _ptr(x), _ptr(y), _ptr(z), _ptr(m), _ptr(wx), _ptr(wy), _ptr(wz),
                        _d(G), _d(r_cut), _d(eps), _ptr(gx), _ptr(gy), _ptr(gz), _ptr(gm))
    return np.stack([gx, gy, gz], axis=1), gm


# ------------------------------------------------------------ tree steps
def wrap(v):
    return np.array([lib().or_wrap(float(t)) for t in np.atleast_1d(v)])


def morton_keys(x, y, z):
    """a1: keys in input order and the wrapped positions."""
    x, y, z = map(_f64, (x, y, z))
    n = x.size
    keys = np.empty(n, dtype=np.uint64)
    ux, uy, uz = np.empty(n), np.empty(n), np.empty(n)
    lib().or_morton_keys(_i64(n), _ptr(x), _ptr(y), _ptr(z), _ptr(keys), _ptr(ux), _ptr(uy), _ptr(uz))
    return keys, ux, uy, uz


def sort_keys(keys):
    """a2: order by (key, original index): (sorted keys, perm)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    ks = np.empty_like(keys)
    perm = np.empty(keys.size, dtype=np.int64)
    lib().or_sort(_i64(keys.size), _ptr(keys), _ptr(ks), _ptr(perm))
    return ks, perm


@dataclass
class Tree:
    level: np.ndarray    # int32
    prefix: np.ndarray   # uint64
    first: np.ndarray    # int64
    count: np.ndarray    # int64
    parent: np.ndarray   # int64 (-1 for the root)
    child: np.ndarray    # int64 [nn, 8], -1 if empty
    leaf: np.ndarray     # uint8

    @property
    def size(self) -> int:
        return int(self.level.size)


def build_tree(keys_sorted, n_leaf: int) -> Tree:
    """a3: cells in DFS preorder."""
    ks = np.ascontiguousarray(keys_sorted, dtype=np.uint64)
    n = ks.size
    nn = int(lib().or_tree_count(_i64(n), _ptr(ks), _i64(n_leaf)))
    t = Tree(np.empty(nn, np.int32), np.empty(nn, np.uint64), np.empty(nn, np.int64), np.empty(nn, np.int64),
             np.empty(nn, np.int64), np.empty((nn, 8), np.int64), np.empty(nn, np.uint8))
    lib().or_tree_fill(_i64(n), _ptr(ks), _i64(n_leaf), _ptr(t.level), _ptr(t.prefix), _ptr(t.first),
                       _ptr(t.count), _ptr(t.parent), _ptr(t.child), _ptr(t.leaf))
    return t


def moments(tree: Tree, ux, uy, uz, m):
    """a4: monopole mass and centre of mass of every cell (sorted-order
    inputs), positions taken at their images nearest the cell's centre."""
    nn = tree.size
    M, X, Y, Z = (np.empty(nn) for _ in range(4))
    lib().or_moments(_i64(nn), _ptr(tree.level), _ptr(tree.prefix), _ptr(tree.first), _ptr(tree.count),
                     _ptr(_f64(ux)), _ptr(_f64(uy)),
                     _ptr(_f64(uz)), _ptr(_f64(m)), _ptr(M), _ptr(X), _ptr(Y), _ptr(Z))
    return M, np.stack([X, Y, Z], axis=1)


def groups(tree: Tree, n_group: int, n: int):
    """a5: (gfirst, gcount) in order of first."""
    gf = np.empty(max(n, 1), np.int64)
    gc = np.empty(max(n, 1), np.int64)
    ng = int(lib().or_groups(_ptr(tree.level), _ptr(tree.first), _ptr(tree.count), _ptr(tree.child),
                             _i64(n_group), _ptr(gf), _ptr(gc)))
    return gf[:ng].copy(), gc[:ng].copy()


def group_bbox(gfirst, gcount, ux, uy, uz):
    ng = gfirst.size
    lo, hi = np.empty((ng, 3)), np.empty((ng, 3))
    lib().or_group_bbox(_i64(ng), _ptr(gfirst), _ptr(gcount), _ptr(_f64(ux)), _ptr(_f64(uy)), _ptr(_f64(uz)),
                        _ptr(lo), _ptr(hi))
    return lo, hi


@dataclass
class Lists:
    poff: np.ndarray   # int64 [ng+1]
    pidx: np.ndarray   # int64 sorted particle indices, ascending within a group
    noff: np.ndarray   # int64 [ng+1]
    nidx: np.ndarray   # int64 node ids (preorder), ascending within a group


def make_lists(tree: Tree, lo, hi, r_cut: float, theta: float, com=None, boxes=None) -> Lists:
    """a6: per-group lists in canonical order (two passes: count, fill).
    With ``com`` ([nn, 3] centres of mass) the opening criterion measures
    the distance to each cell's centre of mass instead of its geometric
    centre (the pruning stays box to box).  With ``boxes`` = (clo, chi)
    ([nn, 3] each, a refitted tree) cells are measured by those boxes."""
    ng = lo.shape[0]
    lo = _f64(lo)
    hi = _f64(hi)
    np_, nn_ = np.empty(ng, np.int64), np.empty(ng, np.int64)
    if com is None:
        cx = cy = cz = None
    else:
        cx, cy, cz = (np.ascontiguousarray(com[:, k], dtype=np.float64) for k in range(3))
    clo = chi = None
    if boxes is not None:
        clo, chi = (_f64(b) for b in boxes)
    args = (_ptr(tree.level), _ptr(tree.prefix), _ptr(tree.first), _ptr(tree.count), _ptr(tree.child),
            _ptr(tree.leaf), _d(r_cut), _d(theta), _ptr(cx), _ptr(cy), _ptr(cz), _ptr(clo), _ptr(chi))
    lib().or_lists_count(_i64(ng), _ptr(lo), _ptr(hi), *args, _ptr(np_), _ptr(nn_))
    poff = np.zeros(ng + 1, np.int64)
    noff = np.zeros(ng + 1, np.int64)
    np.cumsum(np_, out=poff[1:])
    np.cumsum(nn_, out=noff[1:])
    pidx = np.empty(int(poff[-1]), np.int64)
    nidx = np.empty(int(noff[-1]), np.int64)
    lib().or_lists_fill(_i64(ng), _ptr(lo), _ptr(hi), *args, _ptr(poff), _ptr(noff), _ptr(pidx), _ptr(nidx))
    return Lists(poff, pidx, noff, nidx)


class OracleTree:
    """The whole forward structure (a1-a6) for one particle set, plus the
    same-list force (a7, a8) and the fixed-structure adjoint (a9)."""

    def __init__(self, x, y, z, m, params):
        self.params = params
        x, y, z, m = map(_f64, (x, y, z, m))
        self.n = x.size
        self.keys_in, ux, uy, uz = morton_keys(x, y, z)
        self.keys, self.perm = sort_keys(self.keys_in)
        self.ux, self.uy, self.uz = ux[self.perm], uy[self.perm], uz[self.perm]
        self.m = m[self.perm]
        self.tree = build_tree(self.keys, params.n_leaf)
        self.M, self.X = moments(self.tree, self.ux, self.uy, self.uz, self.m)
        self.gfirst, self.gcount = groups(self.tree, params.n_group, self.n)
        self.lo, self.hi = group_bbox(self.gfirst, self.gcount, self.ux, self.uy, self.uz)
        self.lists = make_lists(self.tree, self.lo, self.hi, params.r_cut, params.theta,
                                com=self.X if getattr(params, "mac", 0) == 1 else None)

    @property
    def n_groups(self) -> int:
        return int(self.gfirst.size)

    def refitted(self, x, y, z, m=None):
        """The tree reused at new positions (input order) with the sort
        order, cells and groups held: positions wrapped and taken in the old
        sorted order, moments recomputed, each cell and group measured by
        the box of its particles (moved to the image nearest the cell's
        dyadic centre, or the group's first particle), and the lists built
        on those boxes.  Returns a new OracleTree."""
        import copy

        r = copy.copy(self)
        _, ux, uy, uz = morton_keys(x, y, z)
        r.ux, r.uy, r.uz = ux[self.perm], uy[self.perm], uz[self.perm]
        if m is not None:
            r.m = _f64(m)[self.perm]
        r.M, r.X = moments(self.tree, r.ux, r.uy, r.uz, r.m)
        nn = self.tree.size
        r.clo, r.chi = np.empty((nn, 3)), np.empty((nn, 3))
        t = self.tree
        lib().or_refit_cell_boxes(_i64(nn), _ptr(t.level), _ptr(t.prefix), _ptr(t.first), _ptr(t.count),
                                  _ptr(t.child), _ptr(t.leaf), _ptr(r.ux), _ptr(r.uy), _ptr(r.uz), _ptr(r.clo),
                                  _ptr(r.chi))
        r.lo, r.hi = np.empty((self.n_groups, 3)), np.empty((self.n_groups, 3))
        lib().or_refit_group_bbox(_i64(self.n_groups), _ptr(self.gfirst), _ptr(self.gcount), _ptr(r.ux), _ptr(r.uy),
                                  _ptr(r.uz), _ptr(r.lo), _ptr(r.hi))
        p = self.params
        r.lists = make_lists(t, r.lo, r.hi, p.r_cut, p.theta, com=r.X if getattr(p, "mac", 0) == 1 else None,
                             boxes=(r.clo, r.chi))
        r._S = None
        return r

    def refit_qboxes(self):
        """(qlo, qhi, bounded) of a refitted tree: each cell's box rounded
        outward to multiples of 2^-(level+10), as the list decisions use it;
        bounded is False where a bound lies beyond 32767 such steps from the
        cell's centre (the cell is then never pruned or accepted)."""
        nn = self.tree.size
        qlo, qhi, ok = np.empty((nn, 3)), np.empty((nn, 3)), np.empty(nn, np.uint8)
        lib().or_refit_qboxes(_i64(nn), _ptr(self.tree.level), _ptr(self.tree.prefix), _ptr(self.clo),
                              _ptr(self.chi), _ptr(qlo), _ptr(qhi), _ptr(ok))
        return qlo, qhi, ok.astype(bool)

    def interactions(self) -> int:
        """I = sum over groups of N_i * N_j (the paper's count, Table I)."""
        nj = np.diff(self.lists.poff) + np.diff(self.lists.noff)
        return int(np.sum(self.gcount * nj))

    def force_sorted(self, ux=None, uy=None, uz=None, m=None, sel=None):
        """a7 in sorted order.  Optional inputs replace positions/masses with
        the structure held fixed (moments recomputed from them)."""
        p = self.params
        ux = self.ux if ux is None else _f64(ux)
        uy = self.uy if uy is None else _f64(uy)
        uz = self.uz if uz is None else _f64(uz)
        m = self.m if m is None else _f64(m)
        if ux is self.ux and uy is self.uy and uz is self.uz and m is self.m:
            M, X = self.M, self.X
        else:
            M, X = moments(self.tree, ux, uy, uz, m)
        X0, X1, X2 = (np.ascontiguousarray(X[:, k]) for k in range(3))
        ax, ay, az = np.zeros(self.n), np.zeros(self.n), np.zeros(self.n)
        L = self.lists
        if sel is None:
            sel_arr, nsel = None, -1
        else:
            sel_arr = np.ascontiguousarray(sel, dtype=np.int64)
            nsel = sel_arr.size
        lib().or_tree_force(_i64(self.n_groups), _ptr(self.gfirst), _ptr(self.gcount), _ptr(L.poff), _ptr(L.pidx),
                            _ptr(L.noff), _ptr(L.nidx), _ptr(ux), _ptr(uy), _ptr(uz), _ptr(m), _ptr(M),
                            _ptr(X0), _ptr(X1), _ptr(X2), _d(p.G), _d(p.r_cut), _d(p.eps),
                            _ptr(sel_arr), _i64(nsel), _ptr(ax), _ptr(ay), _ptr(az))
        return np.stack([ax, ay, az], axis=1)

    def force(self):
        """a7 + a8: accelerations in input order."""
        a = np.empty((self.n, 3))
        a[self.perm] = self.force_sorted()
        return a

    def potential(self):
        """Same-list short-range potential in input order (the target itself left out)."""
        p = self.params
        X0, X1, X2 = (np.ascontiguousarray(self.X[:, k]) for k in range(3))
        phi = np.empty(self.n)
        L = self.lists
        lib().or_tree_potential(_i64(self.n_groups), _ptr(self.gfirst), _ptr(self.gcount), _ptr(L.poff),
                                _ptr(L.pidx), _ptr(L.noff), _ptr(L.nidx), _ptr(self.ux), _ptr(self.uy),
                                _ptr(self.uz), _ptr(self.m), _ptr(self.M), _ptr(X0), _ptr(X1), _ptr(X2), _d(p.G),
                                _d(p.r_cut), _d(p.eps), _ptr(phi))
        out = np.empty(self.n)
        out[self.perm] = phi
        return out

    def second_moments(self):
        if getattr(self, "_S", None) is None:
            self._S = second_moments(self.tree, self.ux, self.uy, self.uz, self.m, self.X)
        return self._S

    def quad_correction_sorted(self, sel=None):
        """Quadrupole term of every cell entry of each group's list (sorted order)."""
        p = self.params
        S = self.second_moments()
        X0, X1, X2 = (np.ascontiguousarray(self.X[:, k]) for k in range(3))
        ax, ay, az = np.zeros(self.n), np.zeros(self.n), np.zeros(self.n)
        if sel is None:
            sel_arr, nsel = None, -1
        else:
            sel_arr = np.ascontiguousarray(sel, dtype=np.int64)
            nsel = sel_arr.size
        L = self.lists
        lib().or_tree_quad(_i64(self.n_groups), _ptr(self.gfirst), _ptr(self.gcount), _ptr(L.noff), _ptr(L.nidx),
                           _ptr(self.ux), _ptr(self.uy), _ptr(self.uz), _ptr(X0), _ptr(X1), _ptr(X2), _ptr(S),
                           _d(p.G), _d(p.r_cut), _d(p.eps), _ptr(sel_arr), _i64(nsel), _ptr(ax), _ptr(ay), _ptr(az))
        return np.stack([ax, ay, az], axis=1)

    def force_quadrupole(self):
        """Same-list force with the cells' quadrupole terms, input order."""
        a = np.empty((self.n, 3))
        a[self.perm] = self.force_sorted() + self.quad_correction_sorted()
        return a

    def _inputs(self, ux, uy, uz, m):
        """Sorted positions and masses (the tree's own unless replaced, with
        the structure held fixed) and the cell moments of them."""
        ux = self.ux if ux is None else _f64(ux)
        uy = self.uy if uy is None else _f64(uy)
        uz = self.uz if uz is None else _f64(uz)
        m = self.m if m is None else _f64(m)
        if ux is self.ux and uy is self.uy and uz is self.uz and m is self.m:
            M, X = self.M, self.X
        else:
            M, X = moments(self.tree, ux, uy, uz, m)
        return ux, uy, uz, m, M, [np.ascontiguousarray(X[:, k]) for k in range(3)]

    def adjoint(self, w, ux=None, uy=None, uz=None):
        """a9: (dL/dx [N,3], dL/dm [N]) in input order for L = sum_i w_i . a_i
        (optionally at other sorted positions, structure held fixed)."""
        p = self.params
        w = _f64(w)[self.perm]
        wx, wy, wz = (np.ascontiguousarray(w[:, k]) for k in range(3))
        ux, uy, uz, m, M, (X0, X1, X2) = self._inputs(ux, uy, uz, None)
        gx, gy, gz, gm = (np.empty(self.n) for _ in range(4))
        L = self.lists
        lib().or_tree_adjoint(_i64(self.n), _i64(self.n_groups), _ptr(self.gfirst), _ptr(self.gcount),
                              _ptr(L.poff), _ptr(L.pidx), _ptr(L.noff), _ptr(L.nidx),
                              _i64(self.tree.size), _ptr(self.tree.first), _ptr(self.tree.count),
                              _ptr(self.tree.level), _ptr(self.tree.prefix), _ptr(ux), _ptr(uy), _ptr(uz), _ptr(m), _ptr(M),
                              _ptr(X0), _ptr(X1), _ptr(X2), _ptr(wx), _ptr(wy), _ptr(wz),
                              _d(p.G), _d(p.r_cut), _d(p.eps), _ptr(gx), _ptr(gy), _ptr(gz), _ptr(gm))
        gxs = np.stack([gx, gy, gz], axis=1)
        out_x = np.empty_like(gxs)
        out_m = np.empty_like(gm)
        out_x[self.perm] = gxs
        out_m[self.perm] = gm
        return out_x, out_m

    def force_bound_sorted(self, u_k, u_c=2.0 ** -53, e_abs=0.0, sel=None):
        """Per-particle error magnitude E of the same-list force (sorted order;
        only the groups `sel` if given): the sum over the list of
        m_j ||J|| e_j, e_j the uncertainty of the pair's offset when the group-
        relative offsets and their difference are rounded with unit roundoff
        u_k, every offset is further moved by up to e_abs, and cell centres of
        mass carry their FP64 summation error u_c (2 n_c + 2).  A kernel that
        sums K terms in working precision is then within about (K + pair
        roundings) * E of the exact result."""
        p = self.params
        X0, X1, X2 = (np.ascontiguousarray(self.X[:, k]) for k in range(3))
        E = np.zeros(self.n)
        L = self.lists
        if sel is None:
            sel_arr, nsel = None, -1
        else:
            sel_arr = np.ascontiguousarray(sel, dtype=np.int64)
            nsel = sel_arr.size
        lib().or_tree_force_bound(_i64(self.n_groups), _ptr(self.gfirst), _ptr(self.gcount), _ptr(L.poff),
                                  _ptr(L.pidx), _ptr(L.noff), _ptr(L.nidx), _ptr(self.ux), _ptr(self.uy),
                                  _ptr(self.uz), _ptr(self.m), _ptr(self.M), _ptr(X0), _ptr(X1), _ptr(X2),
                                  _ptr(self.tree.count), _ptr(self.lo), _ptr(self.hi), _d(p.G), _d(p.r_cut),
                                  _d(p.eps), _d(u_k), _d(u_c), _d(e_abs), _ptr(sel_arr), _i64(nsel), _ptr(E))
        return E

    def force_bound(self, u_k, u_c=2.0 ** -53, e_abs=0.0):
        """force_bound_sorted in input order."""
        out = np.empty(self.n)
        out[self.perm] = self.force_bound_sorted(u_k, u_c, e_abs)
        return out

    def adjoint_bound(self, w, u_k, u_c=2.0 ** -53, e_abs=0.0):
        """Per-particle error magnitudes (Ex, Em) of dL/dx and dL/dm, input
        order, under the perturbations of force_bound_sorted: per pair the
        error of J w is |w| (u_k ||J|| + ||dJ/dd|| e) and that of w . F is
        |w| ||J|| e, passed from cells to their particles by the chain rule."""
        p = self.params
        w = _f64(w)[self.perm]
        wx, wy, wz = (np.ascontiguousarray(w[:, k]) for k in range(3))
        X0, X1, X2 = (np.ascontiguousarray(self.X[:, k]) for k in range(3))
        Ex, Em = np.empty(self.n), np.empty(self.n)
        L = self.lists
        lib().or_tree_adjoint_bound(_i64(self.n), _i64(self.n_groups), _ptr(self.gfirst), _ptr(self.gcount),
                                    _ptr(L.poff), _ptr(L.pidx), _ptr(L.noff), _ptr(L.nidx),
                                    _i64(self.tree.size), _ptr(self.tree.first), _ptr(self.tree.count),
                                    _ptr(self.tree.level), _ptr(self.tree.prefix), _ptr(self.ux), _ptr(self.uy), _ptr(self.uz), _ptr(self.m), _ptr(self.M),
                                    _ptr(X0), _ptr(X1), _ptr(X2), _ptr(wx), _ptr(wy), _ptr(wz), _ptr(self.lo),
                                    _ptr(self.hi), _d(p.G), _d(p.r_cut), _d(p.eps), _d(u_k), _d(u_c), _d(e_abs),
                                    _ptr(Ex), _ptr(Em))
        ox, om = np.empty(self.n), np.empty(self.n)
        ox[self.perm] = Ex
        om[self.perm] = Em
        return ox, om

    def loss(self, w, ux=None, uy=None, uz=None, m=None):
        """L = sum_i w_i . a_i with the structure fixed; w in input order."""
        a = self.force_sorted(ux, uy, uz, m)
        return float(np.sum(_f64(w)[self.perm] * a))


def relative_errors(a, ref):
    """Per-particle |a - ref| / |ref| over particles with |ref| > 0, and
    summary statistics (rms, median, p99, max, global L2 ratio)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    nr = np.linalg.norm(ref, axis=1)
    nz = nr > 0
    e = np.linalg.norm(a - ref, axis=1)[nz] / nr[nz]
    if e.size == 0:
        return e, dict(rms=0.0, median=0.0, p99=0.0, max=0.0, l2=0.0, n_zero_ref=int((~nz).sum()))
    stats = dict(rms=float(np.sqrt(np.mean(e * e))), median=float(np.median(e)),
                 p99=float(np.percentile(e, 99)), max=float(e.max()),
                 l2=float(np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300)),
                 n_zero_ref=int((~nz).sum()))
    return e, stats
