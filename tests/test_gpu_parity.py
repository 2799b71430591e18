"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bit-exact: Morton keys, sort permutation, cells (level, prefix, first,
count), groups and their boxes, interaction lists (canonical form).
Floating point, for every particle: |x_i - x_i^ref| <= C E_i with E_i the
oracle's first-order error magnitude of that particle and C the stated count
of roundings (tests/_parity.py); in addition the FP32 force and dL/dx keep
a per-particle rms relative error <= 1e-5 and the FP64 force <= 1e-12 where
the forces do not cancel strongly.
"""
import ctypes as C
import dataclasses
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_1211_4406_amd as srf
import synth
from _parity import U32, U64, check, constant, max_list

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
FP64_TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_inputs(ps):
    x = torch.tensor(ps.positions(), dtype=torch.float64, device="cuda")
    m = torch.tensor(ps.m, dtype=torch.float64, device="cuda")
    return x, m


def gpu_forward(ps, params=None, precision=srf.FP32_REL):
    p = srf.Params.of(params or ps.params, precision)
    x, m = dev_inputs(ps)
    tree = srf.tree_build(x, m, p)
    lists = srf.make_lists(tree, p)
    a = srf.short_range_force(tree, lists, p)
    torch.cuda.synchronize()
    return tree, lists, a.cpu().numpy()


def check_structure(tree, lists, ot):
    ex = tree.export()
    assert np.array_equal(ex["keys"], ot.keys), "keys"
    assert np.array_equal(ex["perm"], ot.perm), "perm"
    assert np.array_equal(ex["level"], ot.tree.level), "cell levels"
    assert np.array_equal(ex["prefix"], ot.tree.prefix), "cell prefixes"
    assert np.array_equal(ex["first"], ot.tree.first), "cell first"
    assert np.array_equal(ex["count"], ot.tree.count), "cell count"
    assert np.array_equal(ex["gfirst"], ot.gfirst), "group first"
    assert np.array_equal(ex["gcount"], ot.gcount), "group count"
    assert np.array_equal(ex["lo"], ot.lo) and np.array_equal(ex["hi"], ot.hi), "group boxes"
    L = lists.export()
    for k in ("poff", "pidx", "noff", "nidx"):
        assert np.array_equal(L[k], getattr(ot.lists, k)), k
    info = lists.info()
    assert info["interactions"] == ot.interactions()
    M, X = tree.moments()
    # different summation orders: bounded by count * unit roundoff (for X
    # times the coordinate range, 1)
    assert np.max(np.abs(M - ot.M) / ot.M / ot.tree.count) < 1e-15
    assert np.all(np.abs(X - ot.X) <= 1e-15 + 2.3e-16 * ot.tree.count[:, None])


def rel_stats(a, ref):
    return oracle.relative_errors(a, ref)[1]


def check_force(ot, a, ref, fp64, what, E=None):
    """Element-wise bound of a force (input order) against the oracle's."""
    if E is None:
        E = ot.force_bound(U64 if fp64 else U32)
    return check(a, ref, E, constant("force", fp64, max_list(ot)), what)


def check_adjoint(ot, w, gx, gm, rx, rm, fp64, what):
    """Element-wise bounds of dL/dx and dL/dm (input order)."""
    Ex, Em = ot.adjoint_bound(w, U64 if fp64 else U32)
    C = constant("adjoint", fp64, max_list(ot))
    return check(gx, rx, Ex, C, what + " dL/dx"), check(gm, rm, Em, C, what + " dL/dm")


# ----------------------------------------------------------------- cases
def case_sets():
    return {
        "cfg1-uniform-4096": synth.make_config(1),
        "clustered-20000": synth.small_clustered(20000, 101, r_cut=0.1, eps=2e-4, theta=0.5, per_halo=1000),
        "clustered-tight-12000": synth.small_clustered(12000, 102, r_cut=0.1, eps=5e-5, theta=0.7, per_halo=3000,
                                                       a_range=(2e-4, 2e-3)),
    }


@pytest.mark.parametrize("name", ["cfg1-uniform-4096", "clustered-20000", "clustered-tight-12000"])
@pytest.mark.parametrize("theta", [0.0, 0.5, 1.0])
def test_structure_and_force_parity(name, theta):
    ps = case_sets()[name]
    params = synth.Params(1.0, ps.params.r_cut, ps.params.eps, theta, 64, 16)
    say(f"[gpu] structure/force {name} theta={theta} n={ps.n}")
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, params)
    ref = ot.force()
    tree, lists, a32 = gpu_forward(ps, params, srf.FP32_REL)
    check_structure(tree, lists, ot)
    st = rel_stats(a32, ref)
    say(f"    fp32 vs oracle: {st}")
    assert st["rms"] <= FP32_TOL
    check_force(ot, a32, ref, False, "fp32 force")
    _, _, a64 = gpu_forward(ps, params, srf.FP64)
    st64 = rel_stats(a64, ref)
    say(f"    fp64 vs oracle: {st64}")
    check_force(ot, a64, ref, True, "fp64 force")
    # the tight halos (eps = 5e-5, scale radii from 2e-4) hold particles
    # whose net force is a strongly cancelling sum (|a_i| far below the sum
    # of its pair terms): there the element-wise bound above is the test and
    # the rms relative error is only reported
    if "tight" not in name:
        assert st64["rms"] <= FP64_TOL


def test_g_and_zero_beyond_cutoff_two_bodies():
    # two particles at chosen separations, across the periodic face
    rc, eps = 0.1, 1e-3
    for r in (0.0004, 0.003, 0.02, 0.049, 0.05, 0.07, 0.09, 0.0999, 0.1 * (1 + 1e-6), 0.12):
        x = np.array([[0.995, 0.5, 0.5], [0.995 + r, 0.5, 0.5]])
        ps = synth.ParticleSet(x[:, 0].copy(), x[:, 1].copy(), x[:, 2].copy(), np.array([0.25, 0.75]),
                               synth.Params(1.0, rc, eps, 0.5, 64, 16))
        _, _, a32 = gpu_forward(ps)
        _, _, a64 = gpu_forward(ps, precision=srf.FP64)
        ref = oracle.brute_force(ps.x, ps.y, ps.z, ps.m, 1.0, rc, eps, method="n2")
        if r >= rc:
            assert np.all(a32 == 0.0) and np.all(a64 == 0.0)
        else:
            # near the cutoff g ~ (2 - xi)^5 amplifies the rounding of r by
            # 5 / (2 - xi): FP64 keeps 1e-12 there, FP32 offsets about 1e-3
            near = 2 * r / rc > 1.99
            assert np.allclose(a64, ref, rtol=1e-12 if near else 1e-13, atol=0)
            assert np.allclose(a32, ref, rtol=1e-3 if near else 5e-6, atol=0)
            assert a32[0, 0] > 0 > a32[1, 0]


def test_edge_cases():
    rng = np.random.default_rng(3)
    p = synth.Params(1.0, 0.1, 1e-3, 0.5, 64, 16)
    cases = {}
    cases["n1"] = np.array([[0.3, 0.4, 0.5]])
    cases["n40"] = rng.random((40, 3))
    cases["n64"] = rng.random((64, 3))
    cases["n65"] = rng.random((65, 3))
    # positions outside the box, negative zero, a tiny negative value, exactly 1.0
    pos = rng.random((300, 3)) * 4.0 - 2.0
    pos[0] = [-1e-17, 1.0, -0.0]
    pos[1] = [1.0 - 2 ** -53, 2.0, -3.0]
    cases["wrapped"] = pos
    # particles exactly on dyadic cell faces
    g = np.arange(16) / 16.0
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    cases["faces"] = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    # 150 coincident particles (a level-21 cell larger than a group) plus a background
    co = np.concatenate([np.full((150, 3), 0.123456789), rng.random((500, 3))])
    cases["coincident"] = co
    for name, pos in cases.items():
        say(f"[gpu] edge case {name} n={len(pos)}")
        n = len(pos)
        ps = synth.ParticleSet(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.full(n, 1.0 / n), p)
        ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p)
        tree, lists, a32 = gpu_forward(ps, p)
        check_structure(tree, lists, ot)
        ref = ot.force()
        if n == 1:
            assert np.all(a32 == 0.0)
            continue
        _, _, a64 = gpu_forward(ps, p, srf.FP64)
        if name == "coincident":
            # coincident pairs have d = 0 and contribute exactly nothing
            assert np.all(np.isfinite(a32))
        # every particle within its element-wise bound: in the sparse sets
        # groups as large as a level-1 cell put FP32 offsets up to 0.5 from
        # the group centre, and some particles feel only pairs right at the
        # cutoff; the bound carries both (offset sizes, the kernel's
        # sensitivity there)
        check_force(ot, a32, ref, False, "fp32 force")
        check_force(ot, a64, ref, True, "fp64 force")
        if name == "faces":
            # a perfect lattice: every force cancels to rounding noise, so
            # compare against the scale of one nearest-neighbour pair force
            scale = (1.0 / n) / (1.0 / 16) ** 2
            assert np.max(np.abs(a64 - ref)) <= 1e-13 * scale
            assert np.max(np.abs(a32 - ref)) <= 1e-5 * scale
            continue
        s64, s32 = rel_stats(a64, ref), rel_stats(a32, ref)
        say(f"    fp64 {s64}")
        say(f"    fp32 {s32}")


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_lists_with_distances_exactly_at_the_thresholds(theta):
    """A 32^3 lattice with r_cut = 5/32: cell and group boxes sit on
    multiples of 1/32, so many squared distances equal r_cut^2 exactly (a
    tie: pruned) and many equal (side / theta)^2 exactly (a tie: not
    accepted).  The walk's FP32 first look must leave every such case to the
    FP64 expressions; the structure and lists must match the oracle's bit
    for bit."""
    g = np.arange(32) / 32.0
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    n = len(pos)
    p = synth.Params(1.0, 5.0 / 32.0, 1e-3, theta, 64, 16)
    ps = synth.ParticleSet(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.full(n, 1.0 / n), p)
    say(f"[gpu] lattice ties theta={theta} n={n}")
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p)
    tree, lists, a32 = gpu_forward(ps, p)
    check_structure(tree, lists, ot)
    assert lists.info()["n_node_entries"] > 0   # accepted cells, some of them next to a tie


@pytest.mark.parametrize("n,distinct", [(4096, 4096), (4097, 4097), (8191, 8191), (100_000, 1000), (70_000, 7)])
def test_sort_tiles_and_repeated_keys(n, distinct):
    """The radix sort at exactly one tile of 4096 keys, one past it, one
    short of two tiles, and with heavily repeated keys (each of `distinct`
    positions taken by many particles, so long runs of equal digits inside
    every tile and level-21 cells cut into groups): keys, permutation (ties
    by input index), cells, groups and lists equal the oracle's."""
    rng = np.random.default_rng(900 + distinct)
    base = rng.random((distinct, 3))
    pos = base[rng.integers(0, distinct, n)] if distinct < n else base
    say(f"[gpu] sort n={n} distinct={distinct}")
    p = synth.Params(1.0, 0.05, 1e-3, 0.5, 64, 16)
    ps = synth.ParticleSet(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.full(n, 1.0 / n), p)
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p)
    tree, lists, a32 = gpu_forward(ps, p)
    check_structure(tree, lists, ot)
    assert np.all(np.isfinite(a32))


@pytest.mark.parametrize("clump", [300, 1024, 1025, 3000])
def test_sort_runs_sharing_the_high_key_word(clump):
    """Clumps of `clump` particles, each inside a cube of side 2e-4 centred in
    a level-11 cell (so every member shares the high 32-bit word of its key
    but not the low word), over a uniform background: the sort orders each
    run by the low word and the index when it holds at most 1024 particles,
    and the tree is built again on the full sort when a run is longer;
    either way keys, permutation, cells, groups and lists equal the
    oracle's."""
    rng = np.random.default_rng(1700 + clump)
    n_clumps, n_bg = 3, 20_000
    cells = rng.integers(0, 2 ** 11, (n_clumps, 3))
    parts = [rng.random((n_bg, 3))]
    for c in cells:
        centre = (c + 0.5) / 2 ** 11
        parts.append(centre + (rng.random((clump, 3)) - 0.5) * 2e-4)
    pos = np.concatenate(parts)[rng.permutation(n_bg + n_clumps * clump)]
    n = len(pos)
    say(f"[gpu] sort runs clump={clump} n={n}")
    p = synth.Params(1.0, 0.05, 1e-4, 0.5, 64, 16)
    ps = synth.ParticleSet(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.full(n, 1.0 / n), p)
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p)
    hi = ot.keys >> np.uint64(32)
    starts = np.flatnonzero(np.concatenate([[True], hi[1:] != hi[:-1], [True]]))
    assert np.diff(starts).max() == clump, "each clump is one run of equal high words"
    tree, lists, a32 = gpu_forward(ps, p)
    check_structure(tree, lists, ot)
    assert np.all(np.isfinite(a32))


def test_lists_with_more_items_than_a_slot():
    """With single-particle leaves and a wide cutoff every group's list holds
    more than 2048 leaves and cells, which overflows the per-group slot of
    the counting walk and takes the second, compacting walk; the lists must
    still equal the oracle's bit for bit."""
    rng = np.random.default_rng(303)
    n = 300_000
    pos = rng.random((n, 3))
    ps = synth.ParticleSet(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.full(n, 1.0 / n),
                           synth.Params(1.0, 0.12, 1e-3, 0.3, 64, 1), "uniform-300k-leaf1")
    say(f"[gpu] list slot overflow n={n}")
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    items = np.diff(ot.lists.poff) + np.diff(ot.lists.noff)   # one item per single-particle leaf or cell
    assert items.max() > 2048
    tree, lists, a32 = gpu_forward(ps)
    check_structure(tree, lists, ot)
    st = sampled_force_check(ps, a32, ot, n_groups=100)
    say(f"    fp32 vs oracle (100 groups): {st}")
    assert st["rms"] <= FP32_TOL


@pytest.mark.parametrize("eps", [2e-4, 1e-2])
def test_far_distance_paths(eps):
    """Far pairs take r = s - eps^2/(2 s) when (2 eps / r_cut)^2 <= 5e-4 and
    the exact square root otherwise (eps = 1e-2 with r_cut = 0.1 gives 0.04):
    force and adjoint agree with the oracle on both paths."""
    ps = synth.small_clustered(8000, 131, r_cut=0.1, eps=eps, theta=0.5, per_halo=800)
    say(f"[gpu] far-distance path eps={eps} n={ps.n}")
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    _, _, a32 = gpu_forward(ps)
    ref = ot.force()
    st = rel_stats(a32, ref)
    say(f"    force: {st}")
    assert st["rms"] <= FP32_TOL
    check_force(ot, a32, ref, False, "fp32 force")
    w = synth.loss_weights(ps.n, 132)
    rx, rm = ot.adjoint(w)
    p = srf.Params.of(ps.params)
    x, m = dev_inputs(ps)
    tree = srf.tree_build(x, m, p)
    lists = srf.make_lists(tree, p)
    gx, gm = srf.short_range_adjoint(tree, lists, p, torch.tensor(w, dtype=torch.float64, device="cuda"))
    gx, gm = gx.cpu().numpy(), gm.cpu().numpy()
    sx = rel_stats(gx, rx)
    say(f"    adjoint: dL/dx {sx}")
    assert sx["rms"] <= FP32_TOL
    check_adjoint(ot, w, gx, gm, rx, rm, False, "fp32")


def test_compensated_force_option():
    """compensated = 1 selects Kahan FP32 partial sums over each tile: the
    result stays within the FP32 tolerance, is no less accurate than plain
    FP32 sums, and is not the plain path's result."""
    ps = case_sets()["clustered-20000"]
    say(f"[gpu] compensated FP32 partials n={ps.n}")
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    ref = ot.force()
    x, m = dev_inputs(ps)
    p0 = srf.Params.of(ps.params, srf.FP32_REL, 0)
    p1 = srf.Params.of(ps.params, srf.FP32_REL, 1)
    tree = srf.tree_build(x, m, p0)
    lists = srf.make_lists(tree, p0)
    a0 = srf.short_range_force(tree, lists, p0).cpu().numpy()
    a1 = srf.short_range_force(tree, lists, p1).cpu().numpy()
    s0, s1 = rel_stats(a0, ref), rel_stats(a1, ref)
    say(f"    plain: {s0}\n    compensated: {s1}")
    assert s1["rms"] <= FP32_TOL and s0["rms"] <= FP32_TOL
    E = ot.force_bound(U32)
    check_force(ot, a0, ref, False, "plain", E)
    check_force(ot, a1, ref, False, "compensated", E)
    assert s1["rms"] <= 1.05 * s0["rms"]
    assert not np.array_equal(a0, a1)
    with pytest.raises(srf.SrfError) as e:
        srf.short_range_force(tree, lists, srf.Params.of(ps.params, srf.FP32_REL, 2))
    assert e.value.status == -1


@pytest.mark.parametrize("name", ["cfg1-uniform-4096", "clustered-20000", "clustered-tight-12000"])
@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_centre_of_mass_mac(name, theta):
    """Centre-of-mass opening criterion.  Its decisions use the FP64 centres
    of mass, which the GPU and the oracle sum in different orders (they agree
    to about 1e-16 per particle of the cell), so a decision may flip where
    side^2 and theta^2 d^2 agree to that level.  Lists must be identical
    except in groups where every differing entry lies under a cell whose
    criterion is that close to the threshold (by the oracle's centres of
    mass); forces must match the oracle on the groups with identical lists."""
    ps = case_sets()[name]
    params = synth.Params(1.0, ps.params.r_cut, ps.params.eps, theta, 64, 16, srf.MAC_COM)
    say(f"[gpu] centre-of-mass MAC {name} theta={theta} n={ps.n}")
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, params)
    tree, lists, a32 = gpu_forward(ps, params, srf.FP32_REL)
    L, R = lists.export(), ot.lists
    t = ot.tree
    same = np.ones(ot.n_groups, bool)
    for g in range(ot.n_groups):
        pg, pr = L["pidx"][L["poff"][g]:L["poff"][g + 1]], R.pidx[R.poff[g]:R.poff[g + 1]]
        ng_, nr = L["nidx"][L["noff"][g]:L["noff"][g + 1]], R.nidx[R.noff[g]:R.noff[g + 1]]
        if np.array_equal(pg, pr) and np.array_equal(ng_, nr):
            continue
        same[g] = False
        cg = 0.5 * (ot.lo[g] + ot.hi[g])
        hg = 0.5 * (ot.hi[g] - ot.lo[g])
        nd = np.setxor1d(ng_, nr)
        border = []
        for c in nd:
            side = 2.0 ** -int(t.level[c])
            dd = np.abs(ot.X[c] - cg)
            dd = np.minimum(dd, 1 - dd)
            gap = np.maximum(dd - hg, 0)
            if abs(side * side - theta * theta * np.sum(gap * gap)) <= 1e-9 * side * side:
                border.append(int(c))
        assert border, f"group {g}: differing cells, none at the threshold"
        def under(c):
            while c >= 0:
                if c in border:
                    return True
                c = int(t.parent[c])
            return False
        assert all(under(int(c)) for c in nd)
        for s_ in np.setxor1d(pg, pr):
            assert any(t.first[c] <= s_ < t.first[c] + t.count[c] for c in border)
    say(f"    groups with identical lists: {same.sum()} of {ot.n_groups}")
    assert (~same).sum() <= max(1, ot.n_groups // 1000)
    ref = ot.force()
    keep = np.zeros(ps.n, bool)
    for g in np.flatnonzero(same):
        keep[ot.perm[ot.gfirst[g]:ot.gfirst[g] + ot.gcount[g]]] = True
    st = rel_stats(a32[keep], ref[keep])
    say(f"    fp32 vs oracle: {st}")
    assert st["rms"] <= FP32_TOL
    # the geometric-centre lists differ from these at theta > 0
    p0 = srf.Params.of(params)
    lists0 = srf.make_lists(tree, dataclasses.replace(p0, mac=srf.MAC_CENTRE))
    if theta > 0 and R.nidx.size:
        assert lists0.info()["n_node_entries"] != lists.info()["n_node_entries"] or \
            not np.array_equal(lists0.export()["nidx"], L["nidx"])
    # lists built with one criterion are refused with the other
    with pytest.raises(srf.SrfError) as e:
        srf.short_range_force(tree, lists0, p0)
    assert e.value.status == -5


EXPAND_BATCH = 128   # items the expansion takes per batch


def max_expand_chunk(ot):
    """Largest number of entries in one batch of EXPAND_BATCH consecutive
    items (leaves and accepted cells, in preorder) of any group's list, from
    the oracle's structure."""
    t, L = ot.tree, ot.lists
    leaf_of = np.full(ot.n, -1)
    for i in np.nonzero(t.leaf)[0]:
        leaf_of[t.first[i]:t.first[i] + t.count[i]] = i
    best = 0
    for g in range(ot.n_groups):
        leaves = np.unique(leaf_of[L.pidx[L.poff[g]:L.poff[g + 1]]])
        cells = L.nidx[L.noff[g]:L.noff[g + 1]]
        ids = np.concatenate([leaves, cells])
        size = np.concatenate([t.count[leaves], np.ones(cells.size, np.int64)])[np.argsort(ids, kind="stable")]
        for c0 in range(0, size.size, EXPAND_BATCH):
            best = max(best, int(size[c0:c0 + EXPAND_BATCH].sum()))
    return best


def test_lists_with_leaves_of_64():
    """Leaves of up to 64 particles: some batches of items expand to more
    entries than the expansion's LDS buffer holds (1024) and take its direct
    path; the lists must equal the oracle's bit for bit."""
    ps = synth.small_clustered(20000, 101, r_cut=0.1, eps=2e-4, theta=0.5, per_halo=1000)
    params = synth.Params(1.0, 0.1, 2e-4, 0.5, 64, 64)
    say(f"[gpu] n_leaf=64 n={ps.n}")
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, params)
    assert max_expand_chunk(ot) > 1024
    tree, lists, a32 = gpu_forward(ps, params)
    check_structure(tree, lists, ot)
    st = rel_stats(a32, ot.force())
    say(f"    force {st}")
    assert st["rms"] <= FP32_TOL


@pytest.mark.parametrize("n_group,n_leaf", [(1, 1), (8, 4), (16, 16), (33, 7)])
def test_other_group_sizes(n_group, n_leaf):
    """Groups and leaves other than the workloads' 64 / 16: bit-exact
    structure and lists, FP32 force and adjoint against the oracle."""
    ps = synth.small_clustered(6000, 151, r_cut=0.1, eps=2e-4, theta=0.5, per_halo=600)
    params = synth.Params(1.0, 0.1, 2e-4, 0.5, n_group, n_leaf)
    say(f"[gpu] n_group={n_group} n_leaf={n_leaf} n={ps.n}")
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, params)
    tree, lists, a32 = gpu_forward(ps, params)
    check_structure(tree, lists, ot)
    assert np.max(ot.gcount) <= n_group
    ref = ot.force()
    st = rel_stats(a32, ref)
    say(f"    force {st}")
    assert st["rms"] <= FP32_TOL
    check_force(ot, a32, ref, False, "fp32 force")
    w = synth.loss_weights(ps.n, 152)
    rx, rm = ot.adjoint(w)
    p = srf.Params.of(params)
    gx, gm = srf.short_range_adjoint(tree, lists, p, torch.tensor(w, dtype=torch.float64, device="cuda"))
    gx, gm = gx.cpu().numpy(), gm.cpu().numpy()
    sx = rel_stats(gx, rx)
    say(f"    adjoint: dL/dx {sx}")
    assert sx["rms"] <= FP32_TOL
    check_adjoint(ot, w, gx, gm, rx, rm, False, "fp32")


def test_work_ordered_on_the_callers_stream():
    """Every call orders its device work on torch's current stream: the path
    run on two side streams in turn (the library's memory cache then hands
    blocks from one stream to the other) gives the default stream's result
    bit for bit (the force has no atomics; the adjoint's atomics are compared
    to rounding)."""
    ps = case_sets()["clustered-20000"]
    p = srf.Params.of(ps.params)
    x, m = dev_inputs(ps)
    w = torch.tensor(synth.loss_weights(ps.n, 161), dtype=torch.float64, device="cuda")

    def run():
        tree = srf.tree_build(x, m, p)
        lists = srf.make_lists(tree, p)
        a = srf.short_range_force(tree, lists, p)
        gx, gm = srf.short_range_adjoint(tree, lists, p, w)
        return a, gx, gm

    a0, gx0, gm0 = run()
    torch.cuda.synchronize()
    for _ in range(2):
        for st in (torch.cuda.Stream(), torch.cuda.Stream()):
            st.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(st):
                a, gx, gm = run()
            st.synchronize()
            assert torch.equal(a, a0)
            assert torch.allclose(gx, gx0, rtol=1e-12, atol=1e-12 * gx0.abs().max().item())
            assert torch.allclose(gm, gm0, rtol=1e-12, atol=1e-12 * gm0.abs().max().item())


def test_inputs_reusable_once_the_stream_passes_the_build():
    """The tree build gathers the sorted particles on the library's second
    stream; the caller's stream waits for that gather before the call
    returns, so inputs overwritten on that stream right after the call leave
    the tree as built from the originals (2^22 particles: a gather long
    enough that a missing wait would let the overwrite reach it)."""
    rng = np.random.default_rng(1717)
    n = 1 << 22
    p = srf.Params(r_cut=0.02, eps=1e-4)
    x = torch.tensor(rng.random((n, 3)), dtype=torch.float64, device="cuda")
    m = torch.tensor(rng.random(n) + 0.5, dtype=torch.float64, device="cuda")
    x0, m0 = x.clone(), m.clone()
    for st in (torch.cuda.current_stream(), torch.cuda.Stream()):
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            x.copy_(x0)
            m.copy_(m0)
            tree = srf.tree_build(x, m, p)
            x.fill_(0.5)
            m.fill_(2.0)
        st.synchronize()
        ref = srf.tree_build(x0, m0, p)
        torch.cuda.synchronize()
        xs, ms = tree.sorted_particles()
        xr, mr = ref.sorted_particles()
        assert np.array_equal(xs, xr) and np.array_equal(ms, mr)
        assert np.array_equal(tree.export()["gfirst"], ref.export()["gfirst"])
        del tree, ref


def test_domain_errors_reported():
    p = srf.Params(r_cut=0.1, eps=1e-3)
    x = torch.rand((100, 3), dtype=torch.float64, device="cuda")
    m = torch.full((100,), 0.01, dtype=torch.float64, device="cuda")
    bad = x.clone()
    bad[17, 1] = float("nan")
    with pytest.raises(srf.SrfError) as e:
        srf.tree_build(bad, m, p)
    assert e.value.status == -2
    bad = x.clone()
    bad[3, 0] = float("inf")
    with pytest.raises(srf.SrfError):
        srf.tree_build(bad, m, p)
    mm = m.clone()
    mm[5] = 0.0
    with pytest.raises(srf.SrfError) as e:
        srf.tree_build(x, mm, p)
    assert e.value.status == -2
    # lists with other params, and force with params that do not match
    tree = srf.tree_build(x, m, p)
    with pytest.raises(srf.SrfError) as e:
        srf.make_lists(tree, srf.Params(r_cut=0.1, eps=1e-3, n_group=32))
    assert e.value.status == -5
    lists = srf.make_lists(tree, p)
    with pytest.raises(srf.SrfError) as e:
        srf.short_range_force(tree, lists, srf.Params(r_cut=0.05, eps=1e-3))
    assert e.value.status == -5
    # eps and G are free
    a = srf.short_range_force(tree, lists, srf.Params(G=2.0, r_cut=0.1, eps=2e-3))
    torch.cuda.synchronize()
    assert torch.isfinite(a).all()


def test_deterministic_forward():
    ps = synth.small_clustered(30000, 111, r_cut=0.04, eps=2e-4, theta=0.5, per_halo=1500)
    t1, l1, a1 = gpu_forward(ps)
    t2, l2, a2 = gpu_forward(ps)
    for k in ("poff", "pidx", "noff", "nidx"):
        assert np.array_equal(l1.export()[k], l2.export()[k])
    assert np.array_equal(a1, a2)


def test_strided_soa_and_aos_inputs_agree():
    ps = synth.small_uniform(5000, 7, r_cut=0.08, eps=5e-4, theta=0.5)
    p = srf.Params.of(ps.params)
    x, m = dev_inputs(ps)
    t1 = srf.tree_build(x, m, p)
    a1 = srf.short_range_force(t1, srf.make_lists(t1, p), p)
    # the same positions inside a wider [N,4] buffer (row stride 4)
    wide = torch.zeros((ps.n, 4), dtype=torch.float64, device="cuda")
    wide[:, :3] = x
    m2 = torch.zeros((ps.n, 2), dtype=torch.float64, device="cuda")
    m2[:, 0] = m
    t = srf.tree_build(wide[:, :3], m2[:, 0], p)
    a2 = srf.short_range_force(t, srf.make_lists(t, p), p)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2)


# --------------------------------------------------------------- adjoint
def adjoint_case(n=16384, seed=121):
    ps = synth.small_clustered(n, seed, r_cut=0.1, eps=2e-4, theta=0.5, per_halo=1024)
    w = synth.loss_weights(ps.n, seed + 1)
    return ps, w


@pytest.mark.parametrize("precision,tol", [(srf.FP32_REL, FP32_TOL), (srf.FP64, 1e-12)])
def test_adjoint_parity(precision, tol):
    ps, w = adjoint_case()
    say(f"[gpu] adjoint precision={precision} n={ps.n}")
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    rx, rm = ot.adjoint(w)
    p = srf.Params.of(ps.params, precision)
    x, m = dev_inputs(ps)
    tree = srf.tree_build(x, m, p)
    lists = srf.make_lists(tree, p)
    wd = torch.tensor(w, dtype=torch.float64, device="cuda")
    gx, gm = srf.short_range_adjoint(tree, lists, p, wd)
    torch.cuda.synchronize()
    gx, gm = gx.cpu().numpy(), gm.cpu().numpy()
    sx = rel_stats(gx, rx)
    em = np.abs(gm - rm) / np.maximum(np.abs(rm), 1e-300)
    say(f"    dL/dx vs oracle: {sx}")
    say(f"    dL/dm vs oracle: rms={np.sqrt(np.mean(em ** 2)):.3e} p99={np.percentile(em, 99):.3e} "
        f"normwise={np.linalg.norm(gm - rm) / np.linalg.norm(rm):.3e}")
    assert sx["rms"] <= tol
    # dL/dm_k = sum_i w_i . F(x_k - x_i) + cell terms: random-signed terms
    # whose absolute sum exceeds the result by 1e4-1e5, so its relative
    # error is only reported; every particle is held to its element-wise
    # bound, which carries that sum
    check_adjoint(ot, w, gx, gm, rx, rm, precision == srf.FP64, "fp64" if precision == srf.FP64 else "fp32")
    # translation invariance of the fixed-structure forward
    assert np.linalg.norm(gx.sum(0)) <= 1e-6 * np.abs(gx).sum()


def test_autograd_function_matches_adjoint():
    ps, w = adjoint_case(8192, 131)
    p = srf.Params.of(ps.params)
    x, m = dev_inputs(ps)
    x.requires_grad_(True)
    m.requires_grad_(True)
    wd = torch.tensor(w, dtype=torch.float64, device="cuda")
    a = srf.ShortRange.apply(x, m, p)
    loss = (a * wd).sum()
    loss.backward()
    tree = srf.tree_build(x.detach(), m.detach(), p)
    lists = srf.make_lists(tree, p)
    gx, gm = srf.short_range_adjoint(tree, lists, p, wd)
    a_ref = srf.short_range_force(tree, lists, p)
    torch.cuda.synchronize()
    assert torch.equal(a.detach(), a_ref)
    assert torch.allclose(x.grad, gx, rtol=1e-9, atol=1e-9 * gx.abs().max().item())
    assert torch.allclose(m.grad, gm, rtol=1e-9, atol=1e-9 * gm.abs().max().item())


# ------------------------------------------------------------ full sizes
def sampled_force_check(ps, a_gpu, ot, n_groups=300, seed=0, fp64=False):
    """Same-list force on a random sample of groups: the per-particle bound
    is asserted, the relative-error statistics returned."""
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(ot.n_groups, min(n_groups, ot.n_groups), replace=False))
    ref_sorted = ot.force_sorted(sel=sel)
    E_sorted = ot.force_bound_sorted(U64 if fp64 else U32, sel=sel)
    idx = np.concatenate([np.arange(ot.gfirst[g], ot.gfirst[g] + ot.gcount[g]) for g in sel])
    ref = ref_sorted[idx]
    got = a_gpu[ot.perm[idx]]
    check(got, ref, E_sorted[idx], constant("force", fp64, max_list(ot)), f"{'fp64' if fp64 else 'fp32'} force, "
          f"{sel.size} groups")
    return rel_stats(got, ref)


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_full_size_config(k):
    say(f"[gpu] full-size workload {k}: generating")
    ps = synth.make_config(k)
    say(f"    n={ps.n}; oracle tree")
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    say("    gpu forward")
    tree, lists, a32 = gpu_forward(ps)
    say("    structure")
    check_structure(tree, lists, ot)
    st = sampled_force_check(ps, a32, ot)
    say(f"    fp32 vs oracle (300 groups): {st}")
    assert st["rms"] <= FP32_TOL


def test_lists_refused_after_their_tree_is_freed():
    """Lists refer to their tree by a generation number: once the tree is
    freed, a new tree (which may reuse the same host address) does not
    accept them, in either free order."""
    ps = synth.small_uniform(3000, 171, r_cut=0.08, eps=5e-4, theta=0.5)
    p = srf.Params.of(ps.params)
    x, m = dev_inputs(ps)
    L = srf.lib()
    cp = p.c()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    cols = [C.c_void_p(x.data_ptr() + 8 * k) for k in range(3)]

    def build():
        h = C.c_void_p()
        assert L.srf_tree_build(ps.n, *cols, 3, C.c_void_p(m.data_ptr()), 1, C.byref(cp), st, C.byref(h)) == 0
        return h

    def lists_of(t):
        h = C.c_void_p()
        assert L.srf_make_lists(t, C.byref(cp), st, C.byref(h)) == 0
        return h

    out = torch.empty((ps.n, 3), dtype=torch.float64, device="cuda")
    ocols = [C.c_void_p(out.data_ptr() + 8 * k) for k in range(3)]
    t1 = build()
    l1 = lists_of(t1)
    assert L.srf_short_range_force(t1, l1, C.byref(cp), *ocols, 3, st) == 0
    addr = t1.value
    L.srf_tree_free(t1)
    reused = False
    for _ in range(8):   # the allocator usually hands the same address back
        t2 = build()
        reused |= t2.value == addr
        assert L.srf_short_range_force(t2, l1, C.byref(cp), *ocols, 3, st) == -5
        assert "another tree" in L.srf_last_error().decode()
        if reused:
            break
        L.srf_tree_free(t2)
    say(f"    new tree at the freed address: {reused}")
    # lists freed before their tree: the tree stays usable
    l2 = lists_of(t2)
    L.srf_lists_free(l2)
    L.srf_lists_free(l1)
    l3 = lists_of(t2)
    assert L.srf_short_range_force(t2, l3, C.byref(cp), *ocols, 3, st) == 0
    torch.cuda.synchronize()
    L.srf_lists_free(l3)
    L.srf_tree_free(t2)


def test_backward_with_an_expanded_gradient():
    """A loss whose gradient reaches the force as an expanded tensor (rows
    sharing memory, stride 0) gives the adjoint of the materialised weights."""
    ps, _ = adjoint_case(4096, 181)
    p = srf.Params.of(ps.params)
    x, m = dev_inputs(ps)
    v = torch.tensor([0.3, -1.2, 0.7], dtype=torch.float64, device="cuda")
    xx = x.clone().requires_grad_(True)
    a = srf.ShortRange.apply(xx, m, p)
    (a.sum(0) @ v).backward()          # dL/da = v broadcast over the rows
    tree = srf.tree_build(x, m, p)
    lists = srf.make_lists(tree, p)
    gx, _ = srf.short_range_adjoint(tree, lists, p, v.expand(ps.n, 3).contiguous())
    torch.cuda.synchronize()
    assert torch.allclose(xx.grad, gx, rtol=1e-12, atol=1e-12 * gx.abs().max().item())
