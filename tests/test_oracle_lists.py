"""Pins of the oracle's interaction lists and same-list tree force.

Lists are checked by brute force: for every group, every particle is covered
at most once (as a particle entry or through exactly one accepted cell),
and every particle within r_cut of a member is covered exactly once (Sec. 2
force sum restricted to r_cut, Fig. 2).  The tree force is checked against
the brute-force sum where the method reduces to it (theta = 0: no cell is
ever accepted) and for convergence as theta -> 0."""
import numpy as np
import pytest

import oracle
import synth


def _sets():
    return {
        "uniform": synth.make_config(1),
        "clustered": synth.small_clustered(4096, 31, r_cut=0.06, eps=3e-4, theta=0.5, per_halo=512),
        "tight": synth.small_clustered(3000, 32, r_cut=0.02, eps=1e-4, theta=0.7, per_halo=1000,
                                       a_range=(2e-4, 2e-3)),
    }


def _coverage_check(ps, theta, n_check_groups=None, mac=0):
    p = synth.Params(ps.params.G, ps.params.r_cut, ps.params.eps, theta, 64, 16, mac)
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p)
    u = np.stack([ot.ux, ot.uy, ot.uz], axis=1)
    L = ot.lists
    t = ot.tree
    groups = range(ot.n_groups) if n_check_groups is None else \
        np.random.default_rng(0).choice(ot.n_groups, min(n_check_groups, ot.n_groups), replace=False)
    for g in groups:
        cov = np.zeros(ps.n, np.int64)
        pl = L.pidx[L.poff[g]:L.poff[g + 1]]
        nl = L.nidx[L.noff[g]:L.noff[g + 1]]
        # canonical order: ascending particle indices, nodes in preorder
        assert np.all(np.diff(pl) > 0) and np.all(np.diff(nl) > 0)
        np.add.at(cov, pl, 1)
        for c in nl:
            cov[t.first[c]:t.first[c] + t.count[c]] += 1
        assert cov.max() <= 1
        mem = u[ot.gfirst[g]:ot.gfirst[g] + ot.gcount[g]]
        d = u[None, :, :] - mem[:, None, :]
        d -= np.rint(d)
        near = np.any(np.sum(d * d, axis=2) < p.r_cut ** 2, axis=0)
        assert np.all(cov[near] == 1)
        # members are always particle entries of their own group
        assert np.all(np.isin(np.arange(ot.gfirst[g], ot.gfirst[g] + ot.gcount[g]), pl))
        # accepted cells satisfy the opening criterion geometrically: the
        # cell side is below theta times the distance from any point of the
        # group box to the cell centre (its centre of mass with mac = 1)
        cg = 0.5 * (ot.lo[g] + ot.hi[g])
        hg = 0.5 * (ot.hi[g] - ot.lo[g])
        for c in nl:
            side = 2.0 ** -int(t.level[c])
            f = int(t.first[c])
            cen = (np.floor(u[f] / side) + 0.5) * side if mac == 0 else ot.X[c]
            dd = np.abs(cen - cg)
            dd = np.minimum(dd, 1 - dd)
            gap = np.maximum(dd - hg, 0)
            assert side < theta * np.sqrt(np.sum(gap * gap)) * (1 + 1e-12)
    return ot


@pytest.mark.parametrize("name", ["uniform", "clustered", "tight"])
@pytest.mark.parametrize("theta", [0.0, 0.5, 1.0])
def test_list_coverage(name, theta):
    ps = _sets()[name]
    ot = _coverage_check(ps, theta, n_check_groups=40)
    if theta == 0.0:
        assert ot.lists.nidx.size == 0


@pytest.mark.parametrize("name", ["uniform", "clustered", "tight"])
def test_theta_zero_equals_brute_force(name):
    ps = _sets()[name]
    p = synth.Params(ps.params.G, ps.params.r_cut, ps.params.eps, 0.0, 64, 16)
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p)
    a = ot.force()
    b = oracle.brute_force(ps.x, ps.y, ps.z, ps.m, p.G, p.r_cut, p.eps)
    _, st = oracle.relative_errors(a, b)
    assert st["max"] < 1e-12


def test_error_falls_as_theta_falls():
    ps = synth.small_clustered(8192, 41, r_cut=0.05, eps=2e-4, theta=0.5, per_halo=1024)
    b = oracle.brute_force(ps.x, ps.y, ps.z, ps.m, 1.0, ps.params.r_cut, ps.params.eps)
    meds = []
    for theta in (1.0, 0.7, 0.5, 0.3, 0.1):
        p = synth.Params(1.0, ps.params.r_cut, ps.params.eps, theta, 64, 16)
        ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p)
        _, st = oracle.relative_errors(ot.force(), b)
        meds.append(st["median"])
    assert all(meds[k + 1] <= meds[k] for k in range(len(meds) - 1)), meds
    assert meds[0] > 0 and meds[-1] < 1e-4


def test_group_count_and_interactions_consistent():
    ps = synth.make_config(1)
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    nj = np.diff(ot.lists.poff) + np.diff(ot.lists.noff)
    assert ot.interactions() == int(np.sum(ot.gcount * nj))
    assert ot.interactions() >= oracle.pair_count(ps.x, ps.y, ps.z, ps.params.r_cut)


@pytest.mark.parametrize("name", ["uniform", "clustered", "tight"])
@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_list_coverage_centre_of_mass_mac(name, theta):
    """Centre-of-mass opening criterion: same coverage rules, every accepted
    cell within theta of its centre of mass."""
    ps = _sets()[name]
    _coverage_check(ps, theta, n_check_groups=40, mac=1)


def test_centre_of_mass_mac_theta0_and_accuracy():
    ps = synth.small_clustered(6000, 62, r_cut=0.1, eps=2e-4, theta=0.7, per_halo=1000)
    p0 = synth.Params(1.0, 0.1, 2e-4, 0.0, 64, 16, 0)
    p1 = synth.Params(1.0, 0.1, 2e-4, 0.0, 64, 16, 1)
    a, b = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p0), oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p1)
    for k in ("poff", "pidx", "noff", "nidx"):
        assert np.array_equal(getattr(a.lists, k), getattr(b.lists, k))
    # measuring to the expansion centre: the normwise error against the
    # direct sum is no worse than with the geometric centre on this set
    ref = oracle.brute_force(ps.x, ps.y, ps.z, ps.m, 1.0, 0.1, 2e-4)
    for theta in (0.5, 0.8, 1.0):
        e = []
        for mac in (0, 1):
            ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, synth.Params(1.0, 0.1, 2e-4, theta, 64, 16, mac))
            e.append(oracle.relative_errors(ot.force(), ref)[1]["l2"])
        assert e[1] <= 1.05 * e[0], (theta, e)
