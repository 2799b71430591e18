"""Pins of the oracle's brute-force short-range sum (the plain definition:
Sec. 2 force sum under periodic boundaries, minimum image, cutoff r_cut)."""
import numpy as np
import pytest

import oracle
import synth


def _bf(ps, method="cells"):
    p = ps.params
    return oracle.brute_force(ps.x, ps.y, ps.z, ps.m, p.G, p.r_cut, p.eps, method=method)


def test_cell_list_equals_all_pairs():
    ps = synth.make_config(1)
    a = _bf(ps)
    b = _bf(ps, "n2")
    _, st = oracle.relative_errors(a, b)
    assert st["max"] < 1e-13


def test_cell_list_equals_all_pairs_clustered():
    ps = synth.small_clustered(3000, 7, r_cut=0.07, eps=3e-4, theta=0.5, per_halo=500)
    a = _bf(ps)
    b = _bf(ps, "n2")
    _, st = oracle.relative_errors(a, b)
    assert st["max"] < 1e-12


def test_momentum_conservation():
    # pairwise antisymmetry of F: sum_i m_i a_i = 0 up to rounding
    ps = synth.small_clustered(4096, 11, r_cut=0.08, eps=5e-4, theta=0.5, per_halo=512)
    a = _bf(ps)
    tot = np.sum(ps.m[:, None] * a, axis=0)
    scale = np.sum(ps.m * np.linalg.norm(a, axis=1))
    assert np.linalg.norm(tot) / scale < 1e-13


def test_translation_invariance():
    ps = synth.make_config(1)
    a = _bf(ps)
    shift = np.array([0.3141, 0.7777, 0.05])
    b = oracle.brute_force(np.mod(ps.x + shift[0], 1.0), np.mod(ps.y + shift[1], 1.0),
                           np.mod(ps.z + shift[2], 1.0), ps.m, 1.0, ps.params.r_cut, ps.params.eps)
    _, st = oracle.relative_errors(b, a)
    assert st["max"] < 1e-9   # positions move by up to one ulp of 1.0


def test_pair_across_periodic_face():
    rc, eps = 0.1, 1e-3
    x = np.array([0.01, 0.99])
    y = np.array([0.5, 0.5])
    z = np.array([0.25, 0.25])
    m = np.array([2.0, 3.0])
    a = oracle.brute_force(x, y, z, m, 1.0, rc, eps, method="n2")
    # the partner of particle 0 sits at -0.01 through the face, 0.02 away
    f = oracle.pair_force(np.array([-0.02, 0.0, 0.0]), rc, eps)
    assert np.allclose(a[0], 3.0 * f, rtol=1e-14)
    assert np.allclose(a[1], -2.0 * f, rtol=1e-14)
    assert a[0][0] < 0 < a[1][0]


def test_zero_beyond_cutoff_and_out_of_box_positions():
    rc, eps = 0.05, 1e-4
    # two particles exactly r_cut apart and one far away: all forces exactly 0
    x = np.array([0.2, 0.25, 0.7])
    y = np.array([0.2, 0.2, 0.7])
    z = np.array([0.2, 0.2, 0.7])
    x[1] = x[0] + rc
    a = oracle.brute_force(x, y, z, np.ones(3), 1.0, rc, eps, method="n2")
    d = (x[1] - x[0]) - rc
    if d >= 0:
        assert np.all(a == 0.0)
    # positions outside [0,1) are the same particles as their wrapped images
    x2 = np.array([-0.8, 1.25, 2.7])
    b = oracle.brute_force(x2, y + 3.0, z - 5.0, np.ones(3), 1.0, 0.1, eps, method="n2")
    c = oracle.brute_force(np.mod(x2, 1.0), np.mod(y + 3.0, 1.0), np.mod(z - 5.0, 1.0), np.ones(3), 1.0, 0.1, eps,
                           method="n2")
    assert np.allclose(b, c, rtol=1e-12, atol=0)


def test_linear_in_mass_and_G():
    ps = synth.make_config(1)
    p = ps.params
    a = oracle.brute_force(ps.x, ps.y, ps.z, ps.m, 1.0, p.r_cut, p.eps)
    b = oracle.brute_force(ps.x, ps.y, ps.z, 3.0 * ps.m, 2.0, p.r_cut, p.eps)
    _, st = oracle.relative_errors(b, 6.0 * a)
    assert st["max"] < 1e-13


def test_pair_count_matches_direct_count():
    ps = synth.make_config(1)
    pos = ps.positions()
    d = pos[:, None, :] - pos[None, :, :]
    d -= np.rint(d)
    r2 = np.sum(d * d, axis=2)
    direct = int(np.sum(r2 < ps.params.r_cut ** 2)) - ps.n
    assert oracle.pair_count(ps.x, ps.y, ps.z, ps.params.r_cut) == direct


def test_selected_targets_match_full_sum():
    ps = synth.small_clustered(5000, 77, r_cut=0.07, eps=3e-4, theta=0.5, per_halo=500)
    p = ps.params
    full = oracle.brute_force(ps.x, ps.y, ps.z, ps.m, p.G, p.r_cut, p.eps)
    sel = np.random.default_rng(2).choice(ps.n, 300, replace=False)
    part = oracle.brute_force_sel(ps.x, ps.y, ps.z, ps.m, p.G, p.r_cut, p.eps, sel)
    assert np.array_equal(part, full[sel])
    # pairs within r_cut summed for the sample: the direct count over its rows
    part2, npairs = oracle.brute_force_sel(ps.x, ps.y, ps.z, ps.m, p.G, p.r_cut, p.eps, sel, count_pairs=True)
    assert np.array_equal(part2, part)
    pos = ps.positions()
    d = pos[sel][:, None, :] - pos[None, :, :]
    d -= np.rint(d)
    r2 = np.sum(d * d, axis=2)
    assert npairs == int(np.sum((r2 < p.r_cut ** 2) & (r2 > 0.0)))
