"""Pins of the oracle's refitted tree (the tree reused after its particles
moved: sort order, cells and groups held, boxes of the actual particles).

  - every cell's box holds an image of each of its particles and is touched
    by one on every face, a leaf's box is exactly that of its particles'
    images nearest the cell's dyadic centre (recomputed directly), no box is
    wider than the cell plus twice the largest move, and every group's box
    is that of its particles' images nearest its first particle;
  - coverage by brute force after the drift: for every group, every particle
    within r_cut of a member is covered exactly once and nothing twice, and
    accepted cells satisfy the opening criterion on their boxes;
  - theta = 0 reduces to the brute-force sum at the new positions;
  - without motion the refitted lists never hold more entries than the
    fresh ones (tight boxes lie inside the dyadic cells)."""
import numpy as np
import pytest

import oracle
import synth


def _drifted(ps, scale, seed, cross=True):
    """Positions moved by up to `scale` per axis, some particles pushed
    across the periodic faces."""
    rng = np.random.default_rng(seed)
    pos = np.stack([ps.x, ps.y, ps.z], axis=1)
    new = pos + scale * (2 * rng.random(pos.shape) - 1)
    if cross:
        k = rng.choice(ps.n, ps.n // 50, replace=False)
        new[k, 0] = np.where(pos[k, 0] < 0.5, pos[k, 0] - 0.7 * scale, pos[k, 0] + 0.7 * scale)
    new = np.mod(new, 1.0)
    new[new >= 1.0] = 0.0
    return new


def _sets():
    return {
        "clustered": synth.small_clustered(4096, 41, r_cut=0.06, eps=3e-4, theta=0.5, per_halo=512),
        "uniform": synth.small_uniform(3000, 42, r_cut=0.08, eps=5e-4, theta=0.5),
    }


def _images_box(v, ref):
    u = v - np.rint(v - ref)
    return u.min(axis=0), u.max(axis=0)


@pytest.mark.parametrize("name", ["clustered", "uniform"])
def test_refitted_boxes_hold_their_particles(name):
    """Each cell box holds an image of each of its particles and is touched
    by one on every face; a leaf's box is exactly that of its particles'
    images nearest its dyadic centre; no box is wider than the cell's side
    plus twice the largest move.  Group boxes are exactly those of the
    images nearest the group's first particle."""
    ps = _sets()[name]
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    scale = 4e-3
    new = _drifted(ps, scale, 1)
    rt = ot.refitted(new[:, 0], new[:, 1], new[:, 2])
    u = np.stack([rt.ux, rt.uy, rt.uz], axis=1)
    t = ot.tree
    for c in range(t.size):
        lv = int(t.level[c])
        side = 2.0 ** -lv
        lo, hi = rt.clo[c], rt.chi[c]
        v = u[t.first[c]:t.first[c] + t.count[c]]
        # some image of each particle lies in the box, and some particle's
        # image lies on each face
        imgs = v[None] + np.array([-1.0, 0.0, 1.0])[:, None, None]
        inside = (imgs >= lo) & (imgs <= hi)
        assert np.all(inside.any(axis=0)), c
        assert np.all((imgs == lo).any(axis=(0, 1))) and np.all((imgs == hi).any(axis=(0, 1))), c
        assert np.all(hi - lo <= side + 2 * scale * (1 + 1e-12)), c
        if t.leaf[c]:
            pf = int(t.prefix[c])
            ijk = [sum(((pf >> (3 * l + b)) & 1) << l for l in range(lv)) for b in (2, 1, 0)]
            cref = (np.array(ijk) + 0.5) * side
            dlo, dhi = _images_box(v, cref)
            assert np.array_equal(dlo, lo) and np.array_equal(dhi, hi), c
    for g in range(ot.n_groups):
        f = int(ot.gfirst[g])
        lo, hi = _images_box(u[f:f + ot.gcount[g]], u[f])
        assert np.array_equal(lo, rt.lo[g]) and np.array_equal(hi, rt.hi[g]), g
    # the sort order, cells and groups are held
    assert np.array_equal(rt.perm, ot.perm) and rt.tree is ot.tree and np.array_equal(rt.gfirst, ot.gfirst)


@pytest.mark.parametrize("name", ["clustered", "uniform"])
def test_rounded_boxes_hold_the_particles(name):
    """The boxes the list decisions use: each cell's box rounded outward to
    multiples of q = 2^-(level+10), within one q of it, holding an image of
    every particle of the cell.  A cell of level <= 6 is always bounded (no
    image lies more than half the box from the cell's centre)."""
    ps = _sets()[name]
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    new = _drifted(ps, 4e-3, 4)
    rt = ot.refitted(new[:, 0], new[:, 1], new[:, 2])
    qlo, qhi, ok = rt.refit_qboxes()
    t = ot.tree
    assert np.all(ok[t.level <= 6])
    u = np.stack([rt.ux, rt.uy, rt.uz], axis=1)
    for c in np.flatnonzero(ok):
        e = int(t.level[c]) + 10
        q = 2.0 ** -e
        for b in (qlo[c], qhi[c]):
            assert np.all(np.ldexp(b, e) == np.rint(np.ldexp(b, e)))
        assert np.all(qlo[c] <= rt.clo[c]) and np.all(qlo[c] > rt.clo[c] - q)
        assert np.all(qhi[c] >= rt.chi[c]) and np.all(qhi[c] < rt.chi[c] + q)
        v = u[t.first[c]:t.first[c] + t.count[c]]
        imgs = v[None] + np.array([-1.0, 0.0, 1.0])[:, None, None]
        assert np.all(((imgs >= qlo[c]) & (imgs <= qhi[c])).any(axis=0)), c


def test_a_particle_moved_far_leaves_its_deep_cell_unbounded_and_covered():
    """One particle of a deep leaf (level >= 7) moved by 0.3 in x: its leaf's
    box no longer fits 32767 steps of its centre, so the cell is unbounded
    (never pruned, never accepted), and every pair within r_cut is still
    covered exactly once for every group."""
    ps = synth.small_clustered(4096, 41, r_cut=0.06, eps=3e-4, theta=0.7, per_halo=2048, a_range=(5e-4, 2e-3))
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    t = ot.tree
    deep = np.flatnonzero(t.leaf.astype(bool) & (t.level >= 7) & (t.count >= 2))
    assert deep.size
    c0 = deep[0]
    k = ot.perm[t.first[c0]]
    new = np.stack([ps.x, ps.y, ps.z], axis=1)
    new[k, 0] = np.mod(new[k, 0] + 0.3, 1.0)
    rt = ot.refitted(new[:, 0], new[:, 1], new[:, 2])
    qlo, qhi, ok = rt.refit_qboxes()
    assert not ok[c0] and ok[t.level <= 6].all()
    u = np.stack([rt.ux, rt.uy, rt.uz], axis=1)
    L = rt.lists
    listed = 0
    for g in range(rt.n_groups):
        cov = np.zeros(ps.n, np.int64)
        np.add.at(cov, L.pidx[L.poff[g]:L.poff[g + 1]], 1)
        for c in L.nidx[L.noff[g]:L.noff[g + 1]]:
            assert ok[c]
            cov[t.first[c]:t.first[c] + t.count[c]] += 1
        assert cov.max() <= 1
        mem = u[rt.gfirst[g]:rt.gfirst[g] + rt.gcount[g]]
        d = u[None, :, :] - mem[:, None, :]
        d -= np.rint(d)
        near = np.any(np.sum(d * d, axis=2) < ps.params.r_cut ** 2, axis=0)
        assert np.all(cov[near] == 1), g
        listed += int(t.first[c0] in L.pidx[L.poff[g]:L.poff[g + 1]])
    assert listed > 0


@pytest.mark.parametrize("name", ["clustered", "uniform"])
@pytest.mark.parametrize("theta", [0.0, 0.5, 1.0])
def test_refitted_list_coverage(name, theta):
    ps = _sets()[name]
    p = synth.Params(ps.params.G, ps.params.r_cut, ps.params.eps, theta, 64, 16)
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p)
    new = _drifted(ps, 4e-3, 2)
    rt = ot.refitted(new[:, 0], new[:, 1], new[:, 2])
    u = np.stack([rt.ux, rt.uy, rt.uz], axis=1)
    L, t = rt.lists, rt.tree
    qlo, qhi, ok = rt.refit_qboxes()
    for g in np.random.default_rng(0).choice(rt.n_groups, min(40, rt.n_groups), replace=False):
        cov = np.zeros(ps.n, np.int64)
        pl = L.pidx[L.poff[g]:L.poff[g + 1]]
        nl = L.nidx[L.noff[g]:L.noff[g + 1]]
        assert np.all(np.diff(pl) > 0) and np.all(np.diff(nl) > 0)
        np.add.at(cov, pl, 1)
        for c in nl:
            cov[t.first[c]:t.first[c] + t.count[c]] += 1
        assert cov.max() <= 1
        mem = u[rt.gfirst[g]:rt.gfirst[g] + rt.gcount[g]]
        d = u[None, :, :] - mem[:, None, :]
        d -= np.rint(d)
        near = np.any(np.sum(d * d, axis=2) < p.r_cut ** 2, axis=0)
        assert np.all(cov[near] == 1)
        assert np.all(np.isin(np.arange(rt.gfirst[g], rt.gfirst[g] + rt.gcount[g]), pl))
        # accepted cells: the larger of the dyadic side and the longest side
        # of the (outward-rounded) box below theta times the distance from
        # the group box to the box's centre
        cg = 0.5 * (rt.lo[g] + rt.hi[g])
        hg = 0.5 * (rt.hi[g] - rt.lo[g])
        for c in nl:
            assert ok[c]
            side = max(np.max(qhi[c] - qlo[c]), 2.0 ** -int(t.level[c]))
            dd = 0.5 * (qlo[c] + qhi[c]) - cg
            dd = np.abs(dd - np.rint(dd))
            gap = np.maximum(dd - hg, 0)
            assert side < theta * np.sqrt(np.sum(gap * gap)) * (1 + 1e-12)
    if theta == 0.0:
        assert L.nidx.size == 0


@pytest.mark.parametrize("name", ["clustered", "uniform"])
def test_refitted_theta_zero_equals_brute_force(name):
    ps = _sets()[name]
    p = synth.Params(ps.params.G, ps.params.r_cut, ps.params.eps, 0.0, 64, 16)
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p)
    new = _drifted(ps, 4e-3, 3)
    rt = ot.refitted(new[:, 0], new[:, 1], new[:, 2])
    a = rt.force()
    bf = oracle.brute_force(new[:, 0], new[:, 1], new[:, 2], ps.m, 1.0, p.r_cut, p.eps, method="n2")
    assert np.linalg.norm(a - bf) <= 1e-13 * np.linalg.norm(bf)


def test_refit_without_motion_prunes_no_less():
    ps = _sets()["clustered"]
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, synth.Params(1.0, 0.06, 3e-4, 0.0, 64, 16))
    rt = ot.refitted(ps.x, ps.y, ps.z)
    assert rt.lists.pidx.size <= ot.lists.pidx.size
    assert np.array_equal(rt.force(), rt.force())
    # at theta = 0 both are the exact sum within r_cut
    assert np.allclose(rt.force(), ot.force(), rtol=1e-12, atol=1e-12 * np.abs(ot.force()).max())


@pytest.mark.parametrize("name", ["clustered", "uniform"])
def test_refitted_centres_of_mass_follow_a_translation(name):
    """Every particle moved by the same vector, some across a face of the
    unit box: each cell's centre of mass (the root aside, which is never a
    source) moves by exactly that vector, and the masses are unchanged --
    also for cells whose particles now sit on both sides of the face."""
    ps = _sets()[name]
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    shift = np.array([-0.0123, 0.0071, 0.0])
    new = np.mod(np.stack([ps.x, ps.y, ps.z], axis=1) + shift, 1.0)
    rt = ot.refitted(new[:, 0], new[:, 1], new[:, 2])
    t = ot.tree
    sel = t.level >= 1
    assert np.array_equal(rt.M, ot.M)
    moved = rt.X[sel] - ot.X[sel]
    assert np.max(np.abs(moved - shift)) <= 1e-12
    # some cell does hold particles on both sides of the face x = 0
    straddle = [c for c in np.nonzero(sel)[0] if np.ptp(new[ot.perm][t.first[c]:t.first[c] + t.count[c], 0]) > 0.5]
    assert straddle


@pytest.mark.parametrize("name", ["clustered", "uniform"])
def test_refitted_force_error_after_a_translation(name):
    """The refitted tree's same-list force at translated positions is as
    close to the brute-force sum as the fresh tree's force at the original
    positions: the monopole error does not grow where cells straddle a
    face of the unit box."""
    ps = _sets()[name]
    p = synth.Params(ps.params.G, ps.params.r_cut, ps.params.eps, 1.0, 64, 16)
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p)
    shift = np.array([-0.0123, 0.0071, 0.0])
    new = np.mod(np.stack([ps.x, ps.y, ps.z], axis=1) + shift, 1.0)
    rt = ot.refitted(new[:, 0], new[:, 1], new[:, 2])
    bf0 = oracle.brute_force(ps.x, ps.y, ps.z, ps.m, 1.0, p.r_cut, p.eps, method="n2")
    bf1 = oracle.brute_force(new[:, 0], new[:, 1], new[:, 2], ps.m, 1.0, p.r_cut, p.eps, method="n2")
    e0 = np.linalg.norm(ot.force() - bf0, axis=1)
    e1 = np.linalg.norm(rt.force() - bf1, axis=1)
    scale = np.max(np.linalg.norm(bf0, axis=1))
    assert rt.lists.nidx.size > 0
    assert np.max(e1) <= 2.0 * np.max(e0) + 1e-12 * scale
    assert np.sqrt(np.mean(e1 ** 2)) <= 1.5 * np.sqrt(np.mean(e0 ** 2)) + 1e-12 * scale


def _fd(rt, w, s, axis, h):
    u = [rt.ux.copy(), rt.uy.copy(), rt.uz.copy()]
    up = [a.copy() for a in u]
    um = [a.copy() for a in u]
    up[axis][s] += h
    um[axis][s] -= h
    return float(np.sum(w[rt.perm] * (rt.force_sorted(*up) - rt.force_sorted(*um)))) / (2 * h)


def _fd_mass(rt, w, s, rel):
    h = rt.m[s] * rel
    mp, mm = rt.m.copy(), rt.m.copy()
    mp[s] += h
    mm[s] -= h
    return float(np.sum(w[rt.perm] * (rt.force_sorted(m=mp) - rt.force_sorted(m=mm)))) / (2 * h)


def _slab():
    """A slab of particles on both sides of the face x = 0 (|x| < 0.08),
    moved by -13/1024 in x (and 7/1024 in y; multiples of the rounding step
    of every refitted box): most cells near the face then hold particles on
    both sides of it, and many are accepted with their centre of mass
    within r_cut of the group."""
    rng = np.random.default_rng(5)
    n = 4000
    x = np.concatenate([rng.random(n // 2) * 0.08, 0.92 + rng.random(n // 2) * 0.08])
    y, z = 0.3 + 0.4 * rng.random(n), 0.3 + 0.4 * rng.random(n)
    p = synth.Params(1.0, 0.06, 3e-4, 1.0, 64, 16)
    ot = oracle.OracleTree(x, y, z, np.full(n, 1.0 / n), p)
    new = np.mod(np.stack([x, y, z], axis=1) + np.array([-13.0, 7.0, 0.0]) / 1024, 1.0)
    return ot, ot.refitted(new[:, 0], new[:, 1], new[:, 2])


def test_refitted_adjoint_matches_finite_differences_across_a_face():
    """The gradient of L = sum w . a on a refitted tree, structure held
    fixed, against central differences of its own forward, for particles of
    accepted cells whose particles sit on both sides of a face of the unit
    box (the mass derivative goes through x_k - X_c at its nearest image)."""
    ot, rt = _slab()
    t = ot.tree
    acc = np.unique(rt.lists.nidx)
    straddle = [c for c in acc if np.ptp(rt.ux[t.first[c]:t.first[c] + t.count[c]]) > 0.5]
    assert len(straddle) > 20
    w = synth.loss_weights(rt.n, 9)
    gx, gm = rt.adjoint(w)
    rng = np.random.default_rng(3)
    ex, em = [], []
    for c in rng.choice(straddle, 12, replace=False):
        for s in rng.choice(np.arange(t.first[c], t.first[c] + t.count[c]), 2, replace=False):
            k = rt.perm[s]
            for a in range(3):
                ex.append(abs(_fd(rt, w, s, a, 1e-7) - gx[k, a]) / np.abs(gx[k]).max())
            em.append(abs(_fd_mass(rt, w, s, 1e-6) - gm[k]) / max(abs(gm[k]), 1e-6 * np.abs(gm).max()))
    assert max(ex) < 1e-4 and max(em) < 1e-4, (max(ex), max(em))


def test_refitted_force_across_a_face_is_translation_covariant():
    """On the slab across the face x = 0: the tree refitted to the moved
    positions and the same tree refitted to the unmoved ones have the same
    lists and the same forces to rounding (moving every particle by one
    vector moves every box and centre of mass by it, also where a cell's
    particles now sit on both sides of the face), and the force stays as
    close to the brute-force sum as the fresh tree's."""
    ot, rt = _slab()
    p = ot.params
    x0 = np.empty((ot.n, 3))
    x1 = np.empty((ot.n, 3))
    x0[ot.perm] = np.stack([ot.ux, ot.uy, ot.uz], axis=1)
    x1[rt.perm] = np.stack([rt.ux, rt.uy, rt.uz], axis=1)
    r0 = ot.refitted(x0[:, 0], x0[:, 1], x0[:, 2])
    for a, b in [(r0.lists.poff, rt.lists.poff), (r0.lists.pidx, rt.lists.pidx), (r0.lists.noff, rt.lists.noff),
                 (r0.lists.nidx, rt.lists.nidx)]:
        assert np.array_equal(a, b)
    m = np.empty(ot.n)
    m[ot.perm] = ot.m
    bf0 = oracle.brute_force(x0[:, 0], x0[:, 1], x0[:, 2], m, 1.0, p.r_cut, p.eps, method="n2")
    bf1 = oracle.brute_force(x1[:, 0], x1[:, 1], x1[:, 2], m, 1.0, p.r_cut, p.eps, method="n2")
    scale = np.max(np.linalg.norm(bf0, axis=1))
    assert np.max(np.linalg.norm(rt.force() - r0.force(), axis=1)) <= 1e-12 * scale
    # so is the quadrupole term (second moments about the centre of mass)
    dq = rt.force_quadrupole() - r0.force_quadrupole()
    assert np.max(np.linalg.norm(dq, axis=1)) <= 1e-12 * scale
    e0 = np.linalg.norm(ot.force() - bf0, axis=1)
    e1 = np.linalg.norm(rt.force() - bf1, axis=1)
    assert np.sqrt(np.mean(e1 ** 2)) <= 1.5 * np.sqrt(np.mean(e0 ** 2))
