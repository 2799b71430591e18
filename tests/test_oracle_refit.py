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
@pytest.mark.parametrize("theta", [0.0, 0.5, 1.0])
def test_refitted_list_coverage(name, theta):
    ps = _sets()[name]
    p = synth.Params(ps.params.G, ps.params.r_cut, ps.params.eps, theta, 64, 16)
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, p)
    new = _drifted(ps, 4e-3, 2)
    rt = ot.refitted(new[:, 0], new[:, 1], new[:, 2])
    u = np.stack([rt.ux, rt.uy, rt.uz], axis=1)
    L, t = rt.lists, rt.tree
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
        # accepted cells: the larger of the dyadic side and the longest box
        # side below theta times the distance from the group box to the
        # cell box's centre
        cg = 0.5 * (rt.lo[g] + rt.hi[g])
        hg = 0.5 * (rt.hi[g] - rt.lo[g])
        for c in nl:
            side = max(np.max(rt.chi[c] - rt.clo[c]), 2.0 ** -int(t.level[c]))
            dd = 0.5 * (rt.clo[c] + rt.chi[c]) - cg
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
