"""Pins of the oracle's Morton keys, sort, octree, moments and groups.

Keys are checked against hand-computed values and against an encoder built
a different way (interleaving binary digit strings); the order against
numpy's lexsort; the tree, moments and groups against the structural
invariants that define them (Sec. 1 octree cells; Sec. 2 particle groups of
Barnes' modified algorithm, with the grouping rule read as stated in the
oracle's header)."""
import numpy as np
import pytest

import oracle
import synth


def key_by_strings(ix, iy, iz):
    bx, by, bz = (format(v, "021b") for v in (ix, iy, iz))
    return int("".join(a + b + c for a, b, c in zip(bx, by, bz)), 2)


def test_hand_computed_keys():
    k = lambda *p: int(oracle.morton_keys(np.array([p[0]]), np.array([p[1]]), np.array([p[2]]))[0][0])
    assert k(0.0, 0.0, 0.0) == 0
    assert k(0.5, 0.0, 0.0) == 1 << 62
    assert k(0.0, 0.5, 0.0) == 1 << 61
    assert k(0.0, 0.0, 0.5) == 1 << 60
    assert k(0.5, 0.5, 0.5) == 7 << 60
    assert k(2.0 ** -21, 0.0, 0.0) == 4
    assert k(0.0, 2.0 ** -21, 0.0) == 2
    assert k(0.0, 0.0, 2.0 ** -21) == 1
    top = (1 << 63) - 1
    assert k(1 - 2.0 ** -53, 1 - 2.0 ** -53, 1 - 2.0 ** -53) == top
    # wrapping: -1e-17 rounds to 1.0 after the shift and maps to 0
    assert k(-1e-17, 0.0, 0.0) == 0
    assert k(1.0, 2.0, -3.0) == 0
    assert k(-0.5, 1.5, 0.0) == (1 << 62) | (1 << 61)


def test_keys_match_string_interleave():
    rng = np.random.default_rng(3)
    pos = rng.random((500, 3)) * 3 - 1
    keys, ux, uy, uz = oracle.morton_keys(pos[:, 0], pos[:, 1], pos[:, 2])
    for i in range(500):
        u = np.mod(pos[i], 1.0)
        u[u == 1.0] = 0.0
        assert np.allclose([ux[i], uy[i], uz[i]], u, rtol=0, atol=1e-15)
        ii = [min(int(np.floor(c * 2 ** 21)), 2 ** 21 - 1) for c in (ux[i], uy[i], uz[i])]
        assert int(keys[i]) == key_by_strings(*ii)


def test_sort_matches_lexsort_with_ties():
    rng = np.random.default_rng(4)
    keys = rng.integers(0, 50, 4000).astype(np.uint64)   # many ties
    ks, perm = oracle.sort_keys(keys)
    ref = np.lexsort((np.arange(keys.size), keys))
    assert np.array_equal(perm, ref)
    assert np.array_equal(ks, keys[ref])


def _sets():
    return [synth.make_config(1),
            synth.small_clustered(6000, 21, r_cut=0.05, eps=2e-4, theta=0.5, per_halo=1000, a_range=(1e-4, 1e-3))]


@pytest.mark.parametrize("k", [0, 1])
def test_tree_invariants(k):
    ps = _sets()[k]
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    t = ot.tree
    n = ps.n
    assert t.level[0] == 0 and t.first[0] == 0 and t.count[0] == n and t.parent[0] == -1
    # preorder == order of (first, level)
    order = np.lexsort((t.level, t.first))
    assert np.array_equal(order, np.arange(t.size))
    leaves_cover = np.zeros(n, np.int64)
    for c in range(t.size):
        lv, f, cnt = int(t.level[c]), int(t.first[c]), int(t.count[c])
        assert cnt >= 1
        shift = 3 * (21 - lv)
        pre = ot.keys[f:f + cnt] >> np.uint64(shift) if lv > 0 else np.zeros(cnt, np.uint64)
        assert np.all(pre == t.prefix[c])
        split = lv == 0 or (lv < 21 and cnt > ps.params.n_leaf)
        assert bool(t.leaf[c]) == (not split)
        kids = [int(ch) for ch in t.child[c] if ch >= 0]
        if split:
            # children tile the parent's range in octant order
            assert sum(int(t.count[ch]) for ch in kids) == cnt
            s = f
            for o in range(8):
                ch = int(t.child[c][o])
                if ch < 0:
                    continue
                assert t.first[ch] == s and t.level[ch] == lv + 1 and t.parent[ch] == c
                assert int(t.prefix[ch]) == int(t.prefix[c]) * 8 + o
                s += int(t.count[ch])
        else:
            assert not kids
            leaves_cover[f:f + cnt] += 1
    assert np.all(leaves_cover == 1)


def test_moments_against_direct_sums():
    ps = synth.small_clustered(6000, 22, r_cut=0.05, eps=2e-4, theta=0.5, per_halo=1000)
    ps.m[:] = np.random.default_rng(1).uniform(0.5, 1.5, ps.n) / ps.n
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    t = ot.tree
    u = np.stack([ot.ux, ot.uy, ot.uz], axis=1)
    cm = np.concatenate([[0.0], np.cumsum(ot.m)])
    for c in range(0, t.size, 7):
        f, cnt = int(t.first[c]), int(t.count[c])
        assert abs(ot.M[c] - (cm[f + cnt] - cm[f])) < 1e-12 * ot.M[c] + 1e-18
        ref = (ot.m[f:f + cnt, None] * u[f:f + cnt]).sum(0) / ot.m[f:f + cnt].sum()
        assert np.allclose(ot.X[c], ref, rtol=0, atol=1e-15)
        # the centre of mass lies inside the cell box
        lv = int(t.level[c])
        side = 2.0 ** -lv
        lo = np.floor(u[f] / side) * side
        assert np.all(ot.X[c] >= lo - 1e-15) and np.all(ot.X[c] <= lo + side + 1e-15)


@pytest.mark.parametrize("k", [0, 1])
def test_group_invariants(k):
    ps = _sets()[k]
    ng_max = ps.params.n_group
    ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, ps.params)
    t = ot.tree
    gf, gc = ot.gfirst, ot.gcount
    # partition of [0, N) in order
    assert gf[0] == 0 and np.all(gf[1:] == gf[:-1] + gc[:-1]) and gf[-1] + gc[-1] == ps.n
    assert np.all(gc >= 1) and np.all(gc <= ng_max)
    # each group lies inside one level-1 cell
    top = ot.keys >> np.uint64(60)
    for f, c in zip(gf, gc):
        assert np.all(top[f:f + c] == top[f])
    # each group is a run of whole candidate cells under one parent; greedy
    # merging: the next group under the same parent could not have been added
    start_of = {int(t.first[c]): [] for c in range(t.size)}
    for c in range(t.size):
        start_of[int(t.first[c])].append(c)
    candidate = np.zeros(t.size, bool)
    for c in range(1, t.size):
        par = int(t.parent[c])
        candidate[c] = t.count[c] <= ng_max and (par == 0 or t.count[par] > ng_max)
    owner = []
    for f, c in zip(gf, gc):
        cells = [cc for cc in start_of[int(f)] if candidate[cc]]
        assert len(cells) == 1
        par = int(t.parent[cells[0]])
        covered, s = 0, int(f)
        while covered < c:
            cs = [cc for cc in start_of[s] if candidate[cc] and int(t.parent[cc]) == par]
            assert len(cs) == 1
            covered += int(t.count[cs[0]])
            s += int(t.count[cs[0]])
        assert covered == c
        owner.append((par, cells[0]))
    for g in range(len(gf) - 1):
        par, _ = owner[g]
        par2, first_cell = owner[g + 1]
        if par == par2 and par != 0 and gf[g] + gc[g] == gf[g + 1]:
            assert gc[g] + t.count[first_cell] > ng_max
    # tight bounding boxes
    u = np.stack([ot.ux, ot.uy, ot.uz], axis=1)
    for g in range(0, len(gf), 5):
        seg = u[gf[g]:gf[g] + gc[g]]
        assert np.array_equal(ot.lo[g], seg.min(0)) and np.array_equal(ot.hi[g], seg.max(0))


def test_small_n_groups_and_coincident_particles():
    # N <= n_group: the root is split anyway and each non-empty octant is a group
    rng = np.random.default_rng(9)
    pos = rng.random((40, 3))
    p = synth.Params(1.0, 0.1, 1e-3, 0.5, 64, 16)
    ot = oracle.OracleTree(pos[:, 0], pos[:, 1], pos[:, 2], np.full(40, 1 / 40), p)
    assert ot.n_groups == len(np.unique(ot.keys >> np.uint64(60)))
    # 150 coincident particles: one level-21 cell cut into chunks of n_group
    pos = np.full((150, 3), 0.123456789)
    ot = oracle.OracleTree(pos[:, 0], pos[:, 1], pos[:, 2], np.full(150, 1 / 150), p)
    assert list(ot.gcount) == [64, 64, 22]
    assert ot.tree.level.max() == 21
