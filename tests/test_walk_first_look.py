"""The list walk's FP32 first look (csrc/lists.hip, classify32) decides a
prune or accept test only when its FP32 value clears the threshold by the
stated margin b(X) = 2.5e-6 sqrt(X) + 2e-6 X + 1e-12; the lists must then be
those of the FP64 expressions (Sec. 2: the group's list holds the cells that
pass the cutoff pruning and the opening criterion).  This checks the margin
argument on a numpy model of both evaluations (float32 arithmetic rounds
each operation, as the kernel compiled without contraction does), on cells
placed within a few margins of either threshold and at random.  Host logic
only: no GPU, no oracle."""
import numpy as np

F32 = np.float32


def gap64(c, cg, half):
    t = np.abs(c - cg)
    t2 = 1.0 - t
    t = np.where(t2 < t, t2, t)
    r = t - half
    return np.where(r > 0.0, r, 0.0)


def gap32(c, cg, half):
    t = np.abs((c - cg).astype(F32))
    t2 = (F32(1.0) - t).astype(F32)
    t = np.where(t2 < t, t2, t)
    r = (t - half).astype(F32)
    return np.where(r > F32(0.0), r, F32(0.0))


def classify64(level, c, mc, cg, hg, rc2, th2):
    side = np.ldexp(1.0, -level)
    hs = side * 0.5
    e = [gap64(c[a], cg[a], hs + hg[a]) for a in range(3)]
    D2 = (e[0] * e[0] + e[1] * e[1]) + e[2] * e[2]
    e = [gap64(mc[a], cg[a], hg[a]) for a in range(3)]
    d2 = (e[0] * e[0] + e[1] * e[1]) + e[2] * e[2]
    return np.where(D2 >= rc2, 0, np.where(side * side < th2 * d2, 1, 3))


def classify32(level, c, mc, cg, hg, rc2, th2):
    cg32 = [cg[a].astype(F32) for a in range(3)]
    hg32 = [hg[a].astype(F32) for a in range(3)]
    c32 = [c[a].astype(F32) for a in range(3)]     # exact: dyadic, 22 significant bits
    mc32 = [mc[a].astype(F32) for a in range(3)]
    rc2f = F32(rc2)
    bp = F32(F32(2.5e-6) * np.sqrt(rc2f)) + F32(F32(2e-6) * rc2f) + F32(1e-12)
    rc_hi, rc_lo = F32(rc2f + bp), F32(rc2f - bp)
    inv_th = F32(1.0 / np.sqrt(th2))
    side = np.ldexp(F32(1.0), -level).astype(F32)
    hs = (side * F32(0.5)).astype(F32)
    e = [gap32(c32[a], cg32[a], (hs + hg32[a]).astype(F32)) for a in range(3)]
    D2 = ((e[0] * e[0]).astype(F32) + (e[1] * e[1]).astype(F32)).astype(F32)
    D2 = (D2 + (e[2] * e[2]).astype(F32)).astype(F32)
    e = [gap32(mc32[a], cg32[a], hg32[a]) for a in range(3)]
    d2 = ((e[0] * e[0]).astype(F32) + (e[1] * e[1]).astype(F32)).astype(F32)
    d2 = (d2 + (e[2] * e[2]).astype(F32)).astype(F32)
    sx = (side * inv_th).astype(F32)
    X = (sx * sx).astype(F32)
    b = ((F32(2.5e-6) * sx).astype(F32) + (F32(2e-6) * X).astype(F32) + F32(1e-12)).astype(F32)
    prune = np.where(D2 >= rc_hi, 1, np.where(D2 < rc_lo, 0, -1))
    acc = np.where(d2 > (X + b).astype(F32), 1, np.where(d2 < (X - b).astype(F32), 0, -1))
    out = np.where(prune == 1, 0, np.where(prune == -1, -1, np.where(acc == 1, 1, np.where(acc == 0, 3, -1))))
    return out


def cells_near(rng, n, level, target, half_of, rc):
    """Cells of `level` and groups placed so that the exact gap vector, with
    `half_of(hs, hg)` subtracted per axis, has length `target` (per sample)."""
    side = np.ldexp(1.0, -level)
    hs = side * 0.5
    i = rng.integers(0, 1 << level, size=(3, n))
    c = (i + 0.5) * side
    hg = rng.uniform(0.0, 0.6 * rc, size=(3, n))
    u = rng.normal(size=(3, n))
    u /= np.linalg.norm(u, axis=0)
    e = np.abs(u) * target
    sgn = np.where(rng.random((3, n)) < 0.5, -1.0, 1.0)
    cg = np.mod(c - sgn * (half_of(hs, hg) + e), 1.0)
    return c, cg, hg


def check(level, c, mc, cg, hg, rc2, th2):
    a = classify64(level, c, mc, cg, hg, rc2, th2)
    b = classify32(level, c, mc, cg, hg, rc2, th2)
    decided = b >= 0
    assert np.array_equal(a[decided], b[decided])
    return decided.mean()


def test_first_look_agrees_near_the_cutoff():
    rng = np.random.default_rng(11)
    for rc, theta in ((0.0234375, 0.5), (0.1, 0.7), (0.005, 0.3)):
        rc2, th2 = rc * rc, theta * theta
        for level in range(2, 16):
            n = 20000
            rel = rng.uniform(-3e-5, 3e-5, n)     # within a few margins of r_cut
            c, cg, hg = cells_near(rng, n, level, rc * (1 + rel), lambda hs, hg: hs + hg, rc)
            check(level, c, c, cg, hg, rc2, th2)


def test_first_look_agrees_near_the_opening_angle():
    rng = np.random.default_rng(12)
    for rc, theta in ((0.0234375, 0.5), (0.1, 0.7), (0.05, 0.3)):
        rc2, th2 = rc * rc, theta * theta
        for level in range(5, 18):
            side = np.ldexp(1.0, -level)
            if 2.0 * side / theta > rc:
                continue
            n = 20000
            rel = rng.uniform(-3e-5, 3e-5, n)
            c, cg, hg = cells_near(rng, n, level, side / theta * (1 + rel), lambda hs, hg: hg, rc)
            check(level, c, c, cg, hg, rc2, th2)


def test_first_look_agrees_with_centres_of_mass_and_at_random():
    rng = np.random.default_rng(13)
    rc, theta = 0.0234375, 0.5
    for level in range(1, 22):
        n = 20000
        side = np.ldexp(1.0, -level)
        i = rng.integers(0, 1 << level, size=(3, n))
        c = (i + 0.5) * side
        mc = c + rng.uniform(-0.5, 0.5, size=(3, n)) * side     # a centre of mass inside the cell
        cg = np.mod(c + rng.normal(scale=2 * rc, size=(3, n)), 1.0)
        hg = rng.uniform(0.0, rc, size=(3, n))
        frac = check(level, c, mc, cg, hg, rc * rc, theta * theta)
        # at random nearly every test is decided in FP32 (the margin is
        # widest, relative to the threshold, for the tiny cells of level 20-21)
        assert frac > 0.99
