"""Seeded synthetic particle sets for the short-range TreePM step.

This module only draws inputs: it holds none of the method's arithmetic, and
both the CPU oracle and the GPU library are fed from it.  The paper's own
workload (a 10240^3 cosmological run with a neutralino-cutoff spectrum,
Sec. "Calculation Setup") is not available, so the sets below stand in for it
with the same ingredients: a periodic unit box, equal masses m = 1/N, a cutoff
radius of a few mean spacings (the paper uses r_cut = 3/N_PM^(1/3) with
N_PM = N/8, i.e. about 7.5 spacings) and a clustered mix whose density peaks
are 10^2..10^3 times the mean, as the paper describes for evolved states
(Sec. "Our Parallel TreePM Code", load-balance discussion).

Every set is returned as float64 SoA columns x, y, z, m.  Positions may be
exactly 1.0 after ``mod 1`` of a tiny negative number; the library wraps them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Params", "ParticleSet", "CONFIGS", "config_params", "make_config",
    "uniform", "plummer_halos", "zeldovich", "clustered", "loss_weights",
]


@dataclass(frozen=True)
class Params:
    """Physical and tree parameters of one short-range evaluation."""
    G: float = 1.0
    r_cut: float = 0.1
    eps: float = 1e-3
    theta: float = 0.5
    n_group: int = 64
    n_leaf: int = 16
    mac: int = 0        # 0: opening distance to the cell's geometric centre, 1: to its centre of mass


@dataclass
class ParticleSet:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    m: np.ndarray
    params: Params
    name: str = ""
    recipe: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def positions(self) -> np.ndarray:
        """[N,3] float64 array (a copy)."""
        return np.stack([self.x, self.y, self.z], axis=1)


# The five workloads.  Sizes, cutoffs, softenings and opening angles are the
# ones the throughput and accuracy experiments run on; `seed` feeds
# numpy.random.default_rng.
CONFIGS = {
    1: dict(name="uniform-4096", n=4096, r_cut=0.1, eps=1e-3, theta=0.5, seed=1001),
    2: dict(name="clustered-2^21", n=1 << 21, r_cut=3.0 / 64, eps=2e-4, theta=0.5, seed=1002,
            halos=512, per_halo=2048, a_range=(1e-3, 1e-2)),
    3: dict(name="zeldovich-256^3", n=1 << 24, r_cut=3.0 / 128, eps=5e-5, theta=0.5, seed=1003,
            grid=256, rms_cells=0.3),
    4: dict(name="clustered-2^20", n=1 << 20, r_cut=3.0 / 64, eps=2e-4, theta=0.5, seed=1004,
            halos=256, per_halo=2048, a_range=(1e-3, 1e-2)),
    5: dict(name="clustered-1.3e7", n=13_000_000, r_cut=3.0 / 256, eps=2e-5, theta=0.5, seed=1005,
            halos=4096, halo_total=9_100_000, a_range=(5e-4, 5e-3)),
}


def config_params(k: int, theta: float | None = None) -> Params:
    c = CONFIGS[k]
    return Params(G=1.0, r_cut=c["r_cut"], eps=c["eps"],
                  theta=c["theta"] if theta is None else theta, n_group=64, n_leaf=16)


def uniform(n: int, rng: np.random.Generator) -> np.ndarray:
    """n i.i.d. uniform points in [0,1)^3, shape [n,3]."""
    return rng.random((n, 3))


def _plummer_radii(count: int, a: float, rng: np.random.Generator, r_max: float = 0.5) -> np.ndarray:
    """Radii from a Plummer sphere of scale radius a, truncated at r_max by redrawing."""
    out = np.empty(count)
    todo = np.arange(count)
    while todo.size:
        u = 1.0 - rng.random(todo.size)            # (0, 1]
        with np.errstate(divide="ignore"):
            r = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        ok = np.isfinite(r) & (r <= r_max)
        out[todo[ok]] = r[ok]
        todo = todo[~ok]
    return out


def plummer_halos(counts, a_range, rng: np.random.Generator) -> np.ndarray:
    """Plummer spheres with uniform centres and log-uniform scale radii.

    counts[h] particles in halo h; returns [sum(counts), 3] positions mod 1.
    """
    counts = np.asarray(counts, dtype=np.int64)
    nh = counts.size
    centres = rng.random((nh, 3))
    a = np.exp(rng.uniform(np.log(a_range[0]), np.log(a_range[1]), nh))
    pos = np.empty((int(counts.sum()), 3))
    o = 0
    for h in range(nh):
        c = int(counts[h])
        r = _plummer_radii(c, a[h], rng)
        d = rng.standard_normal((c, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        pos[o:o + c] = np.mod(centres[h] + r[:, None] * d, 1.0)
        o += c
    return pos


def clustered(n_uniform: int, counts, a_range, rng: np.random.Generator) -> np.ndarray:
    """A uniform background followed by Plummer halos (order: uniform first)."""
    return np.concatenate([uniform(n_uniform, rng), plummer_halos(counts, a_range, rng)], axis=0)


def zeldovich(grid: int, rms_cells: float, rng: np.random.Generator) -> np.ndarray:
    """Lattice displaced by a Gaussian field with density spectrum P(k) ~ k^-2.

    delta_k = FFT(white noise) / |k|, psi_k = i k delta_k / k^2 (Nyquist planes
    zeroed), rescaled so that the rms of |psi| is rms_cells lattice spacings.
    """
    noise = rng.standard_normal((grid, grid, grid))
    nk = np.fft.rfftn(noise)
    del noise
    kx = np.fft.fftfreq(grid) * grid
    kz = np.fft.rfftfreq(grid) * grid
    KX, KY, KZ = np.meshgrid(kx, kx, kz, indexing="ij")
    k2 = KX * KX + KY * KY + KZ * KZ
    k2[0, 0, 0] = 1.0
    delta = nk / np.sqrt(k2)
    delta[0, 0, 0] = 0.0
    del nk
    nyq = (np.abs(KX) == grid // 2) | (np.abs(KY) == grid // 2) | (np.abs(KZ) == grid // 2)
    psi = []
    for K in (KX, KY, KZ):
        comp = 1j * K * delta / k2
        comp[nyq] = 0.0
        psi.append(np.fft.irfftn(comp, s=(grid, grid, grid), axes=(0, 1, 2)))
        del comp
    del KX, KY, KZ, k2, delta
    psi = np.stack([p.reshape(-1) for p in psi], axis=1)
    rms = np.sqrt(np.mean(np.sum(psi * psi, axis=1)))
    psi *= (rms_cells / grid) / rms
    idx = (np.arange(grid) + 0.5) / grid
    Q = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), axis=-1).reshape(-1, 3)
    return np.mod(Q + psi, 1.0)


def _halo_counts_cfg5(total: int, halos: int) -> np.ndarray:
    base, extra = divmod(total, halos)
    counts = np.full(halos, base, dtype=np.int64)
    counts[:extra] += 1
    return counts


def make_config(k: int, theta: float | None = None) -> ParticleSet:
    """The full-size particle set of workload k (1..5), deterministic in its seed."""
    c = CONFIGS[k]
    rng = np.random.default_rng(c["seed"])
    n = c["n"]
    if k == 1:
        pos = uniform(n, rng)
        recipe = dict(kind="uniform")
    elif k in (2, 4):
        counts = np.full(c["halos"], c["per_halo"], dtype=np.int64)
        nu = n - int(counts.sum())
        pos = clustered(nu, counts, c["a_range"], rng)
        recipe = dict(kind="clustered", n_uniform=nu, halos=c["halos"], per_halo=c["per_halo"],
                      a_range=c["a_range"])
    elif k == 3:
        pos = zeldovich(c["grid"], c["rms_cells"], rng)
        recipe = dict(kind="zeldovich", grid=c["grid"], rms_cells=c["rms_cells"])
    elif k == 5:
        counts = _halo_counts_cfg5(c["halo_total"], c["halos"])
        nu = n - c["halo_total"]
        pos = clustered(nu, counts, c["a_range"], rng)
        recipe = dict(kind="clustered", n_uniform=nu, halos=c["halos"], halo_total=c["halo_total"],
                      a_range=c["a_range"])
    else:
        raise ValueError(f"unknown workload {k}")
    assert pos.shape == (n, 3)
    m = np.full(n, 1.0 / n)
    return ParticleSet(np.ascontiguousarray(pos[:, 0]), np.ascontiguousarray(pos[:, 1]),
                       np.ascontiguousarray(pos[:, 2]), m, config_params(k, theta), c["name"], recipe)


def small_clustered(n: int, seed: int, r_cut: float, eps: float, theta: float,
                    halo_frac: float = 0.5, per_halo: int = 512,
                    a_range=(1e-3, 1e-2)) -> ParticleSet:
    """A scaled-down clustered set (uniform background + Plummer halos) for tests."""
    rng = np.random.default_rng(seed)
    nh = max(1, int(round(n * halo_frac / per_halo)))
    counts = np.full(nh, per_halo, dtype=np.int64)
    nu = n - int(counts.sum())
    if nu < 0:
        raise ValueError("too few particles for the halos")
    pos = clustered(nu, counts, a_range, rng)
    m = np.full(n, 1.0 / n)
    p = Params(1.0, r_cut, eps, theta, 64, 16)
    return ParticleSet(np.ascontiguousarray(pos[:, 0]), np.ascontiguousarray(pos[:, 1]),
                       np.ascontiguousarray(pos[:, 2]), m, p, f"clustered-{n}", dict(kind="clustered"))


def small_uniform(n: int, seed: int, r_cut: float, eps: float, theta: float) -> ParticleSet:
    rng = np.random.default_rng(seed)
    pos = uniform(n, rng)
    m = np.full(n, 1.0 / n)
    p = Params(1.0, r_cut, eps, theta, 64, 16)
    return ParticleSet(np.ascontiguousarray(pos[:, 0]), np.ascontiguousarray(pos[:, 1]),
                       np.ascontiguousarray(pos[:, 2]), m, p, f"uniform-{n}", dict(kind="uniform"))


def loss_weights(n: int, seed: int) -> np.ndarray:
    """Loss weights w ~ N(0,1) drawn in float32, shape [n,3], returned as float64."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, 3), dtype=np.float32).astype(np.float64)
