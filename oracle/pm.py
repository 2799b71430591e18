"""FP64 CPU oracle of the long-range (PM) half of the TreePM force, and the
Ewald sum that pins the total -- TEST INFRASTRUCTURE (same import rules as
the rest of ``oracle``).

The force split (Sec. 2): each particle's density is split into an S2
cloud of radius r_cut/2 (the PM part) and the point mass minus that cloud
(the PP part, which vanishes beyond r_cut).  The PM part is computed on a
periodic mesh (the PM steps listed in Sec. 2.2, "Relay Mesh Method": TSC assignment to 27 mesh
points, FFT convolution with the long-range Green's function, four-point
finite differences, interpolation back to the particles):

  rho_m  = sum_p m_p W(x_p - x_m) / H^3,            W = TSC window, H = 1/n
  phi^(k) = -4 pi G S(k)^2 / (k^2 W^(k)^2) rho^(k),  phi^(0) = 0
  a_m    = -D4 phi                                 (fourth-order central differences)
  a_p    = sum_m W(x_p - x_m) a_m

with S(k) = 12 (2 - 2 cos u - u sin u) / u^4, u = |k| r_cut / 2, the Fourier
transform of the S2 shape, and W^(k) = prod_axes sinc(k_a H / 2)^3 the TSC
window's transform (the division deconvolves assignment and
interpolation).  Mesh points sit at x = i H.

The exact reference is the Ewald sum of the periodic Newtonian force of
point masses with the mean density removed, pinned by its independence of
the splitting parameter and by symmetry.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erfc


# ------------------------------------------------------------------- PM
def tsc_stencil(u, n):
    """TSC weights of coordinates u (in mesh units, u = x n) on the mesh
    points i0-1, i0, i0+1 with i0 = round(u): (indices [N,3] mod n, weights
    [N,3])."""
    i0 = np.floor(u + 0.5)
    d = u - i0
    w = np.stack([0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2], axis=1)
    idx = (i0.astype(np.int64)[:, None] + np.arange(-1, 2)[None, :]) % n
    return idx, w


def tsc_assign(x, y, z, m, n):
    """Mass density on the n^3 mesh (mass per unit volume)."""
    ix, wx = tsc_stencil(np.asarray(x) * n, n)
    iy, wy = tsc_stencil(np.asarray(y) * n, n)
    iz, wz = tsc_stencil(np.asarray(z) * n, n)
    rho = np.zeros((n, n, n))
    m = np.asarray(m, dtype=np.float64)
    for a in range(3):
        for b in range(3):
            for c in range(3):
                np.add.at(rho, (ix[:, a], iy[:, b], iz[:, c]), m * wx[:, a] * wy[:, b] * wz[:, c])
    return rho * n ** 3


def tsc_interp(field, x, y, z):
    """TSC interpolation of a mesh field at the particle positions."""
    n = field.shape[0]
    ix, wx = tsc_stencil(np.asarray(x) * n, n)
    iy, wy = tsc_stencil(np.asarray(y) * n, n)
    iz, wz = tsc_stencil(np.asarray(z) * n, n)
    out = np.zeros(ix.shape[0])
    for a in range(3):
        for b in range(3):
            for c in range(3):
                out += field[ix[:, a], iy[:, b], iz[:, c]] * wx[:, a] * wy[:, b] * wz[:, c]
    return out


def s2_shape(u):
    """Fourier transform of the unit-mass S2 cloud, as a function of
    u = k r_cut / 2.  Below u = 0.5 its Taylor series (truncation < 2e-12)
    replaces the closed form, whose O(1) terms cancel to O(u^4) there."""
    u = np.asarray(u, dtype=np.float64)
    out = np.empty_like(u)
    small = u < 0.5
    v = u[small] ** 2
    out[small] = 1.0 + v * (-1.0 / 15.0 + v * (1.0 / 560.0 + v * (-1.0 / 37800.0 + v / 3991680.0)))
    ul = u[~small]
    out[~small] = 12.0 * (2.0 - 2.0 * np.cos(ul) - ul * np.sin(ul)) / ul ** 4
    return out


def wavenumbers(n):
    """k along one axis for numpy's FFT ordering (box side 1)."""
    return 2.0 * np.pi * np.fft.fftfreq(n, d=1.0 / n)


def green(n, r_cut, G):
    """The long-range Green's function on the rfftn grid."""
    k1 = wavenumbers(n)
    kz = 2.0 * np.pi * np.arange(n // 2 + 1)
    KX, KY, KZ = np.meshgrid(k1, k1, kz, indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    H = 1.0 / n

    def sinc(v):
        return np.sinc(v / np.pi)   # sin(v)/v

    W = (sinc(KX * H / 2) * sinc(KY * H / 2) * sinc(KZ * H / 2)) ** 3
    S = s2_shape(np.sqrt(k2) * r_cut / 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        g = -4.0 * np.pi * G * S ** 2 / (k2 * W ** 2)
    g[0, 0, 0] = 0.0
    return g


def pm_potential(rho, r_cut, G):
    n = rho.shape[0]
    return np.fft.irfftn(np.fft.rfftn(rho) * green(n, r_cut, G), s=rho.shape, axes=(0, 1, 2))


def fd4_accel(phi):
    """a = -grad phi by fourth-order central differences on the periodic mesh."""
    n = phi.shape[0]
    out = []
    for ax in range(3):
        d1 = np.roll(phi, -1, axis=ax) - np.roll(phi, 1, axis=ax)
        d2 = np.roll(phi, -2, axis=ax) - np.roll(phi, 2, axis=ax)
        out.append(-(2.0 / 3.0 * d1 - 1.0 / 12.0 * d2) * n)
    return out


def pm_force(x, y, z, m, G, r_cut, n_mesh):
    """Long-range accelerations [N,3] of the particles."""
    x, y, z = (np.mod(np.asarray(v, dtype=np.float64), 1.0) for v in (x, y, z))
    rho = tsc_assign(x, y, z, m, n_mesh)
    phi = pm_potential(rho, r_cut, G)
    acc = fd4_accel(phi)
    return np.stack([tsc_interp(a, x, y, z) for a in acc], axis=1)


# ---------------------------------------------------------------- Ewald
def ewald_force(x, y, z, m, G, alpha=6.0, n_real=2, k_max=12):
    """Periodic Newtonian accelerations of point masses in the unit box with
    the mean density removed, by Ewald summation: real-space images with
    |n_i| <= n_real and wave vectors 2 pi (l, m, n) with |l|,|m|,|n| <= k_max.
    The defaults converge to ~1e-12 relative for alpha = 6."""
    P = np.stack([np.asarray(v, dtype=np.float64) for v in (x, y, z)], axis=1)
    m = np.asarray(m, dtype=np.float64)
    N = P.shape[0]
    acc = np.zeros((N, 3))
    rng_ = np.arange(-n_real, n_real + 1)
    images = np.array(np.meshgrid(rng_, rng_, rng_, indexing="ij")).reshape(3, -1).T.astype(np.float64)
    d0 = P[None, :, :] - P[:, None, :]          # x_j - x_i
    d0 -= np.rint(d0)
    for img in images:
        d = d0 + img
        r2 = np.sum(d * d, axis=2)
        self_ = r2 == 0.0
        r2s = np.where(self_, 1.0, r2)
        r = np.sqrt(r2s)
        f = (erfc(alpha * r) + 2.0 * alpha * r / np.sqrt(np.pi) * np.exp(-alpha * alpha * r2s)) / (r2s * r)
        f = np.where(self_, 0.0, f)
        acc += np.einsum("ij,ijk->ik", f * m[None, :], d)
    kr = np.arange(-k_max, k_max + 1)
    K = np.array(np.meshgrid(kr, kr, kr, indexing="ij")).reshape(3, -1).T
    K = K[np.any(K != 0, axis=1)] * 2.0 * np.pi
    k2 = np.sum(K * K, axis=1)
    coef = 4.0 * np.pi / k2 * np.exp(-k2 / (4.0 * alpha * alpha))
    phase = P @ K.T                              # [N, nk]
    c, s = np.cos(phase), np.sin(phase)
    C = m @ c                                     # sum_j m_j cos(k x_j)
    S = m @ s
    # sum_j m_j sin(k (x_j - x_i)) = S cos(k x_i) - C sin(k x_i)
    acc += ((S[None, :] * c - C[None, :] * s) * coef[None, :]) @ K
    return G * acc

