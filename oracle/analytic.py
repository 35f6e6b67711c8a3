"""Closed-form solutions used to pin the oracle -- TEST INFRASTRUCTURE ONLY.

* image_sum_rigid_box: the image-source solution of Section 4.1 (Eq. an2) with A_j = R^{n_j}
  and R = 1.  For sound-hard walls (Eq. sp5) the 8-image lattice with periods 2L is the exact
  Neumann Green's function of the box.  With a real wavenumber the lattice sum does not
  converge, so it is evaluated with a damped k (Im k > 0) and truncated where
  exp(-Im k R)/R falls below `tol`; the BEM is run with the same complex k.
* sphere_robin_interior: series solution for a unit monopole inside a sphere with the
  impedance condition of Eq. (sp3), beta = 1/zeta:  psi_sc(r) = (ik/4pi) sum_n (2n+1) A_n
  j_n(k r_s) j_n(k r) P_n(cos g),  A_n = -(h_n'(ka) - i beta h_n(ka)) / (j_n'(ka) - i beta j_n(ka)).
"""
from __future__ import annotations

import numpy as np
from scipy import special as sp


def image_sum_rigid_box(L, rs, pts, k, tol=1e-13):
    L = np.asarray(L, float)
    rs = np.asarray(rs, float)
    pts = np.atleast_2d(np.asarray(pts, float))
    k = complex(k)
    if k.imag <= 0:
        raise ValueError("image sum needs a damped wavenumber (Im k > 0)")
    # radius beyond which exp(-Im k R)/R < tol
    Rmax = 1.0
    while np.exp(-k.imag * Rmax) / Rmax > tol:
        Rmax *= 1.2
    nmax = np.ceil(Rmax / (2 * L)).astype(int) + 1
    out = np.zeros(pts.shape[0], np.complex128)
    signs = np.array([[sx, sy, sz] for sx in (1, -1) for sy in (1, -1) for sz in (1, -1)], float)
    ax = [np.arange(-nmax[d], nmax[d] + 1) for d in range(3)]
    P = np.stack(np.meshgrid(*ax, indexing="ij"), -1).reshape(-1, 3) * (2 * L)[None, :]
    for s in signs:
        img = P + (s * rs)[None, :]
        for ip, x in enumerate(pts):
            r = np.linalg.norm(img - x[None, :], axis=1)
            keep = r < Rmax
            rr = r[keep]
            out[ip] += np.sum(np.exp(1j * k * rr) / (4 * np.pi * rr))
    return out


def _h(n, x, d=False):
    return sp.spherical_jn(n, x, d) + 1j * sp.spherical_yn(n, x, d)


def sphere_robin_interior(a, beta, k, rs, pts, nmax=None):
    """Scattered field psi_sc inside a sphere of radius a (centre at the origin)."""
    rs = np.asarray(rs, float)
    pts = np.atleast_2d(np.asarray(pts, float))
    ka = k * a
    if nmax is None:
        nmax = int(ka + 30)
    rsn = np.linalg.norm(rs)
    rn = np.linalg.norm(pts, axis=1)
    if rsn > 0:
        cg = (pts @ rs) / np.where(rn > 0, rn, 1) / rsn
    else:
        cg = np.ones(pts.shape[0])
    out = np.zeros(pts.shape[0], np.complex128)
    for n in range(nmax + 1):
        An = -(_h(n, ka, True) - 1j * beta * _h(n, ka)) / (sp.spherical_jn(n, ka, True) - 1j * beta * sp.spherical_jn(n, ka))
        out += (2 * n + 1) * An * sp.spherical_jn(n, k * rsn) * sp.spherical_jn(n, k * rn) * sp.eval_legendre(n, cg)
    return 1j * k / (4 * np.pi) * out
