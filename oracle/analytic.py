"""Closed-form solutions used to pin the oracle -- TEST INFRASTRUCTURE ONLY.

* image_sum_rigid_box: the image-source solution of Section 4.1 (Eq. an2) with A_j = R^{n_j}
  and R = 1.  For sound-hard walls (Eq. sp5) the 8-image lattice with periods 2L is the exact
  Neumann Green's function of the box.  With a real wavenumber the lattice sum does not
  converge, so it is evaluated with a damped k (Im k > 0) and truncated where
  exp(-Im k R)/R falls below `tol`; the BEM is run with the same complex k.
* image_sum_box: Eq. (an2) with A_j = R^{n_j} for a constant reflection coefficient R, truncated
  by distance and amplitude as in Section 4.1 (the validation solution of the paper's impulse
  responses; an approximation for impedance walls, whose reflection coefficient depends on angle).
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


def image_sum_box(L, rs, pts, k, R, r_max, a_th=1e-7):
    """Eq. (an2): psi(r, k) = G_k(r, r_s) + sum_j A_j G_k(r, r_j) for a box [0,Lx]x[0,Ly]x[0,Lz], the
    images r_j of r_s with A_j = R^{n_j}, n_j the number of wall reflections that make the image
    (per axis: the image at 2 n L + x_s takes |2n| reflections, the one at 2 n L - x_s takes
    |2n - 1|); images farther than r_max from the evaluation point or with |A_j| < a_th are left
    out (Section 4.1: r_max = c T_max, A_th = 1e-7)."""
    L = np.asarray(L, float)
    rs = np.asarray(rs, float)
    pts = np.atleast_2d(np.asarray(pts, float))
    k = complex(k)
    nmax = np.ceil(r_max / (2 * L)).astype(int) + 1
    pos, cnt = [], []
    for d in range(3):
        n = np.arange(-nmax[d], nmax[d] + 1)
        pos.append(np.concatenate([2 * n * L[d] + rs[d], 2 * n * L[d] - rs[d]]))
        cnt.append(np.concatenate([np.abs(2 * n), np.abs(2 * n - 1)]))
    X, Y, Z = np.meshgrid(*pos, indexing="ij")
    CX, CY, CZ = np.meshgrid(*cnt, indexing="ij")
    img = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    nref = (CX + CY + CZ).ravel()
    if R == 0:
        amp = (nref == 0).astype(float)
    else:
        amp = np.power(float(R), nref)
    keep = np.abs(amp) >= a_th
    img, amp = img[keep], amp[keep]
    out = np.zeros(pts.shape[0], np.complex128)
    for ip, x in enumerate(pts):
        r = np.linalg.norm(img - x[None, :], axis=1)
        sel = r < r_max
        rr = r[sel]
        out[ip] = np.sum(amp[sel] * np.exp(1j * k * rr) / (4 * np.pi * rr))
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
