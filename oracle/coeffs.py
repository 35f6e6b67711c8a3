"""Plain definitions of the FMM expansion bases and translation/rotation coefficients --
TEST INFRASTRUCTURE ONLY.

Expansions of Eq. (shft0): S_n^m(r) = h_n(kr) Y_n^m(r/r), R_n^m(r) = j_n(kr) Y_n^m(r/r), n < p.
Y_n^m is the orthonormal spherical harmonic with the associated Legendre function taken
without the Condon-Shortley phase, so that Y_n^{-m} = conj(Y_n^m); with this choice the
zonal seed (Eq. shft1) and the recursions of Section 3.3.1 hold with the a_n^m, b_n^m given
below.  The coaxial coefficients are *defined* by Eq. (shft0.1) (sum over n'):
    F_n^m(r + tau i_z) = sum_{n'} (E|F)^m_{n'n}(tau) R_{n'}^m(r)
and are computed here by projecting the left side onto Y_{n'}^m on a sphere |r| = rho
(Gauss-Legendre in cos(theta); the azimuthal integral is exact because a translation along z
keeps the azimuth).  Rotation coefficients are defined by
    Y_n^m(u) = sum_{m'} T^n_{m m'}(Q) Y_n^{m'}(Q u)
and computed by projection on a product Gauss grid over the sphere.
"""
from __future__ import annotations

import numpy as np
from scipy import special as sp


def idx(n, m):
    return n * n + n + m


def legendre_bar(nmax, x):
    """Orthonormal associated Legendre values P[n, m] (0 <= m <= n <= nmax), no Condon-Shortley
    phase, so that Y_n^m = P[n,|m|] exp(i m phi)."""
    x = np.asarray(x, float)
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    P = np.zeros((nmax + 1, nmax + 1) + x.shape)
    P[0, 0] = 1.0 / np.sqrt(4 * np.pi)
    for m in range(1, nmax + 1):
        P[m, m] = np.sqrt((2 * m + 1) / (2.0 * m)) * s * P[m - 1, m - 1]
    for m in range(nmax + 1):
        if m + 1 <= nmax:
            P[m + 1, m] = np.sqrt(2 * m + 3.0) * x * P[m, m]
        for n in range(m + 2, nmax + 1):
            a = np.sqrt((4.0 * n * n - 1) / (n * n - m * m))
            b = np.sqrt(((n - 1.0) ** 2 - m * m) * (2 * n + 1) / ((2 * n - 3) * (n * n - m * m)))
            P[n, m] = a * x * P[n - 1, m] - b * P[n - 2, m]
    return P


def legendre_order(nmax, m, x):
    """Column m of legendre_bar: P[n] = P_n^m for n = 0..nmax (zero for n < m), the same
    recurrences evaluated for one order only."""
    x = np.asarray(x, float)
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    P = np.zeros((nmax + 1,) + x.shape)
    pmm = np.full(x.shape, 1.0 / np.sqrt(4 * np.pi))
    for q in range(1, m + 1):
        pmm = np.sqrt((2 * q + 1) / (2.0 * q)) * s * pmm
    if m > nmax:
        return P
    P[m] = pmm
    if m + 1 <= nmax:
        P[m + 1] = np.sqrt(2 * m + 3.0) * x * pmm
    for n in range(m + 2, nmax + 1):
        a = np.sqrt((4.0 * n * n - 1) / (n * n - m * m))
        b = np.sqrt(((n - 1.0) ** 2 - m * m) * (2 * n + 1) / ((2 * n - 3) * (n * n - m * m)))
        P[n] = a * x * P[n - 1] - b * P[n - 2]
    return P


def Y(nmax, pts):
    """Y[..., idx(n,m)] for points (..., 3) (direction only)."""
    pts = np.asarray(pts, float)
    r = np.linalg.norm(pts, axis=-1)
    ct = np.where(r > 0, pts[..., 2] / np.where(r > 0, r, 1.0), 1.0)
    phi = np.arctan2(pts[..., 1], pts[..., 0])
    P = legendre_bar(nmax, ct)
    out = np.zeros(pts.shape[:-1] + ((nmax + 1) ** 2,), np.complex128)
    for n in range(nmax + 1):
        for m in range(-n, n + 1):
            out[..., idx(n, m)] = P[n, abs(m)] * np.exp(1j * m * phi)
    return out


def jn(n, x):
    return sp.spherical_jn(n, x)


def hn(n, x):
    return sp.spherical_jn(n, x) + 1j * sp.spherical_yn(n, x)


def basis(kind, nmax, k, pts):
    """R_n^m (kind 'R') or S_n^m (kind 'S') at points (..., 3)."""
    pts = np.asarray(pts, float)
    r = np.linalg.norm(pts, axis=-1)
    out = Y(nmax, pts)
    f = jn if kind == "R" else hn
    for n in range(nmax + 1):
        out[..., n * n:(n + 1) ** 2] *= f(n, k * r)[..., None]
    return out


def a_coef(n, m):
    """a_n^m = sqrt((n+1+|m|)(n+1-|m|)/((2n+1)(2n+3))) for n >= |m|, else 0."""
    m = abs(m)
    if n < m:
        return 0.0
    return np.sqrt((n + 1 + m) * (n + 1 - m) / ((2 * n + 1) * (2 * n + 3)))


def b_coef(n, m):
    """b_n^m = sign(m) sqrt((n-m-1)(n-m)/((2n-1)(2n+1))), sign + for m >= 0, 0 for |m| > n."""
    if abs(m) > n:
        return 0.0
    v = np.sqrt((n - m - 1) * (n - m) / ((2 * n - 1) * (2 * n + 1)))
    return v if m >= 0 else -v


def coaxial_projection(kind, k, tau, p, m, rows=None):
    """(E|F)^m_{n'n}(tau) for n, n' in [|m|, p) by projection; kind 'SR' or 'RR'.
    Each row n' is projected at the radius (from a candidate set) where |j_{n'}(k rho)| is
    largest, so that the division by j_{n'}(k rho) stays well conditioned."""
    m = abs(m)
    rows = list(range(m, p)) if rows is None else list(rows)
    rho_max = 0.6 * tau if kind == "SR" else max(1.5 * tau, (p + 10) / k)
    cands = rho_max * np.linspace(0.15, 1.0, 12)
    out = np.zeros((p, p), np.complex128)
    choice = {}
    for nn in rows:
        vals = np.abs(jn(nn, k * cands))
        choice.setdefault(int(np.argmax(vals)), []).append(nn)
    for ci, nns in choice.items():
        rho = cands[ci]
        Q = 2 * p + int(2 * k * (rho + tau)) + 80
        xg, wg = np.polynomial.legendre.leggauss(Q)
        pts = np.stack([rho * np.sqrt(1 - xg ** 2), 0 * xg, rho * xg], -1)
        sh = pts + np.array([0.0, 0.0, tau])
        B = basis("S" if kind == "SR" else "R", p - 1, k, sh)
        Yr = Y(p - 1, pts)
        for nn in nns:
            jj = jn(nn, k * rho)
            for n in range(m, p):
                out[nn, n] = 2 * np.pi * np.sum(wg * B[:, idx(n, m)] * np.conj(Yr[:, idx(nn, m)])) / jj
    return out


def coaxial_projection_order(kind, k, tau, p, m, rows=None):
    """coaxial_projection evaluated with order m of the basis only (the projection points lie at
    azimuth 0, where Y_n^m reduces to P_n^m(cos theta)): the same definition at a cost linear in
    p per point, for the high truncation numbers of the top octree levels."""
    m = abs(m)
    rows = list(range(m, p)) if rows is None else list(rows)
    rho_max = 0.6 * tau if kind == "SR" else max(1.5 * tau, (p + 10) / k)
    cands = rho_max * np.linspace(0.15, 1.0, 12)
    out = np.zeros((p, p), np.complex128)
    choice = {}
    for nn in rows:
        vals = np.abs(jn(nn, k * cands))
        choice.setdefault(int(np.argmax(vals)), []).append(nn)
    for ci, nns in choice.items():
        rho = cands[ci]
        Q = 2 * p + int(2 * k * (rho + tau)) + 80
        xg, wg = np.polynomial.legendre.leggauss(Q)
        # points in the x-z half plane (azimuth 0): Y_n^m there is P_n^m(cos theta) alone, so only
        # order m of the basis is needed, at the points and at the points shifted by tau along z
        sh_z = rho * xg + tau
        sh_r = np.sqrt(rho * rho * (1 - xg ** 2) + sh_z ** 2)
        Psh = legendre_order(p - 1, m, sh_z / sh_r)
        Pr = legendre_order(p - 1, m, xg)
        f = jn if kind == "RR" else hn
        for nn in nns:
            jj = jn(nn, k * rho)
            for n in range(m, p):
                out[nn, n] = 2 * np.pi * np.sum(wg * f(n, k * sh_r) * Psh[n] * Pr[nn]) / jj
    return out


def sphere_grid(L):
    xg, wg = np.polynomial.legendre.leggauss(L + 1)
    nphi = 2 * L + 2
    ph = 2 * np.pi * np.arange(nphi) / nphi
    ct, P = np.meshgrid(xg, ph, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    pts = np.stack([st * np.cos(P), st * np.sin(P), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    return pts, w


def rotation_projection(nmax, Q):
    """List of T^n(Q), (2n+1)x(2n+1), rows m, cols m' (index m + n)."""
    pts, w = sphere_grid(2 * nmax + 2)
    Yu = Y(nmax, pts)
    YQ = Y(nmax, pts @ np.asarray(Q, float).T)
    out = []
    for n in range(nmax + 1):
        s = slice(n * n, (n + 1) ** 2)
        out.append((Yu[:, s] * w[:, None]).T @ np.conj(YQ[:, s]))
    return out


def rot_y(b):
    c, s = np.cos(b), np.sin(b)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def rot_z(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
