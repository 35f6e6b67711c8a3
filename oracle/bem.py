"""CPU oracle for the collocation BEM (direct and indirect) -- TEST INFRASTRUCTURE ONLY.

Plain FP64 numpy on top of the C routines in bem_oracle.c.  Used by tests/, the smoke
check and the benchmark's CPU-baseline leg; never by the product path.

Definitions followed (paper, Sections 2-3):
  * incident field psi_in = G(r, r_s), unit monopole (Eq. sp6)
  * impedance condition -zeta dpsi/dn + i k psi = 0 with beta = 1/zeta (Eq. sp3),
    so k/(i zeta) = -i k beta and gamma = -(dpsi_in/dn) + i k beta psi_in (Eq. sp7)
  * direct BIE for psi_sc (Eq. dbem4):
        (A x)_i = 1/2 x_i + sum_j M_ij x_j - i k sum_j L_ij beta_j x_j ,   b = L gamma
    with the per-element admittance entering as a column scaling of L
  * field off the surface from Green's representation (Eq. dbem1):
        psi(r) = psi_in(r) + L[dpsi_sc/dn](r) - M[psi_sc](r),  dpsi_sc/dn = gamma + i k beta psi_sc
  * indirect BIE (Eq. ibem5) on two-sided elements, unknowns (psi-, psi+) with the normal
    pointing from the - side (the room) to the + side, k/(i zeta) = -i k beta on each side:
        row 1:  (psi- + psi+)/2 + L[s] + M[m]
        row 2:  (i k beta- psi- - i k beta+ psi+)/2 + L'[s] + M'[m]
    with s = -i k (beta- psi- + beta+ psi+), m = psi- - psi+; right-hand sides
        row 1:  L[g- + g+],   row 2: (g+ - g-)/2 + L'[g- + g+],   g-+ = -+ dpsi_in/dn + i k beta-+ psi_in
    and the field psi = psi_in + L[sigma] + M[mu] (Eq. ibem1) with
    sigma = g- + g+ + i k (beta- psi- + beta+ psi+), mu = psi+ - psi- (Eq. ibem4)
  * combined (Burton-Miller) direct equation: Eq. (dbem3) plus alpha = i/k times its normal
    derivative (see bm_system), same unknown and field as Eq. (dbem4)
  * normal-derivative form, Eq. (dbem5): unknown dpsi_sc/dn (see dpsi_system)
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import build as _build

_lib = None
DEFAULT_ETA = 0.35


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        i64, f64 = ctypes.c_int64, ctypes.c_double
        L.oracle_geometry.argtypes = [i64, dp, ip, dp, dp, dp]
        L.oracle_dense_LM.argtypes = [i64, dp, i64, ip, f64, f64, f64, f64, dp, dp]
        L.oracle_layer_rows.argtypes = [i64, dp, i64, ip, f64, f64, f64, f64, i64, ip, dp, dp, dp]
        L.oracle_field.argtypes = [i64, dp, i64, ip, f64, f64, f64, f64, i64, dp, dp, dp, dp]
        L.oracle_pair.argtypes = [dp, dp, f64, f64, ctypes.c_int, f64, dp]
        L.oracle_dense_LMn.argtypes = [i64, dp, i64, ip, f64, f64, f64, f64, dp, dp, dp, dp]
        L.oracle_layer_rows_n.argtypes = [i64, dp, i64, ip, f64, f64, f64, f64, i64, ip, dp, dp, dp, dp]
        L.oracle_pair4.argtypes = [dp, dp, dp, f64, f64, ctypes.c_int, f64, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _mesh(V, T):
    return np.ascontiguousarray(V, np.float64), np.ascontiguousarray(T, np.int64)


def geometry(V, T):
    """Centroids, unit normals ((v1-v0)x(v2-v0) normalised) and areas of flat triangles."""
    V, T = _mesh(V, T)
    n = T.shape[0]
    c, nrm, a = np.empty((n, 3)), np.empty((n, 3)), np.empty(n)
    lib().oracle_geometry(n, _d(V), _i(T), _d(c), _d(nrm), _d(a))
    return c, nrm, a


def near_cutoff(V, T, factor=1.8):
    """Near cutoff r_c of the accurate-integration rule (reading of Section 3.3, which leaves it
    unspecified): factor times the side sqrt(2 A_mean) of the square cell that two triangles of
    the mean area make.  Pairs with |c_i - c_j|^2 < r_c^2 are integrated accurately."""
    _, _, a = geometry(V, T)
    return factor * math.sqrt(2.0 * math.fsum(a) / a.shape[0])


def dense_LM(V, T, k, rc, eta=DEFAULT_ETA):
    """Dense single- and double-layer matrices L_ij, M_ij (complex, N x N)."""
    V, T = _mesh(V, T)
    n = T.shape[0]
    L = np.empty((n, n), np.complex128)
    M = np.empty((n, n), np.complex128)
    k = complex(k)
    lib().oracle_dense_LM(V.shape[0], _d(V), n, _i(T), k.real, k.imag, float(rc), float(eta), _d(L), _d(M))
    return L, M


def layer_rows(V, T, k, rc, rows, sigma, mu, eta=DEFAULT_ETA):
    """sum_j L_ij sigma_j + M_ij mu_j for the listed collocation rows (matrix-free)."""
    V, T = _mesh(V, T)
    rows = np.ascontiguousarray(rows, np.int64)
    sigma = np.ascontiguousarray(sigma, np.complex128)
    mu = np.ascontiguousarray(mu, np.complex128)
    out = np.empty(rows.shape[0], np.complex128)
    k = complex(k)
    lib().oracle_layer_rows(V.shape[0], _d(V), T.shape[0], _i(T), k.real, k.imag, float(rc), float(eta),
                            rows.shape[0], _i(rows), _d(sigma), _d(mu), _d(out))
    return out


def layer_field(V, T, k, rc, pts, sigma, mu, eta=DEFAULT_ETA):
    """L[sigma](r) + M[mu](r) at off-surface points."""
    V, T = _mesh(V, T)
    pts = np.ascontiguousarray(np.atleast_2d(pts), np.float64)
    sigma = np.ascontiguousarray(sigma, np.complex128)
    mu = np.ascontiguousarray(mu, np.complex128)
    out = np.empty(pts.shape[0], np.complex128)
    k = complex(k)
    lib().oracle_field(V.shape[0], _d(V), T.shape[0], _i(T), k.real, k.imag, float(rc), float(eta),
                       pts.shape[0], _d(pts), _d(sigma), _d(mu), _d(out))
    return out


def pair(x, tri_xyz, k, self=False, eta=DEFAULT_ETA):
    """Accurate (L_j(x), M_j(x)) for one triangle (3x3 vertex array)."""
    x = np.ascontiguousarray(x, np.float64)
    tri = np.ascontiguousarray(tri_xyz, np.float64)
    out = np.empty(4)
    k = complex(k)
    lib().oracle_pair(_d(x), _d(tri), k.real, k.imag, int(self), float(eta), _d(out))
    return out[0] + 1j * out[1], out[2] + 1j * out[3]


def dense_LMn(V, T, k, rc, eta=DEFAULT_ETA):
    """Dense L, M, L', M' (complex, N x N each); L', M' use the normal of the row element."""
    V, T = _mesh(V, T)
    n = T.shape[0]
    out = [np.empty((n, n), np.complex128) for _ in range(4)]
    k = complex(k)
    lib().oracle_dense_LMn(V.shape[0], _d(V), n, _i(T), k.real, k.imag, float(rc), float(eta),
                           *[_d(o) for o in out])
    return tuple(out)


def layer_rows_n(V, T, k, rc, rows, sigma, mu, eta=DEFAULT_ETA):
    """Rows of L[sigma] + M[mu] and of L'[sigma] + M'[mu] at the listed collocation points."""
    V, T = _mesh(V, T)
    rows = np.ascontiguousarray(rows, np.int64)
    sigma = np.ascontiguousarray(sigma, np.complex128)
    mu = np.ascontiguousarray(mu, np.complex128)
    y = np.empty(rows.shape[0], np.complex128)
    yn = np.empty(rows.shape[0], np.complex128)
    k = complex(k)
    lib().oracle_layer_rows_n(V.shape[0], _d(V), T.shape[0], _i(T), k.real, k.imag, float(rc), float(eta),
                              rows.shape[0], _i(rows), _d(sigma), _d(mu), _d(y), _d(yn))
    return y, yn


def pair4(x, nx, tri_xyz, k, self=False, eta=DEFAULT_ETA):
    """Accurate (L, M, L', M') of one triangle at x with normal nx (self: x = centroid)."""
    x = np.ascontiguousarray(x, np.float64)
    nx = np.ascontiguousarray(nx, np.float64)
    tri = np.ascontiguousarray(tri_xyz, np.float64)
    out = np.empty(8)
    k = complex(k)
    lib().oracle_pair4(_d(x), _d(nx), _d(tri), k.real, k.imag, int(self), float(eta), _d(out))
    return tuple(out[2 * q] + 1j * out[2 * q + 1] for q in range(4))


# ----------------------------------------------------------------------------- problem data
def green(x, y, k):
    r = np.linalg.norm(np.asarray(x) - np.asarray(y), axis=-1)
    return np.exp(1j * k * r) / (4 * np.pi * r)


def incident(c, nrm, k, rs):
    """psi_in and dpsi_in/dn at the points c with normals nrm (unit monopole at rs, Eq. sp6)."""
    d = c - np.asarray(rs)[None, :]
    r = np.linalg.norm(d, axis=1)
    G = np.exp(1j * k * r) / (4 * np.pi * r)
    dGdn = G * (1j * k * r - 1.0) * (d * nrm).sum(1) / r ** 2
    return G, dGdn


def gamma(c, nrm, beta, k, rs):
    """gamma = -(dpsi_in/dn + k/(i zeta) psi_in) = -dpsi_in/dn + i k beta psi_in (Eq. sp7)."""
    psi, dpsi = incident(c, nrm, k, rs)
    return -dpsi + 1j * k * beta * psi


def direct_system(V, T, k, beta, rs, rc, eta=DEFAULT_ETA):
    """Dense A and b of Eq. (dbem4); also returns (L, M) and gamma."""
    L, M = dense_LM(V, T, k, rc, eta)
    c, nrm, _ = geometry(V, T)
    n = T.shape[0]
    A = 0.5 * np.eye(n) + M - 1j * k * L * beta[None, :]
    g = gamma(c, nrm, beta, k, rs)
    b = L @ g
    return A, b, (L, M), g


def direct_matvec_rows(V, T, k, beta, rc, x, rows, eta=DEFAULT_ETA):
    """(A x)_i of Eq. (dbem4) for selected rows, without forming A."""
    rows = np.asarray(rows, np.int64)
    y = layer_rows(V, T, k, rc, rows, -1j * k * beta * x, x, eta)
    return 0.5 * x[rows] + y


def direct_rhs_rows(V, T, k, beta, rs, rc, rows, eta=DEFAULT_ETA):
    c, nrm, _ = geometry(V, T)
    g = gamma(c, nrm, beta, k, rs)
    return layer_rows(V, T, k, rc, rows, g, np.zeros_like(g), eta)


def direct_receivers(V, T, k, beta, rs, rc, x, pts, eta=DEFAULT_ETA):
    """psi(r) = G(r, rs) + L[gamma + i k beta x](r) - M[x](r)   (Eq. dbem1)."""
    c, nrm, _ = geometry(V, T)
    g = gamma(c, nrm, beta, k, rs)
    sc = layer_field(V, T, k, rc, pts, g + 1j * k * beta * x, -x, eta)
    return green(pts, np.asarray(rs)[None, :], k) + sc


# ----------------------------------------------------------------------------- indirect formulation
def gamma_pm(c, nrm, beta_m, beta_p, k, rs):
    """g- = -dpsi_in/dn + i k beta- psi_in,  g+ = +dpsi_in/dn + i k beta+ psi_in (Eq. ibem4)."""
    psi, dpsi = incident(c, nrm, k, rs)
    return -dpsi + 1j * k * beta_m * psi, dpsi + 1j * k * beta_p * psi


def indirect_system(V, T, k, beta_m, beta_p, rs, rc, eta=DEFAULT_ETA):
    """Dense 2N x 2N operator and right-hand side of Eq. (ibem5), unknowns (psi-, psi+)."""
    L, M, Lp, Mp = dense_LMn(V, T, k, rc, eta)
    c, nrm, _ = geometry(V, T)
    n = T.shape[0]
    I = np.eye(n)
    bm, bp = beta_m[None, :], beta_p[None, :]
    # s = -ik(bm psi- + bp psi+), m = psi- - psi+
    A = np.block([[0.5 * I - 1j * k * L * bm + M, 0.5 * I - 1j * k * L * bp - M],
                  [np.diag(0.5j * k * beta_m) - 1j * k * Lp * bm + Mp, np.diag(-0.5j * k * beta_p) - 1j * k * Lp * bp - Mp]])
    gm, gp = gamma_pm(c, nrm, beta_m, beta_p, k, rs)
    b = np.concatenate([L @ (gm + gp), 0.5 * (gp - gm) + Lp @ (gm + gp)])
    return A, b


def indirect_matvec_rows(V, T, k, beta_m, beta_p, rc, x, rows, eta=DEFAULT_ETA):
    """Rows (of both blocks) of the Eq. (ibem5) operator applied to x = (psi-, psi+)."""
    n = T.shape[0]
    rows = np.asarray(rows, np.int64)
    pm, pp = x[:n], x[n:]
    s = -1j * k * (beta_m * pm + beta_p * pp)
    y, yn = layer_rows_n(V, T, k, rc, rows, s, pm - pp, eta)
    r1 = 0.5 * (pm[rows] + pp[rows]) + y
    r2 = 0.5j * k * (beta_m[rows] * pm[rows] - beta_p[rows] * pp[rows]) + yn
    return r1, r2


def indirect_rhs_rows(V, T, k, beta_m, beta_p, rs, rc, rows, eta=DEFAULT_ETA):
    c, nrm, _ = geometry(V, T)
    gm, gp = gamma_pm(c, nrm, beta_m, beta_p, k, rs)
    rows = np.asarray(rows, np.int64)
    y, yn = layer_rows_n(V, T, k, rc, rows, gm + gp, np.zeros_like(gm), eta)
    return y, 0.5 * (gp - gm)[rows] + yn


def indirect_receivers(V, T, k, beta_m, beta_p, rs, rc, x, pts, eta=DEFAULT_ETA):
    """psi(r) = G(r, rs) + L[sigma](r) + M[mu](r)  (Eq. ibem1, ibem4)."""
    n = T.shape[0]
    c, nrm, _ = geometry(V, T)
    gm, gp = gamma_pm(c, nrm, beta_m, beta_p, k, rs)
    pm, pp = x[:n], x[n:]
    sigma = gm + gp + 1j * k * (beta_m * pm + beta_p * pp)
    sc = layer_field(V, T, k, rc, pts, sigma, pp - pm, eta)
    return green(pts, np.asarray(rs)[None, :], k) + sc


# ----------------------------------------------------------------------------- combined direct form
# Burton-Miller combination of the direct equation (reading: coupling alpha = i/k).  For the
# scattered field psi on S with v = dpsi/dn = gamma + i k beta psi, Green's representation taken
# to S from the room gives the surface equation of Eq. (dbem3)
#       psi/2 + M[psi] - L[v] = 0,
# and its normal derivative, with the single-layer jump dL[v]/dn -> L'[v] + v/2 from the room side
# (Section 3.2), gives
#       v/2 - L'[v] + M'[psi] = 0.
# The combined equation is the first plus alpha times the second; with v substituted:
#   A psi = psi/2 + (alpha i k / 2) beta psi + M psi - i k L[beta psi] + alpha (M'[psi] - i k L'[beta psi])
#   b     = L[gamma] + alpha (L'[gamma] - gamma / 2)
def bm_alpha(k):
    """Coupling constant of the combined direct equation (reading: alpha = i/k)."""
    return 1j / k


def bm_system(V, T, k, beta, rs, rc, eta=DEFAULT_ETA):
    """Dense A and b of the combined (Burton-Miller) direct equation; also returns gamma."""
    L, M, Lp, Mp = dense_LMn(V, T, k, rc, eta)
    c, nrm, _ = geometry(V, T)
    a = bm_alpha(k)
    A = (np.diag(0.5 + 0.5j * a * k * beta) + M - 1j * k * L * beta[None, :]
         + a * (Mp - 1j * k * Lp * beta[None, :]))
    g = gamma(c, nrm, beta, k, rs)
    b = L @ g + a * (Lp @ g - 0.5 * g)
    return A, b, g


def bm_matvec_rows(V, T, k, beta, rc, x, rows, eta=DEFAULT_ETA):
    """Rows of the combined direct operator applied to x, without forming it."""
    rows = np.asarray(rows, np.int64)
    a = bm_alpha(k)
    y, yn = layer_rows_n(V, T, k, rc, rows, -1j * k * beta * x, x, eta)
    return (0.5 + 0.5j * a * k * beta[rows]) * x[rows] + y + a * yn


def bm_rhs_rows(V, T, k, beta, rs, rc, rows, eta=DEFAULT_ETA):
    c, nrm, _ = geometry(V, T)
    g = gamma(c, nrm, beta, k, rs)
    rows = np.asarray(rows, np.int64)
    a = bm_alpha(k)
    y, yn = layer_rows_n(V, T, k, rc, rows, g, np.zeros_like(g), eta)
    return y + a * (yn - 0.5 * g[rows])


# ----------------------------------------------------------------------------- normal-derivative form
# Eq. (dbem5): unknown v = dpsi_sc/dn.  With the impedance condition psi_sc = zeta (v - gamma) / (i k)
# (zeta = 1/beta) in Eq. (dbem3), multiplied by i k / zeta at the collocation point:
#   A v = v/2 + beta M[zeta v] - i k beta L[v],     b = gamma/2 + beta M[zeta gamma]
# (per element: beta_i on the row, zeta_j on the column).  Needs beta != 0 on every element.
def dpsi_system(V, T, k, beta, rs, rc, eta=DEFAULT_ETA):
    """Dense A and b of Eq. (dbem5); also returns gamma."""
    L, M = dense_LM(V, T, k, rc, eta)
    c, nrm, _ = geometry(V, T)
    zeta = 1.0 / beta
    n = T.shape[0]
    A = 0.5 * np.eye(n) + beta[:, None] * (M * zeta[None, :] - 1j * k * L)
    g = gamma(c, nrm, beta, k, rs)
    b = 0.5 * g + beta * (M @ (zeta * g))
    return A, b, g


def dpsi_matvec_rows(V, T, k, beta, rc, v, rows, eta=DEFAULT_ETA):
    rows = np.asarray(rows, np.int64)
    y = layer_rows(V, T, k, rc, rows, -1j * k * v, v / beta, eta)
    return 0.5 * v[rows] + beta[rows] * y


def dpsi_rhs_rows(V, T, k, beta, rs, rc, rows, eta=DEFAULT_ETA):
    c, nrm, _ = geometry(V, T)
    g = gamma(c, nrm, beta, k, rs)
    rows = np.asarray(rows, np.int64)
    y = layer_rows(V, T, k, rc, rows, np.zeros_like(g), g / beta, eta)
    return 0.5 * g[rows] + beta[rows] * y


def dpsi_to_psi(V, T, k, beta, rs, v):
    """psi_sc on the elements from the normal-derivative unknown: psi_sc = (v - gamma) / (i k beta)."""
    c, nrm, _ = geometry(V, T)
    return (v - gamma(c, nrm, beta, k, rs)) / (1j * k * beta)


# ----------------------------------------------------------------------------- dense solvers
def solve_lu(A, b):
    return np.linalg.solve(A, b)


def gmres(A, b, tol=1e-10, restart=50, maxit=2000, x0=None, precond=None):
    """Plain restarted (flexible) GMRES with modified Gram-Schmidt and Givens rotations.
    `A` is a matrix or a callable; `precond` an optional callable z = P(v).
    Returns (x, iterations, relative residual history)."""
    mv = A if callable(A) else (lambda v: A @ v)
    pc = precond if precond is not None else (lambda v: v)
    n = b.shape[0]
    x = np.zeros(n, np.complex128) if x0 is None else np.array(x0, np.complex128)
    bn = np.linalg.norm(b)
    hist, it = [], 0
    while it < maxit:
        r = b - mv(x)
        beta0 = np.linalg.norm(r)
        hist.append(beta0 / bn)
        if beta0 / bn < tol:
            break
        Vk = np.zeros((restart + 1, n), np.complex128)
        Z = np.zeros((restart, n), np.complex128)
        H = np.zeros((restart + 1, restart), np.complex128)
        cs, sn = np.zeros(restart, np.complex128), np.zeros(restart, np.complex128)
        g = np.zeros(restart + 1, np.complex128)
        g[0] = beta0
        Vk[0] = r / beta0
        j_done = 0
        for j in range(restart):
            Z[j] = pc(Vk[j])
            w = mv(Z[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(Vk[i], w)
                w = w - H[i, j] * Vk[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                Vk[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(abs(H[j, j]), abs(H[j + 1, j]))
            cs[j] = abs(H[j, j]) / den if den else 1.0
            sn[j] = (H[j, j] / abs(H[j, j]) if H[j, j] != 0 else 1.0) * np.conj(H[j + 1, j]) / den if den else 0.0
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            if abs(g[j + 1]) / bn < tol or it >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + Z[:j_done].T @ y
    return x, it, np.array(hist)
