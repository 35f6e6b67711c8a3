"""Pins of the oracle's coefficient definitions (projection integrals) against closed forms
and identities printed in the paper, and against the addition theorem evaluated at points."""
import numpy as np
import pytest

from oracle import coeffs as C


@pytest.mark.parametrize("kind,k,tau", [("SR", 1.0, 5.0), ("SR", 1.0, 40.0), ("RR", 1.0, 5.0), ("RR", 2.0, 30.0)])
def test_zonal_seed_closed_form(kind, k, tau):
    """Eq. (shft1): (S|R)^0_{n'0} = (-1)^n' sqrt(2n'+1) h_n'(k tau), same with j for (R|R)."""
    p = 14
    T = C.coaxial_projection(kind, k, tau, p, 0)
    f = C.hn if kind == "SR" else C.jn
    for nn in range(p):
        ref = (-1) ** nn * np.sqrt(2 * nn + 1) * f(nn, k * tau)
        assert abs(T[nn, 0] - ref) < 1e-10 * max(abs(ref), 1e-3)


@pytest.mark.parametrize("kind", ["SR", "RR"])
def test_addition_theorem_at_points(kind):
    """sum_n' (E|F)^m_{n'n} R_n'^m(r) reproduces F_n^m(r + tau i_z) away from the projection sphere."""
    k, tau, p = 1.3, 4.0, 34
    rng = np.random.default_rng(2)
    pts = rng.normal(size=(6, 3))
    pts *= (0.9 / np.linalg.norm(pts, axis=1))[:, None]
    R = C.basis("R", p - 1, k, pts)
    F = C.basis("S" if kind == "SR" else "R", 8, k, pts + np.array([0, 0, tau]))
    for m in (0, 2, -3):
        T = C.coaxial_projection(kind, k, tau, p, m)
        for n in range(abs(m), 8):
            approx = sum(T[nn, n] * R[:, C.idx(nn, m)] for nn in range(abs(m), p))
            assert np.max(np.abs(approx - F[:, C.idx(n, m)])) < 1e-9 * np.max(np.abs(F[:, C.idx(n, m)]))


@pytest.mark.parametrize("kind", ["SR", "RR"])
def test_coaxial_symmetry_step4(kind):
    """Step 4 of the coaxial algorithm: (E|F)^m_{n'n} = (-1)^{n+n'} (E|F)^m_{nn'}."""
    p = 12
    for m in (0, 1, 4):
        T = C.coaxial_projection(kind, 1.0, 6.0, p, m)
        s = slice(m, p)
        sgn = (-1.0) ** np.add.outer(np.arange(p), np.arange(p))
        assert np.max(np.abs(T[s, s] - (sgn * T.T)[s, s])) < 1e-10 * np.max(np.abs(T[s, s]))


def test_rotation_unitary_and_composition():
    Q1 = C.rot_z(0.4) @ C.rot_y(1.1)
    Q2 = C.rot_y(-0.7) @ C.rot_z(2.0)
    T1, T2, T12 = C.rotation_projection(6, Q1), C.rotation_projection(6, Q2), C.rotation_projection(6, Q2 @ Q1)
    for n in range(7):
        I = np.eye(2 * n + 1)
        assert np.max(np.abs(T1[n] @ T1[n].conj().T - I)) < 1e-12
        assert np.max(np.abs(T1[n] @ T2[n] - T12[n])) < 1e-12


def test_rotation_degree_one_explicit():
    """Degree 1: sqrt(4pi/3) Y_1^0 = z, sqrt(8pi/3) Y_1^{+-1} = x +- i y (no Condon-Shortley
    phase), so T^1(Q) follows from the 3x3 matrix: u = Q^T (Q u)."""
    Q = C.rot_z(0.3) @ C.rot_y(0.8) @ C.rot_z(-1.2)
    T = C.rotation_projection(1, Q)[1]
    # coefficient vectors of Y_1^m in the Cartesian components (x, y, z)
    s1, s0 = np.sqrt(3 / (8 * np.pi)), np.sqrt(3 / (4 * np.pi))
    B = np.array([[s1, -1j * s1, 0], [0, 0, s0], [s1, 1j * s1, 0]])  # rows m=-1,0,1
    # Y_1^m(u) = B[m] . u = B[m] . Q^T v with v = Q u; write in Y_1^{m'}(v): v = Binv Y(v)
    Binv = np.linalg.inv(B)
    T_exp = B @ Q.T @ Binv
    assert np.max(np.abs(T - T_exp)) < 1e-13


def test_order_only_projection_equals_full_projection():
    """The order-only evaluation of the projection agrees with the full one (p = 14, several m)."""
    for kind, ktau in (("SR", 5.0), ("RR", 3.0), ("SR", 12.0)):
        for m in (0, 3, 9):
            A = C.coaxial_projection(kind, 1.0, ktau, 14, m)
            B = C.coaxial_projection_order(kind, 1.0, ktau, 14, m)
            assert np.max(np.abs(A - B)) < 1e-9 * np.max(np.abs(A)), (kind, ktau, m)


def test_order_only_projection_zonal_closed_form_high_degree():
    """Eq. (shft1) at the truncation numbers of the top level of the 5 kHz room (p = 255,
    k tau = 600): (S|R)^0_{n'0} = (-1)^n' sqrt(2n'+1) h_n'(k tau) and the (R|R) analogue."""
    p, kt = 255, 600.0
    rows = [0, 97, 180, 254]
    for kind, f in (("SR", C.hn), ("RR", C.jn)):
        T = C.coaxial_projection_order(kind, 1.0, kt, p, 0, rows=rows)
        for nn in rows:
            ref = (-1) ** nn * np.sqrt(2 * nn + 1) * f(nn, kt)
            assert abs(T[nn, 0] - ref) < 1e-8 * abs(ref), (kind, nn, T[nn, 0], ref)
