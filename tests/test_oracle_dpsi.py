"""Pins of the oracle's normal-derivative form, Eq. (dbem5): its solution converges to the exact
normal derivative when the monopole sits outside the room, its interior field agrees with Eq.
(dbem4)'s, and its operator is Eq. (dbem4)'s similarity transform by the admittance."""
import numpy as np

from oracle import bem
from paper_2103_16073_amd import synth


def test_dpsi_solution_converges_to_exact_normal_derivative():
    """Monopole outside the room: the scattered field -psi_in cancels the incident one (total field
    zero satisfies the impedance condition), so the exact unknown is -dpsi_in/dn at the centroids.
    The Eq. (dbem5) solution converges to it under refinement (Eq. dbem4's unknown -psi_in alongside)."""
    k = 3.0
    r_out = np.array([4.1, 1.3, 0.9])
    e5, e4 = [], []
    for h in (0.5, 0.34):
        room = synth.shoebox(3.0, 2.5, 2.0, h)
        V, T = room.vertices, room.triangles
        c, nrm, area = bem.geometry(V, T)
        rc = 1.8 * np.sqrt(2 * area.mean())
        beta = np.linspace(0.05, 0.3, room.n) * (1 + 0.5j)
        psi_in, dpsi_in = bem.incident(c, nrm, k, r_out)
        A, b, _ = bem.dpsi_system(V, T, k, beta, r_out, rc)
        v = bem.solve_lu(A, b)
        e5.append(np.linalg.norm(v + dpsi_in) / np.linalg.norm(dpsi_in))
        A4, b4, _, _ = bem.direct_system(V, T, k, beta, r_out, rc)
        x = bem.solve_lu(A4, b4)
        e4.append(np.linalg.norm(x + psi_in) / np.linalg.norm(psi_in))
        # the unknowns are tied by the impedance condition: psi_sc = (v - gamma) / (i k beta)
        assert np.allclose(bem.dpsi_to_psi(V, T, k, beta, r_out, v), x, rtol=0, atol=1e-9 * np.abs(x).max())
        print(f"h {h}: N {room.n} dbem5 error {e5[-1]:.3e}, dbem4 error {e4[-1]:.3e}")
    assert e5[1] < 0.75 * e5[0] and e5[1] < 0.05


def test_dpsi_field_matches_direct():
    """Interior source: the field at receivers from the Eq. (dbem5) solution (converted to psi_sc)
    equals Eq. (dbem4)'s: the two operators are similar (A5 = B A4 B^-1, B = diag(beta)) and the
    right-hand sides correspond (b5 = B b4 up to the v/2 - psi terms), so the discrete solutions
    agree to rounding, not only in the limit."""
    room = synth.shoebox(3.0, 2.5, 2.0, 0.34)
    V, T = room.vertices, room.triangles
    k = 4.0
    beta = np.linspace(0.05, 0.3, room.n) + 0.02j
    rs, rec = synth.source_and_receivers(room, 8)
    c, _, area = bem.geometry(V, T)
    rc = 1.8 * np.sqrt(2 * area.mean())
    A4, b4, _, _ = bem.direct_system(V, T, k, beta, rs[0], rc)
    x = bem.solve_lu(A4, b4)
    A5, b5, _ = bem.dpsi_system(V, T, k, beta, rs[0], rc)
    v = bem.solve_lu(A5, b5)
    x5 = bem.dpsi_to_psi(V, T, k, beta, rs[0], v)
    print(f"N {room.n}: surface rel diff {np.linalg.norm(x5 - x) / np.linalg.norm(x):.2e}")
    assert np.linalg.norm(x5 - x) <= 1e-10 * np.linalg.norm(x)
    p4 = bem.direct_receivers(V, T, k, beta, rs[0], rc, x, rec)
    p5 = bem.direct_receivers(V, T, k, beta, rs[0], rc, x5, rec)
    assert np.linalg.norm(p5 - p4) <= 1e-10 * np.linalg.norm(p4)
    # similarity: A5 = B A4 B^-1
    B = np.diag(beta)
    assert np.allclose(A5, B @ A4 @ np.diag(1 / beta), rtol=0, atol=1e-12 * np.abs(A5).max())


def test_dpsi_rows_match_dense_system():
    room = synth.shoebox(3.0, 2.5, 2.0, 0.5)
    V, T = room.vertices, room.triangles
    k = 5.0
    beta = np.linspace(0.05, 0.3, room.n) + 0.02j
    rs, _ = synth.source_and_receivers(room, 2)
    c, _, area = bem.geometry(V, T)
    rc = 1.8 * np.sqrt(2 * area.mean())
    A, b, _ = bem.dpsi_system(V, T, k, beta, rs[0], rc)
    v = synth.complex_normal(room.n, 4)
    rows = np.arange(0, room.n, 5)
    y = bem.dpsi_matvec_rows(V, T, k, beta, rc, v, rows)
    assert np.linalg.norm(y - (A @ v)[rows]) <= 1e-12 * np.linalg.norm(y)
    r = bem.dpsi_rhs_rows(V, T, k, beta, rs[0], rc, rows)
    assert np.linalg.norm(r - b[rows]) <= 1e-12 * np.linalg.norm(r)
