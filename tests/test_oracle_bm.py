"""Pins of the oracle's combined (Burton-Miller) direct equation: exact boundary data of a field
that satisfies the Helmholtz equation in the room make both of its halves vanish as the mesh is
refined, and its solution gives the same interior field as Eq. (dbem4)."""
import numpy as np

from oracle import bem
from paper_2103_16073_amd import synth


def test_bm_solution_converges_to_exact_trace():
    """With the monopole outside the room, the scattered field -psi_in cancels the incident one:
    the total field is zero, which satisfies the Helmholtz equation and the impedance condition
    inside, so the exact surface unknown is -psi_in at the centroids (unique for Re beta > 0).
    The combined system's solution (operator and right-hand side as the oracle builds them)
    converges to it under refinement (measured 21 %, 13.6 %, 9.7 % at N = 296, 696, 1184: first
    order, the collocated hypersingular part with constant elements; Eq. dbem4 gives 6.4 %, 2.9 %,
    1.9 %).  A wrong sign or a dropped term in either half leaves an O(1) error that does not fall."""
    k = 3.0
    r_out = np.array([4.1, 1.3, 0.9])  # outside the 3 x 2.5 x 2 m box
    errs = []
    for h in (0.5, 0.34):
        room = synth.shoebox(3.0, 2.5, 2.0, h)
        V, T = room.vertices, room.triangles
        c, nrm, area = bem.geometry(V, T)
        rc = 1.8 * np.sqrt(2 * area.mean())
        beta = np.linspace(0.05, 0.3, room.n) * (1 + 0.5j)
        exact = -bem.incident(c, nrm, k, r_out)[0]
        A, b, _ = bem.bm_system(V, T, k, beta, r_out, rc)
        x = bem.solve_lu(A, b)
        errs.append(np.linalg.norm(x - exact) / np.linalg.norm(exact))
        print(f"h {h}: N {room.n} error vs exact trace {errs[-1]:.3e}")
    assert errs[1] < 0.75 * errs[0] and errs[1] < 0.15


def test_bm_halves_vanish_on_exact_data():
    """Each half of the combined equation, built from the oracle's L, M, L', M', vanishes on the
    traces (psi, dpsi/dn) of an interior Helmholtz solution up to a discretisation error that
    falls under refinement; flipping the sign of the jump term v/2 leaves an O(1) residual."""
    k = 3.0
    r_out = np.array([4.1, 1.3, 0.9])
    halves = []
    for h in (0.5, 0.34):
        room = synth.shoebox(3.0, 2.5, 2.0, h)
        V, T = room.vertices, room.triangles
        c, nrm, area = bem.geometry(V, T)
        rc = 1.8 * np.sqrt(2 * area.mean())
        psi, v = bem.incident(c, nrm, k, r_out)
        L, M, Lp, Mp = bem.dense_LMn(V, T, k, rc)
        eq1 = 0.5 * psi + M @ psi - L @ v
        eq2 = 0.5 * v - Lp @ v + Mp @ psi
        halves.append((np.linalg.norm(eq1) / np.linalg.norm(psi), np.linalg.norm(eq2) / np.linalg.norm(v)))
        print(f"h {h}: N {room.n} halves {halves[-1][0]:.3e} {halves[-1][1]:.3e}")
    assert halves[1][0] < halves[0][0] < 0.05 and halves[1][1] < halves[0][1] < 0.1
    assert np.linalg.norm(-0.5 * v - Lp @ v + Mp @ psi) / np.linalg.norm(v) > 0.5


def test_bm_matches_direct_inside_closed_room():
    """The combined equation and Eq. (dbem4) discretise the same boundary-value problem: their
    interior fields (Eq. dbem1) agree, and the difference falls under refinement (the combined
    form carries the slower, first-order error of the collocated hypersingular part)."""
    diffs = []
    for h in (0.5, 0.34):
        room = synth.shoebox(3.0, 2.5, 2.0, h)
        V, T = room.vertices, room.triangles
        k = 4.0
        beta = np.full(room.n, 0.2 + 0.05j)
        rs, rec = synth.source_and_receivers(room, 8)
        c, _, area = bem.geometry(V, T)
        rc = 1.8 * np.sqrt(2 * area.mean())
        A, b, _, _ = bem.direct_system(V, T, k, beta, rs[0], rc)
        xd = bem.solve_lu(A, b)
        pd = bem.direct_receivers(V, T, k, beta, rs[0], rc, xd, rec)
        Ab, bb, _ = bem.bm_system(V, T, k, beta, rs[0], rc)
        xb = bem.solve_lu(Ab, bb)
        pb = bem.direct_receivers(V, T, k, beta, rs[0], rc, xb, rec)
        diffs.append(np.linalg.norm(pb - pd) / np.linalg.norm(pd))
        print(f"h {h}: N {room.n} receivers rel diff {diffs[-1]:.3e}, "
              f"surface {np.linalg.norm(xb - xd) / np.linalg.norm(xd):.3e}")
    assert diffs[1] < diffs[0]
    assert diffs[1] < 0.1


def test_bm_rows_match_dense_system():
    """The row routines (used at sizes where no dense matrix fits) reproduce the dense operator
    and right-hand side."""
    room = synth.shoebox(3.0, 2.5, 2.0, 0.5)
    V, T = room.vertices, room.triangles
    k = 5.0
    beta = np.linspace(0.05, 0.3, room.n) + 0.02j
    rs, _ = synth.source_and_receivers(room, 2)
    c, _, area = bem.geometry(V, T)
    rc = 1.8 * np.sqrt(2 * area.mean())
    A, b, _ = bem.bm_system(V, T, k, beta, rs[0], rc)
    x = synth.complex_normal(room.n, 3)
    rows = np.arange(0, room.n, 5)
    y = bem.bm_matvec_rows(V, T, k, beta, rc, x, rows)
    assert np.linalg.norm(y - (A @ x)[rows]) <= 1e-12 * np.linalg.norm(y)
    r = bem.bm_rhs_rows(V, T, k, beta, rs[0], rc, rows)
    assert np.linalg.norm(r - b[rows]) <= 1e-12 * np.linalg.norm(r)
