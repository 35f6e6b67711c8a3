"""Pins of the image-source solution Eq. (an2) with reflection coefficient R (Section 4.1)."""
import numpy as np

from oracle import analytic


L = (3.0, 2.5, 2.0)
RS = np.array([1.1, 0.7, 1.3])


def test_r1_matches_rigid_lattice():
    """R = 1: the pinned rigid-box lattice (damped k, both truncated far beyond the decay)."""
    k = 4.0 + 0.8j
    pts = np.array([[0.4, 1.9, 0.5], [2.6, 0.3, 1.7]])
    a = analytic.image_sum_box(L, RS, pts, k, 1.0, r_max=60.0)
    b = analytic.image_sum_rigid_box(L, RS, pts, k)
    assert np.allclose(a, b, rtol=1e-9, atol=0)


def test_r0_is_free_field():
    pts = np.array([[0.4, 1.9, 0.5], [2.6, 0.3, 1.7]])
    k = 5.0
    a = analytic.image_sum_box(L, RS, pts, k, 0.0, r_max=30.0)
    r = np.linalg.norm(pts - RS[None, :], axis=1)
    assert np.allclose(a, np.exp(1j * k * r) / (4 * np.pi * r), rtol=1e-14, atol=0)


def test_r_minus1_vanishes_on_walls():
    """R = -1 (pressure-release walls): the image sum is the box's Dirichlet Green's function, so it
    vanishes on every wall -- which needs every image's reflection count right (a miscounted image
    breaks the pairwise cancellation across a wall).  Damped k and a large truncation radius."""
    k = 3.0 + 1.0j
    rng = np.random.default_rng(7)
    wall = []
    for d in range(3):
        for side in (0.0, L[d]):
            p = rng.uniform(0.2, 0.8, 3) * np.asarray(L)
            p[d] = side
            wall.append(p)
    wall = np.array(wall)
    v = analytic.image_sum_box(L, RS, wall, k, -1.0, r_max=40.0)
    inside = analytic.image_sum_box(L, RS, np.array([[1.5, 1.2, 1.0]]), k, -1.0, r_max=40.0)
    assert np.max(np.abs(v)) < 1e-9 * abs(inside[0])
    # the same points with R = +1 do not vanish (the check has teeth)
    assert np.min(np.abs(analytic.image_sum_box(L, RS, wall, k, 1.0, r_max=40.0))) > 1e-3
