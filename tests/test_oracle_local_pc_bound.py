"""What a per-leaf learned preconditioner can gain at most (CPU, oracle's dense operator).

The learned slot maps the residual restricted to one octree leaf to a correction on that leaf. The
best such map that is linear is the leaf's diagonal block of the exact inverse A^-1; for residuals of
Gaussian-like spread the best map of any form (the conditional mean) is that linear one.  On the
L-room these blocks give flexible GMRES the same iteration count as the leaf blocks of A itself (the
plain near-field block preconditioner), so a map that sees one leaf has nothing to learn; maps that
see the leaf's 26 neighbours too (rows of A^-1 over the neighbourhood) do cut the iterations, which
sets the ceiling of a wider-input network."""
import numpy as np
import pytest

from oracle import bem
from paper_2103_16073_amd import synth


def uniform_leaves(c, target=64):
    """Cubes of the smallest uniform grid (bounding cube halved per level) whose non-empty cells
    hold at most `target` elements on average (the library's depth rule without the cutoff bound)."""
    lo = c.min(0) - 1e-9
    side = (c.max(0) + 1e-9 - lo).max()
    for depth in range(1, 12):
        d = side / 2 ** depth
        key = np.floor((c - lo) / d).astype(np.int64)
        _, inv = np.unique(key[:, 0] * 4096 * 4096 + key[:, 1] * 4096 + key[:, 2], return_inverse=True)
        if len(c) / (inv.max() + 1) <= target:
            return [np.where(inv == q)[0] for q in range(inv.max() + 1)], d
    raise RuntimeError("no depth")


def block_map(M, rows_of, cols_of):
    maps = [(r, cl, M[np.ix_(r, cl)]) for r, cl in zip(rows_of, cols_of)]

    def pc(v):
        z = np.zeros_like(v)
        for r, cl, B in maps:
            z[r] = B @ v[cl]
        return z
    return pc


@pytest.mark.slow
def test_exact_local_inverse_blocks_gain_nothing_over_leaf_blocks():
    room = synth.lroom(0.3)
    k = synth.wavenumber(250.0)
    V, T = room.vertices, room.triangles
    rs, _ = synth.source_and_receivers(room, 4)
    A, b, _, _ = bem.direct_system(V, T, k, room.beta, rs[0], bem.near_cutoff(V, T))
    c, _, _ = bem.geometry(V, T)
    L, side = uniform_leaves(c)
    Ainv = np.linalg.inv(A)
    cen = np.array([c[i].mean(0) for i in L])
    nbrs = [np.concatenate([L[p] for p in range(len(L)) if np.max(np.abs(cen[p] - cen[q])) < 1.8 * side])
            for q in range(len(L))]
    inv_blocks = [(i, np.linalg.inv(A[np.ix_(i, i)])) for i in L]

    def leaf_blocks(v):
        z = np.zeros_like(v)
        for i, B in inv_blocks:
            z[i] = B @ v[i]
        return z
    its = {}
    for name, pc in (("none", None), ("leaf blocks of A", leaf_blocks), ("leaf blocks of A^-1", block_map(Ainv, L, L)),
                     ("rows of A^-1 over 27 leaves", block_map(Ainv, L, nbrs))):
        x, it, hist = bem.gmres(A, b, tol=1e-8, restart=400, maxit=400, precond=pc)
        assert hist[-1] < 1e-8
        its[name] = it
    print(f"N {room.n}, {len(L)} leaves: iterations {its}")
    assert its["leaf blocks of A"] < its["none"]
    # the exact local inverse does no better than the local blocks of A ...
    assert abs(its["leaf blocks of A^-1"] - its["leaf blocks of A"]) <= 1
    # ... while a map that also sees the neighbouring leaves does
    assert its["rows of A^-1 over 27 leaves"] <= 0.85 * its["leaf blocks of A"]
