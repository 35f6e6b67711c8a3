"""Indirect formulation (Eq. ibem3-ibem5) through the C ABI against the oracle: near entries
of L' and M', the product (all-pairs and FMM), the right-hand side, the solve and the field."""
import numpy as np
import pytest

from oracle import bem
from rc_check import oracle_rc
from paper_2103_16073_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    from paper_2103_16073_amd import fmmbem
    return fmmbem


def make_ctx(F, V, T, k, beta_m, beta_p=None, nsrc=1, rs=None, **opt):
    ctx = F.Context(0, **opt)
    ctx.fmmbem_set_mesh(V, T)
    ctx.fmmbem_set_wavenumber(k)
    ctx.fmmbem_set_admittance(beta_m, beta_p)
    ctx.fmmbem_set_formulation(F.FMMBEM_INDIRECT)
    if rs is not None:
        ctx.fmmbem_set_sources(rs)
    return ctx


def open_room(h=0.17):
    """Shoebox 3 x 2.5 x 2 m with a 1 x 1 m doorway hole in the wall x = 0 (its elements
    removed) and a 1 x 1 m zero-thickness plate at x = 1.5 (two-sided)."""
    room = synth.shoebox(3.0, 2.5, 2.0, h)
    V, T = room.vertices, room.triangles
    c = V[T].mean(1)
    keep = ~((np.abs(c[:, 0]) < 1e-9) & (c[:, 1] > 0.7) & (c[:, 1] < 1.7) & (c[:, 2] < 1.0))
    T = T[keep]
    beta = room.beta[keep]
    # plate: a 1 x 1 m square at x = 1.5 meshed like a wall, normal +x
    m = int(np.ceil(1.0 / h))
    ys, zs = np.linspace(0.8, 1.8, m + 1), np.linspace(0.5, 1.5, m + 1)
    base = V.shape[0]
    pv = np.array([[1.5, y, z] for y in ys for z in zs])
    tris = []
    for i in range(m):
        for j in range(m):
            a, b, cc, d = i * (m + 1) + j, (i + 1) * (m + 1) + j, (i + 1) * (m + 1) + j + 1, i * (m + 1) + j + 1
            tris += [(a, b, cc), (a, cc, d)]
    pt = np.array(tris) + base
    V = np.vstack([V, pv])
    T = np.vstack([T, pt])
    beta = np.concatenate([beta, np.full(pt.shape[0], 0.15)])
    return V, T, beta


def test_near_entries_Lp_Mp_vs_oracle(F):
    room, k = synth.config_room(1)
    ctx = make_ctx(F, room.vertices, room.triangles, k, room.beta)
    r, c, L, M = ctx.fmmbem_near_entries()
    Lp, Mp = ctx.fmmbem_near_entries_n()
    cen, nrm, _ = bem.geometry(room.vertices, room.triangles)
    rng = np.random.default_rng(3)
    off = np.nonzero(r != c)[0]
    sel = np.concatenate([rng.choice(off, 1200, replace=False), np.nonzero(r == c)[0][:300]])
    for e in sel:
        i, j = r[e], c[e]
        ref = bem.pair4(cen[i], nrm[i], room.vertices[room.triangles[j]], k, self=(i == j))
        assert abs(Lp[e] - ref[2]) <= 1e-9 * abs(ref[0]) + 1e-12, (i, j, Lp[e], ref[2])
        assert abs(Mp[e] - ref[3]) <= 1e-9 * abs(ref[3]) + 1e-9, (i, j, Mp[e], ref[3])
    ctx.close()


@pytest.fixture(scope="module")
def dense_ind():
    room, k = synth.config_room(1)
    beta_p = np.full(room.n, 0.1)
    rc_ctx = None
    return room, k, beta_p


def _dense_operator(room, k, beta_m, beta_p, rc):
    L, M, Lp, Mp = bem.dense_LMn(room.vertices, room.triangles, k, rc)
    n = room.n
    I = np.eye(n)
    bm, bp = beta_m[None, :], beta_p[None, :]
    return np.block([[0.5 * I - 1j * k * L * bm + M, 0.5 * I - 1j * k * L * bp - M],
                     [np.diag(0.5j * k * beta_m) - 1j * k * Lp * bm + Mp, np.diag(-0.5j * k * beta_p) - 1j * k * Lp * bp - Mp]])


@pytest.mark.parametrize("leaf_max", [64, 12])
def test_indirect_product_vs_dense(F, dense_ind, leaf_max):
    """The indirect operator: all-pairs product to 1e-10 and FMM product (potential and normal
    derivative of the far field from the same expansions) to 1e-6 against the dense oracle."""
    room, k, beta_p = dense_ind
    ctx = make_ctx(F, room.vertices, room.triangles, k, room.beta, beta_p, leaf_max=leaf_max)
    assert ctx.fmmbem_num_unknowns() == 2 * room.n
    rc = oracle_rc(ctx, room)
    A = _dense_operator(room, k, room.beta, beta_p, rc)
    for seed in (1, 2):
        x = synth.complex_normal(2 * room.n, seed)
        ref = A @ x
        ye = ctx.fmmbem_matvec(x, exact_far=True)[0]
        assert np.linalg.norm(ye - ref) / np.linalg.norm(ref) < 1e-10
        y = ctx.fmmbem_matvec(x)[0]
        e1 = np.linalg.norm(y[:room.n] - ref[:room.n]) / np.linalg.norm(ref[:room.n])
        e2 = np.linalg.norm(y[room.n:] - ref[room.n:]) / np.linalg.norm(ref[room.n:])
        print(f"leaf_max {leaf_max}: row-1 err {e1:.3e}, row-2 err {e2:.3e}")
        assert e1 < 1e-6 and e2 < 1e-6
        # mixed precision: FP32 translations between FP64 P2M and FP64 local derivatives / L2P
        ym = ctx.fmmbem_matvec(x, precision=F.FMMBEM_MIXED)[0]
        m1 = np.linalg.norm(ym[:room.n] - ref[:room.n]) / np.linalg.norm(ref[:room.n])
        m2 = np.linalg.norm(ym[room.n:] - ref[room.n:]) / np.linalg.norm(ref[room.n:])
        print(f"leaf_max {leaf_max}: mixed row-1 err {m1:.3e}, row-2 err {m2:.3e}")
        assert m1 < 1e-4 and m2 < 1e-4
    # the FP64 product is unaffected by a mixed one before it
    y2 = ctx.fmmbem_matvec(x)[0]
    assert np.array_equal(y2, y)
    with pytest.raises(RuntimeError):
        ctx.fmmbem_matvec(x, precision=F.FMMBEM_MIXED, exact_far=True)
    ctx.close()


def test_indirect_full_size_rows_vs_oracle(F):
    """The 6x5x3 m room at 1 kHz (N = 90,972, 181,944 unknowns) in the indirect formulation, a
    different admittance on the + faces: both block rows of the FMM product (FP64 <= 1e-6, mixed
    <= 1e-4) and of the right-hand side (1e-6) on 256 seeded rows against the oracle's matrix-free
    rows of Eq. ibem5."""
    room, k = synth.config_room(2)
    n = room.n
    beta_p = 0.5 * room.beta + 0.05
    rs, _ = synth.source_and_receivers(room, 4)
    ctx = make_ctx(F, room.vertices, room.triangles, k, room.beta, beta_p, rs=rs)
    rc = oracle_rc(ctx, room)
    x = synth.complex_normal(2 * n, 17)
    rows = np.random.default_rng(12).choice(n, 256, replace=False)
    r1, r2 = bem.indirect_matvec_rows(room.vertices, room.triangles, k, room.beta, beta_p, rc, x, rows)
    for prec, tol in ((F.FMMBEM_FP64, 1e-6), (F.FMMBEM_MIXED, 1e-4)):
        y = ctx.fmmbem_matvec(x, precision=prec)[0]
        e1 = np.linalg.norm(y[rows] - r1) / np.linalg.norm(r1)
        e2 = np.linalg.norm(y[n + rows] - r2) / np.linalg.norm(r2)
        print(f"precision {prec}: row-1 {e1:.2e}, row-2 {e2:.2e}")
        assert e1 < tol and e2 < tol
    b = ctx.fmmbem_rhs()[0]
    b1, b2 = bem.indirect_rhs_rows(room.vertices, room.triangles, k, room.beta, beta_p, rs[0], rc, rows)
    assert np.linalg.norm(b[rows] - b1) / np.linalg.norm(b1) < 1e-6
    assert np.linalg.norm(b[n + rows] - b2) / np.linalg.norm(b2) < 1e-6
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_indirect_two_streams_match_one_stream(F, prec):
    """The indirect product on two streams (near field beside P2M and the translations) adds every
    contribution in the same order as on one stream: bitwise equal results (6x5x3 m room at 1 kHz,
    octree depth >= 5)."""
    room, k = synth.config_room(2)
    ctxs = [make_ctx(F, room.vertices, room.triangles, k, room.beta, None, streams=s) for s in (1, 2)]
    x = synth.complex_normal(2 * room.n, 31)
    y1, y2 = (c.fmmbem_matvec(x, precision=prec)[0] for c in ctxs)
    assert ctxs[1].fmmbem_get_info().depth >= 5
    assert np.array_equal(y1, y2)
    for c in ctxs:
        c.close()


def test_indirect_rhs_vs_oracle(F, dense_ind):
    room, k, beta_p = dense_ind
    rs, _ = synth.source_and_receivers(room, 4)
    ctx = make_ctx(F, room.vertices, room.triangles, k, room.beta, beta_p, rs=rs)
    b = ctx.fmmbem_rhs()[0]
    rc = oracle_rc(ctx, room)
    rows = np.arange(0, room.n, 7)
    r1, r2 = bem.indirect_rhs_rows(room.vertices, room.triangles, k, room.beta, beta_p, rs[0], rc, rows)
    assert np.linalg.norm(b[rows] - r1) / np.linalg.norm(r1) < 1e-6
    assert np.linalg.norm(b[room.n + rows] - r2) / np.linalg.norm(r2) < 1e-6
    ctx.close()


def test_indirect_open_room_solve_and_field_vs_lu(F):
    """Open room (doorway hole, two-sided plate): FGMRES with the 2x2 element-block diagonal
    preconditioner agrees with the LU solution of the oracle's dense indirect system, and the
    field at receivers with the oracle's (Eq. ibem1)."""
    V, T, beta = open_room(0.34)
    k = synth.wavenumber(250.0)
    rs = np.array([[2.2, 1.3, 1.1]])
    rec = np.array([[0.8, 0.6, 0.7], [2.5, 2.0, 1.5], [1.2, 1.9, 0.4], [2.7, 0.4, 1.8]])
    ctx = make_ctx(F, V, T, k, beta, None, rs=rs)
    x, rep, rc_ = ctx.fmmbem_solve(0, tol=1e-9, restart=200, maxit=600, precond=F.FMMBEM_PC_DIAG)
    print(f"open room N {T.shape[0]}: iters {rep.iters} rel {rep.rel_res:.2e}")
    assert rc_ == 0 and rep.rel_res < 1e-9
    rc = oracle_rc(ctx, V, T)
    A, b = bem.indirect_system(V, T, k, beta, beta, rs[0], rc)
    x_ref = bem.solve_lu(A, b)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-5
    psi = ctx.fmmbem_eval_field(0, rec, x)
    psi_ref = bem.indirect_receivers(V, T, k, beta, beta, rs[0], rc, x_ref, rec)
    assert np.linalg.norm(psi - psi_ref) / np.linalg.norm(psi_ref) < 1e-5
    # mixed-precision Krylov products (FP32 translations, FP32 Krylov storage) with FP64 restart
    # residuals reach the same FP64 residual target and the same solution
    xm, repm, rcm = ctx.fmmbem_solve(0, tol=1e-7, restart=200, maxit=600, precond=F.FMMBEM_PC_DIAG,
                                     precision=F.FMMBEM_MIXED)
    print(f"open room mixed: iters {repm.iters} restarts {repm.restarts} rel {repm.rel_res:.2e} "
          f"mixed products {repm.matvecs_mixed}")
    assert rcm == 0 and repm.rel_res < 1e-7 and repm.matvecs_mixed > 0
    assert np.linalg.norm(xm - x_ref) / np.linalg.norm(x_ref) < 1e-5
    ctx.close()


def test_indirect_leaf_blocks_vs_lu_and_diag(F):
    """Near-field leaf blocks of the two-sided operator (each leaf's 2 n_b unknowns, inverted):
    on the open room the solution equals the LU solution of the oracle's dense indirect system,
    in fewer FGMRES iterations than with the 2x2 element blocks."""
    V, T, beta = open_room(0.34)
    k = synth.wavenumber(250.0)
    rs = np.array([[2.2, 1.3, 1.1]])
    ctx = make_ctx(F, V, T, k, beta, None, rs=rs)
    xd, repd, rcd = ctx.fmmbem_solve(0, tol=1e-9, restart=200, maxit=600, precond=F.FMMBEM_PC_DIAG)
    xb, repb, rcb = ctx.fmmbem_solve(0, tol=1e-9, restart=200, maxit=600, precond=F.FMMBEM_PC_NEARBLOCK)
    print(f"open room N {T.shape[0]}: iterations diag {repd.iters}, leaf blocks {repb.iters}")
    assert rcd == 0 and rcb == 0 and repb.rel_res < 1e-9
    rc = oracle_rc(ctx, V, T)
    A, b = bem.indirect_system(V, T, k, beta, beta, rs[0], rc)
    x_ref = bem.solve_lu(A, b)
    assert np.linalg.norm(xb - x_ref) / np.linalg.norm(x_ref) < 1e-5
    assert repb.iters < repd.iters
    ctx.close()


def test_indirect_leaf_blocks_6x5x3_room(F):
    """The 6x5x3 m room at 1 kHz (N = 90,972, 2N unknowns) with both preconditioners, mixed
    products, relative residual 1e-6: the leaf blocks converge in fewer iterations and to the same
    solution as the 2x2 element blocks."""
    room, k = synth.config_room(2)
    rs, _ = synth.source_and_receivers(room, 4)
    ctx = make_ctx(F, room.vertices, room.triangles, k, room.beta, None, rs=rs)
    kw = dict(tol=1e-6, restart=400, maxit=400, precision=F.FMMBEM_MIXED)
    xd, repd, rcd = ctx.fmmbem_solve(0, precond=F.FMMBEM_PC_DIAG, **kw)
    xb, repb, rcb = ctx.fmmbem_solve(0, precond=F.FMMBEM_PC_NEARBLOCK, **kw)
    print(f"6x5x3 room, indirect: iterations diag {repd.iters} ({repd.t_solve_s:.2f} s), leaf blocks "
          f"{repb.iters} ({repb.t_solve_s:.2f} s)")
    assert rcd == 0 and rcb == 0 and repb.iters < repd.iters
    assert np.linalg.norm(xb - xd) / np.linalg.norm(xd) < 1e-4
    ctx.close()
