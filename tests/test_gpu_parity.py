"""Parity of the HIP path (through the C ABI) with the CPU oracle, element by element."""
import numpy as np
import pytest

from oracle import bem
from rc_check import oracle_rc
from oracle import coeffs as OC
from paper_2103_16073_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    from paper_2103_16073_amd import fmmbem
    fmmbem.lib()
    return fmmbem


def make_ctx(F, room, k, **opt):
    ctx = F.Context(0, **opt)
    ctx.fmmbem_set_mesh(room.vertices, room.triangles)
    ctx.fmmbem_set_wavenumber(k)
    ctx.fmmbem_set_admittance(room.beta)
    return ctx


# ----------------------------------------------------------------------------- tables
@pytest.mark.parametrize("kind,ktau,p", [("SR", 5.0, 12), ("SR", 40.0, 30), ("RR", 5.0, 12), ("RR", 60.0, 40),
                                         ("SR", 0.6, 10), ("RR", 0.4, 10)])
def test_coaxial_table_vs_projection(F, kind, ktau, p):
    """Device recursion (stabilised for k tau >= 1, original below) against the projection
    definition of the coefficients."""
    blocks = F.fmmbem_coaxial_table(0 if kind == "SR" else 1, ktau, p)
    # errors are measured against the table's scale (the largest |entry| of block m = 0): at the
    # highest m the entries are many orders smaller and only absolute accuracy is meaningful
    scale = np.max(np.abs(blocks[0]))
    for m in sorted({0, 1, 2, p // 3, p - 2}):
        ref = OC.coaxial_projection(kind, 1.0, ktau, p, m)
        got = blocks[m]
        r = ref[m:, m:]
        assert np.max(np.abs(got - r)) < 1e-9 * scale, (m, np.max(np.abs(got - r)) / scale)


def test_coaxial_original_vs_stabilised_overlap(F):
    """Both device schemes agree where the original one is still accurate (k tau = 3)."""
    p = 20
    for kind in (0, 1):
        a = F.fmmbem_coaxial_table(kind, 3.0, p, method=0)
        b = F.fmmbem_coaxial_table(kind, 3.0, p, method=1)
        for m in range(p):
            s = np.max(np.abs(b[m]))
            assert np.max(np.abs(a[m] - b[m])) < 1e-10 * s


def test_coaxial_stable_at_high_ktau(F):
    """k tau = 150, p = 130 (R|R): the stabilised scheme matches the definition; the original
    propagation in n does not (the instability analysed in Section 3.3.1)."""
    p, kt = 130, 150.0
    st = F.fmmbem_coaxial_table(1, kt, p, method=1)
    orig = F.fmmbem_coaxial_table(1, kt, p, method=0)
    m = 40
    ref = OC.coaxial_projection("RR", 1.0, kt, p, m)[m:, m:]
    assert np.max(np.abs(st[m] - ref)) < 1e-9
    assert np.max(np.abs(orig[m] - ref)) > 1.0


@pytest.mark.parametrize("kind,ktau,ms", [("SR", 600.0, (0, 100, 200)), ("RR", 100.0, (0, 120, 230))])
def test_coaxial_table_top_level_of_5khz_room(F, kind, ktau, ms):
    """The stabilised recursion at the truncation number of the top level of the 5 kHz L-room (p =
    255; M2L k tau from about 460, M2M/L2L k tau about 100) against the projection definition on a
    few rows of several orders (errors against the table's scale, as above)."""
    p = 255
    blocks = F.fmmbem_coaxial_table(0 if kind == "SR" else 1, ktau, p)
    scale = np.max(np.abs(blocks[0]))
    for m in ms:
        rows = sorted({m, m + 40, m + 90, p - 1} & set(range(m, p)))
        ref = OC.coaxial_projection_order(kind, 1.0, ktau, p, m, rows=rows)
        for nn in rows:
            err = np.max(np.abs(blocks[m][nn - m] - ref[nn, m:]))
            assert err < 1e-8 * scale, (m, nn, err / scale)


def test_rotation_table_vs_projection(F):
    p = 10
    D = F.fmmbem_rotation_table(p)
    T = OC.rotation_projection(p - 1, OC.rot_y(np.pi / 2))
    for n in range(p):
        assert np.max(np.abs(D[n] - T[n].real)) < 1e-12
        assert np.max(np.abs(T[n].imag)) < 1e-12


def test_rotation_table_orthogonal_high_degree(F):
    D = F.fmmbem_rotation_table(500)
    for n in (100, 300, 499):
        err = np.max(np.abs(D[n] @ D[n].T - np.eye(2 * n + 1)))
        assert err < 1e-12, (n, err)


# ----------------------------------------------------------------------------- near field
def test_near_entries_vs_oracle(F):
    room = synth.shoebox(3.0, 2.5, 2.0, 0.34)
    k = synth.wavenumber(250.0)
    ctx = make_ctx(F, room, k)
    rows, cols, L, M = ctx.fmmbem_near_entries()
    rc = oracle_rc(ctx, room)
    c, _, _ = bem.geometry(room.vertices, room.triangles)
    # same pair set as the oracle's classification
    d2 = ((c[:, None, :] - c[None, :, :]) ** 2).sum(-1)
    near = (d2 < rc * rc) | np.eye(room.n, dtype=bool)
    assert len(rows) == near.sum()
    assert near[rows, cols].all()
    # margin: no pair within 1e-9 (relative) of the cutoff
    assert np.min(np.abs(np.sqrt(d2[~np.eye(room.n, dtype=bool)]) - rc)) > 1e-9 * rc
    sel = np.random.default_rng(0).choice(len(rows), 300, replace=False)
    for e in sel:
        tri = room.vertices[room.triangles[cols[e]]]
        Lr, Mr = bem.pair(c[rows[e]], tri, k, self=(rows[e] == cols[e]))
        assert abs(L[e] - Lr) < 1e-11 * abs(Lr)
        assert abs(M[e] - Mr) < 1e-11 * abs(Lr)
    ctx.close()


# ----------------------------------------------------------------------------- products
@pytest.fixture(scope="module")
def cfg1_dense():
    room, k = synth.config_room(1)
    return room, k


def test_matvec_exact_far_vs_dense(F, cfg1_dense):
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k)
    rc = oracle_rc(ctx, room)
    L, M = bem.dense_LM(room.vertices, room.triangles, k, rc)
    for seed in (1, 2):
        x = synth.complex_normal(room.n, seed)
        ref = 0.5 * x + M @ x - 1j * k * L @ (room.beta * x)
        y = ctx.fmmbem_matvec(x, exact_far=True)[0]
        assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-12
    ctx.close()


@pytest.mark.parametrize("reorth", [0, 1, 2])
def test_solve_gram_schmidt_passes_vs_oracle_lu(F, cfg1_dense, reorth):
    """One classical Gram-Schmidt pass, a second one when needed, or always two: each solve
    reaches the FP64 residual target and agrees with LU, single and batched."""
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k)
    rs, _ = synth.source_and_receivers(room, 4, nsrc=2)
    ctx.fmmbem_set_sources(rs)
    rc = oracle_rc(ctx, room)
    kw = dict(tol=1e-8, restart=200, maxit=200, precond=F.FMMBEM_PC_NEARBLOCK, reorth=reorth)
    x, rep, rc_ = ctx.fmmbem_solve(0, **kw)
    X, reps, rcb = ctx.fmmbem_solve_batch([0, 1], **kw)
    print(f"reorth {reorth}: iters {rep.iters} rel {rep.rel_res:.2e}; batched {[r.iters for r in reps]}")
    assert rc_ == 0 and rep.rel_res < 1e-8 and rcb == 0
    for s, xs in ((0, x), (0, X[0]), (1, X[1])):
        A, b, _, _ = bem.direct_system(room.vertices, room.triangles, k, room.beta, rs[s], rc)
        x_ref = bem.solve_lu(A, b)
        assert np.linalg.norm(xs - x_ref) / np.linalg.norm(x_ref) < 1e-5
    with pytest.raises(F.FmmbemError):
        ctx.fmmbem_solve(0, tol=1e-4, reorth=3)
    ctx.close()


def test_solve_inner_coarse_fmm_vs_oracle_lu(F, cfg1_dense):
    """The inner GMRES on a second FMM with a smaller truncation number (Section 4.3): the outer
    solve still reaches its FP64 target and agrees with LU; every inner product runs on the
    coarser operator; a new admittance reaches that operator before the next solve."""
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k)
    rs, _ = synth.source_and_receivers(room, 4)
    ctx.fmmbem_set_sources(rs)
    rc = oracle_rc(ctx, room)
    for beta in (room.beta, 0.5 * room.beta + 0.05):
        ctx.fmmbem_set_admittance(beta)
        x, rep, rc_ = ctx.fmmbem_solve(0, tol=1e-8, restart=20, maxit=60, inner_iters=8, inner_tol=1e-2,
                                       precision=F.FMMBEM_FP64, inner_p_min=6, inner_p_excess=0.5)
        print(f"coarse inner: outer {rep.iters} inner {rep.inner_iters} coarse {rep.matvecs_coarse} "
              f"fp64 {rep.matvecs_fp64} rel {rep.rel_res:.2e}")
        assert rc_ == 0 and rep.rel_res < 1e-8
        # an inner solve that ends on its iteration cap spends one more product on its true residual
        assert rep.inner_iters <= rep.matvecs_coarse <= rep.inner_iters + rep.iters
        assert rep.inner_iters > 0 and rep.matvecs_mixed == 0
        A, b, _, _ = bem.direct_system(room.vertices, room.triangles, k, beta, rs[0], rc)
        x_ref = bem.solve_lu(A, b)
        assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-5
    ctx.close()


@pytest.mark.parametrize("form", ["dpsi", "bm", "indirect"])
def test_solve_inner_coarse_fmm_other_formulations(F, cfg1_dense, form):
    """The coarser inner operator follows the formulation (Eq. dbem5, the combined form, the
    indirect Eq. ibem5): with it, FGMRES (diagonal preconditioner) reaches the solution of the
    plain solve (both to 1e-8) in fewer outer iterations."""
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k)
    rs, _ = synth.source_and_receivers(room, 4)
    ctx.fmmbem_set_sources(rs)
    f = {"dpsi": F.FMMBEM_DIRECT_DPSI, "bm": F.FMMBEM_DIRECT_BM, "indirect": F.FMMBEM_INDIRECT}[form]
    ctx.fmmbem_set_formulation(f)
    kw = dict(tol=1e-8, restart=300, maxit=900, precond=F.FMMBEM_PC_DIAG, precision=F.FMMBEM_FP64)
    x0, rep0, rc0 = ctx.fmmbem_solve(0, **kw)
    x1, rep1, rc1 = ctx.fmmbem_solve(0, inner_iters=6, inner_tol=1e-2, inner_p_min=4, inner_p_excess=0.0, **kw)
    print(f"{form}: plain {rep0.iters} its; coarse inner: outer {rep1.iters} inner {rep1.inner_iters} "
          f"coarse products {rep1.matvecs_coarse} rel {rep1.rel_res:.2e}")
    assert rc0 == 0 and rc1 == 0 and rep1.matvecs_coarse >= rep1.inner_iters > 0
    assert rep1.iters < rep0.iters
    assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) < 1e-5
    ctx.close()


def test_solve_inner_coarse_fmm_rejects_bad_opts(F, cfg1_dense):
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k)
    rs, _ = synth.source_and_receivers(room, 4)
    ctx.fmmbem_set_sources(rs)
    with pytest.raises(F.FmmbemError) as e:
        ctx.fmmbem_solve(0, tol=1e-4, inner_iters=4, inner_p_min=-1)
    assert e.value.code == F.FMMBEM_EINVAL
    ctx.close()


@pytest.mark.parametrize("leaf_max,lds_budget,lane,mfma,fused", [
    (64, 0, 0, 0, 0), (12, 0, 0, 0, 0), (12, 8192, 0, 0, 0), (64, 8192, 0, 0, 0), (64, 0, 2, 0, 0),
    (12, 0, 2, 0, 0), (64, 0, 2, 2, 0), (12, 0, 2, 2, 0), (64, 0, 2, 0, 1), (12, 0, 2, 0, 1)])
def test_matvec_fmm_vs_dense(F, cfg1_dense, leaf_max, lds_budget, lane, mfma, fused):
    """FP64 FMM product against the oracle's dense operator: relative L2 <= 1e-6, for octrees of
    depth 2 and 3 (so M2M/L2L are exercised), with the whole-vector LDS tiles, the per-degree
    kernels (small LDS budget), the one-job-per-lane kernels (lane=2 forces them), the
    matrix-core tiles (mfma=2 puts every lane batch on them) and the fused LDS-resident tiles
    (fused=1, every lane batch with p_src = p_tgt <= 16)."""
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k, leaf_max=leaf_max, lds_budget=lds_budget, lane_tiles=lane, mfma=mfma, fused=fused)
    if fused:
        assert any(s["mfma"] in (2, 4) for s in ctx.fmmbem_batch_shapes())
    info = ctx.fmmbem_get_info()
    L, M = bem.dense_LM(room.vertices, room.triangles, k, oracle_rc(ctx, room))
    for seed in (1, 2):
        x = synth.complex_normal(room.n, seed)
        ref = 0.5 * x + M @ x - 1j * k * L @ (room.beta * x)
        y = ctx.fmmbem_matvec(x)[0]
        err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        print(f"depth {info.depth} p {list(info.p)[:info.depth + 1]} err {err:.3e}")
        assert err < 1e-6
    ctx.close()


@pytest.mark.parametrize("leaf_max,lds_budget,lane,mfma,fused", [
    (64, 0, 0, 0, 0), (12, 0, 0, 0, 0), (12, 8192, 0, 0, 0), (12, 0, 2, 0, 0), (12, 0, 2, 2, 0), (12, 0, 2, 0, 1)])
def test_matvec_mixed_vs_dense(F, cfg1_dense, leaf_max, lds_budget, lane, mfma, fused):
    """Mixed-precision product (FP32 near field and translations, FP64 tables converted once,
    FP64 densities, P2M and L2P) against the oracle's dense operator: relative L2 <= 1e-4, with
    the LDS tiles, the one-job-per-lane kernels, the FP32 matrix-core tiles and the fused tiles."""
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k, leaf_max=leaf_max, lds_budget=lds_budget, lane_tiles=lane, mfma=mfma, fused=fused)
    info = ctx.fmmbem_get_info()
    L, M = bem.dense_LM(room.vertices, room.triangles, k, oracle_rc(ctx, room))
    for seed in (1, 2):
        x = synth.complex_normal(room.n, seed)
        ref = 0.5 * x + M @ x - 1j * k * L @ (room.beta * x)
        y = ctx.fmmbem_matvec(x, precision=F.FMMBEM_MIXED)[0]
        err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        print(f"mixed depth {info.depth} err {err:.3e}")
        assert err < 1e-4
    # the FP64 product is unaffected by a mixed one before it
    y64 = ctx.fmmbem_matvec(x)[0]
    assert np.linalg.norm(y64 - ref) / np.linalg.norm(ref) < 1e-6
    with pytest.raises(RuntimeError):
        ctx.fmmbem_matvec(x, precision=F.FMMBEM_MIXED, exact_far=True)
    ctx.close()


@pytest.mark.parametrize("kk,leaf_max,p_min,p_leaf", [(None, 12, 20, 20), (16.0, 64, 16, 22)])
def test_matvec_large_leaf_p_vs_dense(F, cfg1_dense, kk, leaf_max, p_min, p_leaf):
    """Leaf truncation above 16: p = 20 takes the slot-sum P2M with more coefficients than threads;
    at k = 16 (leaf kd = 12) the truncation rule itself gives p >= 22 at the leaves, more basis
    slots than threads, and the per-coefficient P2M.  (A p far above what kd needs is not a valid
    test: the singular translation coefficients then amplify round-off, which is why the rule never
    raises p beyond need.)  1 and 4 vectors against the oracle's dense operator (1e-6)."""
    room, k = cfg1_dense
    if kk is not None:
        k = kk
    ctx = make_ctx(F, room, k, leaf_max=leaf_max, p_min=p_min)
    info = ctx.fmmbem_get_info()
    assert info.p[info.depth] >= p_leaf
    L, M = bem.dense_LM(room.vertices, room.triangles, k, oracle_rc(ctx, room))
    X = np.stack([synth.complex_normal(room.n, 60 + s) for s in range(4)])
    Y = ctx.fmmbem_matvec(X)
    y1 = ctx.fmmbem_matvec(X[0])[0]
    for s in range(4):
        ref = 0.5 * X[s] + M @ X[s] - 1j * k * L @ (room.beta * X[s])
        err = np.linalg.norm(Y[s] - ref) / np.linalg.norm(ref)
        print(f"k {k:.2f} depth {info.depth} p {list(info.p)[:info.depth + 1]} vector {s}: {err:.2e}")
        assert err < 1e-6
    assert np.linalg.norm(Y[0] - y1) <= 1e-12 * np.linalg.norm(y1)
    ctx.close()


def test_solve_mixed_inner_vs_oracle_lu(F, cfg1_dense):
    """FGMRES with mixed-precision Krylov products and FP64 restart residuals reaches a 1e-8
    FP64 residual; the solution agrees with the oracle's LU solution."""
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k)
    rs, _ = synth.source_and_receivers(room, 4)
    ctx.fmmbem_set_sources(rs)
    x, rep, rc_ = ctx.fmmbem_solve(0, tol=1e-8, restart=40, maxit=400, precision=F.FMMBEM_MIXED)
    print(f"mixed-inner solve: iters {rep.iters} restarts {rep.restarts} rel {rep.rel_res:.2e}")
    assert rc_ == 0 and rep.rel_res < 1e-8
    rc = oracle_rc(ctx, room)
    A, b, _, _ = bem.direct_system(room.vertices, room.triangles, k, room.beta, rs[0], rc)
    x_ref = bem.solve_lu(A, b)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-5
    ctx.close()


@pytest.mark.parametrize("batched", [False, True])
def test_solve_fp32_basis_vs_fp64_basis(F, cfg1_dense, batched):
    """Mixed-precision solves with the Krylov vectors stored in FP32 (the default for mixed
    products) and in FP64: both reach the FP64 residual target within a few iterations of each
    other, and both solutions agree with the oracle's LU solution."""
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k)
    rs, _ = synth.source_and_receivers(room, 4, nsrc=2)
    ctx.fmmbem_set_sources(rs)
    rc = oracle_rc(ctx, room)
    A, b, _, _ = bem.direct_system(room.vertices, room.triangles, k, room.beta, rs[1], rc)
    x_ref = bem.solve_lu(A, b)
    its = {}
    for b32 in (0, 1):
        kw = dict(tol=1e-6, restart=200, maxit=200, precision=F.FMMBEM_MIXED, basis_fp32=b32)
        if batched:
            X, reps, rc_ = ctx.fmmbem_solve_batch([0, 1], **kw)
            x, rep = X[1], reps[1]
        else:
            x, rep, rc_ = ctx.fmmbem_solve(1, **kw)
        print(f"basis fp32={b32} batched={batched}: iters {rep.iters} rel {rep.rel_res:.2e}")
        assert rc_ == 0 and rep.rel_res < 1e-6
        assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-4
        its[b32] = rep.iters
    assert abs(its[1] - its[0]) <= max(3, its[0] // 10), its
    ctx.close()


def test_solve_inner_outer_vs_oracle_lu(F, cfg1_dense):
    """Flexible GMRES preconditioned by an inner mixed-precision GMRES (Section 4.3): converges
    to the FP64 residual target, agrees with LU, and counts its products by arithmetic."""
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k)
    rs, _ = synth.source_and_receivers(room, 4)
    ctx.fmmbem_set_sources(rs)
    x, rep, rc_ = ctx.fmmbem_solve(0, tol=1e-8, restart=20, maxit=60, inner_iters=8, inner_tol=1e-3,
                                   precision=F.FMMBEM_FP64)
    hist = ctx.fmmbem_solve_history()
    print(f"inner-outer: outer {rep.iters} inner {rep.inner_iters} fp64 {rep.matvecs_fp64} "
          f"mixed {rep.matvecs_mixed} rel {rep.rel_res:.2e}")
    assert rc_ == 0 and rep.rel_res < 1e-8
    assert len(hist) == rep.iters and rep.matvecs_mixed == rep.inner_iters > 0
    assert rep.matvecs_fp64 == rep.iters + rep.restarts
    rc = oracle_rc(ctx, room)
    A, b, _, _ = bem.direct_system(room.vertices, room.triangles, k, room.beta, rs[0], rc)
    x_ref = bem.solve_lu(A, b)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-5
    ctx.close()


@pytest.mark.parametrize("leaf_max,lds_budget,lane,mfma,fused", [
    (12, 0, 0, 0, 0), (12, 8192, 0, 0, 0), (64, 0, 0, 0, 0), (12, 0, 2, 0, 0), (12, 0, 2, 2, 0), (12, 0, 2, 0, 1)])
def test_matvec_multi_rhs(F, cfg1_dense, leaf_max, lds_budget, lane, mfma, fused):
    """Seven vectors in one call (chunks of 4, 2 and 1 vectors sharing kernel evaluations,
    basis functions and translation tables) give the single-vector products and match the
    oracle's dense operator (FP64 <= 1e-6, mixed <= 1e-4)."""
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k, leaf_max=leaf_max, lds_budget=lds_budget, lane_tiles=lane, mfma=mfma, fused=fused)
    info = ctx.fmmbem_get_info()
    L, M = bem.dense_LM(room.vertices, room.triangles, k, oracle_rc(ctx, room))
    X = np.stack([synth.complex_normal(room.n, 20 + s) for s in range(7)])
    for prec, tol_single, tol_oracle in ((F.FMMBEM_FP64, 1e-12, 1e-6), (F.FMMBEM_MIXED, 1e-6, 1e-4)):
        Y = ctx.fmmbem_matvec(X, precision=prec)
        for s in range(7):
            y1 = ctx.fmmbem_matvec(X[s], precision=prec)[0]
            assert np.linalg.norm(Y[s] - y1) / np.linalg.norm(y1) < tol_single
            ref = 0.5 * X[s] + M @ X[s] - 1j * k * L @ (room.beta * X[s])
            assert np.linalg.norm(Y[s] - ref) / np.linalg.norm(ref) < tol_oracle
    # all-pairs product with several vectors
    Ye = ctx.fmmbem_matvec(X[:4], exact_far=True)
    for s in range(4):
        ref = 0.5 * X[s] + M @ X[s] - 1j * k * L @ (room.beta * X[s])
        assert np.linalg.norm(Ye[s] - ref) / np.linalg.norm(ref) < 1e-12
    ctx.close()


def test_solve_batch_vs_single_and_lu(F, cfg1_dense):
    """Three sources solved in lock step with batched products: each solution equals its own
    single-source solve and the oracle's LU solution."""
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k)
    rs, _ = synth.source_and_receivers(room, 4, nsrc=3)
    ctx.fmmbem_set_sources(rs)
    srcs = [0, 1, 2]
    Xb, reps, rc_ = ctx.fmmbem_solve_batch(srcs, tol=1e-8, restart=40, maxit=300)
    assert rc_ == 0
    rc = oracle_rc(ctx, room)
    for s in srcs:
        assert reps[s].status == 0 and reps[s].rel_res < 1e-8
        x1, rep1, rc1 = ctx.fmmbem_solve(s, tol=1e-8, restart=40, maxit=300)
        assert rc1 == 0
        assert np.linalg.norm(Xb[s] - x1) / np.linalg.norm(x1) < 1e-6
        A, b, _, _ = bem.direct_system(room.vertices, room.triangles, k, room.beta, rs[s], rc)
        x_ref = bem.solve_lu(A, b)
        assert np.linalg.norm(Xb[s] - x_ref) / np.linalg.norm(x_ref) < 1e-5
    ctx.close()


@pytest.mark.parametrize("nr,prec", [(1, 0), (4, 0), (1, 1), (3, 1)])
def test_matvec_graph_replays_match_eager(F, cfg1_dense, nr, prec):
    """Products on device vectors replay a captured HIP graph; every replay, with eager
    products, other graphs and synchronisations in between, equals the eager product."""
    import torch
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k, leaf_max=12)
    X = np.stack([synth.complex_normal(room.n, 40 + s) for s in range(nr)])
    ref = ctx.fmmbem_matvec(X, precision=prec)  # eager (host entry point)
    dev = torch.device("cuda:0")
    xd = torch.from_numpy(X).to(dev)
    yd = torch.empty_like(xd)
    other = torch.from_numpy(np.stack([synth.complex_normal(room.n, 90)] * 2)).to(dev)
    oy = torch.empty_like(other)
    for rep in range(4):
        yd.zero_()
        ctx.fmmbem_matvec_dev(xd.data_ptr(), yd.data_ptr(), nrhs=nr, precision=prec)
        torch.cuda.synchronize()
        y = yd.cpu().numpy()
        err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        assert err < 1e-13, (rep, err)
        # unrelated work between replays: an eager product and a graph of another shape
        ctx.fmmbem_matvec(X[:1], precision=prec)
        ctx.fmmbem_matvec_dev(other.data_ptr(), oy.data_ptr(), nrhs=2, precision=1 - prec)
        torch.cuda.synchronize()
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("graphs", [0, 1])
def test_matvec_dev_orders_the_callers_stream(F, cfg1_dense, prec, graphs):
    """fmmbem_matvec_dev on a side stream: work enqueued afterwards on that same stream sees the
    finished product (output first filled with NaN, consumed on the stream with no device-wide
    synchronisation), eager and graph-replayed, equal to the host entry point's product."""
    import torch
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k, leaf_max=12, graphs=graphs)
    X = np.stack([synth.complex_normal(room.n, 50 + s) for s in range(2)])
    ref = ctx.fmmbem_matvec(X, precision=prec)
    st = torch.cuda.Stream()
    xd = torch.from_numpy(X).to("cuda")
    torch.cuda.synchronize()
    for rep in range(3):
        with torch.cuda.stream(st):
            yd = torch.full_like(xd, complex("nan+nanj"))
            ctx.fmmbem_matvec_dev(xd.data_ptr(), yd.data_ptr(), nrhs=2, precision=prec, stream=st.cuda_stream)
            z = yd * 1.0  # consumer on the caller's stream
            zh = torch.empty(z.shape, dtype=z.dtype, pin_memory=True)
            zh.copy_(z, non_blocking=True)
        st.synchronize()
        got = zh.numpy()
        assert np.isfinite(got).all(), rep
        assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref), rep
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_two_streams_match_one_stream(F, prec):
    """The product on two streams (near field and upper levels beside the leaf levels) adds every
    contribution in the same order as on one stream: bitwise equal results, eager and replayed
    from a captured graph, for 1 and 4 vectors (6x5x3 m room at 1 kHz, octree depth >= 5, so
    M2L runs on both streams)."""
    import torch
    room, k = synth.config_room(2)
    ctx1 = make_ctx(F, room, k, streams=1)
    ctx2 = make_ctx(F, room, k, streams=2)
    X = np.stack([synth.complex_normal(room.n, 70 + s) for s in range(4)])
    for nr in (1, 4):
        y1 = ctx1.fmmbem_matvec(X[:nr], precision=prec)
        y2 = ctx2.fmmbem_matvec(X[:nr], precision=prec)
        depth = ctx2.fmmbem_get_info().depth
        print("depth", depth)
        assert depth >= 5  # M2L on both streams, L2L on the side one waiting for the main one
        assert np.array_equal(y1, y2), nr
        dev = torch.device("cuda:0")
        xd = torch.from_numpy(X[:nr]).to(dev)
        for _ in range(3):
            yd = torch.zeros_like(xd)
            ctx2.fmmbem_matvec_dev(xd.data_ptr(), yd.data_ptr(), nrhs=nr, precision=prec)
            torch.cuda.synchronize()
            assert np.array_equal(yd.cpu().numpy().reshape(y1.shape), y1), nr
    ctx1.close()
    ctx2.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_fused_tiles_match_lane_tiles(F, prec):
    """The fused LDS-resident translation tiles against the three-pass lane kernels on the 6x5x3 m
    room at 1 kHz (depth >= 5, runs of several jobs per target at the leaf levels), for 1, 2 and 4
    vectors: FP64 products agree to rounding (1e-12), mixed ones to FP32 rounding (1e-5)."""
    room, k = synth.config_room(2)
    ctx0 = make_ctx(F, room, k, lane_tiles=2, mfma=0, fused=0)
    ctx1 = make_ctx(F, room, k, lane_tiles=2, mfma=0, fused=1)
    # the LDS-resident kernel also where the fixed rule picks the register-resident one (p = 16)
    ctx1.fmmbem_set_batch_shapes([dict(d, mfma=2) for d in ctx1.fmmbem_batch_shapes() if d["mfma"] == 4])
    sh = ctx1.fmmbem_batch_shapes()
    print("fused batches:", [(s["level"], s["kind"], s["jobs"]) for s in sh if s["mfma"] == 2])
    assert sum(s["mfma"] == 2 for s in sh) >= 3
    X = np.stack([synth.complex_normal(room.n, 90 + s) for s in range(4)])
    tol = 1e-12 if prec == 0 else 1e-5
    for nr in (1, 2, 4):
        y0 = ctx0.fmmbem_matvec(X[:nr], precision=prec)
        y1 = ctx1.fmmbem_matvec(X[:nr], precision=prec)
        for s in range(nr):
            err = np.linalg.norm(y1[s] - y0[s]) / np.linalg.norm(y0[s])
            print(f"prec {prec} nr {nr} vector {s}: {err:.2e}")
            assert err < tol
    ctx0.close()
    ctx1.close()


@pytest.mark.parametrize("mode", [3, 4])
def test_register_resident_tiles_vs_lane_tiles_and_oracle(F, mode):
    """The fused p = 16 translation tiles (mode 3: each wavefront's 8 jobs' vectors in its
    registers; mode 4: 8 jobs' vectors in LDS shared by four wavefronts) against the three-pass lane
    kernels on the 6x5x3 m room at 1 kHz: FP64 products of one vector agree to rounding (1e-12) and
    with the oracle's rows (1e-6);
    products of 2 and 4 vectors agree with the lane kernels to 1e-12 (mode 3 runs the LDS-resident
    fused kernel for them; mode 4 runs itself, one workgroup per vector, so that each vector of a
    batched product, FP64 or mixed, equals its product alone); a mixed product of one vector
    runs the FP32 register-resident shape (vectors in LDS): FP32 rounding against the lane kernels,
    1e-4 against the oracle's rows."""
    room, k = synth.config_room(2)
    ctx_l = make_ctx(F, room, k, lane_tiles=2, mfma=0, fused=0)
    ctx_r = make_ctx(F, room, k, lane_tiles=2, mfma=0, fused=1)
    shapes = ctx_r.fmmbem_batch_shapes()
    regs = [d for d in shapes if d["mfma"] == 4]
    print("register-resident batches:", [(d["level"], d["kind"], d["jobs"]) for d in regs])
    assert len(regs) >= 3
    if mode == 3:
        ctx_r.fmmbem_set_batch_shapes([dict(d, mfma=3) for d in regs])
        assert sum(d["mfma"] == 3 for d in ctx_r.fmmbem_batch_shapes()) == len(regs)
    X = np.stack([synth.complex_normal(room.n, 120 + s) for s in range(4)])
    y_l = ctx_l.fmmbem_matvec(X[0])[0]
    y_r = ctx_r.fmmbem_matvec(X[0])[0]
    err = np.linalg.norm(y_r - y_l) / np.linalg.norm(y_l)
    print(f"mode {mode}: one vector vs lane kernels {err:.2e}")
    assert err < 1e-12
    rows = np.random.default_rng(9).choice(room.n, 256, replace=False)
    ref = bem.direct_matvec_rows(room.vertices, room.triangles, k, room.beta, oracle_rc(ctx_r, room), X[0], rows)
    assert np.linalg.norm(y_r[rows] - ref) / np.linalg.norm(ref) < 1e-6
    for nr in (2, 4):
        Yl, Yr = ctx_l.fmmbem_matvec(X[:nr]), ctx_r.fmmbem_matvec(X[:nr])
        assert np.linalg.norm(Yr - Yl) / np.linalg.norm(Yl) < 1e-12, nr
    if mode == 4:
        for prec, tol in ((F.FMMBEM_FP64, 1e-15), (F.FMMBEM_MIXED, 1e-7)):
            Y4 = ctx_r.fmmbem_matvec(X, precision=prec)
            for s in range(4):
                y1 = ctx_r.fmmbem_matvec(X[s], precision=prec)[0]
                d = np.linalg.norm(Y4[s] - y1) / np.linalg.norm(y1)
                print(f"mode 4 precision {prec}: vector {s} of 4 vs alone {d:.1e}")
                assert d <= tol, (prec, s)
    # mixed products of one vector: the FP32 kernel with the vectors in LDS (k_tq_lds)
    ym_l = ctx_l.fmmbem_matvec(X[0], precision=F.FMMBEM_MIXED)[0]
    ym_r = ctx_r.fmmbem_matvec(X[0], precision=F.FMMBEM_MIXED)[0]
    errm = np.linalg.norm(ym_r - ym_l) / np.linalg.norm(ym_l)
    print(f"mode {mode}: mixed product vs lane kernels {errm:.2e}")
    assert errm < 1e-5
    assert np.linalg.norm(ym_r[rows] - ref) / np.linalg.norm(ref) < 1e-4
    # a register-resident shape where p != 16 is rejected
    bad = [dict(d, mfma=3) for d in shapes if d["lane"] and d["mfma"] != 4][:1]
    if bad:
        with pytest.raises(F.FmmbemError):
            ctx_r.fmmbem_set_batch_shapes(bad)
    ctx_l.close()
    ctx_r.close()


def test_matrix_core_tiles_of_32_jobs_vs_64(F):
    """Matrix-core translation tiles of 32 jobs (classes padded to 32, each wavefront one 16-column
    block) against the 64-job tiles on the 6x5x3 m room at 1 kHz with every batch on one-job-per-lane
    tiles and matrix cores: products of 1, 2 and 4 vectors agree to rounding (1e-12), mixed products
    to FP32 rounding (1e-5), and the 32-job product matches the oracle's rows (1e-6)."""
    room, k = synth.config_room(2)
    ctx64 = make_ctx(F, room, k, lane_tiles=2, mfma=2, fused=0)
    ctx32 = make_ctx(F, room, k, lane_tiles=2, mfma=2, fused=0)
    shapes = ctx32.fmmbem_batch_shapes()
    tm = [d for d in shapes if d["lane"] and d["mfma"] == 1]
    assert len(tm) >= 6
    ctx64.fmmbem_set_batch_shapes([dict(d, jt=64) for d in tm])
    assert sum(d["jt"] == 64 for d in ctx64.fmmbem_batch_shapes() if d["lane"] and d["mfma"] == 1) == len(tm)
    ctx32.fmmbem_set_batch_shapes([dict(d, jt=32) for d in tm])
    got = ctx32.fmmbem_batch_shapes()
    assert sum(d["jt"] == 32 for d in got) == len(tm)
    X = np.stack([synth.complex_normal(room.n, 130 + s) for s in range(4)])
    for nr in (1, 2, 4):
        Y64, Y32 = ctx64.fmmbem_matvec(X[:nr]), ctx32.fmmbem_matvec(X[:nr])
        err = np.linalg.norm(Y32 - Y64) / np.linalg.norm(Y64)
        print(f"{nr} vectors: 32-job vs 64-job tiles {err:.2e}")
        assert err < 1e-12, nr
    y = ctx32.fmmbem_matvec(X[0])[0]
    rows = np.random.default_rng(10).choice(room.n, 256, replace=False)
    ref = bem.direct_matvec_rows(room.vertices, room.triangles, k, room.beta, oracle_rc(ctx32, room), X[0], rows)
    assert np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref) < 1e-6
    ym64 = ctx64.fmmbem_matvec(X[0], precision=F.FMMBEM_MIXED)[0]
    ym32 = ctx32.fmmbem_matvec(X[0], precision=F.FMMBEM_MIXED)[0]
    assert np.linalg.norm(ym32 - ym64) / np.linalg.norm(ym64) < 1e-5
    # 32-job tiles exist only on matrix cores
    with pytest.raises(F.FmmbemError):
        ctx32.fmmbem_set_batch_shapes([dict(tm[0], jt=32, mfma=0)])
    ctx64.close()
    ctx32.close()


def test_mixed_products_run_lane_batches_fused(F):
    """With `fused` on, mixed products run every lane batch that may use the fused tiles fused, even
    where its shape is the three-pass lane kernels (as the FP64 autotuner may choose): lane shapes
    replayed onto those batches give the fused context's mixed product bitwise, agree with the
    all-lane mixed product to FP32 rounding (1e-5), and leave the FP64 product on the lane kernels
    (bitwise the all-lane FP64 product)."""
    room, k = synth.config_room(2)
    ctx_l = make_ctx(F, room, k, lane_tiles=2, mfma=0, fused=0)
    ctx_f = make_ctx(F, room, k, lane_tiles=2, mfma=0, fused=1)
    ctx_r = make_ctx(F, room, k, lane_tiles=2, mfma=0, fused=1)
    shapes = ctx_f.fmmbem_batch_shapes()
    assert sum(d["mfma"] >= 2 for d in shapes) >= 3
    ctx_r.fmmbem_set_batch_shapes([dict(d, mfma=0) if d["mfma"] >= 2 else d for d in shapes])
    assert all(d["mfma"] < 2 for d in ctx_r.fmmbem_batch_shapes())
    x = synth.complex_normal(room.n, 43)
    y_l, y_f, y_r = (c.fmmbem_matvec(x, precision=F.FMMBEM_MIXED)[0] for c in (ctx_l, ctx_f, ctx_r))
    assert np.array_equal(y_r, y_f)
    assert np.linalg.norm(y_r - y_l) / np.linalg.norm(y_l) < 1e-5
    assert np.array_equal(ctx_r.fmmbem_matvec(x)[0], ctx_l.fmmbem_matvec(x)[0])
    for c in (ctx_l, ctx_f, ctx_r):
        c.close()


def test_replayed_tile_shapes_match_autotuned(F):
    """Tile shapes recorded from an autotuned context and replayed on a fixed-rule one give the
    same launches and bitwise the same products (FP64 and mixed); a shape that does not fit its
    batch is rejected and changes nothing."""
    room, k = synth.config_room(2)
    ctx_a = make_ctx(F, room, k, autotune=1)
    ctx_r = make_ctx(F, room, k, autotune=0)
    shapes = ctx_a.fmmbem_batch_shapes()
    ctx_r.fmmbem_set_batch_shapes(shapes)
    got = ctx_r.fmmbem_batch_shapes()
    key = lambda d: (d["level"], d["kind"], d["lane"], d["whole"], d["jt"], d["mfma"])
    assert [key(d) for d in got] == [key(d) for d in shapes]
    x = synth.complex_normal(room.n, 41)
    for prec in (0, 1):
        assert np.array_equal(ctx_a.fmmbem_matvec(x, precision=prec), ctx_r.fmmbem_matvec(x, precision=prec))
    bad = dict(shapes[0], lane=1, jt=48, whole=0, mfma=0)
    with pytest.raises(RuntimeError):
        ctx_r.fmmbem_set_batch_shapes([bad])
    assert [key(d) for d in ctx_r.fmmbem_batch_shapes()] == [key(d) for d in shapes]
    ctx_a.close()
    ctx_r.close()


def test_autotuned_tiles_vs_dense(F, cfg1_dense):
    """With autotuning, every batch gets the measured-fastest tile shape; the product (FP64,
    mixed, several vectors) still matches the oracle's dense operator."""
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k, leaf_max=12, autotune=1)
    shapes = ctx.fmmbem_batch_shapes()
    print("tile shapes:", [(s["level"], s["kind"], s["lane"], s["whole"], s["jt"], round(s["ms"], 3)) for s in shapes])
    assert len(shapes) > 0 and all(s["ms"] > 0 for s in shapes)
    info = ctx.fmmbem_get_info()
    L, M = bem.dense_LM(room.vertices, room.triangles, k, oracle_rc(ctx, room))
    X = np.stack([synth.complex_normal(room.n, 60 + s) for s in range(3)])
    ref = np.stack([0.5 * x + M @ x - 1j * k * L @ (room.beta * x) for x in X])
    for prec, tol in ((F.FMMBEM_FP64, 1e-6), (F.FMMBEM_MIXED, 1e-4)):
        Y = ctx.fmmbem_matvec(X, precision=prec)
        for s in range(3):
            assert np.linalg.norm(Y[s] - ref[s]) / np.linalg.norm(ref[s]) < tol
    ctx.close()


def test_rhs_vs_oracle(F, cfg1_dense):
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k)
    rs, _ = synth.source_and_receivers(room, 4)
    ctx.fmmbem_set_sources(rs)
    b = ctx.fmmbem_rhs()[0]
    rc = oracle_rc(ctx, room)
    rows = np.arange(0, room.n, 5)
    ref = bem.direct_rhs_rows(room.vertices, room.triangles, k, room.beta, rs[0], rc, rows)
    assert np.linalg.norm(b[rows] - ref) / np.linalg.norm(ref) < 1e-6
    ctx.close()


def test_solve_and_field_vs_oracle_lu(F, cfg1_dense):
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k)
    rs, rec = synth.source_and_receivers(room, 16)
    ctx.fmmbem_set_sources(rs)
    x, rep, rc_ = ctx.fmmbem_solve(0, tol=1e-9, restart=40, maxit=300)
    assert rc_ == 0 and rep.rel_res < 1e-9
    rc = oracle_rc(ctx, room)
    A, b, _, _ = bem.direct_system(room.vertices, room.triangles, k, room.beta, rs[0], rc)
    x_ref = bem.solve_lu(A, b)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-5
    psi = ctx.fmmbem_eval_field(0, rec, x)
    psi_ref = bem.direct_receivers(room.vertices, room.triangles, k, room.beta, rs[0], rc, x, rec)
    assert np.linalg.norm(psi - psi_ref) / np.linalg.norm(psi_ref) < 1e-10
    ctx.close()


def test_field_many_points_tiled_vs_per_point_and_oracle(F, cfg1_dense):
    """Fields at 6,400 points, enough for the tiled field kernel (8 points per workgroup sharing
    element tiles in LDS), 256 of them 2 cm off element centroids where the near integrals apply:
    equal to the one-workgroup-per-point kernel (the same points in two calls of 3,200) to 1e-13,
    and the points at least 0.3 m from the walls equal to the oracle's Green representation
    (Eq. dbem1) to 1e-10."""
    room, k = cfg1_dense
    ctx = make_ctx(F, room, k)
    rs, rec = synth.source_and_receivers(room, 6144)
    ctx.fmmbem_set_sources(rs)
    V, T = room.vertices, room.triangles
    c = V[T].mean(axis=1)
    nrm = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    sel = np.random.default_rng(12).choice(room.n, 256, replace=room.n < 256)
    pts = np.ascontiguousarray(np.vstack([c[sel] + 0.02 * nrm[sel], rec]))
    x = synth.complex_normal(room.n, 77)
    psi = ctx.fmmbem_eval_field(0, pts, x)
    assert np.isfinite(psi).all()
    part = np.concatenate([ctx.fmmbem_eval_field(0, pts[:3200], x), ctx.fmmbem_eval_field(0, pts[3200:], x)])
    d = np.linalg.norm(psi - part) / np.linalg.norm(part)
    print(f"tiled vs per-point kernel: {d:.2e}")
    assert d < 1e-13
    dn = np.linalg.norm(psi[:256] - part[:256]) / np.linalg.norm(part[:256])
    assert dn < 1e-13
    ref = bem.direct_receivers(V, T, k, room.beta, rs[0], oracle_rc(ctx, room), x, pts[256:])
    err = np.linalg.norm(psi[256:] - ref) / np.linalg.norm(ref)
    print(f"tiled kernel vs oracle: {err:.2e}")
    assert err < 1e-10
    ctx.close()


@pytest.mark.parametrize("cfg,nrows", [(2, 1024), (3, 1024)])
def test_matvec_fmm_sampled_rows_full_size(F, cfg, nrows):
    """Full-size rooms (N = 90,972 at 1 kHz; N = 1,009,576 at 2.5 kHz): the FMM product on seeded
    rows against the oracle's matrix-free rows, relative L2 <= 1e-6 in FP64 and <= 1e-4 mixed."""
    room, k = synth.config_room(cfg)
    ctx = make_ctx(F, room, k)
    info = ctx.fmmbem_get_info()
    x = synth.complex_normal(room.n, 11)
    y = ctx.fmmbem_matvec(x)[0]
    rows = np.random.default_rng(5).choice(room.n, nrows, replace=False)
    ref = bem.direct_matvec_rows(room.vertices, room.triangles, k, room.beta, oracle_rc(ctx, room), x, rows)
    err = np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref)
    ym = ctx.fmmbem_matvec(x, precision=F.FMMBEM_MIXED)[0]
    err_m = np.linalg.norm(ym[rows] - ref) / np.linalg.norm(ref)
    print(f"cfg {cfg} N {room.n} depth {info.depth} p {list(info.p)[:info.depth + 1]} err {err:.3e} "
          f"mixed {err_m:.3e}")
    assert err < 1e-6
    assert err_m < 1e-4
    ctx.close()


def test_matvec_sampled_rows_6M_5khz(F):
    """The L-room at 5 kHz meshed at 0.779 cm (N = 6,032,304; k D > 1,100; octree depth 8, p = 255 at
    the top level): FP64 and mixed products on 256 seeded rows against the oracle's rows of Eq.
    dbem4 (FP64 <= 1e-6, mixed <= 1e-4), fixed-rule tile shapes."""
    room, k = synth.config_room(5)
    assert room.n > 6_000_000
    ctx = make_ctx(F, room, k, autotune=0)
    info = ctx.fmmbem_get_info()
    print(f"N {room.n} depth {info.depth} p {list(info.p)[:info.depth + 1]}")
    assert info.p[2] >= 250
    x = synth.complex_normal(room.n, 11)
    rows = np.random.default_rng(7).choice(room.n, 256, replace=False)
    ref = bem.direct_matvec_rows(room.vertices, room.triangles, k, room.beta, oracle_rc(ctx, room), x, rows)
    for prec, tol in ((F.FMMBEM_FP64, 1e-6), (F.FMMBEM_MIXED, 1e-4)):
        y = ctx.fmmbem_matvec(x, precision=prec)[0]
        assert np.isfinite(y).all()
        err = np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref)
        print(f"precision {prec}: sampled rows rel L2 {err:.3e}")
        assert err < tol
    ctx.close()


def test_matvec_sampled_rows_bench_configuration(F):
    """The 1M L-room in the launch configuration the benchmark times: autotuned context with the
    tile shapes of the committed counter run replayed, products on device vectors (captured-graph
    replays) on a torch stream.  Seeded rows against the oracle's matrix-free rows (FP64 <= 1e-6,
    mixed <= 1e-4); two replays give bitwise the same product."""
    import json
    import os
    import torch
    room, k = synth.config_room(3)
    ctx = make_ctx(F, room, k, autotune=1)
    shapes = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                          "tile_shapes_lroom_1M_fp64.json")
    if os.path.exists(shapes):
        with open(shapes) as fh:
            ctx.fmmbem_set_batch_shapes(json.load(fh))
    info = ctx.fmmbem_get_info()
    x = synth.complex_normal(room.n, 11)
    rows = np.random.default_rng(5).choice(room.n, 1024, replace=False)
    ref = bem.direct_matvec_rows(room.vertices, room.triangles, k, room.beta, oracle_rc(ctx, room), x, rows)
    st = torch.cuda.Stream()
    xd = torch.from_numpy(x).to("cuda")
    yd = torch.empty_like(xd)
    torch.cuda.synchronize()
    for prec, tol in ((F.FMMBEM_FP64, 1e-6), (F.FMMBEM_MIXED, 1e-4)):
        ys = []
        for _ in range(2):
            ctx.fmmbem_matvec_dev(xd.data_ptr(), yd.data_ptr(), 1, precision=prec, stream=st.cuda_stream)
            st.synchronize()
            ys.append(yd.cpu().numpy())
        assert np.array_equal(ys[0], ys[1])
        err = np.linalg.norm(ys[0][rows] - ref) / np.linalg.norm(ref)
        print(f"precision {prec}: sampled rows rel L2 {err:.3e}")
        assert err < tol
    ctx.close()


def test_solve_many_frequencies_vs_single_solves(F):
    """Several frequencies of one room, each with its own mesh (about six elements per wavelength,
    so N and the octree differ) and two sources each, solved together from one thread by
    fmmbem_solve_many: every solution equals the lock-step batched solve of its context bitwise,
    agrees with fmmbem_solve one system at a time (1e-8) and, on the smallest room, with the oracle's
    LU solution; more than one host thread and mismatched options within a context are rejected."""
    import time
    fr = [150.0, 200.0, 250.0, 300.0]
    ctxs, rooms = [], []
    for f in fr:
        room = synth.shoebox(3.0, 2.5, 2.0, synth.SOUND_SPEED / (6.0 * f))
        rs, _ = synth.source_and_receivers(room, 2, nsrc=2)
        ctx = make_ctx(F, room, synth.wavenumber(f))
        ctx.fmmbem_set_sources(rs)
        ctxs.append(ctx)
        rooms.append((room, rs))
    kw = dict(tol=1e-9, restart=150, maxit=300)
    sys_ctx = [c for c in ctxs for _ in range(2)]
    sys_src = [s for _ in ctxs for s in range(2)]
    t0 = time.perf_counter()
    xs, reps, status, rc = F.fmmbem_solve_many(sys_ctx, sys_src, **kw)
    t_many = time.perf_counter() - t0
    t0 = time.perf_counter()
    batch = [c.fmmbem_solve_batch([0, 1], **kw) for c in ctxs]
    t_batch = time.perf_counter() - t0
    print(f"N {[c.fmmbem_num_unknowns() for c in ctxs]}: solve_many {t_many:.3f} s, batched one context at a "
          f"time {t_batch:.3f} s, iterations {[r.iters for r in reps]}")
    assert rc == 0 and status == [0] * len(sys_ctx)
    for i, (c, s) in enumerate(zip(sys_ctx, sys_src)):
        Xb = batch[i // 2][0]
        assert np.array_equal(xs[i], Xb[s])
        x1, rep1, rc1 = c.fmmbem_solve(s, **kw)
        assert rc1 == 0 and np.linalg.norm(xs[i] - x1) <= 1e-8 * np.linalg.norm(x1)
    room, rs = rooms[0]
    rc0 = oracle_rc(ctxs[0], room)
    A, b, _, _ = bem.direct_system(room.vertices, room.triangles, synth.wavenumber(fr[0]), room.beta, rs[1], rc0)
    x_ref = bem.solve_lu(A, b)
    assert np.linalg.norm(xs[1] - x_ref) / np.linalg.norm(x_ref) < 1e-6
    with pytest.raises(F.FmmbemError):
        F.fmmbem_solve_many(ctxs[:2], [0, 0], threads=4, **kw)
    for c in ctxs:
        c.close()


@pytest.mark.skip(reason="solving from several host threads is not offered: a 16-thread sweep of 16 L-room contexts "
                         "(mixed precision) crashed the process with a host segmentation fault whose cause has not "
                         "been shown on the CPU; fmmbem_solve_many now keeps every system in flight from one thread "
                         "and rejects threads > 1, so this case stays off the GPU")
def test_solve_many_concurrent_threads(F):
    """Sixteen L-room frequencies (N about 2.8k-41k, mixed products) solved from 16 host threads, one
    context per thread through fmmbem_solve, must give bitwise the one-thread solutions."""
    import threading
    fr = [300.0 * 1.12 ** i for i in range(16)]
    ctxs = []
    for f in fr:
        room = synth.lroom(synth.SOUND_SPEED / (6.0 * f))
        rs, _ = synth.source_and_receivers(room, 2)
        ctx = make_ctx(F, room, synth.wavenumber(f))
        ctx.fmmbem_set_sources(rs)
        ctxs.append(ctx)
    kw = dict(tol=1e-4, restart=300, maxit=600, precision=F.FMMBEM_MIXED)
    ref = [c.fmmbem_solve(0, **kw)[0] for c in ctxs]
    out = [None] * len(ctxs)

    def work(i):
        out[i] = ctxs[i].fmmbem_solve(0, **kw)[0]

    th = [threading.Thread(target=work, args=(i,)) for i in range(len(ctxs))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for a, b in zip(ref, out):
        assert np.array_equal(a, b)
    for c in ctxs:
        c.close()


def test_low_frequency_products_follow_k(F):
    """Low frequencies (the 8 x 6 x 3 m room, 20-320 Hz, one mesh): the octree's leaves stay at least
    kd_leaf_min / k wide, so the FMM product matches the oracle's rows of Eq. dbem4 (1e-6, 256 seeded
    rows) where leaves of k d = 0.18 gave an O(1) error; on one context the octree is rebuilt when a
    new wavenumber moves that bound (20 -> 320 -> 20 Hz)."""
    room = synth.shoebox(8.0, 6.0, 3.0, synth.SOUND_SPEED / (6.7 * 320.0))
    beta = np.full(room.n, 1.0 / 9.0)
    ctx = F.Context(0)
    ctx.fmmbem_set_mesh(room.vertices, room.triangles)
    ctx.fmmbem_set_admittance(beta)
    x = synth.complex_normal(room.n, 11)
    rows = np.random.default_rng(14).choice(room.n, 256, replace=False)
    depths = []
    for f in (20.0, 320.0, 20.0, 60.0):
        k = synth.wavenumber(f)
        ctx.fmmbem_set_wavenumber(k)
        info = ctx.fmmbem_get_info()
        depths.append(info.depth)
        leaf = 8.0 * (1 + 1e-6) / 2 ** info.depth
        assert info.depth == 2 or k * leaf >= 0.75
        y = ctx.fmmbem_matvec(x)[0]
        ref = bem.direct_matvec_rows(room.vertices, room.triangles, k, beta, oracle_rc(ctx, room), x, rows)
        err = np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref)
        print(f"{f:5.0f} Hz: depth {info.depth}, FMM vs oracle rows {err:.2e}")
        assert err < 1e-6
    assert depths[0] == depths[2] < depths[1]
    ctx.close()


def test_new_wavenumber_keeps_batches_of_unchanged_levels(F):
    """A new wavenumber on the same mesh keeps the translation batches of every level whose
    truncation numbers did not move (only the coaxial tables and the fused tiles' coaxial fragments
    are rebuilt): products after 1000 -> 1005 Hz (few levels' p move) and 1005 -> 1300 Hz (most
    move) equal, bitwise, those of a context set up at the new frequency from scratch (FP64 and
    mixed)."""
    room, _ = synth.config_room(2)
    x = synth.complex_normal(room.n, 57)
    ctx = make_ctx(F, room, synth.wavenumber(1000.0))
    ctx.fmmbem_matvec(x)
    for f in (1005.0, 1300.0):
        k = synth.wavenumber(f)
        ctx.fmmbem_set_wavenumber(k)
        fresh = make_ctx(F, room, k)
        ps = [ctx.fmmbem_get_info().p[l] for l in range(ctx.fmmbem_get_info().depth + 1)]
        print(f"{f:.0f} Hz: p per level {ps}")
        for prec in (0, 1):
            assert np.array_equal(ctx.fmmbem_matvec(x, precision=prec), fresh.fmmbem_matvec(x, precision=prec)), (f, prec)
        fresh.close()
    ctx.close()
