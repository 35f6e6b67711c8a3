"""Learned preconditioner: device network kernels against the numpy reference, training, the
guard, and the preconditioner ablation on the small shoebox (direct BIE)."""
import numpy as np
import pytest

from mlp_ref import forward as ref_forward, loss_grad as ref_loss_grad
from oracle import bem
from rc_check import oracle_rc
from paper_2103_16073_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    from paper_2103_16073_amd import fmmbem
    return fmmbem


def make_ctx(F, room, k, nsrc=1, **opt):
    ctx = F.Context(0, **opt)
    ctx.fmmbem_set_mesh(room.vertices, room.triangles)
    ctx.fmmbem_set_wavenumber(k)
    ctx.fmmbem_set_admittance(room.beta)
    rs, _ = synth.source_and_receivers(room, 4, nsrc=nsrc)
    ctx.fmmbem_set_sources(rs)
    ctx.fmmbem_setup()
    return ctx, rs


def _batch(m, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, 140)).astype(np.float32), rng.standard_normal((m, 128)).astype(np.float32)


def test_mlp_forward_and_gradient_vs_reference(F):
    """Forward pass and mean-squared-error gradient of the hand-written kernels against the
    numpy reference's explicit backprop (same FP16-rounded weights): relative 1e-3, per layer;
    output-bias gradients against central differences of the device loss."""
    room, k = synth.config_room(1)
    ctx, _ = make_ctx(F, room, k)
    ctx.fmmbem_mlp_init(7)
    w = ctx.fmmbem_mlp_get_weights()
    for m in (1, 63, 200):  # ragged row tiles
        X, T = _batch(m, m)
        Y = ctx.fmmbem_mlp_forward(X)
        Yr = ref_forward(w, X)[-1]
        assert np.linalg.norm(Y - Yr) <= 1e-3 * np.linalg.norm(Yr)
        loss, g = ctx.fmmbem_mlp_loss_grad(X, T)
        lr, gr = ref_loss_grad(w, X, T)
        assert abs(loss - lr) <= 1e-3 * lr
        assert np.linalg.norm(g - gr) <= 1e-3 * np.linalg.norm(gr)
        # every layer's block of the gradient
        off = 0
        for i, o in [(140, 128), (128, 128), (128, 128), (128, 128)]:
            blk = slice(off, off + i * o + o)
            assert np.linalg.norm(g[blk] - gr[blk]) <= 1e-3 * np.linalg.norm(gr[blk]) + 1e-12
            off += i * o + o
    # the loss is exactly quadratic in the output-layer biases (FP32 parameters), so a central
    # difference with a large step is exact there and stays far above the FP32 loss resolution
    X, T = _batch(32, 5)
    _, g = ctx.fmmbem_mlp_loss_grad(X, T)
    bias_idx = [len(w) - 128, len(w) - 128 + 5, len(w) - 64, len(w) - 1]
    h = 0.5
    for idx in bias_idx:
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        ctx.fmmbem_mlp_set_weights(wp)
        lp, _ = ctx.fmmbem_mlp_loss_grad(X, T)
        ctx.fmmbem_mlp_set_weights(wm)
        lm, _ = ctx.fmmbem_mlp_loss_grad(X, T)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-3 * abs(g[idx]) + 1e-5, (idx, fd, g[idx])
    ctx.close()


def test_training_reduces_loss_and_solves(F):
    """Training on the plain solver's residual/error pairs of one source lowers the loss; the
    learned preconditioner then solves another source to the FP64 residual target and agrees
    with the oracle's LU solution."""
    room, k = synth.config_room(1)
    ctx, rs = make_ctx(F, room, k, nsrc=2)
    rep = ctx.fmmbem_learned_train(1, epochs=40, batch=256, max_pairs=12, restart=6, tol=1e-9)
    print(f"train: samples {rep.samples} pairs {rep.pairs} loss zero {rep.loss_zero:.3e} "
          f"first {rep.loss_first:.3e} last {rep.loss_last:.3e} data {rep.t_data_s:.2f}s train {rep.t_train_s:.2f}s")
    assert rep.pairs >= 3 and rep.samples > 0
    assert rep.loss_last < rep.loss_first
    x, srep, rc_ = ctx.fmmbem_solve(0, tol=1e-8, restart=60, maxit=300, precond=F.FMMBEM_PC_LEARNED)
    assert rc_ == 0 and srep.rel_res < 1e-8
    rc = oracle_rc(ctx, room)
    A, b, _, _ = bem.direct_system(room.vertices, room.triangles, k, room.beta, rs[0], rc)
    x_ref = bem.solve_lu(A, b)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-5
    ctx.close()


def test_guard_drops_a_bad_network(F):
    """Weights that make the correction useless are dropped by the guard (fallback recorded) and
    the solve still converges with the near-field block preconditioner."""
    room, k = synth.config_room(1)
    ctx, rs = make_ctx(F, room, k, nsrc=2)
    ctx.fmmbem_learned_train(1, epochs=1, batch=256, restart=6, tol=1e-9)
    w = ctx.fmmbem_mlp_get_weights()
    rng = np.random.default_rng(0)
    ctx.fmmbem_mlp_set_weights((rng.standard_normal(w.size) * 3.0).astype(np.float32))
    x, srep, rc_ = ctx.fmmbem_solve(0, tol=1e-8, restart=60, maxit=300, precond=F.FMMBEM_PC_LEARNED)
    print(f"bad network: fallback at {srep.pc_fallback_at}, iters {srep.iters}")
    assert srep.pc_fallback_at >= 1
    assert rc_ == 0 and srep.rel_res < 1e-8
    ctx.close()


def test_preconditioner_ablation(F):
    """Iterations to 1e-8 (FP64 residual) with each preconditioner on one source; every variant
    converges to the same solution.  Reported, with the learned network trained on a different
    source position."""
    room, k = synth.config_room(1)
    ctx, rs = make_ctx(F, room, k, nsrc=2)
    ctx.fmmbem_learned_train(1, epochs=40, batch=256, restart=6, tol=1e-9)
    res = {}
    xs = {}
    for name, pc in (("none", F.FMMBEM_PC_NONE), ("diag", F.FMMBEM_PC_DIAG), ("nearblock", F.FMMBEM_PC_NEARBLOCK),
                     ("learned", F.FMMBEM_PC_LEARNED)):
        x, srep, rc_ = ctx.fmmbem_solve(0, tol=1e-8, restart=100, maxit=400, precond=pc)
        assert rc_ == 0
        res[name] = (srep.iters, srep.pc_fallback_at)
        xs[name] = x
    print("ablation (iterations, fallback):", res)
    for name in xs:
        assert np.linalg.norm(xs[name] - xs["nearblock"]) / np.linalg.norm(xs["nearblock"]) < 1e-6
    ctx.close()
