"""Impulse responses from frequency sweeps (Section 4.1): the total field at receivers for a set of
equispaced frequencies, each from an FGMRES solve through the C ABI, multiplied by the spectrum of
the pulse of Eq. (an3) and summed back into the time domain.  Host orchestration only: every
solve and field evaluation runs in the library."""
from __future__ import annotations

import numpy as np

from . import fmmbem as F
from .synth import SOUND_SPEED


def transfer_functions(vertices, triangles, beta, rs, receivers, freqs, formulation=None, solve_kw=None,
                       ctx_opts=None):
    """psi(r_q, f_m) (total field, incident included; nf x nr) on one mesh for every frequency."""
    receivers = np.atleast_2d(np.asarray(receivers, float))
    kw = dict(tol=1e-6, restart=300, maxit=600)
    kw.update(solve_kw or {})
    ctx = F.Context(0, **(ctx_opts or {}))
    out = np.zeros((len(freqs), receivers.shape[0]), np.complex128)
    iters = []
    try:
        ctx.fmmbem_set_mesh(vertices, triangles)
        ctx.fmmbem_set_admittance(beta)
        if formulation is not None:
            ctx.fmmbem_set_formulation(formulation)
        ctx.fmmbem_set_sources(np.atleast_2d(np.asarray(rs, float)))
        for m, f in enumerate(freqs):
            ctx.fmmbem_set_wavenumber(2.0 * np.pi * f / SOUND_SPEED)
            x, rep, rc = ctx.fmmbem_solve(0, **kw)
            if rc != 0:
                raise RuntimeError(f"FGMRES did not converge at {f} Hz (code {rc}, relative residual "
                                   f"{rep.rel_res:.2e} after {rep.iters} iterations)")
            iters.append(rep.iters)
            out[m] = ctx.fmmbem_eval_field(0, receivers, x)
    finally:
        ctx.close()
    return out, iters


def an3_spectrum(freqs, dt):
    """Spectrum of f(t) = delta(t - dt) - delta(t + dt) (Eq. an3) for the e^{-i w t} convention:
    F(w) = e^{i w dt} - e^{-i w dt} = 2 i sin(w dt)."""
    w = 2.0 * np.pi * np.asarray(freqs, float)
    return 2j * np.sin(w * dt)


def synthesize(H, freqs, spectrum, times):
    """p(r_q, t_n) = sum_m Re[H(m, q) F(m) e^{-i w_m t_n}] (one-sided sum over the equispaced
    positive frequencies, the same for every solution compared)."""
    w = 2.0 * np.pi * np.asarray(freqs, float)
    E = np.exp(-1j * np.outer(np.asarray(times, float), w))  # nt x nf
    return np.real(E @ (H * np.asarray(spectrum)[:, None]))


def receiver_plane(lx, ly, z, spacing):
    """Receivers on the plane z over the whole floor area [0, lx] x [0, ly]: a grid of the given
    spacing, cell-centred (points at (i + 1/2) spacing), so that no receiver lies on a wall."""
    nx, ny = int(round(lx / spacing)), int(round(ly / spacing))
    xs = (np.arange(nx) + 0.5) * (lx / nx)
    ys = (np.arange(ny) + 0.5) * (ly / ny)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, float(z))], 1), (nx, ny)


def synthesize_fft(H, spectrum, nt):
    """The sum of `synthesize` on the time grid t_n = n T / nt (T = 1 / df), by one inverse real FFT
    per receiver (Section 4.1): H and spectrum hold the equispaced frequencies f_m = m df, m = 1..nf,
    nf <= nt / 2.  Returns nt x nr."""
    H = np.atleast_2d(H)
    nf = H.shape[0]
    if nf > nt // 2:
        raise ValueError("more frequencies than the time grid resolves")
    # p(t_n) = sum_m Re[Z_m e^{-i w_m t_n}] = sum_m Re[conj(Z_m) e^{+2 pi i m n / nt}]; irfft weights
    # the bins 1 .. nt/2 - 1 by 2 / nt and the Nyquist bin by 1 / nt
    Z = np.zeros((nt // 2 + 1, H.shape[1]), np.complex128)
    Z[1:nf + 1] = np.conj(H * np.asarray(spectrum)[:, None])
    if nf == nt // 2:
        Z[nf] *= 2.0
    return np.fft.irfft(Z, n=nt, axis=0) * (nt / 2.0)


def sweep_plane(L, zeta, rs, freqs, receivers, bands, epw=6.7, tol=1e-4, wave_n=1_000_000, log=None):
    """Total field at the receivers for every frequency in `freqs`, the shoebox [0, L] with constant
    impedance zeta on every wall (admittance 1 / zeta) and a monopole at rs.  The frequencies are
    split at the band edges `bands` (ascending upper frequencies); each band has its own mesh, of
    `epw` elements per wavelength at the band's top frequency, and as many contexts on it as fit
    `wave_n` elements, which take the band's frequencies in turn: every round sets one wavenumber
    per context and solves them together (fmmbem_solve_many: mixed-precision products, near-field
    leaf blocks, FP64 residuals), then evaluates each field at the receivers.  Returns H (nf x nr),
    the iterations per frequency and a per-band summary."""
    import time
    from . import synth
    freqs = np.asarray(freqs, float)
    receivers = np.ascontiguousarray(np.atleast_2d(receivers), np.float64)
    H = np.zeros((len(freqs), receivers.shape[0]), np.complex128)
    iters = np.zeros(len(freqs), int)
    summary = []
    lo = 0.0
    for fb in bands:
        idx = [i for i, f in enumerate(freqs) if lo < f <= fb]
        lo = fb
        if not idx:
            continue
        t0 = time.perf_counter()
        room = synth.shoebox(*L, SOUND_SPEED / (epw * fb))
        beta = np.full(room.n, 1.0 / zeta, np.complex128)
        nctx = max(1, min(len(idx), wave_n // max(1, room.n)))
        ctxs = []
        for _ in range(nctx):
            c = F.Context(0, autotune=0)
            c.fmmbem_set_mesh(room.vertices, room.triangles)
            c.fmmbem_set_admittance(beta)
            c.fmmbem_set_sources(np.atleast_2d(np.asarray(rs, float)))
            ctxs.append(c)
        t_setup = t_solve = t_field = 0.0
        try:
            for r0 in range(0, len(idx), nctx):
                rnd = idx[r0:r0 + nctx]
                ts = time.perf_counter()
                for c, i in zip(ctxs, rnd):
                    c.fmmbem_set_wavenumber(2.0 * np.pi * freqs[i] / SOUND_SPEED)
                    c.fmmbem_setup()
                t_setup += time.perf_counter() - ts
                ts = time.perf_counter()
                xs, reps, status, _ = F.fmmbem_solve_many(ctxs[:len(rnd)], [0] * len(rnd), tol=tol, restart=400,
                                                          maxit=800, precision=F.FMMBEM_MIXED,
                                                          precond=F.FMMBEM_PC_NEARBLOCK)
                t_solve += time.perf_counter() - ts
                for q, i in enumerate(rnd):
                    if status[q] != 0:
                        raise RuntimeError(f"FGMRES did not converge at {freqs[i]:.0f} Hz (code {status[q]}, "
                                           f"relative residual {reps[q].rel_res:.2e} after {reps[q].iters} iterations)")
                    iters[i] = reps[q].iters
                ts = time.perf_counter()
                for q, i in enumerate(rnd):
                    H[i] = ctxs[q].fmmbem_eval_field(0, receivers, xs[q])
                t_field += time.perf_counter() - ts
                if log:
                    log(f"    {', '.join(f'{freqs[i]:.0f}' for i in rnd)} Hz: iterations "
                        f"{', '.join(str(int(iters[i])) for i in rnd)}")
        finally:
            for c in ctxs:
                c.close()
        s = {"band_hz": [float(freqs[idx[0]]), float(freqs[idx[-1]])], "frequencies": len(idx), "n": room.n,
             "contexts": nctx, "setup_s": t_setup, "solve_s": t_solve, "field_s": t_field,
             "wall_s": time.perf_counter() - t0, "iterations": [int(iters[i]) for i in idx]}
        summary.append(s)
        if log:
            log(f"  band {s['band_hz'][0]:.0f}-{s['band_hz'][1]:.0f} Hz: N {room.n}, {nctx} contexts, setup "
                f"{t_setup:.1f} s, solves {t_solve:.1f} s, field {t_field:.1f} s, iterations "
                f"{min(s['iterations'])}..{max(s['iterations'])}")
    return H, iters, summary
