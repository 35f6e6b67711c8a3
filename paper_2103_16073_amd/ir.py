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
