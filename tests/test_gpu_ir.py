"""Impulse-response synthesis (Section 4.1) against the image-source solution Eq. (an2): the 8 x 6 x 3 m
room with zeta = 9 on every wall (normal-incidence reflection coefficient R = (zeta - 1)/(zeta + 1) =
0.8), the monopole at (3, 2, 1.75) m, receivers in the source's plane, equispaced frequencies 20 Hz
apart (T = 50 ms) up to 320 Hz (FGMRES to 1e-4; 20 Hz lies just below the room's first axial mode) on one mesh of about 6.7 elements per wavelength at the top
frequency, the pulse of Eq. (an3).  The image solution takes R independent of the angle of
incidence, which an impedance wall is not, so the comparison is a validation within that model's
approximation, not parity: the pulse responses agree over the first 25 ms (direct sound and early
reflections)."""
import numpy as np
import pytest

from oracle import analytic
from paper_2103_16073_amd import synth

pytestmark = pytest.mark.gpu


def test_impulse_response_vs_image_sources():
    from paper_2103_16073_amd import ir
    L = (8.0, 6.0, 3.0)
    zeta = 9.0
    fmax, df = 320.0, 20.0
    freqs = np.arange(df, fmax + df / 2, df)
    h = synth.SOUND_SPEED / (6.7 * fmax)
    room = synth.shoebox(*L, h)
    beta = np.full(room.n, 1.0 / zeta)
    rs = np.array([3.0, 2.0, 1.75])
    rec = np.array([[1.5, 1.0, 1.75], [5.0, 4.0, 1.75], [6.5, 1.5, 1.75], [2.0, 4.5, 1.75], [4.2, 2.8, 1.75],
                    [7.0, 5.0, 1.75]])
    H, iters = ir.transfer_functions(room.vertices, room.triangles, beta, rs, rec, freqs,
                                     solve_kw=dict(tol=1e-4, restart=500, maxit=3000, precond=1))
    T = 1.0 / df
    Hi = np.stack([analytic.image_sum_box(L, rs, rec, 2 * np.pi * f / synth.SOUND_SPEED, 0.8,
                                          r_max=synth.SOUND_SPEED * T) for f in freqs])
    ef = np.linalg.norm(H - Hi, axis=1) / np.linalg.norm(Hi, axis=1)
    dt = T / 256
    times = np.arange(0, T, dt)
    F = ir.an3_spectrum(freqs, dt)
    pb = ir.synthesize(H, freqs, F, times)
    pi = ir.synthesize(Hi, freqs, F, times)
    early = times < T / 2  # direct sound and the first reflections
    et = np.linalg.norm(pb[early] - pi[early]) / np.linalg.norm(pi[early])
    corr = np.sum(pb[early] * pi[early]) / np.sqrt(np.sum(pb[early] ** 2) * np.sum(pi[early] ** 2))
    print(f"N {room.n}, iterations {iters}")
    print("per-frequency relative difference:", " ".join(f"{e:.3f}" for e in ef))
    print(f"first 25 ms: relative L2 {et:.3f}, correlation {corr:.4f}")
    # measured: correlation 0.972, relative L2 0.237.  The constant-R image model differs from an
    # impedance wall at oblique incidence, and both frequency responses are sampled every 20 Hz,
    # so late reverberation beyond 50 ms folds back into the BEM's window (not into the truncated
    # image sum); the frequency-domain differences (median 0.46) carry both effects.
    assert np.all(np.isfinite(H)) and corr > 0.95 and et < 0.35


def test_impulse_response_plane_two_bands_vs_image_sources():
    # 32 frequencies to 640 Hz on two band meshes (6.7 elements per wavelength at 320 and 640 Hz),
    # every frequency's field on a receiver plane at the source height, the pulse of Eq. (an3) by one
    # inverse FFT per receiver (256 steps of T / 256), and the image sources on the plane's receivers
    # at least 0.3 m from the walls
    from paper_2103_16073_amd import ir
    L = (8.0, 6.0, 3.0)
    zeta = 9.0
    rs = np.array([3.0, 2.0, 1.75])
    df, nt = 20.0, 256
    freqs = df * np.arange(1, 33)
    rec, (nx, ny) = ir.receiver_plane(L[0], L[1], 1.75, 0.25)
    H, iters, summary = ir.sweep_plane(L, zeta, rs, freqs, rec, [320.0, 640.0], tol=1e-4)
    assert [s["frequencies"] for s in summary] == [16, 16] and np.all(iters > 0)
    T = 1.0 / df
    dt = T / nt
    spec = ir.an3_spectrum(freqs, dt)
    pb = ir.synthesize_fft(H, spec, nt)
    inner = np.where((rec[:, 0] > 0.3) & (rec[:, 0] < 7.7) & (rec[:, 1] > 0.3) & (rec[:, 1] < 5.7)
                     & (np.linalg.norm(rec - rs, axis=1) > 0.2))[0]
    Hi = np.stack([analytic.image_sum_box(L, rs, rec[inner], 2 * np.pi * f / synth.SOUND_SPEED, 0.8,
                                          r_max=synth.SOUND_SPEED * T) for f in freqs])
    pi = ir.synthesize_fft(Hi, spec, nt)
    times = np.arange(nt) * dt
    early = times < T / 2
    a, b = pb[early][:, inner], pi[early]
    et = np.linalg.norm(a - b) / np.linalg.norm(b)
    corr = np.sum(a * b) / np.sqrt(np.sum(a * a) * np.sum(b * b))
    ef = np.linalg.norm(H[:, inner] - Hi, axis=1) / np.linalg.norm(Hi, axis=1)
    print("bands:", [(s["n"], s["contexts"], min(s["iterations"]), max(s["iterations"])) for s in summary])
    print(f"{len(inner)} receivers; per-frequency median relative difference {np.median(ef):.3f}; "
          f"first 25 ms: relative L2 {et:.3f}, correlation {corr:.4f}")
    # measured: 656 receivers, correlation 0.984, relative L2 0.179 over the first 25 ms; iterations
    # 9..26 (14,516 elements) and 25..27 (57,608 elements)
    assert np.all(np.isfinite(pb)) and corr > 0.97 and et < 0.25
