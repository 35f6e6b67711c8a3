"""Host side of the impulse-response synthesis (Section 4.1, Eq. an3): the FFT synthesis against its
definition as a sum over frequencies, the pulse spectrum against the pulse, and the receiver plane."""
import numpy as np

from paper_2103_16073_amd import ir


def test_fft_synthesis_equals_the_frequency_sum():
    rng = np.random.default_rng(3)
    nt, df = 256, 20.0
    dt = 1.0 / df / nt
    t = np.arange(nt) * dt
    for nf in (128, 100, 16):
        f = df * np.arange(1, nf + 1)
        H = rng.normal(size=(nf, 7)) + 1j * rng.normal(size=(nf, 7))
        F = ir.an3_spectrum(f, dt)
        a = ir.synthesize(H, f, F, t)
        b = ir.synthesize_fft(H, F, nt)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_pulse_of_an_on_grid_delay_is_the_finite_delta_pair():
    # H = e^{i w tau} (a wave arriving at tau = j dt): with the full band (nf = nt / 2) the discrete
    # synthesis returns nf [delta(n - j - 1) - delta(n - j + 1)], the pulse f(t - tau) of Eq. (an3)
    # on the time grid
    nt, df = 256, 20.0
    dt = 1.0 / df / nt
    f = df * np.arange(1, nt // 2 + 1)
    F = ir.an3_spectrum(f, dt)
    for j in (5, 37, 200):
        p = ir.synthesize_fft(np.exp(2j * np.pi * f * j * dt)[:, None], F, nt)[:, 0]
        want = np.zeros(nt)
        want[j + 1] = nt // 2
        want[j - 1] = -(nt // 2)
        assert np.abs(p - want).max() < 1e-9


def test_an3_spectrum_is_the_transform_of_the_pulse():
    # f(t) = delta(t - dt) - delta(t + dt): int f(t) e^{i w t} dt = e^{i w dt} - e^{-i w dt}
    dt = 1e-4
    w = 2 * np.pi * np.array([20.0, 700.0, 2560.0])
    assert np.allclose(ir.an3_spectrum(w / (2 * np.pi), dt), np.exp(1j * w * dt) - np.exp(-1j * w * dt), rtol=0,
                       atol=1e-15)


def test_receiver_plane_covers_the_floor_area_off_the_walls():
    pts, (nx, ny) = ir.receiver_plane(8.0, 6.0, 1.75, 0.05)
    assert (nx, ny) == (160, 120) and pts.shape == (160 * 120, 3)
    assert np.all(pts[:, 2] == 1.75)
    assert np.isclose(pts[:, 0].min(), 0.025) and np.isclose(pts[:, 0].max(), 7.975)
    assert np.isclose(pts[:, 1].min(), 0.025) and np.isclose(pts[:, 1].max(), 5.975)
    # no receiver on the source position of the paper's example
    assert np.min(np.linalg.norm(pts - np.array([3.0, 2.0, 1.75]), axis=1)) > 0.03
