"""The space-time spectrum tools on histories whose spectrum is known by
construction: a travelling wave puts its power at its own mode and
frequency, and a sum of two modes is dominated by the stronger."""
import numpy as np
import pytest

from paper_2609_17151_amd import spectrum as SP


def _wave(m, omega, L=2.0, N=128, T=256, dt=0.01, amp=1.0, phase=0.3):
    x = np.arange(N) * L / N
    t = np.arange(T) * dt
    k = 2 * np.pi * m / L
    return amp * np.cos(k * x[None, :] - omega * t[:, None] + phase), L, dt


def test_travelling_wave_mode_and_frequency():
    # omega on an exact FFT bin: 2 pi * 8 / (T dt)
    T, dt = 256, 0.01
    om = 2 * np.pi * 8 / (T * dt)
    h, L, dt = _wave(15, om, T=T, dt=dt)
    h = h + 5.0                                       # the mean is removed
    P, m, omega = SP.spectrum(h, L, dt)
    i, j = np.unravel_index(np.argmax(P), P.shape)
    assert m[j] == 15
    # exp(i(kx - wt)) appears at -omega in numpy's time transform convention
    assert abs(abs(omega[i]) - om) < 1e-9
    assert SP.dominant_mode(h, L, dt) == (15, pytest.approx(L / 15))
    # all the power lies on the dispersion relation omega = (om / k15) k
    k15 = 2 * np.pi * 15 / L
    assert SP.power_near(P, m, omega, lambda k: om / k15 * k, L, width=0.01) == pytest.approx(1.0)


def test_stronger_mode_dominates():
    a, L, dt = _wave(15, 3.0, amp=1.0)
    b, _, _ = _wave(7, 1.0, amp=0.6)
    assert SP.dominant_mode(a + b, L, dt)[0] == 15
    assert SP.dominant_mode(0.5 * a + b, L, dt)[0] == 7


def test_record_samples_every_interval():
    class FakeSim:
        n_nodes = [4]

        def __init__(self):
            self.t = 0

        def step(self, n):
            self.t += n

        def density(self, b=0):
            return np.array([np.zeros(4), np.full(4, float(self.t))])

    h = SP.record(FakeSim(), 1, 16, 5)
    np.testing.assert_array_equal(h[:, 0], [16, 32, 48, 64, 80])
