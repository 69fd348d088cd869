"""Pins of the resampling oracle: identities, exact reproduction at
coinciding samples, hand-worked nearest indices, and a band-limited signal."""

import numpy as np

from oracle import resample as rs


def test_same_step_is_the_identity():
    rng = np.random.default_rng(1)
    d = rng.standard_normal((3, 50))
    for mode in ("nearest", "sinc"):
        # sin(pi k) is about 1e-16, not 0, in floating point
        assert np.allclose(rs.resample(d, 2e-3, 50, 2e-3, mode), d, rtol=0, atol=1e-13)


def test_sinc_upsampling_keeps_the_input_samples():
    # with dt_out = dt_in / 2, output m = 2k + 1 falls on input sample k
    rng = np.random.default_rng(2)
    d = rng.standard_normal((2, 40))
    out = rs.resample(d, 4e-3, 80, 2e-3, "sinc")
    assert np.allclose(out[:, 1::2], d, rtol=0, atol=1e-13)


def test_nearest_hand_worked():
    d = np.arange(10.0)[None, :]            # sample k at t = (k + 1) * 1 ms
    out = rs.resample(d, 1e-3, 4, 2.5e-3, "nearest")
    # t = 2.5, 5.0, 7.5, 10.0 ms -> round half up (2.5 -> 3) -> index t - 1
    assert out.tolist() == [[2.0, 4.0, 7.0, 9.0]]
    out = rs.resample(d, 1e-3, 3, 4e-3, "nearest")       # past the end: clamped
    assert out.tolist() == [[3.0, 7.0, 9.0]]


def test_sinc_reproduces_a_band_limited_signal():
    # a 30 Hz sine sampled at 2 ms (Nyquist 250 Hz) over 2 s, resampled at
    # 0.7 ms: away from the ends the interpolation error is small
    dt, n = 2e-3, 1000
    t = (np.arange(n) + 1.0) * dt
    f = np.sin(2 * np.pi * 30.0 * t)[None, :]
    dto, m = 0.7e-3, 2800
    out = rs.resample(f, dt, m, dto, "sinc")[0]
    to = (np.arange(m) + 1.0) * dto
    mid = (to > 0.5) & (to < 1.5)
    assert np.max(np.abs(out[mid] - np.sin(2 * np.pi * 30.0 * to[mid]))) < 2e-3
