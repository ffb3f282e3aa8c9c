"""Pins of the oracle's spectral broadening against closed forms (no GPU).

Unit-area Gaussians of standard deviation sigma: the profile integrates to the
summed oscillator strength, a single line peaks at f / (sigma sqrt(2 pi)) with
full width at half maximum 2 sqrt(2 ln 2) sigma, and the profile's mean and
variance are the f-weighted mean of the lines and their spread plus sigma^2.
"""
import numpy as np

from oracle import spectra


def test_single_line_peak_and_half_width():
    s = 0.1
    E = spectra.grid(3.0, 1e-5, 200001)   # 3.0 .. 5.0 eV
    S = spectra.broaden([4.0], [0.7], s, E)
    i = int(np.argmax(S))
    assert abs(E[i] - 4.0) < 1e-9
    assert abs(S[i] - 0.7 / (s * np.sqrt(2 * np.pi))) < 1e-12
    half = E[S >= S[i] / 2]
    fwhm = half[-1] - half[0]
    assert abs(fwhm - 2 * np.sqrt(2 * np.log(2)) * s) < 3e-5


def test_area_mean_and_variance():
    rng = np.random.default_rng(5)
    w = rng.uniform(3.0, 6.0, 40)
    f = rng.uniform(0.0, 1.0, 40)
    s = 0.1
    E = spectra.grid(1.0, 1e-4, 80001)    # 1 .. 9 eV, every line far inside
    S = spectra.broaden(w, f, s, E)
    area = np.trapezoid(S, E)
    assert abs(area - f.sum()) < 1e-10 * f.sum()
    mean = np.trapezoid(S * E, E) / area
    var = np.trapezoid(S * (E - mean) ** 2, E) / area
    wm = np.sum(f * w) / f.sum()
    assert abs(mean - wm) < 1e-10
    assert abs(var - (np.sum(f * (w - wm) ** 2) / f.sum() + s * s)) < 1e-10


def test_zero_strength_lines_vanish():
    E = spectra.grid(0.0, 0.01, 1000)
    assert np.abs(spectra.broaden([2.0, 5.0], [0.0, 0.0], 0.1, E)).max() == 0.0
