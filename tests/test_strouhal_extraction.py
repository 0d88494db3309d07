"""The Strouhal number extraction of the cylinder workload (bench.py,
Sec. 3.1: St = f d / U0 from the lift) on synthetic lift series of known
frequency: a pure tone, one with a mean, a harmonic and noise, and one whose
sampling interval does not divide its period."""
import numpy as np
import pytest

from bench import strouhal_from_lift


def _series(st, d_lattice, u0, every, periods, **kw):
    f = st * u0 / d_lattice                       # cycles per step
    t = np.arange(int(periods / f / every)) * every
    x = np.sin(2 * np.pi * f * t + kw.get("phase", 0.3)) + kw.get("mean", 0.0)
    x = x + kw.get("harmonic", 0.0) * np.sin(4 * np.pi * f * t + 1.0)
    rng = np.random.default_rng(kw.get("seed", 0))
    return x + kw.get("noise", 0.0) * rng.standard_normal(len(t))


@pytest.mark.parametrize("st,kw", [(0.2, {}), (0.165, {"mean": 0.7}), (0.19, {"harmonic": 0.3, "noise": 0.05}),
                                   (0.21, {"phase": 2.0}), (0.18, {"noise": 0.15, "seed": 3})])
def test_known_frequency_is_recovered(st, kw):
    d_lattice, u0, every = 42.0, 0.01, 50    # d = 42 streaming distances, 21 000 steps per period at St 0.2
    lift = _series(st, d_lattice, u0, every, periods=10, **kw)
    st_zero, st_fft = strouhal_from_lift(lift, every, d_lattice, u0)
    # noise moves each crossing by about noise / slope
    assert st_zero == pytest.approx(st, rel=1e-2 if kw.get("noise") else 2e-3)
    # the spectrum's resolution is 1 / (8 x the record), about 1 % of f here
    assert st_fft == pytest.approx(st, rel=2e-2)


def test_noise_near_zero_adds_no_crossings():
    # without the hysteresis band every noisy pass through zero would count:
    # a plain sign-change count here gives several times too many crossings
    lift = _series(0.2, 42.0, 0.01, 50, periods=10, noise=0.1, seed=5)
    x = lift - lift.mean()
    plain = np.count_nonzero((x[:-1] < 0) & (x[1:] >= 0))
    assert plain > 15
    st_zero, _ = strouhal_from_lift(lift, 50, 42.0, 0.01)
    assert st_zero == pytest.approx(0.2, rel=1e-2)


def test_too_short_a_record_gives_nan():
    lift = _series(0.2, 42.0, 0.01, 50, periods=1.5)
    st_zero, _ = strouhal_from_lift(lift, 50, 42.0, 0.01)
    assert np.isnan(st_zero)
