"""Host-side pieces of the learned warm start (no GPU): the magnitude
interpolation and the choice of training radii."""
import numpy as np
import pytest

pytest.importorskip("torch")

from paper_2404_14195_amd.warmstart import _Pchip, training_radii  # noqa: E402


def test_pchip_interpolates_and_matches_scipy_inside():
    from scipy.interpolate import PchipInterpolator
    rng = np.random.default_rng(0)
    x = np.sort(rng.uniform(0.15, 0.48, 9))
    y = np.log(0.05 * (0.5 - x) ** 3 + 1e-4)  # monotone decreasing, like log k(r)
    f = _Pchip(x, y)
    for xi, yi in zip(x, y):
        assert f(xi) == pytest.approx(yi, abs=1e-14)
    ref = PchipInterpolator(x, y)
    # same interior slopes (Fritsch-Carlson weighted harmonic mean); only the
    # end-point slopes differ, so compare away from the two end intervals
    for t in np.linspace(x[1], x[-2], 57):
        assert f(t) == pytest.approx(float(ref(t)), abs=1e-12)
    # monotone data stay monotone
    ts = np.linspace(x[0], x[-1], 400)
    assert np.all(np.diff([f(t) for t in ts]) <= 1e-15)


def test_training_radii_are_stratified_and_avoid_held_out():
    rs = training_radii(16, held_out=(0.3, 0.33))
    assert len(rs) == 16 and all(0.15 <= r <= 0.48 for r in rs)
    edges = np.linspace(0.15, 0.48, 17)
    assert all(edges[i] <= r <= edges[i + 1] for i, r in enumerate(rs))
    assert all(abs(r - h) > 0.01 for r in rs for h in (0.3, 0.33))
    assert training_radii(16, held_out=(0.3, 0.33)) == rs  # seeded
