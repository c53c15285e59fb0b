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
    """Stratified along the allowed set: the i-th radius lies in the i-th of n
    equal parts of [lo, hi] minus the held-out neighbourhoods, measured along
    that set (computed here on a fine grid, independently of the function)."""
    for n, lo, hi, held in ((16, 0.15, 0.48, (0.3, 0.33)), (64, 0.15, 0.6, (0.18, 0.33, 0.47, 0.58)),
                            (10, 0.2, 0.45, (0.33,))):
        rs = training_radii(n, lo=lo, hi=hi, held_out=held)
        assert len(rs) == n and all(lo <= r <= hi for r in rs)
        assert all(abs(r - h) > 0.01 for r in rs for h in held)
        grid = np.linspace(lo, hi, 2_000_001)
        ok = np.all(np.abs(grid[:, None] - np.array(held)[None, :]) > 0.01, axis=1)
        along = np.concatenate([[0.0], np.cumsum(ok[1:] * np.diff(grid))])  # allowed length below each grid point
        L = along[-1]
        pos = np.interp(rs, grid, along)
        assert all(i * L / n - 1e-6 <= p <= (i + 1) * L / n + 1e-6 for i, p in enumerate(pos))
        assert training_radii(n, lo=lo, hi=hi, held_out=held) == rs  # seeded
