"""Host-side logic of the benchmark (no GPU): the steady-state extrapolation,
the algorithmic byte counts and the grid convergence index."""
import importlib.util
import math
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


class Geometric:
    """A stand-in solver whose permeability approaches k_inf geometrically:
    k_n = k_inf + a rho^n after n checks."""

    def __init__(self, k_inf, a, rho):
        self.k_inf, self.a, self.rho, self.steps, self.n = k_inf, a, rho, 0, 0

    def run(self, steps):
        self.steps += steps
        self.n += 1

    def permeability(self):
        return self.k_inf + self.a * self.rho ** self.n


def test_settle_aitken_is_exact_on_a_geometric_approach(bench):
    """Aitken's delta-squared recovers the limit of a geometric sequence
    exactly (up to rounding), whatever the check at which the run stops."""
    s = Geometric(0.0438, 3e-3, 0.8)
    k, k_inf, settled = bench._settle(s, 500, 10**9, 1e-6)
    assert settled and s.steps % 500 == 0
    assert abs(k - 0.0438) > 1e-9  # the raw value is still off
    assert k_inf == pytest.approx(0.0438, rel=1e-12)


def test_settle_stops_at_the_cap(bench):
    s = Geometric(1.0, 0.5, 0.999)
    k, k_inf, settled = bench._settle(s, 100, 1000, 1e-12)
    assert not settled and s.steps == 1000


def test_algorithmic_bytes_per_node_step(bench):
    """(4 s_w + s_i) N_L + 6 s_f + n_p [(3 s_w + s_i) N_L + 5 s_f] + n_p [(3 s_w + s_i) N_L + 7 s_f] at N_L = 30,
    n_p = 3: 3648 B (FP32) and 6456 B (FP64); the damped pressure equation adds n_p s_w N_L."""
    assert bench.acm_bytes_per_node_step(30, 4, 4) == 3648
    assert bench.acm_bytes_per_node_step(30, 8, 8) == 6456
    assert bench.acm_bytes_per_node_step(30, 4, 4, edac=True) == 3648 + 3 * 4 * 30
    assert bench.acm_bytes_per_node_step(30, 8, 8, edac=True) == 6456 + 3 * 8 * 30


def test_gci_of_a_hand_computed_series(bench):
    """Appendix B on four grids: errors against the finest, the apparent order
    from a least-squares line through the three coarser (log h, log e), and
    GCI = 1.3 |eps| / (ratio^p - 1) per pair."""
    hs = [0.014, 0.01, 0.007, 0.005]
    X = [4.0, 3.0, 2.5, 2.25]
    t = bench.gci_table(hs, X)
    e = [1.75 / 2.25, 0.75 / 2.25, 0.25 / 2.25]
    lh, le = np.log(hs[:3]), np.log(e)
    p = ((lh - lh.mean()) * (le - le.mean())).sum() / ((lh - lh.mean()) ** 2).sum()
    assert t["p"] == pytest.approx(p, rel=1e-12)
    assert t["e_vs_finest"] == pytest.approx(e, rel=1e-12)
    for row, (xc, xf, hc, hf) in zip(t["pairs"], [(4.0, 3.0, 0.014, 0.01), (3.0, 2.5, 0.01, 0.007),
                                                  (2.5, 2.25, 0.007, 0.005)]):
        eps = abs(xc - xf) / xf
        assert row["h"] == hf and row["eps"] == pytest.approx(eps, rel=1e-12)
        assert row["gci"] == pytest.approx(1.3 * eps / ((hc / hf) ** p - 1.0), rel=1e-12)


def test_hasimoto_drag_limits(bench):
    """Hasimoto's series: an isolated sphere's Stokes drag (K -> 1) as the
    array dilutes, with the leading correction 1.7601 c^(1/3) of the periodic
    images; and the permeability the paper derives from K, d / (6 pi r K),
    falls with the radius."""
    for r in (1e-3, 1e-2):
        c = 4.0 / 3.0 * math.pi * r ** 3
        x = c ** (1.0 / 3.0)
        K = bench.hasimoto_K(r)
        assert abs(K - (1.0 + 1.7601 * x)) <= 5.0 * x * x  # next term is (1.7601 x)^2
    ks = [1.0 / (6.0 * math.pi * r * bench.hasimoto_K(r)) for r in (0.05, 0.1, 0.15, 0.2)]
    assert all(a > b for a, b in zip(ks, ks[1:]))


def test_paper_stop_times_are_the_printed_ones(bench):
    """The physical times to the stopping criterion that Sec. 3.4 prints
    (h_min = 0.007), as the bench reports them beside its own."""
    assert bench.PAPER_STOP_TIME == {0.062: {"mlbm": 3.57, "acm": 3.58}, 0.6526: {"mlbm": 0.04, "acm": 0.39}}
