"""Oracle meshless TRT LBM (Sec. 2.2) pinned by the paper's tables, the
collision invariants and the standard-lattice special case."""
import os
from fractions import Fraction

import numpy as np
import pytest

import nodecloud as nc
import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_d3q15_matches_paper_table():
    e, w, opp = O.lattice(15)
    for line in open(os.path.join(GOLD, "d3q15_paper.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        k, ex, ey, ez, wk = line.split()
        k = int(k)
        assert tuple(e[k]) == (int(ex), int(ey), int(ez))
        assert w[k] == pytest.approx(float(Fraction(wk)), rel=1e-15)
        if k > 0:  # e_k = -e_{k-1} for even k
            assert tuple(e[k + 1]) == tuple(-e[k])
            assert w[k + 1] == w[k]
            assert opp[k] == k + 1 and opp[k + 1] == k


@pytest.mark.parametrize("q", [15, 19])
def test_lattice_isotropy(q):
    e, w, opp = O.lattice(q)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.abs(w @ e).max() < 1e-16
    assert np.allclose(np.einsum("k,ka,kb->ab", w, e, e), np.eye(3) / 3.0, atol=1e-15)
    assert np.array_equal(e[opp], -e)
    # fourth-order isotropy: sum w e_a^2 e_b^2 = 1/9 (a != b), sum w e_a^4 = 1/3
    m4 = np.einsum("k,ka,kb->ab", w, e ** 2, e ** 2)
    assert np.allclose(m4, (np.ones((3, 3)) + 2 * np.eye(3)) / 9.0, atol=1e-15)


@pytest.fixture(scope="module")
def lattice12():
    c = nc.lattice_cloud(12)
    return c, nc.stencils(c.pos, 30)


def textbook_lbm(f, e, w, tau, g_lb, steps, n):
    """Plain lattice BGK with first-order forcing, streaming by array shifts."""
    q = len(w)
    F = f.reshape(n, n, n, q).copy()
    for _ in range(steps):
        rho = F.sum(-1)
        u = F @ e / rho[..., None]
        eu = u @ e.T
        uu = (u * u).sum(-1)[..., None]
        feq = rho[..., None] * w * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * uu)
        force = 3 * w * (e @ g_lb)[None, None, None, :] * rho[..., None]
        post = F - (F - feq) / tau + force
        for k in range(q):
            F[..., k] = np.roll(post[..., k], shift=tuple(e[k].astype(int)), axis=(0, 1, 2))
    return F.reshape(-1, q)


def test_mlbm_on_a_lattice_is_lattice_boltzmann(lattice12):
    """Nodes on a cubic lattice of spacing dx = streaming distance: every
    departure point is a node, interpolation returns the nodal value, and MLBM
    with tau+ = tau- (BGK) is the textbook lattice Boltzmann method."""
    c, S = lattice12
    n = 12
    m = O.MLBM(c.pos, c.n, S, np.zeros((0, 3)), q=19, dx=1.0 / n, tau_plus=0.8, magic=0.09, g=(0.3, 0.1, 0.0))
    assert m.tau_minus == pytest.approx(0.8)
    rng = np.random.default_rng(2)
    u0 = 0.01 * rng.normal(size=(c.n, 3))
    f0 = np.concatenate([O.equilibrium(19, 1, 1.0 + 0.01 * rng.normal(), u0[i]) for i in range(c.n)])
    m.f[:] = f0
    m.run(7)
    e, w, _ = O.lattice(19)
    ref = textbook_lbm(f0, e, w, 0.8, m.g_lb, 7, n)
    assert np.abs(m.f - ref).max() < 1e-13


def test_collision_invariants_on_lattice(lattice12):
    """On the lattice streaming permutes values, so one step conserves total
    mass exactly and adds sum_i rho_i g_lb of momentum (Eq. force_lbm)."""
    c, S = lattice12
    g = np.array([0.002, -0.001, 0.0005])
    m = O.MLBM(c.pos, c.n, S, np.zeros((0, 3)), q=19, dx=1.0 / 12, tau_plus=1.0, magic=1.0, g=(1, 1, 1))
    m.g_lb = g
    rng = np.random.default_rng(3)
    e, w, _ = O.lattice(19)
    m.f[:] = w * (1.0 + 0.05 * rng.uniform(-1, 1, size=(c.n, 19)))
    rho0 = m.f.sum(1)
    mom0 = (m.f @ e).sum(0)
    m.run(1)
    assert m.f.sum() == pytest.approx(rho0.sum(), rel=1e-14)
    assert np.abs((m.f @ e).sum(0) - (mom0 + rho0.sum() * g)).max() < 1e-12


def test_equilibrium_without_force_is_fixed(lattice12):
    c, S = lattice12
    m = O.MLBM(c.pos, c.n, S, np.zeros((0, 3)), q=19, dx=1.0 / 12, tau_plus=0.7, magic=0.25, g=(0, 0, 0))
    u = np.array([0.02, -0.01, 0.005])
    m.f[:] = O.equilibrium(19, c.n, 1.1, u)
    f0 = m.f.copy()
    m.run(3)
    assert np.abs(m.f - f0).max() < 1e-15


def test_shear_wave_decay_sets_viscosity():
    """A shear wave u_x = U sin(2 pi z / L) decays at nu_lb k^2 with
    nu_lb = (tau+ - 1/2)/3 (Eq. lbm_viscosity); the paper's TRT setting
    tau+ = 1, Lambda = 1 (tau- = 5/2)."""
    n = 32
    c = nc.lattice_cloud(n)
    S = nc.stencils(c.pos, 30)
    m = O.MLBM(c.pos, c.n, S, np.zeros((0, 3)), q=19, dx=1.0 / n, tau_plus=1.0, magic=1.0, g=(0, 0, 0))
    assert m.tau_minus == pytest.approx(2.5)
    z = c.pos[:, 2]
    s = np.sin(2 * np.pi * z)
    U = 1e-4
    m.f[:] = np.concatenate([O.equilibrium(19, 1, 1.0, (U * s[i], 0, 0)) for i in range(c.n)])
    steps = 60
    m.run(steps)
    _, u = O.moments(19, m.f)
    amp = 2 * (u[:, 0] * s).mean()
    k = 2 * np.pi / n
    nu_lb = (1.0 - 0.5) / 3.0
    rate = -np.log(amp / U) / steps
    assert rate == pytest.approx(nu_lb * k * k, rel=0.02)


def test_rest_state_preserved_with_grain(small_cloud, small_stencils):
    """Interpolation rows reproduce constants and bounce-back swaps equal
    values, so a fluid at rest without force stays at rest."""
    c, S = small_cloud, small_stencils
    m = O.MLBM(c.pos, c.n_int, S, c.nrm, q=19, h_min=0.02, g=(0, 0, 0))
    f0 = m.f.copy()
    m.run(5)
    assert np.abs(m.f - f0).max() < 1e-14
