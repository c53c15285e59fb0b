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


# --- unknown populations at boundary nodes (Sec. 2.2; Sec. 3.3 touching limit)

def unknown_set(mask_b, q):
    return [k for k in range(q) if mask_b >> k & 1]


@pytest.mark.parametrize("q, n_diag, n_zero", [(19, 6, 6), (15, 7, 0)])
def test_unknown_normal_rule_hand_cases(q, n_diag, n_zero):
    """Counted by hand from the velocity sets: along +x the five velocities
    with e_x = 1 leave from the solid side (one axis and four diagonals in
    both lattices).  Along the cube diagonal the ones with e_x + e_y + e_z > 0
    do: D3Q19 has 3 axes + 3 face diagonals, and 6 face diagonals with zero
    sum that stay known in both directions; D3Q15 has 3 axes + 4 corners."""
    e, _, opp = O.lattice(q)
    nrm = np.array([[1.0, 0.0, 0.0], [1.0, 1.0, 1.0]]) / np.array([[1.0], [np.sqrt(3.0)]])
    m = O.lbm_unknown(q, np.zeros((2, 3)), nrm, "normal")
    ks = unknown_set(int(m[0]), q)
    assert len(ks) == 5 and all(e[k, 0] == 1 for k in ks)
    ks = unknown_set(int(m[1]), q)
    assert len(ks) == n_diag and all(e[k].sum() > 0 for k in ks)
    zero = [k for k in range(1, q) if not (m[1] >> k & 1) and not (m[1] >> opp[k] & 1)]
    assert len(zero) == n_zero


@pytest.mark.parametrize("q", [15, 19])
def test_unknown_normal_rule_one_of_each_pair(small_cloud, q):
    """For a generic normal exactly one population of each opposite pair
    departs from the solid side, and the rest population never does."""
    c = small_cloud
    _, _, opp = O.lattice(q)
    m = O.lbm_unknown(q, c.pos[c.n_int:], c.nrm, "normal")
    assert not (m & 1).any()
    for k in range(1, q):
        assert ((m >> k & 1) ^ (m >> opp[k] & 1)).all()


def test_unknown_solid_rule_single_grain_closed_form(small_cloud):
    """A node x on the sphere |x - c| = r with outward normal n: |x - dx e - c|^2
    = r^2 - 2 dx r (e . n) + dx^2 |e|^2, so the departure point is inside the
    grain iff e . n > dx |e|^2 / (2 r).  Below r = 1/2 no other image reaches
    the cell, so this must be the whole solid rule."""
    c = small_cloud
    assert c.r < 0.5
    dx = 0.013
    e, _, _ = O.lattice(19)
    m = O.lbm_unknown(19, c.pos[c.n_int:], c.nrm, "solid", dx, c.r)
    en = c.nrm @ e.T  # [nb][q]
    thr = dx * (e * e).sum(1) / (2 * c.r)
    decided = np.abs(en - thr) > 1e-9
    expect = (en > thr)
    got = (m[:, None] >> np.arange(19)[None, :] & 1).astype(bool)
    assert decided[:, 1:].mean() > 0.99
    assert (got == expect)[decided].all()
    # and the two rules differ only at near-tangent velocities, 0 < e . n <= thr
    mn = O.lbm_unknown(19, c.pos[c.n_int:], c.nrm, "normal")
    diff = ((m ^ mn)[:, None] >> np.arange(19)[None, :] & 1).astype(bool)
    assert diff.any() and ((en > 0) & (en <= thr + 1e-9))[diff].all()


def test_unknown_solid_rule_overlapping_grains_against_kdtree():
    """For r > 1/2 the neighbouring images of the grain reach into the cell.
    The periodic distance from the departure point to the nearest grain centre,
    from scipy's periodic k-d tree, decides independently; and some departure
    points of the overlapping cell fall into a neighbouring image while their
    own normal says fluid side (the case the rule is for)."""
    from scipy.spatial import cKDTree
    r, dx = 0.52, 0.02
    c = nc.sphere_cloud(r, 0.04, 0.3, 0.08, seed=7)
    e, _, _ = O.lattice(19)
    pb = c.pos[c.n_int:]
    m = O.lbm_unknown(19, pb, c.nrm, "solid", dx, r)
    tree = cKDTree(np.array([[0.5, 0.5, 0.5]]), boxsize=1.0)
    got = (m[:, None] >> np.arange(19)[None, :] & 1).astype(bool)
    dep = pb[:, None, :] - dx * e[None, :, :]  # [nb][q][3]
    d, _ = tree.query(np.mod(dep.reshape(-1, 3), 1.0))
    d = d.reshape(len(pb), 19)
    decided = np.abs(d - r) > 1e-12
    decided[:, 0] = True
    expect = d < r
    expect[:, 0] = False
    assert (got == expect)[decided].all()
    en = c.nrm @ e.T
    assert (got & (en < 0)).any()


def test_rest_state_preserved_with_solid_rule():
    """Bounce-back swaps equal populations at rest under either rule."""
    c = nc.sphere_cloud(0.52, 0.04, 0.3, 0.08, seed=7)
    S = nc.solver_stencils(c, 30)
    m = O.MLBM(c.pos, c.n_int, S, c.nrm, q=15, h_min=c.h_min, magic=1.0, g=(0, 0, 0), rule="solid", r=c.r)
    f0 = m.f.copy()
    m.run(3)
    assert np.abs(m.f - f0).max() < 1e-14


def test_bounce_back_reads_streamed_values():
    """On a periodic lattice the shift rows are Kronecker deltas, so streaming
    is exact lattice streaming: f_k(x) = f_k^post(x - dx e_k).  A node-wise
    equilibrium state without force is its own post-collision state.  At a
    node marked with both k and opp(k) unknown, each takes the other's
    streamed value: f_k(b) = f_opp^0(b + dx e_k) and f_opp(b) =
    f_k^0(b - dx e_k); a one-sided copy would put the first value in both."""
    n = 6
    c = nc.lattice_cloud(n)
    S = nc.stencils(c.pos, 30)
    q = 19
    e, _, opp = O.lattice(q)
    W, info = O.weights(c.pos, S, [("shift", tuple(-e[k] / n)) for k in range(q)])
    assert not info.any()
    rng = np.random.default_rng(2)
    f0 = np.concatenate([O.equilibrium(q, 1, 1.0 + 0.01 * rng.normal(), 0.02 * rng.normal(size=3))
                         for _ in range(c.n)])
    b = c.n - 1  # the last node plays a boundary node
    k = 7
    kb = int(opp[k])
    mask = np.array([(1 << k) | (1 << kb)], dtype=np.uint32)
    f = f0.copy()
    O.lbm_run(q, c.n - 1, S, W, mask, 1.0, 1.0, np.zeros(3), f, 1)

    def node_at(x):
        d = nc.min_image(c.pos - x)
        return int(np.argmin((d * d).sum(1)))

    up = node_at(c.pos[b] + e[k] / n)
    down = node_at(c.pos[b] - e[k] / n)
    assert f[b, k] == pytest.approx(f0[up, kb], abs=1e-15)
    assert f[b, kb] == pytest.approx(f0[down, k], abs=1e-15)
    assert abs(f0[up, kb] - f0[down, k]) > 1e-4  # the two readings differ here


# --- the two relaxation rates of Eq. LBM_collision, each on its own mode ---

@pytest.mark.parametrize("q", [15, 19])
@pytest.mark.parametrize("tau_plus,magic", [(1.0, 1.0), (0.8, 0.25), (0.62, 0.03)])
def test_trt_relaxes_odd_and_even_modes_at_their_own_rates(q, tau_plus, magic):
    """TRT relaxes the symmetric part of f - f^eq at 1/tau+ and the
    antisymmetric part at 1/tau- (Eq. LBM_collision with Lambda =
    (tau+ - 1/2)(tau- - 1/2)).  Add to a uniform moving equilibrium the odd
    mode eps w_k (e_kx (e_ky^2 - e_kz^2) + e_kx e_ky e_kz) (the first term
    lives on the D3Q19 edge vectors, the second on the D3Q15 diagonals), which
    has no mass and no momentum on either lattice (fourth-order isotropy and
    parity), so rho, u and f^eq are unchanged:
    after one step (without forcing, a uniform state streams onto itself) the
    mode must be scaled by exactly 1 - 1/tau-.  The even mode
    eps w_k (e_kx^2 - e_ky^2) likewise has no mass or momentum and must be
    scaled by 1 - 1/tau+.  Taking 1/tau+ for both parts, swapping the two, or
    a sign error in either relaxation term fails one of the two checks."""
    n = 6
    c = nc.lattice_cloud(n)
    S = nc.stencils(c.pos, 27)
    m = O.MLBM(c.pos, c.n, S, np.zeros((0, 3)), q=q, dx=1.0 / n, tau_plus=tau_plus, magic=magic, g=(0, 0, 0))
    tau_minus = 0.5 + magic / (tau_plus - 0.5)
    assert m.tau_minus == pytest.approx(tau_minus, rel=1e-15)
    e, w, _ = O.lattice(q)
    feq = O.equilibrium(q, 1, 1.02, np.array([0.03, -0.02, 0.01]))[0]
    odd = w * (e[:, 0] * (e[:, 1] ** 2 - e[:, 2] ** 2) + e[:, 0] * e[:, 1] * e[:, 2])
    even = w * (e[:, 0] ** 2 - e[:, 1] ** 2)
    for mode in (odd, even):  # neither mode carries mass or momentum
        assert abs(mode.sum()) < 1e-17 and np.abs(mode @ e).max() < 1e-17
    eps = 1e-3
    for mode, tau in ((odd, tau_minus), (even, tau_plus)):
        m.f[:] = feq + eps * mode
        m.run(1)
        expect = feq + (1.0 - 1.0 / tau) * eps * mode
        assert np.abs(m.f - expect).max() < 1e-15
    # the two rates are distinguishable in every case above
    assert abs(1.0 / tau_minus - 1.0 / tau_plus) * eps * np.abs(odd).max() > 1e-7


def test_threads_do_not_change_the_oracle():
    """The MLBM oracle's node loops may run on several host threads (to time
    it on all cores); every node's arithmetic is unchanged, so the state is
    identical bit for bit."""
    c = nc.sphere_cloud(0.3, 0.05, 0.3, 0.1, seed=1)
    S = nc.solver_stencils(c, 30)
    out = []
    try:
        for th in (1, 4):
            assert O.set_threads(th) == th
            m = O.MLBM(c.pos, c.n_int, S, c.nrm, q=19, h_min=c.h_min)
            m.run(30)
            out.append(m.f.copy())
    finally:
        O.set_threads(1)
    assert np.array_equal(out[0], out[1])
