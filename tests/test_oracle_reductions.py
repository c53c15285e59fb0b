"""Oracle geometry, permeability and drag reductions pinned by closed forms,
the divergence theorem and brute force."""
import os

import numpy as np
import pytest

import nodecloud as nc
import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_porosity_matches_paper_pairs():
    for line in open(os.path.join(GOLD, "porosity_paper.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        r, phi, tol = map(float, line.split())
        assert abs(O.porosity(r) - phi) <= tol, (r, O.porosity(r), phi)


@pytest.mark.parametrize("r", [0.3, 0.55, 0.65])
def test_porosity_and_area_brute_force(r):
    rng = np.random.default_rng(7)
    x = rng.uniform(size=(2_000_000, 3))
    phi_mc = (nc.sphere_sdf(x, r) > 0).mean()
    assert O.porosity(r) == pytest.approx(phi_mc, abs=2e-3)
    # area: uniform points on the sphere, fraction that is not covered by an image
    u = rng.normal(size=(1_000_000, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    p = 0.5 + r * u
    inside = np.all((p >= 0) & (p < 1), axis=1)
    assert O.area(r) == pytest.approx(4 * np.pi * r * r * inside.mean(), rel=3e-3)


@pytest.fixture(scope="module")
def plan_small(small_cloud):
    pp = nc.plane_plan(small_cloud, 64, 30)
    pw = O.plane_weights(small_cloud.pos, pp.idx, pp.shift)
    return pp, pw


def test_flux_of_uniform_field(small_cloud, plan_small):
    """v_x = 1 in the fluid: interpolation reproduces constants, so q is the
    fraction of fluid samples, and that tends to the mean open fraction of the
    five planes: (1 + 1 + (1 - pi(r^2 - 0.01))*2 + 1)/5 for r = 0.3."""
    pp, pw = plan_small
    q = O.flux(pp.idx, pw, np.ones(small_cloud.n), 5 * 64 * 64)
    assert q == pytest.approx(pp.n_samples / (5 * 64 * 64), rel=1e-13)
    r = small_cloud.r
    open_frac = [1.0 if abs(x - 0.5) >= r else 1.0 - np.pi * (r * r - (x - 0.5) ** 2) for x in pp.planes]
    assert q == pytest.approx(np.mean(open_frac), abs=2e-3)


def test_flux_of_linear_field(small_cloud, plan_small):
    """A field linear in y and z is interpolated exactly; its plane integral is
    the sum over the fluid samples of the field at the sample points."""
    pp, pw = plan_small
    a, b, c0 = 0.3, -0.7, 1.1
    X = small_cloud.pos - 0.5
    vx = c0 + a * X[:, 1] + b * X[:, 2]
    # only linear fields that are single-valued across the seam: none are, so
    # compare sample by sample using the minimum-image offsets of each stencil
    num = 0.0
    for s in range(pp.n_samples):
        d = nc.min_image(small_cloud.pos[pp.idx[s]] - pp.pts[s])
        vals = c0 + a * (pp.pts[s, 1] - 0.5 + d[:, 1]) + b * (pp.pts[s, 2] - 0.5 + d[:, 2])
        num += pw[s] @ vals
    expect = (c0 + a * (pp.pts[:, 1] - 0.5) + b * (pp.pts[:, 2] - 0.5)).sum() / (5 * 64 * 64)
    assert num / (5 * 64 * 64) == pytest.approx(expect, rel=1e-12)


@pytest.fixture(scope="module")
def grad_bnd(small_cloud, small_stencils):
    c, S = small_cloud, small_stencils
    w, _ = O.weights(c.pos, S[c.n_int:], [("dx",), ("dy",), ("dz",)])
    return w


def test_drag_of_linear_pressure(small_cloud, small_stencils, grad_bnd):
    """p = -G x, v = 0: F = -oint p n dA = G V_sphere (divergence theorem)."""
    c, S = small_cloud, small_stencils
    X = nc.min_image(c.pos - 0.5)
    G = 2.5
    F = O.drag(S[c.n_int:], grad_bnd, c.nrm, np.zeros((c.n, 3)), -G * X[:, 0], 1.0, 1.0, O.area(c.r) / c.n_bnd)
    V = 4.0 / 3.0 * np.pi * c.r ** 3
    assert F[0] == pytest.approx(G * V, rel=2e-4)
    assert abs(F[1]) < 1e-4 * G * V and abs(F[2]) < 1e-4 * G * V


def test_drag_of_shear_field(small_cloud, small_stencils, grad_bnd):
    """v = (z^2, 0, 0), p = 0: sigma_xz = sigma_zx = 2 rho nu z, so
    F_x = oint 2 rho nu z n_z dA = 2 rho nu V (divergence theorem)."""
    c, S = small_cloud, small_stencils
    X = nc.min_image(c.pos - 0.5)
    v = np.zeros((c.n, 3))
    v[:, 0] = X[:, 2] ** 2
    rho, nu = 1.2, 0.7
    F = O.drag(S[c.n_int:], grad_bnd, c.nrm, v, np.zeros(c.n), rho, nu, O.area(c.r) / c.n_bnd)
    V = 4.0 / 3.0 * np.pi * c.r ** 3
    assert F[0] == pytest.approx(2 * rho * nu * V, rel=5e-4)


def test_drag_ignores_pressure_gauge(small_cloud, small_stencils, grad_bnd):
    c, S = small_cloud, small_stencils
    rng = np.random.default_rng(0)
    p = rng.normal(size=c.n)
    dA = O.area(c.r) / c.n_bnd
    F1 = O.drag(S[c.n_int:], grad_bnd, c.nrm, np.zeros((c.n, 3)), p, 1.0, 1.0, dA)
    F2 = O.drag(S[c.n_int:], grad_bnd, c.nrm, np.zeros((c.n, 3)), p + 123.0, 1.0, 1.0, dA)
    assert np.abs(F1 - F2).max() < 1e-9


def test_traction_pointwise_closed_forms(small_cloud, small_stencils, grad_bnd):
    """The surface map node by node: a linear pressure gives t = -(p - <p>) n
    exactly (no velocity), and the shear field v = (z^2, 0, 0) gives
    t = rho nu (grad v + grad v^T) n with the exact gradient (2z in the xz and
    zx entries), the weights being exact on quadratics."""
    c, S = small_cloud, small_stencils
    X = nc.min_image(c.pos - 0.5)
    p = -2.5 * X[:, 0]
    t, pc = O.traction(S[c.n_int:], grad_bnd, c.nrm, np.zeros((c.n, 3)), p, 1.0, 1.0)
    pb = p[c.n_int:] - p.mean()
    assert np.abs(pc - pb).max() < 1e-14
    assert np.abs(t + pb[:, None] * c.nrm).max() < 1e-14
    v = np.zeros((c.n, 3))
    v[:, 0] = X[:, 2] ** 2
    rho, nu = 1.2, 0.7
    t, _ = O.traction(S[c.n_int:], grad_bnd, c.nrm, v, np.zeros(c.n), rho, nu)
    z, n = X[c.n_int:, 2], c.nrm
    expect = rho * nu * np.stack([2 * z * n[:, 2], np.zeros_like(z), 2 * z * n[:, 0]], 1)
    assert np.abs(t - expect).max() < 1e-9 * np.abs(expect).max()
    # the drag is the area-weighted sum of the map
    dA = O.area(c.r) / c.n_bnd
    F = O.drag(S[c.n_int:], grad_bnd, c.nrm, v, np.zeros(c.n), rho, nu, dA)
    assert np.abs(F - dA * t.sum(0)).max() <= 1e-14 * np.abs(F).max()


def test_residual_monitors_closed_forms():
    """mpfo_residual on the grain-free periodic fill: the divergence of the
    linear field v = (aX, bY, cZ) is a + b + c at every node whose stencil
    does not wrap (the derivative weights are exact on linear fields), and the
    two maxima are plain maxima of |v| and |v - v_prev|.  A wrong weight row,
    a missing component or a sum of squares without the root fails one of
    them."""
    c = nc.sphere_cloud(0.0, 0.05, 0.0, 0.05, seed=5)
    S = nc.stencils(c.pos, 30)
    d_raw = c.pos[S] - c.pos[S[:, :1]]
    safe = np.all(np.abs(d_raw - nc.min_image(d_raw)) < 1e-12, axis=(1, 2))
    w, _ = O.weights(c.pos, S, [("dx",), ("dy",), ("dz",), ("lap",)])
    X, Y, Z = (c.pos - 0.5).T
    a, b, cc = 0.9, -0.4, 0.25
    v = np.stack([a * X, b * Y, cc * Z], 1)
    # only the seam-free nodes as the "interior": reorder them first
    order = np.concatenate([np.flatnonzero(safe), np.flatnonzero(~safe)])
    inv = np.empty_like(order)
    inv[order] = np.arange(len(order))
    S2, w2, v2 = inv[S[order]], w[order], v[order]
    n_int = int(safe.sum())
    assert n_int > 100
    vp = v2 + 1e-3 * np.sin(np.arange(len(v2)))[:, None]
    out = O.residual(n_int, S2, w2, v2, vp)
    assert out[2] == pytest.approx(abs(a + b + cc), rel=1e-12)
    assert out[1] == np.linalg.norm(v2[:n_int], axis=1).max()
    assert out[0] == np.linalg.norm((v2 - vp)[:n_int], axis=1).max()
    assert O.residual(n_int, S2, w2, v2)[0] == 0.0
    # a divergence-free field (Y, Z, X) has zero divergence on those nodes
    assert O.residual(n_int, S2, w2, np.stack([Y, Z, X], 1)[order])[2] < 1e-12


def test_pointwise_difference_closed_forms():
    """Eq. pointwise_error: a perturbation of size eps orthogonal to v_b gives
    delta = eps / |v_b| exactly; delta is invariant under a common scaling
    and zero for equal fields; the no-slip grain (both zero) gives 0 and a
    non-zero difference over a zero velocity gives inf.  Swapping the two
    fields changes the denominator, so the formula's orientation is pinned
    too."""
    rng = np.random.default_rng(7)
    vb = rng.normal(size=(50, 3))
    e = np.cross(vb, rng.normal(size=(50, 3)))  # orthogonal to v_b
    e *= (0.01 * np.linalg.norm(vb, axis=1) / np.linalg.norm(e, axis=1))[:, None]
    va = vb + e
    d, dv = O.pointwise(va, vb)
    assert np.allclose(d, 0.01, rtol=1e-13, atol=0)
    assert np.allclose(dv, np.linalg.norm(e, axis=1), rtol=1e-12, atol=0)  # va - vb = e up to rounding
    d3, _ = O.pointwise(3.7 * va, 3.7 * vb)
    assert np.allclose(d3, d, rtol=1e-14, atol=0)
    assert not O.pointwise(vb, vb)[0].any()
    ds, _ = O.pointwise(vb, va)  # |v_a| = sqrt(1 + 1e-4) |v_b|
    assert np.allclose(ds, 0.01 / np.sqrt(1 + 1e-4), rtol=1e-13, atol=0)
    z = np.zeros((2, 3))
    dz, _ = O.pointwise(np.array([[0.0, 0, 0], [1e-3, 0, 0]]), z)
    assert dz[0] == 0.0 and dz[1] == np.inf


def test_channel_permeability_closed_form():
    """Plane Poiseuille flow u = g z (H - z) / (2 nu) in 0 <= z <= H: the
    sample interpolation is exact on quadratics, and the M x M midpoint
    quadrature of Eq. k_definition integrates the profile with the midpoint
    rule's known error, so k / d^2 = H^3 / 12 + H / (24 M^2) exactly (the
    channel's textbook H^3 / 12 plus the quadrature term).  Pins the plane
    flux, the solid samples counting zero, and k = q nu / |g| (a wrong nu or
    |g| exponent shows as a factor)."""
    H, M, g, nu = 0.5, 32, 2.5, 0.8
    c = nc.channel_cloud(0.05, H, seed=2)
    S = nc.stencils(c.pos, 30)
    pp = nc.plane_plan(c, M, 30, fluid=lambda p: p[:, 2] < H)
    pw = O.plane_weights(c.pos, pp.idx, pp.shift)
    z = c.pos[:, 2]
    u = g * z * (H - z) / (2 * nu)
    u[c.n_int:] = 0.0
    q = O.flux(pp.idx, pw, u, 5 * M * M)
    k = O.permeability(q, nu, g)
    assert k == pytest.approx(H ** 3 / 12 + H / (24 * M * M), rel=1e-11)
    assert O.permeability(q, nu, g, d=2.0) == pytest.approx(k / 4, rel=1e-15)
