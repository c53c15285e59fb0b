"""Oracle ACM Navier-Stokes step (Sec. 2.3) pinned by closed forms."""
import numpy as np
import pytest

import nodecloud as nc
import oracle as O
from oracle.steady import steady_solve


@pytest.fixture(scope="module")
def channel():
    c = nc.channel_cloud(0.1, 0.5, seed=0)
    S = nc.stencils(c.pos, 30)
    Sn = nc.neumann_stencils(c, 30)
    return c, S, Sn


def poiseuille(c, H=0.5, g=1.0, nu=1.0):
    z = c.pos[:, 2]
    u = g * z * (H - z) / (2.0 * nu)
    u[c.n_int:] = 0.0
    return u


def test_poiseuille_is_a_fixed_point(channel):
    """Weights are exact on quadratics, so the plane Poiseuille profile, with
    constant pressure, is reproduced exactly by every term of the step."""
    c, S, Sn = channel
    a = O.ACM(c.pos, c.n_int, S, c.nrm, sten_n=Sn, h_min=0.05, v_ref=1e-3)
    u = poiseuille(c)
    a.v[:, 0] = u
    a.run(50)
    assert np.abs(a.v[:, 0] - u).max() < 1e-12 * u.max()
    assert np.abs(a.v[:, 1:]).max() < 1e-12 * u.max()
    assert np.ptp(a.p) < 1e-10


def test_direct_steady_solve_gives_poiseuille(channel):
    c, S, Sn = channel
    w, _ = O.weights(c.pos, S, [("dx",), ("dy",), ("dz",), ("lap",)])
    wn, _ = O.weights(c.pos, Sn, [("dn",)], rowvec=c.nrm)
    v, p, kappa = steady_solve(c.n_int, S, w, Sn, wn[:, 0, :])
    u = poiseuille(c)
    assert np.abs(v[:, 0] - u).max() < 1e-11 * u.max()
    assert abs(kappa) < 1e-10


@pytest.fixture(scope="module")
def box():
    """Periodic fill without a grain, and the nodes whose whole stencil sits
    away from the periodic seam (there a polynomial field is single-valued)."""
    c = nc.sphere_cloud(0.0, 0.05, 0.0, 0.05, seed=5)
    S = nc.stencils(c.pos, 30)
    d_raw = c.pos[S] - c.pos[S[:, :1]]
    safe = np.all(np.abs(d_raw - nc.min_image(d_raw)) < 1e-12, axis=(1, 2))
    return c, S, safe


def test_predictor_terms_exact_on_quadratics(box):
    """With beta = 0 the coupling is inert and one step is the intermediate
    velocity of Eq. MNS_intermediate; for v = (Y^2, Z^2, X^2) the Laplacian
    and the gradients are exact, so v' has a closed form."""
    c, S, safe = box
    X, Y, Z = (c.pos - 0.5).T
    g = np.array([0.7, -0.2, 0.1])
    a = O.ACM(c.pos, c.n, S, np.zeros((0, 3)), dt=1e-4, nu=0.9, beta=0.0, v_ref=1.0, g=g, n_p=1)
    a.v[:] = np.stack([Y * Y, Z * Z, X * X], 1)
    v0 = a.v.copy()
    a.run(1)
    lap = np.array([2.0, 2.0, 2.0])
    adv = np.stack([Z * Z * 2 * Y, X * X * 2 * Z, Y * Y * 2 * X], 1)  # (v . grad) v
    expect = v0 + 1e-4 * (0.9 * lap - adv + g)
    assert safe.sum() > 100
    assert np.abs(a.v[safe] - expect[safe]).max() < 1e-13


def test_pressure_gradient_exact_on_quadratics(box):
    """From rest, without forcing, one coupling iteration turns a quadratic
    pressure q into v = -(dt/rho) grad q (Eq. MNS_velocity) and leaves p
    unchanged (Eq. MNS_pressure with div v' = 0)."""
    c, S, safe = box
    X, Y, Z = (c.pos - 0.5).T
    a = O.ACM(c.pos, c.n, S, np.zeros((0, 3)), dt=2e-4, rho=1.3, g=(0, 0, 0), n_p=1)
    q = X * X + X * Y - 0.5 * Z * Z
    a.p[:] = q
    a.run(1)
    gq = np.stack([2 * X + Y, X, -Z], 1)
    assert np.abs(a.v[safe] + 2e-4 / 1.3 * gq[safe]).max() < 1e-14
    assert np.array_equal(a.p, q)
    # Eq. MNS_C from the new velocity
    assert a.C[0] == pytest.approx(10.0 * max(np.linalg.norm(a.v, axis=1).max(), 1.0), rel=1e-15)


def test_rest_without_force_stays_at_rest(small_cloud, small_stencils):
    c, S = small_cloud, small_stencils
    a = O.ACM(c.pos, c.n_int, S, c.nrm, sten_n=nc.neumann_stencils(c, 30), h_min=0.02, g=(0, 0, 0))
    a.run(5)
    assert not a.v.any() and not a.p.any()


def test_time_steps_match_paper_footnotes():
    rows = [l.split() for l in open(__file__.replace("test_oracle_acm.py", "golden/timestep_paper.txt"))
            if l.strip() and not l.startswith("#")]
    for solver, h, dt, tol in rows:
        h, dt, tol = float(h), float(dt), float(tol)
        got = O.acm_dt(h, 1.0) if solver == "acm" else O.lbm_units(h, 1.0, 1.0, (0, 0, 0), 1.0)["dt"]
        assert abs(got - dt) <= tol * dt, (solver, h, got, dt)


# --- the entropically damped pressure equation (the remedy Sec. 2.3 names) ---

def test_edac_keeps_poiseuille_a_fixed_point(channel):
    """Constant pressure has no gradient and no Laplacian, so the damping and
    advection terms vanish and the Poiseuille profile stays exact."""
    c, S, Sn = channel
    a = O.ACM(c.pos, c.n_int, S, c.nrm, sten_n=Sn, h_min=0.05, v_ref=1e-3, edac=True)
    u = poiseuille(c)
    a.v[:, 0] = u
    a.run(50)
    assert np.abs(a.v[:, 0] - u).max() < 1e-12 * u.max()
    assert np.ptp(a.p) < 1e-10


def stencil_safe(S, safe):
    """Nodes whose own stencil and every neighbour's stencil avoid the seam."""
    return safe & safe[S].all(1)


def test_edac_pressure_diffusion_exact_on_quadratics(box):
    """From rest without forcing (div v' = 0, v' = 0) one coupling iteration
    gives p = q + dt nu lap q with lap q = 2 - 1 = 1, and then v = -(dt/rho)
    grad q (the added constant has no gradient)."""
    c, S, safe = box
    X, Y, Z = (c.pos - 0.5).T
    dt, nu, rho = 2e-4, 0.7, 1.3
    a = O.ACM(c.pos, c.n, S, np.zeros((0, 3)), dt=dt, nu=nu, rho=rho, g=(0, 0, 0), n_p=1, edac=True)
    q = X * X + X * Y - 0.5 * Z * Z
    a.p[:] = q
    a.run(1)
    assert np.abs(a.p[safe] - (q[safe] + dt * nu * 1.0)).max() < 1e-14
    s2 = stencil_safe(S, safe)
    assert s2.sum() > 50
    gq = np.stack([2 * X + Y, X, -Z], 1)
    assert np.abs(a.v[s2] + dt / rho * gq[s2]).max() < 1e-13


def test_edac_pressure_advection_exact_on_quadratics(box):
    """With beta = 0 the compressibility term is off (C = 0) and a
    divergence-free quadratic v = (Y^2, Z^2, X^2) is advanced by the closed form
    of the predictor; the pressure then moves by dt (-v' . grad q + nu lap q)."""
    c, S, safe = box
    X, Y, Z = (c.pos - 0.5).T
    dt, nu = 1e-4, 0.9
    g = np.array([0.7, -0.2, 0.1])
    a = O.ACM(c.pos, c.n, S, np.zeros((0, 3)), dt=dt, nu=nu, beta=0.0, v_ref=1.0, g=g, n_p=1, edac=True)
    v0 = np.stack([Y * Y, Z * Z, X * X], 1)
    a.v[:] = v0
    q = X * X + X * Y - 0.5 * Z * Z
    a.p[:] = q
    a.run(1)
    adv = np.stack([Z * Z * 2 * Y, X * X * 2 * Z, Y * Y * 2 * X], 1)
    vp = v0 + dt * (nu * 2.0 - adv + g)
    gq = np.stack([2 * X + Y, X, -Z], 1)
    expect = q + dt * (-(vp * gq).sum(1) + nu * 1.0)
    assert np.abs(a.p[safe] - expect[safe]).max() < 1e-13
    # the plain method leaves p alone here (C = 0)
    b = O.ACM(c.pos, c.n, S, np.zeros((0, 3)), dt=dt, nu=nu, beta=0.0, v_ref=1.0, g=g, n_p=1)
    b.v[:] = v0
    b.p[:] = q
    b.run(1)
    assert np.array_equal(b.p, q)


def test_nominal_step_on_a_jittered_channel_is_not_stable():
    """The time step 0.1 h_min^2 / (2 nu) of Sec. 2.3 is not stable on every
    node set.  On a plane channel filled with a jittered lattice (jitter
    h / 4) the predictor's RBF-FD Laplacian has a mode that grows by about
    1.6 per step at that step, with or without the pressure coupling, so the
    Poiseuille fixed point is lost within tens of steps; at half the step it
    holds to rounding.  (The sphere-cell clouds of the workloads run stably
    for millions of steps at the nominal step.)"""
    c = nc.channel_cloud(0.02, 0.5, seed=3)
    S, Sn = nc.solver_stencils(c, 30), nc.neumann_stencils(c, 30)
    z = c.pos[:, 2]
    u = z * (0.5 - z) / 2.0
    u[c.n_int:] = 0.0
    dev = {}
    for name, dt in (("nominal", O.acm_dt(c.h_min, 1.0)), ("half", 0.5 * O.acm_dt(c.h_min, 1.0))):
        a = O.ACM(c.pos, c.n_int, S, c.nrm, sten_n=Sn, dt=dt, v_ref=1e-3, beta=0.0)
        a.v[:, 0] = u
        a.run(40)
        dev[name] = np.abs(a.v[:, 0] - u).max() / u.max()
    assert dev["nominal"] > 1e-9  # grown by six orders of magnitude from rounding
    assert dev["half"] < 1e-13


# --- pins of the pressure update (Eq. MNS_pressure) and the Neumann pass ---

def test_pressure_update_coefficient_on_a_linear_field(box):
    """Eq. MNS_pressure with C != 0 and div v' != 0.  From v = (aX, bY, cZ)
    without forcing the predictor is exact: the Laplacian vanishes and
    (v . grad) v = (a^2 X, b^2 Y, c^2 Z), so v' = (a(1 - dt a) X, ...) and
    div v' = a(1 - dt a) + b(1 - dt b) + c(1 - dt c).  The first pressure
    update then gives p = -dt C^2 rho div v' with C = beta |v_ref| (the sound
    speed before the first correction).  Mistakes this catches: C for C^2, a
    dropped rho, div v instead of div v', one divergence term taken from the
    wrong weight row (a transposed operand) and a sign error."""
    c, S, safe = box
    X, Y, Z = (c.pos - 0.5).T
    dt, rho, beta, v_ref = 1e-3, 1.3, 2.0, 0.7
    a_, b_, c_ = 0.9, -0.4, 0.25
    o = O.ACM(c.pos, c.n, S, np.zeros((0, 3)), dt=dt, rho=rho, beta=beta, v_ref=v_ref, g=(0, 0, 0), n_p=1)
    o.v[:] = np.stack([a_ * X, b_ * Y, c_ * Z], 1)
    o.run(1)
    div = a_ * (1 - dt * a_) + b_ * (1 - dt * b_) + c_ * (1 - dt * c_)
    C = beta * v_ref
    expect = -dt * C * C * rho * div
    s2 = stencil_safe(S, safe)  # v' is exact at every stencil node of these
    assert s2.sum() > 50
    assert np.abs(o.p[s2] - expect).max() < 1e-13 * abs(expect)
    # the alternatives named above all miss by far more than the bound
    for wrong in (-dt * C * rho * div, -dt * C * C * div, -dt * C * C * rho * (a_ + b_ + c_),
                  -dt * C * C * rho * (a_ * (1 - dt * a_) + 2 * b_ * (1 - dt * b_)), dt * C * C * rho * div):
        assert abs(wrong - expect) > 1e-6 * abs(expect)


def test_neumann_pass_reproduces_a_field_with_zero_normal_derivative():
    """The boundary update of the coupling iteration solves the discrete
    dp/dn = 0 row for the node's own pressure.  On the plane channel the
    normals are +-z, so any quadratic in x and y alone has zero normal
    derivative; the normal-derivative weights are exact on quadratics, and the
    solved value must be the field's own value at the wall node, whatever the
    wall held before.  From rest without forcing the interior pressure is
    untouched (div v' = 0), so one iteration isolates the pass.  A sign error
    in the solve gives -q at the wall, a wrong self weight a scaled q."""
    c = nc.channel_cloud(0.05, 0.5, seed=4)
    S, Sn = nc.solver_stencils(c, 30), nc.neumann_stencils(c, 30)
    X, Y = c.pos[:, 0] - 0.5, c.pos[:, 1] - 0.5
    q = 1.0 + X * X - 0.5 * X * Y + 0.3 * Y + 0.2 * X - 0.7 * Y * Y
    o = O.ACM(c.pos, c.n_int, S, c.nrm, sten_n=Sn, dt=1e-5, g=(0, 0, 0), n_p=1)
    o.p[:] = q
    o.p[c.n_int:] = 123.0  # the old wall values must not matter
    o.run(1)
    # wall nodes whose Neumann stencil does not wrap in x or y
    d_raw = c.pos[Sn] - c.pos[Sn[:, :1]]
    safe = np.all(np.abs(d_raw - nc.min_image(d_raw)) < 1e-12, axis=(1, 2))
    assert safe.sum() > 200
    pb = o.p[c.n_int:]
    qb = q[c.n_int:]
    assert np.abs(pb[safe] - qb[safe]).max() < 1e-12
    assert np.array_equal(o.p[:c.n_int], q[:c.n_int])  # interior untouched
