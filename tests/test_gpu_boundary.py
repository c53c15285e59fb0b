"""The boundary's run-time signals and the compensated FP32 state, through the
C ABI on the GPU: the flags word and MPF_ERR_DIVERGED, the residual monitors
against the oracle, and MPF_F32_KAHAN against the FP64 oracle."""
import sys

import numpy as np
import pytest

import nodecloud as nc
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def announce(request):
    print(f"\n[gpu-case] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def api():
    from paper_2404_14195_amd import api as A
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return A


@pytest.fixture(scope="module")
def tiny():
    """r = 0.3, h 0.04 -> 0.1: 2,162 nodes, small enough for the oracle to
    reach steady state in seconds."""
    return nc.sphere_cloud(0.3, 0.04, 0.3, 0.1, seed=1)


@pytest.fixture(scope="module")
def disc_tiny(api, tiny):
    from paper_2404_14195_amd.solvers import Discretization
    return Discretization(tiny, nl=30, M=32)


def dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


# ----------------------------------------------------------------- flags word

@pytest.mark.parametrize("precision", [0, 1, 2, 3])
def test_acm_non_finite_state_is_reported(api, disc_tiny, precision):
    """A NaN planted in the state on the host reaches the velocity pass: the
    run returns MPF_ERR_DIVERGED with flags bit 0, and the running max is +inf
    (a NaN magnitude is not dropped by the max)."""
    from paper_2404_14195_amd import MPFDiverged
    from paper_2404_14195_amd.solvers import ACMSolver
    s = ACMSolver(disc_tiny, precision=precision)
    s.run(5)
    v = s.v.cpu()
    v[0, 17] = float("nan")
    s.v.copy_(v)
    with pytest.raises(MPFDiverged):
        s.run(3)
    assert int(s.flags.item()) & 1
    assert s.vmax.item() == float("inf")


def test_acm_courant_limit_is_reported(api, disc_tiny):
    """With a finite state but a stated h_min so small that C dt / h_min > 1,
    only bit 1 is raised."""
    from paper_2404_14195_amd import MPFDiverged
    from paper_2404_14195_amd.solvers import ACMSolver
    s = ACMSolver(disc_tiny, precision=0)
    s.run(3)  # C dt / h_min = 10 * 1e-3 * dt / h_min << 1: nothing raised
    assert int(s.flags.item()) == 0
    s.prm.h_min = 1e-3 * s.prm.dt * s.prm.beta * s.prm.v_ref  # C dt / h_min = 1000
    with pytest.raises(MPFDiverged):
        s.run(1)
    assert int(s.flags.item()) == 2
    assert np.isfinite(s.v.cpu().numpy()).all()


@pytest.mark.parametrize("precision", [0, 1, 2, 3])
def test_mlbm_non_finite_state_is_reported(api, disc_tiny, precision):
    from paper_2404_14195_amd import MPFDiverged
    from paper_2404_14195_amd.solvers import MLBMSolver
    s = MLBMSolver(disc_tiny, q=19, precision=precision)
    s.run(2)
    f = s.f.cpu()
    f[101, 3] = float("nan")
    s.f.copy_(f)
    with pytest.raises(MPFDiverged):
        s.run(2)
    assert int(s.flags.item()) & 1


def test_mlbm_lattice_speed_limit_is_reported(api, disc_tiny):
    """A uniform equilibrium at |u| = 0.7 > c_s: bit 1 only."""
    from paper_2404_14195_amd import MPFDiverged
    from paper_2404_14195_amd.solvers import MLBMSolver
    s = MLBMSolver(disc_tiny, q=19, precision=0)
    api.lbm_init(s.prm, s.f, 1.0, (0.7, 0.0, 0.0))
    with pytest.raises(MPFDiverged):
        s.run(1)
    assert int(s.flags.item()) == 2


def test_runs_without_flags_stay_quiet(api, disc_tiny):
    """No flags word, no check: the call returns normally and the NaN is left
    for the caller to find (here in k)."""
    from paper_2404_14195_amd.solvers import MLBMSolver
    s = MLBMSolver(disc_tiny, q=19, precision=0, check=False)
    f = s.f.cpu()
    f[5, 1] = float("nan")
    s.f.copy_(f)
    s.run(3)
    assert not np.isfinite(s.permeability())


# ----------------------------------------------------------------- residual

@pytest.mark.parametrize("precision", [0, 1, 2])
def test_residual_parity(api, disc_tiny, tiny, precision):
    """mpf_residual against mpfo_residual on a seeded smooth field and a
    seeded previous field (host inputs), each side with its own FP64 weights
    (FP32 copies on the GPU for FP32 weights)."""
    from paper_2404_14195_amd.solvers import ACMSolver
    c = tiny
    s = ACMSolver(disc_tiny, precision=precision)
    rng = np.random.default_rng(21)
    X = c.pos - 0.5
    v = np.stack([np.sin(2 * np.pi * X[:, 1]), np.cos(2 * np.pi * X[:, 2]), X[:, 0] ** 2], 1)
    v[c.n_int:] = 0.0
    vp = v + 1e-3 * rng.normal(size=v.shape)
    if precision == 1:  # the FP32 state holds the rounded values; so does the oracle's input
        v, vp = v.astype(np.float32).astype(np.float64), vp.astype(np.float32).astype(np.float64)
    dt = torch.float32 if precision == 1 else torch.float64
    out = api.residual(disc_tiny.sten, s.w, dev(v.T, dt), c.n_int, dev(vp.T, dt), precision).cpu().numpy()
    w_o, _ = O.weights(c.pos, disc_tiny.sten_host, [("dx",), ("dy",), ("dz",)])
    ref = O.residual(c.n_int, disc_tiny.sten_host, w_o, v, vp)
    tol = 1e-12 if precision == 0 else 2e-6
    print(f"[residual p{precision}] gpu={out} oracle={ref}", flush=True)
    assert out[0] == pytest.approx(ref[0], rel=1e-6 if precision == 1 else 1e-15)
    assert out[1] == pytest.approx(ref[1], rel=1e-6 if precision == 1 else 1e-15)
    assert out[2] == pytest.approx(ref[2], rel=tol)


# ----------------------------------------------------------------- compensated FP32

def _oracle_k(c, disc, o):
    v_o, _ = o.macros()
    pp = disc.plan
    return O.flux(pp.idx, O.plane_weights(c.pos, pp.idx, pp.shift), v_o[:, 0], disc.n_all)


def test_lbm_kahan_settles_with_the_fp64_oracle(api, disc_tiny, tiny):
    """14,000 steps from rest on the 2,162-node cell (k settled to 2e-8 in
    the oracle): the compensated FP32 state's permeability within 5e-6 of the
    FP64 oracle's.  The plain FP32 state is printed beside it; an explicit
    iteration whose state is rounded every step stops about tau ulp short of
    its fixed point (tau ~ 740 steps here, ~4e-5)."""
    from paper_2404_14195_amd import MPF_F32, MPF_F32_KAHAN
    from paper_2404_14195_amd.solvers import MLBMSolver
    c = tiny
    steps = 14000
    o = O.MLBM(c.pos, c.n_int, disc_tiny.sten_host, c.nrm, q=19, h_min=c.h_min)
    o.run(steps)
    k_o = _oracle_k(c, disc_tiny, o)
    ks = {}
    for name, prec in (("fp32", MPF_F32), ("kahan", MPF_F32_KAHAN)):
        g = MLBMSolver(disc_tiny, q=19, precision=prec)
        for _ in range(steps // 1000):
            g.run(1000)
        ks[name] = g.permeability()
    e32, ek = abs(ks["fp32"] / k_o - 1), abs(ks["kahan"] / k_o - 1)
    print(f"[lbm kahan steady] k64={k_o:.12e} fp32 err={e32:.2e} kahan err={ek:.2e}", flush=True)
    assert ek < 5e-6


def test_lbm_kahan_short_parity(api, disc_small, small_cloud):
    """200 steps from rest on the 8k-node cell within 1e-6 of the FP64
    oracle's permeability (the mixed-precision bound; plain FP32 meets 1e-4)."""
    from paper_2404_14195_amd import MPF_F32_KAHAN
    from paper_2404_14195_amd.solvers import MLBMSolver
    c = small_cloud
    g = MLBMSolver(disc_small, q=19, precision=MPF_F32_KAHAN)
    o = O.MLBM(c.pos, c.n_int, disc_small.sten_host, c.nrm, q=19, h_min=c.h_min)
    g.run(200)
    o.run(200)
    k_o, k_g = _oracle_k(c, disc_small, o), g.permeability()
    print(f"[lbm kahan] k={k_g:.12e} k64={k_o:.12e} rel={abs(k_g / k_o - 1):.3e}", flush=True)
    assert k_g == pytest.approx(k_o, rel=1e-6)
    # the state is f + comp: its populations track the oracle's closely
    fg = g.populations()
    assert np.abs(fg - o.f).max() < 1e-6 * np.abs(o.f - O.lattice(19)[1]).max() + 1e-9


@pytest.fixture(scope="module")
def disc_small(api, small_cloud):
    from paper_2404_14195_amd.solvers import Discretization
    return Discretization(small_cloud, nl=30, M=64)


def test_acm_kahan_parity_500_steps(api, disc_small, small_cloud):
    """The plain-ACM workload (8k nodes, 500 steps): the compensated FP32
    state's k within 1e-6 of the FP64 oracle (plain FP32 is held to 1e-4)."""
    from paper_2404_14195_amd import MPF_F32_KAHAN
    from paper_2404_14195_amd.solvers import ACMSolver
    c = small_cloud
    g = ACMSolver(disc_small, precision=MPF_F32_KAHAN)
    g.run(500)
    o = O.ACM(c.pos, c.n_int, disc_small.sten_host, c.nrm, sten_n=nc.neumann_stencils(c, 30), h_min=c.h_min,
              v_ref=1e-3)
    o.run(500)
    pp = disc_small.plan
    k_o = O.flux(pp.idx, O.plane_weights(c.pos, pp.idx, pp.shift), o.v[:, 0], disc_small.n_all)
    k_g = g.permeability()
    print(f"[acm kahan] k={k_g:.12e} k64={k_o:.12e} rel={abs(k_g / k_o - 1):.3e}", flush=True)
    assert k_g == pytest.approx(k_o, rel=1e-6)
    v_true = g.v.double().cpu().numpy() + g.comp[:3].double().cpu().numpy()
    assert np.abs(v_true.T - o.v).max() < 1e-5 * np.abs(o.v).max()


# ----------------------------------------------------------------- pointwise difference

@pytest.mark.parametrize("dta, dtb", [(np.float64, np.float64), (np.float32, np.float64), (np.float32, np.float32)])
def test_pointwise_difference_parity(api, dta, dtb):
    """Eq. pointwise_error element by element against the oracle on seeded
    fields (host inputs, rounded to each side's state type first), with zero
    rows for the no-slip nodes, and the isocontour counts exact."""
    rng = np.random.default_rng(13)
    n, n_int = 70_001, 60_000
    vb = rng.normal(size=(n, 3)) * rng.uniform(0.1, 2.0, size=(n, 1))
    va = vb + rng.normal(size=(n, 3)) * rng.uniform(1e-4, 1.0, size=(n, 1))
    va[n_int:] = vb[n_int:] = 0.0
    va[n_int + 3] = (1e-3, 0.0, 0.0)  # a difference over a zero velocity
    va, vb = va.astype(dta).astype(np.float64), vb.astype(dtb).astype(np.float64)
    tdt = {np.float64: torch.float64, np.float32: torch.float32}
    levels = (1.0, 0.25, 0.05, 0.1, 0.01)
    d, dv, counts = api.pointwise(dev(va.T, tdt[dta]), dev(vb.T, tdt[dtb]), n_count=n_int, levels=levels)
    d_o, dv_o = O.pointwise(va, vb)
    d, dv = d.cpu().numpy(), dv.cpu().numpy()
    fin = np.isfinite(d_o)
    assert np.array_equal(fin, np.isfinite(d)) and d[n_int + 3] == np.inf
    assert np.abs(d[fin] - d_o[fin]).max() <= 1e-14 * np.abs(d_o[fin]).max()
    assert np.abs(dv - dv_o).max() <= 1e-14 * np.abs(dv_o).max()
    assert counts == [int((d_o[:n_int] > t).sum()) for t in levels]


def test_compensated_moments_include_the_remainder():
    """The moments of a compensated FP32 MLBM state are those of hi + lo: the
    velocity equals the FP64 moments of hi + lo formed on the host from the
    two FP32 arrays (same shifted form) to 1e-13, while the FP32 values
    alone give a velocity that differs by more than 1e-10 (relative)."""
    import nodecloud as nc
    from paper_2404_14195_amd import MPF_F32_KAHAN, api
    from paper_2404_14195_amd.solvers import Discretization, MLBMSolver, lattice_vectors
    cloud = nc.sphere_cloud(0.3, 0.04, 0.3, 0.1, seed=1)
    d = Discretization(cloud, nl=30, M=32)
    s = MLBMSolver(d, q=19, precision=MPF_F32_KAHAN)
    s.run(300)
    v, _ = s.macros()
    v = v.cpu().numpy()
    ft = s.f[:, :19].double().cpu().numpy() + s.comp[:, :19].double().cpu().numpy()  # shifted, FP64
    e = np.array(lattice_vectors(19), dtype=np.float64)
    vs = s.units["vel_scale"]
    v_host = (vs * (ft @ e) / (1.0 + ft.sum(1))[:, None]).T
    scale = np.abs(v_host).max()
    assert np.abs(v - v_host).max() <= 1e-13 * scale
    v_hi = api.lbm_moments(s.prm, s.f, vs)[0].cpu().numpy()  # the FP32 values alone
    assert np.abs(v_hi - v_host).max() > 1e-10 * scale
