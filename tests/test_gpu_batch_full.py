"""The batched weight solve at its full benchmark size: the eight cells of
bench.py --weights-batch (21.6M rows, N_L = 30, four operators) in one launch,
FP64 direct and FP32 factors with FP64 refinement.  Every 1000th row of every
cell is checked against the oracle, whose stencils come from the host fixture
(so the GPU stencils of those rows are checked too)."""
import importlib.util
import os
import sys
import time

import numpy as np
import pytest

import nodecloud as nc
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(m):
    print(f"[batch-full] {m}", flush=True)
    sys.stdout.flush()


def test_batched_weights_full_size_sampled():
    from paper_2404_14195_amd import api
    assert torch.cuda.is_available()
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    t0 = time.perf_counter()
    # threads, not processes: this process already holds a GPU context
    _, cells = bench.batch_cells(workers=8, context="threads")
    say(f"{sum(n for _, n in cells)} nodes in 8 cells, fill {time.perf_counter() - t0:.0f}s")
    ops = [("dx",), ("dy",), ("dz",), ("lap",)]
    clouds, samples = [], []
    for pos, n in cells:
        p = torch.as_tensor(np.ascontiguousarray(pos.T), device="cuda")
        clouds.append((p, api.knn(p, 30), None))
        rows = np.arange(0, n, 1000)
        samples.append((rows, nc.stencils(pos, 30, queries=pos[rows])))
        say(f"cell of {n} nodes: {len(rows)} sampled rows, host stencils ({time.perf_counter() - t0:.0f}s)")
    for c, (rows, s_host) in enumerate(samples):
        assert np.array_equal(clouds[c][1][:, rows].T.cpu().numpy(), s_host), c
    refs = [O.weights(pos, s_host, ops)[0] for (pos, _), (rows, s_host) in zip(cells, samples)]
    say(f"oracle weights of {sum(len(r) for r, _ in samples)} rows ({time.perf_counter() - t0:.0f}s)")
    for solve, tol in ((0, 1e-10), (1, 1e-9)):
        api.weights_autotune(clouds[0][0], clouds[0][1], ops, solve=solve, sample_rows=65536)
        res = api.rbffd_weights_batched(clouds, ops, solve=solve)
        torch.cuda.synchronize()
        worst = 0.0
        for c, (rows, _) in enumerate(samples):
            w64, _, info = res[c]
            assert not (info[rows].cpu().numpy() > 0).any()
            w = w64[:, :, rows].cpu().numpy().transpose(2, 0, 1)  # [rows][op][nl]
            scale = np.abs(refs[c]).max(2)
            worst = max(worst, float((np.abs(w - refs[c]).max(2) / scale).max()))
        say(f"solve {solve}: worst row error {worst:.2e} ({time.perf_counter() - t0:.0f}s)")
        assert worst < tol
        del res
        torch.cuda.empty_cache()


@pytest.mark.parametrize("precision, tol", [(0, 1e-11), (2, 1e-6)])
def test_acm_poiseuille_fixed_point_at_full_size(precision, tol):
    """A property that holds at any size, checked where the oracle cannot
    follow: plane Poiseuille flow between walls at z = 0 and H with constant
    pressure is an exact fixed point of the whole ACM step, every weight being
    exact on quadratics.  On a channel of about a million nodes the GPU step
    keeps it over 20 steps: to rounding in FP64, and to the rounding of the
    FP32 weights in mixed precision.  The step is half the nominal one: on
    this jittered lattice the nominal step lets a mode of the Laplacian grow
    (test_oracle_acm shows it on the oracle)."""
    from paper_2404_14195_amd.solvers import ACMSolver, Discretization
    c = nc.channel_cloud(0.008, 0.5, seed=3)
    assert c.n > 900_000
    d = Discretization(c, nl=30, M=16, plan=False)
    s = ACMSolver(d, precision=precision, v_ref=1e-3, dt=0.025 * c.h_min ** 2)
    z = c.pos[:, 2]
    u = z * (0.5 - z) / 2.0  # g = 1, nu = 1
    u[c.n_int:] = 0.0
    s.v[0].copy_(torch.as_tensor(u, dtype=s.v.dtype))
    s.vmax.fill_(float(u.max()))
    s.run(20)
    v = s.v.double().cpu().numpy()
    say(f"Poiseuille on {c.n} nodes, precision {precision}: max |dv_x| / max u = "
        f"{np.abs(v[0] - u).max() / u.max():.2e}")
    assert np.abs(v[0] - u).max() <= tol * u.max()
    assert np.abs(v[1:]).max() <= tol * u.max()
    p = s.p.double().cpu().numpy()
    assert np.ptp(p) <= tol * u.max()


def test_lbm_streamed_weights_parity():
    """The MLBM step on a cell whose weights exceed 512 MiB in every precision
    (about 280k nodes: 1.2 GB FP64, 0.6 GB FP32), where the step streams its
    weights past the caches.  The GPU runs with the oracle's weights from a
    state with O(1e-2) deviations from rest:
    * FP64: the oracle's own weights, within 1e-10 of the deviations plus the
      oracle's rounding floor, as on the small cells;
    * mixed (FP32 weights, FP64 state and arithmetic) and FP32: the oracle's
      weights rounded to FP32, with the oracle run on those same rounded
      values.  The GPU interpolates the shifted populations g = f - w_k and
      adds w_k back, which equals the oracle's sum of w_j f_j only where a
      row's weights sum to one: rounded weights miss that by a few 1e-8, so
      each step may differ by delta = max_k w_k |1 - sum_j w_j| (computed from
      the rounded weights; bound 10 delta per step, for the collision's
      mixing).  Beyond that, mixed differs only in FP64 summation order; FP32
      also stores g in FP32 and sums 30 FP32 products, which bounds its error
      by 5e-6 max|g| per step."""
    from paper_2404_14195_amd.solvers import Discretization, MLBMSolver
    q, nl = 19, 30
    c = nc.sphere_cloud(0.3, 0.0042, 0.16, 0.02, seed=4)
    assert (q - 1) * nl * c.n * 4 > 512 * 2 ** 20
    disc = Discretization(c, nl=nl, M=64)
    say(f"MLBM streamed weights: {c.n} nodes")
    o = O.MLBM(c.pos, c.n_int, disc.sten_host, c.nrm, q=q, h_min=c.h_min)
    e, wk, _ = O.lattice(q)
    rng = np.random.default_rng(11)
    rho0 = 1.0 + 0.01 * rng.normal(size=c.n)
    u0 = 0.02 * rng.normal(size=(c.n, 3))
    f0 = np.concatenate([O.equilibrium(q, 1, rho0[i], u0[i]) for i in range(c.n)])
    say("oracle weights and initial state done")

    def check(precision, tol_rel, floor, per_step=0.0):
        Wd = torch.as_tensor(np.ascontiguousarray(o.W[:, 1:, :].transpose(1, 2, 0)), device="cuda",
                             dtype=torch.float64 if precision == 0 else torch.float32)
        g = MLBMSolver(disc, q=q, precision=precision, W=Wd)
        g.set_populations(f0)
        o.f[:] = f0
        done = 0
        for steps in (1, 2):
            g.run(steps)
            o.run(steps)
            done += steps
            fg = g.populations()
            dev_max = np.abs(o.f - wk).max()
            err = np.abs(fg - o.f).max()
            tol = tol_rel * done * dev_max + floor(o.f, done) + per_step * done
            say(f"precision {precision}, {done} steps: max |df| = {err:.3e} (bound {tol:.3e}, max|g| {dev_max:.3e})")
            assert err <= tol, (precision, done, err, tol)
        del g, Wd
        torch.cuda.empty_cache()

    def floor64(f, steps):
        return 2 * np.finfo(np.float64).eps * np.abs(f).max() * steps

    check(0, 1e-10, floor64)
    o.W[:] = o.W.astype(np.float32).astype(np.float64)  # the FP32 weights, exactly, in FP64
    delta = float((wk[1:] * np.abs(1.0 - o.W[:, 1:, :].sum(axis=2))).max())
    say(f"FP32 weights: max_k w_k |1 - row sum| = {delta:.3e}")
    assert delta < 1e-8
    check(2, 1e-10, floor64, 10 * delta)
    check(1, 5e-6, lambda f, s: 0.0)
