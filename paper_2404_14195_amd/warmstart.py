"""Learned warm start: a network trained on the solvers' own steady fields
predicts the steady velocity and pressure of a new cell, and the explicit
iteration starts from that prediction instead of rest.

This is an addition to the paper's method.  The cold-started solver remains
the reference: a warm-started run converges to the same steady state (the
steady state does not depend on the initial condition), so the prediction
only moves the starting point, and its error is measured against the cold
run's k.

Split of the prediction:
* the field shape comes from the MLP of ``mpf_mlp_*``: per-node features
  (offset from the grain centre, signed distance to the surface, porosity)
  -> (v / U, (p - <p>) / P);
* the magnitudes U = k(r) |g| / nu and P (the spread of p) of a cell come from
  a monotone cubic interpolation of log U and log P over the training radii,
  so every target the network sees is O(1) whatever the porosity.

Everything on the device runs in libmpf kernels; this module only holds the
parameters, shuffles sample indices and moves a few scalars.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import api
from ._lib import MPF_F32, MPF_MIXED


def _init_params(seed: int) -> np.ndarray:
    """U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for every weight and bias."""
    rng = np.random.default_rng(seed)
    sizes = (5, 128, 128, 128, 4)
    parts = []
    for i, o in zip(sizes[:-1], sizes[1:]):
        a = 1.0 / math.sqrt(i)
        parts += [rng.uniform(-a, a, o * i), rng.uniform(-a, a, o)]
    return np.concatenate(parts).astype(np.float32)


class _Pchip:
    """Monotone piecewise-cubic interpolation (Fritsch-Carlson slopes) of
    y(x) over sorted knots; linear extrapolation beyond the end knots."""

    def __init__(self, x, y):
        o = np.argsort(x)
        self.x = np.asarray(x, np.float64)[o]
        self.y = np.asarray(y, np.float64)[o]
        h = np.diff(self.x)
        d = np.diff(self.y) / h
        m = np.zeros_like(self.y)
        if len(self.x) == 2:
            m[:] = d[0]
        else:
            for i in range(1, len(self.x) - 1):
                if d[i - 1] * d[i] > 0:
                    w1, w2 = 2 * h[i] + h[i - 1], h[i] + 2 * h[i - 1]
                    m[i] = (w1 + w2) / (w1 / d[i - 1] + w2 / d[i])
            m[0], m[-1] = d[0], d[-1]
        self.m = m

    def __call__(self, x):
        x = float(x)
        xs, ys, ms = self.x, self.y, self.m
        if x <= xs[0]:
            return ys[0] + ms[0] * (x - xs[0])
        if x >= xs[-1]:
            return ys[-1] + ms[-1] * (x - xs[-1])
        i = int(np.searchsorted(xs, x)) - 1
        h = xs[i + 1] - xs[i]
        t = (x - xs[i]) / h
        h00, h10 = 2 * t ** 3 - 3 * t ** 2 + 1, t ** 3 - 2 * t ** 2 + t
        h01, h11 = -2 * t ** 3 + 3 * t ** 2, t ** 3 - t ** 2
        return h00 * ys[i] + h10 * h * ms[i] + h01 * ys[i + 1] + h11 * h * ms[i + 1]


def steady_fields(solver, check=500, tol=1e-6, max_steps=1_000_000, log=None, log_every=20.0):
    """Run a solver until k changes by less than tol (relative) over two
    successive checks; returns (k, steps).  Raises FloatingPointError if k
    stops being finite and RuntimeError if max_steps pass first."""
    ks = []
    t_log = time.perf_counter()
    while solver.steps < max_steps:
        solver.run(check)
        ks.append(solver.permeability())
        if not math.isfinite(ks[-1]):
            raise FloatingPointError(f"k is {ks[-1]} after {solver.steps} steps")
        if len(ks) > 2 and all(abs(ks[-i] - ks[-i - 1]) <= tol * abs(ks[-1]) for i in (1, 2)):
            return ks[-1], solver.steps
        if log and time.perf_counter() - t_log > log_every:
            log(f"steady: {solver.steps} steps, k = {ks[-1]:.8e}")
            t_log = time.perf_counter()
    raise RuntimeError(f"k not steady after {solver.steps} steps (last {ks[-3:]})")


def steady_fields_many(solvers, check=500, tol=1e-6, max_steps=1_000_000, log=None, log_every=20.0):
    """steady_fields for several solvers at once, each on a stream of its own
    (default priority): small cells leave most of the chip idle, and their
    launches overlap this way.  Every solver takes exactly the steps and
    checks it would take alone, so the results are the same bit for bit.
    Returns [(k, steps)] in the solvers' order."""
    streams = [torch.cuda.Stream() for _ in solvers]
    torch.cuda.synchronize()  # set-up ran on the default stream
    # no end-of-call flag check (it waits for the stream and would serialise
    # the cells); a non-finite k below still stops the run
    checks = [s.check for s in solvers]
    for s in solvers:
        s.check = False
    try:
        return _steady_many(solvers, streams, check, tol, max_steps, log, log_every)
    finally:
        for s, c in zip(solvers, checks):
            s.check = c


def _steady_many(solvers, streams, check, tol, max_steps, log, log_every):
    ks = [[] for _ in solvers]
    out = [None] * len(solvers)
    t_log = time.perf_counter()
    while any(o is None for o in out):
        live = [i for i, o in enumerate(out) if o is None]
        for i in live:
            if solvers[i].steps >= max_steps:
                raise RuntimeError(f"k not steady after {solvers[i].steps} steps (last {ks[i][-3:]})")
            with torch.cuda.stream(streams[i]):
                solvers[i].run(check)
        for i in live:
            with torch.cuda.stream(streams[i]):
                ks[i].append(solvers[i].permeability())
            k = ks[i]
            if not math.isfinite(k[-1]):
                raise FloatingPointError(f"k is {k[-1]} after {solvers[i].steps} steps")
            if len(k) > 2 and all(abs(k[-j] - k[-j - 1]) <= tol * abs(k[-1]) for j in (1, 2)):
                out[i] = (k[-1], solvers[i].steps)
        if log and time.perf_counter() - t_log > log_every:
            log(f"steady: {sum(o is not None for o in out)} of {len(out)} cells settled")
            t_log = time.perf_counter()
    torch.cuda.synchronize()
    return out


class WarmStart:
    """The network, its optimiser state and the training set on the device."""

    def __init__(self, seed: int = 0, device="cuda"):
        self.device = torch.device(device)
        self.master = torch.as_tensor(_init_params(seed), device=self.device)
        self.packed = torch.empty(api.mlp_packed_count(), dtype=torch.bfloat16, device=self.device)
        api.mlp_pack(self.master, self.packed)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.grad = torch.empty_like(self.master)
        self.step = 0
        self.epochs_done = 0
        self._x, self._t = [], []
        self.radii, self.logU, self.logP = [], [], []
        self.X = self.T = None

    # ------------------------------------------------------------ data
    def add_cell(self, disc, v, p, k, g_abs=1.0, nu=1.0):
        """Add the steady state (v [3][n], p [n], device double, physical
        units) of one cell with permeability k as training samples."""
        c = disc.cloud
        U = k * g_abs / nu
        pc = p.double().cpu().numpy()
        pc = pc - pc.mean()
        P = float(np.sqrt((pc * pc).mean()))
        vh = v.double().cpu().numpy()
        t = np.empty((c.n, 4), dtype=np.float32)
        t[:, :3] = vh.T / U
        t[c.n_int:, :3] = 0.0  # no slip on the grain, as the state mapping imposes
        t[:, 3] = pc / P
        self._x.append(api.mlp_features(disc.pos, c.r, disc.phi))
        self._t.append(torch.as_tensor(t, device=self.device))
        self.radii.append(c.r)
        self.logU.append(math.log(U))
        self.logP.append(math.log(P))
        self.X = self.T = None

    def scales(self, r):
        """(U, P) of a cell of radius r, interpolated over the training cells."""
        return math.exp(_Pchip(self.radii, self.logU)(r)), math.exp(_Pchip(self.radii, self.logP)(r))

    @property
    def n_samples(self) -> int:
        return sum(x.shape[0] for x in self._x)

    # ------------------------------------------------------------ training
    def fit(self, epochs: int, batch: int = 8192, lr: float = 2e-3, lr_end: float = 1e-4, seed: int = 0,
            log=None, fused: bool = True):
        """Adam over shuffled minibatches, learning rate decayed
        geometrically from lr to lr_end.  Returns the mean loss per epoch (one
        host read per epoch).  fused: the fused training step
        (mpf_mlp_train_fused), else the separate forward/backward kernels."""
        if self.X is None:
            self.X = torch.cat(self._x).contiguous()
            self.T = torch.cat(self._t).contiguous()
        N = self.X.shape[0]
        ws = api.mlp_fused_workspace(batch, self.device) if fused else api.mlp_train_workspace(batch, self.device)
        train = api.mlp_train_fused if fused else api.mlp_train
        loss_sum = torch.zeros(1, dtype=torch.float64, device=self.device)
        per_epoch = max(1, N // batch)
        total = epochs * per_epoch
        ratio = (lr_end / lr) ** (1.0 / max(1, total - 1))
        perm = torch.empty(per_epoch * batch, dtype=torch.int64, device=self.device)
        hist = []
        t0 = time.perf_counter()
        for ep in range(epochs):
            api.shuffle_rows(N, per_epoch * batch, (seed << 32) + self.epochs_done, perm)
            self.epochs_done += 1
            rate = lr * ratio ** (ep * per_epoch)
            train(self.master, self.packed, self.m, self.v, self.grad, self.X, self.T, perm, batch, self.step, rate,
                  ratio, loss_sum, ws)
            self.step += per_epoch
            hist.append(loss_sum.item() / per_epoch)
            if log:
                log(f"epoch {ep + 1}/{epochs} loss {hist[-1]:.4e} ({time.perf_counter() - t0:.1f}s)")
        return hist

    # ------------------------------------------------------------ inference
    def predict(self, disc, ws=None):
        """Network outputs y [n][4] for the nodes of a cell."""
        c = disc.cloud
        x = api.mlp_features(disc.pos, c.r, disc.phi)
        y = torch.empty((c.n, 4), dtype=torch.float32, device=self.device)
        if ws is None:
            ws = api.mlp_workspace(c.n, False, self.device)
        api.mlp_forward(self.master, self.packed, x, y, ws)
        return y

    def state(self, disc, v, p, vmax=None, network: bool = True):
        """Predicted state of a cell into v [3][n], p [n] (and max |v|).

        The network gives the shape of the field and the interpolation over
        the training radii its magnitude; the velocity is then rescaled so that
        its flux through the permeability planes equals U = k(r) |g| / nu
        exactly.  The flux is the slowest-decaying part of the iteration's
        error, so it is the part worth pinning to the best estimate.

        network=False is the ablation without the network: the same magnitude
        and flux match applied to a shapeless field, a uniform velocity along
        the body force on the interior nodes (zero on the grain) and zero
        pressure, so that a run from it measures what the k(r) lookup and the
        flux matches alone give."""
        U, P = self.scales(disc.cloud.r)
        if network:
            y = self.predict(disc)
        else:
            y = torch.zeros((disc.n, 4), dtype=torch.float32, device=self.device)
            y[:, 0] = 1.0
        api.mlp_to_state(y, disc.n_int, U, P, v, p, vmax, disc.red_ws)
        q = float(api.flux_planes(disc.s_idx, disc.s_w, v[0], disc.n_all, ws=disc.red_ws).item())
        if q > 0.0 and math.isfinite(q):
            api.mlp_to_state(y, disc.n_int, U * U / q, P, v, p, vmax, disc.red_ws)

    def _flux_factor(self, disc, vx):
        """U / q for the current x-velocity, or None if q is not usable."""
        U, _ = self.scales(disc.cloud.r)
        q = float(api.flux_planes(disc.s_idx, disc.s_w, vx, disc.n_all, ws=disc.red_ws).item())
        return U / q if q > 0.0 and math.isfinite(q) else None

    def load_acm(self, solver, burn_in: int = 1000, network: bool = True):
        """Warm-start an ACMSolver in place (v, p and the running max |v|).

        After burn_in steps the velocity is rescaled once more so that its
        flux equals U: the prediction's shape error relaxes through fast modes
        in those steps and shifts the flux, and the slowest mode of the
        approach to steady state has the shape of the steady flow itself, so a
        uniform rescaling removes what the shift left in it.  solver.steps
        counts the burn-in."""
        self.state(solver.d, solver.v, solver.p, solver.vmax, network=network)
        solver.clear_compensation()
        solver.steps = 0
        if burn_in > 0:
            solver.run(burn_in)
            c = self._flux_factor(solver.d, solver.v[0])
            if c is not None:
                solver.scale_velocity(c)

    def load_mlbm(self, solver, burn_in: int = 1000, network: bool = True):
        """Warm-start an MLBMSolver: equilibrium populations of the predicted
        fields, then after burn_in steps the same flux match as load_acm (the
        populations are rebuilt as the equilibrium of the rescaled
        velocity and the current pressure).  solver.steps counts the burn-in.
        network=False: the ablation of state()."""
        d = solver.d
        v = torch.empty((3, d.n), dtype=torch.float64, device=self.device)
        p = torch.empty(d.n, dtype=torch.float64, device=self.device)
        self.state(d, v, p, network=network)
        solver.set_fields(v, p)
        if burn_in > 0:
            solver.run(burn_in)
            v, p = solver.macros()
            c = self._flux_factor(d, v[0])
            if c is not None:
                api.scale(v, c)
                solver.set_fields(v, p)
            solver.steps = burn_in

    # ------------------------------------------------------------ persistence
    def state_dict(self):
        return {"master": self.master.cpu().numpy(), "radii": np.array(self.radii), "logU": np.array(self.logU),
                "logP": np.array(self.logP)}

    def load_state_dict(self, sd):
        self.master.copy_(torch.as_tensor(np.asarray(sd["master"], np.float32)))
        api.mlp_pack(self.master, self.packed)
        self.radii, self.logU, self.logP = list(sd["radii"]), list(sd["logU"]), list(sd["logP"])


def solve_warm(model, make_solver, kind: str = "mlbm", band: float = 0.1, burn_in: int = 1000, check: int = 500,
               tol: float = 1e-7, max_steps: int = 1_000_000, network: bool = True):
    """Steady solve of one cell from the learned prediction, with the plain
    cold-started solver as its fallback.

    make_solver() builds a fresh solver of the cell (from rest).  The warm
    run loads the prediction (``load_mlbm`` or ``load_acm``: prediction,
    burn-in, flux match) and then runs until k changes by at most tol
    (relative) per check.  It is abandoned, and a fresh solver is run from
    rest to the same criterion instead, when the library reports a diverged
    state (MPFDiverged: a non-finite value or a stability limit), when k is
    not finite, or when k at any check leaves the band |k / U - 1| <= band
    around the network's own magnitude estimate U = k(r) (the prediction is
    then not the cell's flow).  Returns a dict with the solver used, k,
    steps, the (steps, k) history of the run that finished, and
    fallback/reason."""
    from ._lib import MPFDiverged
    if kind not in ("mlbm", "acm"):
        raise ValueError("kind is 'mlbm' or 'acm'")
    s = make_solver()
    U, _ = model.scales(s.d.cloud.r)

    def in_band(k):
        return math.isfinite(k) and abs(k / U - 1.0) <= band

    def settle(solver, hist, guard):
        while solver.steps < max_steps:
            solver.run(check)
            k = solver.permeability()
            hist.append((solver.steps, k))
            if not guard(k):
                return f"k = {k:.6e} after {solver.steps} steps"
            if len(hist) > 2 and abs(hist[-1][1] - hist[-2][1]) <= tol * abs(k):
                return None
        raise RuntimeError(f"k not steady after {solver.steps} steps")

    reason = None
    hist = []
    try:
        (model.load_mlbm if kind == "mlbm" else model.load_acm)(s, burn_in=burn_in, network=network)
        k0 = s.permeability()
        hist.append((s.steps, k0))
        reason = None if in_band(k0) else f"prediction k = {k0:.6e}, U(r) = {U:.6e}"
        if reason is None:
            reason = settle(s, hist, in_band)
    except MPFDiverged as e:
        reason = f"diverged: {e}"
    if reason is None:
        return {"solver": s, "k": hist[-1][1], "steps": s.steps, "history": hist, "fallback": False, "reason": None}
    s = make_solver()  # the plain solver from rest
    hist = []
    settle(s, hist, math.isfinite)
    return {"solver": s, "k": hist[-1][1], "steps": s.steps, "history": hist, "fallback": True, "reason": reason}


def training_radii(n: int, seed: int = 5, lo: float = 0.15, hi: float = 0.48, held_out=(0.18, 0.3, 0.33, 0.47),
                   gap: float = 0.01, exclude=()):
    """n radii stratified over [lo, hi] without the gap-neighbourhoods of the
    held-out radii and the intervals in exclude: that allowed set, of total
    length L, is cut into n equal parts of length L / n measured along it,
    and one uniform draw (seeded) is taken in each part.  (A stratum of
    [lo, hi] itself can lie entirely inside an excluded neighbourhood once
    L / n < 2 gap.)  The default range stays below 1/2, where neighbouring
    grains of the simple-cubic array touch."""
    cuts = [(max(lo, h - gap), min(hi, h + gap)) for h in held_out if h + gap > lo and h - gap < hi]
    cuts += [(max(lo, a), min(hi, b)) for a, b in exclude if b > lo and a < hi]
    cuts.sort()
    ivals, a = [], lo
    for c0, c1 in cuts:
        if c0 > a:
            ivals.append((a, c0))
        a = max(a, c1)
    if a < hi:
        ivals.append((a, hi))
    if not ivals:
        raise ValueError("the held-out neighbourhoods cover the whole range")
    length = sum(b - a for a, b in ivals)
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        u = (i + rng.uniform()) * length / n
        for a, b in ivals:
            if u < b - a or (a, b) == ivals[-1]:
                out.append(float(a + min(u, b - a)))
                break
            u -= b - a
    return out


__all__ = ["WarmStart", "solve_warm", "steady_fields", "training_radii", "MPF_F32", "MPF_MIXED"]
