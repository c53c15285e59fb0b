"""Device-resident drivers for the two meshless solvers.

They hold the node cloud, stencils, weights and state in HBM and call the C
ABI (``api``) for every step of the computation, the unit conversions and the
reductions to k and K included; the host only launches and, at checks, reads
back one or three doubles.  Each run call hands the library a flags word (a
non-finite state or a stability limit) and raises MPFDiverged when it comes
back set, unless the solver's ``check`` is False."""
from __future__ import annotations

import math
import time

import numpy as np
import torch

import nodecloud

from . import api
from ._lib import MPF_F32, MPF_F32_KAHAN, MPF_F64, MPF_MIXED, AcmParams, LbmParams, MPFError

# state element type per precision (MPF_MIXED: FP32 weights, FP64 state)
_DT = {MPF_F64: torch.float64, MPF_F32: torch.float32, MPF_MIXED: torch.float64, MPF_F32_KAHAN: torch.float32}


class Discretization:
    """A node cloud on the device: positions [3][n], stencils [nl][n], the
    Neumann stencils of the boundary nodes [nl][nb], normals [3][nb] and the
    plane-sample plan of the permeability."""

    def __init__(self, cloud: nodecloud.Cloud, nl: int = 30, M: int = 64, device="cuda", plan: bool = True):
        self.cloud, self.nl, self.M = cloud, nl, M
        self.n, self.n_int, self.nb = cloud.n, cloud.n_int, cloud.n_bnd
        self.device = torch.device(device)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=self.device)
        self.pos = t(cloud.pos.T, torch.float64)
        # interior rows: nl nearest nodes; surface rows: self + nl - 1 nearest interior nodes
        self.sten = api.solver_stencils(self.pos, self.n_int, nl)
        self._sten_host = None
        self._tiles = None
        self._plans = {}
        self.nrm = t(cloud.nrm.T, torch.float64) if self.nb else torch.zeros((3, 0), dtype=torch.float64,
                                                                               device=self.device)
        # the Neumann rows and the drag's gradient rows use the surface stencils
        self.sn = self.sten[:, self.n_int:].contiguous()
        self.sb = self.sn
        if plan:
            pp = nodecloud.plane_plan(cloud, M, nl)
            self.plan = pp
            self.s_idx = t(pp.idx.T, torch.int32)
            self.s_shift = t(pp.shift.T, torch.float64)
            self.n_all = len(pp.planes) * M * M
            self.s_w = api.rbffd_weights(self.pos, self.s_idx, [("shift_row",)], rowvec=self.s_shift)[0][0].contiguous()
        self.phi, self.area = api.sc_cell(cloud.r) if cloud.r > 0 else (1.0, 0.0)
        self.red_ws = api.reduce_workspace(max(self.n, 5 * M * M), self.device)

    @property
    def tiles(self):
        """The tile plan (64-node tiles) of the stencils for the LDS-staged
        gather (built on first use, once per discretization)."""
        if self._tiles is None:
            try:
                self._tiles = api.TilePlan(self.sten)
            except MPFError:  # a halo over the default capacity: the largest the plan takes
                self._tiles = api.TilePlan(self.sten, h_cap=4096)
        return self._tiles

    def tiles_of(self, tile: int):
        """The tile plan with tiles of 64, 128 or 256 nodes (built on first
        use, once per discretization and size)."""
        if tile == 64:
            return self.tiles
        if tile not in self._plans:
            try:
                self._plans[tile] = api.TilePlan(self.sten, h_cap=16 * tile, tile=tile)
            except MPFError:
                self._plans[tile] = api.TilePlan(self.sten, h_cap=64 * tile, tile=tile)
        return self._plans[tile]

    @property
    def sten_host(self):
        """The same stencils [n][nl] from the host fixture (k-d tree), for
        checks that must not take their inputs from the GPU path."""
        if self._sten_host is None:
            self._sten_host = nodecloud.solver_stencils(self.cloud, self.nl)
        return self._sten_host


class ACMSolver:
    """Artificial-compressibility Navier-Stokes (Sec. 2.3) on a Discretization."""

    def __init__(self, disc: Discretization, precision: int = MPF_F64, nu=1.0, rho=1.0, dt=None, beta=10.0,
                 v_ref=1e-3, g=(1.0, 0.0, 0.0), n_p=3, lanes: int = 0, edac: bool = False, check: bool = True,
                 staged: bool = True, tile: int = 0):
        self.d, self.precision, self.check, self.staged = disc, precision, check, staged
        self.tile = tile or self._block_tile(lanes or self._default_lanes(disc.n_int, precision))
        dt = api.acm_dt(disc.cloud.h_min, nu) if dt is None else dt
        self.prm = AcmParams(nu=nu, rho=rho, dt=dt, beta=beta, v_ref=v_ref, g=(ctypesarr(g)), n_p=n_p,
                             precision=precision, lanes=lanes, edac=int(bool(edac)), h_min=disc.cloud.h_min)
        self.g = tuple(g)
        w64, w32, info = api.rbffd_weights(disc.pos, disc.sten, [("dx",), ("dy",), ("dz",), ("lap",)],
                                           want64=True, want32=precision != MPF_F64)
        wn64, wn32, infon = api.rbffd_weights(disc.pos, disc.sn, [("dn",)], rowvec=disc.nrm, want64=True,
                                              want32=precision != MPF_F64) if disc.nb else (None, None, None)
        self.info = info
        self.w64 = w64
        self.w = w64 if precision == MPF_F64 else w32
        self.wn = (wn64 if precision == MPF_F64 else wn32)[0].contiguous() if disc.nb else None
        self.wg = w64[:3, :, disc.n_int:].contiguous()
        dtp = _DT[precision]
        self.v = torch.zeros((3, disc.n), dtype=dtp, device=disc.device)
        self.p = torch.zeros(disc.n, dtype=dtp, device=disc.device)
        self.vmax = torch.zeros(1, dtype=torch.float64, device=disc.device)
        # compensation terms of v (rows 0-2) and p (row 3) of the compensated FP32 state
        self.comp = torch.zeros((4, disc.n), dtype=torch.float32, device=disc.device) \
            if precision == MPF_F32_KAHAN else None
        self.flags = torch.zeros(1, dtype=torch.int32, device=disc.device)
        self.ws = api.acm_workspace(disc.n, precision, disc.device)
        self.steps = 0

    @staticmethod
    def _block_tile(lanes: int) -> int:
        """The staged passes' tile: one tile per block of 256 lanes (256 nodes
        at one lane per node, 128 at two); 64 where the passes do not stage."""
        return {1: 256, 2: 128}.get(lanes, 64)

    @staticmethod
    def _default_lanes(n_int: int, precision: int) -> int:
        """The library's lanes per node when left to it (before the tile plan
        is considered): 8 up to 12k interior nodes, 2 up to 50k, then 1, and
        2 again above 500k for an FP64 state."""
        fp64 = precision in (MPF_F64, MPF_MIXED)
        return 8 if n_int <= 12000 else 2 if n_int <= 50000 else 2 if fp64 and n_int > 500000 else 1

    def run(self, n_steps: int):
        # the tile plan is built once per discretization and tile size; the
        # library stages where the lanes per node and the halos allow it
        tiles = self.d.tiles_of(self.tile) if self.staged else None
        api.acm_run(self.prm, self.d.n_int, self.d.sten, self.w, self.d.sn, self.wn, self.v, self.p, self.vmax,
                    n_steps, self.ws, comp=self.comp, flags=self.flags if self.check else None, tiles=tiles)
        self.steps += n_steps

    def staged_now(self) -> bool:
        """Whether run() takes the LDS-staged gather: a tile plan, one or two
        lanes per node (as the library picks them: 2 above 12k interior
        nodes, 1 above 50k, and 2 again above 500k for an FP64 state or where
        the halos fit LDS at two lanes but not at one) and a block's halos
        within 64 KiB."""
        if not self.staged:
            return False
        fp64 = self.precision in (MPF_F64, MPF_MIXED)
        rec, val = (32, 8) if fp64 else (16, 4)
        plan = self.d.tiles_of(self.tile)
        ts = getattr(plan, "tile", 64)
        fits = lambda lanes: (lanes <= 2 and ts * lanes <= 256 and
                              (256 // (ts * lanes)) * plan.h_max * (rec + val) <= 64 * 1024)
        lanes = self.prm.lanes or self._default_lanes(self.d.n_int, self.precision)
        if not self.prm.lanes and lanes == 1 and not fits(1) and fits(2):
            lanes = 2
        return fits(lanes)

    def clear_compensation(self):
        """After the state was set from outside (a warm start): the FP32
        values are the state, their compensation is zero."""
        if self.comp is not None:
            self.comp.zero_()

    def scale_velocity(self, c: float):
        """v *= c with its compensation and the running max (flux match)."""
        api.scale(self.v, c)
        if self.comp is not None:
            api.scale(self.comp[:3], c)
        api.scale(self.vmax, c)

    @property
    def time_step(self) -> float:
        """Physical time per step (Sec. 2.3: 0.1 h_min^2 / (2 nu) by default)."""
        return self.prm.dt

    def flux(self):
        return api.flux_planes(self.d.s_idx, self.d.s_w, self.v[0], self.d.n_all, ws=self.d.red_ws)

    def permeability(self) -> float:
        """k/d^2 = q nu / (|g| d^2), Eq. k_definition."""
        return api.permeability(float(self.flux().item()), self.prm.nu, self.g)

    def drag(self):
        """(F [3], K) with K = F_x / (6 pi r phi q mu), Eq. K_definition."""
        d = self.d
        F = api.drag(self.v, self.p, d.sb, self.wg, d.nrm, self.prm.rho, self.prm.nu, d.area / d.nb, ws=d.red_ws)
        F = F.cpu().numpy()
        q = float(self.flux().item())
        K = api.drag_coefficient(F[0], d.cloud.r, d.phi, q, self.prm.rho * self.prm.nu)
        return F, K

    def residual(self, v_prev=None):
        """[max |v - v_prev|, max |v|, rms div v] over the interior (host floats)."""
        return api.residual(self.d.sten, self.w, self.v, self.d.n_int, v_prev, self.precision).cpu().tolist()

    def surface_map(self):
        """Traction sigma n [3][nb] and centred pressure [nb] on the grain
        (device, double): the surface maps of Sec. 3.1."""
        d = self.d
        return api.traction(self.v, self.p, d.sb, self.wg, d.nrm, self.prm.rho, self.prm.nu, ws=d.red_ws)


def ctypesarr(g):
    import ctypes
    return (ctypes.c_double * 3)(*[float(x) for x in g])


def lbm_units(h_min: float, nu: float, tau_plus: float, g, magic: float):
    """dx = h_min / 2 (Sec. 2.2), nu_lb = (tau+ - 1/2)/3 (Eq. lbm_viscosity),
    dt and g_lb from Eq. conversion_factors, tau- from the magic parameter:
    the library's mpf_lbm_units_of."""
    return api.lbm_units(h_min, nu, tau_plus, g, magic)


def lattice_vectors(q: int):
    """e_k in the pairing of the paper's D3Q15 table (rest; odd k listed; even
    k opposite), for building the shift operators of the departure points."""
    base = {15: [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1), (1, 1, -1), (1, -1, 1), (1, -1, -1)],
            19: [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1),
                 (0, 1, -1)]}[q]
    e = [(0, 0, 0)]
    for b in base:
        e.append(b)
        e.append(tuple(-x for x in b))
    return e


def lattice_weights(q: int):
    """w_k of the velocity set in the same order (used only to convert the
    shifted device state for host-side inspection)."""
    w0, w1, w2 = (1 / 3, 1 / 18, 1 / 36) if q == 19 else (2 / 9, 1 / 9, 1 / 72)
    return np.array([w0 if sum(x * x for x in v) == 0 else (w1 if sum(x * x for x in v) == 1 else w2)
                     for v in lattice_vectors(q)])


class MLBMSolver:
    """Meshless TRT lattice Boltzmann (Sec. 2.2) on a Discretization.

    streaming: "shift" interpolates each population at its departure point
    x_i - dx e_k (Eq. LBM_streaming); "taylor" uses the first-order form
    f - dx e_k . grad f instead.  rule: the unknown populations of boundary
    nodes come from the local normal ("normal", Sec. 2.2) or from testing the
    departure point against the grains ("solid", the touching limit of
    Sec. 3.3)."""

    def __init__(self, disc: Discretization, q=19, precision: int = MPF_F64, nu=1.0, tau_plus=1.0, magic=0.25,
                 g=(1.0, 0.0, 0.0), dx=None, W=None, streaming: str = "shift", rule: str = "normal",
                 check: bool = True, staged: bool = True):
        self.d, self.q, self.precision, self.check, self.staged = disc, q, precision, check, staged
        h = disc.cloud.h_min if dx is None else 2.0 * dx
        self.units = u = lbm_units(h, nu, tau_plus, g, magic)
        self.nu, self.g = nu, tuple(g)
        self.prm = LbmParams(q=q, precision=precision, tau_plus=tau_plus, tau_minus=u["tau_minus"],
                             g_lb=ctypesarr(u["g_lb"]))
        e = lattice_vectors(q)
        if streaming not in ("shift", "taylor"):
            raise ValueError(f"unknown streaming {streaming!r}")
        if W is None:
            ops = [(streaming, tuple(-u["dx"] * x for x in e[k])) for k in range(1, q)]
            w64, w32, self.info = api.rbffd_weights(disc.pos, disc.sten, ops, want64=precision == MPF_F64,
                                                    want32=precision != MPF_F64)
            W = w64 if precision == MPF_F64 else w32
        self.W = W
        self.unknown = api.lbm_unknown(q, disc.pos, disc.n_int, disc.nrm, rule, u["dx"], disc.cloud.r)
        dtp = _DT[precision]
        self.f = torch.empty((disc.n, api.record_len(q)), dtype=dtp, device=disc.device)
        self.f_tmp = torch.empty_like(self.f)
        # compensation records of the compensated FP32 state (zero: the
        # equilibrium below is its FP32 value)
        self.comp = torch.zeros_like(self.f) if precision == MPF_F32_KAHAN else None
        self.flags = torch.zeros(1, dtype=torch.int32, device=disc.device)
        api.lbm_init(self.prm, self.f)
        self.steps = 0
        self._v = torch.empty((3, disc.n), dtype=torch.float64, device=disc.device)
        self._p = torch.empty(disc.n, dtype=torch.float64, device=disc.device)
        self._wg = None

    def set_fields(self, v, p):
        """Start from the equilibrium of fields v [3][n], p [n] (device double,
        physical units): a warm start."""
        api.lbm_init_fields(self.prm, self.f, v, p, self.units["vel_scale"])
        if self.comp is not None:
            self.comp.zero_()
        self.steps = 0

    def run(self, n_steps: int):
        api.lbm_run(self.prm, self.d.n_int, self.d.sten, self.W, self.unknown, self.f, self.f_tmp, n_steps,
                    comp=self.comp, flags=self.flags if self.check else None,
                    tiles=self.d.tiles if self.staged else None)
        self.steps += n_steps

    @property
    def time_step(self) -> float:
        """Physical time per step: delta t = nu_lb delta x^2 / nu (Sec. 2.2)."""
        return self.units["dt"]

    def populations(self):
        """Host copy of the state as f [n][q] (unshifted; the compensated
        state adds its remainder in FP64)."""
        f = self.f[:, :self.q].double().cpu().numpy()
        if self.comp is not None:
            f = f + self.comp[:, :self.q].double().cpu().numpy()
        return f + lattice_weights(self.q)

    def set_populations(self, f):
        """Load f [n][q] (unshifted, host) into the device state."""
        buf = np.zeros(tuple(self.f.shape))
        buf[:, :self.q] = np.asarray(f) - lattice_weights(self.q)
        self.f.copy_(torch.as_tensor(buf, dtype=self.f.dtype, device=self.f.device))
        if self.comp is not None:  # the FP32 remainder of the given values
            rem = buf - self.f.double().cpu().numpy()
            self.comp.copy_(torch.as_tensor(rem, dtype=torch.float32, device=self.f.device))

    def macros(self):
        return api.lbm_moments(self.prm, self.f, self.units["vel_scale"], self._v, self._p, comp=self.comp)

    def permeability(self) -> float:
        v, _ = self.macros()
        q = float(api.flux_planes(self.d.s_idx, self.d.s_w, v[0], self.d.n_all, ws=self.d.red_ws).item())
        return api.permeability(q, self.nu, self.g)

    def drag(self):
        d = self.d
        v, p = self.macros()
        v[:, d.n_int:] = 0.0  # the no-slip value on the grain enters the stress
        if self._wg is None:
            self._wg = api.rbffd_weights(d.pos, d.sb, [("dx",), ("dy",), ("dz",)])[0]
        F = api.drag(v, p, d.sb, self._wg, d.nrm, 1.0, self.nu, d.area / d.nb, ws=d.red_ws).cpu().numpy()
        q = float(api.flux_planes(d.s_idx, d.s_w, v[0], d.n_all, ws=d.red_ws).item())
        K = api.drag_coefficient(F[0], d.cloud.r, d.phi, q, self.nu)
        return F, K

    def surface_map(self):
        """Traction sigma n [3][nb] and centred pressure [nb] on the grain
        (device, double), with the no-slip velocity on the grain."""
        d = self.d
        v, p = self.macros()
        v[:, d.n_int:] = 0.0
        if self._wg is None:
            self._wg = api.rbffd_weights(d.pos, d.sb, [("dx",), ("dy",), ("dz",)])[0]
        return api.traction(v, p, d.sb, self._wg, d.nrm, 1.0, self.nu, ws=d.red_ws)


def run_to_paper_criterion(solver, every: int = 10_000, tol: float = 1e-2, max_steps: int = 10_000_000,
                           log=None, log_every: float = 30.0):
    """Run until the paper's stopping criterion (Eq. stopCrit) holds: every
    `every` steps the relative rate of change of the permeability,
    |k(t) - k(t - Dt)| / (k(t) Dt) with Dt = every delta t in physical time,
    is evaluated, and the run stops at the first check where it is below
    `tol` (the paper: every 1e4 steps, tol 1e-2).  The first check compares
    with the state the call started from.  Returns a dict with the steps and
    physical time at the stop (counted from the solver's step 0), k there,
    the last rate and the number of checks; "converged" is False if
    max_steps ran out first.  log: optional callable(str), called about every
    log_every seconds of wall-clock with the progress."""
    if every < 1 or not tol > 0:
        raise ValueError("every must be >= 1 and tol > 0")
    dt = solver.time_step * every
    k = k_prev = solver.permeability()
    rate, checks = math.inf, 0
    t_log = time.perf_counter()
    while solver.steps < max_steps:
        solver.run(every)
        k = solver.permeability()
        checks += 1
        rate = abs(k - k_prev) / (abs(k) * dt) if k != 0 else math.inf
        if not math.isfinite(k):
            raise FloatingPointError(f"permeability is {k} after {solver.steps} steps")
        if rate < tol:
            break
        k_prev = k
        if log and time.perf_counter() - t_log > log_every:
            log(f"{solver.steps} steps, t = {solver.steps * solver.time_step:.4g}, k = {k:.6e}, rate {rate:.3e}")
            t_log = time.perf_counter()
    return {"steps": solver.steps, "time": solver.steps * solver.time_step, "k": k, "rate": rate,
            "checks": checks, "converged": rate < tol}
