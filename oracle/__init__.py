"""CPU FP64 oracle for the meshless pore-flow solvers (arXiv 2404.14195).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  The product library never imports
this package and shares no code with it.

The arithmetic lives in ``mpf_oracle.c`` (plain scalar C, FP64, paper order and
notation); this module is argument marshalling plus a few scalar formulas that
the paper states directly (time steps, unit conversion, drag coefficient).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libmpf_oracle.so")
_lib = None

OPS = {"dx": 0, "dy": 1, "dz": 2, "lap": 3, "dir": 4, "shift": 5, "dn": 6, "shift_row": 7, "taylor": 8}


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-std=c11", "-shared", "-fPIC",
                               os.path.join(_HERE, "mpf_oracle.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        lib = ctypes.CDLL(_SO)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        lib.mpfo_porosity.restype = dbl
        lib.mpfo_porosity.argtypes = [dbl]
        lib.mpfo_area.restype = dbl
        lib.mpfo_area.argtypes = [dbl]
        lib.mpfo_weights.restype = i32
        lib.mpfo_weights.argtypes = [vp, i64, vp, i64, i32, i32, vp, vp, vp, vp, vp]
        lib.mpfo_acm_run.restype = i32
        lib.mpfo_acm_run.argtypes = [i64, i64, i32, vp, vp, vp, vp, dbl, dbl, dbl, dbl, dbl, vp, i32, vp, vp, vp, i32, i32]
        lib.mpfo_lattice.restype = i32
        lib.mpfo_lattice.argtypes = [i32, vp, vp, vp]
        lib.mpfo_lbm_equilibrium.restype = None
        lib.mpfo_lbm_equilibrium.argtypes = [i32, i64, dbl, vp, vp]
        lib.mpfo_lbm_moments.restype = None
        lib.mpfo_lbm_moments.argtypes = [i32, i64, vp, vp, vp]
        lib.mpfo_lbm_run.restype = i32
        lib.mpfo_lbm_run.argtypes = [i32, i64, i64, i32, vp, vp, vp, dbl, dbl, vp, vp, i32]
        lib.mpfo_knn.restype = i32
        lib.mpfo_knn.argtypes = [vp, i64, vp, i64, i32, vp]
        lib.mpfo_lbm_unknown.restype = i32
        lib.mpfo_lbm_unknown.argtypes = [i32, i64, vp, vp, i32, dbl, dbl, vp]
        lib.mpfo_flux.restype = dbl
        lib.mpfo_flux.argtypes = [i64, i32, vp, vp, vp, i64]
        lib.mpfo_drag.restype = None
        lib.mpfo_drag.argtypes = [i64, i32, vp, vp, vp, i64, vp, vp, dbl, dbl, dbl, vp]
        lib.mpfo_traction.restype = None
        lib.mpfo_traction.argtypes = [i64, i32, vp, vp, vp, i64, vp, vp, dbl, dbl, vp, vp]
        lib.mpfo_set_threads.restype = i32
        lib.mpfo_set_threads.argtypes = [i32]
        lib.mpfo_pointwise.restype = None
        lib.mpfo_pointwise.argtypes = [i64, vp, vp, vp, vp]
        lib.mpfo_residual.restype = None
        lib.mpfo_residual.argtypes = [i64, i32, vp, vp, i32, vp, vp, vp]
        _lib = lib
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --- geometry (Sec. 2.4) -------------------------------------------------------

def porosity(r: float) -> float:
    return _load().mpfo_porosity(float(r))


def area(r: float) -> float:
    return _load().mpfo_area(float(r))


# --- stencils (Sec. 2.1) -------------------------------------------------------

def knn(pts, k, queries=None):
    """Indices [m][k] of the k nearest of pts [n][3] to each query (default:
    the points themselves), nearest first; equal distances by index."""
    pts = _c(pts, np.float64).reshape(-1, 3)
    q = pts if queries is None else _c(queries, np.float64).reshape(-1, 3)
    idx = np.zeros((len(q), k), dtype=np.int32)
    if len(q) and _load().mpfo_knn(pts.ctypes.data, len(pts), q.ctypes.data, len(q), int(k), idx.ctypes.data):
        raise ValueError("mpfo_knn: need 1 <= k <= number of points")
    return idx


def solver_stencils(pos, n_int, nl):
    """Interior nodes: their nl nearest nodes.  Boundary nodes [n_int, n):
    the node itself, then its nl - 1 nearest interior nodes."""
    pos = _c(pos, np.float64)
    n_int = int(n_int)
    sten = np.zeros((len(pos), nl), dtype=np.int32)
    if n_int:
        sten[:n_int] = knn(pos, nl, pos[:n_int])
    if len(pos) > n_int:
        sten[n_int:, 0] = np.arange(n_int, len(pos))
        sten[n_int:, 1:] = knn(pos[:n_int], nl - 1, pos[n_int:])
    return sten


# --- weights (Sec. 2.1) --------------------------------------------------------

def weights(pos, sten, ops, rowvec=None):
    """RBF-FD weights for each stencil row.  ops: list of (name, vec) with
    name in OPS.  Returns (w [m][n_ops][nl], info [m])."""
    lib = _load()
    pos = _c(pos, np.float64)
    sten = _c(sten, np.int32)
    m, nl = sten.shape
    kinds = _c([OPS[o[0]] for o in ops], np.int32)
    vec = _c([list(o[1]) if len(o) > 1 and o[1] is not None else [0.0, 0.0, 0.0] for o in ops], np.float64)
    rv = None if rowvec is None else _c(rowvec, np.float64)
    w = np.zeros((m, len(ops), nl))
    info = np.zeros(m, dtype=np.int32)
    rc = lib.mpfo_weights(pos.ctypes.data, len(pos), sten.ctypes.data, m, nl, len(ops), kinds.ctypes.data,
                          vec.ctypes.data, None if rv is None else rv.ctypes.data, w.ctypes.data, info.ctypes.data)
    if rc != 0:
        raise ValueError(f"mpfo_weights failed ({rc})")
    return w, info


# --- ACM (Sec. 2.3) ------------------------------------------------------------

def acm_dt(h_min: float, nu: float) -> float:
    """Time step of the ACM solver: 0.1 h_min^2 / (2 nu) (Sec. 2.3)."""
    return 0.1 * h_min * h_min / (2.0 * nu)


class ACM:
    """ACM state and parameters on one node cloud (defaults: Sec. 2.3).
    edac=True takes the entropically damped pressure equation (see
    mpfo_acm_run)."""

    def __init__(self, pos, n_int, sten, nrm, sten_n=None, nu=1.0, rho=1.0, dt=None, beta=10.0, v_ref=1.0,
                 g=(1.0, 0.0, 0.0), n_p=3, h_min=None, edac=False):
        self.edac = bool(edac)
        self.pos, self.n_int, self.sten, self.nrm = _c(pos, np.float64), int(n_int), _c(sten, np.int32), _c(nrm, np.float64)
        self.n, self.nl = self.sten.shape
        self.nu, self.rho, self.beta, self.v_ref, self.n_p = nu, rho, beta, v_ref, n_p
        self.g = _c(g, np.float64)
        self.dt = dt if dt is not None else acm_dt(h_min, nu)
        self.w, info = weights(self.pos, self.sten, [("dx",), ("dy",), ("dz",), ("lap",)])
        if info.any():
            raise ValueError("singular weight system")
        nb = self.n - self.n_int
        # stencils of the pressure Neumann rows (default: the node's own stencil)
        self.sn = _c(self.sten[self.n_int:] if sten_n is None else sten_n, np.int32)
        if nb:
            wn, info = weights(self.pos, self.sn, [("dn",)], rowvec=self.nrm)
            if info.any():
                raise ValueError("singular weight system")
            self.wn = _c(wn[:, 0, :], np.float64)
        else:
            self.wn = np.zeros((1, self.nl))
            self.sn = np.zeros((1, self.nl), dtype=np.int32)
        self.v = np.zeros((self.n, 3))
        self.p = np.zeros(self.n)
        self.C = np.array([beta * abs(v_ref)])

    def run(self, n_steps: int):
        lib = _load()
        rc = lib.mpfo_acm_run(self.n, self.n_int, self.nl, self.sten.ctypes.data, self.w.ctypes.data,
                              self.sn.ctypes.data, self.wn.ctypes.data, self.nu, self.rho, self.dt, self.beta, self.v_ref,
                              self.g.ctypes.data, self.n_p, self.v.ctypes.data, self.p.ctypes.data,
                              self.C.ctypes.data, int(n_steps), int(self.edac))
        if rc != 0:
            raise RuntimeError("mpfo_acm_run failed")


# --- MLBM (Sec. 2.2) -----------------------------------------------------------

def lattice(q: int):
    lib = _load()
    e = np.zeros((q, 3))
    wk = np.zeros(q)
    opp = np.zeros(q, dtype=np.int32)
    if lib.mpfo_lattice(q, e.ctypes.data, wk.ctypes.data, opp.ctypes.data):
        raise ValueError("q must be 15 or 19")
    return e, wk, opp


def lbm_units(h_min: float, nu: float, tau_plus: float, g, magic: float):
    """Streaming distance dx = h_min/2, nu_lb = (tau+ - 1/2)/3 (Eq.
    lbm_viscosity), dt from nu = dx^2/dt nu_lb and g_lb = g dt^2/dx (Eq.
    conversion_factors), tau- from Lambda = (tau+ - 1/2)(tau- - 1/2)."""
    dx = 0.5 * h_min
    nu_lb = (tau_plus - 0.5) / 3.0
    dt = nu_lb * dx * dx / nu
    g_lb = np.asarray(g, dtype=np.float64) * dt * dt / dx
    tau_minus = 0.5 + magic / (tau_plus - 0.5)
    return dict(dx=dx, dt=dt, nu_lb=nu_lb, g_lb=g_lb, tau_minus=tau_minus)


UNKNOWN_RULES = {"normal": 0, "solid": 1}


def lbm_unknown(q, pos_b, nrm, rule="normal", dx=0.0, r=0.0):
    """Bit mask [nb] of the unknown populations of each boundary node: by the
    local normal (Sec. 2.2) or by testing the departure point against the
    solid (Sec. 3.3, the touching limit)."""
    pos_b = _c(pos_b, np.float64).reshape(-1, 3)
    nrm = _c(nrm, np.float64).reshape(-1, 3)
    mask = np.zeros(len(pos_b), dtype=np.uint32)
    if len(mask) and _load().mpfo_lbm_unknown(q, len(mask), pos_b.ctypes.data, nrm.ctypes.data, UNKNOWN_RULES[rule],
                                              float(dx), float(r), mask.ctypes.data):
        raise ValueError("mpfo_lbm_unknown: bad q, rule or dx")
    return mask


class MLBM:
    """Meshless TRT LBM state on one node cloud.

    streaming "shift" interpolates each population at its departure point
    x_i - dx e_k (Eq. LBM_streaming, L = 1); "taylor" takes the first-order
    estimate f - dx e_k . grad f there instead.  rule picks the unknown
    populations of boundary nodes (lbm_unknown); "solid" needs the grain
    radius r."""

    def __init__(self, pos, n_int, sten, nrm, q=19, h_min=None, nu=1.0, tau_plus=1.0, magic=0.25, g=(1.0, 0.0, 0.0),
                 dx=None, streaming="shift", rule="normal", r=None):
        self.pos, self.n_int, self.sten, self.nrm = _c(pos, np.float64), int(n_int), _c(sten, np.int32), _c(nrm, np.float64)
        self.n, self.nl = self.sten.shape
        self.q = q
        u = lbm_units(h_min if dx is None else 2.0 * dx, nu, tau_plus, g, magic)
        self.units = u
        self.tau_plus, self.tau_minus, self.g_lb = tau_plus, u["tau_minus"], u["g_lb"]
        e, _, _ = lattice(q)
        if streaming not in ("shift", "taylor"):
            raise ValueError(streaming)
        # departure point of population k: x_i - dx e_k
        ops = [(streaming, tuple(-u["dx"] * e[k])) for k in range(q)]
        W, info = weights(self.pos, self.sten, ops)
        if info.any():
            raise ValueError("singular weight system")
        self.W = W
        if rule == "solid" and r is None:
            raise ValueError("the solid rule needs the grain radius r")
        self.unknown = lbm_unknown(q, self.pos[self.n_int:], self.nrm, rule, u["dx"], r or 0.0)
        self.f = equilibrium(q, self.n, 1.0, (0.0, 0.0, 0.0))

    def run(self, n_steps: int):
        rc = _load().mpfo_lbm_run(self.q, self.n, self.n_int, self.nl, self.sten.ctypes.data, self.W.ctypes.data,
                                  self.unknown.ctypes.data, self.tau_plus, self.tau_minus,
                                  _c(self.g_lb, np.float64).ctypes.data, self.f.ctypes.data, int(n_steps))
        if rc != 0:
            raise RuntimeError("mpfo_lbm_run failed")

    def macros(self):
        """Physical velocity [n][3] and pressure [n] (Eq. conversion_factors,
        p_lb = (rho - <rho>) c_s^2)."""
        rho, u = moments(self.q, self.f)
        c = self.units["dx"] / self.units["dt"]
        return u * c, (rho - rho.mean()) / 3.0 * c * c


def equilibrium(q, n, rho, u):
    f = np.zeros((n, q))
    _load().mpfo_lbm_equilibrium(q, n, float(rho), _c(u, np.float64).ctypes.data, f.ctypes.data)
    return f


def moments(q, f):
    f = _c(f, np.float64)
    n = f.shape[0]
    rho = np.zeros(n)
    u = np.zeros((n, 3))
    _load().mpfo_lbm_moments(q, n, f.ctypes.data, rho.ctypes.data, u.ctypes.data)
    return rho, u


def lbm_run(q, n_int, sten, W, unknown, tau_p, tau_m, g_lb, f, n_steps):
    sten = _c(sten, np.int32)
    W = _c(W, np.float64)
    unknown = _c(unknown, np.uint32)
    if len(unknown) != sten.shape[0] - int(n_int):
        raise ValueError("one mask per boundary node")
    rc = _load().mpfo_lbm_run(q, sten.shape[0], int(n_int), sten.shape[1], sten.ctypes.data, W.ctypes.data,
                              unknown.ctypes.data, tau_p, tau_m, _c(g_lb, np.float64).ctypes.data, f.ctypes.data,
                              int(n_steps))
    if rc != 0:
        raise RuntimeError("mpfo_lbm_run failed")


# --- reductions ------------------------------------------------------------------

def plane_weights(pos, plan_idx, plan_shift):
    """Interpolation weights (L = 1) of every plane sample."""
    w, info = weights(pos, plan_idx, [("shift_row",)], rowvec=plan_shift)
    if info.any():
        raise ValueError("singular weight system")
    return w[:, 0, :]


def flux(plan_idx, plan_w, vx, n_all: int) -> float:
    """Mean x-velocity q over the planes (Eq. k_definition)."""
    idx = _c(plan_idx, np.int32)
    sw = _c(plan_w, np.float64)
    vx = _c(vx, np.float64)
    return _load().mpfo_flux(idx.shape[0], idx.shape[1], idx.ctypes.data, sw.ctypes.data, vx.ctypes.data, int(n_all))


def permeability(q: float, nu: float, g_abs: float, d: float = 1.0) -> float:
    """k/d^2 = q nu / (|g| d^2), Eq. k_definition."""
    return q * nu / (g_abs * d * d)


def drag(sb, wg, nrm, v, p, rho, nu, dA):
    """Hydrodynamic force F_H [3] (Eqs. stress_tensor_force, integration_force)."""
    sb = _c(sb, np.int32)
    wg = _c(wg, np.float64)
    nrm = _c(nrm, np.float64)
    v = _c(v, np.float64)
    p = _c(p, np.float64)
    F = np.zeros(3)
    _load().mpfo_drag(sb.shape[0], sb.shape[1], sb.ctypes.data, wg.ctypes.data, nrm.ctypes.data, len(p),
                      v.ctypes.data, p.ctypes.data, rho, nu, dA, F.ctypes.data)
    return F


def traction(sb, wg, nrm, v, p, rho, nu):
    """Traction sigma n [nb][3] at every boundary node and the centred pressure
    [nb] there (the surface maps of Sec. 3.1)."""
    sb = _c(sb, np.int32)
    wg = _c(wg, np.float64)
    nrm = _c(nrm, np.float64)
    v = _c(v, np.float64)
    p = _c(p, np.float64)
    t = np.zeros((sb.shape[0], 3))
    pc = np.zeros(sb.shape[0])
    _load().mpfo_traction(sb.shape[0], sb.shape[1], sb.ctypes.data, wg.ctypes.data, nrm.ctypes.data, len(p),
                          v.ctypes.data, p.ctypes.data, rho, nu, t.ctypes.data, pc.ctypes.data)
    return t, pc


def drag_coefficient(Fx: float, r: float, phi: float, q: float, mu: float) -> float:
    """K = F_H,0 / (6 pi r phi q mu), Eq. K_definition."""
    return Fx / (6.0 * np.pi * r * phi * q * mu)


def residual(n_int, sten, w, v, v_prev=None):
    """[max |v - v_prev|, max |v|, rms div v] over the interior nodes (see
    mpfo_residual); w [n][n_ops >= 3][nl] with d/dx, d/dy, d/dz first."""
    sten, w, v = _c(sten, np.int32), _c(w, np.float64), _c(v, np.float64)
    vp = None if v_prev is None else _c(v_prev, np.float64)
    out = np.zeros(3)
    _load().mpfo_residual(int(n_int), sten.shape[1], sten.ctypes.data, w.ctypes.data, w.shape[1], v.ctypes.data,
                          None if vp is None else vp.ctypes.data, out.ctypes.data)
    return out


def set_threads(n: int) -> int:
    """Host threads of the MLBM oracle's node loops (default 1); the results
    do not depend on it.  Returns the count in effect."""
    return int(_load().mpfo_set_threads(int(n)))


def pointwise(va, vb):
    """(delta [n], dv [n]): the pointwise relative velocity difference of
    Eq. pointwise_error, |v_a - v_b| / |v_b| per node (see mpfo_pointwise)."""
    va, vb = _c(va, np.float64).reshape(-1, 3), _c(vb, np.float64).reshape(-1, 3)
    n = len(va)
    delta, dv = np.zeros(n), np.zeros(n)
    _load().mpfo_pointwise(n, va.ctypes.data, vb.ctypes.data, delta.ctypes.data, dv.ctypes.data)
    return delta, dv


def tile_plan(sten, tile: int = 64):
    """The tile plan of a stencil set, from its definition: tiles of `tile`
    consecutive nodes; halo of a tile = the ascending distinct node indices
    its stencils name; lidx[i][j] = position of sten[i][j] in the halo of
    node i's tile.  sten [n][nl].  Returns (halos: list of arrays, lidx
    [n][nl])."""
    sten = np.asarray(sten)
    n = len(sten)
    halos, lidx = [], np.empty_like(sten)
    for t0 in range(0, n, tile):
        rows = sten[t0:t0 + tile]
        h = np.unique(rows)
        halos.append(h)
        lidx[t0:t0 + tile] = np.searchsorted(h, rows)
    return halos, lidx
