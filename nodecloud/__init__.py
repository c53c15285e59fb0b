"""Seeded synthetic inputs for the meshless pore-flow solvers.

This module prepares what both the CPU oracle and the HIP library consume and
contains none of the solver arithmetic (no weights, no time stepping, no
reductions):

* node clouds in one periodic simple-cubic cell of side d = 1 with a sphere of
  radius r centred in it (paper Sec. 2.4), h-refined towards the grain with a
  linear target spacing h(dist) = min(h0 + slope*dist, hmax);
* stencils: the N_L nearest nodes under the minimum-image convention, the node
  itself first (Sec. 2.1); surface nodes take their N_L - 1 nearest interior
  nodes instead (solver_stencils);
* the plane-sample plan used for the permeability (Eq. k_definition): midpoint
  samples on the five planes x in {0, .2, .4, .6, .8}, each fluid sample with
  its own N_L-nearest stencil and the offset from its nearest node;
* special node sets for the physics checks: a plane channel (Poiseuille) and
  a regular periodic lattice.

Node order: interior nodes first, boundary nodes last, each block in Morton
order so that stencil neighbours sit close in memory.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_libfill.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the node-placement helper with g++ (host code only)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["g++", "-O2", "-shared", "-fPIC", os.path.join(_HERE, "_fill.cpp"), "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        lib = ctypes.CDLL(_SO)
        lib.nc_fill.restype = ctypes.c_int
        lib.nc_fill.argtypes = [ctypes.c_double] * 5 + [ctypes.c_uint64, ctypes.c_int, ctypes.c_int64,
                                                       ctypes.c_void_p, ctypes.c_void_p,
                                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        lib.nc_fill_gauss.restype = ctypes.c_int
        lib.nc_fill_gauss.argtypes = list(lib.nc_fill.argtypes)
        _lib = lib
    return _lib


def min_image(d):
    """Minimum-image displacement in the unit periodic cell."""
    return d - np.rint(d)


def sphere_sdf(x, r):
    """Distance from x ([..., 3]) to the grain surface; > 0 in the fluid."""
    d = min_image(np.asarray(x, dtype=np.float64) - 0.5)
    return np.sqrt((d * d).sum(-1)) - r


def morton_order(x, bits: int = 10):
    """Permutation that sorts points of [0,1)^3 along a Morton curve."""
    g = np.clip((np.asarray(x) * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(len(g), dtype=np.int64)
    for b in range(bits):
        for a in range(3):
            code |= ((g[:, a] >> b) & 1) << (3 * b + a)
    return np.argsort(code, kind="stable")


@dataclass
class Cloud:
    """A node cloud.  pos is [N][3] in [0,1); nodes [0, n_int) are interior,
    nodes [n_int, N) lie on the grain surface with unit normals nrm [N_b][3]
    pointing from the solid into the fluid."""
    pos: np.ndarray
    n_int: int
    nrm: np.ndarray
    r: float = 0.0
    h_min: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.pos)

    @property
    def n_bnd(self) -> int:
        return self.n - self.n_int


def estimate_count(r: float, h0: float, slope: float, hmax: float, hb: float) -> float:
    """Rough node count of a fill: integral of 1/h^3 over the fluid (midpoint
    rule on a 64^3 grid, refined near the grain through h itself) plus the
    surface nodes.  Used only to size the generator's buffers."""
    g = (np.arange(64) + 0.5) / 64
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    d = sphere_sdf(X, r)
    h = np.minimum(h0 + slope * np.maximum(d, 0.0), hmax)
    vol = np.where(d > 0, 1.0 / h ** 3, 0.0).mean()
    # the midpoint rule misses the thin refined shell; add it explicitly
    shell = 4 * np.pi * r * r * min(hmax, 4 * h0) / h0 ** 3
    return vol + shell + 4 * np.pi * r * r / (1.15 * hb * hb)


def gauss_spacing(d, r: float, h_min: float, h_max: float, eps: float = 0.295):
    """The paper's refinement function (Sec. 2.4, Eq. refinement_function) of
    the distance d to the grain: h_max - exp(-t^2 / (2 eps^2)) (h_max - h_min)
    with t = d / (sqrt(3)/2 - r)."""
    t = np.maximum(d, 0.0) / (np.sqrt(3.0) / 2.0 - r)
    return h_max - np.exp(-t * t / (2.0 * eps * eps)) * (h_max - h_min)


def estimate_count_h(r: float, h, hb: float) -> float:
    """Rough node count for a spacing function h(d) (vectorised): integral of
    1/h^3 over the fluid on a 64^3 midpoint grid plus the surface nodes."""
    g = (np.arange(64) + 0.5) / 64
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    d = sphere_sdf(X, r)
    vol = np.where(d > 0, 1.0 / h(np.maximum(d, 0.0)) ** 3, 0.0).mean()
    return vol + 4 * np.pi * r * r / (1.15 * hb * hb)


def _run_fill(fn, args, hb, cap, r, seed, n_cand, meta):
    while True:
        pos = np.zeros((cap, 3))
        nrm = np.zeros((cap, 3))
        n = ctypes.c_int64()
        nb = ctypes.c_int64()
        rc = fn(r, *args, hb, seed, n_cand, cap, pos.ctypes.data, nrm.ctypes.data, ctypes.byref(n), ctypes.byref(nb))
        if rc == 1:
            cap *= 2
            continue
        if rc != 0:
            raise ValueError(f"node fill rejected its arguments (code {rc})")
        return pos, nrm, n.value, nb.value


# The advancing front packs nodes less densely than the generator the paper
# used: with the nominal spacing it places 0.86-0.88 of the paper's printed
# node counts at every radius and resolution.  Scaling the interior spacing by
# this factor (its cube is the mean ratio) reproduces the printed counts.
PAPER_PACKING = 0.951


def gauss_cloud(r: float, h_min: float, seed: int, h_max: float | None = None, eps: float = 0.295,
                hb: float | None = None, n_cand: int = 20, packing: float = PAPER_PACKING) -> Cloud:
    """The paper's discretisation (Sec. 2.4): boundary nodes at h_min, interior
    nodes by the advancing front with the Gaussian refinement function (its
    spacing scaled by `packing`); h_max = 2 h_min and eps = 0.295 unless
    given.  The cloud's h_min is the nominal one (it sets the solvers' steps)."""
    lib = _load()
    h_max = 2.0 * h_min if h_max is None else h_max
    hb = h_min if hb is None else hb
    lo, hi = packing * h_min, packing * h_max
    est = estimate_count_h(r, lambda d: gauss_spacing(d, r, lo, hi, eps), hb)
    cap = max(int(1.5 * est) + 4096, 16384)
    pos, nrm, n, nb = _run_fill(lib.nc_fill_gauss, (lo, hi, eps), hb, cap, r, seed, n_cand, None)
    bpos, bnrm, ipos = pos[:nb], nrm[:nb], pos[nb:n]
    oi = morton_order(ipos)
    ob = morton_order(bpos)
    allpos = np.ascontiguousarray(np.concatenate([ipos[oi], bpos[ob]]))
    return Cloud(pos=allpos, n_int=len(ipos), nrm=np.ascontiguousarray(bnrm[ob]), r=r, h_min=min(h_min, hb),
                 meta=dict(kind="sphere_gauss", r=r, h_min=h_min, h_max=h_max, eps=eps, hb=hb, seed=seed,
                           n_cand=n_cand, packing=packing))


def sphere_cloud(r: float, h0: float, slope: float, hmax: float, seed: int, hb: float | None = None,
                 n_cand: int = 20) -> Cloud:
    """Boundary nodes on the sphere plus an advancing-front fill of the fluid."""
    lib = _load()
    hb = h0 if hb is None else hb
    cap = max(int(1.5 * estimate_count(r, h0, slope, hmax, hb)) + 4096, 16384)
    pos, nrm, n, nb = _run_fill(lib.nc_fill, (h0, slope, hmax), hb, cap, r, seed, n_cand, None)
    bpos, bnrm, ipos = pos[:nb], nrm[:nb], pos[nb:n]
    oi = morton_order(ipos)
    ob = morton_order(bpos)
    allpos = np.ascontiguousarray(np.concatenate([ipos[oi], bpos[ob]]))
    return Cloud(pos=allpos, n_int=len(ipos), nrm=np.ascontiguousarray(bnrm[ob]), r=r, h_min=min(h0, hb),
                 meta=dict(kind="sphere", r=r, h0=h0, slope=slope, hmax=hmax, hb=hb, seed=seed, n_cand=n_cand))


def batch_fill(args):
    """(r, h0, seed) -> (pos [n][3], n) of the cell h(d) = min(h0 + 0.3 d,
    4 h0): one worker's share of a parallel fill of several cells."""
    r, h0, seed = args
    c = sphere_cloud(r, h0, 0.3, 4 * h0, seed=seed)
    return c.pos, c.n


def lattice_cloud(n_side: int) -> Cloud:
    """All nodes of a regular periodic n^3 lattice with spacing 1/n, no grain."""
    a = (np.arange(n_side) + 0.5) / n_side
    g = np.stack(np.meshgrid(a, a, a, indexing="ij"), -1).reshape(-1, 3)
    return Cloud(pos=np.ascontiguousarray(g), n_int=len(g), nrm=np.zeros((0, 3)), r=0.0, h_min=1.0 / n_side,
                 meta=dict(kind="lattice", n_side=n_side))


def channel_cloud(h: float, H: float, seed: int, jitter: float = 0.25) -> Cloud:
    """Plane channel 0 <= z <= H (solid elsewhere), periodic in x and y.

    Wall nodes lie on z = 0 (normal +z) and z = H (normal -z) on a square
    lattice of spacing h; interior nodes sit on a jittered lattice strictly
    inside the channel."""
    rng = np.random.default_rng(seed)
    m = int(round(1.0 / h))
    hx = 1.0 / m
    nz = int(round(H / h))
    hz = H / nz
    a = (np.arange(m) + 0.5) * hx
    X, Y = np.meshgrid(a, a, indexing="ij")
    wall = []
    nrm = []
    for z, nz_sign in ((0.0, 1.0), (H, -1.0)):
        w = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], -1)
        wall.append(w)
        nrm.append(np.tile([0.0, 0.0, nz_sign], (X.size, 1)))
    zi = np.arange(1, nz) * hz
    Xi, Yi, Zi = np.meshgrid(a, a, zi, indexing="ij")
    ip = np.stack([Xi.ravel(), Yi.ravel(), Zi.ravel()], -1)
    ip = ip + rng.uniform(-jitter, jitter, ip.shape) * np.array([hx, hx, hz])
    ip[:, :2] %= 1.0
    bpos = np.concatenate(wall)
    bn = np.concatenate(nrm)
    oi = morton_order(ip)
    ob = morton_order(bpos)
    return Cloud(pos=np.ascontiguousarray(np.concatenate([ip[oi], bpos[ob]])), n_int=len(ip),
                 nrm=np.ascontiguousarray(bn[ob]), r=0.0, h_min=min(hx, hz),
                 meta=dict(kind="channel", h=h, H=H, seed=seed))


def _canonical(pts: np.ndarray, q: np.ndarray, cand: np.ndarray, k: int):
    """Order candidate neighbours by (squared minimum-image distance, index)
    and keep the first k.  The distance is formed operation by operation
    (t = p - q, t - rint(t), x^2 + y^2, + z^2), so exact ties are decided by
    the index, whatever order the tree returned them in.  Also returns the rows
    whose k-th distance equals that of the last candidate: tied neighbours may
    lie beyond the candidates there."""
    t = pts[cand] - q[:, None, :]
    t = t - np.rint(t)
    d2 = t[..., 0] * t[..., 0]
    d2 = d2 + t[..., 1] * t[..., 1]
    d2 = d2 + t[..., 2] * t[..., 2]
    order = np.lexsort((cand, d2), axis=1)
    d2 = np.take_along_axis(d2, order, 1)
    cand = np.take_along_axis(cand, order, 1)
    open_rows = d2[:, k - 1] == d2[:, -1] if cand.shape[1] > k else np.zeros(len(q), dtype=bool)
    return cand[:, :k], open_rows


def _knn(pts: np.ndarray, k: int, q: np.ndarray) -> np.ndarray:
    """k nearest of pts to each query in the canonical order (see _canonical).
    Rows with a tie reaching past the candidates are asked again with more."""
    tree = cKDTree(pts, boxsize=1.0)
    extra = min(8, len(pts) - k)
    _, idx = tree.query(q, k=k + extra)
    out, open_rows = _canonical(pts, q, np.asarray(idx, dtype=np.int64).reshape(len(q), k + extra), k)
    while open_rows.any() and k + extra < len(pts):
        extra = min(4 * extra + 8, len(pts) - k)
        rows = np.where(open_rows)[0]
        _, idx = tree.query(q[rows], k=k + extra)
        sub, still = _canonical(pts, q[rows], np.asarray(idx, dtype=np.int64).reshape(len(rows), k + extra), k)
        out[rows] = sub
        open_rows = np.zeros(len(q), dtype=bool)
        open_rows[rows[still]] = True
    return out


def stencils(pos: np.ndarray, nl: int, queries: np.ndarray | None = None) -> np.ndarray:
    """The nl nearest nodes (minimum image) of each query point, nearest first;
    equal distances in index order.

    With queries=None the queries are the nodes themselves and column 0 is the
    node's own index."""
    pos = np.asarray(pos, dtype=np.float64) % 1.0
    q = pos if queries is None else (np.asarray(queries, dtype=np.float64) % 1.0)
    idx = _knn(pos, nl, q)
    if queries is None:
        own = np.arange(len(pos))
        bad = idx[:, 0] != own
        if bad.any():  # only possible with coincident nodes
            raise ValueError("coincident nodes: a node is not its own nearest neighbour")
    return np.ascontiguousarray(idx.astype(np.int32))


def neumann_stencils(cloud: Cloud, nl: int) -> np.ndarray:
    """Stencils of the pressure Neumann rows of the boundary nodes: the node
    itself followed by its nl-1 nearest interior nodes.

    The plain nl-nearest stencil of a surface node is dominated by other
    surface nodes, and the self weight of its normal derivative can be close to
    zero, which makes solving the Neumann row for the node's own pressure
    unstable; interior neighbours only keep that weight well away from zero."""
    own = np.arange(cloud.n_int, cloud.n, dtype=np.int64)[:, None]
    if cloud.n_bnd == 0:
        return np.zeros((0, nl), dtype=np.int32)
    idx = _knn(np.asarray(cloud.pos[:cloud.n_int]) % 1.0, nl - 1, np.asarray(cloud.pos[cloud.n_int:]) % 1.0)
    return np.ascontiguousarray(np.concatenate([own, idx], 1).astype(np.int32))


def solver_stencils(cloud: Cloud, nl: int) -> np.ndarray:
    """Stencils of every node for the solvers: the nl nearest nodes for
    interior nodes, and for surface nodes the node itself followed by its nl-1
    nearest interior nodes (the stencils of neumann_stencils).

    On the sphere x^2 + y^2 + z^2 is constant, so a surface node whose nearest
    neighbours are mostly other surface nodes (typically two thirds of them)
    gets a nearly singular quadratic block in its saddle system: its
    interpolation weights reach sum |w| ~ 40 on some clouds, and the MLBM
    step, which applies them every step, grows without bound from there.
    Interior neighbours keep sum |w| of those rows near that of interior
    nodes (<= ~5)."""
    sten = stencils(cloud.pos, nl)
    if cloud.n_bnd:
        sten[cloud.n_int:] = neumann_stencils(cloud, nl)
    return sten


@dataclass
class PlanePlan:
    """Midpoint samples of the five cross-sections x = x_p, M x M per plane.

    Only fluid samples are stored: sample s has its nl-nearest stencil
    idx[s] (nearest node first) and offset shift[s] = y_s - x_{idx[s,0]}
    (minimum image).  Solid samples carry zero velocity; the normalisation
    uses all n_planes*M*M samples."""
    pts: np.ndarray
    idx: np.ndarray
    shift: np.ndarray
    plane: np.ndarray
    M: int
    planes: tuple

    @property
    def n_samples(self) -> int:
        return len(self.pts)


def plane_plan(cloud: Cloud, M: int, nl: int, planes=(0.0, 0.2, 0.4, 0.6, 0.8), fluid=None) -> PlanePlan:
    a = (np.arange(M) + 0.5) / M
    Y, Z = np.meshgrid(a, a, indexing="ij")
    pts, pl = [], []
    for k, xp in enumerate(planes):
        p = np.stack([np.full(Y.size, xp), Y.ravel(), Z.ravel()], -1)
        keep = fluid(p) if fluid is not None else sphere_sdf(p, cloud.r) > 0.0
        pts.append(p[keep])
        pl.append(np.full(int(keep.sum()), k, dtype=np.int32))
    pts = np.concatenate(pts)
    pl = np.concatenate(pl)
    idx = stencils(cloud.pos, nl, queries=pts)
    shift = min_image(pts - cloud.pos[idx[:, 0]])
    return PlanePlan(pts=pts, idx=idx, shift=np.ascontiguousarray(shift), plane=pl, M=M, planes=tuple(planes))


# --- workloads ---------------------------------------------------------------

# h(dist) = min(h0 + slope*dist, hmax); the grain surface is sampled at h0.
CONFIGS = {
    # plain ACM, FP64: r = 0.3, h 0.02 -> 0.08 reached at dist 0.2
    "acm_small": dict(r=0.3, h0=0.02, slope=0.3, hmax=0.08, seed=1, nl=30),
    # MLBM D3Q19: r = 0.3, h 0.008 -> 0.04 reached at dist 0.2
    "lbm_mid": dict(r=0.3, h0=0.008, slope=0.16, hmax=0.04, seed=2, nl=30),
    # ACM sweep cell: h 0.002 -> 0.008
    "acm_large": dict(r=0.3, h0=0.002, slope=0.3, hmax=0.008, seed=3, nl=30),
}


def config_cloud(name: str, **over) -> Cloud:
    c = dict(CONFIGS[name])
    c.update(over)
    return sphere_cloud(c["r"], c["h0"], c["slope"], c["hmax"], c["seed"])
