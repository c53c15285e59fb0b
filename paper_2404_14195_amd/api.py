"""Python face of libmpf: one function per C entry point, same names without
the ``mpf_`` prefix.  Tensors must be contiguous and on the current HIP device;
every call is enqueued on torch's current stream."""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (MPF_F32, MPF_F32_KAHAN, MPF_F64, MPF_MIXED, AcmParams, LbmParams, LbmUnits, Tiles, WGeom, WTune,
                   check, ctx, lib, make_ops)

# element type of the state (fields, populations) and of the stencil weights
_ST = {MPF_F64: torch.float64, MPF_F32: torch.float32, MPF_MIXED: torch.float64, MPF_F32_KAHAN: torch.float32}
_WT = {MPF_F64: torch.float64, MPF_F32: torch.float32, MPF_MIXED: torch.float32, MPF_F32_KAHAN: torch.float32}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, shape=None, name="tensor"):
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")


def precision_of(dtype) -> int:
    if dtype == torch.float64:
        return MPF_F64
    if dtype == torch.float32:
        return MPF_F32
    raise TypeError(f"unsupported dtype {dtype}")


def version() -> int:
    return lib().mpf_version()


def sc_cell(r: float):
    """(porosity, grain area) of the simple-cubic cell, from the library."""
    phi = ctypes.c_double()
    area = ctypes.c_double()
    check(lib().mpf_sc_cell(float(r), ctypes.byref(phi), ctypes.byref(area)), "mpf_sc_cell")
    return phi.value, area.value


def rbffd_weights(pos, sten, ops, rowvec=None, want64=True, want32=False):
    """pos [3][n] f64, sten [nl][m] i32; ops: list of (name, vec).  Returns
    (w64 [n_ops][nl][m] or None, w32 or None, info [m])."""
    _need(pos, torch.float64, name="pos")
    _need(sten, torch.int32, name="sten")
    nl, m = sten.shape
    dev = pos.device
    w64 = torch.empty((len(ops), nl, m), dtype=torch.float64, device=dev) if want64 else None
    w32 = torch.empty((len(ops), nl, m), dtype=torch.float32, device=dev) if want32 else None
    info = torch.empty(m, dtype=torch.int32, device=dev)
    if rowvec is not None:
        _need(rowvec, torch.float64, (3, m), "rowvec")
    arr = make_ops(ops)
    ws = weights_workspace(dev)
    check(lib().mpf_rbffd_weights(_p(pos), pos.shape[1], _p(sten), m, nl, len(ops), arr, _p(rowvec), _p(w64), _p(w32),
                                  _p(info), _p(ws), ws.numel(), _stream()), "mpf_rbffd_weights")
    return w64, w32, info


def knn(pts, k: int, qry=None):
    """Indices [k][m] (int32) of the k nearest of pts [3][n] to each query
    qry [3][m] (default: the points themselves), nearest first, minimum image
    in the unit cell; equal distances in index order."""
    _need(pts, torch.float64, name="pts")
    qry = pts if qry is None else qry
    _need(qry, torch.float64, name="qry")
    if pts.dim() != 2 or pts.shape[0] != 3 or qry.dim() != 2 or qry.shape[0] != 3:
        raise ValueError("pts and qry must be [3][n]")
    n, m = pts.shape[1], qry.shape[1]
    idx = torch.empty((k, m), dtype=torch.int32, device=pts.device)
    ws = torch.empty(lib().mpf_knn_workspace(n), dtype=torch.uint8, device=pts.device)
    check(lib().mpf_knn(_p(pts), n, n, _p(qry), m, m, int(k), _p(idx), m, _p(ws), ws.numel(), _stream()), "mpf_knn")
    return idx


def solver_stencils(pos, n_int: int, nl: int):
    """Stencils [nl][n] (int32): interior nodes their nl nearest nodes, surface
    nodes themselves and then their nl - 1 nearest interior nodes."""
    _need(pos, torch.float64, name="pos")
    if pos.dim() != 2 or pos.shape[0] != 3:
        raise ValueError("pos must be [3][n]")
    n = pos.shape[1]
    sten = torch.empty((nl, n), dtype=torch.int32, device=pos.device)
    ws = torch.empty(lib().mpf_knn_workspace(n), dtype=torch.uint8, device=pos.device)
    check(lib().mpf_solver_stencils(_p(pos), n, int(n_int), int(nl), _p(sten), _p(ws), ws.numel(), _stream()),
          "mpf_solver_stencils")
    return sten


def weights_workspace(device) -> torch.Tensor:
    return torch.empty(lib().mpf_weights_workspace(), dtype=torch.uint8, device=device)


def _wgeom(pos, sten, rowvec, w64, w32, info):
    return WGeom(pos=_p(pos), n_nodes=pos.shape[1], sten=_p(sten), m=sten.shape[1], rowvec=_p(rowvec), w64=_p(w64),
                 w32=_p(w32), info=_p(info))


def rbffd_weights_batched(clouds, ops, solve=0, want64=True, want32=False, tune=None):
    """clouds: list of (pos [3][n], sten [nl][m], rowvec or None).  One launch
    over all rows.  Returns [(w64, w32, info)] per cloud."""
    nl = clouds[0][1].shape[0]
    out, geoms = [], (WGeom * len(clouds))()
    for g, (pos, sten, rowvec) in enumerate(clouds):
        _need(pos, torch.float64, name="pos")
        _need(sten, torch.int32, name="sten")
        if sten.shape[0] != nl:
            raise ValueError("all clouds must share the stencil size")
        m = sten.shape[1]
        w64 = torch.empty((len(ops), nl, m), dtype=torch.float64, device=pos.device) if want64 else None
        w32 = torch.empty((len(ops), nl, m), dtype=torch.float32, device=pos.device) if want32 else None
        info = torch.empty(m, dtype=torch.int32, device=pos.device)
        geoms[g] = _wgeom(pos, sten, rowvec, w64, w32, info)
        out.append((w64, w32, info))
    ws = weights_workspace(clouds[0][0].device)
    t = None
    if tune is not None:
        t = WTune(waves_per_block=tune[0], rows_per_wave=tune[1])
    check(lib().mpf_rbffd_weights_batched(ctx(), len(clouds), geoms, nl, len(ops), make_ops(ops), int(solve),
                                          None if t is None else ctypes.byref(t), _p(ws), ws.numel(), _stream()),
          "mpf_rbffd_weights_batched")
    return out


def weights_autotune(pos, sten, ops, solve=0, sample_rows=16384, rowvec=None):
    """Time the candidate tile shapes on the first sample_rows rows; returns
    (waves_per_block, rows_per_wave) and caches it in the device's context."""
    nl, m = sten.shape
    k = min(m, sample_rows)
    w64 = torch.empty((len(ops), nl, m), dtype=torch.float64, device=pos.device)
    info = torch.empty(m, dtype=torch.int32, device=pos.device)
    g = _wgeom(pos, sten, rowvec, w64, None, info)
    ws = weights_workspace(pos.device)
    t = WTune()
    torch.cuda.synchronize()
    check(lib().mpf_weights_autotune(ctx(), nl, len(ops), make_ops(ops), int(solve), ctypes.byref(g), k, ctypes.byref(t),
                                     _p(ws), ws.numel()), "mpf_weights_autotune")
    return t.waves_per_block, t.rows_per_wave


def acm_workspace(n: int, precision: int, device) -> torch.Tensor:
    nbytes = lib().mpf_acm_workspace(n, precision)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def acm_dt(h_min: float, nu: float) -> float:
    """The ACM time step of Sec. 2.3, from the library."""
    out = ctypes.c_double()
    check(lib().mpf_acm_dt(float(h_min), float(nu), ctypes.byref(out)), "mpf_acm_dt")
    return out.value


def acm_run(prm: AcmParams, n_int: int, sten, w, sn, wn, v, p, vmax, n_steps: int, ws=None, comp=None, flags=None,
            tiles: "TilePlan | None" = None):
    """comp: [4][n] float32 for MPF_F32_KAHAN; flags: [1] int32 (the uint32
    word), or None for a call without the end-of-call check; tiles: the plan
    of sten for the LDS-staged gather (one lane per node, FP32 state), or
    None."""
    prec = prm.precision
    dt, dw = _ST[prec], _WT[prec]
    nl, n = sten.shape
    _need(w, dw, (4, nl, n), "w")
    _need(v, dt, (3, n), "v")
    _need(p, dt, (n,), "p")
    _need(vmax, torch.float64, (1,), "vmax")
    if n > n_int:
        _need(wn, dw, (nl, n - n_int), "wn")
        _need(sn, torch.int32, (nl, n - n_int), "sn")
    if comp is not None:
        _need(comp, torch.float32, (4, n), "comp")
    if flags is not None:
        _need(flags, torch.int32, (1,), "flags")
    if ws is None:
        ws = acm_workspace(n, prec, v.device)
    check(lib().mpf_acm_run(ctypes.byref(prm), n, n_int, nl, _p(sten), _p(w), _p(sn), _p(wn),
                            None if tiles is None else ctypes.byref(tiles.rec), _p(v), _p(p), _p(comp), _p(vmax),
                            _p(flags), int(n_steps), _p(ws), ws.numel(), _stream()), "mpf_acm_run")


def record_len(q: int) -> int:
    """Padded length of one node's population record (node-major layout)."""
    return {19: 20, 15: 16}[q]


def lbm_init(prm: LbmParams, f, rho=1.0, u=(0.0, 0.0, 0.0)):
    _need(f, _ST[prm.precision], name="f")
    if f.dim() != 2 or f.shape[1] != record_len(prm.q):
        raise ValueError("f must be [n][qp]")
    uu = (ctypes.c_double * 3)(*[float(x) for x in u])
    check(lib().mpf_lbm_init(ctypes.byref(prm), f.shape[0], float(rho), uu, _p(f), _stream()), "mpf_lbm_init")


def lbm_init_fields(prm: LbmParams, f, v, p, vel_scale: float):
    """Equilibrium state of fields v [3][n], p [n] (double, physical units)."""
    _need(f, _ST[prm.precision], name="f")
    n = f.shape[0]
    _need(v, torch.float64, (3, n), "v")
    _need(p, torch.float64, (n,), "p")
    check(lib().mpf_lbm_init_fields(ctypes.byref(prm), n, _p(v), _p(p), float(vel_scale), _p(f), _stream()),
          "mpf_lbm_init_fields")


def lbm_units(h_min: float, nu: float, tau_plus: float, g, magic: float) -> dict:
    """Lattice units of Sec. 2.2 (Eq. conversion_factors), from the library."""
    out = LbmUnits()
    gg = (ctypes.c_double * 3)(*[float(x) for x in g])
    check(lib().mpf_lbm_units_of(float(h_min), float(nu), float(tau_plus), float(magic), gg, ctypes.byref(out)),
          "mpf_lbm_units_of")
    return dict(dx=out.dx, dt=out.dt, nu_lb=out.nu_lb, g_lb=list(out.g_lb), tau_minus=out.tau_minus,
                vel_scale=out.vel_scale)


class TilePlan:
    """The tile plan of a stencil set (mpf_tile_plan_sized; tile 64, 128 or
    256 nodes): device arrays and the mpf_tiles record that points at them."""

    def __init__(self, sten, h_cap: int = 1024, tile: int = 64):
        nl, n = sten.shape
        _need(sten, torch.int32, name="sten")
        G = int(lib().mpf_tile_count_sized(n, int(tile)))
        self.count = torch.empty(G + 1, dtype=torch.int32, device=sten.device)
        self.halo = torch.empty((G, h_cap), dtype=torch.int32, device=sten.device)
        self.lidx = torch.empty((nl, n), dtype=torch.int16, device=sten.device)  # the uint16 pattern
        hmax = ctypes.c_int32()
        check(lib().mpf_tile_plan_sized(n, nl, _p(sten), int(tile), int(h_cap), _p(self.count), _p(self.halo),
                                        _p(self.lidx), ctypes.byref(hmax), _stream()), "mpf_tile_plan_sized")
        self.h_cap, self.h_max, self.tile = int(h_cap), hmax.value, int(tile)
        self.rec = Tiles(count=_p(self.count), halo=_p(self.halo), lidx=_p(self.lidx), h_cap=self.h_cap,
                         h_max=self.h_max, tile=self.tile)


def lbm_run(prm: LbmParams, n_int: int, sten, W, unknown, f, f_tmp, n_steps: int, comp=None, flags=None,
            tiles: TilePlan | None = None):
    """unknown: [n - n_int] int32 bit masks from lbm_unknown; comp: [n][qp]
    float32 for MPF_F32_KAHAN; flags: [1] int32 or None; tiles: the plan of
    sten for the LDS-staged gather, or None."""
    dt = _ST[prm.precision]
    nl, n = sten.shape
    _need(W, _WT[prm.precision], (prm.q - 1, nl, n), "W")
    _need(f, dt, (n, record_len(prm.q)), "f")
    _need(f_tmp, dt, (n, record_len(prm.q)), "f_tmp")
    if n > n_int:
        _need(unknown, torch.int32, (n - n_int,), "unknown")
    if comp is not None:
        _need(comp, torch.float32, (n, record_len(prm.q)), "comp")
    if flags is not None:
        _need(flags, torch.int32, (1,), "flags")
    check(lib().mpf_lbm_run(ctypes.byref(prm), n, n_int, nl, _p(sten), _p(W), _p(unknown),
                            None if tiles is None else ctypes.byref(tiles.rec), _p(f), _p(f_tmp), _p(comp), _p(flags),
                            int(n_steps), _stream()), "mpf_lbm_run")


def lbm_unknown(q: int, pos, n_int: int, nrm=None, rule: str = "normal", dx: float = 0.0, r: float = 0.0):
    """Bit masks [n - n_int] (int32 holding the uint32 pattern) of the unknown
    populations of the boundary nodes: rule "normal" reads nrm [3][nb],
    "solid" tests the departure points x_b - dx e_k against the grains of
    radius r."""
    _need(pos, torch.float64, name="pos")
    n = pos.shape[1]
    nb = n - int(n_int)
    if rule == "normal":
        _need(nrm, torch.float64, (3, nb), "nrm")
    out = torch.empty(nb, dtype=torch.int32, device=pos.device)
    check(lib().mpf_lbm_unknown(int(q), n, int(n_int), _p(pos), _p(nrm) if rule == "normal" else None,
                                _lib.UNKNOWN_RULE[rule], float(dx), float(r), _p(out) if nb else None, _stream()),
          "mpf_lbm_unknown")
    return out


def lbm_moments(prm: LbmParams, f, vel_scale: float, v=None, p=None, comp=None):
    """comp: the remainders [n][qp] of an MPF_F32_KAHAN state, or None."""
    _need(f, _ST[prm.precision], name="f")
    n = f.shape[0]
    if comp is not None:
        _need(comp, torch.float32, tuple(f.shape), "comp")
    v = torch.empty((3, n), dtype=torch.float64, device=f.device) if v is None else v
    p = torch.empty(n, dtype=torch.float64, device=f.device) if p is None else p
    check(lib().mpf_lbm_moments(ctypes.byref(prm), n, _p(f), _p(comp), float(vel_scale), _p(v), _p(p), _stream()),
          "mpf_lbm_moments")
    return v, p


def reduce_workspace(n_items: int, device) -> torch.Tensor:
    return torch.empty(lib().mpf_reduce_workspace(n_items), dtype=torch.uint8, device=device)


def flux_planes(s_idx, s_w, vx, n_all: int, q_out=None, ws=None):
    nl, ns = s_idx.shape
    _need(s_w, torch.float64, (nl, ns), "s_w")
    q_out = torch.empty(1, dtype=torch.float64, device=vx.device) if q_out is None else q_out
    ws = reduce_workspace(ns, vx.device) if ws is None else ws
    check(lib().mpf_flux_planes(ns, nl, _p(s_idx), _p(s_w), _p(vx), precision_of(vx.dtype), int(n_all), _p(q_out),
                              _p(ws), ws.numel(), _stream()), "mpf_flux_planes")
    return q_out


def flux_planes_noalloc(s_idx, s_w, vx, n_all: int, q_out):
    """flux_planes without a workspace (the library's static partials);
    allocates nothing, so q_out [1] f64 must be given."""
    nl, ns = s_idx.shape
    _need(s_w, torch.float64, (nl, ns), "s_w")
    _need(q_out, torch.float64, (1,), "q_out")
    check(lib().mpf_flux_planes_noalloc(ns, nl, _p(s_idx), _p(s_w), _p(vx), precision_of(vx.dtype), int(n_all),
                                        _p(q_out), _stream()), "mpf_flux_planes_noalloc")
    return q_out


def pointwise(va, vb, n_count=None, levels=(), delta=None, dv=None):
    """Eq. pointwise_error on the device: (delta [n], dv [n], counts) with
    counts[l] the number of the first n_count nodes (default all) whose delta
    exceeds levels[l] (host ints).  va, vb [3][n] float32 or float64."""
    n = va.shape[1]
    for t, name in ((va, "va"), (vb, "vb")):
        if t.dim() != 2 or t.shape[0] != 3 or t.shape[1] != n:
            raise ValueError(f"{name} must be [3][n]")
    delta = torch.empty(n, dtype=torch.float64, device=va.device) if delta is None else delta
    dv = torch.empty(n, dtype=torch.float64, device=va.device) if dv is None else dv
    _need(delta, torch.float64, (n,), "delta")
    _need(dv, torch.float64, (n,), "dv")
    lv = (ctypes.c_double * max(1, len(levels)))(*[float(x) for x in levels])
    counts = torch.empty(max(1, len(levels)), dtype=torch.int64, device=va.device)
    check(lib().mpf_pointwise(n, _p(va), precision_of(va.dtype), _p(vb), precision_of(vb.dtype), _p(delta), _p(dv),
                              n if n_count is None else int(n_count), len(levels), lv, _p(counts), _stream()),
          "mpf_pointwise")
    return delta, dv, [int(x) for x in counts.cpu().tolist()[:len(levels)]]


def permeability(q: float, nu: float, g, d: float = 1.0) -> float:
    """k / d^2 = q nu / (|g| d^2), Eq. k_definition, from the library."""
    out = ctypes.c_double()
    gg = (ctypes.c_double * 3)(*[float(x) for x in g])
    check(lib().mpf_permeability(float(q), float(nu), gg, float(d), ctypes.byref(out)), "mpf_permeability")
    return out.value


def drag_coefficient(Fx: float, r: float, phi: float, q: float, mu: float) -> float:
    """K = F_x / (6 pi r phi q mu), Eq. K_definition, from the library."""
    out = ctypes.c_double()
    check(lib().mpf_drag_coefficient(float(Fx), float(r), float(phi), float(q), float(mu), ctypes.byref(out)),
          "mpf_drag_coefficient")
    return out.value


def residual(sten, w, v, n_int: int, v_prev=None, precision=None, out=None, ws=None):
    """[max |v - v_prev|, max |v|, rms div v] over the interior nodes
    (device double [3]); w [>=3][nl][n] holds d/dx, d/dy, d/dz first."""
    nl, n = sten.shape
    if precision is None:
        precision = MPF_F64 if w.dtype == torch.float64 else (MPF_F32 if v.dtype == torch.float32 else MPF_MIXED)
    _need(w, _WT[precision], name="w")
    _need(v, _ST[precision], (3, n), "v")
    if w.dim() != 3 or w.shape[0] < 3 or tuple(w.shape[1:]) != (nl, n):
        raise ValueError("w must be [>=3][nl][n]")
    if v_prev is not None:
        _need(v_prev, _ST[precision], (3, n), "v_prev")
    out = torch.empty(3, dtype=torch.float64, device=v.device) if out is None else out
    ws = reduce_workspace(n, v.device) if ws is None else ws
    check(lib().mpf_residual(n, int(n_int), nl, _p(sten), _p(w), _p(v), _p(v_prev), int(precision), _p(out), _p(ws),
                             ws.numel(), _stream()), "mpf_residual")
    return out


def drag(v, p, sb, wg, nrm, rho: float, nu: float, dA: float, F_out=None, ws=None):
    n = p.shape[0]
    nl, nb = sb.shape
    _need(wg, torch.float64, (3, nl, nb), "wg")
    _need(nrm, torch.float64, (3, nb), "nrm")
    if v.dtype != p.dtype:
        raise TypeError("v and p must share a dtype")
    F_out = torch.empty(3, dtype=torch.float64, device=v.device) if F_out is None else F_out
    ws = reduce_workspace(max(n, nb), v.device) if ws is None else ws
    check(lib().mpf_drag(n, _p(v), _p(p), precision_of(p.dtype), nb, nl, _p(sb), _p(wg), _p(nrm), float(rho), float(nu),
                       float(dA), _p(F_out), _p(ws), ws.numel(), _stream()), "mpf_drag")
    return F_out


def traction(v, p, sb, wg, nrm, rho: float, nu: float, ws=None):
    """Surface maps: traction sigma n [3][nb] and centred pressure [nb] at the
    boundary nodes (double)."""
    n = p.shape[0]
    nl, nb = sb.shape
    _need(wg, torch.float64, (3, nl, nb), "wg")
    _need(nrm, torch.float64, (3, nb), "nrm")
    if v.dtype != p.dtype:
        raise TypeError("v and p must share a dtype")
    t = torch.empty((3, nb), dtype=torch.float64, device=v.device)
    pc = torch.empty(nb, dtype=torch.float64, device=v.device)
    ws = reduce_workspace(max(n, nb), v.device) if ws is None else ws
    check(lib().mpf_traction(n, _p(v), _p(p), precision_of(p.dtype), nb, nl, _p(sb), _p(wg), _p(nrm), float(rho),
                             float(nu), _p(t), _p(pc), _p(ws), ws.numel(), _stream()), "mpf_traction")
    return t, pc


# ---------------------------------------------------------------- learned warm start

MLP_DESC = _lib.MlpDesc(5, 128, 4, 4)


def mlp_param_count() -> int:
    return int(lib().mpf_mlp_param_count(ctypes.byref(MLP_DESC)))


def mlp_packed_count() -> int:
    return int(lib().mpf_mlp_packed_count(ctypes.byref(MLP_DESC)))


def mlp_workspace(batch: int, train: bool, device="cuda") -> torch.Tensor:
    nbytes = lib().mpf_mlp_workspace(ctypes.byref(MLP_DESC), int(batch), int(bool(train)))
    if nbytes == 0:
        raise ValueError(f"unsupported MLP batch {batch}")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def mlp_pack(master, packed):
    _need(master, torch.float32, (mlp_param_count(),), "master")
    _need(packed, torch.bfloat16, (mlp_packed_count(),), "packed")
    check(lib().mpf_mlp_pack(ctypes.byref(MLP_DESC), _p(master), _p(packed), _stream()), "mpf_mlp_pack")


def mlp_forward(master, packed, x, y, ws, rows=None, train=False):
    """y [B][4] = net(x[rows]) (B = len(rows) or len(x))."""
    _need(x, torch.float32, name="x")
    if x.dim() != 2 or x.shape[1] != 5:
        raise ValueError("x must be [rows][5]")
    B = x.shape[0] if rows is None else rows.shape[0]
    if rows is not None:
        _need(rows, torch.int64, (B,), "rows")
    _need(y, torch.float32, (B, 4), "y")
    check(lib().mpf_mlp_forward(ctypes.byref(MLP_DESC), _p(master), _p(packed), _p(x), _p(rows), _p(y), B,
                                int(bool(train)), _p(ws), ws.numel(), _stream()), "mpf_mlp_forward")


def mlp_backward(packed, dy, grad, ws):
    B = dy.shape[0]
    _need(dy, torch.float32, (B, 4), "dy")
    _need(grad, torch.float32, (mlp_param_count(),), "grad")
    check(lib().mpf_mlp_backward(ctypes.byref(MLP_DESC), _p(packed), _p(dy), _p(grad), B, _p(ws), ws.numel(),
                                 _stream()), "mpf_mlp_backward")


def mlp_mse(y, t, dy, loss, ws, rows=None):
    B = y.shape[0]
    _need(y, torch.float32, (B, 4), "y")
    _need(t, torch.float32, name="t")
    _need(dy, torch.float32, (B, 4), "dy")
    _need(loss, torch.float64, (1,), "loss")
    if rows is not None:
        _need(rows, torch.int64, (B,), "rows")
    check(lib().mpf_mlp_mse(B, _p(y), _p(t), _p(rows), _p(dy), _p(loss), _p(ws), ws.numel(), _stream()),
          "mpf_mlp_mse")


def adam_step(p, g, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    n = p.numel()
    for t, name in ((p, "p"), (g, "g"), (m, "m"), (v, "v")):
        _need(t, torch.float32, (n,), name)
    check(lib().mpf_adam_step(n, _p(p), _p(g), _p(m), _p(v), int(step), float(lr), float(b1), float(b2),
                              float(eps), _stream()), "mpf_adam_step")


def mlp_features(pos, r: float, phi: float, x=None):
    n = pos.shape[1]
    _need(pos, torch.float64, (3, n), "pos")
    if x is None:
        x = torch.empty((n, 5), dtype=torch.float32, device=pos.device)
    _need(x, torch.float32, (n, 5), "x")
    check(lib().mpf_mlp_features(n, _p(pos), float(r), float(phi), _p(x), _stream()), "mpf_mlp_features")
    return x


def mlp_to_state(y, n_int: int, U: float, P: float, v, p, vmax=None, ws=None):
    n = y.shape[0]
    _need(y, torch.float32, (n, 4), "y")
    if v.dtype != p.dtype or v.dtype not in (torch.float32, torch.float64):
        raise TypeError("v and p must share float32 or float64")
    _need(v, v.dtype, (3, n), "v")
    _need(p, v.dtype, (n,), "p")
    if vmax is not None:
        _need(vmax, torch.float64, (1,), "vmax")
    if ws is None:
        ws = reduce_workspace(n, y.device)
    prec = MPF_F32 if v.dtype == torch.float32 else MPF_F64
    check(lib().mpf_mlp_to_state(n, int(n_int), _p(y), float(U), float(P), prec, _p(v), _p(p), _p(vmax), _p(ws),
                                 ws.numel(), _stream()), "mpf_mlp_to_state")


def gemm_bf16(A, Bt, C=None, K=None):
    """C [M][N] = A[:, :K] Bt[:, :K]^T, BF16 in, FP32 out."""
    _need(A, torch.bfloat16, name="A")
    _need(Bt, torch.bfloat16, name="Bt")
    M, lda = A.shape
    N, ldb = Bt.shape
    K = lda if K is None else K
    if C is None:
        C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _need(C, torch.float32, name="C")
    check(lib().mpf_gemm_bf16(M, N, K, _p(A), lda, _p(Bt), ldb, _p(C), C.shape[1], _stream()), "mpf_gemm_bf16")
    return C


def mlp_train_workspace(batch: int, device="cuda") -> torch.Tensor:
    nbytes = lib().mpf_mlp_train_workspace(ctypes.byref(MLP_DESC), int(batch))
    if nbytes == 0:
        raise ValueError(f"unsupported MLP batch {batch}")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def mlp_train(master, packed, m, v, grad, x, t, rows, batch: int, step0: int, lr0: float, lr_ratio: float, loss_sum,
              ws, b1=0.9, b2=0.999, eps=1e-8):
    """len(rows) // batch Adam steps in one call; loss_sum [1] f64 gets the sum
    of their losses."""
    n = mlp_param_count()
    for a, name in ((master, "master"), (m, "m"), (v, "v"), (grad, "grad")):
        _need(a, torch.float32, (n,), name)
    _need(x, torch.float32, name="x")
    _need(t, torch.float32, name="t")
    _need(rows, torch.int64, name="rows")
    _need(loss_sum, torch.float64, (1,), "loss_sum")
    nb = rows.numel() // batch
    check(lib().mpf_mlp_train(ctypes.byref(MLP_DESC), _p(master), _p(packed), _p(m), _p(v), _p(grad), _p(x), _p(t),
                              _p(rows), nb, int(batch), int(step0), float(lr0), float(lr_ratio), float(b1), float(b2),
                              float(eps), _p(loss_sum), _p(ws), ws.numel(), _stream()), "mpf_mlp_train")


def mlp_fused_workspace(batch: int, device="cuda") -> torch.Tensor:
    nbytes = lib().mpf_mlp_fused_workspace(ctypes.byref(MLP_DESC), int(batch))
    if nbytes == 0:
        raise ValueError(f"unsupported MLP batch {batch}")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def mlp_grad_fused(master, packed, x, t, grad, ws, rows=None, loss=None, batch=None):
    """grad (overwritten) and loss [1] f64 of one batch (rows or the first
    batch rows of x, t) by the fused training step."""
    n = mlp_param_count()
    _need(master, torch.float32, (n,), "master")
    _need(grad, torch.float32, (n,), "grad")
    _need(x, torch.float32, name="x")
    _need(t, torch.float32, name="t")
    B = (rows.shape[0] if rows is not None else x.shape[0]) if batch is None else int(batch)
    if rows is not None:
        _need(rows, torch.int64, name="rows")
    if loss is not None:
        _need(loss, torch.float64, (1,), "loss")
    check(lib().mpf_mlp_grad_fused(ctypes.byref(MLP_DESC), _p(master), _p(packed), _p(x), _p(t), _p(rows), B, _p(grad),
                                   _p(loss), _p(ws), ws.numel(), _stream()), "mpf_mlp_grad_fused")


def mlp_train_fused(master, packed, m, v, grad, x, t, rows, batch: int, step0: int, lr0: float, lr_ratio: float,
                    loss_sum, ws, b1=0.9, b2=0.999, eps=1e-8):
    """len(rows) // batch Adam steps of the fused training step in one call."""
    n = mlp_param_count()
    for a_, name in ((master, "master"), (m, "m"), (v, "v"), (grad, "grad")):
        _need(a_, torch.float32, (n,), name)
    _need(rows, torch.int64, name="rows")
    _need(loss_sum, torch.float64, (1,), "loss_sum")
    nb = rows.numel() // batch
    check(lib().mpf_mlp_train_fused(ctypes.byref(MLP_DESC), _p(master), _p(packed), _p(m), _p(v), _p(grad), _p(x),
                                    _p(t), _p(rows), nb, int(batch), int(step0), float(lr0), float(lr_ratio),
                                    float(b1), float(b2), float(eps), _p(loss_sum), _p(ws), ws.numel(), _stream()),
          "mpf_mlp_train_fused")


def shuffle_rows(n: int, count: int, seed: int, rows=None, device="cuda"):
    """rows [count] int64: the first count entries of a seeded permutation of [0, n)."""
    if rows is None:
        rows = torch.empty(count, dtype=torch.int64, device=device)
    _need(rows, torch.int64, (count,), "rows")
    check(lib().mpf_shuffle_rows(int(n), int(count), int(seed) & (2 ** 64 - 1), _p(rows), _stream()),
          "mpf_shuffle_rows")
    return rows


def scale(x, c: float):
    """x *= c in place (float32 or float64, any shape, contiguous)."""
    check(lib().mpf_scale(x.numel(), _p(x), precision_of(x.dtype), float(c), _stream()), "mpf_scale")
