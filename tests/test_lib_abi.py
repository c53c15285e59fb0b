"""libmpf loads on the host, exports every symbol include/mpf.h declares, and
rejects bad arguments before launching anything (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2404_14195_amd import _lib
    return _lib.lib()


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "mpf.h")).read()
    return sorted(set(re.findall(r"\b(mpf_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(lib, s), s


def test_binding_covers_the_header():
    from paper_2404_14195_amd import _lib
    assert sorted(_lib.EXPORTED) == declared_symbols()


def test_error_strings_and_version(lib):
    assert lib.mpf_strerror(0) == b"ok"
    for code in (-1, -2, -3, -4, -5):
        assert lib.mpf_strerror(code) not in (b"", b"unknown error code")
    assert lib.mpf_version() >= 20000


def test_sc_cell_host(lib):
    phi, area = ctypes.c_double(), ctypes.c_double()
    assert lib.mpf_sc_cell(0.3, ctypes.byref(phi), ctypes.byref(area)) == 0
    assert phi.value == pytest.approx(1 - 4 / 3 * 3.141592653589793 * 0.027, rel=1e-15)
    assert lib.mpf_sc_cell(0.8, ctypes.byref(phi), ctypes.byref(area)) == -1


def test_host_argument_checks(lib):
    from paper_2404_14195_amd._lib import AcmParams, LbmParams, make_ops
    ops = make_ops([("dx",)])
    # null pointers, bad sizes: rejected before any launch
    assert lib.mpf_rbffd_weights(None, 10, None, 5, 30, 1, ops, None, None, None, None, None, 0, None) == -1
    fake = ctypes.c_void_p(16)
    big = lib.mpf_weights_workspace()
    assert lib.mpf_rbffd_weights(fake, 10, fake, 5, 30, 0, ops, None, fake, None, fake, fake, big, None) == -1
    assert lib.mpf_rbffd_weights(fake, 10, fake, 5, 31, 1, ops, None, fake, None, fake, fake, big, None) == -3
    assert lib.mpf_rbffd_weights(fake, 10, fake, 5, 30, 1, ops, None, fake, None, fake, fake, 8, None) == -5
    from paper_2404_14195_amd._lib import WGeom, WTune
    geoms = (WGeom * 2)()
    for g in geoms:
        g.pos, g.n_nodes, g.sten, g.m, g.w64, g.info = fake, 10, fake, 5, fake, fake
    assert lib.mpf_rbffd_weights_batched(None, 0, geoms, 30, 1, ops, 0, None, fake, big, None) == -1
    assert lib.mpf_rbffd_weights_batched(None, 17, geoms, 30, 1, ops, 0, None, fake, big, None) == -1
    assert lib.mpf_rbffd_weights_batched(None, 2, geoms, 30, 1, ops, 2, None, fake, big, None) == -1
    bad = WTune(waves_per_block=9, rows_per_wave=1)
    assert lib.mpf_rbffd_weights_batched(None, 2, geoms, 30, 1, ops, 0, ctypes.byref(bad), fake, big, None) == -1
    prm = AcmParams(nu=1, rho=1, dt=1e-5, beta=10, v_ref=1e-3, n_p=3, precision=0)
    assert lib.mpf_acm_run(ctypes.byref(prm), 10, 8, 30, fake, fake, fake, fake, None, fake, fake, None, fake, None, 1, fake, 0,
                           None) == -5  # workspace too small
    prm.lanes = 3
    assert lib.mpf_acm_run(ctypes.byref(prm), 10, 8, 30, fake, fake, fake, fake, None, fake, fake, None, fake, None, 1, fake, 1 << 20,
                           None) == -1
    prm.lanes = 0
    prm.n_p = 0
    assert lib.mpf_acm_run(ctypes.byref(prm), 10, 8, 30, fake, fake, fake, fake, None, fake, fake, None, fake, None, 1, fake, 1 << 20,
                           None) == -1
    lp = LbmParams(q=17, precision=0, tau_plus=1.0, tau_minus=1.0)
    assert lib.mpf_lbm_run(ctypes.byref(lp), 10, 10, 30, fake, fake, None, None, fake, fake, None, None, 1, None) == -1
    lp.q, lp.tau_plus = 19, 0.5
    assert lib.mpf_lbm_run(ctypes.byref(lp), 10, 10, 30, fake, fake, None, None, fake, fake, None, None, 1, None) == -1
    lp.tau_plus = 1.0
    assert lib.mpf_lbm_run(ctypes.byref(lp), 10, 8, 30, fake, fake, None, None, fake, fake, None, None, 1, None) == -1  # no masks
    # remainders are only for the compensated state
    assert lib.mpf_lbm_moments(ctypes.byref(lp), 10, fake, fake, 1.0, fake, fake, None) == -1
    # unknown-population masks: rule, q, normals, dx and r are checked first
    assert lib.mpf_lbm_unknown(19, 10, 10, None, None, 0, 0.0, 0.0, None, None) == 0  # no boundary nodes
    assert lib.mpf_lbm_unknown(19, 10, 8, fake, None, 0, 0.0, 0.0, fake, None) == -1  # normal rule needs nrm
    assert lib.mpf_lbm_unknown(19, 10, 8, fake, fake, 2, 0.01, 0.3, fake, None) == -1  # no such rule
    assert lib.mpf_lbm_unknown(19, 10, 8, fake, None, 1, 0.6, 0.3, fake, None) == -1  # dx >= 1/2
    assert lib.mpf_lbm_unknown(19, 10, 8, fake, None, 1, 0.01, 0.0, fake, None) == -1  # r <= 0
    assert lib.mpf_lbm_unknown(19, 10, 8, None, None, 1, 0.01, 0.3, fake, None) == -1  # solid rule needs pos
    assert lib.mpf_lbm_unknown(17, 10, 8, fake, fake, 0, 0.0, 0.0, fake, None) == -1  # q
    assert lib.mpf_lbm_unknown(19, 10, 11, fake, fake, 0, 0.0, 0.0, fake, None) == -1  # n_int > n
    assert lib.mpf_flux_planes(5, 30, fake, fake, fake, 0, 0, fake, fake, 1 << 20, None) == -1
    assert lib.mpf_drag(10, fake, fake, 0, 2, 30, fake, fake, fake, 1.0, 1.0, 0.1, fake, fake, 8, None) == -5
    prm.n_p, prm.edac = 3, 2
    assert lib.mpf_acm_run(ctypes.byref(prm), 10, 8, 30, fake, fake, fake, fake, None, fake, fake, None, fake, None, 1, fake, 1 << 20,
                           None) == -1  # edac is 0 or 1
    prm.edac = 0
    # a tile plan record is checked like the MLBM step's
    from paper_2404_14195_amd._lib import Tiles
    bad_tiles = Tiles(count=0x1000, halo=0x1000, lidx=0x1000, h_cap=64, h_max=65)  # h_max > h_cap
    assert lib.mpf_acm_run(ctypes.byref(prm), 10, 8, 30, fake, fake, fake, fake, ctypes.byref(bad_tiles), fake, fake,
                           None, fake, None, 1, fake, 1 << 20, None) == -1
    assert lib.mpf_acm_workspace(1000, 0) >= 9 * 1000 * 8  # v, v' records and a second pressure
    assert lib.mpf_acm_workspace(1000, 0) >= 3 * 1000 * 8
    assert lib.mpf_acm_workspace(1000, 1) >= 3 * 1000 * 4


def test_mlp_host_queries_and_checks(lib):
    from paper_2404_14195_amd._lib import MlpDesc
    d = MlpDesc(5, 128, 4, 4)
    assert lib.mpf_mlp_param_count(ctypes.byref(d)) == 34308
    assert lib.mpf_mlp_packed_count(ctypes.byref(d)) > 34308 - 128 * 3  # padded copies of W and W^T
    bad = MlpDesc(5, 64, 4, 4)
    assert lib.mpf_mlp_param_count(ctypes.byref(bad)) == -1
    assert lib.mpf_mlp_workspace(ctypes.byref(bad), 100, 1) == 0
    assert lib.mpf_mlp_workspace(ctypes.byref(d), 0, 1) == 0
    # training needs more than inference; both grow with the batch
    w_inf = lib.mpf_mlp_workspace(ctypes.byref(d), 1000, 0)
    w_tr = lib.mpf_mlp_workspace(ctypes.byref(d), 1000, 1)
    assert 0 < w_inf < w_tr < lib.mpf_mlp_workspace(ctypes.byref(d), 100000, 1)
    fake = ctypes.c_void_p(256)
    assert lib.mpf_mlp_forward(ctypes.byref(bad), fake, fake, fake, None, fake, 10, 0, fake, 1 << 30, None) == -3
    assert lib.mpf_mlp_forward(ctypes.byref(d), fake, fake, fake, None, fake, 10, 1, fake, 64, None) == -5
    assert lib.mpf_mlp_forward(ctypes.byref(d), None, fake, fake, None, fake, 10, 0, fake, 1 << 30, None) == -1
    assert lib.mpf_adam_step(10, fake, fake, fake, fake, 0, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert lib.mpf_adam_step(10, fake, fake, fake, fake, 1, 1e-3, 1.0, 0.999, 1e-8, None) == -1
    assert lib.mpf_gemm_bf16(4, 4, 40, fake, 40, fake, 40, fake, 4, None) == -1  # K not a multiple of 32
    assert lib.mpf_mlp_to_state(10, 11, fake, 1.0, 1.0, 0, fake, fake, None, fake, 1 << 20, None) == -1


def test_scale_host_checks(lib):
    fake = ctypes.c_void_p(256)
    assert lib.mpf_scale(10, None, 0, 2.0, None) == -1
    assert lib.mpf_scale(10, fake, 2, 2.0, None) == -1  # only FP64 or FP32 arrays
    assert lib.mpf_scale(10, fake, 4, 2.0, None) == -1
    assert lib.mpf_scale(0, fake, 0, 2.0, None) == 0    # nothing to do, nothing launched


def test_knn_host_checks(lib):
    fake = ctypes.c_void_p(0x1000)
    ws = lib.mpf_knn_workspace(1000)
    assert ws >= 1000 * (3 * 8 + 4 + 4)  # sorted coordinates, indices, cells
    assert lib.mpf_knn_workspace(10 ** 7) > lib.mpf_knn_workspace(10 ** 6)
    # k in [1, min(64, n)], strides at least the counts, a large enough workspace
    assert lib.mpf_knn(fake, 1000, 1000, fake, 10, 10, 0, fake, 10, fake, ws, None) == -1
    assert lib.mpf_knn(fake, 1000, 1000, fake, 10, 10, 65, fake, 10, fake, ws, None) == -1
    assert lib.mpf_knn(fake, 20, 20, fake, 10, 10, 21, fake, 10, fake, ws, None) == -1
    assert lib.mpf_knn(fake, 1000, 999, fake, 10, 10, 30, fake, 10, fake, ws, None) == -1
    assert lib.mpf_knn(fake, 1000, 1000, fake, 10, 10, 30, fake, 9, fake, ws, None) == -1
    assert lib.mpf_knn(fake, 1000, 1000, fake, 10, 10, 30, fake, 10, fake, ws - 1, None) == -1
    assert lib.mpf_knn(fake, 1000, 1000, None, 0, 0, 30, None, 0, None, 0, None) == 0  # no queries
    assert lib.mpf_solver_stencils(fake, 1000, 20, 30, fake, fake, ws, None) == -1  # surface rows need 29 interior
    assert lib.mpf_solver_stencils(fake, 1000, 900, 65, fake, fake, ws, None) == -1
    assert lib.mpf_solver_stencils(fake, 1000, 900, 30, fake, fake, 100, None) == -1


def test_traction_host_checks(lib):
    fake = ctypes.c_void_p(0x1000)
    ws = lib.mpf_reduce_workspace(100)
    assert lib.mpf_traction(100, fake, fake, 0, 10, 30, fake, fake, fake, 1.0, 1.0, None, fake, fake, ws, None) == -1
    assert lib.mpf_traction(100, fake, fake, 5, 10, 30, fake, fake, fake, 1.0, 1.0, fake, fake, fake, ws, None) == -1
    assert lib.mpf_traction(100, fake, fake, 0, 10, 30, fake, fake, fake, 1.0, 1.0, fake, fake, fake, 8, None) == -5
    assert lib.mpf_traction(100, fake, fake, 0, 0, 30, None, None, None, 1.0, 1.0, None, None, fake, ws, None) == 0


def test_compensated_state_and_flags_checks(lib):
    """MPF_F32_KAHAN needs its compensation buffer and nothing else takes one;
    the new precision is accepted wherever a state type is asked for."""
    from paper_2404_14195_amd._lib import MPF_F32_KAHAN, AcmParams, LbmParams
    fake = ctypes.c_void_p(0x1000)
    big = 1 << 30
    prm = AcmParams(nu=1, rho=1, dt=1e-5, beta=10, v_ref=1e-3, n_p=3, precision=MPF_F32_KAHAN)
    run = lambda comp, ws: lib.mpf_acm_run(ctypes.byref(prm), 10, 8, 30, fake, fake, fake, fake, None, fake, fake, comp,
                                           fake, None, 1, fake, ws, None)
    assert run(None, big) == -1              # compensated state without comp
    assert run(fake, lib.mpf_acm_workspace(10, MPF_F32_KAHAN) - 1) == -5
    prm.precision = 1
    assert run(fake, big) == -1              # comp given to a plain state
    prm.precision, prm.h_min = 1, -1.0
    assert run(None, big) == -1              # negative h_min
    # the compensated workspace also holds the v and v' remainders
    assert lib.mpf_acm_workspace(1000, MPF_F32_KAHAN) >= 17 * 1000 * 4
    lp = LbmParams(q=19, precision=MPF_F32_KAHAN, tau_plus=1.0, tau_minus=1.0)
    assert lib.mpf_lbm_run(ctypes.byref(lp), 10, 10, 30, fake, fake, None, None, fake, fake, None, None, 1, None) == -1
    lp.precision = 0
    assert lib.mpf_lbm_run(ctypes.byref(lp), 10, 10, 30, fake, fake, None, None, fake, fake, fake, None, 1, None) == -1
    lp.precision = 4
    assert lib.mpf_lbm_run(ctypes.byref(lp), 10, 10, 30, fake, fake, None, None, fake, fake, None, None, 1, None) == -1
    assert lib.mpf_scale(0, fake, MPF_F32_KAHAN, 2.0, None) == 0


def test_context_host_checks(lib):
    assert lib.mpf_create(None, 0) == -1
    c = ctypes.c_void_p()
    assert lib.mpf_create(ctypes.byref(c), -1) in (-1, -2)  # no such device (or no GPU at all)
    assert lib.mpf_destroy(None) == 0
    from paper_2404_14195_amd._lib import make_ops, WGeom, WTune
    fake = ctypes.c_void_p(16)
    g = WGeom(pos=fake, n_nodes=10, sten=fake, m=5, w64=fake, info=fake)
    t = WTune()
    # the autotuner stores its choice in a context: none given, nothing tuned
    assert lib.mpf_weights_autotune(None, 30, 1, make_ops([("dx",)]), 0, ctypes.byref(g), 5, ctypes.byref(t), fake,
                                    lib.mpf_weights_workspace()) == -1


def test_unit_conversions_in_the_library(lib):
    """The library's lattice units reproduce the paper's footnoted time steps
    (golden file) and the conversion's own identities; k and K follow Eqs.
    k_definition and K_definition."""
    from paper_2404_14195_amd._lib import LbmUnits
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "timestep_paper.txt"))
            if l.strip() and not l.startswith("#")]
    g3 = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    for solver, h, dt, tol in rows:
        h, dt, tol = float(h), float(dt), float(tol)
        if solver == "acm":
            out = ctypes.c_double()
            assert lib.mpf_acm_dt(h, 1.0, ctypes.byref(out)) == 0
            got = out.value
        else:
            u = LbmUnits()
            assert lib.mpf_lbm_units_of(h, 1.0, 1.0, 1.0, g3, ctypes.byref(u)) == 0
            got = u.dt
        assert abs(got - dt) <= tol * dt, (solver, h, got, dt)
    u = LbmUnits()
    g = (ctypes.c_double * 3)(1.0, -2.0, 0.5)
    assert lib.mpf_lbm_units_of(0.008, 0.7, 0.8, 0.25, g, ctypes.byref(u)) == 0
    assert u.dx == 0.004 and u.nu_lb == pytest.approx(0.1, rel=1e-15)
    assert u.nu_lb * u.dx ** 2 / u.dt == pytest.approx(0.7, rel=1e-15)   # nu in physical units
    assert u.vel_scale == pytest.approx(u.dx / u.dt, rel=1e-15)
    assert (u.tau_minus - 0.5) * (0.8 - 0.5) == pytest.approx(0.25, rel=1e-15)  # the magic parameter
    assert list(u.g_lb) == pytest.approx([x * u.dt ** 2 / u.dx for x in (1.0, -2.0, 0.5)], rel=1e-15)
    assert lib.mpf_lbm_units_of(0.008, 0.7, 0.5, 0.25, g, ctypes.byref(u)) == -1  # tau+ must exceed 1/2
    k, K = ctypes.c_double(), ctypes.c_double()
    g = (ctypes.c_double * 3)(3.0, 0.0, 4.0)  # |g| = 5
    assert lib.mpf_permeability(0.2, 1.5, g, 2.0, ctypes.byref(k)) == 0
    assert k.value == pytest.approx(0.2 * 1.5 / (5.0 * 4.0), rel=1e-15)
    assert lib.mpf_drag_coefficient(2.0, 0.3, 0.887, 0.05, 1.0, ctypes.byref(K)) == 0
    assert K.value == pytest.approx(2.0 / (6 * 3.141592653589793 * 0.3 * 0.887 * 0.05), rel=1e-15)
    assert lib.mpf_drag_coefficient(2.0, 0.3, 0.887, 0.0, 1.0, ctypes.byref(K)) == -1


def test_residual_host_checks(lib):
    fake = ctypes.c_void_p(0x1000)
    ws = lib.mpf_reduce_workspace(100)
    assert lib.mpf_residual(100, 90, 30, fake, fake, fake, None, 0, None, fake, ws, None) == -1
    assert lib.mpf_residual(100, 90, 30, fake, fake, fake, None, 7, fake, fake, ws, None) == -1
    assert lib.mpf_residual(100, 90, 30, fake, fake, fake, None, 0, fake, fake, 8, None) == -5


def test_pointwise_host_checks(lib):
    fake = ctypes.c_void_p(0x1000)
    lv = (ctypes.c_double * 17)(*range(17))
    assert lib.mpf_pointwise(0, fake, 0, fake, 0, fake, None, 0, 0, None, None, None) == -1
    assert lib.mpf_pointwise(10, fake, 5, fake, 0, fake, None, 0, 0, None, None, None) == -1
    assert lib.mpf_pointwise(10, fake, 0, fake, 0, fake, None, 10, 17, lv, fake, None) == -1  # at most 16 levels
    assert lib.mpf_pointwise(10, fake, 0, fake, 0, fake, None, 11, 2, lv, fake, None) == -1   # n_count > n
    assert lib.mpf_pointwise(10, fake, 0, fake, 0, fake, None, 10, 2, lv, None, None) == -1   # counts missing


def test_tile_plan_host_checks(lib):
    fake = ctypes.c_void_p(0x1000)
    hm = ctypes.c_int32()
    assert lib.mpf_tile_count(0) == 0 and lib.mpf_tile_count(64) == 1 and lib.mpf_tile_count(65) == 2
    assert lib.mpf_tile_plan(100, 65, fake, 1024, fake, fake, fake, ctypes.byref(hm), None) == -1  # nl <= 64
    assert lib.mpf_tile_plan(100, 30, fake, 63, fake, fake, fake, ctypes.byref(hm), None) == -1    # h_cap >= 64
    assert lib.mpf_tile_plan(100, 30, fake, 4097, fake, fake, fake, ctypes.byref(hm), None) == -1
    assert lib.mpf_tile_plan(100, 30, None, 1024, fake, fake, fake, ctypes.byref(hm), None) == -1
