"""The tile plan of the LDS-staged gather (mpf_tile_plan) against the
oracle's definition, bit for bit, and the MLBM step with and without it:
the staged records are the same values read from LDS, so every precision
gives the same populations bit for bit."""
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
def disc(small_cloud):
    from paper_2404_14195_amd.solvers import Discretization
    assert torch.cuda.is_available()
    return Discretization(small_cloud, nl=30, M=32)


@pytest.mark.parametrize("nl, tile", [(30, 64), (25, 64), (50, 64), (30, 128), (30, 256), (50, 256)])
def test_tile_plan_equals_the_definition(small_cloud, nl, tile):
    """Halo lists and 16-bit positions equal the oracle's, on the 8k-node
    cell (ragged last tile) and for the host fixture's stencils, for tiles of
    64, 128 and 256 nodes."""
    from paper_2404_14195_amd import api
    S = nc.solver_stencils(small_cloud, nl)
    plan = api.TilePlan(torch.as_tensor(np.ascontiguousarray(S.T), dtype=torch.int32, device="cuda"),
                        h_cap=16 * tile, tile=tile)
    halos, lidx = O.tile_plan(S, tile)
    count = plan.count.cpu().numpy()
    assert len(count) == len(halos) + 1 and count[-1] == max(len(h) for h in halos) == plan.h_max
    halo = plan.halo.cpu().numpy()
    for t, h in enumerate(halos):
        assert count[t] == len(h) and np.array_equal(halo[t, :len(h)], h)
    assert np.array_equal(plan.lidx.cpu().numpy().astype(np.uint16).T, lidx.astype(np.uint16))


def test_tile_plan_rejects_a_small_cap(small_cloud):
    from paper_2404_14195_amd import MPFError, api
    S = nc.solver_stencils(small_cloud, 30)
    with pytest.raises(MPFError, match="unsupported"):
        api.TilePlan(torch.as_tensor(np.ascontiguousarray(S.T), dtype=torch.int32, device="cuda"), h_cap=64)


@pytest.mark.parametrize("precision, q", [(0, 19), (1, 19), (2, 19), (3, 19), (1, 15), (0, 15)])
def test_staged_step_equals_cached_gather(disc, precision, q):
    from paper_2404_14195_amd.solvers import MLBMSolver
    a = MLBMSolver(disc, q=q, precision=precision, staged=True)
    b = MLBMSolver(disc, q=q, precision=precision, staged=False)
    for s in (a, b):
        s.run(37)
    assert torch.equal(a.f, b.f)
    if a.comp is not None:
        assert torch.equal(a.comp, b.comp)


@pytest.mark.parametrize("precision, lanes", [(1, 1), (1, 2), (3, 1), (3, 2), (0, 2), (2, 2)])
@pytest.mark.parametrize("edac", [False, True])
@pytest.mark.parametrize("tile", [64, 0])
def test_staged_acm_equals_cached_gather(disc, precision, lanes, edac, tile):
    """The ACM passes at one and two lanes per node, in every precision (FP32
    and compensated FP32 at both; FP64 and mixed, whose 40-byte halo entries
    fit four 64-node tiles only up to 409 entries, at two), with and without
    the damped pressure equation, on 64-node tiles and on one tile per block
    (256 nodes at one lane, 128 at two): staged and cached gathers give the
    same fields bit for bit (same values, same summation order), including
    the running max |v|."""
    from paper_2404_14195_amd.solvers import ACMSolver
    a = ACMSolver(disc, precision=precision, lanes=lanes, edac=edac, staged=True, tile=tile)
    b = ACMSolver(disc, precision=precision, lanes=lanes, edac=edac, staged=False)
    assert a.tile == (tile or 256 // lanes)
    assert a.staged_now()  # the halo fits: the staged passes run
    for s in (a, b):
        s.run(60)
    assert torch.equal(a.v, b.v) and torch.equal(a.p, b.p) and torch.equal(a.vmax, b.vmax)
    if a.comp is not None:
        assert torch.equal(a.comp, b.comp)


def test_staged_acm_fp32_against_the_oracle(disc):
    """Staged FP32 ACM (one lane per node) against the FP64 oracle: the
    permeability after 500 steps within 1e-4, as for the cached gather."""
    from paper_2404_14195_amd.solvers import ACMSolver
    c = disc.cloud
    g = ACMSolver(disc, precision=1, lanes=1, staged=True)
    o = O.ACM(c.pos, c.n_int, disc.sten_host, c.nrm, sten_n=nc.neumann_stencils(c, 30), h_min=c.h_min, v_ref=1e-3)
    g.run(500)
    o.run(500)
    pp = disc.plan
    q_o = O.flux(pp.idx, O.plane_weights(c.pos, pp.idx, pp.shift), o.v[:, 0], disc.n_all)
    k = g.permeability()
    print(f"[acm staged fp32] k={k:.9e} k64={q_o:.9e} rel={abs(k / q_o - 1):.3e}", flush=True)
    assert k == pytest.approx(q_o, rel=1e-4)


@pytest.fixture(scope="module")
def mid_disc():
    """The 71k-node cell (55,662 interior nodes: one lane per node by default
    for an FP32 state)."""
    from paper_2404_14195_amd.solvers import Discretization
    return Discretization(nc.config_cloud("lbm_mid"), nl=30, M=16)


def test_acm_takes_two_lanes_when_one_lane_halos_do_not_fit(mid_disc):
    """With the lanes left to the library, a tile plan whose halos fit LDS at
    two lanes per node but not at one (here the real plan with its h_max
    raised to 900 > 819: the staged passes size LDS by h_max and copy only
    each tile's own count) runs the two-lane staged passes: the same fields
    bit for bit as lanes = 2 with the plan as built."""
    from types import SimpleNamespace

    from paper_2404_14195_amd import MPF_F32
    from paper_2404_14195_amd._lib import Tiles
    from paper_2404_14195_amd.solvers import ACMSolver
    d = mid_disc
    plan = d.tiles
    assert plan.h_max <= 819 < 900 <= plan.h_cap
    big = SimpleNamespace(rec=Tiles(count=plan.rec.count, halo=plan.rec.halo, lidx=plan.rec.lidx,
                                    h_cap=plan.h_cap, h_max=900), h_max=900, h_cap=plan.h_cap)
    a = ACMSolver(d, precision=MPF_F32, tile=64)  # lanes from the library
    b = ACMSolver(d, precision=MPF_F32, lanes=2, tile=64)
    one = ACMSolver(d, precision=MPF_F32, lanes=1, tile=64)
    try:
        d._tiles = big
        assert a.staged_now()
        a.run(40)
    finally:
        d._tiles = plan
    b.run(40)
    one.run(40)
    assert torch.equal(a.v, b.v) and torch.equal(a.p, b.p) and torch.equal(a.vmax, b.vmax)
    # one lane per node sums in another order: equal to rounding only
    assert torch.allclose(one.v, b.v, rtol=1e-4, atol=1e-9)


@pytest.mark.parametrize("precision, lanes, tile, staged", [(1, 1, 128, True), (3, 1, 128, True), (0, 1, 128, False),
                                                             (1, 2, 256, False), (0, 2, 256, False)])
def test_staged_acm_other_tile_sizes(disc, precision, lanes, tile, staged):
    """Two 128-node tiles per block at one lane per node run staged for an
    FP32 state; for an FP64 state their two halos (over 819 entries each on
    this cell) exceed 64 KiB, and a 256-node tile at two lanes (512 lanes,
    more than a block) is no block's tile: both fall back to the cached
    gather.  Either way the fields equal the cached gather's bit for bit."""
    from paper_2404_14195_amd.solvers import ACMSolver
    a = ACMSolver(disc, precision=precision, lanes=lanes, staged=True, tile=tile)
    b = ACMSolver(disc, precision=precision, lanes=lanes, staged=False)
    if precision == 0 and lanes == 1:
        assert disc.tiles_of(128).h_max > 819
    assert a.staged_now() == staged
    for s in (a, b):
        s.run(60)
    assert torch.equal(a.v, b.v) and torch.equal(a.p, b.p) and torch.equal(a.vmax, b.vmax)
