"""Both solvers on the paper's own discretisation and MLBM setting, through the
C ABI, against the oracle: Gaussian h-refinement (Sec. 2.4, Eq.
refinement_function, the clouds of the Appendix B studies at a coarser
h_min), N_L = 25, D3Q15 TRT with tau+ = 1 and Lambda = 1, and the ACM with
the sound-speed floor v_ref = 1 (C = 10); then the pointwise difference of
Eq. pointwise_error between the two solvers' fields, GPU against oracle."""
import sys

import numpy as np
import pytest

import nodecloud as nc
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NL = 25


@pytest.fixture(autouse=True)
def announce(request):
    print(f"\n[gpu-case] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield
    torch.cuda.synchronize()


@pytest.fixture(scope="module", params=[(0.062, 0.04), (0.6526, 0.03)], ids=["r0.062", "r0.6526"])
def paper_cell(request):
    """The paper's two cross-validation radii on Gaussian clouds: 3,152
    nodes (isolated small grain) and 2,946 nodes (grains overlapping their
    images, porosity 0.1)."""
    from paper_2404_14195_amd.solvers import Discretization
    assert torch.cuda.is_available()
    r, h = request.param
    c = nc.gauss_cloud(r, h, seed=7)
    return c, Discretization(c, nl=NL, M=32)


def _flux(c, d, vx):
    pp = d.plan
    return O.flux(pp.idx, O.plane_weights(c.pos, pp.idx, pp.shift), vx, d.n_all)


def test_paper_cells_both_solvers_and_pointwise_difference(paper_cell):
    from paper_2404_14195_amd import api
    from paper_2404_14195_amd.solvers import ACMSolver, MLBMSolver
    c, d = paper_cell
    # ACM, FP64, each side its own weights
    ga = ACMSolver(d, precision=0, v_ref=1.0)
    oa = O.ACM(c.pos, c.n_int, d.sten_host, c.nrm, sten_n=nc.neumann_stencils(c, NL), h_min=c.h_min, v_ref=1.0)
    ga.run(300)
    oa.run(300)
    va = ga.v.cpu().numpy().T
    assert np.abs(va - oa.v).max() <= 1e-10 * np.abs(oa.v).max()
    assert np.abs(ga.p.cpu().numpy() - oa.p).max() <= 1e-10 * np.abs(oa.p).max()
    assert ga.permeability() == pytest.approx(_flux(c, d, oa.v[:, 0]), rel=1e-10)
    # MLBM, the paper's D3Q15 TRT (tau- = 5/2), FP64, each side its own weights
    gm = MLBMSolver(d, q=15, precision=0, magic=1.0)
    om = O.MLBM(c.pos, c.n_int, d.sten_host, c.nrm, q=15, h_min=c.h_min, magic=1.0)
    assert gm.prm.tau_minus == pytest.approx(2.5) and om.tau_minus == pytest.approx(2.5)
    gm.run(200)
    om.run(200)
    vm_o, _ = om.macros()
    k_g, k_o = gm.permeability(), _flux(c, d, vm_o[:, 0])
    print(f"[paper cell r={c.r}] n={c.n} ACM k={ga.permeability():.10e}; MLBM k gpu={k_g:.10e} "
          f"oracle={k_o:.10e}", flush=True)
    assert k_g == pytest.approx(k_o, rel=1e-8)
    # pointwise difference MLBM vs MNS on the interior nodes: the GPU's from
    # its own states, the oracle's from its own
    vm, _ = gm.macros()
    delta, _, counts = api.pointwise(vm, ga.v, n_count=c.n_int, levels=(1.0, 0.25, 0.05))
    d_o, _ = O.pointwise(vm_o, oa.v)
    delta = delta.cpu().numpy()[:c.n_int]
    d_o = d_o[:c.n_int]
    assert np.abs(delta - d_o).max() <= 1e-6 * np.abs(d_o).max()
    print(f"[paper cell r={c.r}] delta after 200 MLBM / 300 ACM steps: median {np.median(d_o):.3e}, "
          f"counts above 1, 0.25, 0.05: {counts}", flush=True)
