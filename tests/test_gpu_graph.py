"""Long ACM runs on small cells replay a captured HIP graph of 16 steps
(the launch overhead bounds those steps).  The graph holds the same kernels
with the same arguments in the same order as direct launches, so every replay
gives the same fields bit for bit; checked over several calls with eager work
and synchronisation between them."""
import sys

import pytest

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


@pytest.mark.parametrize("precision", [0, 1, 2, 3])
@pytest.mark.parametrize("edac", [False, True])
def test_acm_graph_replays_equal_direct_launches(disc, precision, edac):
    from paper_2404_14195_amd.solvers import ACMSolver
    a = ACMSolver(disc, precision=precision, edac=edac)
    b = ACMSolver(disc, precision=precision, edac=edac)
    for rep in range(3):
        a.run(80)  # five replays of the 16-step graph
        for _ in range(5):
            b.run(16)  # too short for a graph: direct launches
        ka, kb = a.permeability(), b.permeability()  # eager work between the calls
        assert ka == kb
        assert torch.equal(a.v, b.v) and torch.equal(a.p, b.p) and torch.equal(a.vmax, b.vmax)
        if a.comp is not None:
            assert torch.equal(a.comp, b.comp)
    # an odd length: graphs plus a direct remainder
    a.run(37)
    b.run(16), b.run(16), b.run(5)
    assert torch.equal(a.v, b.v) and torch.equal(a.p, b.p)


def test_acm_graph_run_reports_divergence(disc):
    """A NaN planted before a graphed run still ends it with MPF_ERR_DIVERGED."""
    from paper_2404_14195_amd._lib import MPFDiverged
    from paper_2404_14195_amd.solvers import ACMSolver
    s = ACMSolver(disc, precision=1)
    s.run(20)
    s.v[0, 7] = float("nan")
    with pytest.raises(MPFDiverged):
        s.run(64)


def test_acm_run_inside_a_callers_graph_capture(disc):
    """Called on a stream that the caller is capturing (no flags word, so no
    wait inside the call), the run enqueues its kernels directly into the
    caller's graph; three replays, with eager work between them, equal three
    eager runs of the same length bit for bit."""
    from paper_2404_14195_amd.solvers import ACMSolver
    a = ACMSolver(disc, precision=1, check=False)
    b = ACMSolver(disc, precision=1, check=False)
    a.run(10)
    b.run(10)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            a.run(40)
    torch.cuda.synchronize()
    for rep in range(3):
        g.replay()
        b.run(40)
        torch.cuda.synchronize()
        assert a.permeability() == b.permeability()  # eager work between the replays
        assert torch.equal(a.v, b.v) and torch.equal(a.p, b.p) and torch.equal(a.vmax, b.vmax)
