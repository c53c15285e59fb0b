"""The allocation-free flux reduction (mpf_flux_planes_noalloc) against the
workspace form (mpf_flux_planes), through the C ABI: bit-identical results
(same kernels, same fixed summation order) on two calls in a row, the second
with a smaller input, in FP64 and FP32, and the size limit."""
import ctypes
import sys

import numpy as np
import pytest

import nodecloud as nc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def test_noalloc_flux_equals_workspace_flux():
    print("\n[gpu-case] no-alloc flux", flush=True)
    from paper_2404_14195_amd import MPFError, api
    from paper_2404_14195_amd._lib import lib
    assert torch.cuda.is_available()
    c = nc.sphere_cloud(0.3, 0.04, 0.3, 0.1, seed=1)
    pos = dev(c.pos.T, torch.float64)
    sten = api.solver_stencils(pos, c.n_int, 30)
    rng = np.random.default_rng(3)
    for M, dt in ((64, torch.float64), (24, torch.float32), (64, torch.float32), (8, torch.float64)):
        pp = nc.plane_plan(c, M, 30)
        s_idx = dev(pp.idx.T, torch.int32)
        s_w = api.rbffd_weights(pos, s_idx, [("shift_row",)], rowvec=dev(pp.shift.T, torch.float64))[0][0]
        s_w = s_w.contiguous()
        vx = dev(rng.normal(size=c.n), dt)
        n_all = 5 * M * M
        ref = api.flux_planes(s_idx, s_w, vx, n_all).cpu().numpy()
        q = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        api.flux_planes_noalloc(s_idx, s_w, vx, n_all, q)
        got = q.cpu().numpy()
        print(f"[no-alloc] M={M} {dt}: ns={s_idx.shape[1]} ref={ref[0]!r} got={got[0]!r}", flush=True)
        assert got[0] == ref[0]  # bitwise
    assert lib().mpf_flux_planes_noalloc_max() == 8192 * 256
    # beyond the static partials: rejected on the host, nothing launched
    fake = ctypes.c_void_p(0x1000)
    rc = lib().mpf_flux_planes_noalloc(8192 * 256 + 1, 30, fake, fake, fake, 0, 1, fake, None)
    assert rc == -5
    with pytest.raises(MPFError):
        api.check(rc, "mpf_flux_planes_noalloc")
