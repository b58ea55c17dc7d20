"""The allocation-free time step (mhd_dt_device_noalloc) against the workspace
one (mhd_dt_device), through the C ABI: two calls in a row on one GPU, the
second on a smaller grid, then the flag of an unphysical state and its reset.
"""
import numpy as np
import pytest

import oracle as O
from paper_2511_20337_amd import mhd, workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dt_pair(setup, U0, dev):
    ctx = mhd.Context(setup, dev)
    U = torch.from_numpy(U0).to(dev)
    ref = torch.zeros(1, dtype=torch.float64, device=dev)
    got = torch.full((1,), -1.0, dtype=torch.float64, device=dev)
    flag = torch.full((1,), 7, dtype=torch.int32, device=dev)
    ctx.dt_device(U, ref)
    mhd.mhd_dt_device_noalloc(ctx.ctx, U, got, flag)
    torch.cuda.synchronize()
    return float(ref.item()), float(got.item()), int(flag.item())


def test_noalloc_dt_matches_workspace_dt_twice():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dev = torch.device("cuda:0")
    # first a 3D grid that uses all 2048 partials, then a smaller 2D one that
    # uses 4, so the second call reads none of the first call's stale partials
    cases = [W.turbulence_3d(96), W.orszag_tang_2d(32)]
    for setup, U0 in cases:
        ref, got, flag = _dt_pair(setup, U0, dev)
        print("noalloc dt", setup["name"], setup["nx"], ref, got, flush=True)
        assert got == ref  # same kernels, and a minimum is exact in any order
        assert flag == 0
        assert got == pytest.approx(O.dt(O.cfg_from(setup), U0), rel=1e-14)


def test_noalloc_flag_reports_and_resets():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dev = torch.device("cuda:0")
    setup, U0 = W.turbulence_3d(16)
    bad = U0.copy()
    bad[4, 3, 5, 7] = -1.0  # negative total energy: p < 0 at that cell
    _, _, flag = _dt_pair(setup, bad, dev)
    assert flag == 1
    ref, got, flag = _dt_pair(setup, U0, dev)
    assert flag == 0  # the array's flag starts every call at zero
    assert got == ref
