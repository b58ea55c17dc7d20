"""The C ABI on its own: a host program that includes only include/mhd.h and
the HIP runtime (tests/c_abi/step_cli.cpp, compiled by build()) runs steps of
mhd_step_cfl in a child process, and its state and dt must equal, bit for
bit, those of the Python binding on the same input."""
import os
import subprocess

import numpy as np
import pytest

from paper_2511_20337_amd import mhd, workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c_abi", "step_cli")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mhd.lib()
    return torch.device("cuda:0")


def _cases():
    s1, U1 = W.generic_state(3, 20, 18, 37, "vanleer", "hlld", seed=9)
    s2, U2 = W.generic_state(3, 20, 18, 37, "wenoz", "hlld", seed=9)
    s2 = dict(s2, integrator="rk3")
    s3, U3 = W.orszag_tang_2d(32)
    s3 = dict(s3, limiter="minmod", riemann="hll", precision="mixed")
    return {"plm_rk2_3d": (s1, U1), "wenoz_rk3_3d": (s2, U2), "mixed_2d": (s3, U3)}


@pytest.mark.parametrize("case", ["plm_rk2_3d", "wenoz_rk3_3d", "mixed_2d"])
def test_c_abi_program_matches_binding(dev, case, tmp_path):
    assert os.path.exists(EXE), "tests/c_abi/step_cli is missing: run __graft_entry__.build()"
    s, U0 = _cases()[case]
    nsteps = 3
    print("c abi", case, flush=True)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    np.ascontiguousarray(U0, dtype=np.float64).tofile(fin)
    c = mhd.config_from(s)
    args = [str(v) for v in (c.dim, c.nx, c.ny, c.nz, repr(c.xmin), repr(c.xmax), repr(c.ymin),
                             repr(c.ymax), repr(c.zmin), repr(c.zmax), repr(c.gamma), repr(c.cfl),
                             c.limiter, c.riemann, c.precision, c.integrator)]
    r = subprocess.run([EXE, str(fin), str(fout), str(nsteps)] + args, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = np.fromfile(fout, dtype=np.float64)
    assert out.size == U0.size + 1
    ctx = mhd.Context(s, dev)
    U = torch.from_numpy(U0).to(dev)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(nsteps):
        ctx.step_cfl(U, dt)
    ctx.check()
    np.testing.assert_array_equal(out[:-1].reshape(U0.shape), U.cpu().numpy())
    assert out[-1] == dt.item()
