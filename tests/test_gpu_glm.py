"""GLM divergence cleaning on the GPU (nine cell-centred fields) against the
oracle's GLM step: time step, ten CFL steps per field within 1e-12 (FP64)
on 2D/3D and ragged grids with an injected divergence and a non-zero psi,
both solvers and integrators, WENO-Z, the mixed-precision bound, the fused
CFL entry, and the cleaning of an injected div B error."""
import numpy as np
import pytest

import oracle as O
from paper_2511_20337_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2511_20337_amd import mhd
    mhd.lib()
    return torch.device("cuda:0")


def ctx_for(setup, dev, **kw):
    from paper_2511_20337_amd import mhd
    return mhd.Context(setup, dev, **kw)


def rel_err9(got, ref):
    """Per field max |got - ref| / max |ref|; momentum, field and psi take
    their group's scale when they hold only rounding noise."""
    groups = {1: (1, 2, 3), 2: (1, 2, 3), 3: (1, 2, 3), 5: (5, 6, 7), 6: (5, 6, 7),
              7: (5, 6, 7), 8: (5, 6, 7, 8)}
    errs = []
    for q in range(9):
        scale = np.abs(ref[q]).max()
        gs = max(np.abs(ref[g]).max() for g in groups.get(q, (q,)))
        if scale <= 1e-13 * gs:
            scale = gs
        errs.append(float(np.abs(got[q] - ref[q]).max() / (scale if scale > 0 else 1.0)))
    return np.array(errs)


def _case(name):
    if name == "ot2d":
        s, U = W.orszag_tang_2d(64)
    elif name == "turb3d":
        s, U = W.turbulence_3d(32)
    elif name in ("ragged3", "ragged3_hll", "ragged3_rk3", "ragged3_mixed", "ragged3_wenoz"):
        lim = "wenoz" if name == "ragged3_wenoz" else "vanleer"
        s, U = W.generic_state(3, 20, 18, 37, lim, "hll" if name == "ragged3_hll" else "hlld",
                               seed=9)
    else:  # ragged2
        s, U = W.generic_state(2, 28, 20, 1, "minmod", "hlld", seed=4)
    s, U9 = W.glm_from_ct(s, U)
    if name.startswith("ragged"):
        rng = np.random.default_rng(17)
        U9[8] = 0.02 * rng.normal(size=U9[8].shape)  # a cleaning field to transport
        U9[5] += 0.01 * rng.normal(size=U9[5].shape)  # and a divergence to clean
    if name == "ragged3_rk3":
        s = dict(s, integrator="rk3")
    if name == "ragged3_mixed":
        s = dict(s, precision="mixed")
    return s, U9


def _run_gpu(ctx, U0, nsteps, dev):
    U = torch.from_numpy(U0).to(dev)
    dts = []
    for _ in range(nsteps):
        dt = ctx.dt(U)
        dts.append(dt)
        ctx.step(U, dt)
    torch.cuda.synchronize()
    return U.cpu().numpy(), np.array(dts)


@pytest.mark.parametrize("dim", [2, 3])
def test_glm_dt_parity(dev, dim):
    s, U = _case("ragged2" if dim == 2 else "ragged3")
    ctx = ctx_for(s, dev)
    got = ctx.dt(torch.from_numpy(U).to(dev))
    assert got == pytest.approx(O.glm_dt(O.cfg_from(s), U), rel=1e-14)


@pytest.mark.parametrize("case", ["ot2d", "turb3d", "ragged2", "ragged3", "ragged3_hll",
                                  "ragged3_rk3", "ragged3_wenoz", "ragged3_mixed"])
def test_glm_ten_step_parity(dev, case):
    s, U0 = _case(case)
    print("glm 10-step parity", case, flush=True)
    ctx = ctx_for(s, dev)
    got, dts = _run_gpu(ctx, U0, 10, dev)
    c = O.cfg_from(s)
    if case == "ragged3_mixed":
        ref = O.glm_run_dts(c, U0, dts)
        err = rel_err9(got, ref)
        assert (err <= 2e-5).all(), err
        return
    ref, odts = O.glm_run(c, U0, 10)
    np.testing.assert_allclose(dts, odts, rtol=1e-13)
    err = rel_err9(got, ref)
    assert (err <= 1e-12).all(), err


@pytest.mark.parametrize("case", ["ragged2", "ragged3"])
def test_glm_step_cfl_matches_separate_cfl_pass(dev, case):
    """mhd_step_cfl (the CFL bound reduced in the first stage's primitive
    kernel) equals mhd_dt_device + mhd_step_device_dt bit for bit."""
    s, U0 = _case(case)
    ctx = ctx_for(s, dev)
    Ua = torch.from_numpy(U0).to(dev)
    Ub = Ua.clone()
    dta = torch.zeros(1, dtype=torch.float64, device=dev)
    dtb = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(3):
        ctx.dt_device(Ua, dta)
        ctx.step_device_dt(Ua, dta)
        ctx.step_cfl(Ub, dtb)
        assert dta.item() == dtb.item()
        assert torch.equal(Ua, Ub)


@pytest.mark.parametrize("dim", [2, 3])
def test_glm_cleans_an_injected_divergence_on_gpu(dev, dim):
    """The injected div B error of the oracle's cleaning pin, on the GPU at
    twice the oracle's resolution: ten steps against the oracle (1e-12), then
    the L2 norm of div B is below 0.9 of its initial value after ten steps and
    below 0.4 after sixty (measured 0.86 and 0.32 in 2D at 128^2, 0.49 and
    0.27 in 3D at 64^3, as in the oracle at these sizes; in 3D the norm rises
    once, near step 20, where the pulse meets its periodic images)."""
    n = 128 if dim == 2 else 64
    s, U0 = W.glm_divergence_bump(dim, n)
    c = O.cfg_from(s)
    ctx = ctx_for(s, dev)
    got, dts = _run_gpu(ctx, U0, 10, dev)
    ref = O.glm_run_dts(c, U0, dts)
    assert (rel_err9(got, ref) <= 1e-12).all()
    U = torch.from_numpy(got).to(dev)
    d0 = np.sqrt((O.divb_centred(c, U0) ** 2).mean())
    d10 = np.sqrt((O.divb_centred(c, got) ** 2).mean())
    ctx.run(U, 50)
    d60 = np.sqrt((O.divb_centred(c, U.cpu().numpy()) ** 2).mean())
    print("glm div B after 10 and 60 steps", dim, d10 / d0, d60 / d0, flush=True)
    assert d10 < 0.9 * d0 and d60 < 0.4 * d0, (d0, d10, d60)
    ctx.check()


def test_glm_unsupported_calls(dev):
    from paper_2511_20337_amd import mhd
    s, U9 = _case("ragged2")
    ctx = ctx_for(s, dev, with_adjoint=True)
    U = torch.from_numpy(U9).to(dev)
    for call in (lambda: ctx.rhs(U), lambda: ctx.adjoint_step(U, 1e-3, torch.ones_like(U)),
                 lambda: mhd.mhd_dt_device_noalloc(ctx.ctx, U, ctx.dt_dev)):
        with pytest.raises(mhd.MHDError) as e:
            call()
        assert e.value.status == mhd.MHD_ERR_UNSUPPORTED
