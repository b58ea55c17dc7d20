"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar (FP64): per field, max |gpu - oracle| / max |oracle| <= 1e-12 (a field
that is identically zero is scaled by the largest field of its group:
momentum or magnetic field). Mixed precision: stated per-field bounds.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2511_20337_amd import workloads as W
from tests.oracle_patches import oracle_at_samples

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GROUPS = {1: (1, 2, 3), 2: (1, 2, 3), 3: (1, 2, 3), 5: (5, 6, 7), 6: (5, 6, 7), 7: (5, 6, 7)}


def rel_err(got, ref):
    errs = []
    for q in range(8):
        scale = np.abs(ref[q]).max()
        if q in GROUPS:
            # a field that vanishes in exact arithmetic holds only rounding
            # noise, which two correct evaluations need not share: scale it
            # by its group (momentum or magnetic field)
            gscale = max(np.abs(ref[g]).max() for g in GROUPS[q])
            if scale <= 1e-13 * gscale:
                scale = gscale
        scale = scale if scale > 0 else 1.0
        errs.append(float(np.abs(got[q] - ref[q]).max() / scale))
    return np.array(errs)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2511_20337_amd import mhd
    mhd.lib()
    return torch.device("cuda:0")


def ctx_for(setup, dev, **kw):
    from paper_2511_20337_amd import mhd
    return mhd.Context(setup, dev, **kw)


def ragged(dim, lim, solver, precision="fp64"):
    if dim == 2:
        # ragged, non-square grid with Orszag-Tang-like fields
        s2 = W.make_setup("ot_ragged", 2, 28, 20, 1, (0, 1, 0, 1, 0, 1), 5 / 3, 0.4, lim, solver,
                          precision)
        x, y, _ = W.centres(s2)
        dx, dy, _ = W.spacing(s2)
        sh = (1, 20, 28)
        rng = np.random.default_rng(3)
        vx = np.broadcast_to(-np.sin(2 * np.pi * y), sh) + 0.05 * rng.uniform(-1, 1, sh)
        vy = np.broadcast_to(np.sin(2 * np.pi * x), sh) + 0.05 * rng.uniform(-1, 1, sh)
        Az = np.broadcast_to((np.cos(2 * np.pi * (y - dy / 2)) / (2 * np.pi) +
                              np.cos(4 * np.pi * (x - dx / 2)) / (4 * np.pi)) / np.sqrt(4 * np.pi),
                             sh)
        bx, by = W.curl_of_edge_potential(s2, None, None, Az)
        bz = 0.1 * np.cos(2 * np.pi * (x + 2 * y)) * np.ones(sh)
        U = W.assemble(s2, 0.22 + 0.05 * np.sin(2 * np.pi * x) * np.ones(sh), vx, vy,
                       0.2 * np.sin(2 * np.pi * y) * np.ones(sh), 0.13 * np.ones(sh), bx, by, bz)
        return s2, U
    # ragged 13 x 10 x 9 grid, smooth periodic fields
    s3 = W.make_setup("turb_ragged", 3, 13, 10, 9, (0, 1, 0, 1, 0, 1), 5 / 3, 0.3, lim, solver,
                      precision)
    x, y, z = W.centres(s3)
    dx, dy, dz = W.spacing(s3)
    sh = (9, 10, 13)
    rng = np.random.default_rng(4)
    tp = 2 * np.pi

    def f(a, b, c, ph):
        return np.sin(tp * (a * x + b * y + c * z) + ph) * np.ones(sh)
    rho = 1 + 0.2 * f(1, 1, 0, 0.3) + 0.01 * rng.uniform(-1, 1, sh)
    p = 0.9 + 0.2 * f(0, 1, 1, 1.1)
    vx, vy, vz = 0.8 * f(0, 1, 1, 0.2), 0.7 * f(1, 0, 1, 0.9), 0.6 * f(1, 1, 0, 2.0)

    def A(ax, px, py, pz):
        k = [(1, 2, 1), (2, 1, 1), (1, 1, 2)][ax]
        return 0.05 * np.sin(tp * (k[0] * px + k[1] * py + k[2] * pz) + ax) * np.ones(sh)
    bx, by, bz = W.curl_of_edge_potential(s3, A(0, x, y - dy / 2, z - dz / 2),
                                          A(1, x - dx / 2, y, z - dz / 2),
                                          A(2, x - dx / 2, y - dy / 2, z))
    U = W.assemble(s3, rho, vx, vy, vz, p, bx + 0.3, by - 0.2, bz + 0.1)
    return s3, U


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("lim", ["minmod", "vanleer", "wenoz"])
@pytest.mark.parametrize("solver", ["hlld", "hll"])
def test_rhs_parity_fp64(dev, dim, lim, solver):
    s, U = ragged(dim, lim, solver)
    print("rhs parity", s["name"], lim, solver, flush=True)
    ctx = ctx_for(s, dev)
    Ug = torch.from_numpy(U).to(dev)
    got = ctx.rhs(Ug).cpu().numpy()
    ref = O.rhs(O.cfg_from(s), U)
    err = rel_err(got, ref)
    assert (err <= 1e-12).all(), err


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("solver", ["hlld", "hll"])
@pytest.mark.parametrize("lim", ["minmod", "vanleer"])
def test_rhs_parity_degenerate_star_states(dev, dim, solver, lim):
    """A field along x only (B_t = 0 on x-faces), Alfven speed above sound
    speed, and a compact bump in an otherwise exactly uniform state: the
    x-faces outside the bump see identical states with rho (S-u)(S-S_M) equal
    to B_n^2 up to rounding, where HLLD takes its degenerate branch."""
    s, U = W.aligned_field_bump(dim, 24, 16, 8, limiter=lim, riemann=solver)
    print("rhs parity, degenerate star states", dim, lim, solver, flush=True)
    ctx = ctx_for(s, dev)
    got = ctx.rhs(torch.from_numpy(U).to(dev)).cpu().numpy()
    ref = O.rhs(O.cfg_from(s), U)
    assert np.isfinite(got).all()
    err = rel_err(got, ref)
    assert (err <= 1e-12).all(), err


@pytest.mark.parametrize("dim", [2, 3])
def test_dt_parity(dev, dim):
    s, U = ragged(dim, "vanleer", "hlld")
    ctx = ctx_for(s, dev)
    got = ctx.dt(torch.from_numpy(U).to(dev))
    assert got == pytest.approx(O.dt(O.cfg_from(s), U), rel=1e-14)


def _run_gpu(ctx, U0, nsteps, dev):
    U = torch.from_numpy(U0).to(dev)
    dts = []
    for _ in range(nsteps):
        dt = ctx.dt(U)
        dts.append(dt)
        ctx.step(U, dt)
    torch.cuda.synchronize()
    return U.cpu().numpy(), np.array(dts)


@pytest.mark.parametrize("case", ["orszag_tang_128", "turbulence_64", "blast_32",
                                  "kh_64", "ragged2", "ragged2_odd", "ragged3", "ragged3_runs"])
def test_ten_step_parity_fp64(dev, case):
    """Ten CFL steps against the oracle. ragged3_runs (20 x 18 x 37) has
    partial 16 x 16 columns in x and y and z-runs of 16, 16 and 5 planes. In
    3D an even nx takes the two-cell update kernel, an odd one (ragged3
    13 x 10 x 9) the one-cell kernel; 2D grids (ragged2_odd 27 x 20 with a
    partial tile among them) the kernel that forms the EMF with the update."""
    if case == "orszag_tang_128":
        s, U0 = W.orszag_tang_2d(128)
    elif case == "turbulence_64":
        s, U0 = W.turbulence_3d(64)
    elif case == "blast_32":
        s, U0 = W.blast_3d(32, precision="fp64")
    elif case == "kh_64":
        s, U0, _ = W.kelvin_helmholtz_2d(64)
    elif case == "ragged2":
        s, U0 = ragged(2, "minmod", "hlld")
    elif case == "ragged2_odd":
        s, U0 = W.generic_state(2, 27, 20, 1, "vanleer", "hlld", seed=4)
    elif case == "ragged3":
        s, U0 = ragged(3, "vanleer", "hll")
    else:
        s, U0 = W.generic_state(3, 20, 18, 37, "vanleer", "hlld", seed=9)
    print("10-step parity", case, flush=True)
    ctx = ctx_for(s, dev)
    got, dts = _run_gpu(ctx, U0, 10, dev)
    c = O.cfg_from(s)
    ref, odts = O.run(c, U0, 10)
    np.testing.assert_allclose(dts, odts, rtol=1e-13)
    err = rel_err(got, ref)
    assert (err <= 1e-12).all(), err


@pytest.mark.parametrize("case", ["ragged3_runs", "orszag_tang_128", "mixed", "wenoz3", "wenoz2"])
def test_ten_step_parity_rk3(dev, case):
    """SSP-RK3 (Eq. (RK3)): ten CFL steps against the oracle's SSP-RK3, FP64
    to 1e-12 per field; in mixed precision against the oracle's mixed
    variant with the mixed path's stated bound (2e-5)."""
    if case == "ragged3_runs":
        s, U0 = W.generic_state(3, 20, 18, 37, "vanleer", "hlld", seed=9)
    elif case == "orszag_tang_128":
        s, U0 = W.orszag_tang_2d(128)
    elif case == "mixed":
        s, U0 = W.generic_state(3, 20, 18, 37, "vanleer", "hlld", seed=9)
        s = dict(s, precision="mixed")
    elif case == "wenoz3":  # the paper's scheme: WENO-Z + RK3 + HLLD + CT
        s, U0 = W.generic_state(3, 20, 18, 37, "wenoz", "hlld", seed=9)
    else:
        s, U0 = W.orszag_tang_2d(128, limiter="wenoz")
    s = dict(s, integrator="rk3")
    print("rk3 10-step parity", case, flush=True)
    ctx = ctx_for(s, dev)
    got, dts = _run_gpu(ctx, U0, 10, dev)
    ref, odts = O.run(O.cfg_from(s), U0, 10)
    np.testing.assert_allclose(dts, odts, rtol=1e-13 if case != "mixed" else 1e-6)
    err = rel_err(got, ref if case != "mixed" else O.run_dts(O.cfg_from(s), U0, dts))
    assert (err <= (1e-12 if case != "mixed" else 2e-5)).all(), err


def test_orszag_tang_3d_ten_step_parity(dev):
    """The paper's 3D Orszag-Tang problem (its first benchmark) at 32^3, ten
    CFL steps of this path's scheme against the oracle."""
    s, U0 = W.orszag_tang_3d(32)
    ctx = ctx_for(s, dev)
    got, dts = _run_gpu(ctx, U0, 10, dev)
    ref, odts = O.run(O.cfg_from(s), U0, 10)
    np.testing.assert_allclose(dts, odts, rtol=1e-13)
    err = rel_err(got, ref)
    assert (err <= 1e-12).all(), err


def test_orszag_tang_3d_352_wenoz_rk3_sampled_parity(dev):
    """The paper's 3D Orszag-Tang problem at its per-GPU size, 352^3, with the
    paper's scheme (WENO-Z + SSP-RK3 + HLLD + CT with the UCT-HLLD average) as
    the benchmark times it:
    two steps of mhd_step_cfl against the separate CFL pass bit for bit, the
    first dt against the oracle on the whole grid, the state after two steps
    against the oracle at sampled cells (corners and random interior; two RK3
    steps of the +-3-cell stencil reach 24 cells, the patches reach 26), then
    conservation and div B on the whole grid."""
    s, U0 = W.orszag_tang_3d(352, limiter="wenoz")
    s = dict(s, integrator="rk3", emf="uct_hlld")
    print("352^3 wenoz rk3: 2 steps, step_cfl against the separate pass", flush=True)
    ctx = ctx_for(s, dev)
    c = O.cfg_from(s)
    U = torch.from_numpy(U0).to(dev)
    Ub = U.clone()
    dta = torch.zeros(1, dtype=torch.float64, device=dev)
    dtb = torch.zeros(1, dtype=torch.float64, device=dev)
    dts = []
    for step in range(2):
        ctx.dt_device(U, dta)
        ctx.step_device_dt(U, dta)
        ctx.step_cfl(Ub, dtb)
        assert dta.item() == dtb.item(), step
        assert torch.equal(U, Ub), step
        dts.append(dtb.item())
    del Ub
    ctx.check()
    assert dts[0] == pytest.approx(O.dt(c, U0), rel=1e-14)
    print("352^3 wenoz rk3: sampled oracle patches", flush=True)
    got = U.cpu().numpy()
    rng = np.random.default_rng(21)
    cen = [(0, 0, 0), (351, 351, 351), (0, 351, 176), (351, 0, 1)]
    cen += [tuple(int(v) for v in rng.integers(0, 352, 3)) for _ in range(8)]
    ref = oracle_at_samples(s, U0, dts, cen, radius=26)
    g = np.array([got[:, k, j, i] for (k, j, i) in cen])
    scale = np.abs(U0).max(axis=(1, 2, 3))
    scale[5:8] = np.abs(U0[5:8]).max()  # B_z starts at zero: the field's scale
    err = (np.abs(g - ref) / scale).max(axis=0)
    assert (err <= 1e-12).all(), err
    print("352^3 wenoz rk3: invariants", flush=True)
    for q in range(8):
        mag = np.abs(U0[q]).sum() if q < 5 else np.abs(U0[5:8]).sum()
        assert abs(got[q].sum() - U0[q].sum()) <= 1e-12 * mag, q
    div = O.divb(c, got)
    assert np.abs(div).max() * (1 / 352) / np.abs(got[5:]).max() <= 1e-12


def _cp_alfven_gpu_error(dev, n, limiter, integrator):
    """L1 error of B after one period of the 3D CP Alfven wave on the GPU."""
    s, U0, period = W.cp_alfven(n, dim=3, cfl=0.3, limiter=limiter)
    s = dict(s, integrator=integrator)
    ctx = ctx_for(s, dev)
    U = torch.from_numpy(U0).to(dev)
    nsteps = int(math.ceil(period / ctx.dt(U)))
    for _ in range(nsteps):
        ctx.step(U, period / nsteps)
    ctx.check()
    return float(np.mean(np.abs(U.cpu().numpy()[5:8] - U0[5:8]))), s, U0, period, nsteps


def test_cp_alfven_3d_paper_scheme_on_gpu(dev):
    """The paper's scheme (WENO-Z + SSP-RK3 + HLLD + CT) on its second
    benchmark problem, the 3D circularly polarised Alfven wave: after one
    period the L1 error of B at 32^3 is the oracle's; from 64^3 to 256^3 it
    falls at order >= 1.8 (the CT edge values are PLM, so the scheme is second
    order overall) and stays below 0.6 of PLM + SSP-RK2's at every size (the
    oracle: 0.55 at 16^3, 0.52 at 32^3)."""
    e32, s, U0, period, nsteps = _cp_alfven_gpu_error(dev, 32, "wenoz", "rk3")
    ref = O.run_dts(O.cfg_from(s), U0, [period / nsteps] * nsteps)
    e_ref = float(np.mean(np.abs(ref[5:8] - U0[5:8])))
    print("cp-alfven wenoz rk3 32", e32, e_ref, flush=True)
    assert e32 == pytest.approx(e_ref, rel=1e-9)
    errs = []
    for n in (64, 128, 256):
        ew = _cp_alfven_gpu_error(dev, n, "wenoz", "rk3")[0]
        ep = _cp_alfven_gpu_error(dev, n, "vanleer", "rk2")[0]
        print("cp-alfven", n, "wenoz+rk3", ew, "vanleer+rk2", ep, flush=True)
        assert ew <= 0.6 * ep, (n, ew, ep)
        errs.append(ew)
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print("cp-alfven wenoz rk3 orders", orders, flush=True)
    assert min(orders) >= 1.8, orders


def test_cp_alfven_3d_second_order_on_gpu(dev):
    """The paper's second benchmark problem, the 3D circularly polarised
    Alfven wave (k = 2 pi (1,1,1), eps = 0.1), an exact nonlinear solution: after
    one period the GPU result returns to the initial state with an L1 error of
    B that falls at second order, at sizes past the oracle's (64^3 to 256^3).
    (Between 32^3 and 64^3 the rate dips to 1.2-1.4 in the oracle as well,
    whose errors the GPU matches: 1.6749e-3 at 32^3, 6.9851e-4 at 64^3;
    12^3 to 24^3 gives 2.3, 64^3 to 128^3 1.83.)"""
    errs = []
    for n in (64, 128, 256):
        s, U0, period = W.cp_alfven(n, dim=3, cfl=0.3)
        ctx = ctx_for(s, dev)
        U = torch.from_numpy(U0).to(dev)
        nsteps = int(math.ceil(period / ctx.dt(U)))
        for _ in range(nsteps):
            ctx.step(U, period / nsteps)
        ctx.check()
        errs.append(float(np.mean(np.abs(U.cpu().numpy()[5:8] - U0[5:8]))))
        print("cp-alfven", n, nsteps, errs[-1], flush=True)
    orders = [math.log2(errs[q] / errs[q + 1]) for q in range(2)]
    assert min(orders) >= 1.75, (errs, orders)


def test_device_dt_path_matches_host_dt(dev):
    s, U0 = W.turbulence_3d(32)
    ctx = ctx_for(s, dev)
    a, _ = _run_gpu(ctx, U0, 5, dev)
    U = torch.from_numpy(U0).to(dev)
    ctx.run(U, 5)
    np.testing.assert_array_equal(U.cpu().numpy(), a)


@pytest.mark.parametrize("case", ["ragged3_runs", "short_runs", "mixed", "ragged2", "ot2d_128",
                                  "ragged2_1122", "rk3", "wenoz", "wenoz2"])
def test_step_cfl_matches_separate_cfl_pass(dev, case):
    """mhd_step_cfl (the CFL reduction inside the first face kernel) gives
    the dt of mhd_dt_device and the state of mhd_step_device_dt, bit for bit,
    and that dt is the oracle's. ragged3_runs: 20 x 18 x 37 (z-runs of 16, 16,
    5 planes; partial columns); short_runs: 12 x 10 x 7 (one run shorter than
    16); mixed: the first state in mixed precision; ragged2: 2D 28 x 20 (the
    reduction in the tiled face kernel, finished by every workgroup of the
    update; partial 16 x 16 tiles); ot2d_128: 64 whole tiles; ragged2_1122:
    530 x 520, 1122 tiles, more than the update finishes itself, so
    k_cfl_final does; wenoz: the reduction in the WENO-Z primitive kernel (53
    workgroups of 256 cells, the last one holding 8); wenoz2: 2D WENO-Z with
    the separate pass."""
    if case == "ragged3_runs":
        s, U0 = W.generic_state(3, 20, 18, 37, "vanleer", "hlld", seed=9)
    elif case == "short_runs":
        s, U0 = W.generic_state(3, 12, 10, 7, "minmod", "hll", seed=5)
    elif case == "mixed":
        s, U0 = W.generic_state(3, 20, 18, 37, "vanleer", "hlld", seed=9)
        s = dict(s, precision="mixed")
    elif case == "rk3":
        s, U0 = W.generic_state(3, 20, 18, 37, "vanleer", "hlld", seed=9)
        s = dict(s, integrator="rk3")
    elif case == "wenoz":
        s, U0 = W.generic_state(3, 20, 18, 37, "wenoz", "hlld", seed=9)
    elif case == "wenoz2":
        s, U0 = ragged(2, "wenoz", "hlld")
    elif case == "ot2d_128":
        s, U0 = W.orszag_tang_2d(128)
    elif case == "ragged2_1122":
        s, U0 = W.generic_state(2, 530, 520, 1, "vanleer", "hlld", seed=6)
    else:
        s, U0 = ragged(2, "minmod", "hlld")
    print("step_cfl", case, flush=True)
    ctx = ctx_for(s, dev)
    Ua = torch.from_numpy(U0).to(dev)
    Ub = Ua.clone()
    dta = torch.zeros(1, dtype=torch.float64, device=dev)
    dtb = torch.zeros(1, dtype=torch.float64, device=dev)
    for step in range(3):
        ctx.dt_device(Ua, dta)
        ctx.step_device_dt(Ua, dta)
        ctx.step_cfl(Ub, dtb)
        assert dta.item() == dtb.item(), (step, dta.item(), dtb.item())
        np.testing.assert_array_equal(Ua.cpu().numpy(), Ub.cpu().numpy())
        if step == 0:
            assert dtb.item() == pytest.approx(O.dt(O.cfg_from(s), U0), rel=1e-14)
    ctx.check()


def test_full_size_256_sampled_parity_and_invariants(dev):
    """Full 256^3 turbulence in the configuration the benchmark times: the
    time step against the oracle on the whole grid, two steps against the
    oracle at sampled cells (corners, faces and random interior), one step
    of mhd_step_cfl (the benchmark's entry) against the separate CFL pass bit
    for bit, then ten more steps checked for conservation and div B on the
    whole grid."""
    s, U0 = W.turbulence_3d(256)
    print("256^3: dt + 2 steps", flush=True)
    ctx = ctx_for(s, dev)
    U = torch.from_numpy(U0).to(dev)
    c = O.cfg_from(s)
    dt0 = ctx.dt(U)
    assert dt0 == pytest.approx(O.dt(c, U0), rel=1e-14)
    ctx.step(U, dt0)
    dt1 = ctx.dt(U)
    assert dt1 == pytest.approx(O.dt(c, U.cpu().numpy()), rel=1e-14)
    ctx.step(U, dt1)
    got = U.cpu().numpy()
    rng = np.random.default_rng(12)
    cen = [(0, 0, 0), (255, 255, 255), (0, 255, 128), (255, 0, 1), (128, 128, 128)]
    cen += [tuple(int(v) for v in rng.integers(0, 256, 3)) for _ in range(11)]
    ref = oracle_at_samples(s, U0, [dt0, dt1], cen)
    g = np.array([got[:, k, j, i] for (k, j, i) in cen])
    scale = np.abs(U0).max(axis=(1, 2, 3))
    err = (np.abs(g - ref) / scale).max(axis=0)
    assert (err <= 1e-12).all(), err
    print("256^3: the benchmark's step entry against the separate CFL pass", flush=True)
    Ub = U.clone()
    dta = torch.zeros(1, dtype=torch.float64, device=dev)
    dtb = torch.zeros(1, dtype=torch.float64, device=dev)
    ctx.dt_device(U, dta)
    ctx.step_device_dt(U, dta)
    ctx.step_cfl(Ub, dtb)
    assert dta.item() == dtb.item()
    assert torch.equal(U, Ub)
    del Ub
    print("256^3 invariants: 10 more steps", flush=True)
    ctx.run(U, 10)
    Uf = U.cpu().numpy()
    for q in range(8):
        s0, s1 = U0[q].sum(), Uf[q].sum()
        assert abs(s1 - s0) <= 1e-12 * np.abs(U0[q]).sum(), q
    div = O.divb(c, Uf)
    assert np.abs(div).max() * (1 / 256) / np.abs(Uf[5:]).max() <= 1e-12


@pytest.mark.parametrize("n", [4, 5])
def test_minimum_sizes(dev, n):
    for dim in (2, 3):
        s, U0 = W.smooth_random(dim=dim, n=n, seed=2, amp=0.1)
        ctx = ctx_for(s, dev)
        got, _ = _run_gpu(ctx, U0, 2, dev)
        ref, _ = O.run(O.cfg_from(s), U0, 2)
        err = rel_err(got, ref)
        assert (err <= 1e-12).all(), (dim, err)


def test_uniform_state_preserved_bitwise(dev):
    for dim in (2, 3):
        s, U0 = W.uniform(dim=dim, n=8)
        ctx = ctx_for(s, dev)
        U = torch.from_numpy(U0).to(dev)
        ctx.step(U, 0.01)
        np.testing.assert_array_equal(U.cpu().numpy(), U0)


def test_deterministic_bitwise(dev):
    s, U0 = W.turbulence_3d(32)
    ctx = ctx_for(s, dev)
    a, _ = _run_gpu(ctx, U0, 3, dev)
    b, _ = _run_gpu(ctx, U0, 3, dev)
    np.testing.assert_array_equal(a, b)


def test_unphysical_flag_and_errors(dev):
    from paper_2511_20337_amd import mhd
    s, U0 = W.uniform(dim=3, n=8)
    U0 = U0.copy()
    U0[4, 2, 3, 4] = 1e-3  # E below kinetic + magnetic energy: p < 0
    ctx = ctx_for(s, dev)
    U = torch.from_numpy(U0).to(dev)
    with pytest.raises(mhd.Unphysical):
        ctx.dt(U)
    ctx.check()  # flag was cleared by the report
    ctx.step(U, 1e-3)
    with pytest.raises(mhd.Unphysical):
        ctx.check()
    with pytest.raises(mhd.MHDError) as e:
        ctx.step(U, -1.0)
    assert e.value.status == mhd.MHD_ERR_INVALID
    with pytest.raises(mhd.MHDError) as e:
        mhd.mhd_step(ctx.ctx, U, 1e-3, ctx.ws[:1024])
    assert e.value.status == mhd.MHD_ERR_WORKSPACE
    with pytest.raises(mhd.MHDError) as e:
        mhd.mhd_rhs(ctx.ctx, U, U, ctx.ws)
    assert e.value.status == mhd.MHD_ERR_INVALID


# ------------------------------------------------------- mixed precision ---
def test_mixed_precision_parity(dev):
    """Mixed precision (FP32 reconstruction / Riemann / EMF) after 10 steps on
    the low-beta, Mach-3 turbulence: against the oracle's own mixed variant
    and against the FP64 oracle (the stated error of the mixed path). At 64^3
    the scheme (FP64 oracle included) keeps p > 0 for ~35 steps; coarser grids
    lose positivity sooner at this beta."""
    s, U0 = W.turbulence_3d_lowbeta(64)
    ctx = ctx_for(s, dev)
    c64 = O.cfg_from(s, precision="fp64")
    ref64, dts = O.run(c64, U0, 10)
    U = torch.from_numpy(U0).to(dev)
    for dt in dts:
        ctx.step(U, float(dt))
    got = U.cpu().numpy()
    refmx = O.run_dts(O.cfg_from(s), U0, dts)
    e_mx = rel_err(got, refmx)
    e_64 = rel_err(got, ref64)
    print("mixed vs oracle-mixed", e_mx, "\nmixed vs fp64", e_64, flush=True)
    # stated error of the mixed path on this workload (measured <= 2.6e-6 and
    # <= 1.1e-5 per field)
    assert (e_mx <= 2e-5).all(), e_mx
    assert (e_64 <= 1e-4).all(), e_64
    ctx.check()  # positivity kept
    div = O.divb(c64, got)
    assert np.abs(div).max() / 64 / np.abs(got[5:]).max() <= 1e-12


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("solver", ["hlld", "hll"])
def test_rhs_parity_mixed(dev, dim, solver):
    """One right-hand side in mixed precision against the oracle's mixed
    variant: FP32 rounding only (relative to the largest |L| of the field)."""
    s, U = ragged(dim, "vanleer", solver, precision="mixed")
    ctx = ctx_for(s, dev)
    got = ctx.rhs(torch.from_numpy(U).to(dev)).cpu().numpy()
    ref = O.rhs(O.cfg_from(s), U)
    err = rel_err(got, ref)
    assert (err <= 2e-5).all(), err
    ref64 = O.rhs(O.cfg_from(s, precision="fp64"), U)
    assert (rel_err(got, ref64) <= 2e-5).all()


def _gpu_divb_rel(U, s):
    """max |div b| * min(dx) / max |b| of a device state (test-side check)."""
    dx, dy, dz = W.spacing(s)
    bx, by, bz = U[5], U[6], U[7]
    div = (torch.roll(bx, -1, 2) - bx) / dx + (torch.roll(by, -1, 1) - by) / dy + \
        (torch.roll(bz, -1, 0) - bz) / dz
    return float(div.abs().max()) * min(dx, dy, dz) / float(U[5:].abs().max())


@pytest.mark.parametrize("case", ["blast_640", "lowbeta_384"])
def test_full_size_mixed_sampled_parity_and_invariants(dev, case):
    """The large mixed-precision workloads at their full size: the magnetised
    blast at 640^3 (minmod) and the low-beta Mach-3 turbulence at 384^3. The
    time step against the oracle on the whole grid; two steps against the
    oracle's mixed variant (stated FP32 bound) and its FP64 scheme at sampled
    cells; then eight more steps checked for positivity, conservation and
    div b on the whole grid (reductions on the device)."""
    if case == "blast_640":
        s, U0 = W.blast_3d(640)
        n = 640
        # the blast front (r = 0.1, 64 cells from the centre) and random cells
        cen = [(320, 320, 384), (320, 384, 320), (256, 320, 320), (365, 365, 320),
               (320, 275, 275), (0, 0, 0), (639, 639, 639)]
    else:
        s, U0 = W.turbulence_3d_lowbeta(384)
        n = 384
        cen = [(0, 0, 0), (383, 383, 383), (0, 383, 191)]
    rng = np.random.default_rng(21)
    cen += [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(6)]
    assert s["precision"] == "mixed"
    print("%s: dt + 2 steps" % case, flush=True)
    ctx = ctx_for(s, dev)
    U = torch.from_numpy(U0).to(dev)
    dt0 = ctx.dt(U)
    assert dt0 == pytest.approx(O.dt(O.cfg_from(s), U0), rel=1e-14)
    ctx.step(U, dt0)
    dt1 = ctx.dt(U)
    ctx.step(U, dt1)
    idx = torch.tensor(cen, device=dev)
    got = U[:, idx[:, 0], idx[:, 1], idx[:, 2]].T.cpu().numpy()
    ref_mx = oracle_at_samples(s, U0, [dt0, dt1], cen)
    s64 = dict(s, precision="fp64")
    ref_64 = oracle_at_samples(s64, U0, [dt0, dt1], cen)
    scale = np.abs(U0).max(axis=(1, 2, 3))
    mom = np.abs(ref_64[:, 1:4]).max()
    assert mom > 0, "no sample saw motion"
    # fields at rest or absent (momentum, the blast's b_z) take their group's scale
    scale[1:4] = np.maximum(scale[1:4], mom)
    scale[5:8] = np.maximum(scale[5:8], scale[5:8].max())
    e_mx = (np.abs(got - ref_mx) / scale).max(axis=0)
    e_64 = (np.abs(got - ref_64) / scale).max(axis=0)
    print("%s mixed vs oracle-mixed" % case, e_mx, "\nvs fp64", e_64, flush=True)
    assert (e_mx <= 2e-5).all(), e_mx
    assert (e_64 <= 1e-4).all(), e_64
    print("%s invariants: 8 more steps" % case, flush=True)
    sums0 = U.sum(dim=(1, 2, 3)).cpu().numpy()
    abs0 = U.abs().sum(dim=(1, 2, 3)).cpu().numpy()
    ctx.run(U, 8)
    ctx.check()
    sums1 = U.sum(dim=(1, 2, 3)).cpu().numpy()
    # momentum starts at rest in the blast: scale by the sum of |q| after the run too
    absq = np.maximum(abs0, U.abs().sum(dim=(1, 2, 3)).cpu().numpy())
    assert (np.abs(sums1 - sums0) <= 1e-12 * absq).all(), (sums1 - sums0) / absq
    assert _gpu_divb_rel(U, s) <= 1e-12


# ------------------------------------------- the named configurations, full ---
def test_turbulence_256_ten_step_full_grid_parity(dev):
    """The benchmark's configuration (3D turbulence 256^3, FP64, van Leer,
    HLLD, SSP-RK2, C = 0.3): ten CFL steps on the GPU against ten steps of the
    oracle on the whole grid, per field within 1e-12, and the ten time steps
    within 1e-13."""
    s, U0 = W.turbulence_3d(256)
    print("256^3: ten CFL steps on the GPU and in the oracle (whole grid)", flush=True)
    ctx = ctx_for(s, dev)
    got, dts = _run_gpu(ctx, U0, 10, dev)
    ref, odts = O.run(O.cfg_from(s), U0, 10)
    np.testing.assert_allclose(dts, odts, rtol=1e-13)
    err = rel_err(got, ref)
    print("256^3 ten-step per-field error", err, flush=True)
    assert (err <= 1e-12).all(), err


def _field_errors(got, ref):
    """Per-field max-norm and L1 errors, each relative to the reference
    field's max |q| and sum |q| (momentum and field groups share a scale
    when a field is identically zero)."""
    mx, l1 = [], []
    for q in range(8):
        smax, ssum = np.abs(ref[q]).max(), np.abs(ref[q]).sum()
        if smax == 0.0 and q in GROUPS:
            smax = max(np.abs(ref[g]).max() for g in GROUPS[q])
            ssum = max(np.abs(ref[g]).sum() for g in GROUPS[q])
        d = np.abs(got[q] - ref[q])
        mx.append(float(d.max() / smax))
        l1.append(float(d.sum() / ssum))
    return np.array(mx), np.array(l1)


class _C3:
    """State shared by the chunked 50-step comparison below (each chunk
    advances ten steps, so that no single test runs for minutes)."""
    U = None      # GPU mixed-precision state (device)
    ref = None    # FP64 oracle state (host)
    ctx = None
    dts = []


@pytest.mark.parametrize("chunk", range(5))
def test_mixed_lowbeta_256_fifty_steps_vs_fp64_oracle(dev, chunk):
    """Mixed precision on the low-beta, Mach-3 turbulence at 256^3: fifty
    steps on the GPU, and the FP64 oracle over the same fifty time steps on
    the whole grid; the per-field error of the mixed path after 50 steps
    (max-norm and L1, relative) is bounded at the end. Ten steps per chunk."""
    s, U0 = W.turbulence_3d_lowbeta(256)
    if chunk == 0:
        _C3.ctx = ctx_for(s, dev)
        _C3.U = torch.from_numpy(U0).to(dev)
        _C3.ref = U0.copy()
        _C3.dts = []
    assert _C3.U is not None, "the chunks run in order"
    c64 = O.cfg_from(s, precision="fp64")
    dts = []
    for _ in range(10):
        dt = _C3.ctx.dt(_C3.U)
        dts.append(dt)
        _C3.ctx.step(_C3.U, dt)
    torch.cuda.synchronize()
    _C3.dts += dts
    _C3.ref = O.run_dts(c64, _C3.ref, dts)
    got = _C3.U.cpu().numpy()
    mx, l1 = _field_errors(got, _C3.ref)
    print("C3 256^3 after %d steps: max-rel" % len(_C3.dts), mx, "L1-rel", l1, flush=True)
    _C3.ctx.check()  # positivity kept
    if chunk == 4:
        assert len(_C3.dts) == 50
        # stated error of the mixed path after 50 steps: measured at most 6.6e-6
        # (max-norm, rho) and 4.4e-7 (L1, m_y) per field
        assert (mx <= 2e-5).all(), mx
        assert (l1 <= 2e-6).all(), l1
        _C3.U = _C3.ref = _C3.ctx = None


def test_mixed_lowbeta_384_fifty_steps_vs_gpu_fp64(dev):
    """The same comparison at 384^3, where the reference is the GPU FP64 path
    (parity-checked against the oracle above), over the same fifty steps."""
    s, U0 = W.turbulence_3d_lowbeta(384)
    print("C3 384^3: fifty mixed and fifty FP64 steps on the GPU", flush=True)
    ctx = ctx_for(s, dev)
    U = torch.from_numpy(U0).to(dev)
    dts = []
    for _ in range(50):
        dt = ctx.dt(U)
        dts.append(dt)
        ctx.step(U, dt)
    ctx.check()
    got = U.cpu().numpy()
    del U
    ctx64 = ctx_for(dict(s, precision="fp64"), dev)
    R = torch.from_numpy(U0).to(dev)
    for dt in dts:
        ctx64.step(R, dt)
    ref = R.cpu().numpy()
    del R
    mx, l1 = _field_errors(got, ref)
    print("C3 384^3 after 50 steps: max-rel", mx, "L1-rel", l1, flush=True)
    # measured at most 4.0e-6 (max-norm) and 4.3e-7 (L1) per field
    assert (mx <= 2e-5).all(), mx
    assert (l1 <= 2e-6).all(), l1


# --------------------------------------------------- UCT-HLLD edge average ---
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("lim", ["minmod", "vanleer", "wenoz"])
@pytest.mark.parametrize("solver", ["hlld", "hll"])
def test_rhs_parity_uct_hlld(dev, dim, lim, solver):
    """The right-hand side with the UCT-HLLD edge average against the oracle's,
    FP64, per field within 1e-12, on the ragged grids and on the degenerate
    star states (B_t = 0 outside a bump, identical states on the x-faces)."""
    for which in ("ragged", "degenerate"):
        if which == "ragged":
            s, U = ragged(dim, lim, solver)
        else:
            s, U = W.aligned_field_bump(dim, 24, 16, 8, limiter=lim, riemann=solver)
        s = dict(s, emf="uct_hlld")
        ctx = ctx_for(s, dev)
        got = ctx.rhs(torch.from_numpy(U).to(dev)).cpu().numpy()
        ref = O.rhs(O.cfg_from(s), U)
        err = rel_err(got, ref)
        assert (err <= 1e-12).all(), (which, err)


@pytest.mark.parametrize("case", ["ragged3_runs", "orszag_tang_3d_32", "orszag_tang_128",
                                  "wenoz_rk3_3d", "mixed"])
def test_ten_step_parity_uct_hlld(dev, case):
    """Ten CFL steps with the UCT-HLLD average against the oracle: the ragged
    3D grid (partial columns, z-runs of 16, 16 and 5), the paper's 3D
    Orszag-Tang problem, 2D Orszag-Tang, the paper's full scheme (WENO-Z +
    SSP-RK3 + HLLD + UCT-HLLD) in 3D, and mixed precision against the oracle's
    mixed variant (stated bound 2e-5)."""
    if case == "ragged3_runs":
        s, U0 = W.generic_state(3, 20, 18, 37, "vanleer", "hlld", seed=9)
    elif case == "orszag_tang_3d_32":
        s, U0 = W.orszag_tang_3d(32)
    elif case == "orszag_tang_128":
        s, U0 = W.orszag_tang_2d(128)
    elif case == "wenoz_rk3_3d":
        s, U0 = W.generic_state(3, 20, 18, 37, "wenoz", "hlld", seed=9)
        s = dict(s, integrator="rk3")
    else:
        s, U0 = W.generic_state(3, 20, 18, 37, "vanleer", "hlld", seed=9)
        s = dict(s, precision="mixed")
    s = dict(s, emf="uct_hlld")
    print("uct-hlld 10-step parity", case, flush=True)
    ctx = ctx_for(s, dev)
    got, dts = _run_gpu(ctx, U0, 10, dev)
    if case == "mixed":
        ref = O.run_dts(O.cfg_from(s), U0, dts)
        err = rel_err(got, ref)
        assert (err <= 2e-5).all(), err
    else:
        ref, odts = O.run(O.cfg_from(s), U0, 10)
        np.testing.assert_allclose(dts, odts, rtol=1e-13)
        err = rel_err(got, ref)
        assert (err <= 1e-12).all(), err
    c = O.cfg_from(s)
    div = O.divb(c, got)
    assert np.abs(div).max() * min(W.spacing(s)[:s["dim"]]) / np.abs(got[5:]).max() <= 1e-12


def test_uct_hlld_adjoint_is_unsupported(dev):
    from paper_2511_20337_amd import mhd
    s, U = W.generic_state(3, 8, 8, 8, "vanleer", "hlld", seed=2)
    ctx = ctx_for(dict(s, emf="uct_hlld"), dev, with_adjoint=True)
    Ug = torch.from_numpy(U).to(dev)
    with pytest.raises(mhd.MHDError) as e:
        ctx.adjoint_step(Ug, 1e-3, torch.ones_like(Ug))
    assert e.value.status == mhd.MHD_ERR_UNSUPPORTED


def test_orszag_tang_2d_hundred_step_parity(dev):
    """The 2D Orszag-Tang configuration as named, 128^2 with minmod, HLLD and
    C = 0.4, for its full 100 CFL steps against the oracle: the time steps to
    1e-12 and every field to 1e-12 (measured 4.7e-15)."""
    s, U0 = W.orszag_tang_2d(128)
    ctx = ctx_for(s, dev)
    got, dts = _run_gpu(ctx, U0, 100, dev)
    ref, odts = O.run(O.cfg_from(s), U0, 100)
    np.testing.assert_allclose(dts, odts, rtol=1e-12)
    err = rel_err(got, ref)
    print("orszag_tang_2d 128^2 after 100 steps", err, flush=True)
    assert (err <= 1e-12).all(), err


@pytest.mark.parametrize("case", ["orszag_tang_128", "turbulence_32"])
def test_hip_graph_replay_matches_eager(dev, case):
    """Steps captured in a HIP graph (torch.cuda.CUDAGraph around mhd_step_cfl:
    every launch of the step is capturable, with no memset and no host
    synchronisation) replayed three times, with the program's own eager work
    and synchronisations between the replays: each replay equals the same
    steps run eagerly from the same state, bit for bit."""
    s, U0 = W.orszag_tang_2d(128) if case == "orszag_tang_128" else W.turbulence_3d(32)
    ctx = ctx_for(s, dev)
    nstep = 5
    U = torch.from_numpy(U0).to(dev)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    # warm the kernels outside the capture (first launches load code objects)
    W0 = U.clone()
    ctx.step_cfl(W0, dt)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(nstep):
            ctx.step_cfl(U, dt)
    start = torch.from_numpy(U0).to(dev)
    ref = start.clone()
    for _ in range(nstep):
        ctx.step_cfl(ref, dt)
    torch.cuda.synchronize()
    other = torch.ones(1 << 20, dtype=torch.float64, device=dev)
    for rep in range(3):
        U.copy_(start)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(U, ref), (case, rep)
        other.mul_(1.5).add_(1.0)  # eager work between the replays
        ctx.step_cfl(W0, dt)
        torch.cuda.synchronize()
