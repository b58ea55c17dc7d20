"""Pins of the whole oracle step against what the mathematics fixes:
exact solutions (shock tube at B = 0, circularly polarised Alfven wave),
conservation and div B invariants, symmetries, a brute-force 1D reduction,
and finite differences for its forward-mode tangent.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import exact_euler as X
from paper_2511_20337_amd import workloads as W
from tests import ref_mhd1d


# ------------------------------------------------------------ exact Euler --
def test_exact_solver_jump_conditions():
    """The exact solver's shock satisfies Rankine-Hugoniot; its rarefaction
    conserves entropy and the Riemann invariant u + 2c/(g-1)."""
    g = 1.4
    rl, ul, pl, rr, ur, pr = 0.125, 0.0, 0.1, 1.0, 0.0, 1.0  # mirror Sod
    ws = X.wave_structure(rr, -ur, pr, rl, -ul, pl, g)  # standard Sod orientation
    # right shock: mass, momentum, energy fluxes continuous in the shock frame
    S = ws["right"][1]
    r1, u1, p1 = rl, 0.0, pl
    r2, u2, p2 = ws["rho_r"], ws["u"], ws["p"]
    e1 = p1 / (g - 1) + 0.5 * r1 * u1 ** 2
    e2 = p2 / (g - 1) + 0.5 * r2 * u2 ** 2
    assert r1 * (u1 - S) == pytest.approx(r2 * (u2 - S), rel=1e-12)
    assert r1 * u1 * (u1 - S) + p1 == pytest.approx(r2 * u2 * (u2 - S) + p2, rel=1e-12)
    assert e1 * (u1 - S) + p1 * u1 == pytest.approx(e2 * (u2 - S) + p2 * u2, rel=1e-12)
    # left rarefaction: isentropic, invariant u + 2c/(g-1) constant
    r3, p3 = ws["rho_l"], ws["p"]
    assert pr / rr ** g == pytest.approx(p3 / r3 ** g, rel=1e-12)
    c0, c3 = math.sqrt(g * pr / rr), math.sqrt(g * p3 / r3)
    assert 0 + 2 * c0 / (g - 1) == pytest.approx(ws["u"] + 2 * c3 / (g - 1), rel=1e-12)


def test_exact_solver_textbook_sod_star_state():
    # tests/golden/sod_star_state.txt (Toro, Riemann Solvers and Numerical
    # Methods for Fluid Dynamics, test 1): p* = 0.30313, u* = 0.92745
    vals = {}
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "sod_star_state.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    p, u = X.star_state(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4)
    assert p == pytest.approx(vals["p_star"], abs=5e-6)
    assert u == pytest.approx(vals["u_star"], abs=5e-6)


def _sod_l1(n, solver="hlld", lim="vanleer", dim=2, axis=0, t_end=0.2):
    s, U = W.sod_double(n, dim=dim, axis=axis, limiter=lim, riemann=solver)
    c = O.cfg_from(s)
    t = 0.0
    while t < t_end - 1e-14:
        dt = min(O.dt(c, U), t_end - t)
        U = O.step(c, U, dt)
        t += dt
    x = W.centres(s)[axis].ravel()
    # exact: standard Sod at s = 3/2, mirrored Sod at s = 1/2
    ex = np.where(x > 1.0,
                  X.sample(1.0, 0, 1.0, 0.125, 0, 0.1, 1.4, (x - 1.5) / t_end)[0],
                  X.sample(0.125, 0, 0.1, 1.0, 0, 1.0, 1.4, (x - 0.5) / t_end)[0])
    rho = np.moveaxis(U[0], 2 - axis, 0).reshape(len(x), -1)
    # plane-parallel: every transverse row identical
    assert np.ptp(rho, axis=1).max() <= 1e-13
    return np.abs(rho[:, 0] - ex).mean() * 2.0, U, s


@pytest.mark.parametrize("solver", ["hlld", "hll"])
def test_double_sod_converges_to_exact(solver):
    e1, _, _ = _sod_l1(128, solver)
    e2, _, _ = _sod_l1(256, solver)
    order = math.log2(e1 / e2)
    assert e2 < 1e-2  # two Sod problems, dx = 1/128
    assert 0.6 <= order <= 1.1, order


def test_double_sod_same_along_every_axis():
    _, Ux, _ = _sod_l1(64, dim=3, axis=0, t_end=0.1)
    _, Uy, _ = _sod_l1(64, dim=3, axis=1, t_end=0.1)
    _, Uz, _ = _sod_l1(64, dim=3, axis=2, t_end=0.1)
    np.testing.assert_allclose(Ux[0, 0, 0, :], Uy[0, 0, :, 0], rtol=1e-13)
    np.testing.assert_allclose(Ux[0, 0, 0, :], Uz[0, :, 0, 0], rtol=1e-13)
    np.testing.assert_allclose(Ux[1, 0, 0, :], Uy[2, 0, :, 0], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(Ux[1, 0, 0, :], Uz[3, :, 0, 0], rtol=1e-12, atol=1e-14)


# ------------------------------------------------------- CP Alfven wave ----
def _cpa_error(n, dim, eps=0.1, lim="vanleer", solver="hlld"):
    # the time step takes the min over directions, so the summed Courant
    # number is dim * C: C = 0.4 in 2D, 0.3 in 3D
    s, U0, period = W.cp_alfven(n, dim=dim, eps=eps, limiter=lim, riemann=solver,
                                cfl=0.4 if dim == 2 else 0.3)
    c = O.cfg_from(s)
    dt = O.dt(c, U0)
    nsteps = int(math.ceil(period / dt))
    U = O.run_dts(c, U0, np.full(nsteps, period / nsteps))
    # L1 error of the magnetic field components (wave returns after a period)
    return float(np.mean(np.abs(U[5:8] - U0[5:8])))


def test_cp_alfven_2d_second_order():
    e = [_cpa_error(n, 2) for n in (32, 64, 128)]
    o1, o2 = math.log2(e[0] / e[1]), math.log2(e[1] / e[2])
    assert o2 >= 1.8, (e, o1, o2)


def test_cp_alfven_3d_second_order():
    e = [_cpa_error(n, 3) for n in (12, 24)]
    assert math.log2(e[0] / e[1]) >= 1.8, e


@pytest.mark.parametrize("integrator,lo,hi", [("rk2", 1.8, 2.3), ("rk3", 2.7, 3.5)])
def test_ssp_time_order(integrator, lo, hi):
    """Temporal order of the SSP integrators (Sec. 2.2, Eq. (RK3) and its
    two-stage member) on a fixed grid: the 2D circularly polarised Alfven wave
    at 32^2 taken to a quarter period with dt, dt/2 and dt/4 against dt/32;
    the spatial error is the same in every run, so the differences are
    temporal. SSP-RK2 halves to a quarter (order 2), SSP-RK3 to an eighth
    (order 3; measured 2.8 and 3.0). Read as printed, the last RK3 stage
    would not even be consistent (its dt term would be 2/3 dt L)."""
    s, U0, period = W.cp_alfven(32, dim=2, cfl=0.4)
    c = O.cfg_from(dict(s, integrator=integrator))
    T = period / 4
    n0 = int(math.ceil(T / O.dt(c, U0)))

    def run_to_T(ns):
        return O.run_dts(c, U0, np.full(ns, T / ns))
    ref = run_to_T(32 * n0)
    e = [float(np.mean(np.abs(run_to_T(f * n0) - ref))) for f in (1, 2, 4)]
    orders = [math.log2(e[q] / e[q + 1]) for q in range(2)]
    assert all(lo <= o <= hi for o in orders), (e, orders)


def test_wenoz_rk3_scheme_on_cp_alfven():
    """The paper's benchmark scheme (WENO-Z + SSP-RK3 + HLLD + CT) on the 2D
    circularly polarised Alfven wave: after one period the error of B is at
    least halved against van Leer PLM at 32^2 (measured 0.29x) and falls at
    second order from 32^2 to 64^2 (measured 2.10: the CT edge values and the
    one-point face flux are second order)."""
    def err(n, lim):
        s, U0, period = W.cp_alfven(n, dim=2, cfl=0.4, limiter=lim)
        c = O.cfg_from(dict(s, integrator="rk3"))
        ns = int(math.ceil(period / O.dt(c, U0)))
        U = O.run_dts(c, U0, np.full(ns, period / ns))
        return float(np.mean(np.abs(U[5:8] - U0[5:8])))
    e32, e64 = err(32, "wenoz"), err(64, "wenoz")
    assert e32 <= 0.5 * err(32, "vanleer"), e32
    assert math.log2(e32 / e64) >= 1.9, (e32, e64)


def test_linear_alfven_wave_minmod_order():
    e = [_cpa_error(n, 2, eps=1e-6, lim="minmod") for n in (32, 64)]
    assert math.log2(e[0] / e[1]) >= 1.3, e


def test_linear_alfven_wave_vanleer_second_order():
    """The smooth linear wave (amplitude 1e-6) with van Leer: second order
    (measured 1.81 from 32^2 to 64^2 and 1.95 from 64^2 to 128^2)."""
    e = [_cpa_error(n, 2, eps=1e-6, lim="vanleer") for n in (32, 64, 128)]
    o1, o2 = math.log2(e[0] / e[1]), math.log2(e[1] / e[2])
    assert o1 >= 1.75 and o2 >= 1.9, (e, o1, o2)


# --------------------------------------------------------- invariants ------
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("solver", ["hlld", "hll"])
def test_conservation_and_divb(dim, solver):
    if dim == 2:
        s, U = W.orszag_tang_2d(32, riemann=solver)
    else:
        s, U = W.turbulence_3d(16, riemann=solver)
    c = O.cfg_from(s)
    U1, _ = O.run(c, U, 30)
    cells = range(5) if dim == 3 else (0, 1, 2, 3, 4, 7)
    for q in cells:
        scale = np.abs(U[q]).sum() + np.abs(U1[q]).sum()
        assert abs(U1[q].sum() - U[q].sum()) <= 1e-12 * scale
    for q in (5, 6, 7)[: dim]:
        scale = np.abs(U[q]).sum()
        assert abs(U1[q].sum() - U[q].sum()) <= 1e-12 * scale
    dx = min(W.spacing(s)[:dim])
    bmax = np.abs(U1[5:5 + dim]).max()
    assert np.abs(O.divb(c, U1)).max() * dx / bmax <= 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_state_preserved_bitwise(dim):
    s, U = W.uniform(dim=dim, n=8)
    c = O.cfg_from(s)
    for dt in (1e-3, 0.05):
        np.testing.assert_array_equal(O.step(c, U, dt), U)


def test_orszag_tang_point_symmetry():
    """Noise-free OT is symmetric under (x, y) -> (1-x, 1-y) with vectors
    flipped; the scheme keeps that symmetry (up to rounding order)."""
    s, U = W.orszag_tang_2d(64, noise=0.0)
    c = O.cfg_from(s)
    U1, _ = O.run(c, U, 100)

    def mirror(A):
        M = A[:, :, ::-1, ::-1].copy()
        for q in (5, 6):  # staggered: face index f <-> (n - f) mod n
            ax = 3 if q == 5 else 2
            M[q] = np.roll(M[q], 1, axis=ax - 1)
        M[1:4] *= -1
        M[5:8] *= -1
        return M
    np.testing.assert_allclose(mirror(U), U, atol=1e-15)
    scale = np.abs(U1).max(axis=(1, 2, 3))
    err = np.abs(mirror(U1) - U1).max(axis=(1, 2, 3))
    assert (err <= 1e-12 * scale).all(), err / scale


def test_axis_permutation_symmetry_3d():
    """Relabelling axes cyclically (x->y->z->x) commutes with the step."""
    s, U = W.turbulence_3d(12)
    c = O.cfg_from(s)
    dt = O.dt(c, U)

    def rot(A):  # new(x,y,z) components = old(z,x,y); array axes (z,y,x)
        B = np.empty_like(A)
        # new field at (i,j,k) = old at (j? ) : permute spatial axes
        perm = lambda a: np.transpose(a, (1, 0, 2))  # noqa: E731
        perm = lambda a: np.moveaxis(a, (0, 1, 2), (2, 0, 1))  # noqa: E731
        B[0] = perm(A[0])
        B[4] = perm(A[4])
        B[1], B[2], B[3] = perm(A[3]), perm(A[1]), perm(A[2])
        B[5], B[6], B[7] = perm(A[7]), perm(A[5]), perm(A[6])
        return B
    Ur = rot(U)
    np.testing.assert_allclose(O.divb(c, Ur), 0, atol=1e-12)
    A = rot(O.step(c, U, dt))
    B = O.step(c, Ur, dt)
    np.testing.assert_allclose(A, B, rtol=0, atol=1e-13 * np.abs(B).max())


def _hlld_face_flux(WL, WR, bx, g):
    """Face fluxes of the oracle's single-face HLLD solver (pinned on its own
    in test_oracle_units) for the 1D reference scheme."""
    out = np.zeros(WL.shape)
    for f in range(WL.shape[1]):
        out[:, f] = O.riemann(WL[:, f], WR[:, f], bx, gamma=g, solver="hlld")[:7]
    return out


@pytest.mark.parametrize("dim,axis,solver,emf",
                         [(2, 0, "hll", "uct_hll"), (2, 1, "hll", "uct_hll"),
                          (3, 0, "hll", "uct_hll"), (3, 2, "hll", "uct_hll"),
                          (2, 0, "hlld", "uct_hlld"), (2, 1, "hlld", "uct_hlld"),
                          (3, 1, "hlld", "uct_hlld"), (3, 2, "hlld", "uct_hlld"),
                          (3, 0, "hll", "uct_hlld")])
def test_plane_parallel_equals_1d_hll(dim, axis, solver, emf):
    """With no transverse variation the 2D/3D scheme, including the CT EMF,
    reduces to a 1D scheme with the same face solver: with HLL and either
    average, the independently written 1D HLL scheme; with HLLD and the
    UCT-HLLD average, the 1D scheme with the HLLD face flux (the edge EMFs
    equal minus the HLLD fluxes of the transverse field components)."""
    n = 64
    nn = [4, 4, 1 if dim == 2 else 4]
    nn[axis] = n
    s = W.make_setup("plane", dim, nn[0], nn[1], nn[2], (0, 1, 0, 1, 0, 1), 5 / 3, 0.4,
                     "vanleer", solver, emf=emf)
    xs = (np.arange(n) + 0.5) / n
    g = 5 / 3
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * xs)
    un = 0.2 * np.cos(2 * np.pi * xs)
    v1, v2 = 0.3 * np.sin(4 * np.pi * xs), -0.1 + 0.2 * np.cos(2 * np.pi * xs)
    b1, b2 = 0.5 * np.cos(2 * np.pi * xs), 0.4 * np.sin(2 * np.pi * xs + 1)
    p = 0.8 + 0.1 * np.where(xs > 0.5, 1.0, 0.0)
    bn = 0.7
    # place along `axis`: normal = axis, t1 = axis+1, t2 = axis+2 (cyclic)
    comps = {axis: un, (axis + 1) % 3: v1, (axis + 2) % 3: v2}
    bcomp = {axis: np.full(n, bn), (axis + 1) % 3: b1, (axis + 2) % 3: b2}
    shp = [1, 1, 1]
    shp[2 - axis] = n

    def f(a):
        return np.broadcast_to(np.reshape(a, shp), (nn[2], nn[1], nn[0]))
    U = W.assemble(s, f(rho), f(comps[0]), f(comps[1]), f(comps[2]), f(p),
                   f(bcomp[0]), f(bcomp[1]), f(bcomp[2]))
    if dim == 2 and axis != 2:
        pass
    c = O.cfg_from(s)
    E = p / (g - 1) + 0.5 * rho * (un ** 2 + v1 ** 2 + v2 ** 2) + 0.5 * (bn ** 2 + b1 ** 2 + b2 ** 2)
    U1d = np.stack([rho, rho * un, rho * v1, rho * v2, b1, b2, E])
    dt = 0.4 / n / 3.0
    flux = _hlld_face_flux if solver == "hlld" else None
    for _ in range(10):
        U = O.step(c, U, dt)
        U1d = ref_mhd1d.step(U1d, bn, 1.0 / n, dt, g, "vanleer", flux)
    line = [slice(0, 1)] * 3
    line[2 - axis] = slice(None)

    def get(q):
        return U[(q,) + tuple(line)].ravel()
    t1, t2 = (axis + 1) % 3, (axis + 2) % 3
    mapping = [(0, 0), (1 + axis, 1), (1 + t1, 2), (1 + t2, 3), (5 + t1, 4), (5 + t2, 5), (4, 6)]
    for q3, q1 in mapping:
        np.testing.assert_allclose(get(q3), U1d[q1], rtol=1e-12, atol=1e-13)


def test_plane_parallel_hlld_with_uct_hll_is_not_1d_hlld():
    """The mismatch the UCT-HLLD average removes: with HLLD fluxes but the
    HLL-coefficient upwind EMF, the transverse field of a plane-parallel run
    follows the HLL flux, not the HLLD one, so the run departs from the 1D
    HLLD scheme (by far more than round-off) while the cell fields' fluxes
    are HLLD."""
    n = 64
    s = W.make_setup("plane", 2, n, 4, 1, (0, 1, 0, 1, 0, 1), 5 / 3, 0.4, "vanleer", "hlld")
    xs = (np.arange(n) + 0.5) / n
    g = 5 / 3
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * xs)
    un = 0.2 * np.cos(2 * np.pi * xs)
    v1, v2 = 0.3 * np.sin(4 * np.pi * xs), -0.1 + 0.2 * np.cos(2 * np.pi * xs)
    b1, b2 = 0.5 * np.cos(2 * np.pi * xs), 0.4 * np.sin(2 * np.pi * xs + 1)
    p = 0.8 + 0.1 * np.where(xs > 0.5, 1.0, 0.0)
    bn = 0.7

    def f(a):
        return np.broadcast_to(a[None, None, :], (1, 4, n))
    U0 = W.assemble(s, f(rho), f(un), f(v1), f(v2), f(p), f(np.full(n, bn)), f(b1), f(b2))
    E = p / (g - 1) + 0.5 * rho * (un ** 2 + v1 ** 2 + v2 ** 2) + 0.5 * (bn ** 2 + b1 ** 2 + b2 ** 2)
    U1d = np.stack([rho, rho * un, rho * v1, rho * v2, b1, b2, E])
    dt = 0.4 / n / 3.0
    res = {}
    for emf in ("uct_hll", "uct_hlld"):
        c = O.cfg_from(dict(s, emf=emf))
        U = U0
        for _ in range(10):
            U = O.step(c, U, dt)
        res[emf] = U[6, 0, 0, :]  # b_y (t1 of the x-normal)
    R1 = U1d
    for _ in range(10):
        R1 = ref_mhd1d.step(R1, bn, 1.0 / n, dt, g, "vanleer", _hlld_face_flux)
    err_hlld = np.abs(res["uct_hlld"] - R1[4]).max()
    err_hll = np.abs(res["uct_hll"] - R1[4]).max()
    assert err_hlld <= 1e-13
    assert err_hll >= 1e-6, err_hll


# ------------------------------------------------------ tangent vs FD ------
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("lim,solver", [("vanleer", "hlld"), ("minmod", "hll")])
def test_step_jvp_matches_central_differences(dim, lim, solver):
    """The forward-mode tangent of the step against central differences, for
    a perturbation of every stored field (staggered field included), on a
    state with no ties (where the step is differentiable)."""
    s, U = W.generic_state(dim, 12 if dim == 2 else 7, 10 if dim == 2 else 6, 5, lim, solver)
    c = O.cfg_from(s)
    dt = O.dt(c, U)
    rng = np.random.default_rng(9)
    dU = rng.normal(size=U.shape) * np.abs(U).max(axis=(1, 2, 3), keepdims=True)
    h = 1e-7
    fd = (O.step(c, U + h * dU, dt) - O.step(c, U - h * dU, dt)) / (2 * h)
    Unew, jv = O.step_jvp(c, U, dU, dt)
    np.testing.assert_array_equal(Unew, O.step(c, U, dt))
    assert np.abs(jv - fd).max() <= 1e-7 * np.abs(fd).max()
    # dt direction
    _, jdt = O.step_jvp(c, U, np.zeros_like(U), dt, 1.0)
    hd = 1e-7 * dt
    fdt = (O.step(c, U, dt + hd) - O.step(c, U, dt - hd)) / (2 * hd)
    assert np.abs(jdt - fdt).max() <= 1e-7 * np.abs(fdt).max()


# ------------------------------------------------------ mixed precision ----
def test_mixed_precision_close_to_fp64():
    s, U = W.turbulence_3d(16)
    c64 = O.cfg_from(s)
    cmx = O.cfg_from(s, precision="mixed")
    U64, dts = O.run(c64, U, 5)
    Umx = O.run_dts(cmx, U, dts)
    for q in range(8):
        err = np.abs(Umx[q] - U64[q]).max() / np.abs(U64[q]).max()
        assert err < 1e-5, (q, err)
    # div B untouched: still a pure FP64 curl update
    assert np.abs(O.divb(cmx, Umx)).max() / np.abs(Umx[5:]).max() / 16 < 1e-12


@pytest.mark.parametrize("emf", ["uct_hll", "uct_hlld"])
def test_patch_sampling_reproduces_full_grid(emf):
    """The sampled-cell oracle used for full-size GPU checks equals the oracle
    on the whole grid, bit for bit, over two steps (with either edge average)."""
    from tests.oracle_patches import oracle_at_samples
    s, U0 = W.turbulence_3d(32)
    s = dict(s, emf=emf)
    c = O.cfg_from(s)
    d0 = O.dt(c, U0)
    U1 = O.step(c, U0, d0)
    d1 = O.dt(c, U1)
    U2 = O.step(c, U1, d1)
    cen = [(0, 0, 0), (31, 31, 31), (5, 17, 2), (16, 0, 30)]
    r = oracle_at_samples(s, U0, [d0, d1], cen)
    for n, (k, j, i) in enumerate(cen):
        np.testing.assert_array_equal(r[n], U2[:, k, j, i])
