"""Pins of the oracle's GLM divergence cleaning (nine cell-centred fields).

The (B_n, psi) face problem against the characteristic relations of its
linear system; plane-parallel runs with no normal-field jump against the
independent 1D scheme; conservation of eight fields and the exact decay of
the sum of psi; a uniform state kept; an injected div B error carried away
and damped.
"""
import numpy as np
import pytest

import oracle as O
from paper_2511_20337_amd import workloads as W
from tests import ref_mhd1d


def _hlld_face_flux(WL, WR, bx, g):
    out = np.zeros(WL.shape)
    for f in range(WL.shape[1]):
        out[:, f] = O.riemann(WL[:, f], WR[:, f], bx, gamma=g, solver="hlld")[:7]
    return out


@pytest.mark.parametrize("solver", ["hlld", "hll"])
def test_glm_face_characteristics(solver):
    """The interface values of (B_n, psi) keep the outgoing characteristic
    variables psi +- c_h B_n of each side (the linear subsystem's exact
    solution), the fluxes of B_n and psi are psi* and c_h^2 B_n*, and the
    rest of the face is the MHD problem with the normal field B_n*."""
    rng = np.random.default_rng(41)
    for _ in range(500):
        wl = np.array([rng.uniform(0.3, 2), rng.normal(), rng.normal(), rng.normal(),
                       rng.normal(), rng.normal(), rng.uniform(0.1, 2)])
        wr = np.array([rng.uniform(0.3, 2), rng.normal(), rng.normal(), rng.normal(),
                       rng.normal(), rng.normal(), rng.uniform(0.1, 2)])
        bnl, bnr, psil, psir = rng.normal(size=4)
        ch = rng.uniform(0.5, 5.0)
        F = O.glm_face(wl, wr, bnl, bnr, psil, psir, ch, solver=solver)
        psi_s, bn_s = F[7], F[8] / ch ** 2
        assert psi_s + ch * bn_s == pytest.approx(psil + ch * bnl, rel=1e-13, abs=1e-13)
        assert psi_s - ch * bn_s == pytest.approx(psir - ch * bnr, rel=1e-13, abs=1e-13)
        mhd = O.riemann(wl, wr, bn_s, solver=solver)[:7]
        np.testing.assert_allclose(F[:7], mhd, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("dim,axis,solver", [(2, 0, "hll"), (2, 1, "hlld"), (3, 2, "hll"),
                                             (3, 0, "hlld")])
def test_glm_plane_parallel_equals_1d(dim, axis, solver):
    """With a uniform normal field and psi = 0 the cleaning field stays zero
    and the GLM scheme reduces to the 1D scheme with the same face solver."""
    n = 64
    nn = [4, 4, 1 if dim == 2 else 4]
    nn[axis] = n
    s = W.make_setup("plane", dim, nn[0], nn[1], nn[2], (0, 1, 0, 1, 0, 1), 5 / 3, 0.4,
                     "vanleer", solver)
    s["divb"] = "glm"
    xs = (np.arange(n) + 0.5) / n
    g = 5 / 3
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * xs)
    un = 0.2 * np.cos(2 * np.pi * xs)
    v1, v2 = 0.3 * np.sin(4 * np.pi * xs), -0.1 + 0.2 * np.cos(2 * np.pi * xs)
    b1, b2 = 0.5 * np.cos(2 * np.pi * xs), 0.4 * np.sin(2 * np.pi * xs + 1)
    p = 0.8 + 0.1 * np.where(xs > 0.5, 1.0, 0.0)
    bn = 0.7
    comps = {axis: un, (axis + 1) % 3: v1, (axis + 2) % 3: v2}
    bcomp = {axis: np.full(n, bn), (axis + 1) % 3: b1, (axis + 2) % 3: b2}
    shp = [1, 1, 1]
    shp[2 - axis] = n

    def f(a):
        return np.broadcast_to(np.reshape(a, shp), (nn[2], nn[1], nn[0]))
    E = p / (g - 1) + 0.5 * rho * (un ** 2 + v1 ** 2 + v2 ** 2) + 0.5 * (bn ** 2 + b1 ** 2 + b2 ** 2)
    U = np.zeros((9, nn[2], nn[1], nn[0]))
    U[0] = f(rho)
    for d in range(3):
        U[1 + d] = f(rho * comps[d])
        U[5 + d] = f(bcomp[d])
    U[4] = f(E)
    c = O.cfg_from(s)
    U1d = np.stack([rho, rho * un, rho * v1, rho * v2, b1, b2, E])
    dt = 0.4 / n / 3.0
    U = O.glm_run_dts(c, U, [dt] * 10)
    flux = _hlld_face_flux if solver == "hlld" else None
    for _ in range(10):
        U1d = ref_mhd1d.step(U1d, bn, 1.0 / n, dt, g, "vanleer", flux)
    line = [slice(0, 1)] * 3
    line[2 - axis] = slice(None)

    def get(q):
        return U[(q,) + tuple(line)].ravel()
    t1, t2 = (axis + 1) % 3, (axis + 2) % 3
    mapping = [(0, 0), (1 + axis, 1), (1 + t1, 2), (1 + t2, 3), (5 + t1, 4), (5 + t2, 5), (4, 6)]
    for q3, q1 in mapping:
        np.testing.assert_allclose(get(q3), U1d[q1], rtol=1e-12, atol=1e-13)
    assert np.all(U[5 + axis] == bn)
    assert np.all(U[8] == 0.0)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("integrator", ["rk2", "rk3"])
def test_glm_conservation_and_psi_decay(dim, integrator):
    """Eight fields are conserved to round-off; the sum of psi, conserved by
    the flux divergence, falls by exactly exp(-alpha C) per step (with
    c_h = C Delta_min / dt the damping factor exp(-alpha c_h dt / Delta_min)
    does not depend on dt)."""
    s, U8 = W.generic_state(dim, 16 if dim == 2 else 10, 12 if dim == 2 else 9, 8, "vanleer",
                            "hlld", seed=5)
    s, U = W.glm_from_ct(dict(s, integrator=integrator), U8)
    rng = np.random.default_rng(3)
    U[8] = 0.05 * rng.normal(size=U[8].shape)
    U[5] += 0.02 * rng.normal(size=U[5].shape)  # a divergence to clean
    c = O.cfg_from(s)
    sums0 = U.reshape(9, -1).sum(axis=1)
    abs0 = np.abs(U).reshape(9, -1).sum(axis=1)
    Un, dts = O.glm_run(c, U, 6)
    sums1 = Un.reshape(9, -1).sum(axis=1)
    for q in range(8):
        assert abs(sums1[q] - sums0[q]) <= 1e-12 * abs0[q], q
    decay = np.exp(-O.GLM_ALPHA * s["cfl"]) ** 6
    assert sums1[8] == pytest.approx(sums0[8] * decay, rel=1e-11, abs=1e-13 * abs0[8])


def test_glm_uniform_state_preserved():
    s, U8 = W.generic_state(3, 8, 8, 8, "vanleer", "hlld", seed=1)
    s, U = W.glm_from_ct(s, U8)
    for q, v in enumerate((1.3, 0.2, -0.1, 0.3, 5.0, 0.4, -0.7, 0.2, 0.0)):
        U[q] = v
    Un, _ = O.glm_run(O.cfg_from(s), U, 3)
    np.testing.assert_allclose(Un, U, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_glm_cleans_an_injected_divergence(dim):
    """A div B error injected at rest is carried away at c_h and damped: the
    L2 norm of the central-difference div B falls after every ten steps and
    ends below 0.35 of its initial value after 60 steps (2D, 64^2; measured
    0.28) / 40 steps (3D, 32^3; measured 0.25); psi takes the error up."""
    s, U = W.glm_divergence_bump(dim, 64 if dim == 2 else 32)
    c = O.cfg_from(s)
    d = [np.sqrt((O.divb_centred(c, U) ** 2).mean())]
    for _ in range(6 if dim == 2 else 4):
        U, _ = O.glm_run(c, U, 10)
        d.append(np.sqrt((O.divb_centred(c, U) ** 2).mean()))
    assert all(b < a for a, b in zip(d, d[1:])), d
    assert d[-1] < 0.35 * d[0], d
    assert np.abs(U[8]).max() > 0.0
