"""Seeded synthetic initial conditions.

This module is the only code shared by the GPU library's callers and the
oracle's: it turns an analytic initial condition into the stored state and
holds none of the time-stepping arithmetic (no reconstruction, Riemann solve,
EMF, update or time step).

State layout: float64 array ``(8, nz, ny, nx)`` = (rho, m_x, m_y, m_z, E,
b_x, b_y, b_z), x fastest. b_d is the face-normal magnetic field on the lower
d-face of each cell; in 2D (nz == 1) field 7 is the cell-centred B_z.
Staggered fields are built as the discrete curl of an edge-centred vector
potential, so the discrete divergence vanishes to round-off, plus a uniform
field set as constant face values. The total energy follows the ideal EOS of
the paper's Eq. (Energy), with the cell-centred field taken as the mean of the
two faces of the cell.

Each generator returns ``(setup, U)``; ``setup`` is a plain dict naming the
grid, box, adiabatic index, Courant number, limiter, Riemann solver and
precision, from which each side builds its own configuration structure.
"""
from __future__ import annotations

import math

import numpy as np

FIELDS = ("rho", "mx", "my", "mz", "E", "bx", "by", "bz")


def make_setup(name, dim, nx, ny, nz, box, gamma, cfl, limiter, riemann="hlld",
               precision="fp64", emf="uct_hll"):
    return {"name": name, "dim": int(dim), "nx": int(nx), "ny": int(ny), "nz": int(nz),
            "box": tuple(float(b) for b in box), "gamma": float(gamma), "cfl": float(cfl),
            "limiter": limiter, "riemann": riemann, "precision": precision, "emf": emf}


def spacing(setup):
    b = setup["box"]
    return ((b[1] - b[0]) / setup["nx"], (b[3] - b[2]) / setup["ny"],
            (b[5] - b[4]) / setup["nz"])


def centres(setup):
    """Cell-centre coordinates as broadcastable arrays (z, y, x order)."""
    b = setup["box"]
    dx, dy, dz = spacing(setup)
    x = b[0] + (np.arange(setup["nx"]) + 0.5) * dx
    y = b[2] + (np.arange(setup["ny"]) + 0.5) * dy
    z = b[4] + (np.arange(setup["nz"]) + 0.5) * dz
    return x[None, None, :], y[None, :, None], z[:, None, None]


def faces(setup, axis):
    """Coordinates of the lower faces along ``axis`` (0 = x, 1 = y, 2 = z);
    the other two coordinates are cell centres."""
    x, y, z = centres(setup)
    dx, dy, dz = spacing(setup)
    if axis == 0:
        x = x - 0.5 * dx
    elif axis == 1:
        y = y - 0.5 * dy
    else:
        z = z - 0.5 * dz
    return x, y, z


def assemble(setup, rho, vx, vy, vz, p, bx, by, bz):
    """Stored state from cell-centre primitives and the staggered field."""
    shape = (setup["nz"], setup["ny"], setup["nx"])
    g = setup["gamma"]
    rho, vx, vy, vz, p, bx, by, bz = [np.asarray(a, dtype=np.float64) for a in
                                      (rho, vx, vy, vz, p, bx, by, bz)]

    def face_mean(b, axis):
        # a constant field is its own face average (and rolling a broadcast
        # view of a scalar is needlessly slow on large grids)
        return b if b.ndim == 0 else 0.5 * (b + np.roll(b, -1, axis=axis))
    bcx = face_mean(bx, 2)
    bcy = face_mean(by, 1)
    bcz = face_mean(bz, 0) if setup["dim"] == 3 else bz
    U = np.empty((8,) + shape)
    U[0] = rho
    U[1] = rho * vx
    U[2] = rho * vy
    U[3] = rho * vz
    U[4] = p / (g - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz) + \
        0.5 * (bcx * bcx + bcy * bcy + bcz * bcz)
    U[5] = bx
    U[6] = by
    U[7] = bz
    return np.ascontiguousarray(U)


def curl_of_edge_potential(setup, Ax, Ay, Az):
    """Staggered field b = curl A from a potential sampled at edge centres:
    A_x at (i, j-1/2, k-1/2), A_y at (i-1/2, j, k-1/2), A_z at (i-1/2, j-1/2, k)
    (each stored at index (k, j, i)). In 2D only A_z is used."""
    dx, dy, dz = spacing(setup)
    nxt = lambda a, ax: np.roll(a, -1, axis=ax)  # noqa: E731  value at index + 1
    if setup["dim"] == 2:
        bx = (nxt(Az, 1) - Az) / dy
        by = -(nxt(Az, 2) - Az) / dx
        return bx, by
    bx = (nxt(Az, 1) - Az) / dy - (nxt(Ay, 0) - Ay) / dz
    by = (nxt(Ax, 0) - Ax) / dz - (nxt(Az, 2) - Az) / dx
    bz = (nxt(Ay, 2) - Ay) / dx - (nxt(Ax, 1) - Ax) / dy
    return bx, by, bz


# ---------------------------------------------------------------------------
# Band-limited random fields on the unit cube (periodic), sampled at any grid
# offset; the same seed gives the same continuous field at every resolution.

def band_modes(seed, kmin=1.0, kmax=4.0, solenoidal=True):
    """Complex Gaussian vector coefficients on integer wave vectors with
    kmin <= |k| <= kmax (units of 2 pi / L), projected solenoidal."""
    kk = int(math.floor(kmax))
    r = np.arange(-kk, kk + 1)
    K = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)  # (kx, ky, kz)
    kn = np.sqrt((K * K).sum(1))
    K = K[(kn >= kmin) & (kn <= kmax)]
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((len(K), 3)) + 1j * rng.standard_normal((len(K), 3))
    if solenoidal:
        k2 = (K * K).sum(1)[:, None]
        C = C - K * ((K * C).sum(1)[:, None] / k2)
    return K.astype(np.float64), C


def band_sample(K, C, n, offset, comp):
    """Re sum_k C_k exp(2 pi i k.x) at x = (index + offset) / n on an n^3 grid.
    offset = (ox, oy, oz) in cells; returns array (n, n, n) in (z, y, x) order.
    Evaluated as a separable contraction over the (small) band of modes."""
    kk = int(np.abs(K).max())
    m = 2 * kk + 1
    dense = np.zeros((m, m, m), dtype=np.complex128)  # [kz, ky, kx]
    Ki = K.astype(np.int64) + kk
    np.add.at(dense, (Ki[:, 2], Ki[:, 1], Ki[:, 0]), C[:, comp])
    ks = np.arange(-kk, kk + 1)[:, None]
    idx = np.arange(n)[None, :]
    ex = np.exp(2j * np.pi * ks * (idx + offset[0]) / n)  # [kx, x]
    ey = np.exp(2j * np.pi * ks * (idx + offset[1]) / n)  # [ky, y]
    ez = np.exp(2j * np.pi * ks * (idx + offset[2]) / n)  # [kz, z]
    t1 = np.einsum("abc,cx->abx", dense, ex)               # [kz, ky, x]
    t2 = np.einsum("abx,by->ayx", t1, ey).reshape(m, n * n)  # [kz, y*x]
    out = ez.real.T @ t2.real - ez.imag.T @ t2.imag        # real part, [z, y*x]
    return out.reshape(n, n, n)


# ---------------------------------------------------------------------------
# Workloads

def orszag_tang_2d(n=128, noise=1e-4, seed=1, limiter="minmod", riemann="hlld",
                   cfl=0.4, precision="fp64"):
    """2D Orszag-Tang vortex on [0,1]^2, gamma = 5/3, rho = 25/(36 pi),
    p = 5/(12 pi), v = (-sin 2 pi y, sin 2 pi x) plus seeded uniform noise of
    amplitude ``noise`` on v_x, v_y, B = (-sin 2 pi y, sin 4 pi x)/sqrt(4 pi)
    from A_z = [cos(2 pi y)/(2 pi) + cos(4 pi x)/(4 pi)]/sqrt(4 pi)."""
    s = make_setup("orszag_tang_2d", 2, n, n, 1, (0, 1, 0, 1, 0, 1), 5.0 / 3.0, cfl,
                   limiter, riemann, precision)
    x, y, _ = centres(s)
    shape = (1, n, n)
    rho = np.full(shape, 25.0 / (36.0 * np.pi))
    p = np.full(shape, 5.0 / (12.0 * np.pi))
    vx = np.broadcast_to(-np.sin(2 * np.pi * y), shape).copy()
    vy = np.broadcast_to(np.sin(2 * np.pi * x), shape).copy()
    if noise:
        rng = np.random.default_rng(seed)
        vx += rng.uniform(-noise, noise, shape)
        vy += rng.uniform(-noise, noise, shape)
    dx, dy, _ = spacing(s)
    xe = x - 0.5 * dx
    ye = y - 0.5 * dy
    Az = np.broadcast_to((np.cos(2 * np.pi * ye) / (2 * np.pi) +
                          np.cos(4 * np.pi * xe) / (4 * np.pi)) / np.sqrt(4 * np.pi), shape)
    bx, by = curl_of_edge_potential(s, None, None, Az)
    return s, assemble(s, rho, vx, vy, 0.0, p, bx, by, 0.0)


def orszag_tang_3d(n=352, limiter="vanleer", riemann="hlld", cfl=0.3, precision="fp64"):
    """3D Orszag-Tang vortex, the paper's first benchmark problem (Sec. 4.1):
    [0,1]^3 periodic, gamma = 5/3, rho = 25/9, p = 5/3,
    v = (-zeta sin 2 pi y, zeta sin 2 pi x, 0.2 sin 2 pi z) with
    zeta = 1 + sin(2 pi z)/5, B = (-sin 2 pi y, sin 4 pi x, 0) from
    A_z = cos(2 pi y)/(2 pi) + cos(4 pi x)/(4 pi). (The paper runs it with
    WENO-Z and RK3; here it runs with this path's scheme.)"""
    s = make_setup("orszag_tang_3d", 3, n, n, n, (0, 1, 0, 1, 0, 1), 5.0 / 3.0, cfl, limiter,
                   riemann, precision)
    x, y, z = centres(s)
    shape = (n, n, n)
    zeta = 1.0 + np.sin(2 * np.pi * z) / 5.0
    vx = np.broadcast_to(-zeta * np.sin(2 * np.pi * y), shape)
    vy = np.broadcast_to(zeta * np.sin(2 * np.pi * x), shape)
    vz = np.broadcast_to(0.2 * np.sin(2 * np.pi * z), shape)
    dx, dy, _ = spacing(s)
    xe = x - 0.5 * dx
    ye = y - 0.5 * dy
    Az = np.broadcast_to(np.cos(2 * np.pi * ye) / (2 * np.pi) + np.cos(4 * np.pi * xe) / (4 * np.pi),
                         shape)
    zero = np.zeros(shape)
    bx, by, bz = curl_of_edge_potential(s, zero, zero, Az)
    return s, assemble(s, 25.0 / 9.0, vx, vy, vz, 5.0 / 3.0, bx, by, bz)


def turbulence_3d(n=256, mach=1.0, beta=None, B0=0.1, dB_rel=None, dB_rms=0.1,
                  seed_v=2, seed_a=3, limiter="vanleer", riemann="hlld", cfl=0.3,
                  precision="fp64"):
    """3D decaying turbulence on [0,1]^3: rho = 1, p = 1, gamma = 5/3; random-
    phase solenoidal velocity band-limited to 1 <= |k| <= 4 scaled to rms
    Mach ``mach``; uniform B0 along x plus the curl of a band-limited random
    vector potential scaled to rms ``dB_rms``. With ``beta`` given, B0 =
    sqrt(2 p / beta) and (with ``dB_rel``) dB_rms = dB_rel * B0."""
    s = make_setup("turbulence_3d", 3, n, n, n, (0, 1, 0, 1, 0, 1), 5.0 / 3.0, cfl,
                   limiter, riemann, precision)
    g = s["gamma"]
    rho0, p0 = 1.0, 1.0
    if beta is not None:
        B0 = math.sqrt(2.0 * p0 / beta)
    if dB_rel is not None:
        dB_rms = dB_rel * B0
    K, C = band_modes(seed_v)
    v = [band_sample(K, C, n, (0.5, 0.5, 0.5), c) for c in range(3)]
    vrms = math.sqrt(float(np.mean(v[0] ** 2 + v[1] ** 2 + v[2] ** 2)))
    scale = mach * math.sqrt(g * p0 / rho0) / vrms
    v = [a * scale for a in v]
    KA, CA = band_modes(seed_a, solenoidal=False)
    Ax = band_sample(KA, CA, n, (0.5, 0.0, 0.0), 0)
    Ay = band_sample(KA, CA, n, (0.0, 0.5, 0.0), 1)
    Az = band_sample(KA, CA, n, (0.0, 0.0, 0.5), 2)
    bx, by, bz = curl_of_edge_potential(s, Ax, Ay, Az)
    brms = math.sqrt(float(np.mean(bx ** 2 + by ** 2 + bz ** 2)))
    f = dB_rms / brms
    bx, by, bz = bx * f + B0, by * f, bz * f
    return s, assemble(s, rho0, v[0], v[1], v[2], p0, bx, by, bz)


def turbulence_3d_lowbeta(n=256, **kw):
    """The 3D turbulence at rms Mach 3 and plasma beta 0.01 (B0 = sqrt(200)
    along x, dB_rms = 0.1 B0), stressing the pressure recovery."""
    kw.setdefault("precision", "mixed")
    return turbulence_3d(n=n, mach=3.0, beta=0.01, dB_rel=0.1, **kw)


def kh_mode_basis(setup, phases):
    """Per-mode shape of the v_y perturbation: sin(2 pi m x + phi_m) times two
    Gaussian envelopes centred on the shear layers y = +-1/4."""
    x, y, _ = centres(setup)
    env = np.exp(-((y - 0.25) / 0.1) ** 2) + np.exp(-((y + 0.25) / 0.1) ** 2)
    return [np.broadcast_to(np.sin(2 * np.pi * (m + 1) * x + phases[m]) * env,
                            (1, setup["ny"], setup["nx"])) for m in range(len(phases))]


def kelvin_helmholtz_2d(n=512, amps=None, nmodes=16, seed=4, limiter="vanleer",
                        riemann="hlld", cfl=0.4, precision="fp64"):
    """2D Kelvin-Helmholtz on [0,1] x [-1/2,1/2], periodic: rho = 1, p = 2.5,
    B_x = 0.1, gamma = 5/3; a double shear layer v_x = [tanh((y+1/4)/0.05) -
    tanh((y-1/4)/0.05) - 1]/2 (locally 0.5 tanh of the distance to each layer),
    and a v_y perturbation sum_m A_m sin(2 pi m x + phi_m) env(y), m = 1..16,
    A_m = 1e-2 by default, phases seeded. Returns (setup, U, phases)."""
    s = make_setup("kelvin_helmholtz_2d", 2, n, n, 1, (0, 1, -0.5, 0.5, 0, 1), 5.0 / 3.0,
                   cfl, limiter, riemann, precision)
    if amps is None:
        amps = np.full(nmodes, 1e-2)
    amps = np.asarray(amps, dtype=np.float64)
    rng = np.random.default_rng(seed)
    phases = rng.uniform(0.0, 2 * np.pi, len(amps))
    x, y, _ = centres(s)
    shape = (1, n, n)
    vx = np.broadcast_to(0.5 * (np.tanh((y + 0.25) / 0.05) - np.tanh((y - 0.25) / 0.05) - 1.0),
                         shape)
    basis = kh_mode_basis(s, phases)
    vy = sum(a * b for a, b in zip(amps, basis))
    U = assemble(s, 1.0, vx, vy, 0.0, 2.5, 0.1, 0.0, 0.0)
    return s, U, phases


def blast_3d(n=640, seed=5, limiter="minmod", riemann="hlld", cfl=0.3, precision="mixed",
             p_in=10.0):
    """3D magnetised blast on [-1/2,1/2]^3: rho = 1 + 1e-3 U(-1,1) (seeded),
    p = p_in for cell centres with r < 0.1 else 0.1, B = (1,1,0)/sqrt(2), v = 0."""
    s = make_setup("blast_3d", 3, n, n, n, (-0.5, 0.5, -0.5, 0.5, -0.5, 0.5), 5.0 / 3.0, cfl,
                   limiter, riemann, precision)
    x, y, z = centres(s)
    rng = np.random.default_rng(seed)
    rho = 1.0 + 1e-3 * rng.uniform(-1.0, 1.0, (n, n, n))
    r2 = x * x + y * y + z * z
    p = np.where(r2 < 0.01, p_in, 0.1)
    b = 1.0 / math.sqrt(2.0)
    return s, assemble(s, rho, 0.0, 0.0, 0.0, p, b, b, 0.0)


def sod_double(n, dim=2, axis=0, limiter="vanleer", riemann="hlld", cfl=0.4, ntrans=4,
               gamma=1.4):
    """B = 0 double shock tube on a periodic box of length 2 along ``axis``:
    (rho, p) = (1, 1) for 1/2 < s < 3/2, (0.125, 0.1) elsewhere, v = 0.
    The two interfaces (s = 1/2 and 3/2) launch mirror-image Riemann problems
    that do not interact before t ~ 0.3. The transverse extent has ``ntrans``
    cells."""
    nn = [ntrans, ntrans, 1 if dim == 2 else ntrans]
    nn[axis] = n
    box = [0.0, 1.0, 0.0, 1.0, 0.0, 1.0]
    box[2 * axis + 1] = 2.0
    s = make_setup("sod_double", dim, nn[0], nn[1], nn[2], box, gamma, cfl, limiter, riemann)
    c = centres(s)[axis]
    inside = (c > 0.5) & (c < 1.5)
    rho = np.where(inside, 1.0, 0.125)
    p = np.where(inside, 1.0, 0.1)
    return s, assemble(s, rho, 0.0, 0.0, 0.0, p, 0.0, 0.0, 0.0)


def cp_alfven(n, dim=2, eps=0.1, rho0=1.0, p0=0.1, B0=1.0, limiter="vanleer",
              riemann="hlld", cfl=0.4, gamma=5.0 / 3.0, kdir=None):
    """Circularly polarised Alfven wave on the unit square/cube, wave vector
    k = 2 pi (1,1) in 2D or 2 pi (1,1,1) in 3D: B = B0 e1 + eps (sin phi e2 +
    cos phi e3), v = -(eps / sqrt(rho0)) (sin phi e2 + cos phi e3) with
    phi = k.x, e1 = k/|k| and (e1, e2, e3) orthonormal. In 3D ``kdir``
    (integer vector) overrides the wave vector direction. It is an exact
    nonlinear solution travelling at the Alfven speed B0/sqrt(rho0) along e1
    (for any eps); one period is |k|^-1 2 pi sqrt(rho0)/B0. Returns
    (setup, U, period)."""
    if dim == 2:
        s = make_setup("cp_alfven_2d", 2, n, n, 1, (0, 1, 0, 1, 0, 1), gamma, cfl, limiter,
                       riemann)
        kv = np.array([1.0, 1.0, 0.0])
        e2 = np.array([-1.0, 1.0, 0.0]) / math.sqrt(2.0)
    else:
        s = make_setup("cp_alfven_3d", 3, n, n, n, (0, 1, 0, 1, 0, 1), gamma, cfl, limiter,
                       riemann)
        kv = np.array([1.0, 1.0, 1.0] if kdir is None else kdir, dtype=np.float64)
        t = np.array([0.0, 0.0, 1.0]) if abs(kv[2]) < 0.5 * np.linalg.norm(kv) else \
            np.array([1.0, 0.0, 0.0])
        e2 = np.cross(kv, t)
        e2 = e2 / np.linalg.norm(e2)
        if kdir is None:
            e2 = np.array([-1.0, 1.0, 0.0]) / math.sqrt(2.0)
    e1 = kv / np.linalg.norm(kv)
    e3 = np.cross(e1, e2)
    kvec = 2 * np.pi * kv
    x, y, z = centres(s)
    shape = (s["nz"], s["ny"], s["nx"])

    def phase(px, py, pz):
        return kvec[0] * px + kvec[1] * py + (kvec[2] * pz if dim == 3 else 0.0)

    ph = phase(x, y, z)
    va = -eps / math.sqrt(rho0)
    v = [np.broadcast_to(va * (np.sin(ph) * e2[c] + np.cos(ph) * e3[c]), shape) for c in range(3)]
    # B = B0 e1 + curl A with A = (eps/|k|) (sin phi e2 + cos phi e3): curl of
    # that A is eps (sin phi e2 + cos phi e3) for this right-handed triad.
    kn = float(np.linalg.norm(kvec))
    dx, dy, dz = spacing(s)

    def A(c, px, py, pz):
        pp = phase(px, py, pz)
        return np.broadcast_to((eps / kn) * (np.sin(pp) * e2[c] + np.cos(pp) * e3[c]), shape)

    if dim == 2:
        Az = A(2, x - 0.5 * dx, y - 0.5 * dy, z)
        bx, by = curl_of_edge_potential(s, None, None, Az)
        bx = bx + B0 * e1[0]
        by = by + B0 * e1[1]
        bz = np.broadcast_to(B0 * e1[2] + eps * (np.sin(ph) * e2[2] + np.cos(ph) * e3[2]), shape)
    else:
        Ax = A(0, x, y - 0.5 * dy, z - 0.5 * dz)
        Ay = A(1, x - 0.5 * dx, y, z - 0.5 * dz)
        Az = A(2, x - 0.5 * dx, y - 0.5 * dy, z)
        bx, by, bz = curl_of_edge_potential(s, Ax, Ay, Az)
        bx = bx + B0 * e1[0]
        by = by + B0 * e1[1]
        bz = bz + B0 * e1[2]
    U = assemble(s, rho0, v[0], v[1], v[2], p0, bx, by, bz)
    period = 2 * np.pi / kn * math.sqrt(rho0) / B0
    return s, U, period


def uniform(dim=3, n=8, rho=1.3, v=(0.3, -0.2, 0.1), p=0.7, B=(0.4, -0.25, 0.6),
            limiter="vanleer", riemann="hlld", cfl=0.4, gamma=5.0 / 3.0):
    """Uniform state (every field constant)."""
    s = make_setup("uniform", dim, n, n, n if dim == 3 else 1, (0, 1, 0, 1, 0, 1), gamma, cfl,
                   limiter, riemann)
    return s, assemble(s, rho, v[0], v[1], v[2], p, B[0], B[1], B[2])


def smooth_random(dim=3, n=16, seed=7, amp=0.05, limiter="vanleer", riemann="hlld",
                  cfl=0.3, gamma=5.0 / 3.0, Bmean=(0.3, 0.2, -0.1)):
    """Smooth, low-amplitude random perturbation of a uniform magnetised state
    (band |k| <= 2 on the unit box), for adjoint and Jacobian tests."""
    shape = (n, n, n) if dim == 3 else (1, n, n)
    s = make_setup("smooth_random", dim, n, n, n if dim == 3 else 1, (0, 1, 0, 1, 0, 1), gamma,
                   cfl, limiter, riemann)
    rng = np.random.default_rng(seed)
    x, y, z = centres(s)
    fields = []
    for _ in range(5):
        f = np.zeros(shape)
        for _m in range(3):
            k = rng.integers(-2, 3, 3)
            if not k.any():
                k[0] = 1
            ph = rng.uniform(0, 2 * np.pi)
            arg = 2 * np.pi * (k[0] * x + k[1] * y + (k[2] * z if dim == 3 else 0.0)) + ph
            f = f + np.sin(arg) * rng.uniform(0.5, 1.0)
        fields.append(f)
    rho = 1.0 + amp * fields[0]
    p = 0.8 + amp * fields[1]
    vx, vy, vz = 0.4 + amp * fields[2], -0.3 + amp * fields[3], (0.2 + amp * fields[4])
    dx, dy, dz = spacing(s)
    kA = [rng.integers(1, 3, 3) for _ in range(3)]
    phA = rng.uniform(0, 2 * np.pi, 3)

    def Aof(c, px, py, pz):
        k = kA[c]
        arg = 2 * np.pi * (k[0] * px + k[1] * py + (k[2] * pz if dim == 3 else 0.0)) + phA[c]
        return np.broadcast_to(amp * np.sin(arg) / (2 * np.pi), shape)

    if dim == 2:
        bx, by = curl_of_edge_potential(s, None, None, Aof(2, x - 0.5 * dx, y - 0.5 * dy, z))
        bz = Bmean[2] + amp * fields[0]
    else:
        bx, by, bz = curl_of_edge_potential(
            s, Aof(0, x, y - 0.5 * dy, z - 0.5 * dz), Aof(1, x - 0.5 * dx, y, z - 0.5 * dz),
            Aof(2, x - 0.5 * dx, y - 0.5 * dy, z))
        bz = bz + Bmean[2]
    return s, assemble(s, rho, vx, vy, vz, p, bx + Bmean[0], by + Bmean[1], bz)


def generic_state(dim, nx, ny, nz, limiter="vanleer", riemann="hlld", seed=1, cfl=0.3,
                  gamma=5.0 / 3.0):
    """Magnetised state on any (ragged) grid with no symmetry: each field is a
    sum of two oblique modes plus seeded cell noise, and the staggered field
    is the discrete curl of such a potential. No two faces or cells hold
    bit-identical values, so the step has no tie in a limiter or min/max at
    this state (such ties are kinks, where directional derivatives are not
    linear)."""
    s = make_setup("generic", dim, nx, ny, nz if dim == 3 else 1, (0, 1, 0, 1, 0, 1), gamma,
                   cfl, limiter, riemann)
    x, y, z = centres(s)
    sh = (s["nz"], ny, nx)
    rng = np.random.default_rng(seed)
    tp = 2 * np.pi

    def f():
        out = np.zeros(sh)
        for _ in range(2):
            a, b, c = rng.integers(1, 3, 3) * rng.choice([-1, 1], 3)
            out = out + np.sin(tp * (a * x + b * y + (c * z if dim == 3 else 0)) +
                               rng.uniform(0, tp))
        return out + 0.2 * rng.uniform(-1, 1, sh)
    rho = 1.0 + 0.05 * f()
    p = 0.6 + 0.05 * f()
    vx, vy, vz = 0.3 + 0.1 * f(), -0.2 + 0.1 * f(), 0.1 + 0.1 * f()

    def A():
        return 0.03 * f() / tp
    if dim == 2:
        bx, by = curl_of_edge_potential(s, None, None, A())
        bz = 0.2 + 0.05 * f()
    else:
        bx, by, bz = curl_of_edge_potential(s, A(), A(), A())
        bz = bz - 0.15
    return s, assemble(s, rho, vx, vy, vz, p, bx + 0.4, by + 0.25, bz)


WORKLOADS = {
    "orszag_tang_2d": orszag_tang_2d,
    "turbulence_3d": turbulence_3d,
    "turbulence_3d_lowbeta": turbulence_3d_lowbeta,
    "kelvin_helmholtz_2d": kelvin_helmholtz_2d,
    "blast_3d": blast_3d,
}


def aligned_field_bump(dim=3, nx=24, ny=8, nz=8, axes=(0, 1, 2), limiter="vanleer",
                       riemann="hlld", cfl=0.3, B0=1.0, p0=0.1):
    """Uniform plasma in a uniform field B = (B0, 0, 0) whose Alfven speed
    exceeds the sound speed (rho = 1, p = p0), with v = (0.3, -0.2, 0.1), and a
    smooth compact bump in rho, p and every velocity component around the box
    centre that varies only along `axes`. Outside the bump the state is
    exactly uniform, so the x-faces there see identical states with B_t = 0,
    where the HLLD star state is degenerate (rho (S-u)(S-S_M) = B_n^2). Inside
    it every primitive varies, so no velocity is uniform only up to the
    rounding of m / rho (which would put limiters at ties that rounding
    decides)."""
    nz = nz if dim == 3 else 1
    s = make_setup("aligned_field_bump", dim, nx, ny, nz, (0, 1, 0, 1, 0, 1), 5.0 / 3.0, cfl,
                   limiter, riemann)
    x, y, z = centres(s)
    r2 = np.zeros((nz, ny, nx))
    for ax, c in ((0, x), (1, y), (2, z)):
        if ax in axes and (ax < 2 or dim == 3):
            r2 = r2 + ((c - 0.5) / 0.22) ** 2
    bump = np.where(r2 < 1.0, np.cos(0.5 * np.pi * np.sqrt(np.minimum(r2, 1.0))) ** 2, 0.0)
    rho = 1.0 + 0.3 * bump
    p = p0 * (1.0 + 0.5 * bump)
    vx = 0.3 + 0.1 * bump
    vy = -0.2 + 0.2 * bump
    vz = 0.1 + 0.05 * bump
    return s, assemble(s, rho, vx, vy, vz, p, B0, 0.0, 0.0)


# ---------------------------------------------------------------------------
# GLM divergence cleaning: nine cell-centred fields (rho, m, E, B, psi)

def glm_from_ct(setup, U):
    """The GLM form of a stored state: the cell-centred field (the mean of
    the two faces; in 2D b_x, b_y averaged and B_z as stored), the same
    total energy (which already uses that cell-centred field) and psi = 0.
    Returns (setup with divb = 'glm', U9)."""
    s = dict(setup, divb="glm")
    U9 = np.zeros((9,) + U.shape[1:])
    U9[:5] = U[:5]
    U9[5] = 0.5 * (U[5] + np.roll(U[5], -1, axis=2))
    U9[6] = 0.5 * (U[6] + np.roll(U[6], -1, axis=1))
    U9[7] = 0.5 * (U[7] + np.roll(U[7], -1, axis=0)) if setup["dim"] == 3 else U[7]
    return s, np.ascontiguousarray(U9)


def glm_divergence_bump(dim=2, n=64, amp=0.1, width=0.08, riemann="hlld", limiter="vanleer",
                        cfl=0.3):
    """Uniform plasma at rest (rho = 1, p = 1) in a field B = (B0 + amp g(r), 0, 0)
    with B0 = 0.5 and g a Gaussian of the given width about the box centre:
    div B = amp dg/dx is not zero, and psi = 0. The cleaning carries the
    error away at c_h and damps it."""
    nz = n if dim == 3 else 1
    s = make_setup("glm_divergence_bump", dim, n, n, nz, (0, 1, 0, 1, 0, 1), 5.0 / 3.0, cfl,
                   limiter, riemann)
    s["divb"] = "glm"
    x, y, z = centres(s)
    r2 = (x - 0.5) ** 2 + (y - 0.5) ** 2 + ((z - 0.5) ** 2 if dim == 3 else 0.0)
    shape = (nz, n, n)
    bx = np.broadcast_to(0.5 + amp * np.exp(-r2 / width ** 2), shape)
    U9 = np.zeros((9,) + shape)
    U9[0] = 1.0
    U9[4] = 1.0 / (s["gamma"] - 1.0) + 0.5 * bx * bx
    U9[5] = bx
    return s, np.ascontiguousarray(U9)
