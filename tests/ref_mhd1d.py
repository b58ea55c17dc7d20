"""Independent one-dimensional reference for the plane-parallel pin.

A deliberately separate, vectorised numpy implementation of the 1D ideal-MHD
scheme (constant normal field B_x; cell-centred (rho, m, B_y, B_z, E)):
piecewise-linear limited reconstruction of (rho, u, v, w, B_y, B_z, p), the
HLL flux with the wave-speed bounds S_L = min(u_L, u_R) - max(c_fL, c_fR),
S_R = max(u_L, u_R) + max(c_fL, c_fR), and two-stage SSP Runge-Kutta.

A plane-parallel problem run by the 2D/3D scheme with the HLL solver and the
upwind constrained-transport EMF must reproduce this to round-off: with no
transverse variation the edge EMFs reduce to the HLL fluxes of the transverse
field components.
"""
import numpy as np


def _slope(lim, dm, dp):
    out = np.zeros_like(dm)
    pos = dm * dp > 0
    if lim == "minmod":
        out[pos] = np.where(np.abs(dm[pos]) <= np.abs(dp[pos]), dm[pos], dp[pos])
    else:
        out[pos] = 2 * dm[pos] * dp[pos] / (dm[pos] + dp[pos])
    return out


def _flux_and_cons(W, bx, g):
    rho, u, v, w, by, bz, p = W
    B2 = bx * bx + by * by + bz * bz
    pt = p + 0.5 * B2
    E = p / (g - 1) + 0.5 * rho * (u * u + v * v + w * w) + 0.5 * B2
    Uc = np.stack([rho, rho * u, rho * v, rho * w, by, bz, E])
    F = np.stack([rho * u, rho * u * u + pt - bx * bx, rho * u * v - bx * by,
                  rho * u * w - bx * bz, u * by - v * bx, u * bz - w * bx,
                  (E + pt) * u - bx * (u * bx + v * by + w * bz)])
    return Uc, F


def _cf(W, bx, g):
    rho, _, _, _, by, bz, p = W
    gp = g * p
    B2 = bx * bx + by * by + bz * bz
    a = gp + B2
    return np.sqrt((a + np.sqrt(np.maximum(0.0, a * a - 4 * gp * bx * bx))) / (2 * rho))


def rhs(Uc, bx, dx, g, lim, flux=None):
    """Uc: (7, n) = (rho, m_x, m_y, m_z, B_y, B_z, E); periodic. flux: an
    optional face flux flux(WL, WR, bx, g) -> (7, n) in place of the HLL one
    (used to check the scheme against another single-face solver)."""
    rho = Uc[0]
    u, v, w = Uc[1] / rho, Uc[2] / rho, Uc[3] / rho
    by, bz = Uc[4], Uc[5]
    p = (g - 1) * (Uc[6] - 0.5 * (Uc[1] * u + Uc[2] * v + Uc[3] * w) -
                   0.5 * (bx * bx + by * by + bz * bz))
    W = np.stack([rho, u, v, w, by, bz, p])
    dm = W - np.roll(W, 1, axis=1)
    dp = np.roll(W, -1, axis=1) - W
    S = _slope(lim, dm, dp)
    # face f is the lower face of cell f: left state from cell f-1, right from f
    WL = np.roll(W + 0.5 * S, 1, axis=1)
    WR = W - 0.5 * S
    if flux is not None:
        Fh = flux(WL, WR, bx, g)
        return -(np.roll(Fh, -1, axis=1) - Fh) / dx
    UL, FL = _flux_and_cons(WL, bx, g)
    UR, FR = _flux_and_cons(WR, bx, g)
    cmax = np.maximum(_cf(WL, bx, g), _cf(WR, bx, g))
    SL = np.minimum(WL[1], WR[1]) - cmax
    SR = np.maximum(WL[1], WR[1]) + cmax
    Fh = (SR * FL - SL * FR + SL * SR * (UR - UL)) / (SR - SL)
    Fh = np.where(SL >= 0, FL, Fh)
    Fh = np.where(SR <= 0, FR, Fh)
    return -(np.roll(Fh, -1, axis=1) - Fh) / dx


def step(Uc, bx, dx, dt, g, lim, flux=None):
    U1 = Uc + dt * rhs(Uc, bx, dx, g, lim, flux)
    return 0.5 * (Uc + (U1 + dt * rhs(U1, bx, dx, g, lim, flux)))
