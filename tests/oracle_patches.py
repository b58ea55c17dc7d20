"""Oracle values at sampled cells of a large grid.

One stage changes a cell only through cells a bounded distance away: with
PLM, faces need two cells on each side and the edge EMFs reconstruct face
values one more cell across (3 cells); with WENO-Z the face stencil spans
three cells below and two above the face, and primitive recovery reads the
upper staggered face, so a stage reaches 4 cells. After s stages the reach is
s times that. Running the oracle on the periodic (2r+1)^3 patch around a
cell, with the grid's own spacing, therefore reproduces that cell's result
exactly while the reach stays below r; the radius is derived from the
limiter, the integrator's stage count and the number of steps, and checked.
Wrapping the patch periodically puts artificial jumps on its border; on
violent workloads (low beta, Mach 3) they may drive border cells unphysical,
which is allowed: like any other border value they reach at most the same
distance inward, and the sampled centre must come out finite.
"""
import numpy as np

import oracle as O
from paper_2511_20337_amd import workloads as W


def stage_reach(limiter):
    """Cells one stage reaches: 4 with WENO-Z, 3 with PLM."""
    return 4 if limiter == "wenoz" else 3


def required_radius(setup, nsteps):
    stages = 3 if setup.get("integrator", "rk2") == "rk3" else 2
    return stage_reach(setup["limiter"]) * stages * nsteps


def oracle_at_samples(setup, U0, dts, centres, radius=None):
    """Oracle state after len(dts) steps at the cells `centres` (k, j, i).
    radius defaults to the reach plus two cells of margin; a given radius
    must exceed the reach."""
    reach = required_radius(setup, len(dts))
    if radius is None:
        radius = reach + 2
    assert radius > reach, (radius, reach)
    dx, dy, dz = W.spacing(setup)
    m = 2 * radius + 1
    sp = W.make_setup("patch", 3, m, m, m, (0, m * dx, 0, m * dy, 0, m * dz), setup["gamma"],
                      setup["cfl"], setup["limiter"], setup["riemann"], setup["precision"])
    sp = dict(sp, integrator=setup.get("integrator", "rk2"), emf=setup.get("emf", "uct_hll"))
    c = O.cfg_from(sp)
    out = []
    for (k, j, i) in centres:
        ik = np.arange(k - radius, k + radius + 1) % setup["nz"]
        ij = np.arange(j - radius, j + radius + 1) % setup["ny"]
        ii = np.arange(i - radius, i + radius + 1) % setup["nx"]
        P = np.ascontiguousarray(U0[:, ik][:, :, ij][:, :, :, ii])
        P = O.run_dts(c, P, dts, allow_unphysical=True)
        v = P[:, radius, radius, radius]
        assert np.isfinite(v).all(), (k, j, i)
        out.append(v)
    return np.array(out)
