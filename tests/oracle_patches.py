"""Oracle values at sampled cells of a large grid.

One RK stage changes a cell only through cells at most 3 away (faces need two
cells on each side, the edge EMFs one more transverse face), so k stages
reach 3k cells. Running the oracle on the periodic (2r+1)^3 patch around a
cell, with the grid's own spacing, therefore reproduces that cell's result
exactly while 3k < r: r = 14 covers two RK2 steps (four stages) with margin.
Wrapping the patch periodically puts artificial jumps on its border; on
violent workloads (low beta, Mach 3) they may drive border cells unphysical,
which is allowed: like any other border value they reach at most 3k cells
inward, and the sampled centre must come out finite.
"""
import numpy as np

import oracle as O
from paper_2511_20337_amd import workloads as W


def oracle_at_samples(setup, U0, dts, centres, radius=14):
    dx, dy, dz = W.spacing(setup)
    m = 2 * radius + 1
    sp = W.make_setup("patch", 3, m, m, m, (0, m * dx, 0, m * dy, 0, m * dz), setup["gamma"],
                      setup["cfl"], setup["limiter"], setup["riemann"], setup["precision"])
    sp = dict(sp, integrator=setup.get("integrator", "rk2"))
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
