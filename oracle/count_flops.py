"""ORACLE — test infrastructure.

Prints the algorithmic floating-point operations per cell of one right-hand
side evaluation of the method, per phase, on the benchmark workload (3D
turbulence generator, van Leer, HLLD) and on the 3D Orszag-Tang problem with
WENO-Z, counted by running the oracle's own
step with an operation-counting scalar: every add/sub, mul, div and sqrt is
one flop. These are the figures bench.py uses for the ALU roofline entry.

    python -m oracle.count_flops [n]
"""
import json
import sys

import oracle as O
from paper_2511_20337_amd import workloads as W


def main(n=64):
    s, U = W.turbulence_3d(n)
    r = O.count_ops(O.cfg_from(s), U)
    cells = n ** 3
    out = {k: {kk: vv / cells for kk, vv in v.items()} for k, v in r.items()}
    per = {k: sum(v.values()) for k, v in out.items()}
    print(json.dumps({"workload": "turbulence_3d_%d" % n, "ops_per_cell": out,
                      "flops_per_cell": per,
                      "faces_kernel_flops_per_cell": per["prims"] + per["faces"],
                      "rhs_flops_per_cell": sum(per.values())}, indent=1))
    # the WENO-Z face phase on the 3D Orszag-Tang problem (primitives are
    # recovered by a kernel of their own there, so the face kernel is "faces")
    s, U = W.orszag_tang_3d(n, limiter="wenoz")
    r = O.count_ops(O.cfg_from(s), U)
    per = {k: sum(v.values()) / cells for k, v in r.items()}
    print(json.dumps({"workload": "orszag_tang_3d_%d wenoz" % n, "flops_per_cell": per,
                      "weno_faces_kernel_flops_per_cell": per["faces"]}, indent=1))


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 64)
