"""Writes c5_oracle_gradient.txt: the oracle's spring-stiffness gradient on the
differentiation workload (256 x 256 periodic Stokes, mu = 1, dt = 1e-3,
membrane of 1024 points, kappa_i = 1e3 (1 + 0.5 u_i), u_i ~ U[-1, 1] with
seed 1; loss 0.5 ||u - u_target||^2 with u_target solved at the kappa field
of seed 2; right-hand side seed 0).

Every number comes from the oracle alone: the forward and target solves and
the adjoint solve L_IB^T lam = (u - u_target, 0) by the oracle's FGMRES with
its V-cycle to a 1e-13 reduction, then dL/dkappa_e = -lam^T (dL_IB/dkappa_e) w
(Eq. matrix-impib with the stiffness of spring e alone).

    python tests/golden/make_c5_gradient.py      # about two minutes on 8 cores
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.solver import Problem, spring_gradient  # noqa: E402

OUT = os.path.join(HERE, "c5_oracle_gradient.txt")


def main():
    wl = W.diff_256(field_seed=1)
    wt = W.diff_256(field_seed=2)
    b = W.rhs(wl.N, 0)
    P = Problem(wl)
    w, iw = P.solve(b, rtol=1e-13, max_it=400)
    ut, it = Problem(wt).solve(b, rtol=1e-13, max_it=400)
    n2 = 2 * wl.N * wl.N
    rhs = np.zeros_like(w)
    rhs[:n2] = w[:n2] - ut[:n2]
    lam, il = P.solve(rhs, rtol=1e-13, max_it=400)
    g = spring_gradient(wl, w, lam)
    loss = 0.5 * float(np.dot(w[:n2] - ut[:n2], w[:n2] - ut[:n2]))
    with open(OUT, "w") as f:
        f.write("# Oracle gradient dLoss/dkappa_e of the differentiation workload, written by\n")
        f.write("# tests/golden/make_c5_gradient.py (oracle only; see its docstring for the inputs).\n")
        f.write(f"# forward {iw['iters']} iterations (true rel. res. {iw['rel_res_true']:.3e}), "
                f"target {it['iters']}, adjoint {il['iters']} ({il['rel_res_true']:.3e})\n")
        f.write(f"# loss {loss:.17e}\n")
        f.write(f"# {len(g)} springs, one value per line in spring order\n")
        for v in g:
            f.write(f"{v:.17e}\n")
    print(OUT, len(g), loss)


if __name__ == "__main__":
    main()
