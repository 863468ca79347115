"""Write the oracle reference for the 131072-node, 64-hole workload.

Calls only the CPU oracle (`oracle/`) and the input generator (`workloads/`):
  * the level-parallel RS of Sections 2.2-2.7 with the bordered root of
    Section 3.2 at ID tolerance 1e-10, with the "key20" pivot rule (the rule
    the GPU library uses) and with the default plain max-norm rule;
  * the direct RS solution of the first right-hand-side column of the
    benchmark (16 columns from exterior point forces, seed 3);
  * the discrete solution of the augmented system (eq. backwardeq) to a
    relative residual below 1e-13, reached by float64 iterative refinement
    with the exact operator applied on the fly and the oracle's RS as the
    inner solver.  That solution does not depend on any pivot choice.

Output: c3_reference.npz (solutions, per-box ranks, residuals) and
c3_reference.txt (the figures in text).  Run: python tests/golden/make_reference_c3.py
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import stokes  # noqa: E402
from oracle.rs import RSFactorization, RSParams  # noqa: E402
from workloads import boundary_data, exterior_forces_for_geometry, workload_circle40_64holes  # noqa: E402


def rel_residual(g, x, f):
    rhs = np.vstack([f, np.zeros((3 * g.n_holes, f.shape[1]))])
    r = rhs - stokes.apply_system(g, x)
    return r, float(np.max(np.linalg.norm(r, axis=0) / np.linalg.norm(f, axis=0)))


def ranks_of(rs):
    ids = sorted(rs.fac)
    return (np.array([rs.fac[b].level for b in ids], np.int32), np.array([rs.fac[b].I.size for b in ids], np.int32),
            np.array([rs.fac[b].k for b in ids], np.int32), np.array(ids, np.int32))


def main():
    log = []

    def say(msg):
        print(msg, flush=True)
        log.append(msg)

    g = workload_circle40_64holes()
    f = boundary_data(g, exterior_forces_for_geometry(g, 16, seed=3))[:, :1]
    say("workload: circle R=40 (16384 nodes) + 64 ellipses (1792 nodes), N=%d, p=%d, rhs column 0 of 16 (seed 3)"
        % (g.n_nodes, g.n_holes))
    out = {}
    for rule in ("key20", "max"):
        t0 = time.perf_counter()
        rs = RSFactorization(g, RSParams(tol=1e-10, pivot=rule)).factor()
        t1 = time.perf_counter()
        x = rs.solve(f)
        r, res = rel_residual(g, x, f)
        lev, nn, kk, ids = ranks_of(rs)
        say("pivot %s: factor %.1f s, levels %d, root %d, direct relative residual %.3e"
            % (rule, t1 - t0, rs.L, rs.I0.size, res))
        out["levels_" + rule], out["n_" + rule], out["k_" + rule], out["box_" + rule] = lev, nn, kk, ids
        out["res_direct_" + rule] = np.array([res])
        if rule == "key20":
            out["x_direct_key20"] = x
            xr = x.copy()
            for it in range(1, 8):
                xr = xr + rs.solve(r)
                r, res = rel_residual(g, xr, f)
                say("refinement %d: relative residual %.3e" % (it, res))
                if res <= 1e-13:
                    break
            out["x_ref"] = xr
            out["res_ref"] = np.array([res])
    out["f"] = f
    np.savez_compressed(os.path.join(HERE, "c3_reference.npz"), **out)
    with open(os.path.join(HERE, "c3_reference.txt"), "w") as fh:
        fh.write("# Oracle reference for the 64-hole workload (written by make_reference_c3.py)\n")
        fh.write("# Section 3.2 eq. backwardeq system; RS of Sections 2.2-2.7 at ID tolerance 1e-10\n")
        for m in log:
            fh.write(m + "\n")


if __name__ == "__main__":
    main()
