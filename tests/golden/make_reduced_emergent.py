"""Write tests/golden/<config>_nz<N>_emergent.txt: emergent Stokes profiles of
the two-term workloads (the Mg II-like doublet, cfg3, and the Ly-alpha-like
line, cfg4) on their full frequency and angular grids but with N heights of the
same seeded generator, from the FP64 oracle solved to a relative residual of
1e-11; optionally in the angle-averaged mode.  Calls only the oracle.

    python tests/golden/make_reduced_emergent.py cfg3 3
    python tests/golden/make_reduced_emergent.py cfg4 2 [aa]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import transfer as T   # noqa: E402
import workloads                    # noqa: E402


def main():
    name, n_z = sys.argv[1], int(sys.argv[2])
    aa = len(sys.argv) > 3 and sys.argv[3] == "aa"
    prob = getattr(workloads, name)(n_z=n_z)
    t0 = time.time()
    op = T.setup(prob, {"aa": aa})
    print(f"setup {time.time() - t0:.1f}s", flush=True)
    sol = T.solve(op, tol=1e-11)
    print(f"solve done {time.time() - t0:.1f}s", flush=True)
    up = op.ang["mu"] > 0
    em = sol[-1][up]
    rows = [[o, n, *em[o, n]] for o in range(em.shape[0]) for n in range(0, em.shape[1], 4)]
    tag = f"{name}_nz{n_z}{'_aa' if aa else ''}"
    out = os.path.join(HERE, f"{tag}_emergent.txt")
    np.savetxt(out, np.array(rows), fmt=["%d", "%d", "%.17e", "%.17e", "%.17e", "%.17e"],
               header=f"{name} generator on {n_z} heights{' (angle-averaged PRD)' if aa else ''}, FP64 oracle "
                      "solve to 1e-11; every 4th frequency; columns: outgoing mu>0 direction index, frequency index, I, Q, U, V at z_max")
    print("wrote", out, em.shape, f"{time.time() - t0:.1f}s")


if __name__ == "__main__":
    main()
