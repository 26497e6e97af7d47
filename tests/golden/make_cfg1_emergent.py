"""Write tests/golden/cfg1_emergent.txt: the emergent Stokes profiles of the
two-level slab workload (N_z = 40, N_nu = 31 on [-8, 8], 2 + 2 mu x 4 chi,
horizontal 20 G field) from the FP64 oracle, solved to a relative residual of
1e-12.  Calls only the oracle.

    python tests/golden/make_cfg1_emergent.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import transfer as T   # noqa: E402
from workloads import cfg1          # noqa: E402


def main():
    prob = cfg1()
    op = T.setup(prob)
    sol = T.solve(op, tol=1e-12)
    up = op.ang["mu"] > 0
    em = sol[-1][up]                                  # [o_up][n][4] at the top
    rows = []
    for o in range(em.shape[0]):
        for n in range(em.shape[1]):
            rows.append([o, n, *em[o, n]])
    out = os.path.join(HERE, "cfg1_emergent.txt")
    np.savetxt(out, np.array(rows), fmt=["%d", "%d", "%.17e", "%.17e", "%.17e", "%.17e"],
               header="two-level slab workload (cfg1), FP64 oracle solve to 1e-12; "
                      "columns: outgoing mu>0 direction index, frequency index, I, Q, U, V at z_max")
    print("wrote", out, em.shape)


if __name__ == "__main__":
    main()
