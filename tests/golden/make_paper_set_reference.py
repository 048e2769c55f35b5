"""Write the FP64 oracle's whole march of the paper's workload on the grid
of set k of Table 0 (Sec. 4: N_theta tau-points and the power of two nearest
N_rho rows, e.g. 448 x 1024 for set 1; random medium, regularised
multiplier, N_sigma steps to Sigma = 120), sampled on 16 rows at the middle
and the end of the march, to paper_set<k>_oracle_rows.npz.  The
regularisation uses the machine epsilon of the working precision, so the
march is written once for eps = 2^-53 (the FP64 reference) and once for
eps = 2^-24 (the FP32 reference).

Only the oracle (oracle/) and the seeded input generator are called.  Set 1
takes a few minutes on a few CPU cores, set 2 about a quarter of an hour:

    python tests/golden/make_paper_set_reference.py 1 [f64,f32]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_2103_06080_amd import inputs as I  # noqa: E402

EPS = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}


def main(k, tags):
    out_path = os.path.join(HERE, "paper_set%d_oracle_rows.npz" % k)
    n_y = I.PAPER_SET_GRIDS[k][1]
    rows = np.arange(0, n_y, n_y // 16)
    out = {"rows": rows}
    t0 = time.time()
    for tag in tags:
        p = I.paper_set(k, reg_eps=EPS[tag])
        half = p.n_steps // 2
        u = oracle.run(p, n_steps=half, first=0, u=p.u0.copy())
        out["%s_step%d" % (tag, half)] = u[rows].copy()
        u = oracle.run(p, n_steps=p.n_steps - half, first=half, u=u)
        out["%s_step%d" % (tag, p.n_steps)] = u[rows].copy()
        out["%s_norm_step%d" % (tag, p.n_steps)] = np.array(np.linalg.norm(u))
        print("%s done after %.0f s" % (tag, time.time() - t0), flush=True)
        np.savez(out_path, **out)
        print("wrote", out_path, flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 1, sys.argv[2].split(",") if len(sys.argv) > 2 else list(EPS))
