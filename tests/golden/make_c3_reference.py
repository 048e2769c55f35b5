"""Write the FP64 oracle's march of the inhomogeneous-medium workload
(8192 x 4096, seed 0, nl(x), D(x), absorption) at steps 500, 1000, 1500 and
2000, sampled on rows, to c3_seed0_oracle_rows.npz.

Only the oracle (oracle/) and the seeded input generator are called; the
march is taken in four 500-step segments (each segment starts from the
previous segment's physical field).  Takes hours on a few CPU cores:

    OMP_NUM_THREADS=6 python tests/golden/make_c3_reference.py
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

OUT = os.path.join(HERE, "c3_seed0_oracle_rows.npz")
SEGMENT = 500
ROWS_FINAL = np.arange(0, 4096, 256)          # 16 rows at step 2000
ROWS_MID = np.array([0, 1024, 2048, 3072])    # 4 rows at steps 500, 1000, 1500


def main():
    p = I.c3()
    u = p.u0.copy()
    out = {"rows_final": ROWS_FINAL, "rows_mid": ROWS_MID, "seed": np.array(0), "segment": np.array(SEGMENT)}
    t0 = time.time()
    for g in range(p.n_steps // SEGMENT):
        u = oracle.run(p, n_steps=SEGMENT, first=g * SEGMENT, u=u)
        s = (g + 1) * SEGMENT
        rows = ROWS_FINAL if s == p.n_steps else ROWS_MID
        out["u_step%d" % s] = u[rows].copy()
        out["norm_step%d" % s] = np.array(np.linalg.norm(u))
        print("step %d done after %.0f s" % (s, time.time() - t0), flush=True)
        np.savez(OUT + ".partial.npz", **out)
    np.savez(OUT, **out)
    os.remove(OUT + ".partial.npz")
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
