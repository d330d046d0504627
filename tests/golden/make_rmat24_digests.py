"""Write the per-level golden digests of the R-MAT scale-24 workload.

Calls only the seeded generator (``graphgen``) and the CPU oracle
(``oracle``): multi-level Louvain (Alg. 3 around Alg. 2, 20 sweeps per level)
and LPA (Alg. 1, 20 sweeps) on R-MAT scale 24, edge factor 16,
(a, b, c) = (0.57, 0.19, 0.19), seed 2, unit weights.  For every attempted
level it stores the digests described in ``digests.py``.  The GPU test and
bench.py compare the library's results at full size against this file.

Takes about six minutes on eight cores:
    python tests/golden/make_rmat24_digests.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, HERE)

import graphgen  # noqa: E402
import oracle  # noqa: E402
from digests import write_digests  # noqa: E402

OUT = os.path.join(HERE, "rmat24_seed2_digests.json")


def main():
    t = time.time()
    g = graphgen.rmat(24, 16, seed=2)
    print(f"generated n={g.n} nnz={g.nnz} in {time.time() - t:.1f}s", flush=True)
    write_digests(oracle, g, "R-MAT scale 24, edge factor 16, (a, b, c) = (0.57, 0.19, 0.19), symmetrised, loops "
                  "and duplicates removed, unit weights, seed 2",
                  "tests/golden/make_rmat24_digests.py (graphgen + oracle only)", OUT)


if __name__ == "__main__":
    main()
