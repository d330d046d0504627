"""Write the per-level golden digests of the LFR-style workload.

Calls only the seeded generator (``graphgen``) and the CPU oracle
(``oracle``): multi-level Louvain (Alg. 3 around Alg. 2, 20 sweeps per level)
and LPA (Alg. 1, 20 sweeps) on the LFR-style graph with 10,000,000 vertices
(degree exponent 2.5, mean degree 20, max degree 5,000, community sizes
50-20,000 with exponent 1.5, mixing 0.3, weights 1..8), seed 3.  For every
attempted level it stores the digests described in ``digests.py``.  The GPU
test compares the library's results at full size against this file.

Takes a few minutes on eight cores:
    python tests/golden/make_lfr10m_digests.py
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

OUT = os.path.join(HERE, "lfr10m_seed3_digests.json")


def main():
    t = time.time()
    g, _ = graphgen.lfr(10_000_000, seed=3)
    print(f"generated n={g.n} nnz={g.nnz} in {time.time() - t:.1f}s", flush=True)
    write_digests(oracle, g, "LFR-style, n = 10,000,000, degree exponent 2.5, mean degree 20, max degree 5,000, "
                  "community sizes 50-20,000 (exponent 1.5), mixing 0.3, weights 1..8, seed 3",
                  "tests/golden/make_lfr10m_digests.py (graphgen + oracle only)", OUT)


if __name__ == "__main__":
    main()
