"""Write the per-level golden digests of the R-MAT scale-24 workload.

Calls only the seeded generator (``graphgen``) and the CPU oracle
(``oracle``): multi-level Louvain (Alg. 3 around Alg. 2, 20 sweeps per level)
and LPA (Alg. 1, 20 sweeps) on R-MAT scale 24, edge factor 16,
(a, b, c) = (0.57, 0.19, 0.19), seed 2, unit weights.  For every attempted
level it stores n, nnz, n_next, Q_start, Q_end, acceptance, the per-sweep
move counts, a SHA-256 of the level's renumbered labels (int32, little
endian) and, for accepted levels, a SHA-256 of the coarse graph the level
produces (offsets, indices, weights as int32 with the community's internal
weight on the diagonal counted twice, columns sorted).  The GPU test and
bench.py compare the library's results at full size against this file.

Takes about six minutes on eight cores:
    python tests/golden/make_rmat24_digests.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "rmat24_seed2_digests.json")


def sha(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype="<i4").tobytes())
    return h.hexdigest()


def main():
    t = time.time()
    g = graphgen.rmat(24, 16, seed=2)
    print(f"generated n={g.n} nnz={g.nnz} in {time.time() - t:.1f}s", flush=True)
    t = time.time()
    res = oracle.louvain(g, max_sweeps=20, keep_graphs=True)
    print(f"oracle louvain: {len(res.levels)} levels in {time.time() - t:.1f}s", flush=True)
    levels = []
    for lvl, rec in enumerate(res.levels):
        d = {"level": lvl, "n": rec.n, "nnz": rec.nnz, "n_next": rec.n_next, "q_start": rec.q_start,
             "q_end": rec.q_end, "accepted": bool(rec.accepted), "sweeps": rec.sweeps,
             "moves": [int(x) for x in rec.moves], "labels_sha256": sha(rec.labels)}
        if rec.accepted:
            co = res.graphs[lvl + 1]
            d["coarse_nnz"] = co.nnz
            d["coarse_sha256"] = sha(co.off, co.idx, co.a)
        levels.append(d)
        print(json.dumps(d), flush=True)
    t = time.time()
    lp = oracle.lpa(g, max_sweeps=20)
    print(f"oracle lpa in {time.time() - t:.1f}s", flush=True)
    out = {
        "workload": "R-MAT scale 24, edge factor 16, (a, b, c) = (0.57, 0.19, 0.19), symmetrised, loops and "
                    "duplicates removed, unit weights, seed 2",
        "n": g.n, "nnz": g.nnz, "max_sweeps": 20,
        "louvain": {"M": res.M, "q_int": res.q_int, "final_labels_sha256": sha(res.final_labels),
                    "levels": levels},
        "lpa": {"moves": [int(x) for x in lp.moves], "labels_sha256": sha(lp.labels), "q_int": lp.q_int},
        "written_by": "tests/golden/make_rmat24_digests.py (graphgen + oracle only)",
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
