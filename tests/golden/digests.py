"""Per-level golden digests of a full-size workload, from the CPU oracle.

Shared by the scripts that write ``*_digests.json`` beside this file: it
calls only the oracle (``oracle``): multi-level Louvain (Alg. 3 around
Alg. 2) and LPA (Alg. 1).  For every attempted level it stores n, nnz,
n_next, Q_start, Q_end, acceptance, the per-sweep move counts, a SHA-256 of
the level's renumbered labels (int32, little endian) and, for accepted
levels, a SHA-256 of the coarse graph the level produces (offsets, indices,
weights as int32 with the community's internal weight on the diagonal
counted twice, columns sorted).
"""
import hashlib
import json
import time

import numpy as np


def sha(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype="<i4").tobytes())
    return h.hexdigest()


def write_digests(oracle, g, workload: str, written_by: str, out_path: str, max_sweeps: int = 20):
    t = time.time()
    res = oracle.louvain(g, max_sweeps=max_sweeps, keep_graphs=True)
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
    lp = oracle.lpa(g, max_sweeps=max_sweeps)
    print(f"oracle lpa in {time.time() - t:.1f}s", flush=True)
    out = {
        "workload": workload,
        "n": g.n, "nnz": g.nnz, "max_sweeps": max_sweeps,
        "louvain": {"M": res.M, "q_int": res.q_int, "final_labels_sha256": sha(res.final_labels),
                    "levels": levels},
        "lpa": {"moves": [int(x) for x in lp.moves], "labels_sha256": sha(lp.labels), "q_int": lp.q_int},
        "written_by": written_by,
    }
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(f"wrote {out_path}", flush=True)
