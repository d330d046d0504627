"""Continuous-batching server through the C ABI: every job's partition equals
the oracle's for its graph alone, whatever else shares its packed levels, the
admission order, the memory budget or the in-flight limit."""
import sys
import threading
import time

import numpy as np
import pytest

import bruteforce as bf
import graphgen
import oracle
import paper_2507_06471_amd as lvp

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def job_mix(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        kind = t % 6
        if kind == 0:
            n = int(rng.integers(1, 40))
            g = bf.to_csr(n, bf.random_graph(rng, n, float(rng.uniform(0.05, 0.4)), 9, True))
        elif kind == 1:
            g = graphgen.sbm(int(rng.integers(300, 3000)), 64, 0.08, 0.001, seed=int(rng.integers(1 << 30)))
        elif kind == 2:
            g = graphgen.rmat(int(rng.integers(9, 14)), seed=int(rng.integers(1 << 30)))
        elif kind == 3:
            g, _ = graphgen.lfr(int(rng.integers(2000, 6000)), kmax=300, smin=20, smax=600,
                                seed=int(rng.integers(1 << 30)))
        elif kind == 4:
            n = int(rng.integers(0, 20))
            g = graphgen.CSR(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), None)
        else:
            g = graphgen.rmat(12, seed=int(rng.integers(1 << 30)))
            g.weights = graphgen.pair_weights(g, 1, 5, seed=int(rng.integers(1 << 30)))
        g.name = f"job{seed}.{t}"
        out.append(g)
    return out


def check(g, labels, info):
    want = oracle.louvain(g)
    assert info["status"] == 0, g.name
    assert np.array_equal(labels, want.final_labels), g.name
    assert (info["q_int"], info["m"], info["q"]) == (want.q_int, want.M, want.q), g.name
    assert info["levels"] == sum(1 for lv in want.levels if lv.accepted), g.name


@pytest.mark.parametrize("max_jobs,budget", [(0, 0), (3, 0), (64, 40 << 20)])
def test_concurrent_jobs_equal_each_graph_alone(max_jobs, budget):
    graphs = job_mix(1, 30)
    say(f"server max_jobs={max_jobs} budget={budget} jobs={len(graphs)}")
    with lvp.Server(mem_budget=budget, max_jobs=max_jobs) as srv:
        tickets = [None] * len(graphs)

        def client(part):
            for i in part:
                tickets[i] = srv.submit(graphs[i])
                time.sleep(0.002 * (i % 3))

        threads = [threading.Thread(target=client, args=(range(k, len(graphs), 3),)) for k in range(3)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        for g, t in zip(graphs, tickets):
            assert srv.wait(t, 60000)
            labels, info = srv.result(t, g.n)
            check(g, labels, info)
        st = srv.stats()
        say(f"stats {st}")
        assert st["completed"] == len(graphs) and st["in_flight"] == 0 and st["mem_in_use"] == 0
        if max_jobs == 3:
            assert st["max_batch"] <= 3


def test_jobs_join_while_others_run():
    big = graphgen.rmat(16, seed=9)
    small = job_mix(2, 12)
    with lvp.Server() as srv:
        tb = srv.submit(big)
        time.sleep(0.01)
        ts = [srv.submit(g) for g in small]
        for g, t in zip(small, ts):
            srv.wait(t)
            check(g, *srv.result(t, g.n))
        srv.wait(tb)
        check(big, *srv.result(tb, big.n))
        assert srv.stats()["max_batch"] >= 2


def test_bad_job_fails_alone_and_cancel():
    good = graphgen.sbm(1000, 50, 0.1, 0.002, seed=3)
    bad = graphgen.CSR(2, np.array([0, 1, 2], np.int32), np.array([1, 1], np.int32), None)  # asymmetric
    with lvp.Server(max_jobs=1) as srv:
        t1 = srv.submit(good)
        t2 = srv.submit(bad)
        t3 = srv.submit(good)
        srv.cancel(t3)
        srv.wait(t1)
        check(good, *srv.result(t1, good.n))
        srv.wait(t2)
        with pytest.raises(lvp.LvError) as ei:
            srv.result(t2, bad.n)
        assert ei.value.status == 3
        srv.wait(t3)
        with pytest.raises(lvp.LvError) as ei:
            srv.result(t3, good.n)
        assert ei.value.status == 10
        with pytest.raises(lvp.LvError) as ei:
            srv.poll(t3)
        assert ei.value.status == 12


def test_too_large_and_destroy_with_pending_jobs():
    g = graphgen.rmat(12, seed=1)
    with lvp.Server(mem_budget=1 << 20) as srv:
        with pytest.raises(lvp.LvError) as ei:
            srv.submit(g)
        assert ei.value.status == 9
    srv = lvp.Server()
    for _ in range(5):
        srv.submit(g)
    srv.close()  # must not hang or leak: pending jobs are cancelled


def test_device_resident_submissions_and_staging():
    # jobs submitted from device memory (copied device to device) mixed with
    # host submissions; every job equals the oracle's result for its graph
    gs = job_mix(77, 18)
    with lvp.Server(max_jobs=4) as srv:
        tickets = [srv.submit(g, device=(i % 2 == 0)) for i, g in enumerate(gs)]
        for g, t in zip(gs, tickets):
            assert srv.wait(t, 120000)
            labels, info = srv.result(t, g.n)
            assert info["status"] == 0
            want = oracle.louvain(g)
            assert np.array_equal(labels, want.final_labels), g.name
            assert info["q_int"] == want.q_int
        st = srv.stats()
        assert st["completed"] == len(gs) and st["in_flight"] == 0 and st["mem_in_use"] == 0
