"""Serving loop: continuous batching of partition requests.

A request's result must not depend on the requests it shares the GPU with:
every result from the server equals the partition of that graph alone
(plain entry point, and the CPU oracle for the small graphs), whether it ran
alone or in a mix of concurrently submitted requests.  Also covers the
memory-budget refusal, per-request error isolation and the timing record.
"""
import threading

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sc():
    import paper_1404_4797_amd as m
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m.load()
    return m


def say(*a):
    print(*a, flush=True)


def requests():
    gs = synth.batch_mix(16, seed=9, n_lo_log2=8, n_hi_log2=14)
    return [(g, g["k"], g["eps"], g["seed"]) for g in gs]


OPTS = dict(coarsest_nodes=300)


def test_results_equal_solo_and_oracle(sc):
    reqs = requests()
    say("serve mix of", len(reqs))
    with sc.Server(slots=3, max_batch=4, **OPTS) as sv:
        ids = [sv.submit(g, k, e, s) for g, k, e, s in reqs]
        res = [sv.wait(i) for i in ids]
    for (g, k, e, s), r in zip(reqs, res):
        ref = oracle.partition(g, k, e, s, **OPTS)
        assert np.array_equal(r["part"], ref["part"])
        assert r["cut"] == ref["cut"] and np.array_equal(r["block_weights"], ref["block_weights"])
        assert r["status"] == ref["status"]
        assert r["submit_ms"] <= r["start_ms"] <= r["done_ms"] and r["batch_size"] >= 1
    assert max(r["batch_size"] for r in res) > 1  # some requests did share a batch


def test_alone_equals_in_mix(sc):
    reqs = requests()
    probe = reqs[5]
    with sc.Server(slots=1, max_batch=1, **OPTS) as sv:
        alone = sv.wait(sv.submit(*probe))
    assert alone["batch_size"] == 1
    with sc.Server(slots=2, max_batch=16, **OPTS) as sv:
        ids = []
        lock = threading.Lock()

        def client(chunk):
            for q in chunk:
                rid = sv.submit(*q)
                with lock:
                    ids.append((q is probe, rid))

        th = [threading.Thread(target=client, args=(reqs[i::3],)) for i in range(3)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        out = {rid: sv.wait(rid) for _, rid in ids}
    mixed = out[[rid for is_probe, rid in ids if is_probe][0]]
    assert np.array_equal(mixed["part"], alone["part"]) and mixed["cut"] == alone["cut"]
    plain = sc.partition(probe[0], probe[1], probe[2], probe[3], **OPTS)
    assert np.array_equal(plain["part"], alone["part"])


def test_budget_and_errors(sc):
    g = synth.ba(2000, 4, seed=3)
    with sc.Server(slots=1, hbm_budget=1 << 20, **OPTS) as sv:  # smaller than any request
        with pytest.raises(sc.SclapError) as e:
            sv.submit(g, 2, 0.03, 1)
        assert e.value.status == sc.ERR_NO_MEMORY
    bad = synth.from_edges(5, [(0, 1), (1, 2), (2, 3), (3, 4)], weights=[1, 2, 3, 4])
    bad = dict(bad)
    w = bad["adjwgt"].copy()
    w[0] = 7  # (0,1) now differs from its twin (1,0): not symmetric
    bad["adjwgt"] = w
    good = synth.rgg(600, seed=4)
    with sc.Server(slots=1, max_batch=8, **OPTS) as sv:
        i_good = sv.submit(good, 4, 0.03, 5)
        i_bad = sv.submit(bad, 2, 0.03, 6)
        r_good = sv.wait(i_good)
        with pytest.raises(sc.SclapError) as e:
            sv.wait(i_bad)
        assert e.value.status == sc.ERR_NOT_SYMMETRIC
    ref = oracle.partition(good, 4, 0.03, 5, **OPTS)
    assert np.array_equal(r_good["part"], ref["part"])
