"""Mesh-type workloads of the paper's benchmark set (delX: Delaunay
triangulations; rggX: random geometric graphs with radius 0.55 sqrt(ln n/n);
Section 5.1 benchmark set) on the GPU, bit for bit against the oracle:
several multilevel configurations, V-cycles and degree order, and the
Delaunay 2^18 workload against the stored digest of the oracle's output.
These graphs have low, even degrees (no hub or workgroup rows) and no
isolated nodes, the opposite regime to R-MAT.
"""
import hashlib
import json
import os

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


MESHES = {
    "del13": lambda: synth.delaunay(1 << 13, seed=2),
    "del15": lambda: synth.delaunay(1 << 15, seed=4),
    "rgg14_paper": lambda: synth.rgg_paper(1 << 14, seed=5),
}


@pytest.mark.parametrize("gname", list(MESHES))
@pytest.mark.parametrize("k", [2, 16, 64])
@pytest.mark.parametrize("opts", [dict(coarsest_nodes=500), dict(coarsest_nodes=500, vcycles=2),
                                  dict(coarsest_nodes=2000, degree_order=1)])
def test_mesh_partition_parity(sc, gname, k, opts):
    g = MESHES[gname]()
    say("mesh", gname, k, opts)
    r = sc.partition_dev(sc.to_device(g, "cuda"), k, 0.03, 3, **opts)
    ref = oracle.partition(g, k, 0.03, 3, **opts)
    assert r["stats"]["level_n"] == ref["level_n"] and r["stats"]["visits"] == ref["visits"]
    assert np.array_equal(r["part"].cpu().numpy(), ref["part"])
    assert r["cut"] == ref["cut"] and np.array_equal(r["block_weights"], ref["block_weights"])
    assert r["status"] == ref["status"]


def test_del18_digest(sc, golden_dir):
    with open(os.path.join(golden_dir, "oracle_digests.json")) as f:
        w = json.load(f)["workloads"]["del18_k16"]
    g = synth.delaunay(w["graph"]["n"], seed=w["graph"]["seed"])
    assert hashlib.sha256(g["adjncy"].tobytes()).hexdigest() == w["input_sha256"]
    r = sc.partition_dev(sc.to_device(g, "cuda"), w["k"], w["eps"], w["seed"], **w["opts"])
    part = r["part"].cpu().numpy().astype(np.int32)
    assert r["stats"]["level_n"] == w["level_n"]
    assert r["cut"] == w["cut"] and r["block_weights"].tolist() == w["block_weights"]
    assert hashlib.sha256(part.tobytes()).hexdigest() == w["part_sha256"]
