"""The allocation-free cut entry point (sclap_cut_dev_noalloc) against the
allocating one (sclap_cut_dev) through the C ABI: identical cut and block
weights on two calls in a row, the second on a smaller input (the workspace
keeps the first call's contents), and the size limit rejected before any work."""
import numpy as np
import pytest

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


def _part(n, k, seed):
    return torch.tensor(np.random.default_rng(seed).integers(0, k, size=max(n, 1)).astype(np.int32)[:n],
                        device="cuda")


def test_noalloc_cut_matches_cut_dev_twice(sc):
    big = synth.rmat(15, 16, seed=21, weighted=True)
    big["vwgt"] = np.random.default_rng(5).integers(0, 7, size=big["n"]).astype(np.int32)
    small = synth.ba(3000, 4, seed=22, weighted=True)
    for g, k, seed in ((big, 300, 1), (small, 5, 2)):
        print("noalloc cut: n=%d S=%d k=%d" % (g["n"], int(g["xadj"][-1]), k), flush=True)
        d = sc.to_device(g, "cuda")
        p = _part(g["n"], k, seed)
        c0, bw0 = sc.cut_dev(d, p, k)
        c1, bw1 = sc.cut_dev_noalloc(d, p, k)
        assert c1 == c0 and np.array_equal(bw1, bw0)
        assert int(bw1.sum()) == int(g["vwgt"].sum())


def test_noalloc_cut_edge_cases(sc):
    # edgeless graph (no slot tiles), one block, and the largest k
    n = 1000
    g = {"n": n, "xadj": np.zeros(n + 1, dtype=np.int64), "adjncy": np.zeros(0, dtype=np.int32),
         "adjwgt": None, "vwgt": None}
    d = sc.to_device(g, "cuda")
    c, bw = sc.cut_dev_noalloc(d, _part(n, 1, 3), 1)
    assert c == 0 and bw.tolist() == [n]
    h = synth.rgg(5000, seed=23, weighted=True)
    dh = sc.to_device(h, "cuda")
    p = _part(h["n"], 65536, 4)
    c0, bw0 = sc.cut_dev(dh, p, 65536)
    c1, bw1 = sc.cut_dev_noalloc(dh, p, 65536)
    assert c1 == c0 and np.array_equal(bw1, bw0)


def test_noalloc_cut_rejects_beyond_workspace(sc):
    g = synth.ba(500, 2, seed=24)
    d = sc.to_device(g, "cuda")
    with pytest.raises(sc.SclapError):
        sc.cut_dev_noalloc(d, _part(g["n"], 4, 5), 65537)
    bad = _part(g["n"], 4, 6)
    bad[7] = 4  # a block id outside [0, k)
    with pytest.raises(sc.SclapError):
        sc.cut_dev_noalloc(d, bad, 4)
    c0, bw0 = sc.cut_dev(d, _part(g["n"], 4, 6), 4)
    c1, bw1 = sc.cut_dev_noalloc(d, _part(g["n"], 4, 6), 4)
    assert c1 == c0 and np.array_equal(bw1, bw0)
