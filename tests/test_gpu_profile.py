"""Per-kernel timing (sclap_profile_begin / sclap_profile_begin_only /
sclap_profile_end): timing never changes a result, every launch group of a
partition is reported when all are timed, and only the named group when one
is selected; the totals are cleared by the end call.
"""
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


def test_profiling_all_and_one_kernel(sc):
    g = synth.rmat(14, 16, seed=3)
    d = sc.to_device(g, "cuda")
    ref = oracle.partition(g, 8, 0.03, 2, coarsest_nodes=500)

    sc.profile_begin()
    r_all = sc.partition_dev(d, 8, 0.03, 2, coarsest_nodes=500)
    torch.cuda.synchronize()
    all_stats = sc.profile_end()
    assert np.array_equal(r_all["part"].cpu().numpy(), ref["part"]) and r_all["cut"] == ref["cut"]
    # label propagation, admission and contraction groups are all there
    for name in ("lp_apply", "contract_count", "contract_emit"):
        assert name in all_stats and all_stats[name]["launches"] > 0, name
    assert any(k.startswith("lp_eval") or k.startswith("lp_refine") for k in all_stats)
    assert all(v["ms"] >= 0 for v in all_stats.values())

    sc.profile_begin(only="lp_apply")
    r_one = sc.partition_dev(d, 8, 0.03, 2, coarsest_nodes=500)
    torch.cuda.synchronize()
    one = sc.profile_end()
    assert np.array_equal(r_one["part"].cpu().numpy(), ref["part"]) and r_one["cut"] == ref["cut"]
    assert list(one) == ["lp_apply"]
    assert one["lp_apply"]["launches"] == all_stats["lp_apply"]["launches"]

    # the totals were cleared, and without profiling nothing is recorded
    sc.profile_begin(only="no_such_kernel")
    sc.partition_dev(d, 8, 0.03, 2, coarsest_nodes=500)
    torch.cuda.synchronize()
    assert sc.profile_end() == {}


def test_gather_probe(sc):
    # the measurement helper: positive pass times for 4- and 1-byte labels,
    # an error for other label widths, and an edgeless graph takes no time
    g = synth.rmat(16, 16, seed=4)
    d = sc.to_device(g, "cuda")
    t4 = sc.gather_probe_dev(d, 4, reps=2)
    t1 = sc.gather_probe_dev(d, 1, reps=2)
    assert t4 > 0 and t1 > 0
    with pytest.raises(sc.SclapError):
        sc.gather_probe_dev(d, 2)
    n = 100
    e = {"n": n, "xadj": np.zeros(n + 1, dtype=np.int64), "adjncy": np.zeros(0, dtype=np.int32)}
    assert sc.gather_probe_dev(sc.to_device(e, "cuda"), 4) == 0.0
