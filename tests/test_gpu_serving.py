"""GPU tests of the serving loop: jobs of mixed size and (r, s) submitted
together run concurrently on worker streams, and each result is identical to
the same job decomposed alone (and to the CPU oracle where it is small)."""
import numpy as np
import pytest

from oracle import oracle
from paper_2111_10980_amd import inputs

pytestmark = pytest.mark.gpu


def _nd():
    import paper_2111_10980_amd as nd
    return nd


def _canon(rcl, kap):
    rcl = np.asarray(rcl)
    kap = np.asarray(kap).view(np.uint32)
    if rcl.shape[0] == 0:
        return rcl, kap
    order = np.lexsort(rcl.T[::-1])
    return rcl[order], kap[order]


def job_mix(seed=3, count=24):
    rng = np.random.default_rng(seed)
    jobs = [(inputs.worked_example(), 3, 4), (inputs.complete_graph(12), 2, 4),
            (inputs.csr_from_edges(0, [], []), 1, 2), (inputs.csr_from_edges(7, [], []), 2, 3)]
    while len(jobs) < count:
        r = int(rng.integers(1, 4))
        s = r + int(rng.integers(1, 3))
        g = inputs.rmat(int(rng.integers(6, 12)), int(rng.integers(8, 17)),
                        int(rng.integers(0, 2**31)))
        jobs.append((g, r, s))
    return jobs


@pytest.mark.parametrize("workers,budget", [(4, 0), (3, 200 << 20), (2, 1)])
def test_each_result_identical_alone_and_in_the_mix(workers, budget):
    nd = _nd()
    jobs = job_mix()
    dev = [nd.to_device(g) for g, _, _ in jobs]
    alone = []
    for (g, r, s), (rp, col) in zip(jobs, dev):
        one = nd.decompose(rp, col, r, s)
        alone.append(_canon(one.rcliques.cpu().numpy(), one.kappa.cpu().numpy()))
    print(f"[serving] workers={workers} budget={budget} jobs={len(jobs)}", flush=True)
    with nd.Server(workers, budget) as sv:
        ids = [sv.submit(rp, col, r, s) for (g, r, s), (rp, col) in zip(jobs, dev)]
        # take results in reverse order so later jobs finish while earlier wait
        got = {j: sv.result(j) for j in reversed(ids)}
    for i, j in enumerate(ids):
        res = got[j].decomposition
        x = _canon(res.rcliques.cpu().numpy(), res.kappa.cpu().numpy())
        for u, v in zip(x, alone[i]):
            np.testing.assert_array_equal(u, v)
        assert got[j].queue_ms >= 0 and got[j].service_ms >= 0


def test_served_results_match_oracle():
    nd = _nd()
    jobs = job_mix(seed=11, count=10)
    dev = [nd.to_device(g) for g, _, _ in jobs]
    with nd.Server(4) as sv:
        ids = [sv.submit(rp, col, r, s) for (g, r, s), (rp, col) in zip(jobs, dev)]
        for (g, r, s), j in zip(jobs, ids):
            res = sv.result(j).decomposition
            ref = oracle.decompose(g.n, g.row_ptr, g.col, r, s)
            rc, kp = _canon(res.rcliques.cpu().numpy(), res.kappa.cpu().numpy())
            np.testing.assert_array_equal(rc, ref.rcliques)
            np.testing.assert_array_equal(kp.astype(np.uint64), ref.kappa)
            assert res.stats["n_s"] == ref.n_s


def test_failed_job_does_not_disturb_others():
    nd = _nd()
    import torch
    good = nd.to_device(inputs.complete_graph(8))
    rp = torch.tensor([0, 1, 2], dtype=torch.int64, device="cuda")
    col = torch.tensor([1, 5], dtype=torch.int32, device="cuda")  # id 5 out of range
    with nd.Server(2) as sv:
        a = sv.submit(*good, 2, 3)
        b = sv.submit(rp, col, 2, 3)
        c = sv.submit(*good, 3, 4)
        with pytest.raises(nd.NdError) as e:
            sv.result(b)
        assert e.value.name == "ND_EGRAPH"
        ra = sv.result(a).decomposition
        rc = sv.result(c).decomposition
    assert ra.rcliques.shape[0] == 28 and int(ra.kappa.max()) == 6
    assert rc.rcliques.shape[0] == 56 and int(rc.kappa.max()) == 5


def test_server_argument_errors():
    nd = _nd()
    with pytest.raises(nd.NdError):
        nd.nd_server_create(0)
    g = nd.to_device(inputs.complete_graph(4))
    with nd.Server(1) as sv:
        with pytest.raises(nd.NdError):
            sv.submit(*g, 3, 3)
        with pytest.raises(nd.NdError):
            nd.nd_server_wait(sv.handle, 12345, 0)
