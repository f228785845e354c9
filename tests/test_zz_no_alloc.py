"""nd_run_noalloc: the run with the library's static device workspace, for
callers that cannot allocate.  Its outputs must equal nd_run's bit for bit
(canonical row order on both sides), on two calls in a row -- the second on
a smaller graph, over the contents the first left in the static array -- and
a plan that needs more than the static workspace is refused."""
import numpy as np
import pytest

from paper_2111_10980_amd import inputs

pytestmark = pytest.mark.gpu


def _nd():
    import paper_2111_10980_amd as nd
    return nd


def _outputs(nd, plan, r, runner):
    import torch
    n_r, ws_bytes, _ = nd.nd_plan_sizes(plan)
    rcl = torch.full((n_r, r), -1, dtype=torch.int32, device="cuda")
    kap = torch.full((n_r,), -1, dtype=torch.int32, device="cuda")
    cnt = torch.full((n_r,), -1, dtype=torch.int32, device="cuda")
    st = runner(plan, rcl, kap, cnt, ws_bytes)
    return (rcl.cpu().numpy(), kap.cpu().numpy(), cnt.cpu().numpy(), st,
            nd.nd_round_trace(plan))


def _with_nd_run(nd):
    def run(plan, rcl, kap, cnt, ws_bytes):
        return nd.nd_run(plan, nd.workspace(ws_bytes), rcl, kap, cnt, ws_bytes=ws_bytes)
    return run


def _with_noalloc(nd):
    def run(plan, rcl, kap, cnt, ws_bytes):
        assert ws_bytes <= nd.ND_NOALLOC_WORKSPACE_BYTES
        return nd.nd_run_noalloc(plan, rcl, kap, cnt)
    return run


def _compare(g, r, s):
    nd = _nd()
    import torch
    rp, col = nd.to_device(g)
    print(f"[noalloc] n={g.n} m={g.m} r={r} s={s}", flush=True)
    ref_plan = nd.nd_plan_create(rp, col, r, s, canonical=True)
    plan = nd.nd_plan_create(rp, col, r, s, canonical=True)
    try:
        want = _outputs(nd, ref_plan, r, _with_nd_run(nd))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        got = _outputs(nd, plan, r, _with_noalloc(nd))
        free1 = torch.cuda.mem_get_info()[0]
    finally:
        nd.nd_plan_destroy(ref_plan)
        nd.nd_plan_destroy(plan)
    for a, b in zip(want[:3], got[:3]):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(want[4], got[4]):
        np.testing.assert_array_equal(a, b)
    assert got[3]["n_s"] == want[3]["n_s"] and got[3]["rounds"] == want[3]["rounds"]
    # the outputs were allocated before the first reading; the run itself
    # takes no device memory (torch's allocator is untouched in between)
    print(f"[noalloc] free device memory before/after: {free0} {free1}", flush=True)
    assert free1 >= free0 - (2 << 20)


def test_noalloc_matches_nd_run_twice_second_smaller():
    """Two calls in a row on the shared static workspace, the second with a
    smaller input; (3,4) on the s = r+1 path, (2,4) on the s >= r+2 path."""
    _compare(inputs.rmat(11, 8, 61), 3, 4)
    _compare(inputs.rmat(9, 8, 62), 3, 4)
    _compare(inputs.planted_er(2000, 8.0, 3, 8, 16, 63), 2, 4)
    _compare(inputs.planted_er(300, 6.0, 2, 6, 10, 64), 2, 4)


def test_noalloc_refuses_a_plan_larger_than_the_static_workspace():
    nd = _nd()
    import torch
    g = inputs.rmat(14, 16, 65)
    rp, col = nd.to_device(g)
    plan = nd.nd_plan_create(rp, col, 3, 4)
    try:
        n_r, ws_bytes, _ = nd.nd_plan_sizes(plan)
        assert ws_bytes > nd.ND_NOALLOC_WORKSPACE_BYTES
        rcl = torch.empty((n_r, 3), dtype=torch.int32, device="cuda")
        kap = torch.empty((n_r,), dtype=torch.int32, device="cuda")
        with pytest.raises(nd.NdError) as e:
            nd.nd_run_noalloc(plan, rcl, kap)
        assert e.value.name == "ND_ENOMEM"
    finally:
        nd.nd_plan_destroy(plan)
