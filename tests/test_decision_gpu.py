"""Decision-graph summaries on the GPU (through the C ABI) against the
decision-graph oracle, on the GPU's own dpc_run / dpc_approx_run outputs (which
other tests check against the DPC oracles): top-k ids, deltas and rhos bit for
bit, the suggested delta_min and its count, and the histogram counts."""
import math
import sys

import numpy as np
import pytest

from oracle import decision_oracle as D
from paper_2207_04649_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_04649_amd import dpc as binding
    binding.lib()
    return binding


def check(dpc, rho_t, delta_t, rho_min, k, d_cut, re, de, ctx=""):
    rho, delta = rho_t.cpu().numpy(), delta_t.cpu().numpy()
    top = dpc.dpc_decision_top(rho_t, delta_t, rho_min, k)
    dmin_t, cent_t = dpc.dpc_decision_suggest(top, d_cut)
    counts = dpc.dpc_decision_histogram(rho_t, delta_t, torch.tensor(re, dtype=torch.float64, device="cuda"),
                                        torch.tensor(de, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    ids, dl, rh = D.top_delta(rho, delta, rho_min, k)
    c = int(top["count"].item())
    assert c == ids.size, ctx
    assert np.array_equal(top["ids"][:c].cpu().numpy(), ids), ctx
    assert np.array_equal(top["deltas"][:c].cpu().numpy().view(np.int64), dl.view(np.int64)), ctx
    assert np.array_equal(top["rhos"][:c].cpu().numpy(), rh), ctx
    want_dmin, want_c = D.suggest_delta_min(dl, d_cut)
    if want_dmin is None:
        assert math.isnan(float(dmin_t.item())) and int(cent_t.item()) == 0, ctx
    else:
        assert float(dmin_t.item()) == want_dmin and int(cent_t.item()) == want_c, ctx
    assert np.array_equal(counts.cpu().numpy(), D.histogram(rho, delta, re, de)), ctx
    return top, float(dmin_t.item())


def test_on_run_outputs(dpc):
    for name, approx in (("blobs_1m", False), ("blobs_1m", True), ("walks_4m", False)):
        job = getattr(inputs, name)()
        print(f"decision graph on {name} approx={approx}", flush=True)
        sys.stdout.flush()
        pts = torch.from_numpy(job.pts).cuda()
        out = (dpc.dpc_approx_run if approx else dpc.dpc_run)(pts, job.d_cut, job.rho_min, job.delta_min)
        re = [1, 2, 5, 10, 20, 50, 100, 200, 500, 1e4, 1e9]
        de = [0.0, job.d_cut / 2, job.d_cut, 2 * job.d_cut, 5 * job.d_cut, 20 * job.d_cut, 100 * job.d_cut, math.inf]
        for k in (1, 100, 4096):
            check(dpc, out["rho"], out["delta"], job.rho_min, k, job.d_cut, re, de, (name, approx, k))


def test_ties_and_edge_cases(dpc):
    rng = np.random.default_rng(8)
    n = 200000
    rho = torch.from_numpy(rng.integers(1, 6, n).astype(np.int32)).cuda()
    dl = rng.integers(0, 4, n).astype(np.float64)
    dl[[5, 9000]] = math.inf
    delta = torch.from_numpy(dl).cuda()
    for k, rho_min in ((1, 1), (333, 3), (4096, 1), (10, 6)):
        check(dpc, rho, delta, rho_min, k, 0.5, list(range(7)), [0.0, 1.0, 2.0, 3.0], (k, rho_min))
    # more bins than the per-block histogram holds
    check(dpc, rho, delta, 1, 5, 0.5, list(np.linspace(0, 6, 301)), list(np.linspace(0, 3, 41)), "wide")
    one_r = torch.tensor([3], dtype=torch.int32, device="cuda")
    one_d = torch.tensor([math.inf], dtype=torch.float64, device="cuda")
    check(dpc, one_r, one_d, 1, 4, 1.0, [0.0, 10.0], [0.0, math.inf], "single")


def test_errors(dpc):
    r = torch.ones(10, dtype=torch.int32, device="cuda")
    d = torch.ones(10, dtype=torch.float64, device="cuda")
    for k in (0, dpc.DECISION_TOP_MAX + 1):
        with pytest.raises(dpc.DpcError) as e:
            dpc.dpc_decision_top(r, d, 1, k)
        assert e.value.status == dpc.DPC_EINVAL
    with pytest.raises(dpc.DpcError) as e:
        dpc.dpc_decision_top(r, d, 1, 5, ws=torch.empty(1024, dtype=torch.uint8, device="cuda"))
    assert e.value.status == dpc.DPC_EWORKSPACE
