"""Serving on the GPU: requests against resident layers go through the
continuous-batching scheduler (two slots, batches overlapping on two
streams); every result equals the same request run alone and the oracle,
bit-exactly."""
import numpy as np
import pytest

from gpu_helpers import log, random_cts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_14497_amd import pcmm
    pcmm.lib()
    return pcmm


def test_alone_equals_in_the_mix(dev, orc):
    import torch
    from paper_2504_14497_amd.serving import DONE, GpuExecutor, Request, Server
    rng = np.random.default_rng(12)
    n, l = 40, 3
    layers = [(rng.integers(-128, 128, size=(24, n)).astype(np.int8), 8),
              (rng.integers(-8, 8, size=(17, n)).astype(np.int8), 4),
              (rng.integers(0, 4, size=(30, n)).astype(np.uint8), 2)]
    plan = dev.Plan([(W, bits, l, dev.AFFINE, dev.cussen_cfg(4, dev.GROUP_AUTO)) for W, bits in layers])
    plan.make_resident()
    torch.cuda.synchronize()
    reqs, Xh = [], []
    for k in range(14):
        li = k % 3
        X = random_cts(orc, n, l, 1200 + k)
        Xh.append(X)
        reqs.append(Request(rid=k, layer=li, X=dev.DevPoints.from_host(X.reshape(-1, 128), n, l, 2),
                            C=dev.DevPoints.empty(layers[li][0].shape[0], l, 2, dev.AFFINE)))
    ex = GpuExecutor(plan, torch.empty(1 << 30, dtype=torch.uint8, device="cuda"), slots=2, count=len(layers))
    srv = Server(ex, budget=ex.ws.numel(), slots=2, max_batch=5)
    log("serving: submit", len(reqs))
    for r in reqs[:6]:
        srv.submit(r)
    srv.poll()                      # two batches in flight
    for r in reqs[6:]:
        srv.submit(r)               # arrive while the device is busy
    srv.drain()
    torch.cuda.synchronize()
    assert all(r.state == DONE for r in reqs)
    assert max(n_ for _, n_, _ in srv.batches) > 1
    log("serving: alone")
    ws = torch.empty(plan.selected_workspace_bytes([0]), dtype=torch.uint8, device="cuda")
    for r, X in zip(reqs, Xh):
        alone = dev.DevPoints.empty(r.C.rows, l, 2, dev.AFFINE)
        plan.run_selected([r.layer], [r.X], [alone], ws)
        torch.cuda.synchronize()
        got = r.C.to_host()
        assert (got == alone.to_host()).all(), r.rid
        assert (got == orc.pcmm_cussen(layers[r.layer][0], X)).all(), r.rid


def test_selected_runs_validate(dev, orc):
    import torch
    W = np.random.default_rng(1).integers(0, 16, size=(5, 6)).astype(np.uint8)
    plan = dev.Plan([(W, 4, 2, dev.AFFINE, None)])
    X = dev.DevPoints.from_host(random_cts(orc, 6, 2, 1300).reshape(-1, 128), 6, 2, 2)
    C = dev.DevPoints.empty(5, 2, 2, dev.AFFINE)
    ws = torch.empty(1 << 24, dtype=torch.uint8, device="cuda")
    with pytest.raises(dev.PCMMError):
        plan.run_selected([0], [X], [C], ws)      # not resident yet
    plan.make_resident()
    with pytest.raises(dev.PCMMError):
        plan.run_selected([1], [X], [C], ws)      # no such problem
    plan.run_selected([0, 0], [X, X], [C, dev.DevPoints.empty(5, 2, 2, dev.AFFINE)], ws)
    torch.cuda.synchronize()
