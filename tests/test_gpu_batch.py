"""GPU parity of the uneven batch at its real shapes: 64 Cussen PC-MMs (m, n, l
uniform in 32..512, A unsigned with bit-width uniform over 1, 2, 4, 8,
ciphertexts of uniform 8-bit messages; seed 4) compiled into one plan and run
as one table build, one persistent accumulation, one reduction and one
normalisation per phase (the plan packs the problems into phases of at most
14 GB of workspace).

Every output is a unique group element (Alg. 3 ENSURE), so the bar is bit-exact
equality of canonical affine bytes.  For every problem: the autotuned plan and
the g = 1 plan agree on all outputs; at least 8 sampled outputs (the four
corners included) equal the oracle's closed form of Eq. (ahe_5_elgamal); and one
whole output column equals the oracle's own Alg. 3 run on ciphertexts the
oracle encrypted from the same seed.
"""
import concurrent.futures as cf

import numpy as np
import pytest

from gpu_helpers import log, sample_positions
from paper_2504_14497_amd import workloads as W

pytestmark = pytest.mark.gpu

HOST_THREADS = 16
PHASE_LIMIT = 14_000_000_000  # bytes of regions per phase of a compiled plan


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_14497_amd import pcmm
    pcmm.lib()
    return pcmm


def test_uneven_batch_at_real_shapes_matches_oracle(dev, orc):
    import torch
    bw = W.batch_workload()
    assert len(bw.shapes) == 64
    As, msgs, sks, Bd = [], [], [], []
    log("batch: keygen + encrypt of", len(bw.shapes), "problems")
    for sh in bw.shapes:
        A, msg = W.make_inputs(sh)
        sk, pk = dev.keygen(sh.seed)
        As.append(A)
        msgs.append(msg)
        sks.append(int.from_bytes(sk, "big"))
        Bd.append(dev.encrypt(pk, msg, sh.seed))
    torch.cuda.synchronize()
    auto = dev.Plan([(A, sh.bits, sh.l, dev.AFFINE, dev.cussen_cfg(4, dev.GROUP_AUTO))
                     for A, sh in zip(As, bw.shapes)])
    g1 = dev.Plan([(A, sh.bits, sh.l, dev.AFFINE, dev.cussen_cfg(4, 1)) for A, sh in zip(As, bw.shapes)])
    groups = [auto.stats(k)["group"] for k in range(len(bw.shapes))]
    log("batch: autotuned groups", groups)
    # the problems' regions add up to far more than one phase may hold, so the
    # run goes in phases whose workspace is the largest phase's (plus the image)
    for plan in (auto, g1):
        total = sum(plan.stats(k)["workspace_bytes"] for k in range(len(bw.shapes)))
        assert total > PHASE_LIMIT
        assert plan.workspace_bytes() <= PHASE_LIMIT + (64 << 20), (plan.workspace_bytes(), total)
    ws = torch.empty(max(auto.workspace_bytes(), g1.workspace_bytes()), dtype=torch.uint8, device="cuda")
    log("batch: run the autotuned plan, workspace", ws.numel())
    C_auto = auto.outputs()
    auto.run(Bd, C_auto, ws)
    torch.cuda.synchronize()
    log("batch: run the g = 1 plan")
    C_g1 = g1.outputs()
    g1.run(Bd, C_g1, ws)
    torch.cuda.synchronize()
    del ws
    got = [c.to_host() for c in C_auto]
    for k in range(len(bw.shapes)):
        assert (C_g1[k].to_host() == got[k]).all(), f"problem {k}: autotuned and g = 1 plans differ"

    def closed_form(k):
        sh = bw.shapes[k]
        ii, jj = sample_positions(sh.m, sh.l, 8, sh.seed)
        want = orc.pcmm_closed_form(As[k], sh.l, sks[k], msgs[k], sh.seed, ii, jj, nthreads=1)
        return k, bool((got[k][ii, jj] == want).all()), len(ii)

    def whole_column(k):
        sh = bw.shapes[k]
        j = (7 * k) % sh.l
        _, opk = orc.keygen(sh.seed)
        B = orc.encrypt_columns(opk, msgs[k], [j], sh.seed, nthreads=1)
        want = orc.pcmm_cussen(As[k], B, cols=[j], nthreads=1)
        return k, j, bool((got[k][:, j] == want[:, j]).all())

    log("batch: oracle closed form on sampled outputs and one whole column per problem")
    with cf.ThreadPoolExecutor(HOST_THREADS) as ex:
        sampled = list(ex.map(closed_form, range(len(bw.shapes))))
        columns = list(ex.map(whole_column, range(len(bw.shapes))))
    bad = [k for k, ok, _ in sampled if not ok]
    assert not bad, f"sampled outputs differ from the closed form in problems {bad}"
    assert all(cnt >= 8 for _, _, cnt in sampled)
    bad = [(k, j) for k, j, ok in columns if not ok]
    assert not bad, f"whole columns differ from the oracle's Alg. 3 in (problem, column) {bad}"
