"""GPU parity of compiled plans (pcmm_plan_*): several uneven Cussen PC-MMs
run together (one table build, one persistent accumulation, one reduction,
one normalisation) equal the oracle bit-exactly; a plan runs again on fresh
ciphertexts; a run captured into a hipGraph replays bit-exactly; the
autotuner's choice is reported and gives the same group elements."""
import numpy as np
import pytest

from gpu_helpers import log, random_cts

pytestmark = pytest.mark.gpu

AFF, JAC = 2, 3


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_14497_amd import pcmm
    pcmm.lib()
    return pcmm


# (m, n, l, bits, signed, group, k_split, c_form)
PROBLEMS = [
    (7, 5, 3, 4, False, 1, 0, AFF),
    (33, 17, 9, 2, False, 2, 0, AFF),
    (1, 1, 1, 8, True, 1, 0, AFF),
    (16, 40, 6, 8, False, -1, 0, JAC),     # autotuned group, Jacobian output
    (5, 0, 4, 4, False, 1, 0, AFF),        # empty inner dimension: identity outputs
    (0, 5, 4, 4, False, 1, 0, AFF),        # no rows
    (70, 9, 2, 1, False, 3, 0, AFF),
    (12, 33, 5, 8, True, 2, 4, AFF),       # signed, split-k
    (130, 20, 3, 4, True, -1, 2, AFF),
]


def _make(dev, orc, problems, seed):
    rng = np.random.default_rng(seed)
    spec, Bh, Bd = [], [], []
    for k, (m, n, l, bits, signed, g, split, form) in enumerate(problems):
        if signed:
            A = rng.integers(-(1 << (bits - 1)), 1 << (bits - 1), size=(m, n)).astype(np.int8)
        else:
            A = rng.integers(0, 1 << bits, size=(m, n)).astype(np.uint8)
        B = random_cts(orc, n, l, seed * 100 + k) if n * l else np.zeros((n, l, 128), np.uint8)
        Bh.append(B)
        Bd.append(dev.DevPoints.from_host(B.reshape(-1, 128), n, l, 2) if n * l
                  else dev.DevPoints.empty(n, l, 2, dev.AFFINE))
        spec.append((A, bits, l, form, dev.cussen_cfg(4, g, split)))
    return spec, Bh, Bd


def _affine(dev, C, form):
    return (dev.normalize(C) if form == JAC else C).to_host()


def _expected(orc, A, B, m, l):
    if m * l == 0:
        return np.zeros((m, l, 128), np.uint8)
    if A.shape[1] == 0:
        return np.zeros((m, l, 128), np.uint8)
    return orc.pcmm_cussen(A, B)


def test_plan_of_uneven_problems_matches_oracle(dev, orc):
    import torch
    spec, Bh, Bd = _make(dev, orc, PROBLEMS, 3)
    log("plan: create", len(spec), "problems")
    plan = dev.Plan(spec)
    for i, (A, bits, l, form, cfg) in enumerate(spec):
        st = plan.stats(i)
        assert 1 <= st["group"] <= 4
        if PROBLEMS[i][5] > 0:
            assert st["group"] == PROBLEMS[i][5]
    for rnd in range(2):
        if rnd == 1:  # the same plan on fresh ciphertexts
            _, Bh, Bd = _make(dev, orc, PROBLEMS, 4)
        log("plan: run", rnd)
        C = plan.run(Bd)
        torch.cuda.synchronize()
        for i, (A, bits, l, form, cfg) in enumerate(spec):
            m = A.shape[0]
            got = _affine(dev, C[i], form)
            want = _expected(orc, A, Bh[i], m, l)
            assert (got == want).all(), (rnd, i, PROBLEMS[i])
    plan.close()


def test_plan_equals_single_calls(dev, orc):
    """The batched run and per-problem pcmm_cussen calls give the same bytes."""
    import torch
    probs = [(40, 64, 7, 4, False, 1, 0, AFF), (64, 31, 10, 8, True, 1, 0, AFF), (9, 70, 3, 2, False, 2, 0, AFF)]
    spec, Bh, Bd = _make(dev, orc, probs, 5)
    plan = dev.Plan(spec)
    C = plan.run(Bd)
    for i, (A, bits, l, form, cfg) in enumerate(spec):
        Cs, _ = dev.cussen(A, bits, Bd[i], cfg=cfg)
        torch.cuda.synchronize()
        assert (Cs.to_host() == C[i].to_host()).all(), i


def test_plan_run_in_hip_graph_replays(dev, orc):
    import torch
    probs = [(20, 12, 5, 4, False, 1, 0, AFF), (8, 30, 4, 8, True, 2, 2, AFF), (50, 7, 3, 1, False, 1, 0, AFF)]
    spec, Bh, Bd = _make(dev, orc, probs, 6)
    plan = dev.Plan(spec)
    ws = torch.empty(plan.workspace_bytes(), dtype=torch.uint8, device="cuda")
    C = plan.outputs()
    plan.run(Bd, C, ws)
    torch.cuda.synchronize()
    ref = [c.to_host() for c in C]
    want = [_expected(orc, s[0], Bh[i], s[0].shape[0], s[2]) for i, s in enumerate(spec)]
    assert all((r == w).all() for r, w in zip(ref, want))
    log("plan: capture")
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            plan.run(Bd, C, ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    other_spec, _, other_Bd = _make(dev, orc, [(6, 6, 6, 4, False, 1, 0, AFF)], 7)
    other = dev.Plan(other_spec)
    for r in range(3):
        for c in C:
            c.t.zero_()
        other.run(other_Bd)          # eager work on the same device between replays
        torch.cuda.synchronize()
        log("plan: replay", r)
        g.replay()
        torch.cuda.synchronize()
        for i, c in enumerate(C):
            assert (c.to_host() == ref[i]).all(), (r, i)


def test_autotuned_group_gives_same_result(dev, orc):
    import torch
    rng = np.random.default_rng(8)
    A = rng.integers(0, 4, size=(96, 48)).astype(np.uint8)
    B = random_cts(orc, 48, 4, 800)
    Bd = dev.DevPoints.from_host(B.reshape(-1, 128), 48, 4, 2)
    C1, st1 = dev.cussen(A, 2, Bd, cfg=dev.cussen_cfg(4, 1))
    Ca, sta = dev.cussen(A, 2, Bd, cfg=dev.cussen_cfg(4, dev.GROUP_AUTO))
    torch.cuda.synchronize()
    assert st1["group"] == 1 and 1 <= sta["group"] <= 4
    assert (C1.to_host() == Ca.to_host()).all()
    assert (Ca.to_host() == orc.pcmm_cussen(A, B)).all()


def test_plan_rejects_bad_runs(dev, orc):
    spec, Bh, Bd = _make(dev, orc, [(4, 3, 2, 4, False, 1, 0, AFF)], 9)
    plan = dev.Plan(spec)
    wrong = dev.DevPoints.empty(3, 5, 2, dev.AFFINE)  # l mismatch
    with pytest.raises(dev.PCMMError):
        plan.run([wrong])
    with pytest.raises(ValueError):
        plan.run(Bd + Bd)
    import torch
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(dev.PCMMError) as ei:
        plan.run(Bd, workspace=small)
    assert ei.value.code == -3
