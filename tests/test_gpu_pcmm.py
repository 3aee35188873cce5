"""GPU parity of PC-MM: schoolbook (Sec. 3.1) and Cussen (Alg. 3 with Alg. 2).

Every output is a unique group element, so the bar is bit-exact equality of
the canonical affine bytes.  Small and ragged shapes are compared element by
element with the oracle's PC-MM on oracle-made inputs; the full-size workloads
(in the launch configuration the benchmark uses) are compared on sampled
outputs with the oracle's closed form of Eq. (ahe_5_elgamal), with every output
also checked between the two GPU methods, and by decryption.
"""
import numpy as np
import pytest

from gpu_helpers import log, random_cts, sample_positions
from paper_2504_14497_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_14497_amd import pcmm
    pcmm.lib()
    return pcmm


def _upload(dev, B):
    n, l, _ = B.shape
    return dev.DevPoints.from_host(B.reshape(-1, 128), n, l, 2)


def _run_both(dev, A, bits, Bd, cfg=None):
    Cs = dev.schoolbook(A, bits, Bd).to_host()
    Cc, st = dev.cussen(A, bits, Bd, cfg=cfg)
    return Cs, Cc.to_host(), st


def test_tiny_workload_vs_oracle(dev, orc):
    sh = W.TINY
    A, msg = W.make_inputs(sh)
    sk, pk = orc.keygen(sh.seed)
    B = orc.encrypt(pk, msg, sh.seed)
    log("tiny", sh)
    Cs, Cc, st = _run_both(dev, A, sh.bits, _upload(dev, B))
    want = orc.pcmm_cussen(A, B)
    assert (want == orc.pcmm_schoolbook(A, B)).all()
    assert (Cs == want).all()
    assert (Cc == want).all()
    assert st["level_mults"] > 0


RAGGED = [
    W.PCMMShape(1, 1, 1, 4, False, 4, seed=101),
    W.PCMMShape(3, 5, 7, 3, False, 4, seed=102),
    W.PCMMShape(65, 33, 17, 4, False, 4, seed=103),
    W.PCMMShape(20, 30, 10, 8, True, 8, seed=104),
    W.PCMMShape(130, 9, 3, 2, False, 4, seed=105),
    W.PCMMShape(7, 70, 2, 1, False, 4, seed=106),
    W.PCMMShape(40, 12, 33, 8, False, 8, seed=107),
]


@pytest.mark.parametrize("sh", RAGGED, ids=lambda s: f"{s.m}x{s.n}x{s.l}_t{s.bits}{'s' if s.signed else 'u'}")
def test_ragged_shapes_vs_oracle(dev, orc, sh):
    A, _ = W.make_inputs(sh)
    B = random_cts(orc, sh.n, sh.l, sh.seed)
    log("ragged", sh)
    Cs, Cc, _ = _run_both(dev, A, sh.bits, _upload(dev, B))
    want = orc.pcmm_cussen(A, B)
    assert (Cs == want).all()
    assert (Cc == want).all()


@pytest.mark.parametrize("group", [1, 2, 3, 4])
@pytest.mark.parametrize("rounds", [1, 2, 4])
def test_cussen_configurations_vs_oracle(dev, orc, group, rounds):
    rng = np.random.default_rng(group * 10 + rounds)
    B = random_cts(orc, 24, 6, 200)
    want = {}
    for name, A, bits in (("u4", rng.integers(0, 16, size=(40, 24)).astype(np.uint8), 4),
                          ("s3", rng.integers(-4, 4, size=(40, 24)).astype(np.int8), 3)):
        ref = orc.pcmm_cussen(A, B)
        Bd = _upload(dev, B)
        for split in (1, 2, 4):
            cfg = dev.CussenCfg(rounds, group, split, 0)
            log("cfg", name, group, rounds, split)
            C, st = dev.cussen(A, bits, Bd, cfg=cfg)
            assert (C.to_host() == ref).all(), (name, group, rounds, split)
        # small LDS chunks (one group staged at a time)
        C, _ = dev.cussen(A, bits, Bd, cfg=dev.CussenCfg(rounds, group, 2, 1))
        assert (C.to_host() == ref).all()


@pytest.mark.parametrize("split", [8, 16, 64])
def test_deep_split_k_vs_oracle(dev, orc, split):
    """Split-k with several partial sums per reduction lane (the reduction
    adds partials sequentially before its shuffle tree), more splits than
    column groups on some of them, signed codes."""
    rng = np.random.default_rng(split)
    B = random_cts(orc, 70, 3, 210)
    A = rng.integers(-8, 8, size=(9, 70)).astype(np.int8)
    ref = orc.pcmm_cussen(A, B)
    Bd = _upload(dev, B)
    for group in (1, 2):
        log("split", split, "group", group)
        C, st = dev.cussen(A, 4, Bd, cfg=dev.CussenCfg(4, group, split, 0))
        assert st["k_split"] == split
        assert (C.to_host() == ref).all(), (split, group)


@pytest.mark.parametrize("bits,signed", [(12, True), (16, False), (16, True), (9, False)])
def test_wide_plaintexts_vs_oracle(dev, orc, bits, signed):
    """9..16-bit plaintexts (16-bit arrays): schoolbook and Cussen (g = 1..3)
    equal the oracle; the vector case n = l = 1 too."""
    rng = np.random.default_rng(bits * 2 + signed)
    lo, hi = (-(1 << (bits - 1)), 1 << (bits - 1)) if signed else (0, 1 << bits)
    dt = np.int16 if signed else np.uint16
    A = rng.integers(lo, hi, size=(70, 9)).astype(dt)
    A[3, :] = hi - 1  # the extreme value and repeats down a column
    A[5, :] = lo
    B = random_cts(orc, 9, 3, 900 + bits)
    ref = orc.pcmm_cussen(A, B)
    Bd = _upload(dev, B)
    log("wide", bits, signed)
    assert (dev.schoolbook(A, bits, Bd).to_host() == ref).all()
    for group in (1, 2, 3):
        C, st = dev.cussen(A, bits, Bd, cfg=dev.CussenCfg(4, group, 0, 0))
        assert (C.to_host() == ref).all(), group
    v = A[:, :1].copy()
    Bv = _upload(dev, B[:1, :1].copy())
    C, _ = dev.cussen(v, bits, Bv)
    assert (C.to_host() == orc.pcmm_cussen(v, B[:1, :1].copy())).all()


def test_exceptional_cases_vs_oracle(dev, orc):
    # equal ciphertexts down a column (accumulator meets P = Q, tables meet
    # P = Q through repeated differences), opposite ones (P = -Q) and an
    # identity point in B
    B = random_cts(orc, 6, 3, 300)
    B[1] = B[0]
    B[3] = B[0]
    for j in range(3):
        for h in range(2):
            P_ = bytes(B[0, j, 64 * h:64 * h + 64])
            B[2, j, 64 * h:64 * h + 64] = np.frombuffer(orc.pt_neg(P_), dtype=np.uint8)
    B[5, 1] = 0  # an infinity point inside B
    A = np.array([[1, 1, 0, 0, 0, 2], [1, 0, 1, 0, 3, 0], [3, 3, 6, 1, 0, 1], [2, 0, 2, 5, 1, 1],
                  [1, 2, 3, 4, 5, 6], [7, 7, 7, 7, 7, 7], [-1, 1, 1, -1, 2, -2], [0, 0, 0, 0, 0, 0],
                  # an identity accumulator meets an identity entry (column 1: 3 B[5] is
                  # the identity), first from the start, then after P + (-P)
                  [0, 0, 0, 0, 0, 3], [1, 0, 1, 0, 0, 1], [1, 0, 1, 0, 0, -2]],
                 dtype=np.int8)
    want = orc.pcmm_cussen(A, B)
    Bd = _upload(dev, B)
    log("exceptional")
    Cs, Cc, _ = _run_both(dev, A, 4, Bd)
    assert (Cs == want).all()
    assert (Cc == want).all()
    for g in (2, 3):
        C, _ = dev.cussen(A, 4, Bd, cfg=dev.CussenCfg(4, g, 2, 0))
        assert (C.to_host() == want).all()
    assert (want[7] == 0).all()
    assert (want[8:11, 1] == 0).all()


def test_combination_lanes_sharing_an_inversion(dev, orc):
    """The combinations' backward pass gives a thread two (group, pair)
    lanes, t and t + H (H = half the lanes in whole wavefronts), which share
    one inversion.  With 2 groups of 80 pairs (160 lanes, H = 128) the lanes
    of group 1's pairs 48..79 share threads with group 0's pairs 0..31.
    Group 1's columns hold equal ciphertexts (B row 3 = row 2), so its equal
    digits meet x_a = x_b: those lanes take the checked passes and the third
    pass while their partners in group 0 take the fast path.  Equal to the
    oracle everywhere."""
    rng = np.random.default_rng(123)
    A = rng.integers(0, 16, size=(20, 4)).astype(np.uint8)
    A[:6, 2] = A[:6, 3]           # equal digits in group 1: chords with x_a = x_b
    A[6, 2:] = [5, 5]
    B = random_cts(orc, 4, 40, 456)
    B[3] = B[2]
    want = orc.pcmm_cussen(A, B)
    Bd = _upload(dev, B)
    log("combination lanes sharing an inversion")
    C, st = dev.cussen(A, 4, Bd, cfg=dev.CussenCfg(4, 2, 1, 0))
    assert st["group"] == 2 and st["combo_adds"] > 0
    assert (C.to_host() == want).all()


@pytest.mark.parametrize("m,n,l,bits,signed,g", [(50, 1, 5, 8, True, 1), (40, 2, 3, 4, False, 2),
                                                 (33, 3, 2, 2, False, 3), (20, 1, 4, 4, False, 1)])
def test_direct_outputs_of_one_column_group(dev, orc, m, n, l, bits, signed, g):
    """n <= g: every row has at most one code, so each affine output is its
    table entry written directly (no accumulation additions, no
    normalisation).  Zero rows give the identity, one ciphertext of B is the
    identity, and the table's combinations (g > 1) feed the outputs.  Equal
    to the oracle on every output, and to the Jacobian-output path (which
    accumulates and leaves normalisation to the caller)."""
    rng = np.random.default_rng(91 + m)
    lo, hi = (-(1 << (bits - 1)), 1 << (bits - 1)) if signed else (0, 1 << bits)
    A = rng.integers(lo, hi, size=(m, n)).astype(np.int8 if signed else np.uint8)
    A[3] = 0          # a zero row: identity outputs
    A[5] = A[4]       # repeated rows share a table entry
    B = random_cts(orc, n, l, 300 + m)
    B[0, l - 1] = 0   # an identity ciphertext
    want = orc.pcmm_cussen(A, B)
    Bd = _upload(dev, B)
    C, st = dev.cussen(A, bits, Bd, cfg=dev.CussenCfg(4, g, 1, 0))
    assert st["group"] == g and st["k_split"] == 1, st
    assert (C.to_host() == want).all()
    Cj, _ = dev.cussen(A, bits, Bd, c_form=dev.JACOBIAN, cfg=dev.CussenCfg(4, g, 1, 0))
    assert (dev.normalize(Cj).to_host() == want).all()
    assert (want[3] == 0).all()


def test_degenerate_sizes(dev, orc):
    B = random_cts(orc, 3, 4, 400)
    Bd = _upload(dev, B)
    log("degenerate")
    # zero rows
    C, _ = dev.cussen(np.zeros((0, 3), np.uint8), 4, Bd)
    assert C.to_host().shape == (0, 4, 128)
    # A = 0 -> every output is the identity
    for method in ("schoolbook", "cussen"):
        A = np.zeros((5, 3), np.uint8)
        out = dev.schoolbook(A, 4, Bd) if method == "schoolbook" else dev.cussen(A, 4, Bd)[0]
        assert (out.to_host() == 0).all()
    # empty inner dimension
    B0 = dev.DevPoints.empty(0, 4, 2, dev.AFFINE)
    C, _ = dev.cussen(np.zeros((2, 0), np.uint8), 4, B0)
    assert (C.to_host() == 0).all()
    # the identity matrix returns B; A = e_i e_k^T picks one ciphertext
    I = np.eye(3, dtype=np.uint8)
    C, _ = dev.cussen(I, 1, Bd)
    assert (C.to_host() == B).all()
    E = np.zeros((4, 3), np.uint8)
    E[2, 1] = 1
    C = dev.cussen(E, 1, Bd)[0].to_host()
    assert (C[2] == B[1]).all() and (C[[0, 1, 3]] == 0).all()


def test_caller_stage_events(dev, orc):
    """Stage events handed in by the caller are recorded (also on the paths
    that launch no stage pipeline) and do not change the result."""
    import torch
    B = random_cts(orc, 6, 5, 600)
    Bd = _upload(dev, B)
    A = np.random.default_rng(6).integers(0, 16, size=(7, 6), dtype=np.uint8)
    stream = torch.cuda.current_stream()
    log("stage events")
    for A_, Bd_ in ((A, Bd), (np.zeros((2, 0), np.uint8), dev.DevPoints.empty(0, 5, 2, dev.AFFINE)),
                    (np.zeros((0, 6), np.uint8), Bd)):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(dev.STAGE_EVENTS)]
        for e in evs:
            e.record(stream)
        torch.cuda.synchronize()
        C, _ = dev.cussen(A_, 4, Bd_, cfg=dev.cussen_cfg(4, 1, stage_events=evs))
        torch.cuda.synchronize()
        if A_.size:
            assert (C.to_host() == orc.pcmm_cussen(A_, B)).all()
        dts = [evs[i].elapsed_time(evs[i + 1]) for i in range(dev.STAGE_EVENTS - 1)]
        assert all(d >= 0 for d in dts)
        assert abs(sum(dts) - evs[0].elapsed_time(evs[-1])) < 1e-2
    with pytest.raises(ValueError):
        dev.cussen_cfg(4, 1, stage_events=evs[:3])


def test_out_of_range_is_rejected(dev, orc):
    B = random_cts(orc, 2, 2, 500)
    Bd = _upload(dev, B)
    with pytest.raises(dev.PCMMError) as ei:
        dev.cussen(np.array([[16, 0]], np.uint8), 4, Bd)
    assert ei.value.code == -2
    with pytest.raises(dev.PCMMError) as ei:
        dev.schoolbook(np.array([[-3, 0]], np.int8), 2, Bd)
    assert ei.value.code == -2


def _full_size(dev, orc, sh, cfg=None, n_samples=24, check_schoolbook=True, whole_columns=(0, -1)):
    """The benchmark's path: GPU keygen + encrypt from the seed, Cussen with the
    default (autotuned-free) configuration, canonical affine output.  Sampled
    outputs are compared with the oracle's closed form and the columns
    `whole_columns` (negative: from the end) with the oracle's own Alg. 3 on
    ciphertexts it encrypted from the same seed."""
    import torch
    A, msg = W.make_inputs(sh)
    log("full size", sh.name, "keygen+encrypt")
    sk, pk = dev.keygen(sh.seed)
    Bd = dev.encrypt(pk, msg, sh.seed)
    log("full size", sh.name, "cussen")
    Cc, st = dev.cussen(A, sh.bits, Bd, cfg=cfg)
    torch.cuda.synchronize()
    C = Cc.to_host()
    ii, jj = sample_positions(sh.m, sh.l, n_samples, sh.seed)
    osk = int.from_bytes(sk, "big")
    log("full size", sh.name, "closed form on", len(ii), "outputs")
    want = orc.pcmm_closed_form(A, sh.l, osk, msg, sh.seed, ii, jj)
    got = C[ii, jj]
    assert (got == want).all()
    cols = sorted({j % sh.l for j in whole_columns})
    if cols:
        log("full size", sh.name, "oracle Alg. 3 on whole columns", cols)
        _, opk = orc.keygen(sh.seed)
        Bo = orc.encrypt_columns(opk, msg, cols, sh.seed)
        Co = orc.pcmm_cussen(A, Bo, cols=cols)
        assert (C[:, cols] == Co[:, cols]).all()
    # decryption of the sampled outputs gives (A.B) G
    AB = A.astype(np.int64) @ msg.astype(np.int64)
    p_, b_, gx, gy, q = orc.curve_params()
    G = orc.generator()
    M = dev.decrypt_to_points(sk, Cc).to_host()
    for i, j in list(zip(ii, jj))[:6]:
        assert bytes(M[i, j]) == orc.ladder_big(int(AB[i, j]) % q, G)
    if check_schoolbook:
        log("full size", sh.name, "schoolbook")
        Cs = dev.schoolbook(A, sh.bits, Bd).to_host()
        assert (Cs == C).all()
    return st


def test_full_size_large_t4(dev, orc):
    st = _full_size(dev, orc, W.LARGE_T4)
    assert st["accum_adds"] == int(np.count_nonzero(W.make_inputs(W.LARGE_T4)[0]))


def test_full_size_large_t2(dev, orc):
    _full_size(dev, orc, W.LARGE_T2, check_schoolbook=False)
    _full_size(dev, orc, W.LARGE_T2, cfg=dev_cfg(3), n_samples=8, check_schoolbook=False, whole_columns=(5,))


def dev_cfg(group):
    from paper_2504_14497_amd import pcmm
    return pcmm.CussenCfg(4, group, 0, 0)


def test_full_size_signed128(dev, orc):
    _full_size(dev, orc, W.SIGNED128)
    _full_size(dev, orc, W.SIGNED128, cfg=dev_cfg(2), n_samples=8, check_schoolbook=False, whole_columns=(5,))


def test_full_size_serve_layer(dev, orc):
    # 256 x 1024 times 1024 x 8: the split-k path with the wavefront reduction
    _full_size(dev, orc, W.SERVE_LAYER, n_samples=12, check_schoolbook=False)


def test_long_inner_dimension_in_one_split(dev, orc):
    """n = 40000 columns with the inner dimension unsplit: one split holds more
    column groups than a code list may (its group index is kept in 15 bits),
    so the accumulation walks two lists; Cussen equals schoolbook and the
    closed form on every output."""
    from paper_2504_14497_amd import pcmm
    sh = W.PCMMShape(m=3, n=40000, l=2, bits=2, signed=False, msg_bits=4, seed=57, name="long_n")
    _full_size(dev, orc, sh, cfg=pcmm.CussenCfg(4, 1, 1, 0), n_samples=6, whole_columns=())


@pytest.mark.parametrize("m,l,bits,signed,coop", [(300, 1, 8, False, True), (257, 2, 12, True, True),
                                                  (200, 1, 16, False, True), (130, 4, 8, True, True),
                                                  (97, 1, 4, False, True), (97, 1, 1, False, False)])
def test_narrow_tables_built_cooperatively(dev, orc, m, l, bits, signed, coop):
    """Few output columns: the run pads its groups to whole wavefronts, and
    W <= 64 lanes share each level-1 chain (ragged blocks, each started by a
    ladder to its first entry) where a cost model of chain depth and
    wavefronts per SIMD prefers it; the 1-bit case (one entry, no chain)
    keeps one lane per chain in the padded build.  Cussen equals schoolbook and the
    closed form on every output."""
    from paper_2504_14497_amd import pcmm
    sh = W.PCMMShape(m=m, n=3, l=l, bits=bits, signed=signed, msg_bits=8, seed=61 + m, name="narrow")
    st = _full_size(dev, orc, sh, cfg=pcmm.CussenCfg(4, 1, 0, 0), n_samples=m * l, whole_columns=())
    if coop:
        assert 2 <= st["coop_lanes"] <= 64, st
    else:
        assert st["coop_lanes"] == 0, st
