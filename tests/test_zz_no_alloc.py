"""pcmm_cussen_static: the Cussen PC-MM whose workspace is the library's static
device array (for callers that cannot allocate device memory).

On the GPU its output must equal pcmm_cussen's byte for byte (and the
oracle's), on two calls in a row whose second problem is smaller, so the
second call runs on a scratch that still holds the first call's contents.
On the CPU: a problem larger than the array is refused before any device call.
"""
import ctypes

import numpy as np
import pytest

from gpu_helpers import log, random_cts
from paper_2504_14497_amd import pcmm, workloads as W


def test_static_scratch_refuses_oversized_problem():
    # 512 x 512 x 512 at 4 bits needs far more than the static array; the
    # matrices' device pointers are never touched (nothing is queued)
    A = np.random.default_rng(7).integers(0, 16, (512, 512)).astype(np.uint8)
    ws = pcmm.cussen_workspace_bytes(A, 4, 512, pcmm.AFFINE, None)
    assert ws > pcmm.STATIC_SCRATCH_BYTES
    ld = 512 * 512
    B = pcmm.Mat(512, 512, 2, pcmm.AFFINE, ld, 0x1000)
    C = pcmm.Mat(512, 512, 2, pcmm.AFFINE, ld, 0x2000)
    rc = pcmm.lib().pcmm_cussen_static(A.ctypes.data_as(ctypes.c_void_p), 512, 512, 4, 0, ctypes.byref(B),
                                       ctypes.byref(C), None, None, None)
    assert rc == -6  # PCMM_ETOOLARGE
    assert "static scratch" in pcmm.strerror(-6)


@pytest.mark.gpu
def test_static_scratch_equals_workspace_call(orc):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pcmm.lib()
    # the second call's problem is smaller than the first's
    shapes = [W.PCMMShape(70, 45, 21, 4, False, 4, seed=401),
              W.PCMMShape(16, 16, 16, 4, True, 4, seed=402)]
    for rep, sh in enumerate(shapes):
        A, _ = W.make_inputs(sh)
        B = random_cts(orc, sh.n, sh.l, 500 + rep)
        ws = pcmm.cussen_workspace_bytes(A, sh.bits, sh.l, pcmm.AFFINE, None)
        assert ws <= pcmm.STATIC_SCRATCH_BYTES
        log("static scratch call", rep, sh, "workspace", ws)
        Bd = pcmm.DevPoints.from_host(B.reshape(-1, 128), sh.n, sh.l, 2)
        Cs, st_s = pcmm.cussen_static(A, sh.bits, Bd)
        got = Cs.to_host()
        Cw, st_w = pcmm.cussen(A, sh.bits, Bd)
        torch.cuda.synchronize()
        want = Cw.to_host()
        assert (got == want).all(), f"call {rep}: static-scratch output differs from pcmm_cussen"
        assert (want == orc.pcmm_cussen(A, B)).all(), f"call {rep}: pcmm_cussen differs from the oracle"
        assert st_s["accum_adds"] == st_w["accum_adds"] and st_s["group"] == st_w["group"]
