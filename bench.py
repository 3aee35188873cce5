#!/usr/bin/env python3
"""Benchmark: PC-MM/s and point-additions/s of Cussen PC-MM on one MI355X.

Workload (default): A 512 x 512 uniform unsigned 4-bit, B 512 x 512 EC-ElGamal
ciphertexts on P-256 of uniform 4-bit messages (seeded, synthetic).  One step
is one complete PC-MM by Cussen's method (Alg. 3 with Alg. 2, N = 4 rounds,
one column of A per compression): the host compression plan, its upload, the
table build with batched inversion, the gather-and-add accumulation and the
affine normalisation of C, with A on the host and B already resident in HBM.
The schoolbook method (Sec. 3.1) runs on the same inputs for the speedup.

Prints one JSON line.  `--gpus N` with N > 1 is refused: the benchmark runs
on one GPU (the design of a sharded run is documented separately).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PC-MM/s + point-adds/s at 512x512 4-bit; Cussen vs schoolbook, batched vs single"

# MI355X figures used for the roofline (the path is bound by 32-bit VALU work):
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane-ops/s; the
# 32x32 -> 64-bit multiply-add issues at full rate on gfx950 (measured by the
# probe in the diagnostics), so the INT32 multiply-add peak is the same figure.
PEAK_INT32_MAD = 256 * 64 * 2.4e9
HBM_PEAK_GBS = 8000.0

# algorithmic 32x32 multiply-adds of the textbook 8 x 32-bit field operations:
# a product is 64, a square 36 (the 28 cross products counted once); the P-256
# Montgomery reduction needs none (its digits of p are 0, 1 and 2^32 - 1)
MADS_MUL, MADS_SQR = 64, 36
MADS_MIXED_ADD = 8 * MADS_MUL + 2 * MADS_SQR        # 584 (XYZZ madd-2008-s, 8M + 2S)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the kernels' code (fp.hpp, ec.hpp, common.hpp, k_cussen.hip)
    with // comments and whitespace removed, so that edits of comments alone
    keep counters taken on the same code valid."""
    import re
    h = hashlib.sha256()
    for f in ("fp.hpp", "ec.hpp", "common.hpp", "k_cussen.hip"):
        with open(os.path.join(ROOT, "paper_2504_14497_amd", "csrc", f), encoding="utf-8") as fh:
            code = re.sub(r"//[^\n]*", "", fh.read())
        h.update("".join(code.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(workload):
    """HBM bytes per launch of the accumulation kernel from the committed
    counter summary, or None if missing or taken on different kernel source."""
    path = os.path.join(ROOT, "profiles", f"accumulate_{workload}_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def load_table_traffic(workload):
    """HBM bytes of one table stage (digit tables and combinations) from the
    committed counter summary, or None if missing or taken on other source."""
    path = os.path.join(ROOT, "profiles", f"table_{workload}_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_run")


def cpu_baseline(sh, A, target_seconds, threads):
    """The CPU oracle's Cussen PC-MM on a bounded sample of output columns.

    The sample's ciphertexts are encrypted by the oracle itself (same seed and
    nonce indices as the full matrix), so the sampled columns of the GPU
    result can be compared with it."""
    import oracle
    from paper_2504_14497_amd import workloads as W
    _, msg = W.make_inputs(sh)
    sk, pk = oracle.keygen(sh.seed)
    t0 = time.time()
    B = oracle.encrypt_columns(pk, msg, [0], sh.seed, nthreads=threads)
    t_enc = time.time() - t0
    t0 = time.time()
    oracle.pcmm_cussen(A, B, cols=[0], nthreads=1)
    t_one = time.time() - t0
    ncols = int(target_seconds / max(t_one, 1e-3) * threads)
    ncols = max(1, min(sh.l, (ncols // threads) * threads if ncols >= threads else ncols))
    cols = list(range(ncols))
    log(f"cpu baseline: one column {t_one:.2f} s, its encryption {t_enc:.2f} s; "
        f"sampling {ncols} columns on {threads} threads")
    B = oracle.encrypt_columns(pk, msg, cols, sh.seed, nthreads=threads)
    t0 = time.time()
    C = oracle.pcmm_cussen(A, B, cols=cols, nthreads=threads)
    dt = time.time() - t0
    return {"value": (ncols / sh.l) / dt, "unit": "PC-MM/s", "cores": threads, "kind": "oracle",
            "sample": f"{ncols} of {sh.l} output columns of the same workload (all {sh.m} rows, both "
                      f"points, compression of all {sh.n} columns of A), scaled by {sh.l}/{ncols}; "
                      f"{dt:.1f} s wall on {threads} threads",
            "threads": threads, "nproc": os.cpu_count(), "physical_cores": physical_cores(),
            "cpu_model": cpu_model(),
            "one_thread_pcmm_per_s": 1.0 / (t_one * sh.l),
            "one_thread_sample": f"output column 0 alone on one thread ({t_one:.2f} s), scaled by {sh.l}",
            "thread_cap": "the oracle runs at most 16 threads, the host CPU share of one GPU"}, C, cols


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def physical_cores():
    """Distinct (physical id, core id) pairs in /proc/cpuinfo, or None."""
    try:
        cores, phys = set(), None
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("physical id"):
                    phys = line.split(":", 1)[1].strip()
                elif line.startswith("core id"):
                    cores.add((phys, line.split(":", 1)[1].strip()))
        return len(cores) or None
    except OSError:
        return None


def time_region(fn, reps, stream):
    """Mean ms per call of fn() over `reps` back-to-back calls on `stream`."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


# issued 32x32 -> 64-bit multiply-adds of one product in the library's field
# form (nine 29-bit limbs): 81 partial products + 4 per quotient digit of the
# Montgomery reduction (9 digits)
ISSUED_MADS_MUL = 81 + 4 * 9


def field_mul_leg(blocks=2048):
    """Field-multiplication throughput (one dependent chain of products per
    lane, 8 wavefronts per SIMD) and the issue rates of single instructions
    (8 independent chains per lane), from the library's probe kernels."""
    from paper_2504_14497_amd import pcmm
    kinds = {"v_mad_u64_u32": (0, 4000), "v_add3_u32": (1, 4000), "v_xor_b32": (5, 4000),
             "v_fma_f64": (4, 4000), "fe_mul": (2, 2000), "mixed_add": (3, 200)}
    rates = {}
    for name, (kind, iters) in kinds.items():
        pcmm.diag_probe(kind, iters // 10, blocks)  # warm-up
        sec, ops = pcmm.diag_probe(kind, iters, blocks)
        rates[name] = ops / sec
    peak = PEAK_INT32_MAD
    mad_rate = rates["v_mad_u64_u32"]
    fe = rates["fe_mul"]
    return {"what": "probe kernels, 2048 workgroups x 256 lanes; fe_mul: x = x * y mod p in the library's "
                    "Montgomery form, one dependent chain per lane; instruction rates: 8 independent chains "
                    "per lane, lane-dependent operands",
            "fe_mul_per_s": fe,
            "algorithmic_mads_per_mul": MADS_MUL, "issued_mads_per_mul": ISSUED_MADS_MUL,
            "algorithmic_tops": fe * MADS_MUL / 1e12,
            "frac_of_peak": fe * MADS_MUL / peak,
            "frac_of_measured_mad_rate": fe * MADS_MUL / mad_rate,
            "issued_mad_frac_of_measured_mad_rate": fe * ISSUED_MADS_MUL / mad_rate,
            "mixed_adds_per_s": rates["mixed_add"],
            "mixed_add_frac_of_peak": rates["mixed_add"] * MADS_MIXED_ADD / peak,
            "lane_ops_per_s": {k: v for k, v in rates.items() if k not in ("fe_mul", "mixed_add")},
            "peak_lane_ops_per_s": peak}


def config_leg(sh, reps, school_reps):
    """A paper-shaped workload besides the headline: Cussen with the autotuned
    column group and with g = 1 against schoolbook, on GPU-encrypted inputs
    (A on the host, B resident in HBM; each call includes host planning and
    the affine normalisation of C)."""
    import torch
    from paper_2504_14497_amd import pcmm, workloads as W
    stream = torch.cuda.current_stream()
    A, msg = W.make_inputs(sh)
    _, pk = pcmm.keygen(sh.seed)
    B = pcmm.encrypt(pk, msg, sh.seed)
    out = {"workload": f"{sh.name}: A {sh.m}x{sh.n} uniform {'signed' if sh.signed else 'unsigned'} {sh.bits}-bit "
                       f"x B {sh.n}x{sh.l} ciphertexts of uniform {sh.msg_bits}-bit messages (seed {sh.seed})",
           "unit": "PC-MM/s"}
    results = {}
    for key, group in (("cussen_autotuned", pcmm.GROUP_AUTO), ("cussen_g1", 1)):
        cfg = pcmm.cussen_cfg(4, group)
        ws = torch.empty(pcmm.cussen_workspace_bytes(A, sh.bits, sh.l, pcmm.AFFINE, cfg), dtype=torch.uint8,
                         device="cuda")
        C = pcmm.DevPoints.empty(sh.m, sh.l, 2, pcmm.AFFINE)
        _, st = pcmm.cussen(A, sh.bits, B, cfg=cfg, workspace=ws, out=C)
        torch.cuda.synchronize()
        ms = time_region(lambda: pcmm.cussen(A, sh.bits, B, cfg=cfg, workspace=ws, out=C), reps, stream)
        results[key] = C
        out[key] = {"value": 1e3 / ms, "ms_per_step": ms, "group": st["group"], "k_split": st["k_split"],
                    "accum_adds_per_column": st["accum_adds"], "table_adds_per_column": st["table_adds"],
                    "workspace_mb": ws.numel() / 1e6}
        del ws
    wss = torch.empty(pcmm.lib().pcmm_schoolbook_workspace(sh.m, sh.n, sh.l, pcmm.AFFINE), dtype=torch.uint8,
                      device="cuda")
    Cs = pcmm.schoolbook(A, sh.bits, B, workspace=wss)
    torch.cuda.synchronize()
    ms_s = time_region(lambda: pcmm.schoolbook(A, sh.bits, B, workspace=wss), school_reps, stream)
    out["schoolbook"] = {"value": 1e3 / ms_s, "ms_per_step": ms_s}
    out["speedup_autotuned_vs_schoolbook"] = ms_s / out["cussen_autotuned"]["ms_per_step"]
    out["speedup_autotuned_vs_g1"] = out["cussen_g1"]["ms_per_step"] / out["cussen_autotuned"]["ms_per_step"]
    out["same_output"] = bool(torch.equal(results["cussen_autotuned"].t, Cs.t)
                              and torch.equal(results["cussen_g1"].t, Cs.t))
    return out


def batch_leg(reps):
    """64 uneven PC-MMs (m, n, l ~ U{32..512}, t ~ U{1, 2, 4, 8}, 8-bit
    messages): separate pcmm_cussen calls, separate cached plans, one batched
    plan (eager), and the batched plan replayed from a hipGraph."""
    import torch
    from paper_2504_14497_amd import pcmm, workloads as W
    bw = W.batch_workload()
    stream = torch.cuda.current_stream()
    As, Bs = [], []
    for sh in bw.shapes:
        A, msg = W.make_inputs(sh)
        _, pk = pcmm.keygen(sh.seed)
        As.append(A)
        Bs.append(pcmm.encrypt(pk, msg, sh.seed))
    torch.cuda.synchronize()
    count = len(As)
    cfg1 = pcmm.cussen_cfg(4, pcmm.GROUP_AUTO)  # column group and split from the autotuner
    t0 = time.time()
    plan = pcmm.Plan([(A, sh.bits, sh.l, pcmm.AFFINE, cfg1) for A, sh in zip(As, bw.shapes)])
    t_plan = time.time() - t0
    ws = torch.empty(plan.workspace_bytes(), dtype=torch.uint8, device="cuda")
    Cb = plan.outputs()
    # separate calls share one workspace of the largest single size
    single_ws = max(pcmm.cussen_workspace_bytes(A, sh.bits, sh.l, pcmm.AFFINE, cfg1)
                    for A, sh in zip(As, bw.shapes))
    ws1 = torch.empty(single_ws, dtype=torch.uint8, device="cuda")
    Cs = plan.outputs()

    def singles():
        for k in range(count):
            pcmm.cussen(As[k], bw.shapes[k].bits, Bs[k], cfg=cfg1, workspace=ws1, out=Cs[k])

    plans1 = [pcmm.Plan([(A, sh.bits, sh.l, pcmm.AFFINE, cfg1)]) for A, sh in zip(As, bw.shapes)]
    Cp = plan.outputs()

    def cached():
        for k in range(count):
            plans1[k].run([Bs[k]], [Cp[k]], ws1)

    def batched():
        plan.run(Bs, Cb, ws)

    singles()
    cached()
    batched()
    torch.cuda.synchronize()
    same = all(torch.equal(Cs[k].t, Cb[k].t) and torch.equal(Cp[k].t, Cb[k].t) for k in range(count))
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            plan.run(Bs, Cb, ws)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    for c in Cb:
        c.t.zero_()
    g.replay()
    torch.cuda.synchronize()
    same = same and all(torch.equal(Cs[k].t, Cb[k].t) for k in range(count))
    ms = {"single_calls": time_region(singles, reps, stream),
          "single_cached_plans": time_region(cached, reps, stream),
          "batched": time_region(batched, reps, stream),
          "batched_graph": time_region(g.replay, reps, stream)}
    acc = sum(2 * sh.l * plan.stats(k)["accum_adds"] for k, sh in enumerate(bw.shapes))
    chosen = [{"m": sh.m, "n": sh.n, "l": sh.l, "bits": sh.bits, "group": plan.stats(k)["group"],
               "k_split": plan.stats(k)["k_split"], "workspace_mb": round(plan.stats(k)["workspace_bytes"] / 1e6, 1)}
              for k, sh in enumerate(bw.shapes)]
    out = {"workload": f"{count} PC-MMs, m, n, l uniform in 32..512, A unsigned with bit-width uniform over "
                       f"(1, 2, 4, 8), ciphertexts of uniform 8-bit messages, Cussen N=4, column group and "
                       f"split chosen by the autotuner per problem (seed {bw.seed})",
           "unit": "PC-MM/s", "reps": reps, "same_output": bool(same), "host_plan_s": t_plan,
           "workspace_gb": ws.numel() / 1e9, "mixed_adds": acc, "tuned": chosen}
    for k, v in ms.items():
        out[k] = {"ms": v, "pcmm_per_s": count * 1000.0 / v}
    out["speedup_batched_graph_vs_single_calls"] = ms["single_calls"] / ms["batched_graph"]
    out["speedup_batched_graph_vs_cached_plans"] = ms["single_cached_plans"] / ms["batched_graph"]
    del ws, ws1
    return out


def vector_leg(ms, ts, l_batch, reps):
    """Vector x ciphertext-scalar (PC-MM with n = 1): an m-entry plaintext
    vector times one ciphertext (latency of one call), and times l_batch
    ciphertexts in one call (throughput), by schoolbook and Cussen."""
    import torch
    from paper_2504_14497_amd import pcmm, workloads as W
    stream = torch.cuda.current_stream()
    out = []
    for t in ts:
        for m in ms:
            sh = W.PCMMShape(m, 1, l_batch, t, False, 8, seed=1000 + 17 * t + m, name=f"vec{m}_t{t}")
            A, msg = W.make_inputs(sh)
            _, pk = pcmm.keygen(sh.seed)
            Bl = pcmm.encrypt(pk, msg, sh.seed)
            B1 = pcmm.encrypt(pk, msg[:, :1].copy(), sh.seed)
            row = {"m": m, "t": t}
            for l, B, key in ((1, B1, "one"), (l_batch, Bl, "batch")):
                cfg = pcmm.cussen_cfg(4, 1)
                wsc = torch.empty(pcmm.cussen_workspace_bytes(A, t, l, pcmm.AFFINE, cfg), dtype=torch.uint8,
                                  device="cuda")
                wss = torch.empty(pcmm.lib().pcmm_schoolbook_workspace(m, 1, l, pcmm.AFFINE), dtype=torch.uint8,
                                  device="cuda")
                C = pcmm.DevPoints.empty(m, l, 2, pcmm.AFFINE)
                Cc, _ = pcmm.cussen(A, t, B, cfg=cfg, workspace=wsc, out=C)
                Cs = pcmm.schoolbook(A, t, B, workspace=wss)
                torch.cuda.synchronize()
                same = bool(torch.equal(Cc.t, Cs.t))
                ms_c = time_region(lambda: pcmm.cussen(A, t, B, cfg=cfg, workspace=wsc, out=C), reps, stream)
                ms_s = time_region(lambda: pcmm.schoolbook(A, t, B, workspace=wss), reps, stream)
                if key == "one":
                    row.update({"cussen_us": ms_c * 1e3, "schoolbook_us": ms_s * 1e3,
                                "speedup": ms_s / ms_c, "same_output": same})
                else:
                    row.update({"cussen_products_per_s": l / (ms_c * 1e-3),
                                "schoolbook_products_per_s": l / (ms_s * 1e-3),
                                "batch_speedup": ms_s / ms_c, "batch_same_output": same})
            out.append(row)
    return {"what": f"a uniform unsigned t-bit m-vector times one EC-ElGamal ciphertext (n = l = 1; latency of "
                    f"one call incl. host planning and normalisation), and times {l_batch} ciphertexts in one "
                    f"call (products/s)", "reps": reps, "rows": out,
            "context": "paper (Raspberry Pi 5, m = 512, t = 4): schoolbook 59153.174 us, Cussen 399.094 us"}


# algorithmic 32x32 multiply-adds of one 6144-bit Montgomery product (192
# words: 192^2 for the product and 192^2 for the reduction, operand scanning)
MADS_PAILLIER_MUL = 2 * 192 * 192


def paillier_leg(m, n, l, bits, reps, school_reps):
    """Paillier PC-MM (Sec. "Extension to Paillier Encryption"), 3072-bit n:
    GPU encryption of the n x l ciphertexts (6148 products mod n^2 each,
    which gives the per-product rate), then Cussen and schoolbook PC-MM of an
    m x n unsigned bits-bit A on them."""
    import numpy as np
    import torch
    from paper_2504_14497_amd import paillier, pcmm, workloads as W
    stream = torch.cuda.current_stream()
    key_seed = 41
    t0 = time.time()
    nmod, _, _ = W.paillier_key(key_seed)
    key_s = time.time() - t0
    rng = W.rng_for(key_seed + 1)
    A = W.gen_plain_matrix(rng, m, n, bits, False)
    msg = torch.from_numpy(W.paillier_messages(rng, n, l, 16)).cuda()
    ctx = paillier.Paillier(nmod)
    B = ctx.encrypt(msg, seed=key_seed)
    torch.cuda.synchronize()
    # the product rate: encryption of 16384 ciphertexts (16 wavefronts per
    # SIMD), 6148 products mod n^2 each (2 per bit of the 3072-bit exponent n)
    enc_count = 16384
    msg_rate = torch.from_numpy(W.paillier_messages(rng, 128, enc_count // 128, 16)).cuda()
    ctx.encrypt(msg_rate, seed=key_seed + 2)
    enc_ms = time_region(lambda: ctx.encrypt(msg_rate, seed=key_seed + 2), 3, stream)
    products_per_ct = 2 * 3072 + 4
    mul_per_s = enc_count * products_per_ct / (enc_ms * 1e-3)
    cfg = pcmm.cussen_cfg(4, 1)
    wsc = torch.empty(ctx.cussen_workspace_bytes(A, bits, l, cfg), dtype=torch.uint8, device="cuda")
    C = torch.empty((m, l, paillier.WORDS), dtype=torch.int32, device="cuda")
    Cc, st = ctx.cussen(A, bits, B, cfg=cfg, workspace=wsc, out=C)
    Cs = ctx.schoolbook(A, bits, B)
    torch.cuda.synchronize()
    same = bool(torch.equal(Cc, Cs))
    ms_c = time_region(lambda: ctx.cussen(A, bits, B, cfg=cfg, workspace=wsc, out=C), reps, stream)
    ms_s = time_region(lambda: ctx.schoolbook(A, bits, B), school_reps, stream)
    # executed products mod n^2 per PC-MM: Alg. 4 powers of `level_mults`
    # (<= 2 bits products each), table products, accumulation products, plus
    # the conversions of B in and C out
    cussen_products = l * (st["table_adds"] + st["accum_adds"]) + n * l + m * l
    power_products = l * st["level_mults"] * 2 * bits
    nz = int(np.count_nonzero(A))
    school_products = l * nz * (2 * bits + 1) + n * l + m * l
    tops = mul_per_s * MADS_PAILLIER_MUL / 1e12
    return {"what": f"Paillier PC-MM, 3072-bit n (6144-bit ciphertexts): A {m}x{n} uniform unsigned {bits}-bit x "
                    f"B {n}x{l} GPU-encrypted uniform 16-bit messages; Cussen N=4, g=1 vs schoolbook (Alg. 4 "
                    "powers); canonical ciphertexts out",
            "cussen": {"pcmm_per_s": 1e3 / ms_c, "ms": ms_c,
                       "products_mod_n2": cussen_products + power_products,
                       "products_per_s": (cussen_products + power_products) / (ms_c * 1e-3)},
            "schoolbook": {"pcmm_per_s": 1e3 / ms_s, "ms": ms_s, "products_mod_n2": school_products,
                           "products_per_s": school_products / (ms_s * 1e-3)},
            "speedup_cussen_vs_schoolbook": ms_s / ms_c, "same_output": same,
            "encrypt": {"ciphertexts_per_s": enc_count / (enc_ms * 1e-3), "ms": enc_ms, "count": enc_count,
                        "products_per_ciphertext": products_per_ct},
            "product_rate": {"products_mod_n2_per_s": mul_per_s,
                             "mads_per_product": MADS_PAILLIER_MUL,
                             "achieved_TOPs": tops, "peak_TOPs": PEAK_INT32_MAD / 1e12,
                             "frac": tops * 1e12 / PEAK_INT32_MAD,
                             "source": "encryption kernel over 16384 ciphertexts (the r^n power: 2 products "
                                       "per exponent bit), 3 timed launches"},
            "key_generation_s": key_s,
            "context": "the paper reports no Paillier timings; it expects speedups similar to EC-ElGamal's"}


def serve_leg(n_requests, fractions, budget_gb, slots, max_batch, overlap_min=1):
    """Encrypted linear layers served by the continuous-batching scheduler:
    4 static layers W (256 x 1024, uniform signed 8-bit, resident plans),
    requests X (1024 x 8 ciphertexts of uniform 8-bit messages, a fresh
    matrix per request, resident in HBM) picking a layer uniformly; Poisson
    arrivals at fractions of the measured capacity."""
    import ctypes
    import numpy as np
    import torch
    from paper_2504_14497_amd import pcmm, workloads as W
    from paper_2504_14497_amd.serving import (DONE, GpuExecutor, Request, Server, latency_summary,
                                              poisson_arrivals, run_arrivals)
    base = W.SERVE_LAYER
    stream = torch.cuda.current_stream()
    layers = []
    for k in range(4):
        sh = W.PCMMShape(base.m, base.n, base.l, base.bits, True, base.msg_bits, seed=base.seed + k,
                         name=f"layer{k}")
        layers.append(W.make_inputs(sh)[0])
    cfg = pcmm.cussen_cfg(4, 1)
    t0 = time.time()
    plan = pcmm.Plan([(Wk, base.bits, base.l, pcmm.AFFINE, cfg) for Wk in layers])
    plan.make_resident()
    t_plan = time.time() - t0
    n, l, m = base.n, base.l, base.m
    rng = np.random.default_rng(base.seed)
    msg = torch.from_numpy(rng.integers(0, 1 << base.msg_bits, size=(n_requests * n, l)).astype(np.int32))
    _, pk = pcmm.keygen(base.seed)
    big = pcmm.encrypt(pk, msg.numpy(), base.seed)  # one call; request k owns rows k*n .. k*n + n - 1
    per = n * l

    def view(k):
        v = pcmm.DevPoints.__new__(pcmm.DevPoints)
        v.t, v.rows, v.cols, v.npts, v.form = big.t, n, l, 2, pcmm.AFFINE
        v.mat = pcmm.Mat(n, l, 2, pcmm.AFFINE, big.mat.ld, big.mat.d + k * per * 4)
        return v

    X = [view(k) for k in range(n_requests)]
    Cs = [pcmm.DevPoints.empty(m, l, 2, pcmm.AFFINE) for _ in range(n_requests)]
    which = rng.integers(0, 4, size=n_requests)
    ws = torch.empty(int(budget_gb * 1e9), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    ex = GpuExecutor(plan, ws, slots=slots, count=4)

    def fresh_requests(count):
        return [Request(rid=k, layer=int(which[k]), X=X[k], C=Cs[k]) for k in range(count)]

    def run(rate, count):
        srv = Server(ex, budget=ws.numel(), slots=slots, max_batch=max_batch, overlap_min=overlap_min)
        reqs = fresh_requests(count)
        arr = poisson_arrivals(count, rate, seed=17) if rate else np.zeros(count)
        wall = run_arrivals(srv, reqs, arr)
        torch.cuda.synchronize()
        assert all(r.state == DONE for r in reqs)
        sizes = [b for _, b, _ in srv.batches]
        out = latency_summary(reqs)
        out.update({"offered_req_per_s": rate, "achieved_req_per_s": count / wall,
                    "mean_batch": float(np.mean(sizes)), "batches": len(sizes)})
        return out

    run(0, min(64, n_requests))                     # warm-up
    burst = run(0, min(512, n_requests))             # all at once: capacity
    capacity = burst["achieved_req_per_s"]
    sweep = [dict(run(f * capacity, n_requests), fraction=f) for f in fractions]
    # identity: requests of the last sweep re-run alone equal their mixed results
    wsa = torch.empty(plan.selected_workspace_bytes([0]), dtype=torch.uint8, device="cuda")
    same = True
    for k in range(0, n_requests, max(1, n_requests // 8)):
        alone = pcmm.DevPoints.empty(m, l, 2, pcmm.AFFINE)
        plan.run_selected([int(which[k])], [X[k]], [alone], wsa)
        torch.cuda.synchronize()
        same = same and bool(torch.equal(alone.t, Cs[k].t))
    # full decryption of served outputs (bounded discrete log), checked against
    # the exact integer products
    bound = n * (1 << (base.bits - 1)) * ((1 << base.msg_bits) - 1)
    t0 = time.time()
    table = pcmm.DlogTable(20)
    torch.cuda.synchronize()
    t_table = time.time() - t0
    ks = list(range(min(64, n_requests)))
    # decrypt request by request inside one timed region
    msg_np = msg.numpy()
    outs = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    pcmm.decrypt(b"\x00" * 31 + b"\x01", Cs[0], bound, table)  # warm-up (wrong key: values unused)
    sk, _ = pcmm.keygen(base.seed)
    torch.cuda.synchronize()
    e0.record(stream)
    for k in ks:
        outs.append(pcmm.decrypt(sk, Cs[k], bound, table))
    e1.record(stream)
    torch.cuda.synchronize()
    ms_dec = e0.elapsed_time(e1)
    exact = all(bool((outs[x].cpu().numpy() == layers[int(which[k])].astype(np.int64)
                      @ msg_np[k * n:(k + 1) * n].astype(np.int64)).all()) for x, k in enumerate(ks))
    decrypt = {"elements": len(ks) * m * l, "ms": ms_dec, "elements_per_s": len(ks) * m * l / (ms_dec * 1e-3),
               "log2_baby": 20, "bound": bound, "table_build_s": t_table, "exact_integer_products": exact}
    return {"workload": f"4 layers W {m}x{n} uniform signed {base.bits}-bit (plans resident), requests X "
                        f"{n}x{l} ciphertexts of uniform {base.msg_bits}-bit messages, a fresh X per request, "
                        f"layer uniform; Poisson arrivals; Cussen N=4 g=1",
            "requests_per_rate": n_requests, "slots": slots, "max_batch": max_batch, "overlap_min": overlap_min,
            "budget_gb": budget_gb, "request_workspace_mb": plan.selected_workspace_bytes([0]) / 1e6,
            "host_plan_s": t_plan, "capacity_req_per_s": capacity, "burst": burst, "sweep": sweep,
            "alone_equals_mix": same, "decrypt": decrypt}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large512_t4")
    ap.add_argument("--group", type=int, default=-1,
                    help="Cussen column group g (-1 = the library's autotuner, 0 or 1 = one column per code, "
                         "Alg. 3 as printed)")
    ap.add_argument("--k-chunk", type=int, default=0, help="column groups per code list of the accumulation (0 = library default)")
    ap.add_argument("--k-split", type=int, default=0, help="split of the inner dimension (0 = library default)")
    ap.add_argument("--school-steps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-reps", type=int, default=3, help="timed repetitions of each batch form")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-PC-MM batch comparison")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving sweep")
    ap.add_argument("--no-vector", action="store_true", help="skip the vector x ciphertext-scalar microbench")
    ap.add_argument("--no-paillier", action="store_true", help="skip the Paillier PC-MM leg")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the signed 128^3 8-bit and 512^3 2-bit workloads")
    ap.add_argument("--no-field", action="store_true", help="skip the field-multiply and instruction-rate probes")
    ap.add_argument("--paillier-shape", default="64,64,64,4", help="m,n,l,bits of the Paillier PC-MM leg")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per arrival rate")
    ap.add_argument("--serve-fractions", default="0.25,0.5,0.75,1.0,1.25",
                    help="arrival rates as fractions of the measured capacity")
    ap.add_argument("--serve-budget-gb", type=float, default=40.0, help="workspace budget of the server")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run the plain copy kernel over BYTES (read BYTES, write BYTES) three "
                         "times, to scale the HBM byte counters of a profiler run")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2504_14497_amd import costmodel as cm
    from paper_2504_14497_amd import pcmm, workloads as W

    pcmm.lib()
    if args.calibrate_copy:
        nbytes = args.calibrate_copy // 16 * 16
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            pcmm.diag_copy(src, dst)
        torch.cuda.synchronize()
        assert bool((dst == 1).all())
        print(json.dumps({"calibrate_copy_bytes": nbytes, "launches": 3}), flush=True)
        return
    dev = pcmm.device_info()
    sh = W.NAMED[args.workload]
    A, msg = W.make_inputs(sh)
    log(f"device {dev}; workload {sh}")
    sk, pk = pcmm.keygen(sh.seed)
    B = pcmm.encrypt(pk, msg, sh.seed)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    C = pcmm.DevPoints.empty(sh.m, sh.l, 2, pcmm.AFFINE)
    cfg = pcmm.cussen_cfg(4, args.group, args.k_split, args.k_chunk)
    ws = torch.empty(pcmm.cussen_workspace_bytes(A, sh.bits, sh.l, pcmm.AFFINE, cfg),
                     dtype=torch.uint8, device="cuda")
    # one set of stage events per timed step, recorded by the library on the
    # launch stream without waiting (host planning of step k+1 overlaps the
    # kernels of step k exactly as without them)
    step_events = [[torch.cuda.Event(enable_timing=True) for _ in range(pcmm.STAGE_EVENTS)]
                   for _ in range(args.steps)]
    for evs in step_events:
        for e in evs:
            e.record(stream)
    step_cfgs = [pcmm.cussen_cfg(4, args.group, args.k_split, args.k_chunk, stage_events=evs)
                 for evs in step_events]
    for _ in range(args.warmup):
        pcmm.cussen(A, sh.bits, B, cfg=cfg, workspace=ws, out=C)
    torch.cuda.synchronize()

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    stats = []
    torch.cuda.synchronize()
    t_wall = time.time()
    host_ms = []
    e0.record(stream)
    for k in range(args.steps):
        t_call = time.perf_counter()
        _, st = pcmm.cussen(A, sh.bits, B, cfg=step_cfgs[k], workspace=ws, out=C)
        host_ms.append((time.perf_counter() - t_call) * 1e3)
        stats.append(st)
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.time() - t_wall
    ms_step = e0.elapsed_time(e1) / args.steps
    pcmm_per_s = 1000.0 / ms_step

    st0 = stats[0]
    per_col_muls, per_col_adds = st0["level_mults"], st0["level_adds"]
    paper_adds = (4 * sh.bits * sh.l * per_col_muls + 2 * sh.l * per_col_adds
                  + 2 * sh.m * sh.l * (sh.n - 1))
    executed_adds = 2 * sh.l * (st0["table_adds"] + st0["accum_adds"])
    step_gpu_ms = [evs[0].elapsed_time(evs[-1]) for evs in step_events]
    # device idle before each step (from the previous step's end, or from the
    # timed region's start): host planning that the queue did not hide
    idle_ms = [e0.elapsed_time(step_events[0][0])] + [
        step_events[k][-1].elapsed_time(step_events[k + 1][0]) for k in range(args.steps - 1)]
    names = ("ms_upload", "ms_table", "ms_accumulate", "ms_reduce", "ms_normalize")
    stage = {k: float(np.mean([evs[i].elapsed_time(evs[i + 1]) for evs in step_events]))
             for i, k in enumerate(names)}
    stage["ms_total"] = float(np.mean([evs[0].elapsed_time(evs[-1]) for evs in step_events]))

    # the same PC-MM with its plan compiled once (a static A served against ciphertexts)
    plan = pcmm.Plan([(A, sh.bits, sh.l, pcmm.AFFINE, cfg)])
    wsp = torch.empty(plan.workspace_bytes(), dtype=torch.uint8, device="cuda")
    Cp = plan.outputs()
    plan.run([B], Cp, wsp)
    ms_cached = time_region(lambda: plan.run([B], Cp, wsp), args.steps, stream)
    cached_same = bool(torch.equal(Cp[0].t, C.t))
    del wsp
    # the autotuned group for this shape
    tuned = pcmm.cussen_plan_stats(A, sh.bits, pcmm.cussen_cfg(4, pcmm.GROUP_AUTO))

    # schoolbook on the same inputs
    Cs = pcmm.DevPoints.empty(sh.m, sh.l, 2, pcmm.AFFINE)
    wss = torch.empty(pcmm.lib().pcmm_schoolbook_workspace(sh.m, sh.n, sh.l, pcmm.AFFINE),
                      dtype=torch.uint8, device="cuda")
    pcmm.schoolbook(A, sh.bits, B, workspace=wss)
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record(stream)
    for _ in range(args.school_steps):
        Cs = pcmm.schoolbook(A, sh.bits, B, workspace=wss)
    s1.record(stream)
    torch.cuda.synchronize()
    ms_school = s0.elapsed_time(s1) / args.school_steps
    same = bool((Cs.to_host() == C.to_host()).all())

    # Strassen (the paper's third method, schoolbook leaves) on the same inputs
    strassen = []
    for depth in (1, 2, 3):
        wst = torch.empty(pcmm.strassen_workspace_bytes(sh.m, sh.n, sh.l, pcmm.AFFINE, depth),
                          dtype=torch.uint8, device="cuda")
        Cst, sst = pcmm.strassen(A, sh.bits, B, depth=depth, workspace=wst)
        torch.cuda.synchronize()
        same_st = bool(torch.equal(Cst.t, C.t))
        ms_st = time_region(lambda: pcmm.strassen(A, sh.bits, B, depth=depth, workspace=wst), args.school_steps,
                            stream)
        strassen.append({"depth": depth, "value": 1000.0 / ms_st, "unit": "PC-MM/s", "ms_per_step": ms_st,
                         "leaf_bits": sst["leaf_bits"], "leaves": sst["leaves"],
                         "block_point_adds": sst["block_adds"], "same_output_as_cussen": same_st,
                         "paper_model_point_adds_per_s": (cm.strassen_equiv_adds(sh.n, sh.bits) / (ms_st * 1e-3)
                                                          if sh.m == sh.n == sh.l and sh.n & (sh.n - 1) == 0
                                                          else None)})
        del wst

    # roofline of the dominant kernel (accumulation): algorithmic multiply-adds
    madds = 2 * sh.l * st0["accum_adds"]
    acc_ms = stage["ms_accumulate"]
    achieved = madds * MADS_MIXED_ADD / (acc_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_INT32_MAD / 1e12,
                "unit": "TOP/s (32x32->64-bit multiply-adds)", "frac": achieved / (PEAK_INT32_MAD / 1e12),
                "traffic": load_traffic(sh.name), "kernel": "accumulate_kernel",
                "kernel_ms": acc_ms, "mixed_adds_per_launch": madds,
                "mads_per_mixed_add": MADS_MIXED_ADD}

    # the table stage (digit tables, combinations): algorithmic bytes are
    # every table entry written once (72 B: an x and a y granule) and B read
    # once (128 B per ciphertext); it is latency- and traffic-bound rather
    # than ALU-bound
    tab_ms = stage["ms_table"]
    tab_bytes = st0["table_entries"] * 2 * sh.l * 72 + sh.n * sh.l * 128
    table_roofline = {"bound": "hbm", "kernels": ["table_build_kernel", "combo_forward_kernel",
                                                  "combo_backward_kernel"],
                      "achieved": tab_bytes / (tab_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": tab_bytes / (tab_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": load_table_traffic(sh.name),
                      "algorithmic_bytes": tab_bytes, "stage_ms": tab_ms,
                      "point_additions": st0["table_adds"] * 2 * sh.l,
                      "point_additions_per_s": st0["table_adds"] * 2 * sh.l / (tab_ms * 1e-3)}

    out = {
        "metric": METRIC, "value": pcmm_per_s, "unit": "PC-MM/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic (seeded uniform plaintexts; ciphertexts encrypted on the GPU)",
        "config": {"workload": f"{sh.name}: A {sh.m}x{sh.n} uniform {'signed' if sh.signed else 'unsigned'} "
                               f"{sh.bits}-bit x B {sh.n}x{sh.l} EC-ElGamal/P-256 ciphertexts of uniform "
                               f"{sh.msg_bits}-bit messages; Cussen N=4, "
                               f"{'autotuned column group g=%d' % st0['group'] if args.group < 0 else 'g=%d' % max(args.group, 1)}"
                               f", canonical affine output",
                   "m": sh.m, "n": sh.n, "l": sh.l, "bits": sh.bits, "seed": sh.seed},
        "point_adds_per_s": paper_adds / (ms_step * 1e-3),
        "paper_model_point_adds": paper_adds,
        "executed_point_adds_per_s": executed_adds / (ms_step * 1e-3),
        "stage_ms": stage,
        "step_gpu_ms": {"median": float(np.median(step_gpu_ms)), "min": float(np.min(step_gpu_ms)),
                        "max": float(np.max(step_gpu_ms))},
        "idle_ms_before_step": [round(x, 3) for x in idle_ms],
        "host_ms_per_call": [round(x, 3) for x in host_ms],
        "cached_plan": {"value": 1000.0 / ms_cached, "unit": "PC-MM/s", "ms_per_step": ms_cached,
                        "same_output": cached_same},
        "autotuned_group": tuned["group"],
        "group": st0["group"], "k_split": st0["k_split"],
        "wall_s": t_wall,
        "schoolbook": {"value": 1000.0 / ms_school, "unit": "PC-MM/s", "ms_per_step": ms_school,
                       "point_adds_per_s": cm.schoolbook_equiv_adds(sh.m, sh.n, sh.l, sh.bits)
                       / (ms_school * 1e-3), "same_output_as_cussen": same},
        "speedup_cussen_vs_schoolbook": ms_school / ms_step,
        "strassen": strassen,
        "speedup_cussen_vs_best_strassen": min(x["ms_per_step"] for x in strassen) / ms_step,
        "roofline": roofline,
        "table_roofline": table_roofline,
        "device": dev,
    }
    if not args.no_field:
        out["field_mul"] = field_mul_leg()
    del ws
    if not args.no_configs:
        out["configs"] = {x.name: config_leg(x, 5, 1) for x in (W.SIGNED128, W.LARGE_T2)}
    if not args.no_batch:
        out["batch"] = batch_leg(args.batch_reps)
    if not args.no_vector:
        out["vector"] = vector_leg((8, 64, 512), (4, 8, 16), 4096, 20)
    if not args.no_paillier:
        pm, pn, pl_, pb = (int(x) for x in args.paillier_shape.split(","))
        log("paillier leg", pm, pn, pl_, pb)
        out["paillier"] = paillier_leg(pm, pn, pl_, pb, 3, 1)
    if not args.no_serve:
        torch.cuda.empty_cache()
        out["serving"] = serve_leg(args.serve_requests, [float(x) for x in args.serve_fractions.split(",")],
                                   args.serve_budget_gb, slots=2, max_batch=32, overlap_min=4)
    if not args.no_cpu_baseline:
        threads = max(1, min(os.cpu_count() or 1, 16))
        base, Corc, cols = cpu_baseline(sh, A, args.cpu_seconds, threads)
        Cg = C.to_host()
        base["parity_on_sample"] = bool((Cg[:, cols] == Corc[:, cols]).all())
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
