"""Benchmark of the nTT sweep on one MI355X.

A step is one full pass of the hot path over the 32^5 workload (33.5M entries from
rank-8 U[0,1) TT cores with 1% multiplicative noise): ntt_decompose (4 stages x 500
MU iterations at ranks 8, FP32) followed by ntt_rel_error (Eq.(3), fused, FP64 sums).
The input tensor is resident in HBM before the timed region starts.

value = algorithmic GFLOP of the sweep per step (4mkr + 4(m+k)r^2 per iteration,
summed over stages) / seconds per step.  One JSON line is printed.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "nTT GFLOP/s & decomps/s, p50/p99 latency; BF16 vs FP32 at equal rel. error"


def progress(msg):
    """Progress of the benchmark phases (stderr; the result is the one JSON line on stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFS = 157.3
BF16_MFMA_PEAK_TFS = 2500.0
EXTRAS = ("precision_mode", "paper_workload", "rank_rule", "bcd", "streamed", "batched", "serving")


def profiled_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the rocprofv3 summaries under
    profiles/ (a line `traffic: kernel=... workload=... bytes=... source=... source_sha16=...`,
    the kernel name written without spaces,
    FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings).  None when no summary
    has it, or when the kernel's source file changed since the counters were taken."""
    import glob
    import hashlib
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(f):
            if not line.startswith("traffic:"):
                continue
            kv = dict(t.split("=", 1) for t in line[len("traffic:"):].split() if "=" in t)
            if kv.get("kernel") != kernel.replace(" ", "") or kv.get("workload") != workload:
                continue
            src = os.path.join(ROOT, kv.get("source", ""))
            if not os.path.isfile(src):
                return None
            sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
            return float(kv["bytes"]) if sha == kv.get("source_sha16") else None
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tt32x5_r8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the precision-mode, paper-workload, batched and serving measurements")
    ap.add_argument("--extras", default=",".join(EXTRAS),
                    help="comma-separated subset of the extra measurements: " + ", ".join(EXTRAS))
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-max-mb", type=float, default=1000.0)
    ap.add_argument("--serve-rates", default="0.8",
                    help="comma-separated arrival rates as fractions of the saturated rate")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (for scaling "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE readings) and exit")
    return ap.parse_args()


def _oracle_mu_rate(X, W, H, r, eps, seconds):
    """MU iterations of the oracle on X for about `seconds`: (iterations, seconds, GFLOP/s)."""
    import oracle as O
    m, k = X.shape
    t0 = time.perf_counter()
    n = 0
    while True:
        W, H = O.mu_step(X, W, H, eps)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or n >= 500:
            break
    return n, el, n * (4.0 * m * k * r + 4.0 * (m + k) * r * r) / el / 1e9


def cpu_baseline(A, w, seconds, bcd_seconds=0.0):
    """The FP64 oracle on this host, on a bounded sample: MU iterations of stage 1 with
    all host cores, then with one thread."""
    import numpy as np
    import oracle as O
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    X = A.reshape(A.shape[0], -1).astype(np.float64)
    m, k = X.shape
    r = w.target_ranks[1]
    W, H = O.init_factors(w.seed, 1, m, r, k)
    n, el, rate = _oracle_mu_rate(X, W, H, r, w.eps, seconds)
    with threadpool_limits(limits=1):
        n1, el1, rate1 = _oracle_mu_rate(X, W, H, r, w.eps, seconds / 3)
    out = {"value": rate, "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
           "sample": f"{n} MU iterations of stage 1 ({m}x{k}, r={r}) of the same workload, "
                     f"NumPy FP64, {el:.1f} s",
           "one_thread": {"value": rate1, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
                          "sample": f"{n1} MU iterations of the same stage 1, NumPy FP64 limited to "
                                    f"one thread, {el1:.1f} s"}}
    if bcd_seconds > 0:
        # the BCD oracle (Alg.3) on the same first unfolding: ms per iteration
        W0, H0 = O.init_factors(w.seed, 1, m, r, k)
        t0 = time.perf_counter()
        O.bcd_nmf(X, W0, H0, 1)
        nb = max(2, min(64, int(bcd_seconds / (time.perf_counter() - t0))))
        t0 = time.perf_counter()
        O.bcd_nmf(X, W0, H0, nb)
        el = time.perf_counter() - t0
        out["bcd"] = {"ms_per_iter": el * 1e3 / nb, "kind": "oracle",
                      "sample": f"{nb} BCD iterations of stage 1 ({m}x{k}, r={r}), NumPy FP64, {el:.1f} s"}
    return out


def precision_mode(ntt, S, torch, cpu_seconds=0.0):
    """128^4 rank-16 workload: FP32 sweep vs BF16 mode (last 20 iterations FP32).  For each
    mode, the roofline of the dominant kernel, the stage-1 pass, from HIP events around each
    launch of a profiled sweep (BF16 mode: every iteration on the BF16 copy); with
    cpu_seconds > 0, the oracle's MU iterations on the same first unfolding."""
    import numpy as np
    w = S.workload("tt128x4_r16")
    A_host = w.tensor()
    A = torch.from_numpy(A_host).cuda()
    out = {"workload": f"{w.name}: {w.note}"}
    progress("precision mode: 128^4 tensor generated")
    m, k, r = w.dims[0], int(np.prod(w.dims[1:])), w.target_ranks[1]
    kernels = {"fp32": "k_mu_pass_LW<2, 4, false, true>", "bf16": "k_mu_pass_LWB<2, 4, true>"}
    for name, prec in (("fp32", ntt.NTT_PREC_FP32), ("bf16", ntt.NTT_PREC_BF16_MIXED)):
        plan = ntt.Plan(w.dims, w.target_ranks, w.iters, eps=w.eps, seed=w.seed, precision=prec,
                        fp32_tail_iters=w.fp32_tail)
        res = ntt.decompose(A, w.target_ranks, w.iters, plan=plan, want_report=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ntt.decompose(A, w.target_ranks, w.iters, plan=plan, cores=res.cores)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        gflop = res.report["total_gflop"]
        out[name] = {"ms": ms, "gflop_per_s": gflop / (ms * 1e-3),
                     "mfma_frac_fp32_peak": gflop / (ms * 1e-3) / (FP32_MFMA_PEAK_TFS * 1e3),
                     "decomps_per_s": 1e3 / ms, "rel_error": ntt.rel_error(A, res.cores),
                     "stage_ms": res.report["ms"]}
        pplan = ntt.Plan(w.dims, w.target_ranks, w.iters, eps=w.eps, seed=w.seed, precision=prec,
                         fp32_tail_iters=0, flags=ntt.NTT_PROFILE)
        prep = ntt.decompose(A, w.target_ranks, w.iters, plan=pplan)
        pass_ms = prep.report["pass_ms"][0]
        xbytes = 2.0 if name == "bf16" else 4.0
        bytes_launch = xbytes * m * k + 8.0 * r * k + 4.0 * m * r
        flop_launch = 4.0 * m * k * r + 4.0 * (m + k) * r * r
        ach = bytes_launch / (pass_ms * 1e-3) / 1e9
        kern = kernels[name]
        traffic = profiled_traffic(kern, w.name)
        out[name]["roofline"] = {
            "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": f"{kern} stage 1 ({m}x{k}, r={r})", "pass_ms": pass_ms,
            "bytes_per_launch": bytes_launch,
            "tflops": flop_launch / (pass_ms * 1e-3) / 1e12,
            "mfma_peak_tflops": BF16_MFMA_PEAK_TFS if name == "bf16" else FP32_MFMA_PEAK_TFS}
        progress(f"precision mode: {name} {ms:.1f} ms, stage-1 pass {pass_ms * 1e3:.1f} us "
                 f"({ach:.0f} GB/s)")
    out["bf16_speedup"] = out["fp32"]["ms"] / out["bf16"]["ms"]
    out["rel_error_gap"] = abs(out["bf16"]["rel_error"] - out["fp32"]["rel_error"])
    del A
    if cpu_seconds > 0:
        from threadpoolctl import threadpool_info, threadpool_limits
        import oracle as O
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        X = A_host.reshape(m, k).astype(np.float64)
        W0, H0 = O.init_factors(w.seed, 1, m, r, k)
        n, el, rate = _oracle_mu_rate(X, W0, H0, r, w.eps, cpu_seconds)
        with threadpool_limits(limits=1):
            n1, el1, rate1 = _oracle_mu_rate(X, W0, H0, r, w.eps, cpu_seconds / 2)
        out["cpu_baseline"] = {
            "value": rate, "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} MU iterations of stage 1 ({m}x{k}, r={r}), NumPy FP64, {el:.1f} s",
            "one_thread": {"value": rate1, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
                           "sample": f"{n1} MU iterations of stage 1, one thread, {el1:.1f} s"}}
        del X
    return out


def paper_workload(ntt, S, torch):
    """The paper's workload size on one GPU: 256^4 FP32 (17 GB) from rank-10 TT cores,
    ranks 10, 100 MU iterations per stage; then the rank sweep r in {2, 4, 8, 16}."""
    w = S.workload("tt256x4_r10")
    A = _tt_on_gpu(ntt, S, torch, w)
    progress("paper workload: 256^4 tensor formed on the device")
    out = {"workload": f"{w.name}: {w.note}"}
    for r in (10, 2, 4, 8, 16):
        ranks = (1, r, r, r, 1)
        plan = ntt.Plan(w.dims, ranks, w.iters, eps=w.eps, seed=w.seed)
        res = ntt.decompose(A, ranks, w.iters, plan=plan, want_report=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ntt.decompose(A, ranks, w.iters, plan=plan, cores=res.cores)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        out[f"r{r}"] = {"ms": ms, "gflop_per_s": res.report["total_gflop"] / (ms * 1e-3),
                        "gflop": res.report["total_gflop"], "rel_error": ntt.rel_error(A, res.cores),
                        "stage_ms": res.report["ms"], "compression": res.report["compression_ratio"]}
        progress(f"paper workload: ranks {r}: {ms:.1f} ms")
    # the paper times both NMF methods on this workload (Fig.5): BCD at ranks 10
    ranks = (1, 10, 10, 10, 1)
    plan = ntt.Plan(w.dims, ranks, w.iters, seed=w.seed, nmf="bcd")
    res = ntt.decompose(A, ranks, w.iters, plan=plan, want_report=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ntt.decompose(A, ranks, w.iters, plan=plan, cores=res.cores)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    out["bcd_r10"] = {"ms": ms, "rel_error": ntt.rel_error(A, res.cores), "stage_ms": res.report["ms"],
                      "corrections": res.report["corrections"]}
    progress(f"paper workload: BCD ranks 10: {ms:.1f} ms")
    del A
    return out


def rank_rule(ntt, S, torch):
    """Compression against relative error with the rank rule of Alg.2 (the style of the
    paper's Fig.8, which draws it for both NMF methods), on the 128^4 workload, rank caps
    16, for the paper's thresholds, with MU and with BCD."""
    w = S.workload("tt128x4_r16")
    A = torch.from_numpy(w.tensor()).cuda()
    caps = (1, 16, 16, 16, 1)
    out = {"workload": f"{w.name}: {w.note}; rank caps 16", "points": []}
    for nmf, eps in [(n, e) for n in ("mu", "bcd") for e in (0.5, 0.25, 0.125, 0.075, 0.01, 0.005, 0.001)]:
        plan = ntt.Plan(w.dims, caps, w.iters, eps=w.eps, seed=w.seed, rank_eps=eps, nmf=nmf)
        res = ntt.decompose(A, caps, w.iters, plan=plan)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ntt.decompose(A, caps, w.iters, plan=plan)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        out["points"].append({"nmf": nmf, "rank_eps": eps, "ranks": res.ranks, "ms": ms,
                              "compression": res.report["compression_ratio"],
                              "rel_error": ntt.rel_error(A, res.cores),
                              "stage_ms": res.report["ms"]})
        progress(f"rank rule: {nmf} eps {eps}: ranks {res.ranks}, {ms:.1f} ms")
    del A
    return out


def bcd(ntt, S, torch, mu_err, mu_ms):
    """The sweep with the BCD NMF of Alg.3 (extrapolation cap 0.9999) on the 32^5 workload
    at the same ranks and iteration count as the MU sweep: time, error, dropped iterations,
    and the bytes each stage-1 iteration moves (two X passes: the H step and the products)."""
    w = S.workload("tt32x5_r8")
    A = torch.from_numpy(w.tensor()).cuda()
    plan = ntt.Plan(w.dims, w.target_ranks, w.iters, seed=w.seed, nmf="bcd")
    res = ntt.decompose(A, w.target_ranks, w.iters, plan=plan)
    torch.cuda.synchronize()
    runs = []
    for _ in range(3):
        t0 = time.perf_counter()
        res = ntt.decompose(A, w.target_ranks, w.iters, plan=plan)
        torch.cuda.synchronize()
        runs.append((time.perf_counter() - t0) * 1e3)
    ms = min(runs)
    err = ntt.rel_error(A, res.cores)
    m, k, r = 32, 32 ** 4, 8
    it_ms = res.report["ms"][0] / w.iters
    # per iteration: X twice, the kept H (and the kept H before it while extrapolating),
    # the candidate H written and read back
    bytes_it = 8.0 * m * k + 16.0 * r * k
    out = {"workload": f"{w.name}: {w.note}; BCD (Alg.3), delta 0.9999", "ms": ms,
           "rel_error": err, "mu_rel_error": mu_err, "mu_ms": mu_ms,
           "corrections": res.report["corrections"], "stage_ms": res.report["ms"],
           "stage1_ms_per_iter": it_ms,
           "stage1_gbs": bytes_it / (it_ms * 1e-3) / 1e9, "stage1_bytes_per_iter": bytes_it,
           # a whole stage-1 iteration (step, H step, products, reduction) against HBM
           "roofline": {"bound": "hbm", "achieved": bytes_it / (it_ms * 1e-3) / 1e9,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": bytes_it / (it_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                        "kernel": "BCD stage-1 iteration (32x1048576, r=8), four launches"}}
    progress(f"bcd: {ms:.1f} ms, rel err {err:.4e} (MU {mu_err:.4e}), corrections "
             f"{res.report['corrections']}")
    del A
    return out


def streamed(ntt, S, torch, iters=3, cols=1 << 20):
    """The out-of-core first stage on the paper's workload: the 256^4 FP32 tensor (17.2 GB)
    in pinned host memory, stage 1 streamed in blocks of 2^20 columns (1 GB of X each),
    a few MU iterations per stage; against the same iterations with the tensor resident."""
    w = S.workload("tt256x4_r10")
    Ad = _tt_on_gpu(ntt, S, torch, w)
    Ah = torch.empty(tuple(Ad.shape), dtype=torch.float32, pin_memory=True)
    Ah.copy_(Ad)
    torch.cuda.synchronize()
    progress("streamed: 256^4 tensor in pinned host memory")
    ranks = w.target_ranks
    out = {"workload": f"{w.name}: {w.note}; {iters} MU iterations per stage, stage 1 streamed "
                       f"from pinned host memory in blocks of {cols} columns"}
    for mode in ("resident", "streamed"):
        kw = {"stream_cols": cols} if mode == "streamed" else {}
        A = Ah if mode == "streamed" else Ad
        plan = ntt.Plan(w.dims, ranks, iters, seed=w.seed, **kw)
        res = ntt.decompose(A, ranks, iters, plan=plan, want_report=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ntt.decompose(A, ranks, iters, plan=plan, cores=res.cores)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        # stage 1 passes over X in both modes: the norm, T iterations, the final objective
        passes = iters + 2
        x_bytes = 4.0 * Ad.numel()
        out[mode] = {"ms": ms, "stage_ms": res.report["ms"], "rel_error": ntt.rel_error(Ad, res.cores),
                     "stage1_ms_per_x_pass": res.report["ms"][0] / passes,
                     "stage1_x_gbs": x_bytes * passes / (res.report["ms"][0] * 1e-3) / 1e9}
        progress(f"streamed: {mode}: {ms:.1f} ms, stage 1 {res.report['ms'][0]:.1f} ms")
    # the paper's large-tensor workflow: ranks chosen by the rule of Alg.2 while X stays in
    # host memory (caps 8, so that every unfolding's shorter side is at most 2048;
    # threshold 0.01)
    caps = (1, 8, 8, 8, 1)
    plan = ntt.Plan(w.dims, caps, iters, seed=w.seed, stream_cols=cols, rank_eps=0.01)
    t0 = time.perf_counter()
    res = ntt.decompose(Ah, caps, iters, plan=plan)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    out["streamed_rank_rule"] = {"rank_eps": 0.01, "caps": list(caps), "ranks": res.ranks, "ms": ms,
                                 "stage_ms": res.report["ms"], "rel_error": ntt.rel_error(Ad, res.cores),
                                 "compression": res.report["compression_ratio"]}
    progress(f"streamed: rank rule: ranks {res.ranks}, {ms:.1f} ms")
    del Ad, Ah
    return out


def _tt_on_gpu(ntt, S, torch, w):
    cores = [torch.from_numpy(c).cuda() for c in S.random_cores(w.dims, w.gen_ranks, w.seed)]
    return ntt.reconstruct(cores)


def batched(ntt, S, torch, count=256):
    """256 tensors, d in {3,4,5}, n in [8,64], true ranks in [2,12], T = 200, FP32."""
    mix = S.batched_mix(count)
    tensors = [_tt_on_gpu(ntt, S, torch, w) for w in mix]
    progress(f"batched: {count} tensors generated")
    ranks = [w.target_ranks for w in mix]
    seeds = [w.seed for w in mix]
    cores, reps, b = ntt.decompose_batch(tensors, ranks, mix[0].iters, seeds)
    torch.cuda.synchronize()
    progress("batched: warm-up batch done")
    t0 = time.perf_counter()
    cores, reps, b = ntt.decompose_batch(tensors, ranks, mix[0].iters, seeds, batch=b, cores=cores)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    gflop = sum(r["total_gflop"] for r in reps)
    # algorithmic HBM bytes: per MU iteration of a stage, X read once, H read and written,
    # W read (4mk + 8rk + 4mr), as for the headline kernel
    nbytes = 0.0
    for w, r in zip(mix, reps):
        e = r["eff_ranks"]
        for l in range(len(w.dims) - 1):
            m, k, rr = e[l] * w.dims[l], math.prod(w.dims[l + 1:]), e[l + 1]
            nbytes += r["iters"][l] * (4.0 * m * k + 8.0 * rr * k + 4.0 * m * rr)
    out = {"problems": count, "entries": int(sum(t.numel() for t in tensors)), "s": sec,
           "decomps_per_s": count / sec, "gflop_per_s": gflop / sec,
           "hbm_bytes": nbytes, "hbm_gbs": nbytes / sec / 1e9,
           "hbm_frac": nbytes / sec / 1e9 / HBM_PEAK_GBS,
           "mean_stage_rel_err": float(sum(sum(r["stage_rel_err"]) / len(r["stage_rel_err"]) for r in reps) / count)}
    del tensors, cores
    return out


def serving_inputs(ntt, S, torch, n_req, max_mb):
    """The request stream's tensors in pinned host memory (how requests arrive), shared by
    both precisions: generated on the device from their TT cores and copied into 2 GiB
    pinned chunks, packed first-fit by decreasing size (one allocation per chunk)."""
    import numpy as np
    reqs = S.serving_stream(n_req, max_bytes=max_mb * 1e6)
    t0 = time.perf_counter()
    chunk = 1 << 29                       # floats (2 GiB)
    sizes = [int(np.prod(q.work.dims)) for q in reqs]
    pad = [(n + 63) // 64 * 64 for n in sizes]
    fill, where = [], {}
    for i in sorted(range(len(reqs)), key=lambda i: -pad[i]):
        need = max(pad[i], 64)
        c = next((c for c in range(len(fill)) if fill[c] + need <= max(chunk, need)), None)
        if c is None:
            fill.append(0)
            c = len(fill) - 1
        where[i] = (c, fill[c])
        fill[c] += need
    pools = [torch.empty(max(chunk, f), dtype=torch.float32, pin_memory=True) for f in fill]
    t1 = time.perf_counter()
    host = [None] * len(reqs)
    for i, q in enumerate(reqs):
        g = _tt_on_gpu(ntt, S, torch, q.work)
        c, off = where[i]
        h = pools[c][off:off + sizes[i]].view(tuple(q.work.dims))
        h.copy_(g)
        host[i] = h
        del g
    torch.cuda.synchronize()
    progress(f"serving: {len(reqs)} requests, {sum(sizes) * 4 / 1e9:.1f} GB in {len(pools)} pinned "
             f"chunks ({t1 - t0:.1f} s to allocate, {time.perf_counter() - t1:.1f} s to generate)")
    return reqs, host


def serving(ntt, S, torch, reqs, host, precision, rates):
    """Poisson stream of TT-generated requests (d in 3..6, 1 MB..max_mb log-uniform, r 4..32):
    a short warm-up, then saturated (all at t = 0) to find the service rate mu and, after
    that run, each request's relative error (Eq.(3)) against its input; then arrivals at the
    given fractions of mu."""
    import numpy as np
    n_req = len(reqs)
    need = sum(h.numel() * 4 for h in host)
    arena = int(min(64 << 30, 3 * need + (1 << 30)))

    def run(arrivals, subset=None, errors=None):
        order = list(range(n_req)) if subset is None else list(subset)
        srv = ntt.Server(arena, max_slots=16, iters_per_tick=25)
        t_start = time.perf_counter()
        pending, done, lat, gfl = list(order), {}, [], 0.0
        ids, kept = {}, []
        while pending or len(done) < len(order):
            now = time.perf_counter() - t_start
            while pending and arrivals[pending[0]] <= now:
                i = pending.pop(0)
                q = reqs[i].work
                ids[srv.submit(host[i], q.target_ranks, q.iters, seed=q.seed, precision=precision,
                               fp32_tail_iters=20)] = i
            srv.tick()
            for rid, i in list(ids.items()):
                inf = srv.info(rid)
                if inf["state"] == ntt.NTT_REQ_DONE:
                    lat.append(inf["t_finish"] - inf["t_submit"])
                    gfl += inf["gflop"]
                    done[i] = inf["t_finish"]
                    if errors is None:
                        srv.release(rid)
                    else:
                        kept.append((rid, i))
                    del ids[rid]
                elif inf["state"] in (ntt.NTT_REQ_REJECTED, ntt.NTT_REQ_CANCELLED):
                    raise RuntimeError("request not served")
        span = time.perf_counter() - t_start
        for rid, i in kept:                  # after the timed span: Eq.(3) on the device
            errors[i] = ntt.rel_error(host[i].to("cuda:0"), srv.cores(rid))
            srv.release(rid)
        srv.close()
        progress(f"serving run: {len(order)} requests in {span:.2f} s")
        lat = np.array(lat)
        return {"decomps_per_s": len(order) / span, "gflop_per_s": gfl / span,
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3)}

    small = sorted(range(n_req), key=lambda i: host[i].numel())[:8]
    run([0.0] * n_req, subset=sorted(small))  # warm-up: first launches of the kernel variants
    errors = [None] * n_req
    sat = run([0.0] * n_req, errors=errors)
    mu = sat["decomps_per_s"]
    out = {"saturated": sat, "rel_error": errors}
    for frac in rates:
        rate = frac * mu
        gaps = -np.log(1.0 - S.uniform01(5, 0x301, (n_req,)).astype(np.float64)) / rate
        out[f"rate_{frac}mu"] = run(list(np.cumsum(gaps) - gaps[0]))
    return out


def serving_both(ntt, S, torch, n_req, max_mb, rates):
    """FP32 and BF16-mixed serving of the same stream; per-request errors summarised, with
    the BF16/FP32 error ratio (the comparison at equal relative error)."""
    import numpy as np
    reqs, host = serving_inputs(ntt, S, torch, n_req, max_mb)
    res = {}
    for name, prec in (("fp32", ntt.NTT_PREC_FP32), ("bf16", ntt.NTT_PREC_BF16_MIXED)):
        res[name] = serving(ntt, S, torch, reqs, host, prec, rates)
    e32, e16 = (np.array(res[k].pop("rel_error"), dtype=np.float64) for k in ("fp32", "bf16"))
    for k, e in (("fp32", e32), ("bf16", e16)):
        res[k]["rel_error"] = {"median": float(np.median(e)), "mean": float(e.mean()), "max": float(e.max())}
    ratio = e16 / np.maximum(e32, 1e-300)
    sizes = np.array([h.numel() * 4 for h in host], dtype=np.float64)
    res["bf16_over_fp32_error"] = {"median": float(np.median(ratio)), "max": float(ratio.max())}
    res["requests"] = n_req
    res["bytes"] = {"total": float(sizes.sum()), "max": float(sizes.max()), "median": float(np.median(sizes))}
    res["note"] = (f"{n_req} requests of the serving stream recipe (d 3..6, ranks 4..32, T=200), sizes "
                   f"log-uniform from 1 MB to {max_mb:g} MB before rounding the modes, inputs in pinned "
                   f"host memory; arrivals saturated, then Poisson at "
                   f"{', '.join(str(r) for r in rates)} of the saturated rate")
    del host
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    import synth as S
    from paper_2008_01340_amd import ntt

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n}), flush=True)
        return

    w = S.workload(args.workload)
    A_host = w.tensor()
    dev = torch.device("cuda:0")
    A = torch.from_numpy(A_host).to(dev)
    d = len(w.dims)
    plan = ntt.Plan(w.dims, w.target_ranks, w.iters, eps=w.eps, seed=w.seed)
    nbytes, eff, comp = plan.workspace()
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    cores = [torch.empty((eff[k], w.dims[k], eff[k + 1]), dtype=torch.float32, device=dev)
             for k in range(d)]
    tt_ws_bytes = ntt.ntt_tt_workspace(w.dims, eff)
    tt_ws = torch.empty(tt_ws_bytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    core_ptrs = [c.data_ptr() for c in cores]

    def step():
        ntt.ntt_decompose(plan, stream, ws.data_ptr(), A.data_ptr(), core_ptrs, want_report=False)
        return ntt.ntt_rel_error(w.dims, eff, A.data_ptr(), core_ptrs, tt_ws.data_ptr(),
                                 tt_ws_bytes, stream)

    progress(f"{w.name}: input resident, warm-up")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        err = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el * 1e3 / args.steps
    progress(f"{w.name}: {ms:.2f} ms per step")

    # stage shapes and algorithmic flops
    shapes = []
    for l in range(1, d):
        m = eff[l - 1] * w.dims[l - 1]
        k = int(np.prod(w.dims[l:]))
        shapes.append((m, k, eff[l]))
    gflop = sum(w.iters * (4.0 * m * k * r + 4.0 * (m + k) * r * r) for m, k, r in shapes) * 1e-9

    # per-stage times of the same (graph-replayed) sweep, from stage-boundary HIP events
    rep_graph = ntt.ntt_decompose(plan, stream, ws.data_ptr(), A.data_ptr(), core_ptrs)

    # dominant kernel: the fused X pass of stage 1, timed per launch with HIP events
    prof_plan = ntt.Plan(w.dims, w.target_ranks, w.iters, eps=w.eps, seed=w.seed,
                         flags=ntt.NTT_PROFILE)
    rep = ntt.ntt_decompose(prof_plan, stream, ws.data_ptr(), A.data_ptr(), core_ptrs)
    m1, k1, r1 = shapes[0]
    bytes_per_launch = 4.0 * m1 * k1 + 8.0 * r1 * k1 + 4.0 * m1 * r1
    pass_ms = rep["pass_ms"][0]
    achieved = bytes_per_launch / (pass_ms * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": gflop / (ms * 1e-3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.note}", "dims": list(w.dims), "ranks": eff,
                   "mu_iters_per_stage": w.iters, "precision": "fp32", "eps": w.eps},
        "decomps_per_s": 1e3 / ms,
        "gflop_per_step": gflop,
        "rel_error": err,
        "stage_ms": rep_graph["ms"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": profiled_traffic("k_mu_pass_r8m<32>", w.name),
                     "kernel": f"k_mu_pass_r8m<32> stage 1 ({m1}x{k1}, r={r1})",
                     "pass_ms": pass_ms, "bytes_per_launch": bytes_per_launch},
    }
    extras = [] if args.no_extras else [e for e in args.extras.split(",") if e]
    unknown = [e for e in extras if e not in EXTRAS]
    if unknown:
        raise SystemExit(f"unknown extras {unknown}; choose from {', '.join(EXTRAS)}")
    if extras:
        del A
        torch.cuda.empty_cache()
    if "precision_mode" in extras:
        out["precision_mode"] = precision_mode(ntt, S, torch, 0.0 if args.no_cpu_baseline else 8.0)
        torch.cuda.empty_cache()
    if "paper_workload" in extras:
        out["paper_workload"] = paper_workload(ntt, S, torch)
        torch.cuda.empty_cache()
    if "rank_rule" in extras:
        out["rank_rule"] = rank_rule(ntt, S, torch)
        torch.cuda.empty_cache()
    if "bcd" in extras:
        out["bcd"] = bcd(ntt, S, torch, err, ms)
        torch.cuda.empty_cache()
    if "streamed" in extras:
        out["streamed"] = streamed(ntt, S, torch)
        torch.cuda.empty_cache()
    if "batched" in extras:
        out["batched"] = batched(ntt, S, torch)
        torch.cuda.empty_cache()
    if "serving" in extras:
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        out["serving"] = serving_both(ntt, S, torch, args.serve_requests, args.serve_max_mb, rates)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A_host, w, args.cpu_seconds,
                                           4.0 if "bcd" in extras else 0.0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
