#!/usr/bin/env python3
"""Benchmark: time to feasibility gap <= 1e-6, multilevel vs plain, on one MI355X.

Headline workload (default): compressive PCP, 2000 x 2000, rank-50 Gaussian low-rank
part, 10% corruptions U[-10, 10], 60% of entries observed, 3 levels (n_H = 250),
float32 data (Gram accumulated and eigensolved in float64).

One step = one complete multilevel solve from the initial point to FG <= 1e-6
(every step of the hot path: restriction, coarse Gram, eigensolve, coarse SVT,
prolongation, fused soft threshold / mask / dual step / feasibility gap).
The plain method (levels = 0, the same kernels with R = I) is timed on the same
input for the speedup.  Inputs are resident in HBM before the timed region.
The speedup is a time to the same feasibility gap, not to the same recovery: the
relative errors of L and S against the generating L0 and S0 at the stop are
reported beside it for both methods (on Q for S in the compressive workloads).

The default line also carries, under "configs", the two tall workloads at their own
precision and at float32: the 76800 x 400 video stand-in (bf16 tiers, as its
workload states: bfloat16 GEMMs) and the 262144 x 200 hyperspectral stand-in
(bf16x3: split-bfloat16 compensated products), each multilevel vs plain with
iterations, ranks, recovery errors and the roofline of its dominant kernel; the
achieved HBM bandwidth of the standalone restrict, prolong and shrink at the
hyperspectral shape under "streaming"; and a short summary of the Frank-Wolfe
comparison (ML-FWT vs FW-T) under "fw".

Prints ONE JSON line.  Options: --steps K --warmup W --gpus N (N must be 1)
--workload {c1,c2,c3,c5,fw1,fw2,fw3,fw4} --no-plain --no-cpu --no-fw --no-configs --no-stream
--prec {fp32,bf16,bf16x3}.

The fw workloads measure the unconstrained-CPCP solvers of the Frank-Wolfe comparison
(Table 2 sizes): one step = one ML-FWT solve to the 1e-3 tolerance (relative objective
change), beside FW-T on the same input.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-rel-err 1e-6 (s) & iters/s: multilevel vs plain PCP on 1 MI355X"

HBM_PEAK = 8.0e12          # bytes/s
FP64_PEAK = 78.6e12        # flop/s, dense FP64 (vector and matrix)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16", "bf16x3"],
                    help="arithmetic of the coarse SVT's Gram and reconstruction products")
    ap.add_argument("--no-fw", action="store_true", help="skip the Frank-Wolfe summary of the default line")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the tall workloads (c3, c5) of the default line")
    ap.add_argument("--config-steps", type=int, default=3, help="timed multilevel solves per tall-workload entry")
    ap.add_argument("--no-stream", action="store_true", help="skip the streaming-kernel bandwidth summary")
    ap.add_argument("--stream-only", action="store_true",
                    help="measure only the standalone streaming entry points (restrict, prolong, shrink) and print "
                         "their bandwidth summary as one JSON line")
    ap.add_argument("--rnorm", type=int, default=0, choices=[0, 1, 2],
                    help="restriction normalisation of the multilevel solve: 0 orthonormal, 1 P/||P||_2, 2 P "
                         "(ablation; the plain solve is unaffected)")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="run one elementwise copy of MIB MiB (read MIB, write MIB) before the solves, "
                         "the reference kernel for scaling HBM byte counters")
    return ap.parse_args()


def describe(w):
    import paper_2206_13369_amd as mlp
    masked = w.Q is not None
    kind = "CPCP" if masked else "PCP"
    obs = f", {w.Q.mean():.0%} observed" if masked else ""
    return (f"{w.name}: {kind} {w.m}x{w.n}, rank {w.rank}{obs}, {w.levels} levels "
            f"(n_H={mlp.coarse_dim(w.n, w.levels)}), FG<=1e-6; {w.recipe}")


def recovery_errors(w, r, dev):
    """Relative Frobenius errors of the returned L and S against the generating L0 and
    S0 (S on the observed entries for the compressive problem: off Q it is not
    identifiable), computed on the device outside the timed region."""
    import torch
    L0 = torch.from_numpy(w.L0).to(dev)
    S0 = torch.from_numpy(w.S0).to(dev)
    L = r.L.double()
    S = r.S.double()
    if w.Q is not None:
        Q = torch.from_numpy(w.Q).to(dev)
        S0 = torch.where(Q, S0, torch.zeros_like(S0))
    eL = float(torch.linalg.norm(L - L0) / torch.linalg.norm(L0))
    eS = float(torch.linalg.norm(S - S0) / torch.linalg.norm(S0))
    del L0, S0, L, S
    return round(eL, 6), round(eS, 6)


def algorithmic_work(cls, w, nH, plain, sweeps, msvt=None):
    """(bound, amount per launch) of the method's own work for one launch of a kernel
    class: HBM bytes the kernel must move ("hbm"), or float64 flops ("mfma" for the
    matrix-core products, "alu" for the latency-bound Jacobi rounds).  `sweeps` is the
    per-iteration Jacobi sweep count of the solve; `msvt` = (products, launches) of the
    matrix-function SVT's product kernel in one solve."""
    m, n = w.m, w.n
    masked = w.Q is not None
    k = n if plain else nH
    if cls == "epilogue":
        # read D, read state, write state, (mask bits), read M_P, write next M_P
        return "hbm", 12.0 * m * n + 8.0 * m * k + (m * n / 8.0 if masked else 0.0)
    if cls == "init_restrict":
        return "hbm", 4.0 * m * n + 4.0 * m * k + (m * n / 8.0 if masked else 0.0)
    if cls == "finalize":
        return "hbm", 16.0 * m * n + 4.0 * m * k
    if cls == "gram":
        # G = M_P^T M_P on float64 MFMA: 2 m k^2 flops over 4 m k bytes; the bound is
        # whichever side of the float64 ridge (9.8 flop/B) the intensity k/2 falls on
        flops, byts = 2.0 * m * k * k, 4.0 * m * k
        return ("mfma", flops) if flops / byts > FP64_PEAK / HBM_PEAK else ("hbm", byts)
    if cls == "msvt_mm":
        # N x N x N float64 products (N = n_H padded to 64), one or two per launch
        if not msvt or not msvt[1]:
            return None, None
        N = int(math.ceil(k / 64.0)) * 64
        return "mfma", 2.0 * N ** 3 * msvt[0] / msvt[1]
    sw = (sum(sweeps) / len(sweeps)) if sweeps else 0.0
    if cls == "coarse_svt_small":
        # rounds of the circle method: ne/2 rotations; each 2x2 tile of A (ne/2)^2 tiles,
        # 24 flops; each (row, pair) of the factor ne * ne/2 items, 6 flops; plus six
        # 64^3 float64 MFMA products (C G C, warm start, T = C W, K = T T^T)
        ne = k + (k & 1)
        per_round = (ne // 2) ** 2 * 24.0 + ne * (ne // 2) * 6.0
        return "alu", sw * (ne - 1) * per_round + 6 * 2.0 * 64 ** 3
    N = int(math.ceil(k / 64.0)) * 64
    npairs = N // 64
    if cls == "jacobi_apply":
        # off-diagonal A tiles (two 64^3 products) + V tiles (one), float64
        return "mfma", 2.0 * (2 * 64 ** 3) * (npairs * (npairs - 1) // 2) + 2.0 * 64 ** 3 * (N // 64) * npairs
    if cls == "jacobi_pairs":
        # 32 rounds of 32 rotations on a 64x64 block and its 64x64 factor
        return "alu", npairs * 32 * 32 * (64 * 6 + 64 * 6)
    return None, None


def fw_pass_bytes(w, nH, plain):
    """Algorithmic HBM bytes of one Frank-Wolfe pass over the data: read D and the mask
    bits; ML-FWT reads and writes the coarse state Z and writes the restricted gradient
    (m x n_H each); FW-T reads and writes the dense L and writes the gradient."""
    m, n = w.m, w.n
    bits = m * n / 8.0 if w.Q is not None else 0.0
    if plain:
        return 4.0 * m * n * 4 + bits
    return 4.0 * m * n + bits + 12.0 * m * nH


def fw_bench(w, dev, steps, plain=True, cpu=True):
    """ML-FWT (and FW-T) solves to the 1e-3 tolerance on a resident input: time per solve,
    iterations, per-kernel breakdown, the roofline of the ML pass, the oracle's time."""
    import numpy as np
    import torch

    import paper_2206_13369_amd as mlp
    D = torch.from_numpy(w.D).to(dev)
    Q = torch.from_numpy(w.Q.astype(np.uint8)).to(dev)
    nH = mlp.coarse_dim(w.n, w.levels)

    def run(levels, ws):
        return mlp.cpcp_fwt(D, Q, w.lam_L, w.lam, levels=levels, tol=w.tol, workspace=ws, history=1000)

    ws = torch.empty(mlp.fwt_workspace_bytes(w.m, w.n, w.levels, True), dtype=torch.uint8, device=dev)
    run(w.levels, ws)   # warm-up
    torch.cuda.synchronize()
    mlp.profile_enable(True)
    run(w.levels, ws)
    torch.cuda.synchronize()
    prof = {k: v for k, v in mlp.profile_read().items() if v[0] > 0}
    mlp.profile_enable(False)
    t0 = time.perf_counter()
    for _ in range(steps):
        r = run(w.levels, ws)
    torch.cuda.synchronize()
    ml_s = (time.perf_counter() - t0) / steps
    mlp.profile_enable(["fw_pass"])
    for _ in range(steps):
        run(w.levels, ws)
    torch.cuda.synchronize()
    pl, pms = mlp.profile_read()["fw_pass"]
    mlp.profile_enable(False)
    roof = roofline("fw_pass", "hbm", fw_pass_bytes(w, nH, False), pms / 1e3 / max(pl, 1), pl)
    if roof is not None:
        roof["traffic"] = measured_traffic(w.name, "fw_pass")
    out = dict(workload=f"{w.name}: CPCP {w.m}x{w.n}, rank {w.rank}, {w.Q.mean():.0%} observed, "
                        f"{w.levels} levels (n_H={nH}), to 1e-3 relative objective change; {w.recipe}",
               ml_time_s=round(ml_s, 6), ml_iters=r.iters, ml_f=r.f,
               ml_ms_per_iter=round(ml_s * 1e3 / max(r.iters, 1), 4),
               ml_kernel_ms_per_solve={k: round(v[1], 4) for k, v in prof.items()},
               ml_launches_per_solve={k: v[0] for k, v in prof.items()},
               roofline=roof)
    del ws
    if plain:
        wsp = torch.empty(mlp.fwt_workspace_bytes(w.m, w.n, 0, True), dtype=torch.uint8, device=dev)
        mlp.profile_enable(True)
        rp = run(0, wsp)
        torch.cuda.synchronize()
        pprof = {k: v for k, v in mlp.profile_read().items() if v[0] > 0}
        mlp.profile_enable(False)
        t0 = time.perf_counter()
        rp = run(0, wsp)
        torch.cuda.synchronize()
        pl_s = time.perf_counter() - t0
        pw = pprof.get("fw_power", (0, 0.0))
        out.update(plain_time_s=round(pl_s, 6), plain_iters=rp.iters, plain_f=rp.f,
                   plain_ms_per_iter=round(pl_s * 1e3 / max(rp.iters, 1), 4),
                   plain_power_steps=rp.power_steps,
                   plain_us_per_power_step=round(pw[1] * 1e3 / max(rp.power_steps, 1), 2),
                   plain_kernel_ms_per_solve={k: round(v[1], 4) for k, v in pprof.items()},
                   speedup_vs_plain=round(pl_s / ml_s, 2),
                   per_iter_speedup=round((pl_s / max(rp.iters, 1)) / (ml_s / max(r.iters, 1)), 2))
        del wsp
    if cpu:
        import oracle.fwt as ofw
        try:
            from threadpoolctl import threadpool_info
            cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
        except Exception:
            cores = os.cpu_count()
        K = 2
        tc0 = time.perf_counter()
        ofw.fwt(w.D, w.lam_L, w.lam, Q=w.Q, levels=w.levels, fixed_iters=K)
        tc = time.perf_counter() - tc0
        out["cpu_baseline"] = dict(value=round(tc / K * r.iters, 3), unit="s", cores=cores, kind="oracle",
                                   sample=f"{K} ML-FWT iterations of the FP64 oracle on the same input "
                                          f"({tc:.2f} s), scaled to the GPU's {r.iters} iterations")
    return out


def stream_bench(dev, m=262144, n=200, levels=4, reps=10):
    """Achieved HBM bandwidth of the standalone streaming entry points (restrict, prolong,
    shrink) at the hyperspectral workload's shape.  The 210 MB operand fits the 256 MB
    Infinity Cache, so back-to-back launches read it partly from there; the HBM figure is
    the median of `reps` single launches each preceded by a read of a 768 MiB buffer
    (clean lines only, so the timed launch evicts without write-backs), timed by events
    on the stream the library launches on (torch's current stream).  Algorithmic bytes =
    what each call must read and write once.  The back-to-back (cache-warm) rate is
    reported beside it."""
    import torch

    import paper_2206_13369_amd as mlp
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    X = torch.randn((m, n), generator=g, device=dev, dtype=torch.float32)
    nH = mlp.coarse_dim(n, levels)
    XH = mlp.restrict(X, levels)
    Y = torch.empty_like(X)
    flush = torch.ones(768 * 1024 * 1024 // 4, device=dev, dtype=torch.float32)
    sink = torch.empty(1, device=dev, dtype=torch.float32)
    cases = {
        "restrict": (lambda: mlp.restrict(X, levels), 4.0 * m * n + 4.0 * m * nH),
        "prolong": (lambda: mlp.prolong(XH, n, levels), 4.0 * m * nH + 4.0 * m * n),
        "shrink": (lambda: mlp.shrink(X, 0.5, out=Y), 8.0 * m * n),
        "copy (torch, reference)": (lambda: Y.copy_(X), 8.0 * m * n),
    }
    out = {"shape": f"{m}x{n}, {levels} levels (n_H={nH})", "timing": "cold: one launch after a 768 MiB read; "
           "warm: mean of back-to-back launches"}
    for name, (fn, byts) in cases.items():
        for _ in range(3):
            fn()
        ts = []
        for _ in range(reps):
            torch.sum(flush, 0, out=sink[0])
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        t = sorted(ts)[len(ts) // 2]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(2 * reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        tw = e0.elapsed_time(e1) / 1e3 / (2 * reps)
        out[name] = dict(avg_launch_us=round(t * 1e6, 2), algorithmic_bytes=byts,
                         achieved_GBps=round(byts / t / 1e9, 1), frac=round(byts / t / HBM_PEAK, 4),
                         warm_launch_us=round(tw * 1e6, 2), warm_GBps=round(byts / tw / 1e9, 1))
    del X, XH, Y, flush
    torch.cuda.empty_cache()
    return out


def sources_sha256():
    """Hash of the kernel sources: HBM traffic measured for other sources is not reused."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2206_13369_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(csrc, name), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "mlpcp.h"), "rb").read())
    return h.hexdigest()


def measured_traffic(workload, cls):
    """HBM bytes per launch of a kernel class from the rocprofv3 FETCH_SIZE / WRITE_SIZE
    runs recorded in profiles/hbm_traffic.json, if they were taken on these sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    data = json.load(open(path))
    if data.get("sources_sha256") != sources_sha256():
        return None
    return data.get("workloads", {}).get(workload, {}).get(cls)


def roofline(cls, bound, amount, avg_s, launches):
    if bound is None or not launches:
        return None
    if bound == "hbm":
        ach = amount / avg_s / 1e9
        return dict(bound="hbm", achieved=round(ach, 2), peak=HBM_PEAK / 1e9, unit="GB/s",
                    frac=round(ach / (HBM_PEAK / 1e9), 4), traffic=None, kernel=cls,
                    avg_launch_us=round(avg_s * 1e6, 2), launches=launches, algorithmic_bytes_per_launch=amount)
    ach = amount / avg_s / 1e12
    return dict(bound=bound, achieved=round(ach, 4), peak=FP64_PEAK / 1e12, unit="TFLOP/s",
                frac=round(ach / (FP64_PEAK / 1e12), 5), traffic=None, kernel=cls,
                avg_launch_us=round(avg_s * 1e6, 2), launches=launches, algorithmic_flops_per_launch=amount)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {a.gpus} is not supported (the solver is single-GPU; "
              "the multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2206_13369_amd as mlp
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if a.stream_only:
        if a.calib_copy:
            src = torch.ones(a.calib_copy << 18, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            torch.mul(src, 1.0, out=dst)
            torch.cuda.synchronize()
            del src, dst
        print(json.dumps({"streaming": stream_bench(dev)}))
        return
    if a.workload.startswith("fw"):
        w = synth.fw_config(a.workload)
        if a.calib_copy:
            src = torch.ones(a.calib_copy << 18, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            torch.mul(src, 1.0, out=dst)
            torch.cuda.synchronize()
            del src, dst
        fb = fw_bench(w, dev, a.steps, plain=not a.no_plain, cpu=not a.no_cpu)
        out = {
            "metric": "time to 1e-3 (s): multilevel FW-T (ML-FWT) vs FW-T, unconstrained CPCP, 1 MI355X",
            "value": fb["ml_time_s"], "unit": "s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "ms_per_step": round(fb["ml_time_s"] * 1e3, 4), "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": fb.pop("workload")},
            "roofline": fb.pop("roofline"), "cpu_baseline": fb.pop("cpu_baseline", None),
        }
        out.update(fb)
        print(json.dumps(out))
        return
    t_gen = time.time()
    w = synth.config(a.workload)
    t_gen = time.time() - t_gen
    print(f"[bench] workload {w.name} {w.m}x{w.n} generated in {t_gen:.1f}s", file=sys.stderr, flush=True)
    if a.calib_copy:
        src = torch.ones(a.calib_copy << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    hb = ialm_bench(w, dev, a.steps, a.warmup, a.prec, plain=not a.no_plain, plain_steps=a.plain_steps,
                    rnorm=a.rnorm, tol=a.tol)
    ml_s = hb["time_s"]

    cpu = None
    if not a.no_cpu:
        import oracle
        try:
            from threadpoolctl import threadpool_info
            cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
        except Exception:
            cores = os.cpu_count()
        tc0 = time.perf_counter()
        ref = oracle.ialm(w.D, w.lam, w.mu0, Q=w.Q, levels=w.levels, tol=a.tol, max_iter=60)
        tc1 = time.perf_counter()
        cpu = dict(value=round(tc1 - tc0, 3), unit="s", cores=cores, kind="oracle",
                   sample=f"one full multilevel FP64 oracle solve of the same input to FG<=1e-6 "
                          f"({ref.iters} iterations, {ref.iters/(tc1-tc0):.2f} iters/s)",
                   iters=ref.iters)
        print(f"[bench] oracle: {tc1-tc0:.2f}s, {ref.iters} iters", file=sys.stderr, flush=True)

    configs = None
    if not a.no_configs and a.workload == "c2":
        configs = {}
        for name, prec in (("c3", "bf16"), ("c5", "bf16x3")):
            wc = synth.config(name)
            entry = {"workload": describe(wc)}
            for pr in (prec, "fp32"):
                r = ialm_bench(wc, dev, a.config_steps, 1, pr, plain=not a.no_plain, plain_steps=1, tol=a.tol,
                               breakdown=False)
                r.pop("kernel_ms_per_solve", None)
                r.pop("launches_per_solve", None)
                r.pop("plain_kernel_ms_per_solve", None)
                r.pop("kernel_rooflines", None)
                entry[pr] = r
            configs[name] = entry
            del wc
            torch.cuda.empty_cache()

    streaming = None
    if not a.no_stream and a.workload == "c2":
        streaming = stream_bench(dev)
        print(f"[bench] streaming kernels (cold / cache-warm): " + ", ".join(
            f"{k} {v['achieved_GBps']} / {v['warm_GBps']} GB/s" for k, v in streaming.items() if isinstance(v, dict)),
            file=sys.stderr, flush=True)

    fw = None
    if not a.no_fw and a.workload == "c2":
        wf = synth.fw_config("fw2")
        fw = fw_bench(wf, dev, 3, plain=not a.no_plain, cpu=False)
        print(f"[bench] fw2 ML-FWT {fw['ml_time_s']*1e3:.2f} ms ({fw['ml_iters']} iters), FW-T "
              f"{fw.get('plain_time_s', float('nan'))*1e3:.2f} ms", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": round(ml_s, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ml_s * 1e3, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.prec == "fp32" else a.prec + "/f32",
        "restriction": ["orthonormal P (P^T P)^-1/2", "P / ||P||_2", "P"][a.rnorm],
        "data": "synthetic",
        "config": {"workload": describe(w)},
        "speedup_basis": "time to the same feasibility gap FG <= 1e-6 (Sec. 4 stopping measure), not to the same "
                         "recovery; err_L0 / err_S0 give each method's relative error to the generating L0, S0",
    }
    out.update({k: v for k, v in hb.items() if k not in ("time_s",)})
    out["roofline"] = out.pop("roofline")
    out["cpu_baseline"] = cpu
    out["configs"] = configs
    out["streaming"] = streaming
    out["fw"] = fw
    print(json.dumps(out))


def ialm_bench(w, dev, steps, warmup, prec, *, plain=True, plain_steps=1, rnorm=0, tol=1e-6, breakdown=True):
    """Multilevel (and plain) solves of one workload to FG <= tol on a resident input:
    mean time per solve over `steps` timed solves, iterations, ranks, recovery errors,
    the per-kernel breakdown of one solve and the roofline of its dominant kernel."""
    import numpy as np
    import torch

    import paper_2206_13369_amd as mlp
    D = torch.from_numpy(w.D).to(dev)
    Q = torch.from_numpy(w.Q.astype(np.uint8)).to(dev) if w.Q is not None else None
    nH = mlp.coarse_dim(w.n, w.levels)

    def run(levels, ws, pr=prec):
        kw = dict(levels=levels, tol=tol, max_iter=500, want_y=False, workspace=ws, history=600, prec=pr,
                  r_norm=rnorm if levels > 0 else 0)
        if Q is None:
            return mlp.pcp_solve(D, w.lam, w.mu0, **kw)
        return mlp.cpcp_solve(D, Q, w.lam, w.mu0, **kw)

    ws_ml = torch.empty(mlp.workspace_bytes(w.m, w.n, mlp.default_opts(levels=w.levels)), dtype=torch.uint8,
                        device=dev)
    for i in range(max(warmup, 1)):
        r = run(w.levels, ws_ml)
        print(f"[bench] {w.name} {prec} warmup {i}: iters {r.iters} fg {r.fg:.2e}", file=sys.stderr, flush=True)
    # per-kernel breakdown of one solve (every launch bracketed by events)
    torch.cuda.synchronize()
    mlp.profile_enable(True)
    run(w.levels, ws_ml)
    torch.cuda.synchronize()
    prof = mlp.profile_read()
    mlp.profile_enable(False)
    kernel_ms = {k: round(v[1], 4) for k, v in prof.items() if v[0] > 0}
    launches = {k: v[0] for k, v in prof.items() if v[0] > 0}
    dom = max(kernel_ms.items(), key=lambda kv: kv[1])[0]

    # timed region: `steps` solves, no instrumentation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(steps):
        results.append(run(w.levels, ws_ml))
    torch.cuda.synchronize()
    ml_s = (time.perf_counter() - t0) / steps
    r = results[-1]
    del results
    eL, eS = recovery_errors(w, r, dev)
    print(f"[bench] {w.name} {prec} multilevel: {ml_s*1e3:.2f} ms/solve, {r.iters} iters, fg {r.fg:.2e}, "
          f"rank {r.rank}, errL0 {eL:.3g}, errS0 {eS:.3g}; dominant kernel {dom}; Gram bf16/split iters "
          f"{r.gram_bf16_iters}/{r.gram_split_iters}; partial-eigensolve iters {r.partial_eig_iters}; "
          f"matrix-function SVT iters {r.msvt_iters} ({r.msvt_products} products, flags {r.msvt_flags})",
          file=sys.stderr, flush=True)

    # the same solves with HIP events around the dominant kernel class only
    torch.cuda.synchronize()
    mlp.profile_enable([dom])
    ti0 = time.perf_counter()
    for _ in range(steps):
        run(w.levels, ws_ml)
    torch.cuda.synchronize()
    inst_s = (time.perf_counter() - ti0) / steps
    dom_launches, dom_ms = mlp.profile_read()[dom]
    mlp.profile_enable(False)
    del ws_ml

    out = dict(time_s=ml_s, prec=prec, iters=r.iters, iters_per_s=round(r.iters / ml_s, 2), fg=r.fg, rank=r.rank,
               err_L0=eL, err_S0=eS, tau_margin=r.tau_margin, partial_eig_iters=r.partial_eig_iters,
               msvt_iters=r.msvt_iters, msvt_products=r.msvt_products,
               gram_tiers={"bf16": r.gram_bf16_iters, "split": r.gram_split_iters})
    if plain:
        ws_pl = torch.empty(mlp.workspace_bytes(w.m, w.n, mlp.default_opts(levels=0)), dtype=torch.uint8,
                            device=dev)
        torch.cuda.synchronize()
        mlp.profile_enable(True)       # warm-up solve, also the plain kernel breakdown
        rp = run(0, ws_pl)
        torch.cuda.synchronize()
        pprof = mlp.profile_read()
        mlp.profile_enable(False)
        tp0 = time.perf_counter()
        for _ in range(plain_steps):
            rp = run(0, ws_pl)
        torch.cuda.synchronize()
        plain_s = (time.perf_counter() - tp0) / plain_steps
        peL, peS = recovery_errors(w, rp, dev)
        print(f"[bench] {w.name} {prec} plain: {plain_s*1e3:.1f} ms/solve, {rp.iters} iters, fg {rp.fg:.2e}, "
              f"rank {rp.rank}, errL0 {peL:.3g}, errS0 {peS:.3g}; partial-eigensolve iters {rp.partial_eig_iters}; "
              f"matrix-function SVT iters {rp.msvt_iters}",
              file=sys.stderr, flush=True)
        out.update(plain_time_s=round(plain_s, 5), plain_iters=rp.iters,
                   plain_iters_per_s=round(rp.iters / plain_s, 3), plain_rank=rp.rank, plain_fg=rp.fg,
                   plain_err_L0=peL, plain_err_S0=peS, speedup_vs_plain=round(plain_s / ml_s, 2),
                   plain_partial_eig_iters=rp.partial_eig_iters, plain_msvt_iters=rp.msvt_iters,
                   plain_kernel_ms_per_solve={k: round(v[1], 3) for k, v in pprof.items() if v[0] > 0})
        del ws_pl, rp

    sweeps = r.sweeps_history
    msvt = (r.msvt_products, launches.get("msvt_mm", 0))
    bound, amount = algorithmic_work(dom, w, nH, False, sweeps, msvt)
    roof = roofline(dom, bound, amount, dom_ms / 1e3 / max(dom_launches, 1), dom_launches)
    if roof is not None:
        roof["traffic"] = measured_traffic(w.name, dom)
    others = {}
    for cls in kernel_ms:
        bd, am = algorithmic_work(cls, w, nH, False, sweeps, msvt)
        rf = roofline(cls, bd, am, kernel_ms[cls] / 1e3 / launches[cls], launches[cls])
        if rf is not None:
            others[cls] = {k: rf[k] for k in ("bound", "achieved", "unit", "frac", "avg_launch_us")}
            others[cls]["traffic"] = measured_traffic(w.name, cls)
    out.update(instrumented_ms_per_step=round(inst_s * 1e3, 4), kernel_ms_per_solve=kernel_ms,
               launches_per_solve=launches, sweeps_per_iteration=sweeps, kernel_rooflines=others, roofline=roof)
    del r, D, Q
    return out


if __name__ == "__main__":
    main()
