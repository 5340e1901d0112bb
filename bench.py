"""Benchmark: Gibbs sweeps per second of the Horseshoe Probit sampler on one
MI355X, at N = 1,000,000 rows and p = 1000 predictors.

One step = one full Gibbs sweep (z | beta over all rows fused with X^T z;
lambda, tau; the float64 Cholesky draw of beta; nu, xi; the draw record).
Inputs are seeded synthetic data (the paper's Section 6.1 design with an
intercept and 10 nonzero coefficients) resident in HBM before timing starts.

Prints one JSON line.  `value` is the float32-X sweep rate (X is 4.0 GB); the
line also carries
  roofline      the sweep kernel (one fused launch per sweep; its z pass is the
                N x p stream): algorithmic bytes per launch (N p 4 + N) over
                its mean duration from HIP events on the library's stream,
                against the 8 TB/s HBM peak; traffic = hardware-counted HBM
                bytes per launch while the stored counter reading matches the
                current kernel sources (else null)
  bf16          the same workload with X stored in bfloat16 (2.0 GB): its own
                sweep rate and roofline (N p 2 + N bytes per launch)
  batch         the batched form: 64 uneven float32 datasets (one chain each)
                plus 16 chains sharing the N = 1e6, p = 1000 bfloat16 design,
                one graph replay per batched sweep: chain-sweeps/s batched and
                the same chains swept one at a time, with the roofline of the
                whole batched sweep (one read of every distinct design)
  rare_event    the stand-in for the data of Section 6.2 (N = 1,295,848,
                p = 141, mean outcome 0.0048): 10,000 sweeps (2,500 burn-in) as
                the paper ran, with the lag-1 autocorrelation and effective
                sample size of the coefficients and the truncated-normal
                branch mix
  large_p       N = 1e6, p = 1e4 (40 GB float32 X, generated on the GPU):
                sweeps/s and the fraction of the FP64 matrix-core peak its
                factorisation and passes reach
  streamed      the same float32 workload with X in pinned host memory,
                streamed through the GPU every sweep: its rate against the
                measured host-to-device link
  read_ceiling  a plain streaming read of the same X (16-byte non-temporal
                loads, nothing else) on this GPU: what the z pass could reach
  cpu_baseline  the float64 oracle timed on this host on a bounded sample of
                the same workload (whole sweeps), all cores and one thread
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gibbs sweeps/sec and HBM GB/s at N=1e6,p=1000; chain-sweeps/sec batched vs plain"
HBM_PEAK_GBPS = 8000.0
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--N", type=int, default=1_000_000)
    ap.add_argument("--p", type=int, default=1000)
    ap.add_argument("--only", choices=["f32", "bf16", "batch", "rare", "streamed", "large_p"], default=None,
                    help="run one form only and print its own line (for profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="built-in launch shapes (no autotuner)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--traffic-json", default=TRAFFIC_JSON)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device twice (a plain copy kernel of known "
                         "size, to scale hardware byte counters)")
    return ap.parse_args()


def kernel_fingerprint():
    """Hash of the library's sources with comments and layout removed: stored
    counter readings apply only to the same code, whatever its comments say."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1608_04329_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(csrc, name), encoding="utf-8") as f:
                text = f.read()
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
            text = " ".join(text.split())
            h.update(name.encode() + b"\0" + text.encode())
    return h.hexdigest()[:16]


def stored_traffic(path, workload):
    """Counted HBM bytes per launch (or per batched sweep) for this workload,
    if they were taken at the current kernel sources."""
    try:
        with open(path) as f:
            t = json.load(f).get(workload)
    except (OSError, ValueError):
        return None
    if not t or t.get("kernel_fingerprint") != kernel_fingerprint():
        return None
    return t.get("bytes")


def roofline(bytes_per_launch, ms, traffic):
    achieved = bytes_per_launch / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic}


def host_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    ram = round(int(line.split()[1]) / 2**20, 1)
                    break
    except OSError:
        pass
    return model, os.cpu_count(), ram


def cpu_baseline(d, seconds):
    """Whole oracle sweeps on the same data, on all host cores and on one."""
    import numpy as np
    from oracle import oracle as orc
    # one-time Gram in float64 (untimed, like the GPU's creation step)
    G = np.zeros((d.p, d.p))
    step = 1 << 16
    for r in range(0, d.N, step):
        xb = d.X[r:r + step].astype(np.float64)
        G += xb.T @ xb

    def time_sweeps(threads, budget):
        orc.set_threads(threads)
        ch = orc.Chain(d.p)
        n = 0
        t0 = time.perf_counter()
        while True:
            ch.sweep_once(d.X, d.y, G, seed=1)
            n += 1
            el = time.perf_counter() - t0
            if el >= budget or n >= 200:
                return n, el

    model, nproc, ram = host_info()
    threads = max(1, min(nproc or 1, orc.max_threads()))
    na, ea = time_sweeps(threads, seconds / 2)
    n1, e1 = time_sweeps(1, seconds / 2)
    orc.set_threads(threads)
    return {"value": round(na / ea, 4), "unit": "sweeps/s", "cores": threads, "kind": "oracle",
            "sample": f"{na} whole float64 oracle sweeps of the same N={d.N}, p={d.p} float32 workload "
                      f"from the cold start on {threads} threads (OpenMP over rows; the p-side is "
                      f"serial), {ea:.1f} s; Gram formed beforehand (untimed)",
            "single_thread": {"value": round(n1 / e1, 4), "cores": 1,
                              "sample": f"{n1} sweeps on one thread, {e1:.1f} s"},
            "cpu_model": model, "nproc": nproc, "ram_gb": ram}


def run_single(a, d, x_type, traffic_path):
    """One chain on design d with X stored as x_type: sweeps/s and the roofline
    of the sweep kernel."""
    import torch

    from paper_1608_04329_amd import hsp
    t0 = time.perf_counter()
    s = hsp.Sampler(d.X, d.y, seed=1, x_type=x_type, max_draws=max(64, a.steps + a.warmup),
                    autotune=not a.no_tune)
    plan = s.plan()
    print(f"[bench] {x_type}: sampler created (X copied, Gram formed, launch plan {plan[4]}) in "
          f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    s.sweep(a.warmup)
    s.sync()
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.sweep(a.steps)
    s.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms, sweep_ms, _ = s.timing()
    clamps, maxatt = s.counters()
    s.set_timing(False)
    ceil_ms, ceil_bytes = hsp.hsp_read_ceiling(s.h, 10)
    s.close()
    esz = 4 if x_type == "f32" else 2
    nbytes = d.N * d.p * esz + d.N  # X once, y once
    workload = f"horseshoe_probit_gibbs_N{d.N}_p{d.p}_x{x_type}"
    print(f"[bench] {x_type}: {a.steps} sweeps in {elapsed:.3f}s; sweep kernel {kernel_ms:.4f} ms per "
          f"launch (events)", file=sys.stderr, flush=True)
    return {
        "workload": workload,
        "value": round(a.steps / elapsed, 3),
        "unit": "sweeps/s",
        "ms_per_step": round(1e3 * elapsed / a.steps, 5),
        "kernel_ms": round(kernel_ms, 5),
        "sweep_ms_events": round(sweep_ms, 5),
        "hbm_gbps": round(nbytes / (elapsed / a.steps) / 1e9, 1),
        "algorithmic_bytes_per_launch": nbytes,
        "read_ceiling": {"gbps": round(ceil_bytes / (ceil_ms * 1e-3) / 1e9, 1),
                         "ms_per_pass": round(ceil_ms, 5),
                         "kernel": "plain 16-byte non-temporal streaming read of the same X"},
        "max_tn_proposals": int(maxatt),
        "lambda_clamps": int(clamps),
        "launch_plan": {"group_blocks": plan[0], "z_blocks": plan[1], "z_static_pct": plan[2],
                        "z_unit": plan[3], "chosen": plan[4]},
        "roofline": roofline(nbytes, kernel_ms, stored_traffic(traffic_path, workload)),
    }


def run_streamed(a, d, sweeps=20):
    """The same workload with X kept in pinned host memory and streamed through
    the GPU in row chunks every sweep (the form for designs beyond device
    memory): bound by the host-to-device link, reported against the link's
    own measured rate."""
    import torch

    from paper_1608_04329_amd import hsp
    t0 = time.perf_counter()
    s = hsp.Sampler(d.X, d.y, seed=1, max_draws=64, x_stream=True)
    print(f"[bench] streamed: sampler created (pinned copy, Gram) in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    s.sweep(2)
    s.sync()
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.sweep(sweeps)
    s.sync()
    elapsed = time.perf_counter() - t0
    _, sweep_ms, _ = s.timing()
    s.set_timing(False)
    link_ms, link_bytes = hsp.hsp_read_ceiling(s.h, 3)
    s.close()
    nbytes = d.N * d.p * 4 + d.N
    link_gbps = link_bytes / (link_ms * 1e-3) / 1e9
    achieved = nbytes / (sweep_ms * 1e-3) / 1e9
    return {
        "workload": f"horseshoe_probit_gibbs_N{d.N}_p{d.p}_xf32_streamed_from_host",
        "value": round(sweeps / elapsed, 3), "unit": "sweeps/s", "sweeps": sweeps,
        "ms_per_step": round(1e3 * elapsed / sweeps, 4),
        "link_gbps_measured": round(link_gbps, 1),
        "roofline": {"bound": "host-to-device link", "achieved": round(achieved, 1), "peak": round(link_gbps, 1),
                     "unit": "GB/s", "frac": round(achieved / link_gbps, 4), "traffic": None,
                     "peak_source": "plain host-to-device copies of the same pinned X, measured in this run"},
    }


def run_large_p(a, N=1_000_000, p=10_000, sweeps=20):
    """The point the paper could not run (Sections 6.1 and 7: N = 1e6,
    p = 1e4, a 40 GB float32 X): data generated on the GPU (X iid N(0,1) with
    an intercept column, 10 nonzero coefficients ~ U(-3, 3), probit y), the
    sweep timed as for the main workload.  Its floor is the float64
    factorisation (p^3 / 3 flops) as much as the pass over X."""
    import numpy as np
    import torch

    from paper_1608_04329_amd import hsp
    t0 = time.perf_counter()
    g = torch.Generator(device="cuda")
    g.manual_seed(14)
    X = torch.randn((N, p), generator=g, device="cuda", dtype=torch.float32)
    X[:, 0] = 1.0
    gc = torch.Generator()
    gc.manual_seed(14)
    idx = torch.randperm(p, generator=gc)[:10]
    beta_true = torch.zeros(p, dtype=torch.float32)
    beta_true[idx] = (torch.rand(10, generator=gc) * 6.0 - 3.0)
    eps = torch.randn(N, generator=g, device="cuda", dtype=torch.float32)
    y = ((X @ beta_true.cuda()) + eps > 0).to(torch.uint8)
    del eps
    torch.cuda.synchronize()
    print(f"[bench] large p: data N={N} p={p} generated on the GPU in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    s = hsp.Sampler(X, y, seed=1, max_draws=64, autotune=not a.no_tune)
    del X, y
    torch.cuda.empty_cache()
    plan = s.plan()
    print(f"[bench] large p: sampler created (copy, Gram, schedule, plan {plan[4]}) in "
          f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    s.sweep(3)
    s.sync()
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.sweep(sweeps)
    s.sync()
    elapsed = time.perf_counter() - t0
    kernel_ms, _, _ = s.timing()
    s.set_timing(False)
    betas, taus, _ = s.draws()
    s.close()
    nbytes = N * p * 4 + N
    flops = p ** 3 / 3.0 + 2.0 * p * p + 4.0 * N * p
    workload = f"horseshoe_probit_gibbs_N{N}_p{p}_xf32"
    hbm = roofline(nbytes, kernel_ms, stored_traffic(a.traffic_json, workload))
    fp64 = {"bound": "mfma", "achieved": round(flops / (kernel_ms * 1e-3) / 1e12, 2), "peak": 78.6,
            "unit": "TFLOP/s", "frac": round(flops / (kernel_ms * 1e-3) / 1e12 / 78.6, 4), "traffic": None,
            "flops_per_launch": flops, "flops_counted": "p^3/3 Cholesky + 2p^2 solves + 4Np for X beta and X^T z"}
    return {
        "workload": workload,
        "value": round(sweeps / elapsed, 3), "unit": "sweeps/s", "sweeps": sweeps,
        "ms_per_step": round(1e3 * elapsed / sweeps, 4), "kernel_ms": round(kernel_ms, 4),
        "launch_plan": {"group_blocks": plan[0], "z_blocks": plan[1], "chosen": plan[4]},
        "finite_draws": bool(np.isfinite(betas).all() and np.all(taus > 0)),
        "roofline": fp64 if fp64["frac"] >= hbm["frac"] else hbm,
        "roofline_hbm": hbm, "roofline_fp64": fp64,
    }


def ess_and_acf(x):
    """Lag-1 autocorrelation and effective sample size of each column of x
    (draws x coefficients): ESS = n / (1 + 2 sum_k rho_k), the sum cut by
    Geyer's initial monotone sequence of paired autocorrelations."""
    import numpy as np
    n = x.shape[0]
    xc = x - x.mean(0)
    f = np.fft.rfft(xc, n=2 * n, axis=0)
    acov = np.fft.irfft(f * np.conj(f), axis=0)[:n] / n
    rho = acov / np.maximum(acov[0], 1e-300)
    ess = np.empty(x.shape[1])
    for j in range(x.shape[1]):
        r = rho[:, j]
        pairs = r[0:n - 1:2] + r[1:n:2]
        m = np.argmax(pairs <= 0) if np.any(pairs <= 0) else pairs.size
        g = np.minimum.accumulate(pairs[:m]) if m else np.zeros(0)
        ess[j] = n / max(1e-12, -1.0 + 2.0 * g.sum())
    return rho[1], ess


def run_rare(a, sweeps=10_000, burn=2_500):
    """The rare-event stand-in for the data of Section 6.2 (N = 1,295,848,
    p = 141, mean outcome 0.0048): the paper's run length, mixing reported."""
    import numpy as np
    import torch

    import synth
    from paper_1608_04329_amd import hsp
    t0 = time.perf_counter()
    d = synth.rare_event()
    print(f"[bench] rare-event data generated in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    s = hsp.Sampler(d.X, d.y, seed=1, max_draws=sweeps, debug_store_z=True)
    s.sweep(2)
    s.sync()
    s.set_state(np.zeros(d.p), np.ones(d.p), np.ones(d.p), 1.0, 1.0, 0)
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.sweep(sweeps)
    s.sync()
    elapsed = time.perf_counter() - t0
    kernel_ms, _, _ = s.timing()
    s.set_timing(False)
    betas, taus, _ = s.draws()
    _, att, _ = s.debug()
    # Section 5's variant: rows reordered by y* x_i beta after burn-in, then
    # the same sweep timed again
    s.sort_rows()
    s.sweep(20)
    s.sync()
    s.set_timing(True)
    s.sweep(2000)
    s.sync()
    kernel_ms_sorted, _, _ = s.timing()
    s.close()
    gauss = (att & (1 << 30)) != 0
    rho1, ess = ess_and_acf(betas[burn:])
    nbytes = d.N * d.p * 4 + d.N
    workload = f"horseshoe_probit_rare_event_N{d.N}_p{d.p}_ybar{d.y.mean():.4f}_xf32"
    return {
        "workload": workload,
        "value": round(sweeps / elapsed, 2), "unit": "sweeps/s",
        "sweeps": sweeps, "burn_in": burn, "seconds_for_run": round(elapsed, 3),
        "kernel_ms": round(kernel_ms, 5),
        "roofline": roofline(nbytes, kernel_ms, stored_traffic(a.traffic_json, workload)),
        "acf_lag1": {"min": round(float(rho1.min()), 4), "median": round(float(np.median(rho1)), 4),
                     "max": round(float(rho1.max()), 4), "intercept": round(float(rho1[0]), 4)},
        "ess": {"min": round(float(ess.min()), 1), "median": round(float(np.median(ess)), 1),
                "intercept": round(float(ess[0]), 1)},
        "tn_gauss_branch_fraction": round(float(gauss.mean()), 5),
        "kernel_ms_rows_sorted": round(kernel_ms_sorted, 5),
        "intercept_posterior_mean": round(float(betas[burn:, 0].mean()), 4),
        "intercept_true": round(float(d.beta_true[0]), 4),
    }


def batch_data(big=None):
    """The 64 uneven datasets and the shared N = 1e6, p = 1000 design (big, if
    already generated: the same seeded design as the single-chain workload)."""
    import synth
    shapes = synth.batch_shapes(64, seed=1000)
    ds = [synth.batch_dataset(k, N, p) for k, (N, p) in enumerate(shapes)]
    if big is None:
        beta_true, _ = synth.sparse_beta(1000, 10, 13)
        big = synth.probit_design(1_000_000, 1000, beta_true, 13, True, "n1000000_p1000")
    return ds, big


def run_batch(a, traffic_path, data=None):
    """Chain-sweeps/s of the batched form against the same chains swept one by one."""
    import torch

    from paper_1608_04329_amd import hsp
    t0 = time.perf_counter()
    ds, big = data if data is not None else batch_data()
    print(f"[bench] batch data ready in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    datasets = [(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), "f32") for d in ds]
    datasets.append((torch.from_numpy(big.X).cuda(), torch.from_numpy(big.y).cuda(), "bf16"))
    counts = [1] * len(ds) + [16]
    b = hsp.Batch(datasets, counts, seed=1, max_draws=64, autotune=not a.no_tune)
    del datasets
    torch.cuda.empty_cache()
    nchains = len(b)
    b.sweep(a.warmup)
    b.sync()
    b.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.sweep(a.steps)
    b.sync()
    elapsed = time.perf_counter() - t0
    ms_ev, _ = b.timing()
    b.set_timing(False)
    bplan = b.plan()
    batched = nchains * a.steps / elapsed
    print(f"[bench] batch: {a.steps} sweeps of {nchains} chains in {elapsed:.3f}s "
          f"({ms_ev:.3f} ms per batched sweep by events)", file=sys.stderr, flush=True)
    # plain: every chain swept on its own, one after another
    t0 = time.perf_counter()
    for c in b.chains:
        c.sweep(a.steps)
    for c in b.chains:
        c.sync()
    elapsed_plain = time.perf_counter() - t0
    plain = nchains * a.steps / elapsed_plain
    b.close()
    # one read of every distinct design (and its y) per batched sweep
    nbytes = sum(d.N * d.p * 4 + d.N for d in ds) + big.N * big.p * 2 + big.N
    workload = "horseshoe_probit_batch_64uneven_f32_plus_16chains_N1e6_p1000_bf16"
    return {
        "workload": workload,
        "value": round(batched, 1),
        "unit": "chain-sweeps/s",
        "chains": nchains, "datasets": len(ds) + 1,
        "ms_per_step": round(1e3 * elapsed / a.steps, 4),
        "batched_sweep_ms_events": round(ms_ev, 4),
        "plain_chain_sweeps_per_s": round(plain, 1),
        "batched_over_plain": round(batched / plain, 3),
        "launch_plan": {"mc_blocks": bplan[0], "z_bandwidth_pct": bplan[1], "packs": bplan[2],
                        "chosen": bplan[3]},
        "algorithmic_bytes_per_step": nbytes,
        "roofline": roofline(nbytes, ms_ev, stored_traffic(traffic_path, workload)),
    }


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (several GPUs "
              "would each sweep a row shard of X and sum X^T z across them).", file=sys.stderr)
        sys.exit(2)
    import torch

    import synth

    torch.cuda.set_device(0)
    if a.copy_calibration:
        n = a.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 2 copies of {a.copy_calibration} MiB", file=sys.stderr,
              flush=True)
        del src, dst

    common = {"metric": METRIC, "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic"}
    if a.only == "batch":
        r = run_batch(a, a.traffic_json)
        out = dict(common, value=r["value"], unit=r["unit"], ms_per_step=r["ms_per_step"], dtype="f32+bf16",
                   config={"workload": r["workload"], "chains": r["chains"], "datasets": r["datasets"]},
                   roofline=r["roofline"], batch=r)
        print(json.dumps(out), flush=True)
        return

    if a.only == "large_p":
        r = run_large_p(a)
        out = dict(common, value=r["value"], unit=r["unit"], ms_per_step=r["ms_per_step"], dtype="f32+f64",
                   config={"workload": r["workload"]}, roofline=r["roofline"], large_p=r)
        out["steps"], out["warmup"] = r["sweeps"], 3
        print(json.dumps(out), flush=True)
        return

    if a.only == "rare":
        r = run_rare(a)
        out = dict(common, value=r["value"], unit=r["unit"], ms_per_step=round(1e3 / r["value"], 5),
                   dtype="f32", config={"workload": r["workload"]}, roofline=r["roofline"], rare_event=r)
        out["steps"], out["warmup"] = r["sweeps"], 0
        print(json.dumps(out), flush=True)
        return

    t0 = time.perf_counter()
    beta_true, _ = synth.sparse_beta(a.p, min(10, a.p - 1), 13)
    d = synth.probit_design(a.N, a.p, beta_true, 13, True, f"n{a.N}_p{a.p}")
    print(f"[bench] data N={a.N} p={a.p} generated in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)

    if a.only == "streamed":
        r = run_streamed(a, d)
        out = dict(common, value=r["value"], unit=r["unit"], ms_per_step=r["ms_per_step"], dtype="f32",
                   config={"workload": r["workload"], "N": a.N, "p": a.p}, roofline=r["roofline"], streamed=r)
        out["steps"], out["warmup"] = r["sweeps"], 2
        print(json.dumps(out), flush=True)
        return

    if a.only == "bf16":
        r = run_single(a, d, "bf16", a.traffic_json)
        out = dict(common, value=r["value"], unit=r["unit"], ms_per_step=r["ms_per_step"], dtype="bf16",
                   config={"workload": r["workload"], "N": a.N, "p": a.p, "x_storage": "bf16"},
                   roofline=r["roofline"], bf16=r)
        print(json.dumps(out), flush=True)
        return

    f32 = run_single(a, d, "f32", a.traffic_json)
    out = dict(common, value=f32["value"], unit="sweeps/s", ms_per_step=f32["ms_per_step"], dtype="f32",
               config={"workload": f32["workload"], "N": a.N, "p": a.p, "x_storage": "f32",
                       "n_side_arith": "f32", "p_side_arith": "f64", "chains": 1},
               hbm_gbps=f32["hbm_gbps"], kernel_ms=f32["kernel_ms"], sweep_ms_events=f32["sweep_ms_events"],
               kernel_fingerprint=kernel_fingerprint(), read_ceiling=f32["read_ceiling"],
               max_tn_proposals=f32["max_tn_proposals"], lambda_clamps=f32["lambda_clamps"],
               roofline=f32["roofline"])
    if a.only != "f32":
        out["bf16"] = run_single(a, d, "bf16", a.traffic_json)
        if a.N == 1_000_000 and a.p == 1000:
            data = batch_data(d)
            out["batch"] = run_batch(a, a.traffic_json, data)
            del data
            out["rare_event"] = run_rare(a)
            out["streamed"] = run_streamed(a, d)
            try:
                out["large_p"] = run_large_p(a)
            except Exception as e:  # reported, never fatal to the main line
                out["large_p"] = {"error": f"{type(e).__name__}: {e}"}
    if not a.no_cpu_baseline and a.only is None:
        print("[bench] timing the float64 oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(d, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
