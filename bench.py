"""Benchmark: Gibbs sweeps per second of the Horseshoe Probit sampler on one
MI355X, at N = 1,000,000 rows and p = 1000 predictors (X float32, 4 GB).

One step = one full Gibbs sweep (z | beta over all rows fused with X^T z;
lambda, tau; the float64 Cholesky draw of beta; nu, xi; the draw record).
Inputs are seeded synthetic data (the paper's Section 6.1 design with an
intercept and 10 nonzero coefficients) resident in HBM before timing starts.

Prints one JSON line.  Also reports:
  roofline      the sweep kernel (one fused launch per sweep; its z pass is the
                N x p stream): algorithmic bytes per launch (N p 4 + N) over
                its mean duration from HIP events on the library's stream,
                against the 8 TB/s HBM peak; traffic = hardware-counted HBM
                bytes per launch when the stored counter reading matches the
                current kernel sources
  read_ceiling  a plain streaming read of the same X (16-byte non-temporal
                loads, nothing else) on this GPU: what the z pass could reach
  cpu_baseline  the float64 oracle timed on this host on a bounded sample of
                the same workload (whole sweeps, one thread)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gibbs sweeps/sec and HBM GB/s at N=1e6,p=1000; chain-sweeps/sec batched vs plain"
HBM_PEAK_GBPS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--N", type=int, default=1_000_000)
    ap.add_argument("--p", type=int, default=1000)
    ap.add_argument("--x-type", default="f32", choices=["f32", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "sweep_kernel_traffic.json"))
    ap.add_argument("--batch", action="store_true",
                    help="the batched form instead: 64 uneven float32 datasets (one chain each) "
                         "and 16 chains sharing the N=1e6, p=1000 design in bfloat16; reports "
                         "chain-sweeps/s batched and plain")
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


def cpu_baseline(d, seconds):
    """Whole oracle sweeps on the same data until `seconds` have elapsed."""
    import numpy as np
    from oracle import oracle as orc
    # one-time Gram in float64 (untimed, like the GPU's creation step)
    G = np.zeros((d.p, d.p))
    step = 1 << 16
    for r in range(0, d.N, step):
        xb = d.X[r:r + step].astype(np.float64)
        G += xb.T @ xb
    ch = orc.Chain(d.p)
    n = 0
    t0 = time.perf_counter()
    while True:
        ch.sweep_once(d.X, d.y, G, seed=1)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or n >= 50:
            break
    return {"value": n / el, "unit": "sweeps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} whole float64 oracle sweeps of the same N={d.N}, p={d.p} workload "
                      f"from the cold start, single thread, {el:.1f} s; Gram formed beforehand "
                      f"(untimed)"}


def run_batch(a):
    """Chain-sweeps/s of the batched form against the same chains swept one by one."""
    import numpy as np
    import torch

    import synth
    from paper_1608_04329_amd import hsp

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    shapes = synth.batch_shapes(64, seed=1000)
    ds = [synth.batch_dataset(k, N, p) for k, (N, p) in enumerate(shapes)]
    beta_true, _ = synth.sparse_beta(1000, 10, 13)
    big = synth.probit_design(1_000_000, 1000, beta_true, 13, True, "n1000000_p1000")
    print(f"[bench] batch data generated in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    datasets = [(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), "f32") for d in ds]
    datasets.append((torch.from_numpy(big.X).cuda(), torch.from_numpy(big.y).cuda(), "bf16"))
    counts = [1] * len(ds) + [16]
    b = hsp.Batch(datasets, counts, seed=1, max_draws=64)
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
    batched = nchains * a.steps / elapsed
    print(f"[bench] batched: {a.steps} sweeps of {nchains} chains in {elapsed:.3f}s "
          f"({ms_ev:.3f} ms per batched sweep by events)", file=sys.stderr, flush=True)
    # plain: every chain swept on its own, one after another
    t0 = time.perf_counter()
    for c in b.chains:
        c.sweep(a.steps)
    for c in b.chains:
        c.sync()
    elapsed_plain = time.perf_counter() - t0
    plain = nchains * a.steps / elapsed_plain
    out = {
        "metric": "chain-sweeps/sec, batched vs plain",
        "value": round(batched, 1),
        "unit": "chain-sweeps/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(1e3 * elapsed / a.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16",
        "data": "synthetic",
        "config": {"workload": "horseshoe_probit_batch_64uneven_f32_plus_16chains_N1e6_p1000_bf16",
                   "chains": nchains, "datasets": len(ds) + 1},
        "plain_chain_sweeps_per_s": round(plain, 1),
        "batched_over_plain": round(batched / plain, 3),
    }
    b.close()
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (several GPUs "
              "would each sweep a row shard of X and sum X^T z across them).", file=sys.stderr)
        sys.exit(2)
    if a.batch:
        run_batch(a)
        return
    import numpy as np
    import torch

    import synth
    from paper_1608_04329_amd import hsp

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
    t0 = time.perf_counter()
    beta_true, idx = synth.sparse_beta(a.p, min(10, a.p - 1), 13)
    d = synth.probit_design(a.N, a.p, beta_true, 13, True, f"n{a.N}_p{a.p}")
    print(f"[bench] data N={a.N} p={a.p} generated in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    s = hsp.Sampler(d.X, d.y, seed=1, x_type=a.x_type, max_draws=max(64, a.steps + a.warmup))
    print(f"[bench] sampler created (X copied, Gram formed) in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)

    s.sweep(a.warmup)
    s.sync()
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.sweep(a.steps)
    s.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    zpass_ms, sweep_ms, n_timed = s.timing()
    clamps, maxatt = s.counters()
    s.set_timing(False)
    ceil_ms, ceil_bytes = hsp.hsp_read_ceiling(s.h, 10)
    print(f"[bench] {a.steps} sweeps in {elapsed:.3f}s; sweep kernel {zpass_ms:.4f} ms per launch, "
          f"{sweep_ms:.4f} ms per sweep (events)", file=sys.stderr, flush=True)

    esz = 4 if a.x_type == "f32" else 2
    zbytes = a.N * a.p * esz + a.N  # X once, y once
    value = a.steps / elapsed
    achieved = zbytes / (zpass_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(a.traffic_json):
        try:
            t = json.load(open(a.traffic_json))
            if (t.get("workload") == d.name and t.get("x_type") == a.x_type
                    and t.get("kernel_fingerprint") == kernel_fingerprint()):
                traffic = t.get("bytes_per_launch")
        except (OSError, ValueError):
            traffic = None
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(1e3 * elapsed / a.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.x_type == "f32" else "bf16",
        "data": "synthetic",
        "config": {"workload": f"horseshoe_probit_gibbs_N{a.N}_p{a.p}_x{a.x_type}",
                   "N": a.N, "p": a.p, "x_storage": a.x_type, "n_side_arith": "f32",
                   "p_side_arith": "f64", "chains": 1},
        "hbm_gbps": round(zbytes / (elapsed / a.steps) / 1e9, 1),
        "kernel_ms": round(zpass_ms, 5),
        "sweep_ms_events": round(sweep_ms, 5),
        "kernel_fingerprint": kernel_fingerprint(),
        "read_ceiling": {"gbps": round(ceil_bytes / (ceil_ms * 1e-3) / 1e9, 1),
                         "ms_per_pass": round(ceil_ms, 5),
                         "kernel": "plain 16-byte non-temporal streaming read of the same X"},
        "max_tn_proposals": int(maxatt),
        "lambda_clamps": int(clamps),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic},
    }
    s.close()
    if not a.no_cpu_baseline:
        print("[bench] timing the float64 oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(d, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
