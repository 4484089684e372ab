"""Benchmark of the grouped multi-density J/K build on one MI355X.

One step = one esmf_fock_build over the resident screened integral store of
the workload (all m densities in one pass).  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--workload slab1000|chain400|box40]
                  [--prec fp64|mixed] [--no-cpu-baseline] [--no-parity]

Only --gpus 1 is supported: the build runs on a single GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "J+K Fock builds/s (N=1000, m=8) FP64 vs mixed at 1e-8 Ha; p50/p99 latency"
PEAK_FP64 = 78.6e12      # MI355X FP64 vector/matrix, FLOP/s
PEAK_FP32 = 157.3e12     # MI355X FP32 vector/matrix, FLOP/s
PEAK_HBM = 8.0e12        # MI355X HBM3E, B/s
MAIN_KERNELS = ["paper_2002_00322_amd/csrc/kernels.hip", "paper_2002_00322_amd/csrc/fock_mfma.hip"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name):
    import workloads as wl
    if name == "slab1000":
        return wl.config3()
    if name == "chain400":
        return wl.config2()
    if name == "box40":
        return wl.config1()
    raise SystemExit(f"unknown workload {name}")


def kernel_source_sha():
    h = hashlib.sha256()
    for rel in MAIN_KERNELS:
        p = os.path.join(ROOT, rel)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_sha, workload_name, prec):
    """HBM bytes per launch of the main kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p)).get(f"{workload_name}:{prec}")
    except (ValueError, OSError):
        return None
    if not rec or rec.get("kernel_source_sha") != kernel_sha:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(c, nq_total, target_s=12.0):
    """The oracle's grouped build on a bounded sample of the same workload:
    the unique quartets whose outer pair index lies in a leading range, timed
    on the host cores, scaled to builds/s of the full workload."""
    import oracle
    n = c["alpha"].shape[0]
    npair = n * (n + 1) // 2
    end = max(1, npair // 400)
    t0 = time.time()
    _, _, nv = oracle.jk_canonical_range(c["centers"], c["alpha"], c["tau"], c["D"], 0, end)
    dt = time.time() - t0
    # grow the range until the sample takes a meaningful time
    while dt < target_s / 2 and end < npair:
        scale = min(8.0, max(2.0, target_s / max(dt, 1e-3)))
        end = min(npair, int(end * scale) + 1)
        t0 = time.time()
        _, _, nv = oracle.jk_canonical_range(c["centers"], c["alpha"], c["tau"], c["D"], 0, end)
        dt = time.time() - t0
    rate = nv / dt  # quartets per second (all m densities)
    return {"value": rate / nq_total, "unit": "builds/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"outer pairs [0,{end}) of {npair}: {nv} of {nq_total} unique quartets, "
                      f"{dt:.1f} s, all {c['D'].shape[0]} densities"}


def parity_sample(c, j, k, nsamp=48, seed=11):
    import oracle
    rng = np.random.default_rng(seed)
    m, n = c["D"].shape[0], c["alpha"].shape[0]
    i = rng.integers(0, m, nsamp)
    p = rng.integers(0, n, nsamp)
    q = rng.integers(0, n, nsamp)
    Jr, Kr = oracle.jk_entries(c["centers"], c["alpha"], c["tau"], c["D"], i, p, q)
    jh = j[i, p, q].cpu().numpy()
    kh = k[i, p, q].cpu().numpy()
    return {"samples": int(nsamp), "max_abs_dJ": float(np.max(np.abs(jh - Jr))),
            "max_abs_dK": float(np.max(np.abs(kh - Kr)))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="slab1000")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GB",
                    help="only run a plain device-to-device copy of this many GB (to scale "
                         "rocprofv3 FETCH_SIZE/WRITE_SIZE readings), then exit")
    args = ap.parse_args()
    if args.copy_calibration > 0:
        import torch
        n = int(args.copy_calibration * 1e9) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the build is "
                                   "single-GPU (multi-GPU sharding is described, not built)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    import paper_2002_00322_amd as pa

    c = workload(args.workload)
    m, n = c["D"].shape[0], c["alpha"].shape[0]
    prec = pa.PREC_FP64 if args.prec == "fp64" else pa.PREC_MIXED
    storage = pa.STORE_FP64 if args.prec == "fp64" else pa.STORE_FP32
    log(f"workload {c['name']} N={n} m={m} tau={c['tau']} prec={args.prec}")
    t0 = time.time()
    st = pa.EriStore(c["centers"], c["alpha"], c["tau"], storage=storage)
    prep_s = time.time() - t0
    info = st.info()
    log(f"prepared in {prep_s:.2f} s: {info}")
    d = torch.from_numpy(np.ascontiguousarray(c["D"])).to("cuda:0").contiguous()
    j = torch.empty_like(d)
    k = torch.empty_like(d)
    stream = torch.cuda.current_stream()
    for w in range(args.warmup):
        pa.fock_build(st, d, j, k, prec=prec)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} done")
    pa.timing_enable(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.time()
    ev0.record(stream)
    for s in range(args.steps):
        pa.fock_build(st, d, j, k, prec=prec)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - t0
    pa.timing_enable(False)
    kern_ms, kern_n = pa.timing_collect()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step (wall {wall:.3f} s), main kernel "
        f"{kern_ms / max(kern_n, 1):.3f} ms")
    builds_s = 1000.0 / ms_step
    nq = info["nquartets_kept"]
    flops = 20.0 * m * nq            # J: 2 FMA, K: 8 FMA per unique quartet per density
    kernel_s = kern_ms / max(kern_n, 1) / 1000.0
    peak = PEAK_FP64 if args.prec == "fp64" else PEAK_FP32
    sha = kernel_source_sha()
    traffic = traffic_from_profile(sha, c["name"], args.prec)
    eri_bytes = nq * (8 if args.prec == "fp64" else 4)
    out = {
        "metric": METRIC, "value": builds_s, "unit": "builds/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32+f64",
        "data": "synthetic (seeded s-type basis and transition densities)",
        "config": {"workload": c["name"], "nbf": n, "m": m, "tau": c["tau"],
                   "prec": args.prec, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": flops / kernel_s / 1e12,
                     "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": flops / kernel_s / peak, "traffic": traffic,
                     "kernel_ms": kernel_s * 1e3,
                     "algorithmic_flops_per_launch": flops,
                     "hbm_algorithmic_GBps": eri_bytes / kernel_s / 1e9,
                     "hbm_frac": eri_bytes / kernel_s / PEAK_HBM,
                     "kernel_source_sha": sha},
        "prepare_s": prep_s,
        "store": {"nquartets_kept": nq, "nblocks": info["nblocks"],
                  "nelements_stored": info["nelements_stored"],
                  "device_GB": info["device_bytes"] / 1e9,
                  "workspace_GB": info["workspace_bytes"] / 1e9},
    }
    if not args.no_parity:
        out["parity"] = parity_sample(c, j, k)
        log(f"parity {out['parity']}")
    st.release()
    del d, j, k
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, nq)
        log(f"cpu baseline {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
