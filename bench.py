"""Benchmark of the grouped multi-density J/K build on one MI355X.

One step = one esmf_fock_build over the resident screened integral store of
the workload (all m densities in one pass).  Prints ONE JSON line: the
headline leg (FP64 by default) with its roofline and per-build p50/p99, the
other precisions' legs with their error against the FP64 result, the
integral-direct leg, the integral-direct build of the 10x10x5 slab (whose
stored integrals would not fit in the device), one ESMF objective step (nine
densities, one m=9 build, E_2) and a GVP step, an s/p/d Cartesian-basis leg,
the 64-molecule batched leg, the serving mix at two arrival rates (p50/p99),
and the oracle's CPU rate from one full timed build of the same workload on
the host cores (the only use of the oracle here).

  python bench.py [--steps K] [--warmup W] [--workload slab1000|chain400|box40]
                  [--prec fp64|mixed|store32] [--no-mixed] [--no-batched]
                  [--no-cpu-baseline] [--no-esmf] [--no-direct-deep] [--no-serving]
  python bench.py --serving [--rates 50,100,...] [--iters 20] [--budget-gb 200]
      (the serving mix: admission by footprint, Poisson arrivals, p50/p99)
  python bench.py --record-traffic FETCH_DIR WRITE_DIR --workload slab1000
      (after rocprofv3 --pmc FETCH_SIZE / --pmc WRITE_SIZE runs of this script:
       writes the contraction kernel's HBM bytes per launch to
       profiles/traffic.json, tagged with the kernel source hash)

Only --gpus 1 is supported: the build runs on a single GPU.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "J+K Fock builds/s (N=1000, m=8) FP64 vs mixed at 1e-8 Ha; p50/p99 latency"
PEAK_FP64 = 78.6e12      # MI355X FP64 vector/matrix, FLOP/s
PEAK_FP32 = 157.3e12     # MI355X FP32 vector/matrix, FLOP/s
PEAK_HBM = 8.0e12        # MI355X HBM3E, B/s
# the contraction's sources, and the runtime that cuts its work items and
# sizes its partial tiles (both set the bytes a launch moves)
MAIN_KERNELS = ["paper_2002_00322_amd/csrc/kernels.hip", "paper_2002_00322_amd/csrc/fock_mfma.hip",
                "paper_2002_00322_amd/csrc/eri_device.h", "paper_2002_00322_amd/csrc/boys_table.h",
                "paper_2002_00322_amd/csrc/internal.h", "paper_2002_00322_amd/csrc/runtime.cpp"]


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


def _code_only(text):
    """Source text without comments and blank lines: edits to comments do
    not change the kernels a traffic record was taken on."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def kernel_source_sha():
    h = hashlib.sha256()
    for rel in MAIN_KERNELS:
        p = os.path.join(ROOT, rel)
        if os.path.exists(p):
            h.update(_code_only(open(p).read()).encode())
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


FETCH_SCALE = 2.0   # bytes per FETCH_SIZE KiB unit / 1024: a 4 GB copy reads 2.0e6 KiB
WRITE_SCALE = 1.0   # a 4 GB copy writes 3.9e6 KiB


def record_traffic(fetch_dir, write_dir, workload_name):
    """Mean FETCH_SIZE / WRITE_SIZE per dispatch of the contraction kernel (per
    precision) from two rocprofv3 --pmc runs, scaled by the copy calibration,
    into profiles/traffic.json."""
    import csv
    import glob

    modes = {"0": "fp64", "1": "mixed", "2": "store32", "3": "direct", "4": "mixed_fp64_store"}
    keys = [m + w for m in modes.values() for w in ("", "_wide")]
    kernels = {}

    def per_prec(d, counter):
        # two-visit kernel fock_mfma_kernel<mode, skip, occupancy, chain, J
        # width> (a J width of 16 is the wide contraction) and the fused
        # kernel fock_fused_kernel<mode, skip, occupancy, chain, band>
        vals = {k: [] for k in keys}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for row in csv.DictReader(open(f)):
                name = row.get("Kernel_Name", "")
                if row.get("Counter_Name") != counter:
                    continue
                kern = "fock_mfma_kernel<" if "fock_mfma_kernel<" in name else \
                    "fock_fused_kernel<" if "fock_fused_kernel<" in name else None
                if kern is None:
                    continue
                args = [a.strip() for a in name.split(kern, 1)[1].split(">", 1)[0].split(",")]
                wide = kern == "fock_mfma_kernel<" and args[-1] == "16"
                key = modes.get(args[0], "fp64") + ("_wide" if wide else "")
                vals[key].append(float(row["Counter_Value"]))
                kernels[key] = kern[:-1]
        return {k: (sum(v) / len(v) if v else None, len(v)) for k, v in vals.items()}

    fe = per_prec(fetch_dir, "FETCH_SIZE")
    wr = per_prec(write_dir, "WRITE_SIZE")
    p = os.path.join(ROOT, "profiles", "traffic.json")
    sha = kernel_source_sha()
    data = json.load(open(p)) if os.path.exists(p) else {}
    # records taken on other kernel sources are stale: dropped
    data = {k: v for k, v in data.items() if v.get("kernel_source_sha") == sha}
    for prec in keys:
        (f, nf), (w, nw) = fe[prec], wr[prec]
        if f is None or w is None:
            continue
        data[f"{workload_name}:{prec}"] = {
            "kernel": kernels.get(prec, "fock_mfma_kernel"), "kernel_source_sha": sha,
            "fetch_KiB_per_dispatch": f, "write_KiB_per_dispatch": w,
            "dispatches": [nf, nw], "fetch_scale": FETCH_SCALE, "write_scale": WRITE_SCALE,
            "hbm_bytes_per_launch": 1024.0 * (FETCH_SCALE * f + WRITE_SCALE * w)}
    json.dump(data, open(p, "w"), indent=1, sort_keys=True)
    print(json.dumps(data), flush=True)


def host_cpu():
    """The host's CPU as lscpu and /proc/cpuinfo describe it (model name,
    family/model/stepping, sockets and cores), and the cores this process may
    use."""
    info = {}
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                info[k.strip()] = v.strip()
    except (OSError, ValueError):
        pass
    model = info.get("Model name")
    if not model:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    keys = ("Vendor ID", "CPU family", "Model", "Stepping", "Socket(s)", "Core(s) per socket",
            "Thread(s) per core", "CPU(s)", "CPU max MHz", "L3 cache")
    detail = {k: info[k] for k in keys if k in info}
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return model, detail, usable


def cpu_baseline(c, nq_total, chunks=4):
    """One full build of the workload by the oracle's grouped loop (every
    unique screened quartet, all m densities), timed on the host cores.  It
    runs as a few calls over ranges of the outer pair index of about equal
    work, so that a progress line appears between them; the time is their
    sum."""
    import oracle
    n = c["alpha"].shape[0]
    npair = n * (n + 1) // 2
    cuts = [0] + [int(npair * np.sqrt(x / chunks)) for x in range(1, chunks)] + [npair]
    dt, nv = 0.0, 0
    for a, b in zip(cuts[:-1], cuts[1:]):
        t0 = time.time()
        _, _, v = oracle.jk_canonical_range(c["centers"], c["alpha"], c["tau"], c["D"], a, b)
        dt += time.time() - t0
        nv += v
        log(f"cpu baseline: outer pairs [{a}, {b}) of {npair} in {dt:.1f} s so far")
    model, detail, usable = host_cpu()
    # the chain of 400 functions (m = 8): the median of five full builds
    import workloads as wl
    c2 = wl.config2()
    ts = []
    for _ in range(5):
        t0 = time.time()
        oracle.jk_canonical(c2["centers"], c2["alpha"], c2["tau"], c2["D"])
        ts.append(time.time() - t0)
    log(f"cpu baseline: chain400 builds {', '.join(f'{x:.3f}' for x in ts)} s")
    return {"value": 1.0 / dt, "unit": "builds/s", "cores": oracle.num_threads(),
            "kind": "oracle", "cpu_model": model, "cpu_detail": detail, "nproc": os.cpu_count(),
            "usable_cpus": usable, "seconds_per_build": dt, "quartets_visited": nv,
            "nquartets_kept_gpu": nq_total,
            "chain400_median_s_per_build": float(np.median(ts)), "chain400_builds": 5,
            "sample": f"full build: all {nv} unique screened quartets of {c['name']} "
                      f"(N={n}, m={c['D'].shape[0]}, tau={c['tau']}) in {dt:.1f} s "
                      f"({chunks} calls over outer-pair ranges); chain400: median of 5 full builds"}


def pctl(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def timed_builds(pa, st, d, j, k, prec, steps, warmup, stream):
    """W untimed builds, then K builds bracketed by synchronisations; HIP
    events around every build on the build stream give per-build latencies,
    the library's own events the contraction kernel's duration."""
    import torch
    for _ in range(warmup):
        pa.fock_build(st, d, j, k, prec=prec, stream=stream)
    torch.cuda.synchronize()
    pa.timing_enable(True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.time()
    evs[0].record(stream)
    for s in range(steps):
        pa.fock_build(st, d, j, k, prec=prec, stream=stream)
        evs[s + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.time() - t0
    pa.timing_enable(False)
    kern_ms, kern_n = pa.timing_collect()
    lat = [evs[s].elapsed_time(evs[s + 1]) for s in range(steps)]
    total = evs[0].elapsed_time(evs[steps])
    return {"ms_per_step": total / steps, "wall_s": wall, "lat": lat,
            "kernel_ms": kern_ms / max(kern_n, 1)}


def roofline(flops, kernel_ms, peak, traffic, eri_bytes=None, bound="mfma"):
    """bound: "mfma" for the matrix-core contractions (their intensity is
    above the ridge), "alu" where vector arithmetic bounds the kernel (the
    integral-direct build evaluates its integrals)."""
    ks = kernel_ms / 1000.0
    out = {"bound": bound, "achieved": flops / ks / 1e12, "peak": peak / 1e12,
           "unit": "TFLOP/s", "frac": flops / ks / peak, "traffic": traffic}
    if eri_bytes:
        # attainable = min(peak, arithmetic intensity x HBM bandwidth)
        attain = min(peak, flops / eri_bytes * PEAK_HBM)
        out["attainable_TFLOPs"] = attain / 1e12
        out["frac_of_attainable"] = flops / ks / attain
    return out


def direct_deep_leg(pa, steps, warmup, stream):
    """The 10x10x5 slab (1000 s functions, m = 8) on an integral-direct handle:
    a molecule whose stored FP64 integrals would not fit in the device, built
    with every integral recomputed in each build (the plan and pair data are
    all the handle holds)."""
    import torch
    import workloads as wl
    c = wl.config3_deep()
    m = c["D"].shape[0]
    t0 = time.time()
    st = pa.EriStore(c["centers"], c["alpha"], c["tau"], storage=pa.STORE_DIRECT)
    torch.cuda.synchronize()
    prep_s = time.time() - t0
    info = st.info()
    log(f"direct deep: prepared in {prep_s:.2f} s: {info}")
    d = torch.from_numpy(np.ascontiguousarray(c["D"])).to("cuda:0")
    j = torch.empty_like(d)
    k = torch.empty_like(d)
    t = timed_builds(pa, st, d, j, k, pa.PREC_FP64, steps, warmup, stream)
    nq = info["nquartets_kept"]
    r = {"workload": c["name"], "nbf": int(c["alpha"].shape[0]), "m": m, "ms_per_step": t["ms_per_step"],
         "kernel_ms": t["kernel_ms"], "prepare_s": prep_s, "nquartets_kept": nq, "nblocks": info["nblocks"],
         "fp64_store_GB": info["fp64_store_bytes"] / 1e9,
         "stored_build_workspace_GB": info["workspace_bytes_plan"][0] / 1e9,
         "device_GB": torch.cuda.mem_get_info()[1] / 1e9,
         "handle_GB": info["device_bytes"] / 1e9, "workspace_GB": info["workspace_bytes"] / 1e9,
         "quartets_per_s": nq / (t["kernel_ms"] / 1000.0)}
    log(f"direct deep: {t['ms_per_step']:.1f} ms/step, kernel {t['kernel_ms']:.1f} ms")
    st.release()
    del d, j, k
    torch.cuda.empty_cache()
    return r


def esmf_leg(pa, st, c, steps, warmup, stream, sha, compare=True, n_occ=40, seed=9):
    """One ESMF objective step on the workload's FP64 store: the nine
    densities from a seeded state (No = 40 occupied rows of an orthogonal V),
    one grouped build of all nine (the two symmetric ones marked, so that all
    nine fit one pass over the integrals), and E_2 from the first two.  HIP
    events split each step into its three parts; the build is also timed
    without the flags (two passes) for comparison.  Then the GVP form: a
    pass over D1, D2, A, the energy gradient as the multipliers, and a pass
    over the six densities that depend on it."""
    import torch
    import workloads as wl
    n = c["alpha"].shape[0]
    n_occ = min(n_occ, n // 2)
    es = wl.esmf_state(n, n_occ, seed)
    ins = [torch.from_numpy(np.ascontiguousarray(es[k])).to("cuda:0")
           for k in ("theta", "gamma", "sigma", "mu", "R", "Phi")]
    d = torch.empty((9, n, n), dtype=torch.float64, device="cuda:0")
    j, k = torch.empty_like(d), torch.empty_like(d)

    def step(ev=None, symmetric=pa.ESMF_SYMMETRIC):
        if ev:
            ev[0].record(stream)
        pa.nine_densities(*ins, d=d, stream=stream)
        if ev:
            ev[1].record(stream)
        pa.fock_build(st, d, j, k, stream=stream, symmetric=symmetric)
        if ev:
            ev[2].record(stream)
        e2 = pa.energy_two_body(d, j, k, es["n2"], es["c0"], stream=stream)
        if ev:
            ev[3].record(stream)
        return e2
    for _ in range(max(warmup, 1)):
        step()
    torch.cuda.synchronize()
    pa.timing_enable(True)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for s in range(steps):
        e2 = step(evs[s])
    torch.cuda.synchronize()
    pa.timing_enable(False)
    kern_ms, kern_n = pa.timing_collect()
    parts = np.array([[ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])]
                      for ev in evs])
    total = evs[0][0].elapsed_time(evs[-1][3]) / steps
    kms = kern_ms / max(kern_n, 1)
    # the same step without the symmetry flags: two passes (groups of 8 + 1)
    two_pass_ms = None
    if compare:
        ev2 = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(3)]
        step(symmetric=None)
        for s in range(3):
            step(ev2[s], symmetric=None)
        torch.cuda.synchronize()
        two_pass_ms = float(np.mean([ev[1].elapsed_time(ev[2]) for ev in ev2]))
    flops = 20.0 * 9 * st.info()["nquartets_kept"]
    # the GVP form: pass 1 builds D1, D2, A; the energy gradient replaces the
    # multipliers; pass 2 builds the six densities that depend on it
    g_dev = torch.from_numpy(np.ascontiguousarray(es["G"])).to("cuda:0")
    d3 = torch.empty((3, n, n), dtype=torch.float64, device="cuda:0")
    j3, k3 = torch.empty_like(d3), torch.empty_like(d3)
    j6 = torch.empty((6, n, n), dtype=torch.float64, device="cuda:0")
    k6 = torch.empty_like(j6)

    def gvp(ev=None):
        if ev:
            ev[0].record(stream)
        pa.nine_densities(*ins, d=d, stream=stream)
        d3.copy_(d[:3])
        pa.fock_build(st, d3, j3, k3, stream=stream, symmetric=(1, 0, 1))
        if ev:
            ev[1].record(stream)
        gr = pa.energy_gradient(ins[0], ins[1], ins[2], g_dev, d3, j3, k3, es["c0"], es["n2"], stream=stream)
        pa.nine_densities(ins[0], ins[1], ins[2], gr["sigma"], gr["theta"], gr["gamma"], d=d, stream=stream)
        if ev:
            ev[2].record(stream)
        pa.fock_build(st, d[3:], j6, k6, stream=stream)
        if ev:
            ev[3].record(stream)
        return gr
    gvp()
    torch.cuda.synchronize()
    gsteps = max(3, steps // 2)
    evg = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(gsteps)]
    for s in range(gsteps):
        gr = gvp(evg[s])
    torch.cuda.synchronize()
    gp = np.array([[ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])]
                   for ev in evg])
    gvp_out = {"steps": gsteps, "ms_per_step": evg[0][0].elapsed_time(evg[-1][3]) / gsteps,
               "pass1_ms": float(gp[:, 0].mean()), "gradient_and_densities_ms": float(gp[:, 1].mean()),
               "pass2_ms": float(gp[:, 2].mean()), "E": float(gr["energy"][2].item())}
    return {"workload": f"{c['name']}: nine densities (No={n_occ}, Nv={n - n_occ}), one grouped "
                        f"FP64 build (m=9, Theta^T Theta and A marked symmetric: one pass), E_2",
            "ms_per_step": total, "steps_per_s": 1000.0 / total,
            "densities_ms": float(parts[:, 0].mean()), "build_ms": float(parts[:, 1].mean()),
            "energy_ms": float(parts[:, 2].mean()), "kernel_ms": kms,
            "roofline": dict(roofline(flops, kms, PEAK_FP64, traffic_from_profile(sha, c["name"], "fp64_wide"),
                                      8.0 * st.info()["nquartets_kept"]),
                             kernel="fock_mfma_kernel (16 J columns)", kernel_ms=kms,
                             algorithmic_flops_per_launch=flops),
            "E2": float(e2.item()), "build_ms_without_symmetry_flags": two_pass_ms,
            "gvp_two_pass": gvp_out, "densities_scaling": densities_scaling_leg(pa, stream, steps)}


def esmf_gemm_flops(n, no, nv):
    """FLOP of the matrix products in the nine densities and in the energy
    gradient, as written (2 M N K per product): the O(N^2 N_o) work that
    grows fastest with N."""
    dens = (3 * 2 * no * n * nv + 2 * 2 * no * no * nv + 2 * 2 * no * n * no + 11 * 2 * n * n * no)
    grad = (5 * 2 * no * n * n + 2 * no * n * nv + 2 * no * no * nv + 2 * no * no * n + 2 * no * n * no
            + 2 * nv * n * no + 2 * no * nv * n + 2 * no * nv * no)
    return float(dens), float(grad)


def densities_scaling_leg(pa, stream, steps, n=8000, no=800, seed=21):
    """The O(N^2 N_o) part of an ESMF step at a size where it dominates:
    nine densities and the energy gradient at N = 8000, N_o = 800 from seeded
    normal matrices generated on the device (their values only set the
    timing).  Reported against the FP64 matrix-core peak."""
    import torch
    nv = n - no
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)

    def rnd(*shape):
        return torch.randn(*shape, generator=g, dtype=torch.float64, device="cuda:0") / np.sqrt(shape[-1])
    theta, gamma, sigma, mu, r, phi = rnd(no, n), rnd(nv, n), rnd(no, nv), rnd(no, nv), rnd(no, n), rnd(nv, n)
    gm = rnd(n, n)
    d = torch.empty((9, n, n), dtype=torch.float64, device="cuda:0")
    j3, k3 = rnd(3, n, n), rnd(3, n, n)
    pa.nine_densities(theta, gamma, sigma, mu, r, phi, d=d, stream=stream)
    pa.energy_gradient(theta, gamma, sigma, gm, d[:3], j3, k3, 0.9, 1.3, stream=stream)
    torch.cuda.synchronize()
    reps = max(3, steps // 4)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
    for e in ev:
        e[0].record(stream)
        pa.nine_densities(theta, gamma, sigma, mu, r, phi, d=d, stream=stream)
        e[1].record(stream)
        pa.energy_gradient(theta, gamma, sigma, gm, d[:3], j3, k3, 0.9, 1.3, stream=stream)
        e[2].record(stream)
    torch.cuda.synchronize()
    dms = float(np.median([e[0].elapsed_time(e[1]) for e in ev]))
    gms = float(np.median([e[1].elapsed_time(e[2]) for e in ev]))
    fd, fg = esmf_gemm_flops(n, no, nv)
    out = {"workload": f"nine densities and energy gradient, N={n}, No={no}, Nv={nv} (seeded normal inputs)",
           "densities_ms": dms, "densities_tflops": fd / dms / 1e9, "gradient_ms": gms,
           "gradient_tflops": fg / gms / 1e9, "peak_tflops": PEAK_FP64 / 1e12,
           "densities_frac": fd / dms / 1e9 / (PEAK_FP64 / 1e12),
           "gradient_frac": fg / gms / 1e9 / (PEAK_FP64 / 1e12)}
    del theta, gamma, sigma, mu, r, phi, gm, d, j3, k3
    torch.cuda.empty_cache()
    return out


def cart_leg(pa, steps, warmup, stream, nsites=72, m=8):
    """A basis with angular momentum: a chain of 72 sites, each with two s,
    two p and one d primitive shell (1008 Cartesian functions), tau 1e-10,
    m = 8 transition densities (N_o = 40); FP64 store and builds."""
    import torch
    import workloads as wl
    A, al, L = wl.spd_chain(nsites)
    n = al.shape[0]
    t0 = time.time()
    st = pa.EriStore(A, al, 1e-10, lmn=L)
    torch.cuda.synchronize()
    prep = time.time() - t0
    info = st.info()
    d = torch.from_numpy(np.ascontiguousarray(wl.transition_densities(n, m, 40, 701, 702))).to("cuda:0")
    j, k = torch.empty_like(d), torch.empty_like(d)
    t = timed_builds(pa, st, d, j, k, pa.PREC_FP64, steps, warmup, stream)
    flops = 20.0 * m * info["nquartets_kept"]
    out = {"workload": f"spd chain: {nsites} sites x (2 s + 2 p + 1 d shells) = {n} Cartesian functions, "
                       f"m={m}, tau 1e-10", "prepare_s": prep, "ms_per_step": t["ms_per_step"],
           "builds_per_s": 1000.0 / t["ms_per_step"], "kernel_ms": t["kernel_ms"],
           "latency_p50_ms": pctl(t["lat"], 50), "latency_p99_ms": pctl(t["lat"], 99),
           "roofline": roofline(flops, t["kernel_ms"], PEAK_FP64, None, 8.0 * info["nquartets_kept"]),
           "store": {"nquartets_kept": info["nquartets_kept"], "nblocks": info["nblocks"],
                     "device_GB": info["device_bytes"] / 1e9}}
    st.release()
    # contracted functions: 48 sites x (s of 3, s of 1, p of 2, d of 1 primitives)
    sites = np.zeros((48, 3))
    sites[:, 0] = wl.SPACING * np.arange(48)
    cen, lm, off, pe, pc = wl.contracted_basis(sites)
    nc = cen.shape[0]
    t0 = time.time()
    st = pa.EriStore.contracted(cen, lm, off, pe, pc, 1e-10)
    torch.cuda.synchronize()
    prep_c = time.time() - t0
    info = st.info()
    d = torch.from_numpy(np.ascontiguousarray(wl.transition_densities(nc, m, 40, 703, 704))).to("cuda:0")
    j, k = torch.empty_like(d), torch.empty_like(d)
    t = timed_builds(pa, st, d, j, k, pa.PREC_FP64, steps, warmup, stream)
    flops = 20.0 * m * info["nquartets_kept"]
    out["contracted"] = {
        "workload": f"contracted chain: 48 sites x (s[3] + s[1] + p[2] + d[1]) = {nc} functions, "
                    f"{int(off[-1])} primitives, m={m}, tau 1e-10",
        "prepare_s": prep_c, "ms_per_step": t["ms_per_step"], "builds_per_s": 1000.0 / t["ms_per_step"],
        "kernel_ms": t["kernel_ms"], "tflops": flops / (t["kernel_ms"] / 1000.0) / 1e12,
        "nquartets_kept": info["nquartets_kept"], "device_GB": info["device_bytes"] / 1e9}
    st.release()
    return out


def batched_leg(pa, steps, warmup):
    """The 64-molecule batch (chains, N 50..600, m 2..10) as one batched
    build per step on a non-default stream (captured once, then replayed)."""
    import torch
    import workloads as wl
    mols = wl.batch_workload()
    t0 = time.time()
    stores = [pa.EriStore(c["centers"], c["alpha"], c["tau"]) for c in mols]
    prep = time.time() - t0
    ds = [torch.from_numpy(np.ascontiguousarray(c["D"])).to("cuda:0") for c in mols]
    js = [torch.empty_like(d) for d in ds]
    ks = [torch.empty_like(d) for d in ds]
    s = torch.cuda.Stream()
    for _ in range(max(warmup, 1)):
        pa.fock_build_batched(stores, ds, js, ks, stream=s)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(s)
    for i in range(steps):
        pa.fock_build_batched(stores, ds, js, ks, stream=s)
        ev[i + 1].record(s)
    torch.cuda.synchronize()
    lat = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    ms = ev[0].elapsed_time(ev[steps]) / steps
    nq = sum(st.info()["nquartets_kept"] for st in stores)
    flops = sum(20.0 * c["D"].shape[0] * st.info()["nquartets_kept"] for c, st in zip(mols, stores))
    out = {"workload": "64 chains, N 50..600, m 2..10, tau 1e-10 (seeds 401+i)",
           "molecules": len(mols), "ms_per_batch": ms, "molecule_builds_per_s": 1000.0 * len(mols) / ms,
           "batch_p50_ms": pctl(lat, 50), "batch_p99_ms": pctl(lat, 99),
           "nquartets_kept": nq, "tflops": flops / (ms / 1000.0) / 1e12, "prepare_s": prep}
    for st in stores:
        st.release()
    return out


def serving_leg(pa, rates, iters, budget, ws_limit, nstreams, max_group, max_inflight, ring=4,
                seed=7, sessions=None):
    """The serving mix (32 sessions, chains and two-layer slabs, N 100..1500,
    m in {4, 8}, 20 iterations each) at each arrival rate, on a fresh server:
    - rolling admission: sessions are admitted in order while their store
      fits the HBM budget left; a session whose 20 iterations are done is
      closed, and waiting sessions are admitted as its budget frees up (one
      whose store alone exceeds the budget is rejected);
    - open-loop Poisson arrivals, each one the next iteration of the next
      active session in round-robin order (FIFO within a session, at most
      `ring` outstanding per session, the depth of its output buffers);
    - every iteration draws fresh W (seeded by session and iteration) and forms
      its densities D = C_occ W C_virt^T on the GPU, on the submitting stream,
      and submits with no host synchronisation (the server orders the build
      after the producer stream).
    Latency is submit-to-completion (the server's clock) and arrival-to-
    completion (including the wait for a ring slot)."""
    import collections
    import queue
    import threading
    import torch
    import workloads as wl
    sess = wl.serving_sessions(iters=iters) if sessions is None else sessions
    dev = torch.device("cuda:0")
    out = {"sessions": len(sess), "budget_GB": budget / 1e9, "workspace_limit_GB": ws_limit / 1e9,
           "nstreams": nstreams, "max_group": max_group, "max_inflight": max_inflight, "iterations": iters,
           "ring": ring, "rates": []}
    for lam in rates:
        srv = pa.Server(prec=pa.PREC_FP64, nstreams=nstreams, max_group=max_group, max_inflight=max_inflight,
                        hbm_budget_bytes=budget, workspace_limit_bytes=ws_limit)
        rng = np.random.default_rng(seed)
        waiting = collections.deque(range(len(sess)))
        active = {}          # session index -> state
        rejected, admitted_at = [], {}
        finished = queue.Queue()
        t0 = time.perf_counter()

        def admit():
            while waiting:
                x = waiting[0]
                s = sess[x]
                try:
                    sid, fp = srv.open_session(s["centers"], s["alpha"], s["tau"])
                except pa.OutOfMemory as e:
                    if e.footprint > budget:
                        rejected.append({"session": s["name"], "footprint_GB": e.footprint / 1e9})
                        log(f"serving: rejected {s['name']} ({e.footprint / 1e9:.1f} GB)")
                        waiting.popleft()
                        continue
                    return
                waiting.popleft()
                n = s["alpha"].shape[0]
                no = min(40, n // 2)
                C = torch.from_numpy(wl.orthonormal(n, s["seed"] + 7000)).to(dev)
                bufs = [tuple(torch.empty((s["m"], n, n), dtype=torch.float64, device=dev) for _ in range(3))
                        for _ in range(ring)]
                active[x] = {"sid": sid, "fp": fp, "co": C[:, :no].contiguous(), "cvt": C[:, no:].T.contiguous(),
                             "no": no, "nv": n - no, "m": s["m"], "next": 0, "done": 0, "out": 0, "bufs": bufs}
                admitted_at[x] = time.perf_counter() - t0

        admit()
        lat, lat_arr = [], []
        errors = []
        q = queue.Queue()

        def collector():
            while True:
                item = q.get()
                if item is None:
                    return
                x, rid, t_arr = item
                try:
                    lat.append(srv.wait(rid))
                    lat_arr.append((time.perf_counter() - t_arr) * 1000.0)
                except Exception as e:  # report, but never leave the driver waiting
                    errors.append(repr(e))
                finished.put(x)

        th = threading.Thread(target=collector)
        th.start()
        ok = False
        try:
            gen = torch.Generator(device=dev)
            order = collections.deque()
            start = time.perf_counter() + 0.005
            t_next = start
            while active or waiting:
                # completions: free ring slots, close finished sessions, admit
                while True:
                    try:
                        x = finished.get_nowait()
                    except queue.Empty:
                        break
                    st = active[x]
                    st["out"] -= 1
                    st["done"] += 1
                    if st["done"] == iters:
                        srv.close_session(st["sid"])
                        del active[x]
                        admit()
                if not active:
                    if waiting:
                        admit()
                        if not active:   # not even alone: the budget is taken by nothing else
                            s = sess[waiting.popleft()]
                            rejected.append({"session": s["name"], "footprint_GB": None})
                        continue
                    break
                # the next arrival of the Poisson process
                now = time.perf_counter()
                if t_next > now:
                    time.sleep(min(t_next - now, 0.002))
                    continue
                t_arr = t_next
                cand = [x for x in sorted(active) if active[x]["next"] < iters and active[x]["out"] < ring]
                if not cand:
                    time.sleep(0.0002)   # every active session waits on its ring: the arrival queues
                    continue
                # round-robin: the first candidate after the last one served
                x = cand[0]
                if order:
                    later = [c for c in cand if c > order[-1]]
                    x = later[0] if later else cand[0]
                order.append(x)
                st = active[x]
                it = st["next"]
                d, j, k = st["bufs"][it % ring]
                gen.manual_seed(seed * 1000003 + sess[x]["seed"] * 131 + it)
                W = torch.randn((st["m"], st["no"], st["nv"]), generator=gen, device=dev, dtype=torch.float64)
                W /= float(np.sqrt(st["no"] * st["nv"]))
                torch.matmul(st["co"], torch.matmul(W, st["cvt"]), out=d)
                rid = srv.submit(st["sid"], d, j, k)
                st["next"] += 1
                st["out"] += 1
                q.put((x, rid, t_arr))
                t_next += rng.exponential(1.0 / lam)
            ok = not errors
        finally:
            # the collector ends and the server goes, whatever the loop raised
            # (an exception here must not leave a thread waiting forever)
            q.put(None)
            th.join()
            if not ok or errors:
                srv.destroy()
        busy = time.perf_counter() - start
        if errors or not ok:
            raise RuntimeError(f"serving requests failed: {errors[:3]}")
        stt = srv.stats()
        srv.destroy()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        r = {"offered_req_per_s": lam, "requests": len(lat), "served_req_per_s": len(lat) / busy,
             "seconds": busy, "latency_p50_ms": pctl(lat, 50), "latency_p99_ms": pctl(lat, 99),
             "from_arrival_p50_ms": pctl(lat_arr, 50), "from_arrival_p99_ms": pctl(lat_arr, 99),
             "groups": stt["groups_launched"], "mean_group_size": len(lat) / max(stt["groups_launched"], 1),
             "max_group_size": stt["max_group_size"], "sessions_rejected": len(rejected),
             "admitted_after_start": sum(1 for v in admitted_at.values() if v > 0.5)}
        out["rates"].append(r)
        out["rejected"] = rejected
        log(f"serving: rate {lam}/s: {len(lat)} requests in {busy:.2f} s, p50 {r['latency_p50_ms']:.2f} ms "
            f"p99 {r['latency_p99_ms']:.2f} ms, {r['admitted_after_start']} sessions admitted while others ran")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="slab1000")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "mixed", "store32"],
                    help="precision of the headline leg")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the legs of the other precisions (mixed on both stores, store32)")
    ap.add_argument("--legs", default="",
                    help="comma-separated precision legs to run (fp64, mixed, store32, mixed_fp64_store, "
                         "direct), the headline first; default: all that the --no-* flags leave")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-molecule batched leg")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (default variant)")
    ap.add_argument("--no-direct", action="store_true",
                    help="skip the integral-direct leg (FP64 integrals recomputed in every build)")
    ap.add_argument("--no-direct-deep", action="store_true",
                    help="skip the integral-direct build of the 10x10x5 slab (a stored build would not fit)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true",
                    help="no effect (the benchmark takes no oracle samples; parity is in tests/)")
    ap.add_argument("--no-esmf", action="store_true",
                    help="skip the ESMF step leg (nine densities, one m=9 build, E_2)")
    ap.add_argument("--no-cart", action="store_true",
                    help="skip the s/p/d Cartesian-basis leg (1008-function chain)")
    ap.add_argument("--no-esmf-compare", action="store_true",
                    help="in the ESMF leg, skip timing the build without symmetry flags")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GB",
                    help="only run a plain device-to-device copy of this many GB (to scale "
                         "rocprofv3 FETCH_SIZE/WRITE_SIZE readings), then exit")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the probe of the device's FP64 matrix-core, FMA and copy rates")
    ap.add_argument("--serving", action="store_true",
                    help="run only the serving mix (Poisson arrivals, p50/p99) and print its JSON")
    ap.add_argument("--rates", default="50,100,200,500,1000,2000")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg of the default run")
    ap.add_argument("--serving-rates", default="50,500",
                    help="arrival rates (req/s) of the default run's serving leg")
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--workspace-gb", type=float, default=64.0)
    ap.add_argument("--nstreams", type=int, default=4)
    ap.add_argument("--max-group", type=int, default=16)
    ap.add_argument("--max-inflight", type=int, default=2)
    args = ap.parse_args()
    if args.record_traffic:
        record_traffic(args.record_traffic[0], args.record_traffic[1], args.workload)
        return
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

    if args.serving:
        rates = [float(x) for x in args.rates.split(",")]
        out = {"metric": "serving latency (ESMF session mix)", "n_gpus": 1,
               "data": "synthetic (seeded s-type basis and transition densities)",
               "serving": serving_leg(pa, rates, args.iters, args.budget_gb * 1e9,
                                      args.workspace_gb * 1e9, args.nstreams, args.max_group,
                                      args.max_inflight)}
        print(json.dumps(out), flush=True)
        return

    c = workload(args.workload)
    m, n = c["D"].shape[0], c["alpha"].shape[0]
    stream = torch.cuda.current_stream()
    d = torch.from_numpy(np.ascontiguousarray(c["D"])).to("cuda:0").contiguous()
    sha = kernel_source_sha()
    legs = [args.prec] + ([] if args.no_mixed else
                          [p for p in ("fp64", "mixed", "store32", "mixed_fp64_store") if p != args.prec])
    if not args.no_direct:
        legs.append("direct")
    if args.legs:
        legs = [x for x in args.legs.split(",") if x]
        if legs[0] != args.prec:
            raise SystemExit("--legs must start with the headline precision (--prec)")
    precs = {"fp64": pa.PREC_FP64, "mixed": pa.PREC_MIXED, "store32": pa.PREC_STORE32,
             "mixed_fp64_store": pa.PREC_MIXED,
             "direct": pa.PREC_FP64}
    storages = {"fp64": pa.STORE_FP64, "mixed": pa.STORE_FP32, "store32": pa.STORE_FP32,
                "mixed_fp64_store": pa.STORE_FP64,
                "direct": pa.STORE_DIRECT}
    res = {}
    for leg in legs:
        prec = precs[leg]
        storage = storages[leg]
        log(f"workload {c['name']} N={n} m={m} tau={c['tau']} prec={leg}")
        t0 = time.time()
        st = pa.EriStore(c["centers"], c["alpha"], c["tau"], storage=storage)
        torch.cuda.synchronize()
        prep_s = time.time() - t0
        info = st.info()
        log(f"prepared in {prep_s:.2f} s: {info}")
        j = torch.empty_like(d)
        k = torch.empty_like(d)
        tune = None
        if not args.no_tune:
            tune = pa.fock_tune(st, m, prec=prec)
            log(f"{leg}: tuner {tune}")
        t = timed_builds(pa, st, d, j, k, prec, args.steps, args.warmup, stream)
        log(f"{leg}: timed {args.steps} steps: {t['ms_per_step']:.3f} ms/step (wall "
            f"{t['wall_s']:.3f} s), main kernel {t['kernel_ms']:.3f} ms, p50 "
            f"{pctl(t['lat'], 50):.3f} p99 {pctl(t['lat'], 99):.3f} ms")
        nq = info["nquartets_kept"]
        flops = 20.0 * m * nq            # J: 2 FMA, K: 8 FMA per unique quartet per density
        # integral stream read per launch (none for the integral-direct leg)
        eri_bytes = nq * {"fp64": 8, "mixed": 4, "store32": 4, "mixed_fp64_store": 8, "direct": 0}[leg]
        r = {"ms_per_step": t["ms_per_step"], "builds_per_s": 1000.0 / t["ms_per_step"],
             "fock_pairs_per_s": m * 1000.0 / t["ms_per_step"],
             "latency_p50_ms": pctl(t["lat"], 50), "latency_p99_ms": pctl(t["lat"], 99),
             "kernel_ms": t["kernel_ms"], "prepare_s": prep_s, "tuner": tune,
             "roofline": roofline(flops, t["kernel_ms"], PEAK_FP32 if leg.startswith("mixed") else PEAK_FP64,
                                  traffic_from_profile(sha, c["name"], leg), eri_bytes,
                                  bound="alu" if leg == "direct" else "mfma"),
             "algorithmic_flops_per_launch": flops,
             "hbm_algorithmic_GBps": eri_bytes / (t["kernel_ms"] / 1000.0) / 1e9,
             "hbm_frac": eri_bytes / (t["kernel_ms"] / 1000.0) / PEAK_HBM,
             "store": {"nquartets_kept": nq, "nblocks": info["nblocks"],
                       "nelements_stored": info["nelements_stored"],
                       "device_GB": info["device_bytes"] / 1e9,
                       "workspace_GB": info["workspace_bytes"] / 1e9}}
        if leg == "fp64" and not args.no_esmf:
            r["esmf_step"] = esmf_leg(pa, st, c, args.steps, args.warmup, stream, sha,
                                      compare=not args.no_esmf_compare)
            log(f"esmf step {r['esmf_step']}")
        r["_jk"] = (j, k)
        st.release()
        del st
        res[leg] = r
    for leg in ("mixed", "store32", "mixed_fp64_store", "direct"):
        if "fp64" in res and leg in res:
            j64, k64 = res["fp64"]["_jk"]
            jm, km = res[leg]["_jk"]
            dj = float((jm - j64).abs().max())
            dk = float((km - k64).abs().max())
            df = float((2.0 * (jm - j64) - (km - k64)).abs().max())
            res[leg]["vs_fp64"] = {"max_abs_dJ": dj, "max_abs_dK": dk, "max_abs_dF": df,
                                   "within_1e-8": bool(max(dj, dk) <= 1e-8)}
            log(f"{leg} vs fp64: {res[leg]['vs_fp64']}")
    for r in res.values():
        r.pop("_jk")
    del d
    torch.cuda.empty_cache()
    head = res[args.prec]
    out = {
        "metric": METRIC, "value": head["builds_per_s"], "unit": "builds/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed": "f32+f64", "store32": "f32 store, f64 math"}[args.prec],
        "data": "synthetic (seeded s-type basis and transition densities)",
        "config": {"workload": c["name"], "nbf": n, "m": m, "tau": c["tau"],
                   "prec": args.prec, "parallelism": "single GPU"},
        "roofline": dict(head["roofline"], kernel="fock_mfma_kernel", kernel_ms=head["kernel_ms"],
                         kernel_source_sha=sha,
                         algorithmic_flops_per_launch=head["algorithmic_flops_per_launch"],
                         hbm_algorithmic_GBps=head["hbm_algorithmic_GBps"],
                         hbm_frac=head["hbm_frac"]),
        "latency_ms": {"p50": head["latency_p50_ms"], "p99": head["latency_p99_ms"]},
        "fock_pairs_per_s": head["fock_pairs_per_s"],
        "prepare_s": head["prepare_s"],
        "tuner": head["tuner"],
        "store": head["store"],
    }
    if "esmf_step" in head:
        out["esmf_step"] = head.pop("esmf_step")
    for leg, r in res.items():
        if leg != args.prec:
            if "esmf_step" in r:
                out["esmf_step"] = r.pop("esmf_step")
            out[leg] = r
    if not args.no_direct and not args.no_direct_deep:
        out["direct_deep"] = direct_deep_leg(pa, min(args.steps, 3), min(args.warmup, 1), stream)
    if not args.no_cart:
        out["cart"] = cart_leg(pa, args.steps, args.warmup, stream)
        log(f"cart {out['cart']}")
        torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = batched_leg(pa, args.steps, args.warmup)
        log(f"batched {out['batched']}")
        torch.cuda.empty_cache()
    if not args.no_serving:
        # the serving mix at two arrival rates (the full sweep: --serving)
        out["serving"] = serving_leg(pa, [float(x) for x in args.serving_rates.split(",")], args.iters,
                                     args.budget_gb * 1e9, args.workspace_gb * 1e9, args.nstreams, args.max_group,
                                     args.max_inflight)
        out["serving_latency_ms"] = {str(int(r["offered_req_per_s"])): {"p50": r["latency_p50_ms"],
                                                                         "p99": r["latency_p99_ms"]}
                                     for r in out["serving"]["rates"]}
        log(f"serving {out['serving_latency_ms']}")
        torch.cuda.empty_cache()
    if not args.no_peaks:
        # the published peaks the roofline divides by, measured on this device
        pk = pa.probe_peaks(8 << 30, stream)
        out["device_peaks_measured"] = pk
        log(f"measured peaks {pk}")
        if args.prec != "mixed":
            rf = out["roofline"]
            rf["measured_peak"] = pk["fp64_mfma_tflops"]
            rf["frac_of_measured_peak"] = rf["achieved"] / pk["fp64_mfma_tflops"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, head["store"]["nquartets_kept"])
        log(f"cpu baseline {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
