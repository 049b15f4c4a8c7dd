#!/usr/bin/env python3
"""Throughput of the periodic RPA hot path on one MI355X.

One step = one full RPA correlation energy of the workload: device Philox generation
of B for every q, chi0 for every (q, w) point, Pi = V^(1/2) chi0 V^(1/2), the Cholesky
log-det and the q/w quadrature, all in librpa's kernels, with the inputs (band
energies, V^(1/2), weights, the Philox seed) resident in HBM before timing starts.

Prints one JSON line: (q, w) points per second, the roofline position of the dominant
kernel (chi0) from HIP events recorded on its stream, and the CPU oracle timed on a
bounded sample of the same workload on the host cores.
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

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}
PREC_CODE = {"fp64": 0, "fp32": 1, "bf16x3": 2}
WORKLOADS = {
    "slab3x3_naux384": "slab_3x3_384",
    "gamma_real_naux128": "gamma_real_128",
    "slab6x6_naux1200": "slab_6x6_1200",
    "slab3x3_naux2400": "slab_3x3_2400",
    "slab3x3_dual_naux384": "slab_3x3_dual_384",
    "slab3x3_ao_naux384": "slab_3x3_ao_384",
}


def chi0_flops_per_point(s):
    """Algorithmic flops of chi0 for one (q, w) point: Hermitian half of B^H W B."""
    M, N = s.M, s.naux
    return (4.0 if s.is_complex else 1.0) * M * N * (N + 1)


def code_hash(text):
    """Hash of a source text's code: // comments, trailing blanks and empty lines are left
    out, so a change of comments alone keeps the counter records of a kernel valid."""
    lines = []
    for ln in text.splitlines():
        i = ln.find("//")
        if i >= 0:
            ln = ln[:i]
        ln = ln.rstrip()
        if ln:
            lines.append(ln)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()[:16]


def kernel_source_hash(name):
    p = os.path.join(ROOT, "paper_2505_06021_amd", "csrc", name)
    return code_hash(open(p).read())


def traffic_from_profiles(workload, prec):
    """HBM bytes per chi0 launch from committed counter runs, if the kernel is unchanged."""
    src = {"fp64": "chi0_f64.hip", "fp32": "chi0_mixed.hip", "bf16x3": "chi0_bf16.hip"}[prec]
    f = os.path.join(ROOT, "profiles", f"chi0_{prec}_{workload}_traffic.json")
    if not os.path.exists(f) or not os.path.exists(os.path.join(ROOT, "paper_2505_06021_amd", "csrc", src)):
        return None
    d = json.load(open(f))
    if d.get("kernel_source_sha256_16") != kernel_source_hash(src):
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(make, budget_s=12.0, max_points=24):
    """The oracle as it stands, on the first points of the workload, on the host cores."""
    from oracle import rpa_oracle as orc
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    s = make()
    pts = [(q, j) for q in range(s.nq) for j in range(s.nw)]
    t0 = time.perf_counter()
    n = 0
    for (q, j) in pts[:max_points]:
        orc.point(s, q, j)
        n += 1
        if time.perf_counter() - t0 > budget_s and n >= 2:
            break
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "points/s", "cores": int(threads), "kind": "oracle",
            "sample": f"first {n} (q, w) points of the workload in q-major order, "
                      f"{dt:.1f} s, NumPy FP64 with host Philox B"}


def serving(args):
    """Replay the Poisson job stream through rpa_submit/rpa_poll (continuous batching) and
    compare with the same jobs run one at a time in FP64 (FIFO replay of measured service
    times).  Prints one JSON line."""
    import numpy as np
    import torch
    from paper_2505_06021_amd import inputs, rpa

    jobs = inputs.serving_jobs(args.jobs, rate=args.rate, seed=77)
    t_gen = time.perf_counter()
    systems = []
    for i, j in enumerate(jobs):
        systems.append(inputs.make_job_system(j))
        if i % 32 == 31:
            print(f"[serve] inputs {i + 1}/{len(jobs)} ({time.perf_counter() - t_gen:.0f} s)",
                  file=sys.stderr, flush=True)
    prec = PREC_CODE[args.prec]
    ctx = rpa.Context(0, hbm_limit=int(args.hbm_limit_gb * 1e9))
    ctx.energy(systems[0], prec=prec)                   # warm the library and kernels
    torch.cuda.synchronize()
    ids = []
    t0 = time.perf_counter()
    for j, s in zip(jobs, systems):
        delay = t0 + j["arrival"] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        ids.append(ctx.submit(s, prec=prec))
        if len(ids) % 32 == 0:
            print(f"[serve] submitted {len(ids)} at {time.perf_counter() - t0:.1f} s "
                  f"{ctx.stats()}", file=sys.stderr, flush=True)
    res = []
    for n, (jid, s) in enumerate(zip(ids, systems)):
        r, _ = ctx.poll(jid, timeout_ms=-1)
        res.append(r)
        if n % 64 == 63:
            print(f"[serve] collected {n + 1}", file=sys.stderr, flush=True)
    st = ctx.stats()
    lat = np.array([r["t_done"] - r["t_submit"] for r in res])
    first = min(r["t_submit"] for r in res)
    last = min(r["t_done"] for r in res), max(r["t_done"] for r in res)
    npts = sum(r["npoints"] for r in res)
    span = last[1] - first
    # the same jobs one at a time in FP64: service times and reference energies
    svc, dE, rel = [], [], []
    for n, (s, r) in enumerate(zip(systems, res)):
        ta = time.perf_counter()
        E64, _ = ctx.energy(s, prec=0)
        svc.append(time.perf_counter() - ta)
        dE.append(abs(r["E"] - E64))
        rel.append(abs(r["E"] - E64) / abs(E64))
        if n % 32 == 31:
            print(f"[serve] fp64 reference {n + 1}/{len(jobs)}", file=sys.stderr, flush=True)
    ctx.close()
    arr = np.array([j["arrival"] for j in jobs])
    fin, t = [], 0.0
    for a, sv in zip(arr, svc):
        t = max(t, a) + sv
        fin.append(t)
    fifo_lat = np.array(fin) - arr
    line = {
        "metric": "serving: (q,w) RPA points/s with p50/p99 job latency",
        "value": npts / span,
        "unit": "points/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": span * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64"}[args.prec],
        "data": "synthetic job stream (seeded Poisson arrivals, log-uniform N_aux)",
        "config": {"workload": "serving_stream", "jobs": len(jobs), "rate_per_s": args.rate,
                   "naux": "log-U[200,1500]", "grids": "1x1x1 | 2x2x1 | 3x3x1", "nw": "U{8..16}",
                   "chi0_precision": args.prec, "hbm_limit": st["hbm_limit"],
                   "workers": int(os.environ.get("RPA_SERVE_WORKERS", "4"))},
        "serving": {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                    "max_s": float(lat.max()), "points": int(npts), "span_s": span,
                    "hbm_high_water": st["hbm_high_water"],
                    "fused_contraction_launches": st.get("fused_launches"),
                    "fused_sub_batches": st.get("fused_groups"),
                    "unfused_sub_batches": st.get("solo_groups"),
                    "max_abs_dE_vs_fp64_Ha": float(max(dE)), "max_rel_dE_vs_fp64": float(max(rel)),
                    "p50_abs_dE_vs_fp64_Ha": float(np.percentile(dE, 50)),
                    "jobs_above_1e-6_Ha": int(sum(1 for x in dE if x > 1e-6)),
                    "worst_job": {k: jobs[int(np.argmax(dE))][k] for k in ("id", "naux", "nocc", "nvirt", "grid", "nw")},
                    "fifo_fp64": {"p50_s": float(np.percentile(fifo_lat, 50)),
                                  "p99_s": float(np.percentile(fifo_lat, 99)),
                                  "points_per_s": npts / (fin[-1] - arr[0]) if fin else None,
                                  "total_service_s": float(sum(svc))}},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="slab3x3_naux384", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default="fp64", choices=sorted(PREC_CODE))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", action="store_true",
                    help="replay the serving job stream instead of the single-system step")
    ap.add_argument("--jobs", type=int, default=256)
    ap.add_argument("--rate", type=float, default=4.0)
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a plain 1 GiB device copy first (scale reference for HBM counters)")
    ap.add_argument("--hbm-limit-gb", type=float, default=200.0,
                    help="device-memory admission limit of the serving context")
    ap.add_argument("--host-inputs", action="store_true",
                    help="hand the inputs over as host buffers, so each step includes their "
                         "host-to-device copies (a PCIe-inclusive rate; the default keeps them in HBM)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the (q, w) points would shard by q across GPUs; this library runs on one).",
              file=sys.stderr, flush=True)
        sys.exit(2)

    if args.serve:
        serving(args)
        return

    import torch
    from paper_2505_06021_amd import inputs, rpa

    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)   # writes 1 GiB
        dst = torch.empty_like(src)
        torch.add(src, 1.0, out=dst)          # an elementwise kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        print("[bench] calibration: fill writes 1 GiB; add reads 1 GiB and writes 1 GiB",
              file=sys.stderr, flush=True)
        del src, dst

    make = getattr(inputs, WORKLOADS[args.workload])
    s = make()
    npts = s.nq * s.nw
    ctx = rpa.Context(0)
    m = rpa._Marshal(s, device=not args.host_inputs)   # inputs resident in HBM before timing
    prec = PREC_CODE[args.prec]
    print(f"[bench] {args.workload} prec={args.prec} points/step={npts} warmup={args.warmup} "
          f"steps={args.steps}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        E, _ = ctx.energy(s, prec=prec, marshal=m)
        print(f"[bench] warmup {i} E={E:.12f}", file=sys.stderr, flush=True)
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        E, eps = ctx.energy(s, prec=prec, marshal=m)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = ctx.profile_read()
    ctx.profile(False)
    ctx.close()
    ms_step = (t1 - t0) * 1e3 / args.steps
    print(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step", file=sys.stderr, flush=True)

    launches, ms = kt["chi0"]
    pts_per_launch = args.steps * npts / max(launches, 1)
    flops_launch = chi0_flops_per_point(s) * pts_per_launch
    # split-BF16 issues three MFMA products per real product; its peak is the BF16 one
    issued_launch = flops_launch * (3.0 if args.prec == "bf16x3" else 1.0)
    avg_s = ms * 1e-3 / max(launches, 1)
    achieved = issued_launch / avg_s / 1e12 if avg_s > 0 else 0.0
    algorithmic = flops_launch / avg_s / 1e12 if avg_s > 0 else 0.0
    peak = PEAK_TFLOPS[args.prec]
    traffic = traffic_from_profiles(args.workload, args.prec)

    check = None
    gold = os.path.join(ROOT, "tests", "golden", f"{args.workload}.json")
    check = {"E": E}   # the energy of the last timed step (Ha per cell)
    if os.path.exists(gold):
        g = json.load(open(gold))
        check = {"E": E, "E_oracle": g["E"], "rel_err": abs(E - g["E"]) / abs(g["E"])}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(make)

    line = {
        "metric": "(q,w) RPA points/s",
        "value": npts / (ms_step * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64"}[args.prec],
        "data": "synthetic (seeded Philox B, Haar-random V, GL frequencies)" +
                ("; inputs handed over as host buffers (PCIe-inclusive)" if args.host_inputs else ""),
        "config": {"workload": args.workload, "grid": list(s.grid), "nk": s.nk, "nq": s.nq, "nk_occ": s.nk_occ, "nbas": s.nbas,
                   "nocc": s.nocc, "nvirt": s.nvirt, "naux": s.naux, "nw": s.nw,
                   "is_complex": s.is_complex, "chi0_precision": args.prec,
                   "B": "Philox4x32-10 on device", "parallelism": "single GPU",
                   "chi0_tile_config": sorted({v for k, v in rpa.tuned().items()
                                               if k.startswith({"fp64": "f64_", "fp32": "f32_",
                                                                "bf16x3": "bf16_"}[args.prec])})},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": "chi0", "flops_per_launch": issued_launch,
                     "algorithmic_flops_per_launch": flops_launch,
                     "algorithmic_TFLOPs": algorithmic,
                     "avg_launch_ms": avg_s * 1e3, "launches": launches},
        "kernels_ms_per_step": {k: v[1] / args.steps for k, v in kt.items()},
        "check": check,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
