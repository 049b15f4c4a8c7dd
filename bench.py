#!/usr/bin/env python3
"""Throughput of the periodic RPA hot path on one MI355X.

One step = the whole hot path for one q-point of the workload and all of its imaginary
frequencies: device Philox generation of B(q), chi0 for every (q, w) point of that q,
Pi = V^(1/2) chi0 V^(1/2) and the Cholesky log-det, all in librpa's kernels, with the
inputs (band energies, V^(1/2), frequency nodes, the Philox seed) resident in HBM before
timing starts.  Steps visit the q-points in turn; once every q has been visited, the
energy E = sum_q zeta_q sum_j W_j eps(q, w_j) / (2 pi) is assembled from the timed steps.

The default workload is the largest single-GPU configuration (3x3x1 k-grid, N_occ 96,
N_virt 900, N_aux 2400, 16 frequencies) in FP64; the FP32 and split-BF16 contractions of
the same workload are timed over one sweep of the q-points next to it and their energies
compared with the FP64 one.

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

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "f16x3": 2500.0}
PREC_CODE = {"fp64": 0, "fp32": 1, "bf16x3": 2, "f16x3": 3}
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
    src = {"fp64": "chi0_f64.hip", "fp32": "chi0_mixed.hip", "bf16x3": "chi0_bf16.hip", "f16x3": "chi0_bf16.hip"}[prec]
    f = os.path.join(ROOT, "profiles", f"chi0_{prec}_{workload}_traffic.json")
    if not os.path.exists(f) or not os.path.exists(os.path.join(ROOT, "paper_2505_06021_amd", "csrc", src)):
        return None
    d = json.load(open(f))
    if d.get("kernel_source_sha256_16") != kernel_source_hash(src):
        return None
    return d.get("bytes_per_launch")


def host_info():
    """BLAS library, its threads, and the host's physical and logical cores."""
    import numpy as np   # noqa: F401  (loads the BLAS whose thread pool is reported)
    info = {"blas": None, "threads": os.cpu_count() or 1,
            "logical_cores": os.cpu_count(), "physical_cores": None}
    try:
        import psutil
        info["physical_cores"] = psutil.cpu_count(logical=False)
    except Exception:
        pass
    try:
        from threadpoolctl import threadpool_info
        pools = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if pools:
            info["blas"] = f"{pools[0].get('internal_api')} {pools[0].get('version')}"
            info["threads"] = max(int(i.get("num_threads", 1)) for i in pools)
    except Exception:
        pass
    return info


def cpu_baseline(make, budget_s=12.0, max_points=24):
    """The oracle as it stands, on the first points of the workload, on the host cores."""
    from oracle import rpa_oracle as orc
    hi = host_info()
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
    return {"value": n / dt, "unit": "points/s", "cores": int(hi["threads"]), "kind": "oracle",
            "blas": hi["blas"], "physical_cores": hi["physical_cores"],
            "logical_cores": hi["logical_cores"],
            "sample": f"first {n} (q, w) points of the workload in q-major order, "
                      f"{dt:.1f} s, NumPy FP64 with host Philox B"}


def cpu_baseline_slice(s, nocc_sample=8):
    """The oracle on one (q, w) point of a workload too large to time whole on the host:
    chi0 over a slice of the point's contraction rows (the first k-point and its first
    nocc_sample occupied bands), then Pi and the Cholesky log-det at the full N_aux.  The
    oracle's chi0 costs the same per contraction row everywhere (B rows from the host
    Philox stream, then the weighted rank update), so the point's time is the slice's
    chi0 time scaled by the ratio of rows plus the full-size Pi and log-det time."""
    import dataclasses

    import numpy as np
    from oracle import rpa_oracle as orc
    hi = host_info()
    nocc = min(nocc_sample, s.nocc)
    part = dataclasses.replace(
        s, nk=1, nocc=nocc, kq=np.zeros((s.nq, 1), dtype=np.int32),
        eps_occ=np.ascontiguousarray(s.eps_occ[s.kq[0, :1], :nocc]),
        eps_virt=np.ascontiguousarray(s.eps_virt[:1]), zeta_k=np.ones(1))
    t0 = time.perf_counter()
    c = orc.chi0(part, 0, s.omega[0])
    t1 = time.perf_counter()
    orc.trace_log(orc.pi_matrix(s.vhalf[0], c / s.nk))
    t2 = time.perf_counter()
    rows_full, rows_part = s.M, part.M
    per_point = (t1 - t0) * rows_full / rows_part + (t2 - t1)
    return {"value": 1.0 / per_point, "unit": "points/s", "cores": int(hi["threads"]), "kind": "oracle",
            "blas": hi["blas"], "physical_cores": hi["physical_cores"],
            "logical_cores": hi["logical_cores"],
            "sample": f"one (q, w) point extrapolated from a slice: oracle chi0 over {rows_part} of the "
                      f"point's {rows_full} contraction rows (first k-point, first {nocc} occupied bands) "
                      f"in {t1 - t0:.1f} s, scaled by {rows_full / rows_part:.0f}, plus the full-size "
                      f"Pi and Cholesky log-det ({t2 - t1:.1f} s): {per_point:.0f} s per point; "
                      f"NumPy FP64 with host Philox B"}


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
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64", "f16x3": "f16x3+f64"}[args.prec],
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


def run_steps(ctx, s, m, prec, steps, q0=0, label=""):
    """`steps` steps of one q each (q = q0, q0 + 1, ... mod nq); returns {q: eps[nw]}."""
    import numpy as np
    out = {}
    for i in range(steps):
        q = (q0 + i) % s.nq
        eps = ctx.points(s, [q] * s.nw, s.omega, prec=prec, marshal=m)
        out[q] = np.asarray(eps)
        if label:
            print(f"[bench] {label} step {i} q={q} eps[0]={eps[0]:.10f}", file=sys.stderr, flush=True)
    return out


def energy_of(s, eps_by_q):
    """E from a full set of per-q integrands (None unless every q is there)."""
    if len(eps_by_q) < s.nq:
        return None
    return math.fsum(float(s.zeta_q[q]) * float(s.weight[j]) * float(eps_by_q[q][j]) / (2.0 * math.pi)
                     for q in range(s.nq) for j in range(s.nw))


def chi0_roofline(s, kt, steps, prec_name):
    """Roofline of the chi0 contraction from the HIP-event kernel times of `steps` steps."""
    launches, ms = kt["chi0"]
    pts_per_launch = steps * s.nw / max(launches, 1)
    flops_launch = chi0_flops_per_point(s) * pts_per_launch
    # the split 16-bit contractions issue three MFMA products per real product; their peak
    # is the BF16/FP16 one
    issued_launch = flops_launch * (3.0 if prec_name in ("bf16x3", "f16x3") else 1.0)
    avg_s = ms * 1e-3 / max(launches, 1)
    achieved = issued_launch / avg_s / 1e12 if avg_s > 0 else 0.0
    algorithmic = flops_launch / avg_s / 1e12 if avg_s > 0 else 0.0
    peak = PEAK_TFLOPS[prec_name]
    return {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "kernel": "chi0", "flops_per_launch": issued_launch,
            "algorithmic_flops_per_launch": flops_launch, "algorithmic_TFLOPs": algorithmic,
            "avg_launch_ms": avg_s * 1e3, "launches": launches}


def golden_check(workload, s, eps_by_q, prec_name):
    """Compare the steps' eps with the stored oracle values of the workload."""
    tol = {"fp64": 1e-10, "fp32": 1e-8, "bf16x3": 2e-7, "f16x3": 1e-8}[prec_name]
    out = []
    for name in (f"{workload}.json", f"{workload}_sampled.json"):
        path = os.path.join(ROOT, "tests", "golden", name)
        if not os.path.exists(path):
            continue
        g = json.load(open(path))
        if "points" in g:
            pts = [(p["iq"], p["j"], p["eps"]) for p in g["points"]]
        else:
            pts = [(q, j, g["eps"][q][j]) for q in range(len(g["eps"])) for j in range(len(g["eps"][q]))]
        # scale of a point: the largest |eps| among the stored points of its q (ln det and
        # Tr Pi cancel at large omega, where a point's own |eps| is no scale)
        qmax = {}
        for q, j, ref in pts:
            qmax[q] = max(qmax.get(q, 0.0), abs(ref))
        for q, j, ref in pts:
            if q in eps_by_q:
                out.append((q, j, abs(float(eps_by_q[q][j]) - ref) / qmax[q]))
    if not out:
        return None
    worst = max(r for _, _, r in out)
    return {"points_checked": len(out), "max_err_eps_over_q_scale": worst, "tol": tol, "ok": worst <= tol}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=18)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="slab3x3_naux2400", choices=sorted(WORKLOADS))
    ap.add_argument("--step", default="q", choices=["q", "energy"],
                    help="one step = one q-point and its frequencies (default), or one full rpa_energy "
                         "call over every point of the workload")
    ap.add_argument("--mixed", default="fp32,bf16x3,f16x3",
                    help="reduced-precision contractions timed beside an FP64 run ('none' to skip)")
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

    import numpy as np
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
    t_in = time.perf_counter()
    s = make()
    ctx = rpa.Context(0)
    m = rpa._Marshal(s, device=not args.host_inputs)   # inputs resident in HBM before timing
    prec = PREC_CODE[args.prec]
    npts = s.nw if args.step == "q" else s.nq * s.nw      # points per step
    print(f"[bench] {args.workload} prec={args.prec} points/step={npts} (one q) nq={s.nq} "
          f"warmup={args.warmup} steps={args.steps} (inputs {time.perf_counter() - t_in:.1f} s)",
          file=sys.stderr, flush=True)
    if args.step == "q":
        run_steps(ctx, s, m, prec, args.warmup, label="warmup")
    else:
        for i in range(args.warmup):
            E_w, _ = ctx.energy(s, prec=prec, marshal=m)
            print(f"[bench] warmup {i} E={E_w:.12f}", file=sys.stderr, flush=True)
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eps_by_q = {}
    E_energy = None
    for i in range(args.steps):
        if args.step == "q":
            q = i % s.nq
            eps_by_q[q] = np.asarray(ctx.points(s, [q] * s.nw, s.omega, prec=prec, marshal=m))
        else:
            E_energy, grid = ctx.energy(s, prec=prec, marshal=m)
            eps_by_q = {q: grid[q] for q in range(s.nq)}
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = ctx.profile_read()
    ctx.profile(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    print(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step", file=sys.stderr, flush=True)
    roof = chi0_roofline(s, kt, args.steps * npts // s.nw, args.prec)
    roof["traffic"] = traffic_from_profiles(args.workload, args.prec)
    E = energy_of(s, eps_by_q) if E_energy is None else E_energy
    check = {"E": E, "q_visited": sorted(eps_by_q)}
    gold = os.path.join(ROOT, "tests", "golden", f"{args.workload}.json")
    if E is not None and os.path.exists(gold):
        g = json.load(open(gold))
        if "E" in g:
            check.update(E_oracle=g["E"], rel_err=abs(E - g["E"]) / abs(g["E"]))
    check["sampled"] = golden_check(args.workload, s, eps_by_q, args.prec)
    tiles = {p: sorted({v for k, v in rpa.tuned().items()
                        if k.startswith({"fp64": "f64_", "fp32": "f32_", "bf16x3": "bf16_", "f16x3": "bf16_"}[p])})
             for p in PREC_CODE}

    # the reduced-precision contractions of the same workload: one sweep of the q-points
    mixed = {}
    wanted = [] if args.mixed == "none" or args.prec != "fp64" else args.mixed.split(",")
    for pname in wanted:
        pc = PREC_CODE[pname]
        run_steps(ctx, s, m, pc, 1, label=f"{pname} warmup")
        ctx.profile(True)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        eq = run_steps(ctx, s, m, pc, s.nq)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        kq = ctx.profile_read()
        ctx.profile(False)
        Em = energy_of(s, eq)
        r = chi0_roofline(s, kq, s.nq, pname)
        dmax = max(float(np.max(np.abs(eq[q] - eps_by_q[q]) / np.abs(eps_by_q[q])))
                   for q in eq if q in eps_by_q) if eps_by_q else None
        mixed[pname] = {"value": s.nq * s.nw / (tb - ta), "unit": "points/s",
                        "ms_per_step": (tb - ta) * 1e3 / s.nq, "steps": s.nq,
                        "chi0_frac_of_peak": r["frac"], "chi0_peak_TFLOPs": r["peak"],
                        "chi0_avg_launch_ms": r["avg_launch_ms"],
                        "chi0_algorithmic_TFLOPs": r["algorithmic_TFLOPs"],
                        "E": Em, "abs_dE_vs_fp64_Ha_per_cell": abs(Em - E) if (Em is not None and E is not None) else None,
                        "max_rel_deps_vs_fp64": dmax,
                        "sampled": golden_check(args.workload, s, eq, pname),
                        "chi0_tile_config": sorted({v for k, v in rpa.tuned().items()
                                                    if k.startswith({"fp32": "f32_", "bf16x3": "bf16_",
                                                                     "f16x3": "bf16_"}[pname])})}
        print(f"[bench] {pname}: {mixed[pname]['value']:.3f} points/s, dE {mixed[pname]['abs_dE_vs_fp64_Ha_per_cell']}",
              file=sys.stderr, flush=True)
    ctx.close()

    cpu = None
    if not args.no_cpu_baseline:
        # the oracle of a large point takes many minutes on the host: time a slice of one
        cpu = cpu_baseline_slice(s) if s.M * s.naux > 5e8 else cpu_baseline(make)

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
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64", "f16x3": "f16x3+f64"}[args.prec],
        "data": "synthetic (seeded Philox B, Haar-random V, GL frequencies)" +
                ("; inputs handed over as host buffers (PCIe-inclusive)" if args.host_inputs else ""),
        "config": {"workload": args.workload, "grid": list(s.grid), "nk": s.nk, "nq": s.nq, "nk_occ": s.nk_occ, "nbas": s.nbas,
                   "nocc": s.nocc, "nvirt": s.nvirt, "naux": s.naux, "nw": s.nw,
                   "is_complex": s.is_complex, "chi0_precision": args.prec,
                   "step": ("one q-point: B(q) generation and all of its frequencies" if args.step == "q" else
                            "one RPA energy: every (q, w) point and the quadrature"),
                   "B": "Philox4x32-10 on device", "parallelism": "single GPU",
                   "chi0_tile_config": tiles[args.prec]},
        "roofline": roof,
        "kernels_ms_per_step": {k: v[1] / args.steps for k, v in kt.items()},
        "check": check,
        "mixed_precision": mixed or None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
