"""Benchmark of the matrix-free H.v / TPQ hot path on one MI355X.

Workload (default): Kitaev-Heisenberg model on the 24-site periodic
honeycomb cluster (K = -1, J = 0.1, link directions drawn per link), full
2^24 space, microcanonical TPQ (l = 1.5) with 16 samples interleaved in one
batched product, complex64 storage, FP64 reductions and observables.
One step = one batched TPQ step (16 H.v products + fused reductions); the
K timed steps are one hphi_tpq_run call (graph replays after the first step).

Also measured in the same run:
  * the plain FP64 single-vector path (same Hamiltonian, one complex128
    vector per step) in samples*iterations/s;
  * the product alone, as a step calls it, timed with HIP events on the
    stream it is launched on, for the roofline (algorithmic bytes = dim *
    nvec * 16 B), next to a plain 2 GiB device copy;
  * the mixed-precision gate outside the timed region: all 16 samples for
    the configured 2000 steps in complex64 and in complex128 from the same
    psi_0, every step's energy compared, and the complex64 state re-evaluated
    with an FP64 product every 500 steps;
  * the C oracle on a bounded row slice of the same workload (host cores,
    median of 3 runs).

Other workloads (--workload): hubbard18, heis_chain16, hubbard_4x3, tri24,
kagome36 (Lanczos over 9,075,135,300 rows), kh_honeycomb24_cma.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "H·v products/s and achieved HBM GB/s; batched mixed TPQ vs plain FP64 Lanczos"


def _events_ms(fn, reps, torch):
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        fn()
    end.record()
    end.synchronize()
    return start.elapsed_time(end) / reps


def run_tpq(hp, ham, psi, steps, warmup, l, torch):
    """Run warmup + timed TPQ steps; returns (ms per step, final buffers, obs of the last step)."""
    a = psi
    b = torch.empty_like(a)
    nvec = 1 if a.dim() == 1 else a.shape[1]
    obs = [torch.empty(4 * nvec, dtype=torch.float64, device="cuda") for _ in range(2)]
    scale = None
    k = 1

    def step():
        nonlocal a, b, scale, k
        o = obs[k & 1]
        hp.hphi_tpq_step(ham, a, b, l, k, scale, o)
        a, b = b, a
        scale = o[3 * nvec:4 * nvec]
        k += 1

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
    return ms, a, scale, obs[(k - 1) & 1], k - 1


def cpu_baseline(w, terms, v_host, dim, nvec, target_s=4.0):
    """The C oracle on the host cores, scaled to H.v products/s: a contiguous row slice sized for
    about target_s seconds (whole products if one takes less), one warm-up run, then the median
    of 3 timed runs."""
    import numpy as np
    from oracle import c_oracle
    rows = np.arange(0, 4096, dtype=np.uint64)
    t0 = time.perf_counter()
    c_oracle.rows_hv(terms, rows, v_host)
    dt = time.perf_counter() - t0
    n = int(min(dim, max(4096, 4096 * target_s / max(dt, 1e-6))))
    rows = np.arange(0, n, dtype=np.uint64)
    c_oracle.rows_hv(terms, rows, v_host)       # warm-up
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        c_oracle.rows_hv(terms, rows, v_host)
        times.append(time.perf_counter() - t0)
    dt = sorted(times)[1]
    rate = (n / dim) * nvec / dt
    what = f"rows 0..{n - 1} of {dim}" if n < dim else f"whole products ({dim} rows each)"
    return {"value": rate, "unit": "H·v products/s", "cores": c_oracle.threads(), "kind": "oracle",
            "sample": f"C oracle (hv_oracle.c, OpenMP), {what}, {nvec} complex64 vectors, median of 3 runs "
                      f"({', '.join(f'{t:.2f}' for t in times)} s) after a warm-up, scaled by dim/rows",
            "host": host_cpu()}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "plan.cpp"):
        with open(os.path.join(ROOT, "paper_1703_03637_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def schedule_key(sched) -> str:
    if isinstance(sched, dict) and "pinned" in sched:
        parts = sched["pinned"].split(",")
        return ",".join(parts + ["1", "1"][len(parts) - 5:] if len(parts) < 7 else parts)
    return ",".join(str(sched[k]) for k in ("windowed", "window_kb", "max_passes", "lanes_per_row",
                                            "blocks_per_cu", "stage_tables", "nt_streams"))


def measured_traffic(sched):
    """HBM bytes per batched product (FETCH_SIZE and WRITE_SIZE, scaled by a
    copy kernel) from the committed PMC summary, if it was taken on the
    current kernel sources for this schedule; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_kh_honeycomb24_tpq_b16_c64.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    entry = rec.get("schedules", {}).get(schedule_key(sched))
    return None if entry is None else entry.get("hbm_bytes_per_product")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="kh_honeycomb24",
                    choices=("kh_honeycomb24", "kh_honeycomb24_cma", "hubbard18", "heis_chain16", "hubbard_4x3",
                             "tri24", "kagome36"),
                    help="kh_honeycomb24: the headline (24-site Kitaev-Heisenberg TPQ, 16 complex64 samples); "
                         "hubbard18: the paper's 18-site Hubbard cluster at half filling (2,363,904,400 rows); "
                         "heis_chain16 / hubbard_4x3: FP64 Lanczos; tri24: the 13 Sz sectors of the 24-site "
                         "triangular torus as one batched FP32 Lanczos; kh_honeycomb24_cma: the headline product "
                         "through the dense-block (continuous-memory-access) variant; kagome36: the 36-site kagome "
                         "Sz = 0 sector (9,075,135,300 rows), Lanczos in FP32 storage with FP64 refinement and in "
                         "FP64, from the same start vector")
    ap.add_argument("--cluster-bits", type=int, default=6, help="kh_honeycomb24_cma: sites per dense cluster")
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 20; 5 for hubbard18)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 3; 1 for hubbard18)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--gate-steps", type=int, default=2000,
                    help="kh_honeycomb24: length of the complex64-vs-FP64 trajectory compared outside the timed "
                         "region (the configured 2000 TPQ steps; 0 skips it)")
    ap.add_argument("--kernel-only", action="store_true",
                    help="kagome36: only time the FP32 and FP64 products of the start vector (profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run three 1 GiB device copies (reference kernel for the PMC byte counters) and exit")
    ap.add_argument("--schedule", default="",
                    help="pin the product schedule 'windowed,window_kb,max_passes,lanes_per_row,blocks_per_cu"
                         "[,stage_tables[,nt_streams]]' for both paths instead of autotuning (used for profiling "
                         "runs)")
    args = ap.parse_args()
    big = args.workload == "hubbard18"
    lanczos_mode = args.workload in ("heis_chain16", "hubbard_4x3", "tri24")
    if args.workload == "kagome36":
        args.steps = 100 if args.steps is None else args.steps
        args.warmup = 0 if args.warmup is None else args.warmup
    if args.steps is None:
        args.steps = 5 if big else (200 if lanczos_mode else 20)
    if args.warmup is None:
        args.warmup = 1 if big else (20 if lanczos_mode else 3)
    if args.schedule:
        keys = ("HPHI_WINDOWED", "HPHI_L2_WINDOW_KB", "HPHI_PASSES", "HPHI_LPR", "HPHI_BLOCKS_PER_CU",
                "HPHI_STAGE_TABLES", "HPHI_NT_STREAMS")
        for k, val in zip(keys, args.schedule.split(",")):
            os.environ[k] = val
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "3 copies of 1 GiB (read 1 GiB + write 1 GiB each)"}))
        return
    import paper_1703_03637_amd as hp
    from synth.configs import workload
    from synth.vectors import device_uniform
    if big:
        run_hubbard18(args, hp, torch, np)
        return
    if lanczos_mode:
        run_lanczos(args, hp, torch, np)
        return
    if args.workload == "kh_honeycomb24_cma":
        run_cma(args, hp, torch, np)
        return
    if args.workload == "kagome36":
        run_kagome36(args, hp, torch, np)
        return

    run_headline(args, hp, torch, np)


def run_headline(args, hp, torch, np):
    """The headline: batched complex64 TPQ on the 24-site Kitaev-Heisenberg honeycomb."""
    from synth.configs import workload
    w = workload("kh_honeycomb24")
    nvec, ns, l = w.nvec, w.basis.n_sites, w.tpq_l
    basis = hp.hphi_basis_build(w.basis)
    ham = hp.hphi_ham_build(basis, w.terms)
    dim = basis.dim

    # ---- start vectors: seeded Gaussian, drawn on the device (one seed per sample)
    def gauss(seed, n, dt):
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        x = torch.randn((dim, n, 2), generator=g, device="cuda", dtype=torch.float64)
        return torch.view_as_complex(x).to(dt).contiguous()

    psi_b = torch.empty((dim, nvec), dtype=torch.complex64, device="cuda")
    for bb, s in enumerate(w.seeds):
        psi_b[:, bb] = gauss(s, 1, torch.complex64)[:, 0]
    psi_1 = psi_b[:, 0].to(torch.complex128).contiguous()     # same psi_0 as sample 0

    # ---- schedule autotuning (set-up, outside the timed region)
    if args.schedule:
        sched_b = sched_1 = {"pinned": args.schedule}
    else:
        sched_b = hp.hphi_hv_tune(ham, psi_b)
        sched_1 = hp.hphi_hv_tune(ham, psi_1)
    torch.cuda.empty_cache()

    # ---- batched mixed-precision TPQ (headline), then the plain FP64 single-vector path: K timed
    # steps, one hphi_tpq_step call each; the same K steps as one graph-replayed hphi_tpq_run call
    # (its set-up included) are reported beside them
    ms_b, st_b = run_tpq_steps(hp, ham, psi_b, args.steps, args.warmup, l, torch)
    ms_1, st_1 = run_tpq_steps(hp, ham, psi_1, args.steps, args.warmup, l, torch)
    ms_bg, _ = run_tpq_graph(hp, ham, psi_b, args.steps, args.warmup, l, torch)
    # the same call over ten times as many steps: the graph instantiation amortized
    long_steps = 10 * args.steps
    ms_bg_long, _ = run_tpq_graph(hp, ham, psi_b, long_steps, 0, l, torch)

    # ---- dominant kernel alone: the batched product exactly as a step calls it (a, b, input scale,
    # reductions), HIP events on the stream it runs on; and one eager step per call for comparison
    cur, oth, scale = st_b
    red = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")
    obs = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")

    def hv_once():
        hp.hphi_hv(ham, cur, oth, a=-1.0 / ns, b=l, in_scale=scale, reduce=red)

    def step_once():
        hp.hphi_tpq_step(ham, cur, oth, l, args.steps + args.warmup + 1, scale, obs)

    hv_once()
    torch.cuda.synchronize()
    k_ms = min(_events_ms(hv_once, args.kernel_reps, torch) for _ in range(3))
    step_ev_ms = min(_events_ms(step_once, args.kernel_reps, torch) for _ in range(3))
    alg_bytes = dim * nvec * 8 * 2                      # read v once, write u once (complex64)
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    copy_gbps = copy_reference(torch)

    value = nvec / (ms_b * 1e-3)                        # H.v products per second
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "H·v products/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_b,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "kh_honeycomb24_tpq_b16_c64", "model": "Kitaev-Heisenberg honeycomb",
                   "n_sites": ns, "dim": dim, "nvec": nvec, "K": -1.0, "J": 0.1, "tpq_l": l,
                   "storage": "complex64", "reductions": "fp64",
                   "timed_call": "hphi_tpq_step, one call per step"},
        "graph_run": {"ms_per_step": ms_bg, "call": "hphi_tpq_run over the same K steps (graph instantiation "
                                                      "and the first, eager step included)",
                      "ms_per_step_long": ms_bg_long, "long_steps": long_steps},
        "hbm_gbps_step": alg_bytes / (ms_b * 1e-3) / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(sched_b),
                     "kernel": "one batched product call as a TPQ step makes it (all passes + reduction)",
                     "kernel_ms": k_ms, "step_ms_events": step_ev_ms, "algorithmic_bytes": alg_bytes,
                     "copy_gbps": copy_gbps, "frac_of_copy": achieved / copy_gbps, "schedule": sched_b},
        "fp64_single_vector": {"ms_per_step": ms_1, "samples_iterations_per_s": 1.0 / (ms_1 * 1e-3),
                               "schedule": sched_1,
                               "batched_samples_iterations_per_s": value,
                               "speedup": value * ms_1 * 1e-3},
    }
    del cur, oth, st_b, st_1
    torch.cuda.empty_cache()
    if args.gate_steps > 0:
        res["energy_check"] = energy_gate(hp, ham, psi_b, l, ns, args.gate_steps, torch, np)
    if not args.no_cpu:
        v_host = psi_b.cpu().numpy()
        res["cpu_baseline"] = cpu_baseline(w, w.terms, v_host, dim, nvec)
    print(json.dumps(res), flush=True)


def run_tpq_steps(hp, ham, psi, steps, warmup, l, torch):
    """W untimed steps, then exactly K timed hphi_tpq_step calls; returns (ms per timed step,
    (buffer holding the state, the other buffer, its scale))."""
    ms, a, scale, _, _ = run_tpq(hp, ham, psi.clone(), steps, warmup, l, torch)
    b = torch.empty_like(a)
    return ms, (a, b, scale)


def run_tpq_graph(hp, ham, psi, steps, warmup, l, torch):
    """W untimed steps, then exactly K timed steps in one hphi_tpq_run call (graph replays);
    returns (ms per timed step, (buffer holding the state, the other buffer, its scale))."""
    a = psi.clone()
    b = torch.empty_like(a)
    scale = None
    k = 1
    if warmup > 0:
        log = hp.hphi_tpq_run(ham, a, b, l, k, warmup)
        scale = log[warmup - 1, 3].contiguous()
        if warmup % 2:
            a, b = b, a
        k += warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    log = hp.hphi_tpq_run(ham, a, b, l, k, steps, in_scale=scale)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
    if steps > 0:
        scale = log[steps - 1, 3].contiguous()
        if steps % 2:
            a, b = b, a
    return ms, (a, b, scale)


def energy_gate(hp, ham, psi_b, l, ns, n_steps, torch, np, chunk=500):
    """The mixed-precision gate over a whole trajectory, outside the timed region: all samples run
    n_steps TPQ steps in complex64 storage and, from the same psi_0, in complex128 (FP64 path).
    Every step's energy per site u_k (an FP64 reduction of the stored state) is compared; at every
    `chunk` steps the complex64 state is also re-evaluated with a separate FP64 product."""
    nvec = psi_b.shape[1]
    bufs = {torch.complex64: [psi_b.clone(), torch.empty_like(psi_b)],
            torch.complex128: [psi_b.to(torch.complex128), None]}
    bufs[torch.complex128][1] = torch.empty_like(bufs[torch.complex128][0])
    scales = {torch.complex64: None, torch.complex128: None}
    logs = {torch.complex64: [], torch.complex128: []}
    red = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")
    strict = []
    k = 1
    t0 = time.perf_counter()
    while k <= n_steps:
        n = min(chunk, n_steps - k + 1)
        u_eval = {}
        for dt in (torch.complex64, torch.complex128):
            a, b = bufs[dt]
            log = hp.hphi_tpq_run(ham, a, b, l, k, n, in_scale=scales[dt])
            logs[dt].append(log.cpu().numpy())
            if n % 2:
                bufs[dt] = [b, a]
            scales[dt] = log[n - 1, 3].contiguous()
            x = (bufs[dt][0].to(torch.complex128) * scales[dt].to(torch.complex128)).contiguous()
            hp.hphi_hv(ham, x, reduce=red, write=False)
            r = red.cpu().numpy().reshape(4, nvec)
            u_eval[dt] = r[1] / r[0] / ns
            del x
        k += n
        rel = np.abs(u_eval[torch.complex64] - u_eval[torch.complex128]) / np.abs(u_eval[torch.complex128])
        strict.append({"step": k - 1, "max_rel_err": float(rel.max())})
    lo = np.concatenate(logs[torch.complex64])
    hi = np.concatenate(logs[torch.complex128])
    du = np.abs(lo[:, 0, :] - hi[:, 0, :])
    rel = du / np.abs(hi[:, 0, :])
    worst = np.unravel_index(np.argmax(rel), rel.shape)
    # near infinite temperature u_k passes through zero, where a relative error is not defined: the
    # gate reads |du/u| over the steps with |u_k| >= 0.01 (0.02 of the energy range), and the
    # absolute error over all steps is reported beside it
    sel = np.abs(hi[:, 0, :]) >= 1e-2
    rel_sel = float(rel[sel].max()) if sel.any() else float("nan")
    drel_beta = np.abs(lo[1:, 2, :] - hi[1:, 2, :]) / np.abs(hi[1:, 2, :])
    return {"steps": n_steps, "samples": nvec, "reference": "complex128 FP64 path from the same psi_0",
            "max_rel_err": float(rel.max()), "max_rel_err_at": {"step": int(worst[0]), "sample": int(worst[1]),
                                                                "u": float(hi[worst[0], 0, worst[1]])},
            "max_rel_err_where_abs_u_ge_0.01": rel_sel, "steps_with_abs_u_below_0.01": int((~sel).sum()),
            "max_abs_err": float(du.max()), "final_rel_err": float(rel[-1].max()),
            "final_u": [float(x) for x in hi[-1, 0, :4]], "final_beta": float(hi[-1, 2, :].mean()),
            "beta_max_rel_err": float(drel_beta.max()), "fp64_reevaluation": strict,
            "gate": 1e-8, "passed": bool(rel_sel <= 1e-8 and max(x["max_rel_err"] for x in strict) <= 1e-8),
            "seconds": time.perf_counter() - t0}


def copy_reference(torch, nbytes=2 << 30, reps=5):
    """Plain device copy of 2 GiB (read + write), GB/s by HIP events: the measured bandwidth
    ceiling the roofline fraction is also quoted against."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    ms = min(_events_ms(lambda: b.copy_(a), reps, torch) for _ in range(3))
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def run_lanczos(args, hp, torch, np):
    """Lanczos workloads: one step = one iteration of every problem's
    recurrence (product with the fused alpha sums, update with the fused
    norm, device-side scalars, graph replays).  value = products per second
    over all problems; roofline = the product on the largest problem timed
    alone with HIP events; the FP64 refinement reported per problem."""
    from synth.configs import workload
    from synth.vectors import device_uniform
    name = args.workload
    w = workload("tri24_allsz" if name == "tri24" else name)
    descs = [w.basis] + list(w.extra_bases)
    dt = {"c128": torch.complex128, "f32": torch.float32, "f64": torch.float64, "c64": torch.complex64}[w.dtype]
    cplx = dt.is_complex
    bases = [hp.hphi_basis_build(d) for d in descs]
    hams = [hp.hphi_ham_build(b, w.terms) for b in bases]
    x0 = [device_uniform(b.dim, 0, w.seeds[k % len(w.seeds)], cplx, dt) for k, b in enumerate(bases)]
    hp.hphi_lanczos(hams, x0, args.warmup, refine=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = hp.hphi_lanczos(hams, x0, args.steps, refine=False)
    torch.cuda.synchronize()
    dt_s = time.perf_counter() - t0
    products = sum(r["n_done"] for r in res)
    steps_done = max(r["n_done"] for r in res)
    ms_step = dt_s * 1e3 / steps_done
    ref = hp.hphi_lanczos(hams, x0, args.steps, refine=True)
    # dominant kernel: the product on the largest problem, alone, HIP events
    big = max(range(len(bases)), key=lambda k: bases[k].dim)
    v = x0[big]
    u = torch.empty_like(v)
    hp.hphi_hv(hams[big], v, u)
    torch.cuda.synchronize()
    k_ms = _events_ms(lambda: hp.hphi_hv(hams[big], v, u), max(5, args.kernel_reps), torch)
    esize = v.element_size()
    alg_bytes = bases[big].dim * esize * 2
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    # per step: product reads v_k and v_{k-1}, writes w; update reads w and v_k, writes w
    step_bytes = sum(b.dim for b in bases) * esize * 6
    out = {
        "metric": METRIC,
        "value": products / dt_s,
        "unit": "H·v products/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.dtype,
        "data": "synthetic",
        "config": {"workload": f"{name}_lanczos_{w.dtype}", "problems": len(bases),
                   "dims": [b.dim for b in bases], "n_terms": len(w.terms), "iterations": args.steps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"one product on the largest problem (dim {bases[big].dim})", "kernel_ms": k_ms,
                     "algorithmic_bytes": alg_bytes},
        "step_gbps": step_bytes / (ms_step * 1e-3) / 1e9,
        "refined": [{"dim": b.dim, "e0_ritz": r["e0_ritz"], "e0_refined": r["e0_refined"],
                     "residual": r["residual"]} for b, r in list(zip(bases, ref))[:4]],
    }
    if not args.no_cpu:
        from oracle import c_oracle
        d = descs[big]
        vh = v.cpu().numpy().astype(np.complex128)
        rows_n = 4096
        while True:
            cfg = c_oracle.unrank_counted(d, np.arange(min(rows_n, bases[big].dim)))
            t0 = time.perf_counter()
            c_oracle.rows_hv_counted(d, w.terms, cfg, vh)
            dtc = time.perf_counter() - t0
            if dtc >= 10.0 or rows_n >= bases[big].dim:
                break
            rows_n = int(min(bases[big].dim, rows_n * min(50.0, 12.0 / max(dtc, 1e-3))))
        n_rows = len(cfg)
        reps, t0 = 0, time.perf_counter()
        while True:
            c_oracle.rows_hv_counted(d, w.terms, cfg, vh)
            reps += 1
            dtc = time.perf_counter() - t0
            if n_rows < bases[big].dim or dtc >= 10.0:
                break
        out["cpu_baseline"] = {"value": reps * (n_rows / bases[big].dim) / dtc, "unit": "H·v products/s",
                               "cores": c_oracle.threads(), "kind": "oracle",
                               "sample": f"C oracle (hv_oracle.c, OpenMP, counting ranks), {reps} x rows "
                                         f"0..{n_rows - 1} of the largest problem ({bases[big].dim} rows), "
                                         f"{dtc:.1f} s"}
    print(json.dumps(out), flush=True)


def run_hubbard18(args, hp, torch, np):
    """The paper's 18-site Hubbard TPQ workload on one GPU: four complex64
    samples in one batched product (headline of this mode) against the plain
    FP64 single-vector path, with the energy check, the HIP-event roofline of
    the batched product and the C oracle (targets ranked by counting)."""
    from synth.configs import workload
    w = workload("hubbard18_tpq")
    nvec, ns, l = 4, w.basis.n_sites, w.tpq_l
    basis = hp.hphi_basis_build(w.basis)
    ham = hp.hphi_ham_build(basis, w.terms)
    dim = basis.dim

    def gauss(seed, n, dt):
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        x = torch.empty((dim, n, 2), device="cuda", dtype=torch.float32).normal_(generator=g)
        return torch.view_as_complex(x).to(dt).contiguous()

    psi_b = gauss(w.seeds[0], nvec, torch.complex64)                 # 75.6 GB
    psi_1 = psi_b[:, 0].to(torch.complex128).contiguous()            # 37.8 GB, same psi_0 as sample 0
    ms_b, fin_b, _, _, k_b = run_tpq(hp, ham, psi_b, args.steps, args.warmup, l, torch)
    # dominant kernel alone: the batched product, HIP events on its stream
    out = psi_b if fin_b.data_ptr() != psi_b.data_ptr() else torch.empty_like(fin_b)
    sc = torch.ones(nvec, dtype=torch.float64, device="cuda")

    def hv_once():
        hp.hphi_hv(ham, fin_b, out, a=-1.0 / ns, b=l, in_scale=sc)

    hv_once()
    torch.cuda.synchronize()
    k_ms = _events_ms(hv_once, max(2, args.kernel_reps // 5), torch)
    x64 = fin_b[:, 0].to(torch.complex128).contiguous()
    del psi_b, fin_b, out
    torch.cuda.empty_cache()
    ms_1, fin_1, _, _, k_1 = run_tpq(hp, ham, psi_1, args.steps, args.warmup, l, torch)
    assert k_b == k_1
    red = torch.empty(4, dtype=torch.float64, device="cuda")
    hp.hphi_hv(ham, x64, reduce=red, write=False)
    r = red.cpu().numpy()
    u_mixed = r[1] / r[0] / ns
    hp.hphi_hv(ham, fin_1, reduce=red, write=False)
    r = red.cpu().numpy()
    u_fp64 = r[1] / r[0] / ns
    alg_bytes = dim * nvec * 8 * 2
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    value = nvec / (ms_b * 1e-3)
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "H·v products/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_b,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "hubbard18_tpq_b4_c64", "model": "Hubbard, 18-site tilted square cluster",
                   "n_sites": ns, "dim": dim, "nvec": nvec, "t": 1.0, "U": 8.0, "n_up": 9, "n_dn": 9,
                   "tpq_l": l, "storage": "complex64", "reductions": "fp64"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "one batched product call (hv_kernel, sector, 36-bit)", "kernel_ms": k_ms,
                     "algorithmic_bytes": alg_bytes},
        "fp64_single_vector": {"ms_per_step": ms_1, "samples_iterations_per_s": 1.0 / (ms_1 * 1e-3),
                               "batched_samples_iterations_per_s": value, "speedup": value * ms_1 * 1e-3,
                               "tpq_steps_per_hour": 3600.0 / (ms_1 * 1e-3)},
        "energy_check": {"step": k_b, "u_mixed_fp64_eval": u_mixed, "u_fp64_path": u_fp64,
                         "rel_err": abs(u_mixed - u_fp64) / abs(u_fp64), "gate": 1e-8},
    }
    if not args.no_cpu:
        from oracle import c_oracle
        v_host = fin_1.cpu().numpy()
        rows_n = 4096
        while True:       # grow the row slice until the oracle works for 10-30 s
            cfg = c_oracle.unrank_counted(w.basis, np.arange(rows_n))
            t0 = time.perf_counter()
            c_oracle.rows_hv_counted(w.basis, w.terms, cfg, v_host)
            dt = time.perf_counter() - t0
            if dt >= 10.0 or rows_n >= dim:
                break
            rows_n = int(min(dim, rows_n * min(50.0, 12.0 / max(dt, 1e-3))))
        res["cpu_baseline"] = {"value": (rows_n / dim) / dt, "unit": "H·v products/s", "cores": c_oracle.threads(),
                               "kind": "oracle",
                               "sample": f"C oracle (hv_oracle.c, OpenMP, targets ranked by counting), rows "
                                         f"0..{rows_n - 1} of {dim}, one complex128 vector, {dt:.1f} s, "
                                         f"scaled by dim/rows"}
    print(json.dumps(res), flush=True)


def run_cma(args, hp, torch, np):
    """The headline product (24-site Kitaev-Heisenberg, 16 complex64 vectors, with the TPQ step's
    a, b and reductions) through the dense-block variant, next to the pull product."""
    from synth.configs import workload
    from synth.vectors import device_uniform
    w = workload("kh_honeycomb24")
    nvec, ns, l, m = w.nvec, w.basis.n_sites, w.tpq_l, args.cluster_bits
    basis = hp.hphi_basis_build(w.basis)
    ham = hp.hphi_ham_build(basis, w.terms)
    dim = basis.dim
    clusters = hp.hphi_hv_cma_plan(ham, m)
    psi = device_uniform(dim, nvec, 915, True, torch.complex64)
    u = torch.empty_like(psi)
    red = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")

    def cma():
        hp.hphi_hv_cma(ham, psi, u, cluster_bits=m, a=-1.0 / ns, b=l, reduce=red)

    for _ in range(args.warmup):
        cma()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cma()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k_ms = _events_ms(cma, max(5, args.kernel_reps), torch)
    red_cma = red.cpu().numpy().copy()
    u_cma = u[:4096].cpu().numpy().copy()
    # the pull product on the same input, tuned as in the headline run
    sched = hp.hphi_hv_tune(ham, psi)

    def pull():
        hp.hphi_hv(ham, psi, u, a=-1.0 / ns, b=l, reduce=red)

    pull()
    torch.cuda.synchronize()
    p_ms = _events_ms(pull, max(5, args.kernel_reps), torch)
    red_pull = red.cpu().numpy()
    u_pull = u[:4096].cpu().numpy()
    V = dim * nvec * 8                                   # bytes of one 16-vector complex64 array
    n_c = len(clusters)
    # per cluster: read v, write u, and read u after the first (the last cluster also finishes the product)
    alg_bytes = n_c * 2 * V + (n_c - 1) * V
    flops = n_c * 2.0 * dim * (1 << m) * (2 * nvec)
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    out = {
        "metric": "H·v products/s (dense-block variant)",
        "value": args.steps / dt,
        "unit": "H·v products/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "kh_honeycomb24_cma_b16_c64", "n_sites": ns, "dim": dim, "nvec": nvec,
                   "cluster_bits": m, "clusters": n_c, "storage": "complex64",
                   "block_sums": "fp32 (MFMA)", "reductions": "fp64"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "one dense-block product call (all clusters)", "kernel_ms": k_ms,
                     "algorithmic_bytes": alg_bytes},
        "mfma": {"flop_per_product": flops, "achieved_tflops": flops / (k_ms * 1e-3) / 1e12,
                 "peak_tflops": 157.3, "frac": flops / (k_ms * 1e-3) / 1e12 / 157.3},
        "pull_product": {"ms": p_ms, "schedule": sched, "speedup_of_pull": k_ms / p_ms},
        "agreement": {"max_rel_reduction_diff": float(np.max(np.abs(red_cma - red_pull) /
                                                             np.maximum(np.abs(red_pull), 1e-300))),
                      "max_abs_u_diff_first_4096_rows": float(np.abs(u_cma - u_pull).max())},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, w.terms, psi.cpu().numpy(), dim, nvec)
    print(json.dumps(out), flush=True)


def run_kagome36(args, hp, torch, np):
    """The 36-site kagome Heisenberg torus, Sz = 0 (9,075,135,300 rows, 36-bit split rank tables):
    K Lanczos steps with FP32 storage, the second pass and FP64 refinement; then the FP64 path from
    the same start vector (upcast), its eigenvector written over the start vector so that the run
    fits the 288 GB of one GPU (v0 + two work vectors + nothing else: 218 GB).  The energies of
    the two runs are compared (no independent value exists at this size).  value = products/s of
    the FP32 run (both passes and the two refinement products)."""
    from synth.configs import workload
    from oracle import c_oracle
    w = workload("kagome36_sz0")
    n_iter = args.steps
    os.environ.setdefault("HPHI_PROGRESS", "10")     # the library reports every 10 Lanczos steps on stderr
    basis = hp.hphi_basis_build(w.basis)
    ham = hp.hphi_ham_build(basis, w.terms)
    dim = basis.dim
    g = torch.Generator(device="cuda")
    g.manual_seed(w.seeds[0])
    v0 = torch.empty(dim, dtype=torch.float32, device="cuda").normal_(generator=g)   # 36.3 GB
    if args.kernel_only:
        prod = {}
        for label, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
            x = v0 if dt == torch.float32 else v0.to(dt)
            u = torch.empty_like(x)
            hp.hphi_hv(ham, x, u)
            torch.cuda.synchronize()
            k_ms = _events_ms(lambda: hp.hphi_hv(ham, x, u), 2, torch)
            prod[label] = {"product_ms": k_ms, "gbps": dim * x.element_size() * 2 / (k_ms * 1e-3) / 1e9}
            print(f"[kagome36] {label} product {k_ms:.1f} ms", file=sys.stderr, flush=True)
            del x, u
            torch.cuda.empty_cache()
        print(json.dumps({"workload": "kagome36_sz0_products", "dim": dim, "products": prod}), flush=True)
        return
    out = {}
    for label, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        if dt == torch.float64:
            v0 = v0.to(torch.float64)                    # 72.6 GB, the same start vector upcast
            torch.cuda.empty_cache()
        work = torch.empty(2 * dim, dtype=dt, device="cuda")
        x_out = v0 if dt == torch.float64 else torch.empty(dim, dtype=torch.float64, device="cuda")
        u = work[:dim]
        hp.hphi_hv(ham, v0, u)
        torch.cuda.synchronize()
        k_ms = _events_ms(lambda: hp.hphi_hv(ham, v0, u), 2, torch)
        print(f"[kagome36] {label}: product {k_ms:.1f} ms; {n_iter} Lanczos steps + second pass + refinement",
              file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        r = hp.hphi_lanczos([ham], [v0], n_iter, work=[work], x_out=[x_out])[0]
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        products = 2 * r["n_done"] + 2
        esize = v0.element_size()
        out[label] = {"seconds": sec, "products": products, "products_per_s": products / sec,
                      "ms_per_iteration": sec * 1e3 / (2 * r["n_done"]), "product_ms": k_ms,
                      "product_gbps": dim * esize * 2 / (k_ms * 1e-3) / 1e9, "n_done": r["n_done"],
                      "e0_ritz": r["e0_ritz"], "e0_refined": r["e0_refined"], "variance": r["variance"],
                      "residual": r["residual"],
                      "peak_memory_gb": torch.cuda.max_memory_allocated() / 1e9}
        print(f"[kagome36] {label}: {json.dumps(out[label])}", file=sys.stderr, flush=True)
        del work, x_out, u, r      # r holds the eigenvector (x_out) too
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats()
    f32, f64 = out["fp32"], out["fp64"]
    res = {
        "metric": METRIC,
        "value": f32["products_per_s"],
        "unit": "H·v products/s",
        "n_gpus": 1,
        "steps": n_iter,
        "warmup": 0,
        "ms_per_step": f32["ms_per_iteration"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "kagome36_sz0_lanczos", "n_sites": 36, "dim": dim, "bonds": len(w.terms),
                   "split_bits": 18, "iterations": n_iter, "storage": "f32 (and f64)", "refine": "fp64"},
        "roofline": {"bound": "hbm", "achieved": f32["product_gbps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": f32["product_gbps"] / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "one FP32 product (hv_kernel, sector, 36-bit)", "kernel_ms": f32["product_ms"],
                     "algorithmic_bytes": dim * 4 * 2},
        "runs": out,
        "energy_check": {"e0_fp32_refined": f32["e0_refined"], "e0_fp64_refined": f64["e0_refined"],
                         "rel_diff": abs(f32["e0_refined"] - f64["e0_refined"]) / abs(f64["e0_refined"]),
                         "gate": 1e-8, "reference": "FP64 GPU run from the same start vector (no independent value "
                                                     "at this size)"},
    }
    if not args.no_cpu:
        rows_n = 1 << 16
        while True:
            cfg = c_oracle.unrank_counted(w.basis, np.arange(rows_n))
            t0 = time.perf_counter()
            c_oracle.rows_hv_counted_ondemand(w.basis, w.terms, cfg, 5)
            dtc = time.perf_counter() - t0
            if dtc >= 8.0 or rows_n >= 1 << 24:
                break
            rows_n = int(rows_n * min(16.0, 10.0 / max(dtc, 1e-3)))
        res["cpu_baseline"] = {"value": (rows_n / dim) / dtc, "unit": "H·v products/s", "cores": c_oracle.threads(),
                               "kind": "oracle",
                               "sample": f"C oracle (hv_oracle.c, OpenMP, counting ranks, input evaluated on demand), "
                                         f"rows 0..{rows_n - 1} of {dim}, {dtc:.1f} s, extrapolated by dim/rows",
                               "host": host_cpu()}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
