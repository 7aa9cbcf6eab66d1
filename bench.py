#!/usr/bin/env python
"""Throughput of the separable-SOAP + GAP energy/forces hot path on one MI355X.

A step is one pass of the whole path over one batch of structures already
resident in HBM: neighbour list, descriptor (c_nlm, power spectrum, q), GAP
energies, the adjoint chain and the forces.  Default workload: 262144 atoms in a
periodic 138 A cube (0.1 atoms/A^3, minimum distance 1.2 A), r_cut 5.5 A,
sigma 0.5 A, n_max = l_max = 10, zeta = 4 against 4000 random unit sparse
descriptors with N(0,1) weights, in the workload's mixed-precision mode (BF16
GAP contractions) with the FP64 path timed alongside.  The 4096-atom
workload (n_max = l_max = 8, M = 2000) is timed as well and reported under
"workloads".  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "fp64_TFs": 78.6,  # vector and matrix
    "fp32_TFs": 157.3,
    "bf16_TFs": 2500.0,
}
RMSE_BAR = 1e-4  # eV/A, force RMSE of a mixed mode against the FP64 path


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def workload_setup(name, precision, dev):
    import numpy as np
    import torch

    import synth
    from paper_1905_02142_amd import Soap, SoapParams

    w = synth.workload(name)
    ss = w["structures"]
    pos = np.concatenate([x.positions for x in ss])
    cells = np.stack([x.cell for x in ss])
    pbc = np.stack([x.pbc for x in ss]).astype(np.int32)
    so = np.cumsum([0] + [x.n_atoms for x in ss]).astype(np.int32) if len(ss) > 1 else None
    kw = dict(n_max=w["n_max"], l_max=w["l_max"], r_cut=w["r_cut"], sigma0_r=w["sigma"], sigma0_perp=w["sigma"],
              n_species=w["n_species"])
    soap = Soap(SoapParams(precision=precision, **kw))
    t = lambda a, dt=None: torch.tensor(np.ascontiguousarray(a), device=dev, dtype=dt)
    gap = bool(w["M"])
    st = dict(w=w, structures=ss, n_atoms=len(pos), cells=cells, pbc=pbc, so=so, kw=kw, soap=soap, pos=t(pos),
              spec=t(w["species"], torch.int32), gap=gap, qs=t(w["q_sparse"]) if gap else None,
              al=t(w["alpha"]) if gap else None)
    return st


def cpu_oracle_rate(st, budget_s=10.0, precision="ld", threads=None, neighbours=True):
    """The oracle's atoms/s on a bounded sample of centres spread evenly over the
    workload: descriptor and, with a sparse set, GAP energies and the pair
    gradients of those centres; with ``neighbours`` also the oracle's own
    (brute-force) neighbour search for them, else the lists are built before the
    clock starts (the paper's timings exclude the neighbour list).  The sample is
    sized from a pilot to take about ``budget_s``; a workload that takes less than
    half of it whole is run whole, in as many passes as fill about two thirds of
    it.  ``threads``: OpenMP threads (None: all host cores)."""
    import numpy as np

    import oracle

    log(f"oracle leg: {precision}, {threads or 'all'} threads, neighbour search {'timed' if neighbours else 'before'}")
    w, ss = st["w"], st["structures"]
    p = oracle.Params(**st["kw"])
    offs = np.cumsum([0] + [x.n_atoms for x in ss])
    all_threads = oracle.num_threads(precision)
    oracle.set_num_threads(threads if threads else all_threads, precision)

    def run(k):
        log(f"  oracle sample of {k} centres")
        # centres: every (N/k)-th atom of the concatenated workload
        picks = np.unique(np.linspace(0, offs[-1] - 1, k).astype(np.int64))
        jobs = []
        t_nl = time.perf_counter()
        for b, x in enumerate(ss):
            c = picks[(picks >= offs[b]) & (picks < offs[b + 1])] - offs[b]
            if len(c):
                jobs.append((b, x, c, None if neighbours else oracle.neighbors(x.positions, x.cell, x.pbc,
                                                                               p.r_cut, centres=c)))
        t0 = time.perf_counter() if not neighbours else t_nl
        run.wall = time.perf_counter() - t_nl  # untimed list building counts against the budget
        for b, x, c, nl in jobs:
            if nl is None:
                nl = oracle.neighbors(x.positions, x.cell, x.pbc, p.r_cut, centres=c)
            spec = w["species"][offs[b]:offs[b + 1]]
            q, _ = oracle.descriptor(p, nl, spec, precision=precision)
            if st["gap"]:
                e, qbar, _ = oracle.gap(q, w["q_sparse"], w["alpha"], w["zeta"], precision=precision)
                oracle.descriptor_vjp(p, nl, spec, qbar, precision=precision)
        t1 = time.perf_counter()
        run.wall += t1 - t0
        return len(picks), t1 - t0

    try:
        run(min(offs[-1], 2))  # one-time set-up (tables, library) outside the timing
        k, t = run(min(offs[-1], 4))
        for _ in range(3):  # grow the sample until it takes about the budget (wall time, lists included)
            if run.wall >= 0.5 * budget_s or k >= offs[-1]:
                break
            k, t = run(int(min(offs[-1], max(k + 1, k * 0.8 * budget_s / max(run.wall, 1e-3)))))
        passes = 1
        if k >= offs[-1] and t < 0.5 * budget_s:
            passes = int(np.ceil(2.0 * budget_s / 3.0 / max(t, 1e-3)))
            t = sum(run(k)[1] for _ in range(passes))
        used = oracle.num_threads(precision)
    finally:
        oracle.set_num_threads(all_threads, precision)
    what = "descriptors" + (", GAP energies and pair gradients" if st["gap"] else "")
    what = ("their neighbour lists, " if neighbours else "") + what + (
        "" if neighbours else "; neighbour lists built before the clock")
    arith = "x87 extended precision" if precision == "ld" else "FP64"
    return {"value": round(k * passes / t, 2), "unit": "atoms/s", "cores": used, "kind": "oracle",
            "arithmetic": arith,
            "sample": f"{k} of {offs[-1]} centres evenly spread over the workload ({what}), "
                      + (f"{passes} passes, " if passes > 1 else "") + f"{t:.1f} s"}


def measured_ceilings(dev):
    """Measured HBM and matrix-core ceilings on this GPU: a 1 GiB device-to-device
    copy (read + write bytes), and square GEMMs through torch (hipBLASLt) in BF16
    (8192^3) and FP64 (4096^3)."""
    import torch

    out = {}
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    out["hbm_copy_GBs"] = round(2 * src.numel() * 8 * reps / (time.perf_counter() - t0) / 1e9, 1)
    del src, dst
    for name, dt, n, reps in (("bf16_gemm_TFs", torch.bfloat16, 8192, 20), ("fp64_gemm_TFs", torch.float64, 4096, 10)):
        a = torch.randn(n, n, device=dev, dtype=dt)
        b = torch.randn(n, n, device=dev, dtype=dt)
        c = a @ b
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            c = a @ b
        torch.cuda.synchronize()
        out[name] = round(2.0 * n ** 3 * reps / (time.perf_counter() - t0) / 1e12, 1)
        del a, b, c
    torch.cuda.empty_cache()
    return out


# stages that are exactly one kernel (the roofline is quoted for one kernel)
SINGLE_KERNEL = {"descriptor": "k_descriptor", "pair_adjoint": "k_pair_adjoint", "pair_prep": "k_pair_prep",
                 "pair_angular": "k_pair_prep", "gap_qbar": "k_qbar", "force_gather": "k_force_gather"}


def algorithmic_work(stage, N, P, M, K, n, l_max, nch):
    """(amount, unit) of the algorithmic work of one launch of a stage.

    Floating-point counts are the method's own arithmetic (FMA = 2 flop), not the
    instructions a kernel happens to issue; bytes are the unavoidable HBM traffic."""
    L2 = (l_max + 1) ** 2
    nab = nch * (nch + 1) // 2
    if stage in ("gap_scores", "gap_qbar"):
        return 2.0 * N * M * K, "flop"
    if stage == "gap_fused":  # both contractions in one pass
        return 4.0 * N * M * K, "flop"
    if stage == "pair_prep":
        # per pair: overlap recursion (~5 FMA per order), orthonormal transform (n^2 FMA),
        # and the derivative of both
        return P * 2.0 * (2 * (5 * (n + 3) + n * n)), "flop"
    if stage == "pair_angular":
        # per pair: ilexp (~4 FMA per order) and its derivative, azimuthal powers (4 FMA per order)
        return P * 2.0 * (8 * (l_max + 2) + 4 * (l_max + 1)), "flop"
    if stage == "descriptor":
        # c accumulation (n L^2 FMA per pair, Eq. (08)) + power spectrum (L^2 FMA per channel pair, Eq. (09))
        return 2.0 * P * n * L2 + 2.0 * N * nab * L2, "flop"
    if stage == "pair_adjoint":
        # cbar = M c per atom (n_ch^2 L^2 FMA), then per pair the U and V contractions
        # (2 n L^2 FMA) and the gradient terms (~5 FMA per slot)
        return 2.0 * N * nch * nch * L2 + 2.0 * P * (2 * n * L2 + 5 * L2), "flop"
    if stage == "force_gather":
        return P * (4 + 2 * 24) + N * 24 + (N + 1) * 4, "byte"
    if stage == "neighbors":
        return N * 24 * 2 + P * (4 * 4 + 24), "byte"
    return 0.0, "flop"


# HBM bytes per launch of the dominant kernel from FETCH_SIZE / WRITE_SIZE counter
# runs (scaled by what the counters read for a plain device copy), kept with the
# profiles; used only while the kernel's source file is unchanged since the runs
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def measured_traffic(kernel, workload, precision):
    import hashlib

    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    for t in rec.get("kernels", []):
        if t.get("kernel") != kernel or t.get("workload") != workload or t.get("precision") != precision:
            continue
        try:
            with open(os.path.join(ROOT, t["source"]), "rb") as f:
                sha = hashlib.sha256(f.read()).hexdigest()
        except OSError:
            return None
        return t["bytes_per_launch"] if sha == t.get("source_sha256") else None
    return None


def run_mode(workload, precision, steps, warmup, dev, autotune=True, sync_neighbors=False, graph=False):
    """Time `steps` whole steps of a workload in one precision mode; per-stage
    times from five profiled steps; the dominant kernel timed inside the timed
    region; optionally the same step captured once in a graph and replayed."""
    import torch

    from paper_1905_02142_amd import _lib
    from paper_1905_02142_amd.soap import NeighbourList

    log(f"{workload} {precision}: set-up")
    st = workload_setup(workload, precision, dev)
    soap, w = st["soap"], st["w"]
    N = st["n_atoms"]
    geo = (st["cells"], st["pbc"])
    nl = soap.neighbors(st["pos"], *geo, struct_offsets=st["so"])
    n_pairs = nl.n_pairs
    if not sync_neighbors:
        # a list with a 25 % reserve over the current count, as a dynamics run would keep
        nl = NeighbourList(N, n_pairs + n_pairs // 4 + 256, dev)
        soap.neighbors(st["pos"], *geo, struct_offsets=st["so"], nl=nl)
    M = w["M"]
    e = torch.empty(N, dtype=torch.float64, device=dev)
    F = torch.empty(N, 3, dtype=torch.float64, device=dev)
    ab = torch.empty(max(M, 1), dtype=torch.float64, device=dev)
    q = torch.empty(N, max(soap.dim, 1), dtype=torch.float64, device=dev)

    def step():
        if sync_neighbors:
            soap.neighbors(st["pos"], *geo, struct_offsets=st["so"], nl=nl)
        else:
            soap.neighbors_async(st["pos"], *geo, nl, struct_offsets=st["so"])
        if st["gap"]:
            soap.energy_forces(nl, st["spec"], st["qs"], st["al"], w["zeta"], out=(e, F, ab))
        else:  # a workload without a sparse set times the descriptor alone
            soap.descriptor(nl, st["spec"], out=q)

    if autotune:  # the neighbour build's cell_split, then the GAP call's launch shapes
        soap.autotune_neighbors(st["pos"], *geo, nl, struct_offsets=st["so"])
    if not autotune or not st["gap"]:
        tuning = soap.tuning
    else:
        tuning = soap.autotune(nl, st["spec"], st["qs"], st["al"], w["zeta"])

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # per-stage times from a short pass with every stage's events
    _lib.soap_profile_read(soap.ctx)
    _lib.soap_profile(soap.ctx, True)
    for _ in range(5):
        step()
    torch.cuda.synchronize()
    _lib.soap_profile(soap.ctx, False)
    stages = _lib.soap_profile_read(soap.ctx)
    per_step = {k: v[0] / 5.0 for k, v in stages.items() if v[1] and k in SINGLE_KERNEL}
    dominant = max(per_step, key=per_step.get)
    # the timed region records events around the dominant kernel only
    _lib.soap_profile_stages(soap.ctx, [dominant])
    torch.cuda.synchronize()
    log(f"{workload} {precision}: timing {steps} steps")
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if not sync_neighbors:  # the last build's count and error bits (raises on overflow or bad input)
        assert soap.check_neighbors(nl) == n_pairs
        nl.n_pairs = _lib.SOAP_PAIRS_DEFERRED
    _lib.soap_profile(soap.ctx, False)
    timed = _lib.soap_profile_read(soap.ctx)[dominant]
    res = dict(st=st, soap=soap, w=w, N=N, n_pairs=n_pairs, M=M, stages=stages, tuning=tuning, dominant=dominant,
               dominant_ms=timed[0] / timed[1], ms=(t1 - t0) * 1e3 / steps, value=N * steps / (t1 - t0),
               e=e.cpu().numpy(), F=F.cpu().numpy(), ab=ab.cpu().numpy(), graph=None)
    if graph and not sync_neighbors:
        # the whole step (neighbour build with the count left on the device, descriptor,
        # GAP, adjoint, forces) captured once and replayed
        g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            step()
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        assert soap.check_neighbors(nl) == n_pairs
        res["graph"] = {"ms_per_step": round((t1 - t0) * 1e3 / steps, 4), "value": round(N * steps / (t1 - t0), 1)}
        del g
    return res


def rate_fn(run, prec_key, P):
    """rate(stage, avg_ms) -> (bound, peak, unit, achieved) for one launch of a stage of this run."""
    w = run["w"]
    n, l_max, nch = w["n_max"], w["l_max"], w["n_max"] * w["n_species"]
    gemm_peak = {"fp64": PEAK["fp64_TFs"], "f32": PEAK["fp32_TFs"], "bf16": PEAK["bf16_TFs"],
                 "bf16x3": PEAK["bf16_TFs"], "bf16ps": PEAK["bf16_TFs"]}[prec_key]

    def rate(name, avg_ms):
        work, unit = algorithmic_work(name, run["N"], P, run["M"], w["K"], n, l_max, nch)
        if unit == "flop":
            bound, peak, u = ("mfma", gemm_peak, "TFLOP/s") if name.startswith("gap") else ("alu", PEAK["fp64_TFs"],
                                                                                           "TFLOP/s")
            achieved = work / (avg_ms * 1e-3) / 1e12
        else:
            bound, peak, u = "hbm", PEAK["hbm_GBs"], "GB/s"
            achieved = work / (avg_ms * 1e-3) / 1e9
        return bound, peak, u, achieved

    return rate


def summarise(run, prec_key):
    """Per-stage rooflines (from the profiled pass) and the dominant kernel's (timed region)."""
    P = run["n_pairs"]
    rate = rate_fn(run, prec_key, P)
    per_stage = {}
    for name, (tot, cnt) in run["stages"].items():
        if cnt == 0:
            continue
        avg_ms = tot / cnt
        bound, peak, u, achieved = rate(name, avg_ms)
        per_stage[name] = dict(avg_ms=avg_ms, launches_per_step=cnt / 5.0, share=tot / 5.0 / run["ms"], bound=bound,
                               achieved=achieved, peak=peak, unit=u, frac=achieved / peak)
    dom = run["dominant"]
    bound, peak, u, achieved = rate(dom, run["dominant_ms"])
    roof = {"kernel": SINGLE_KERNEL[dom], "bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": u,
            "frac": round(achieved / peak, 4), "avg_launch_ms": round(run["dominant_ms"], 5)}
    return per_stage, roof


def compare(mixed, ref):
    import numpy as np

    dF = mixed["F"] - ref["F"]
    rmse = float(np.sqrt(np.mean(dF ** 2)))
    rms = float(np.sqrt(np.mean(ref["F"] ** 2)))
    return {"value": round(ref["value"], 1), "ms_per_step": round(ref["ms"], 4),
            "speedup_of_mixed": round(mixed["value"] / ref["value"], 3),
            "force_rmse_eV_per_A": rmse, "force_rmse_rel_to_rms_force": rmse / rms,
            "force_rmse_within_bar": rmse <= RMSE_BAR,
            "energy_max_abs_err": float(np.abs(mixed["e"] - ref["e"]).max()), "rms_force_eV_per_A": rms}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="box262144_n10l10")
    ap.add_argument("--precision", default="auto", choices=["auto", "fp64", "f32", "bf16", "bf16x3", "bf16ps"],
                    help="GAP contraction precision (the rest of the path is FP64, except the power spectrum and "
                         "its adjoint in bf16ps); auto: the workload's mixed mode (the lowest precision within "
                         "the 1e-4 eV/A force RMSE bar there).  The FP64 path is timed alongside any other mode "
                         "and the force error against it reported")
    ap.add_argument("--also", default="box4096_n8l8",
                    help="comma-separated extra workloads timed the same way (mixed mode and FP64 path), "
                         "reported under 'workloads'; 'none' for none")
    ap.add_argument("--graph", action="store_true",
                    help="also time the whole step captured once in a HIP graph and replayed (always done for "
                         "batched workloads)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0, help="seconds per oracle leg")
    ap.add_argument("--no-ceilings", action="store_true", help="skip the measured copy / GEMM ceilings")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--sync-neighbors", action="store_true",
                    help="read the pair count back to the host in every step (soap_build_neighbors) instead of "
                         "leaving it on the device (soap_build_neighbors_async, checked after the timed region)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, run a plain 512 MiB device-to-device copy three times "
                         "(the reference kernel for scaling FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              f"the multi-GPU decomposition is not run here", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth

    dev = torch.device("cuda:0")

    def mode_of(name):
        w = synth.WORKLOADS[name]
        if args.precision != "auto":
            return args.precision
        return w.get("mixed", "fp64") if w["M"] else "fp64"

    def measure(name, steps, warmup, graph):
        mode = mode_of(name)
        main_run = run_mode(name, mode, steps, warmup, dev, not args.no_autotune, args.sync_neighbors, graph)
        ref = None
        if mode != "fp64" and main_run["st"]["gap"]:
            ref = run_mode(name, "fp64", steps, warmup, dev, not args.no_autotune, args.sync_neighbors, graph)
        return mode, main_run, ref

    graph_main = args.graph or args.workload.startswith("batch")
    mode, main_run, ref = measure(args.workload, args.steps, args.warmup, graph_main)
    st, w, N = main_run["st"], main_run["w"], main_run["N"]
    per_stage, roofline = summarise(main_run, mode)
    roofline["traffic"] = measured_traffic(roofline["kernel"], args.workload, mode)
    fp64_path = None
    if ref is not None:
        fp64_path = compare(main_run, ref)
        _, rref = summarise(ref, "fp64")
        fp64_path["roofline"] = rref
        if ref["graph"]:
            fp64_path["graph_replay"] = ref["graph"]
    # release the main workload's device buffers before the extra workloads
    main_soap = main_run.pop("soap")
    main_run["st"].pop("soap")
    del main_soap
    if ref is not None:
        ref.pop("soap")
        ref["st"].pop("soap")
    torch.cuda.empty_cache()

    extra = {}
    for name in [x for x in args.also.split(",") if x and x != "none" and x != args.workload]:
        m2, r2, f2 = measure(name, args.steps, args.warmup, args.graph or name.startswith("batch"))
        _, roof2 = summarise(r2, m2)
        roof2["traffic"] = measured_traffic(roof2["kernel"], name, m2)
        extra[name] = {"precision": m2, "value": round(r2["value"], 1), "ms_per_step": round(r2["ms"], 4),
                       "n_atoms": r2["N"], "n_pairs": r2["n_pairs"], "roofline": roof2,
                       "fp64_path": compare(r2, f2) if f2 is not None else None}
        if r2["graph"]:
            extra[name]["graph_replay"] = r2["graph"]
        r2.pop("soap")
        r2["st"].pop("soap")
        if f2 is not None:
            f2.pop("soap")
            f2["st"].pop("soap")
        torch.cuda.empty_cache()

    ceilings = None if args.no_ceilings else measured_ceilings(dev)
    if ceilings:
        roofline["measured_peak"] = {"hbm": ceilings["hbm_copy_GBs"],
                                     "mfma": ceilings["fp64_gemm_TFs" if mode == "fp64" else "bf16_gemm_TFs"]}.get(
            roofline["bound"])

    if args.calibrate_copy:  # the reference copy for the HBM byte counters, after everything else
        src = torch.ones(1 << 26, dtype=torch.float64, device=dev)  # 512 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        b = args.cpu_budget
        cpu = cpu_oracle_rate(st, b)
        cpu["legs"] = {
            "fp64_build": cpu_oracle_rate(st, b, precision="f64"),
            "one_core": cpu_oracle_rate(st, b, threads=1),
            "without_neighbour_build": cpu_oracle_rate(st, b, neighbours=False),
        }

    out = {
        "metric": "atomic environments/s (descriptor+forces+GAP kernel)",
        "value": round(main_run["value"], 1),
        "unit": "atoms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if mode == "fp64" else f"f64 (GAP contraction {mode})",
        "data": "synthetic",
        "config": {"workload": args.workload, "structures": len(st["structures"]), "n_atoms": N,
                   "n_pairs": main_run["n_pairs"],
                   "path": "descriptor, GAP energies and forces" if st["gap"] else "descriptor only (no sparse set)",
                   "r_cut": w["r_cut"], "n_max": w["n_max"], "l_max": w["l_max"], "n_species": w["n_species"],
                   "M": main_run["M"], "zeta": w["zeta"], "K": w["K"], "precision": mode,
                   "tuning": main_run["tuning"],
                   "neighbour_build": "sync" if args.sync_neighbors else "async, count checked after the timed steps"},
        "roofline": roofline,
        "fp64_path": fp64_path,
        "graph_replay": main_run["graph"],
        "stages": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                   for k, v in per_stage.items()},
        "workloads": extra,
        "measured_ceilings": ceilings,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
