#!/usr/bin/env python
"""Throughput of the separable-SOAP + GAP energy/forces hot path on one MI355X.

A step is one pass of the whole path over one structure already resident in
HBM: neighbour list, descriptor (c_nlm, power spectrum, q), GAP energies,
the adjoint chain and the forces.  Default workload: 4096 atoms in a periodic
34.5 A cube (0.1 atoms/A^3, minimum distance 1.2 A), r_cut 5 A, sigma 0.5 A,
n_max = l_max = 8, zeta = 4 against 2000 random unit sparse descriptors with
N(0,1) weights.  Prints one JSON line.
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


def workload_setup(name, precision, dev):
    import numpy as np
    import torch

    import synth
    from paper_1905_02142_amd import Soap, SoapParams

    w = synth.workload(name)
    if len(w["structures"]) != 1:
        raise SystemExit("bench.py times single-structure workloads")
    s = w["structures"][0]
    kw = dict(n_max=w["n_max"], l_max=w["l_max"], r_cut=w["r_cut"], sigma0_r=w["sigma"], sigma0_perp=w["sigma"],
              n_species=w["n_species"])
    soap = Soap(SoapParams(precision=precision, **kw))
    t = lambda a, dt=None: torch.tensor(np.ascontiguousarray(a), device=dev, dtype=dt)
    st = dict(w=w, s=s, kw=kw, soap=soap, pos=t(s.positions), spec=t(w["species"], torch.int32),
              qs=t(w["q_sparse"]), al=t(w["alpha"]))
    return st


# stages that are exactly one kernel (the roofline is quoted for one kernel)
SINGLE_KERNEL = {"descriptor": "k_descriptor", "pair_adjoint": "k_pair_adjoint", "pair_prep": "k_pair_prep",
                 "gap_qbar": "k_qbar", "force_gather": "k_force_gather"}


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
        # derivative of both, ilexp (~4 FMA per order) and its derivative, azimuthal powers
        return P * 2.0 * (2 * (5 * (n + 3) + n * n) + 8 * (l_max + 2) + 4 * (l_max + 1)), "flop"
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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="box4096_n8l8")
    ap.add_argument("--precision", default="bf16", choices=["fp64", "f32", "bf16", "bf16x3"],
                    help="GAP contraction precision (the rest of the path is FP64); the FP64 path is timed "
                         "alongside any other mode and the force error against it reported")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
              f"the multi-GPU decomposition is described in DESIGN.md and not run here", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1905_02142_amd import _lib
    from paper_1905_02142_amd.soap import NeighbourList

    dev = torch.device("cuda:0")

    def run_mode(precision, steps, warmup):
        st = workload_setup(args.workload, precision, dev)
        soap, w, s = st["soap"], st["w"], st["s"]
        N = s.n_atoms
        nl = soap.neighbors(st["pos"], s.cell, s.pbc)
        n_pairs = nl.n_pairs
        if not args.sync_neighbors:
            # a list with a 25 % reserve over the current count, as a dynamics run would keep
            nl = NeighbourList(N, n_pairs + n_pairs // 4 + 256, dev)
            soap.neighbors(st["pos"], s.cell, s.pbc, nl=nl)
        M = w["M"]
        e = torch.empty(N, dtype=torch.float64, device=dev)
        F = torch.empty(N, 3, dtype=torch.float64, device=dev)
        ab = torch.empty(M, dtype=torch.float64, device=dev)

        def step():
            if args.sync_neighbors:
                soap.neighbors(st["pos"], s.cell, s.pbc, nl=nl)
            else:
                soap.neighbors_async(st["pos"], s.cell, s.pbc, nl)
            soap.energy_forces(nl, st["spec"], st["qs"], st["al"], w["zeta"], out=(e, F, ab))

        tuning = soap.tuning if args.no_autotune else soap.autotune(nl, st["spec"], st["qs"], st["al"], w["zeta"])

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
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if not args.sync_neighbors:  # the last build's count and error bits (raises on overflow or bad input)
            assert soap.check_neighbors(nl) == n_pairs
        _lib.soap_profile(soap.ctx, False)
        timed = _lib.soap_profile_read(soap.ctx)[dominant]
        res = dict(st=st, soap=soap, w=w, s=s, N=N, nl=nl, M=M, stages=stages, tuning=tuning, dominant=dominant,
                   dominant_ms=timed[0] / timed[1],
                   ms=(t1 - t0) * 1e3 / steps, value=N * steps / (t1 - t0),
                   e=e.cpu().numpy(), F=F.cpu().numpy(), ab=ab.cpu().numpy())
        return res

    main_run = run_mode(args.precision, args.steps, args.warmup)
    st, soap, w, s, N, nl, M = (main_run[k] for k in ("st", "soap", "w", "s", "N", "nl", "M"))
    stages, ms, value = main_run["stages"], main_run["ms"], main_run["value"]
    fp64_path = None
    if args.precision != "fp64":
        ref = run_mode("fp64", args.steps, args.warmup)
        dF = main_run["F"] - ref["F"]
        fp64_path = {"value": round(ref["value"], 1), "ms_per_step": round(ref["ms"], 4),
                     "speedup_of_mixed": round(value / ref["value"], 3),
                     "force_rmse_eV_per_A": float(np.sqrt(np.mean(dF ** 2))),
                     "force_rmse_rel_to_rms_force": float(np.sqrt(np.mean(dF ** 2)) / np.sqrt(np.mean(ref["F"] ** 2))),
                     "energy_max_abs_err": float(np.abs(main_run["e"] - ref["e"]).max()),
                     "rms_force_eV_per_A": float(np.sqrt(np.mean(ref["F"] ** 2)))}

    # roofline of every stage (from the per-stage pass); the dominant kernel's, timed inside the
    # timed region, goes in "roofline"
    P, K = nl.n_pairs, soap.dim
    n, l_max, nch = w["n_max"], w["l_max"], w["n_max"] * w["n_species"]
    gemm_peak = {"fp64": PEAK["fp64_TFs"], "f32": PEAK["fp32_TFs"], "bf16": PEAK["bf16_TFs"],
                 "bf16x3": PEAK["bf16_TFs"]}[args.precision]

    def rate(name, avg_ms):
        work, unit = algorithmic_work(name, N, P, M, K, n, l_max, nch)
        if unit == "flop":
            bound, peak, u = ("mfma", gemm_peak, "TFLOP/s") if name.startswith("gap") else ("alu", PEAK["fp64_TFs"],
                                                                                           "TFLOP/s")
            achieved = work / (avg_ms * 1e-3) / 1e12
        else:
            bound, peak, u = "hbm", PEAK["hbm_GBs"], "GB/s"
            achieved = work / (avg_ms * 1e-3) / 1e9
        return bound, peak, u, achieved

    per_stage = {}
    for name, (tot, cnt) in stages.items():
        if cnt == 0:
            continue
        avg_ms = tot / cnt
        bound, peak, u, achieved = rate(name, avg_ms)
        per_stage[name] = dict(avg_ms=avg_ms, launches_per_step=cnt / 5.0, share=tot / 5.0 / ms, bound=bound,
                               achieved=achieved, peak=peak, unit=u, frac=achieved / peak)
    dom = main_run["dominant"]
    bound, peak, u, achieved = rate(dom, main_run["dominant_ms"])
    roofline = {"kernel": SINGLE_KERNEL[dom], "bound": bound, "achieved": round(achieved, 3), "peak": peak,
                "unit": u, "frac": round(achieved / peak, 4),
                "traffic": measured_traffic(SINGLE_KERNEL[dom], args.workload, args.precision),
                "avg_launch_ms": round(main_run["dominant_ms"], 5)}

    if args.calibrate_copy:  # the reference copy for the HBM byte counters, after everything else
        src = torch.ones(1 << 26, dtype=torch.float64, device=dev)  # 512 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        okw = dict(st["kw"])
        p = oracle.Params(**okw)
        t2 = time.perf_counter()
        oracle.energy_forces(p, s.positions, s.cell, s.pbc, w["species"], w["q_sparse"], w["alpha"], w["zeta"])
        t3 = time.perf_counter()
        cpu = {"value": round(N / (t3 - t2), 2), "unit": "atoms/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"the full workload once ({N} atoms: brute-force neighbour list, descriptor, GAP "
                         f"energies and forces), {t3 - t2:.1f} s"}

    out = {
        "metric": "atomic environments/s (descriptor+forces+GAP kernel)",
        "value": round(value, 1),
        "unit": "atoms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else f"f64 (GAP contraction {args.precision})",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_atoms": N, "n_pairs": P, "r_cut": w["r_cut"], "n_max": n,
                   "l_max": w["l_max"], "n_species": w["n_species"], "M": M, "zeta": w["zeta"], "K": K,
                   "precision": args.precision, "tuning": main_run["tuning"],
                   "neighbour_build": "sync" if args.sync_neighbors else "async, count checked after the timed steps"},
        "roofline": roofline,
        "fp64_path": fp64_path,
        "stages": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                   for k, v in per_stage.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
