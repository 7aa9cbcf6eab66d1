"""Descriptor timing over a grid of basis sizes on the speed-test structure of
Sec. III.D: 10000 random atoms in a periodic 46.371 A cube, no two closer than
0.7 A (r_cut 5 A and sigma 0.5 A, which that section does not give).

As in that test the neighbour list is excluded: it is built once (it depends on
r_cut only) and every timed call is one soap_descriptor, i.e. the expansion
coefficients and the descriptor vectors of all 10000 atoms in FP64.  The time is
also split with the library's stage events into the three parts the paper's
timing figure uses (Sec. III.D):
  radial   (pair_prep):    per-pair radial basis values b_n (Sec. III.A),
  angular  (pair_angular): per-pair ilexp and azimuthal factors (Sec. III.C),
  vector   (descriptor):   the real harmonics' polynomial part, the c_nlm
                           reduction over neighbours, the power spectrum and the
                           normalisation (the harmonics cannot be timed apart
                           from the reduction they feed).
The kernels are compiled for basis buckets (n_max, l_max) = (6, 6), (8, 6),
(8, 8), (10, 10), (12, 12); a smaller basis runs with the sizes of the smallest
bucket that holds it (the padding channels and records are zeros), so the times
are flat inside a bucket.

    python -m paper_1905_02142_amd.speedtest [--n 3 12] [--l 3 12] [--reps 20]

prints one JSON line per (n_max, l_max).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

WORKLOAD = "speed10000_n10l10"


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, nargs=2, default=(3, 12), metavar=("LO", "HI"), help="n_max range")
    ap.add_argument("--l", type=int, nargs=2, default=(3, 12), metavar=("LO", "HI"), help="l_max range")
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args(argv)

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch

    import synth

    from . import _lib
    from .soap import Soap, SoapParams

    dev = torch.device("cuda:0")
    w = synth.workload(WORKLOAD)
    s = w["structures"][0]
    N = s.n_atoms
    pos = torch.tensor(s.positions, device=dev)
    spec = torch.zeros(N, dtype=torch.int32, device=dev)
    nl = None
    for n in range(args.n[0], args.n[1] + 1):
        for l in range(args.l[0], args.l[1] + 1):
            soap = Soap(SoapParams(n_max=n, l_max=l, r_cut=w["r_cut"], sigma0_r=w["sigma"], sigma0_perp=w["sigma"]))
            if nl is None:
                nl = soap.neighbors(pos, s.cell, s.pbc)
            for _ in range(3):
                soap.descriptor(nl, spec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.reps):
                soap.descriptor(nl, spec)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / args.reps
            # the split, from a second pass with stage events
            _lib.soap_profile_read(soap.ctx)
            _lib.soap_profile(soap.ctx, True)
            for _ in range(args.reps):
                soap.descriptor(nl, spec)
            torch.cuda.synchronize()
            _lib.soap_profile(soap.ctx, False)
            st = _lib.soap_profile_read(soap.ctx)
            split = {k: round(v[0] / v[1], 5) for k, v in st.items() if v[1]}
            parts = {"radial": split.get("pair_prep", 0.0), "angular": split.get("pair_angular", 0.0),
                     "vector": split.get("descriptor", 0.0)}
            print(json.dumps({"workload": WORKLOAD, "n_max": n, "l_max": l, "K": soap.dim, "n_atoms": N,
                              "n_pairs": nl.n_pairs, "ms_per_call": round(ms, 5),
                              "atoms_per_s": round(N / (ms * 1e-3), 1), "stage_ms": split,
                              "paper_split_ms": parts}), flush=True)
            soap.close()


if __name__ == "__main__":
    main()
