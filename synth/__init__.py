"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmark.

This module holds no arithmetic of the descriptor or of the GAP model: it only
places atoms, draws species labels, sparse descriptor rows and weights.  Every
generator takes an explicit seed and uses numpy's PCG64 ``default_rng``, so the
same call returns the same arrays on every machine.

Structures stand in for the paper's speed-test system (Sec. "Speed"): atoms
placed uniformly at random in a periodic cube with a minimum pair distance
(random sequential addition), at a density near 0.1 atoms per cubic Angstrom.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Structure",
    "rsa_box",
    "rsa_two_density_box",
    "draw_species",
    "sparse_set",
    "sparse_weights",
    "batch_of_structures",
    "workload",
    "WORKLOADS",
]


@dataclass
class Structure:
    """One periodic structure: positions (N, 3) in Angstrom and cell rows (3, 3)."""

    positions: np.ndarray
    cell: np.ndarray
    pbc: np.ndarray

    @property
    def n_atoms(self) -> int:
        return int(self.positions.shape[0])


class _Grid:
    """Cell grid over a periodic cube, cell side >= d_min, fixed slots per cell."""

    def __init__(self, box, d_min):
        self.n = max(1, int(math.floor(box / d_min)))
        self.size = box / self.n
        self.cap = 8
        self.slots = np.full((self.n, self.n, self.n, self.cap), -1, dtype=np.int64)
        self.count = np.zeros((self.n, self.n, self.n), dtype=np.int64)
        off = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)])
        self.off = off if self.n >= 3 else np.unique(off % self.n, axis=0)

    def cell_of(self, x):
        return np.floor(x / self.size).astype(np.int64) % self.n

    def neighbours(self, cells):
        """Indices of accepted atoms in the 27 cells around each row of ``cells`` (B, 3)."""
        c = (cells[:, None, :] + self.off[None, :, :]) % self.n
        return self.slots[c[..., 0], c[..., 1], c[..., 2]].reshape(len(cells), -1)

    def add(self, cell, idx):
        a, b, c = cell
        k = self.count[a, b, c]
        if k == self.cap:
            grow = np.full(self.slots.shape[:3] + (self.cap,), -1, dtype=np.int64)
            self.slots = np.concatenate([self.slots, grow], axis=3)
            self.cap *= 2
        self.slots[a, b, c, k] = idx
        self.count[a, b, c] = k + 1


def _rsa_fill(rng, n_target, lo, hi, box, d_min, grid, pos, n_have, max_tries):
    """Random sequential addition into the slab lo <= z < hi of a periodic cube.

    Candidates are drawn in blocks; each is accepted iff its minimum-image
    distance to every atom accepted before it (earlier blocks and earlier
    candidates of its own block) is >= d_min, which is the sequential rule.
    """
    d2 = d_min * d_min
    tries = 0
    block = 2048
    n_end = n_have + n_target
    while n_have < n_end:
        if tries > max_tries:
            raise RuntimeError(f"random sequential addition stalled after {tries} candidates")
        cand = rng.random((block, 3))
        cand[:, :2] *= box
        cand[:, 2] = lo + cand[:, 2] * (hi - lo)
        cells = grid.cell_of(cand)
        nb = grid.neighbours(cells)
        d = pos[np.maximum(nb, 0)] - cand[:, None, :]
        d -= box * np.round(d / box)
        r2 = np.einsum("bkc,bkc->bk", d, d)
        r2[nb < 0] = np.inf
        ok = r2.min(axis=1) >= d2 if r2.shape[1] else np.ones(block, bool)
        new_pos = []
        for bi in np.nonzero(ok)[0]:
            c = cand[bi]
            if new_pos:
                e = np.asarray(new_pos) - c
                e -= box * np.round(e / box)
                if np.min(np.einsum("ij,ij->i", e, e)) < d2:
                    continue
            pos[n_have] = c
            grid.add(cells[bi], n_have)
            new_pos.append(c)
            n_have += 1
            if n_have == n_end:
                tries += int(bi) + 1
                break
        else:
            tries += block
    return n_have


def rsa_box(n_atoms: int, box: float, d_min: float, seed: int) -> Structure:
    """``n_atoms`` uniform random atoms in a periodic cube of side ``box`` with
    all minimum-image pair distances >= ``d_min`` (random sequential addition)."""
    rng = np.random.default_rng(seed)
    grid = _Grid(box, d_min)
    pos = np.zeros((n_atoms, 3))
    _rsa_fill(rng, n_atoms, 0.0, box, box, d_min, grid, pos, 0, 1000 * n_atoms + 10000)
    return Structure(pos, np.eye(3) * box, np.ones(3, dtype=np.int32))


def rsa_two_density_box(n_dense: int, n_sparse: int, box: float, d_min: float, seed: int) -> Structure:
    """Cube of side ``box``: ``n_dense`` atoms in z < box/2 and ``n_sparse`` atoms
    in z >= box/2, minimum distance enforced across the interface and the
    periodic boundaries (uneven neighbour counts)."""
    rng = np.random.default_rng(seed)
    grid = _Grid(box, d_min)
    pos = np.zeros((n_dense + n_sparse, 3))
    k = _rsa_fill(rng, n_dense, 0.0, 0.5 * box, box, d_min, grid, pos, 0, 1000 * n_dense + 10000)
    _rsa_fill(rng, n_sparse, 0.5 * box, box, box, d_min, grid, pos, k, 1000 * n_sparse + 10000)
    return Structure(pos, np.eye(3) * box, np.ones(3, dtype=np.int32))


def draw_species(n_atoms: int, probs, seed: int) -> np.ndarray:
    """i.i.d. species labels 0..len(probs)-1 with the given probabilities (int32)."""
    rng = np.random.default_rng(seed)
    p = np.asarray(probs, dtype=np.float64)
    return rng.choice(len(p), size=n_atoms, p=p / p.sum()).astype(np.int32)


def sparse_set(m: int, k: int, seed: int) -> np.ndarray:
    """``m`` sparse descriptor rows of length ``k``: N(0,1) entries, each row scaled to unit norm."""
    rng = np.random.default_rng(seed)
    q = rng.standard_normal((m, k))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def sparse_weights(m: int, seed: int) -> np.ndarray:
    """``m`` GAP weights alpha_s ~ N(0,1)."""
    return np.random.default_rng(seed).standard_normal(m)


def batch_of_structures(n_struct: int, n_lo: int, n_hi: int, rho_lo: float, rho_hi: float,
                        d_min: float, seed: int) -> list[Structure]:
    """Independent periodic cubes: atom counts log-uniform in [n_lo, n_hi],
    densities uniform in [rho_lo, rho_hi] atoms per cubic Angstrom."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n_struct):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        rho = rng.uniform(rho_lo, rho_hi)
        box = (n / rho) ** (1.0 / 3.0)
        out.append(rsa_box(n, box, d_min, seed * 1000 + b))
    return out


# Named workloads: descriptor hyper-parameters and system recipe.  Values in
# Angstrom.  ``sigma`` is sigma_0r = sigma_0perp; alpha_r = alpha_perp = a = 0.
# ``mixed`` names the mixed-precision mode run on a workload with a sparse set:
# the lowest-precision one whose force RMSE against the fp64 path stays within
# 1e-4 eV/A there (the 256-cell batch, at zeta = 2, needs split BF16; the
# three-species slab, 24 channels, also takes its power spectrum on the matrix
# cores, where that is faster than the FP64 one).
WORKLOADS = {
    "box64_n6l6": dict(n_atoms=64, box=8.6, d_min=1.2, r_cut=3.7, sigma=0.5, n_max=6, l_max=6,
                       n_species=1, M=0, zeta=0, seed=1001),
    "box4096_n8l8": dict(n_atoms=4096, box=34.5, d_min=1.2, r_cut=5.0, sigma=0.5, n_max=8, l_max=8,
                         n_species=1, M=2000, zeta=4, seed=1002, mixed="bf16"),
    "slab32768_3sp_n8l8": dict(n_atoms=32768, box=(32768 / 0.06) ** (1.0 / 3.0), d_min=1.2, r_cut=5.0,
                               sigma=0.5, n_max=8, l_max=8, n_species=3, M=2000, zeta=4, seed=1003, mixed="bf16ps",
                               species_probs=(0.5, 0.3, 0.2)),
    "batch256_n8l6": dict(n_struct=256, n_lo=16, n_hi=2048, rho_lo=0.05, rho_hi=0.12, d_min=1.2,
                          r_cut=4.5, sigma=0.5, n_max=8, l_max=6, n_species=1, M=1000, zeta=2,
                          seed=5004, mixed="bf16x3"),
    "box262144_n10l10": dict(n_atoms=262144, box=138.0, d_min=1.2, r_cut=5.5, sigma=0.5, n_max=10,
                             l_max=10, n_species=1, M=4000, zeta=4, seed=1005, mixed="bf16"),
    # the paper's speed-test structure (Sec. III.D): 10000 random atoms in a 46.371 A
    # cube, no two closer than 0.7 A; descriptor only.  r_cut and sigma are not given
    # there: 5 A and 0.5 A as in the 4096-atom workload; n_max, l_max are swept 3..12
    "speed10000_n10l10": dict(n_atoms=10000, box=46.371, d_min=0.7, r_cut=5.0, sigma=0.5, n_max=10,
                              l_max=10, n_species=1, M=0, zeta=0, seed=1006),
}


def workload(name: str):
    """Build the structure(s), species, sparse set and weights of a named workload.

    Returns a dict with ``structures`` (list), ``species`` (concatenated int32),
    ``q_sparse`` (M, K) or None, ``alpha`` (M,) or None, and the hyper-parameters.
    ``K`` depends on the descriptor size: K = n_ch (n_ch + 1) / 2 * (l_max + 1)
    with n_ch = n_species * n_max.
    """
    w = dict(WORKLOADS[name])
    if name.startswith("batch"):
        structs = batch_of_structures(w["n_struct"], w["n_lo"], w["n_hi"], w["rho_lo"], w["rho_hi"],
                                      w["d_min"], w["seed"])
    elif name.startswith("slab"):
        n = w["n_atoms"]
        box = w["box"]
        # half the volume at 0.1, half at 0.02 atoms / A^3 -> 5:1 split of the atoms
        n_dense = int(round(n * 5.0 / 6.0))
        structs = [rsa_two_density_box(n_dense, n - n_dense, box, w["d_min"], w["seed"])]
    else:
        structs = [rsa_box(w["n_atoms"], w["box"], w["d_min"], w["seed"])]
    n_total = sum(s.n_atoms for s in structs)
    c = int(str(w["seed"])[-1])
    if w["n_species"] > 1:
        species = draw_species(n_total, w["species_probs"], 4000 + c)
    else:
        species = np.zeros(n_total, dtype=np.int32)
    n_ch = w["n_species"] * w["n_max"]
    K = n_ch * (n_ch + 1) // 2 * (w["l_max"] + 1)
    qs = alpha = None
    if w["M"]:
        qs = sparse_set(w["M"], K, 2000 + c)
        alpha = sparse_weights(w["M"], 3000 + c)
    w.update(structures=structs, species=species, q_sparse=qs, alpha=alpha, K=K)
    return w
