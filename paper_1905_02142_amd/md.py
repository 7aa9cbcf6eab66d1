"""Molecular dynamics driven by the GAP forces of this library.

Velocity Verlet in eV, A, amu and fs.  The neighbour list is built with a Verlet
skin (soap_set_neighbor_skin): pairs out to r_cut + skin are listed and those
beyond r_cut weigh exactly zero, so one list serves every step until some atom
may have moved more than skin / 2 since the build; each step only refreshes the
pair vectors from the new positions (soap_update_pair_vectors).  Only then is the
list rebuilt, into the same buffers, with the pair count left on the device.  One timestep
(half kick, drift, forces, half kick) is captured once in a graph and replayed,
so a step issues no host-side launches.  The array operations of the
integrator are plain torch element-wise work; all of the force evaluation runs in
the library's kernels.
"""
from __future__ import annotations

import torch

from . import _lib
from .soap import NeighbourList, Soap

# (eV / A) / amu -> A / fs^2
ACC = 9.648533212e-3


class GapMD:
    """NVE dynamics of one periodic structure.

    positions: (N, 3) float64 on the device; masses: (N,) amu; species: (N,)
    int32; q_sparse, alpha, zeta: the GAP model; dt: fs; skin: A.
    """

    def __init__(self, soap: Soap, positions, masses, cell, pbc, species, q_sparse, alpha, zeta: int,
                 dt: float = 0.5, skin: float = 0.4, velocities=None, reserve: float = 0.3):
        self.soap, self.cell, self.pbc = soap, cell, pbc
        self.dt, self.skin = float(dt), float(skin)
        dev = positions.device
        self.pos = positions.to(torch.float64).contiguous().clone()
        n = self.pos.shape[0]
        self.vel = (torch.zeros_like(self.pos) if velocities is None
                    else velocities.to(torch.float64).contiguous().clone())
        self.inv_m = (ACC / masses.to(torch.float64)).reshape(n, 1).contiguous()
        self.mass = masses.to(torch.float64).reshape(n, 1).contiguous()
        self.spec = species.to(torch.int32).contiguous()
        self.qs = q_sparse.to(torch.float64).contiguous()
        self.al = alpha.to(torch.float64).contiguous()
        self.zeta = int(zeta)
        soap.set_neighbor_skin(self.skin)
        first = soap.neighbors(self.pos, cell, pbc)
        self.nl = NeighbourList(n, int(first.n_pairs * (1.0 + reserve)) + 256, dev)
        self.pos_at_build = torch.empty_like(self.pos)
        self.rebuilds = -1
        self._rebuild()
        self.e = torch.empty(n, dtype=torch.float64, device=dev)
        self.F = torch.empty(n, 3, dtype=torch.float64, device=dev)
        self.ab = torch.empty(self.qs.shape[0], dtype=torch.float64, device=dev)
        self._forces()  # forces of the initial positions; also sizes the workspace
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step_ops()
        self.steps = 0

    def _forces(self):
        self.soap.energy_forces(self.nl, self.spec, self.qs, self.al, self.zeta, out=(self.e, self.F, self.ab))

    def _step_ops(self):
        h = 0.5 * self.dt
        self.vel.add_(self.F * self.inv_m, alpha=h)
        self.pos.add_(self.vel, alpha=self.dt)
        self.soap.update_pair_vectors(self.nl, self.pos)
        self._forces()
        self.vel.add_(self.F * self.inv_m, alpha=h)

    def _rebuild(self):
        self.soap.neighbors_async(self.pos, self.cell, self.pbc, self.nl)
        self.pairs = self.soap.check_neighbors(self.nl)  # raises if the reserve was too small
        # the captured step reads the pair count on the device, so it stays valid
        # for every rebuilt list
        self.nl.n_pairs = _lib.SOAP_PAIRS_DEFERRED
        self.pos_at_build.copy_(self.pos)
        self.rebuilds += 1

    def step(self, n: int = 1) -> None:
        """n timesteps; before each, the list is rebuilt if the coming drift could
        take some atom further than skin / 2 from its position at the last build."""
        for _ in range(n):
            disp = (self.pos - self.pos_at_build).norm(dim=1).max()
            # a bound on the coming drift: |v + dt F / 2m| dt
            drift = (self.vel + (0.5 * self.dt) * self.F * self.inv_m).norm(dim=1).max() * self.dt
            if (disp + drift).item() > 0.5 * self.skin:
                self._rebuild()
                if drift.item() > 0.5 * self.skin:
                    raise ValueError("one step moves atoms further than skin / 2: raise the skin or lower dt")
            self.graph.replay()
            self.steps += 1

    def energies(self):
        """(potential, kinetic) in eV at the current step."""
        kin = 0.5 * (self.mass * self.vel * self.vel).sum() / ACC
        return float(self.e.sum().item()), float(kin.item())
