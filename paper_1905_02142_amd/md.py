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

The host does not wait for the device every step.  Steps run in chunks of
``check_every`` replays; inside the graph each step marks, on the device, every
atom that is further than skin / 2 from its position at the last build (the one
condition under which the list may miss a pair inside r_cut).  After a chunk the
host reads the marks once: if none is set, every step of the chunk used a valid
list; if one is, the chunk is undone from a copy of the state taken before it and
run again one step at a time, rebuilding the list before any step whose drift
could reach the limit.  Between chunks the list is also rebuilt ahead of time
when the coming chunk would probably reach the limit, so that repeats are rare.
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
                 dt: float = 0.5, skin: float = 0.4, velocities=None, reserve: float = 0.3, check_every: int = 10):
        self.soap, self.cell, self.pbc = soap, cell, pbc
        self.dt, self.skin = float(dt), float(skin)
        self.check_every = max(1, int(check_every))
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
        self.moved = torch.zeros(n, dtype=torch.bool, device=dev)  # atoms beyond skin / 2 since the build
        self.rebuilds = -1
        self._rebuild()
        self.e = torch.empty(n, dtype=torch.float64, device=dev)
        self.F = torch.empty(n, 3, dtype=torch.float64, device=dev)
        self.ab = torch.empty(self.qs.shape[0], dtype=torch.float64, device=dev)
        self._forces()  # forces of the initial positions; also sizes the workspace
        self.captures = 0
        self._capture()
        self.steps = 0
        self.host_syncs = 0  # host waits for the device inside step()
        self.repeated_chunks = 0

    def _capture(self):
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step_ops()
        # a later growth of the library's workspace frees memory the graph names
        self._ws_gen = _lib.soap_workspace_generation(self.soap.ctx)
        self.captures += 1

    def _forces(self):
        self.soap.energy_forces(self.nl, self.spec, self.qs, self.al, self.zeta, out=(self.e, self.F, self.ab))

    def _step_ops(self):
        h = 0.5 * self.dt
        self.vel.add_(self.F * self.inv_m, alpha=h)
        self.pos.add_(self.vel, alpha=self.dt)
        d = self.pos - self.pos_at_build
        lim2 = (0.5 * self.skin) ** 2
        torch.logical_or(self.moved, d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2] > lim2,
                         out=self.moved)
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
        self.moved.zero_()
        self.rebuilds += 1

    def _reach(self):
        """(atoms marked, largest displacement since the build, coming drift |v + dt F / 2m| dt)
        in one read-back."""
        disp = (self.pos - self.pos_at_build).norm(dim=1).max()
        drift = (self.vel + (0.5 * self.dt) * self.F * self.inv_m).norm(dim=1).max() * self.dt
        self.host_syncs += 1
        marked, disp, drift = torch.stack([self.moved.any().to(torch.float64), disp, drift]).tolist()
        return marked > 0, disp, drift

    def _checked_step(self):
        """One step after the host has checked the list: rebuilt first if the coming
        drift could take some atom further than skin / 2 from its position at the build."""
        _, disp, drift = self._reach()
        if disp + drift > 0.5 * self.skin:
            if drift > 0.5 * self.skin:
                raise ValueError("one step moves atoms further than skin / 2: raise the skin or lower dt")
            self._rebuild()
        self.graph.replay()

    def step(self, n: int = 1) -> None:
        """n timesteps, in chunks of check_every graph replays with one host read-back each."""
        done = 0
        while done < n:
            k = min(self.check_every, n - done)
            if _lib.soap_workspace_generation(self.soap.ctx) != self._ws_gen:
                self._capture()
            saved = [t.clone() for t in (self.pos, self.vel, self.e, self.F, self.ab)]
            for _ in range(k):
                self.graph.replay()
            marked, disp, drift = self._reach()
            if marked:
                # some step of the chunk ran on a list that may miss pairs: undo it and
                # take its steps one at a time
                for t, v in zip((self.pos, self.vel, self.e, self.F, self.ab), saved):
                    t.copy_(v)
                self.moved.zero_()
                self.repeated_chunks += 1
                for _ in range(k):
                    self._checked_step()
            elif disp + k * drift > 0.5 * self.skin:
                self._rebuild()  # ahead of a chunk that would probably reach the limit
            done += k
            self.steps += k

    def energies(self):
        """(potential, kinetic) in eV at the current step."""
        kin = 0.5 * (self.mass * self.vel * self.vel).sum() / ACC
        return float(self.e.sum().item()), float(kin.item())
