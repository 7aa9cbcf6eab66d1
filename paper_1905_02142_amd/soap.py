"""Torch-facing wrapper of the C ABI: device memory and streams come from PyTorch,
every computation is one call into libsoap.so (see include/soap.h)."""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib

PRECISIONS = {"fp64": _lib.SOAP_FP64, "f32": _lib.SOAP_MIXED_F32, "bf16": _lib.SOAP_MIXED_BF16,
              "bf16x3": _lib.SOAP_MIXED_BF16X3, "bf16ps": _lib.SOAP_MIXED_BF16_PS}
RADIAL_PRECISIONS = {"auto": _lib.SOAP_RADIAL_AUTO, "fp64": _lib.SOAP_RADIAL_FP64, "dd": _lib.SOAP_RADIAL_DD}


@dataclass(frozen=True)
class SoapParams:
    """Hyper-parameters (Eq. (15), Sec. III.B); r_soft None means no buffer zone."""

    n_max: int
    l_max: int
    r_cut: float
    sigma0_r: float
    sigma0_perp: float
    n_species: int = 1
    r_soft: float | None = None
    n_f: float = 4.0
    alpha_r: float = 0.0
    alpha_perp: float = 0.0
    a: float = 0.0
    central_weight: float = 1.0
    l_weight: int = 0
    precision: str = "fp64"
    radial_precision: str = "auto"  # "auto": double-double in the fp64 mode for n_max >= 8

    def c_struct(self) -> _lib.soap_params:
        return _lib.soap_params(self.n_max, self.l_max, self.n_species, self.r_cut,
                                self.r_cut if self.r_soft is None else self.r_soft, self.n_f,
                                self.sigma0_r, self.sigma0_perp, self.alpha_r, self.alpha_perp, self.a,
                                self.central_weight, self.l_weight, PRECISIONS[self.precision],
                                RADIAL_PRECISIONS[self.radial_precision])

    @property
    def dim(self) -> int:
        nch = self.n_max * self.n_species
        return nch * (nch + 1) // 2 * (self.l_max + 1)


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


class NeighbourList:
    """Device CSR neighbour list (soap_nlist) backed by torch tensors."""

    def __init__(self, n_atoms: int, capacity: int, device):
        self.device = device
        self.n_atoms = n_atoms
        self.offsets = torch.empty(n_atoms + 1, dtype=torch.int32, device=device)
        self._alloc(capacity)
        self.n_pairs = 0
        self.n_structures = 1

    def _alloc(self, capacity: int):
        cap = max(1, int(capacity))
        dev = self.device
        self.capacity = cap
        self.j = torch.empty(cap, dtype=torch.int32, device=dev)
        self.img = torch.empty(cap, dtype=torch.int32, device=dev)
        self.rev = torch.empty(cap, dtype=torch.int32, device=dev)
        self.center = torch.empty(cap, dtype=torch.int32, device=dev)
        self.dx = torch.empty(cap, dtype=torch.float64, device=dev)
        self.dy = torch.empty(cap, dtype=torch.float64, device=dev)
        self.dz = torch.empty(cap, dtype=torch.float64, device=dev)

    @property
    def deferred(self) -> bool:
        """True while the pair count is on the device only (after an async build)."""
        return self.n_pairs == _lib.SOAP_PAIRS_DEFERRED

    def c_struct(self) -> _lib.soap_nlist:
        return _lib.soap_nlist(self.n_atoms, self.n_structures, self.n_pairs, self.capacity,
                               _ptr(self.offsets), _ptr(self.j), _ptr(self.img), _ptr(self.rev),
                               _ptr(self.center), _ptr(self.dx), _ptr(self.dy), _ptr(self.dz))

    def image(self) -> torch.Tensor:
        """Lattice translations T of the pairs, shape (n_pairs, 3)."""
        if self.deferred:
            raise RuntimeError("pair count not read back yet: call Soap.check_neighbors first")
        v = self.img[: self.n_pairs].to(torch.int64)
        return torch.stack([((v >> 20) & 1023) - 512, ((v >> 10) & 1023) - 512, (v & 1023) - 512], 1)


class Soap:
    """One descriptor configuration on the current HIP device."""

    def __init__(self, params: SoapParams):
        self.params = params
        self._cp = params.c_struct()
        self.ctx = _lib.soap_create(self._cp)
        self.dim = _lib.soap_descriptor_dim(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            _lib.soap_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- neighbours
    def neighbors(self, positions: torch.Tensor, cells, pbc, struct_offsets=None,
                  nl: NeighbourList | None = None, capacity: int | None = None) -> NeighbourList:
        """soap_build_neighbors; grows the list and retries once on capacity overflow."""
        pos = positions.contiguous()
        assert pos.dtype == torch.float64 and pos.is_cuda
        n = pos.shape[0]
        cells = np.ascontiguousarray(np.asarray(cells, dtype=np.float64).reshape(-1, 9))
        pbc = np.ascontiguousarray(np.asarray(pbc, dtype=np.int32).reshape(-1, 3))
        ns = cells.shape[0]
        so = None if struct_offsets is None else np.ascontiguousarray(np.asarray(struct_offsets, dtype=np.int32))
        if nl is None or nl.n_atoms != n:
            cap = capacity if capacity is not None else max(64, n * 64)
            nl = NeighbourList(n, cap, pos.device)
        for _ in range(2):
            c = nl.c_struct()
            st = _lib.soap_build_neighbors(self.ctx, n, pos.data_ptr(), cells.ctypes.data, pbc.ctypes.data,
                                           None if so is None else so.ctypes.data, ns, c, _stream())
            if st == _lib.SOAP_EOVERFLOW:
                nl._alloc(int(c.n_pairs * 1.1) + 64)
                continue
            nl.n_pairs = int(c.n_pairs)
            nl.n_structures = ns
            return nl
        raise _lib.SoapError(_lib.SOAP_EOVERFLOW, "neighbour list still overflows after growing")

    def neighbors_async(self, positions: torch.Tensor, cells, pbc, nl: NeighbourList,
                        struct_offsets=None) -> NeighbourList:
        """soap_build_neighbors_async into an existing list: no host synchronisation,
        nl.n_pairs becomes SOAP_PAIRS_DEFERRED until check_neighbors."""
        pos = positions.contiguous()
        assert pos.dtype == torch.float64 and pos.is_cuda and pos.shape[0] == nl.n_atoms
        cells = np.ascontiguousarray(np.asarray(cells, dtype=np.float64).reshape(-1, 9))
        pbc = np.ascontiguousarray(np.asarray(pbc, dtype=np.int32).reshape(-1, 3))
        so = None if struct_offsets is None else np.ascontiguousarray(np.asarray(struct_offsets, dtype=np.int32))
        c = nl.c_struct()
        _lib.soap_build_neighbors_async(self.ctx, nl.n_atoms, pos.data_ptr(), cells.ctypes.data, pbc.ctypes.data,
                                        None if so is None else so.ctypes.data, cells.shape[0], c, _stream())
        nl.n_pairs = int(c.n_pairs)
        nl.n_structures = cells.shape[0]
        return nl

    def check_neighbors(self, nl: NeighbourList) -> int:
        """soap_neighbors_check: waits for the stream, stores and returns the pair count of
        the last build; raises SoapError on overflow or invalid positions."""
        st, n = _lib.soap_neighbors_check(self.ctx, nl.c_struct(), _stream())
        if st == _lib.SOAP_EOVERFLOW:
            raise _lib.SoapError(st, f"neighbour list needs {n} pairs, capacity {nl.capacity}")
        nl.n_pairs = n
        return n

    # ---------------------------------------------------------------- descriptor
    def descriptor(self, nl: NeighbourList, species: torch.Tensor, with_norm: bool = False, out=None):
        q = torch.empty(nl.n_atoms, self.dim, dtype=torch.float64, device=nl.device) if out is None else out
        assert q.dtype == torch.float64 and q.is_contiguous() and q.shape == (nl.n_atoms, self.dim)
        pn = torch.empty(nl.n_atoms, dtype=torch.float64, device=nl.device)
        sp = species.to(torch.int32).contiguous()
        _lib.soap_descriptor(self.ctx, nl.c_struct(), sp.data_ptr(), q.data_ptr(), pn.data_ptr(), _stream())
        return (q, pn) if with_norm else q

    def descriptor_grad(self, nl: NeighbourList, species: torch.Tensor, q_bar: torch.Tensor,
                        pos_grad: torch.Tensor | None = None) -> torch.Tensor:
        if pos_grad is None:
            pos_grad = torch.zeros(nl.n_atoms, 3, dtype=torch.float64, device=nl.device)
        sp = species.to(torch.int32).contiguous()
        qb = q_bar.to(torch.float64).contiguous()
        _lib.soap_descriptor_grad(self.ctx, nl.c_struct(), sp.data_ptr(), qb.data_ptr(), pos_grad.data_ptr(),
                                  _stream())
        return pos_grad

    def descriptor_jacobian(self, nl: NeighbourList, species: torch.Tensor, k0: int = 0, k1: int | None = None):
        """soap_descriptor_jacobian: (k1 - k0, 3, n_pairs) with [k, x, p] = d q_{i,k} / d (d_p)_x
        for pair p of centre i (d_p = r_j + T - r_i)."""
        k1 = self.dim if k1 is None else k1
        bound = nl.capacity if nl.deferred else max(nl.n_pairs, 1)
        jac = torch.empty(max(k1 - k0, 0), 3, bound, dtype=torch.float64, device=nl.device)
        sp = species.to(torch.int32).contiguous()
        _lib.soap_descriptor_jacobian(self.ctx, nl.c_struct(), sp.data_ptr(), int(k0), int(k1), jac.data_ptr(), _stream())
        return jac if nl.deferred else jac[:, :, : nl.n_pairs]

    def energy_forces(self, nl: NeighbourList, species: torch.Tensor, q_sparse: torch.Tensor,
                      alpha: torch.Tensor, zeta: int, forces: bool = True, alpha_grad: bool = True,
                      out=None):
        """gap_energy_forces: (e_atom, forces or None, dE/dalpha or None)."""
        dev = nl.device
        qs = q_sparse.to(torch.float64).contiguous()
        al = alpha.to(torch.float64).contiguous()
        M = qs.shape[0]
        if out is None:
            e = torch.empty(nl.n_atoms, dtype=torch.float64, device=dev)
            F = torch.empty(nl.n_atoms, 3, dtype=torch.float64, device=dev) if forces else None
            ab = torch.empty(M, dtype=torch.float64, device=dev) if alpha_grad else None
        else:
            e, F, ab = out
        sp = species.to(torch.int32).contiguous()
        _lib.gap_energy_forces(self.ctx, nl.c_struct(), sp.data_ptr(), qs.data_ptr(), al.data_ptr(), M, int(zeta),
                               e.data_ptr(), _ptr(F), _ptr(ab), _stream())
        return e, F, ab

    def update_pair_vectors(self, nl: NeighbourList, positions: torch.Tensor) -> None:
        """soap_update_pair_vectors: the list's d_p from the current positions (a reused skin list)."""
        pos = positions.contiguous()
        assert pos.dtype == torch.float64 and pos.is_cuda
        _lib.soap_update_pair_vectors(self.ctx, nl.c_struct(), pos.data_ptr(), _stream())

    def set_neighbor_skin(self, skin: float) -> None:
        """soap_set_neighbor_skin: later lists reach r_cut + skin (pairs beyond r_cut weigh zero)."""
        _lib.soap_set_neighbor_skin(self.ctx, skin)

    # ---------------------------------------------------------------- tuning
    @property
    def tuning(self) -> dict:
        return _lib.soap_get_tuning(self.ctx).as_dict()

    def set_tuning(self, gap_fused: int = 0, gap_slices: int = 0, prep_block: int = 256, cell_split: int = 2,
                   gap_tile: int = 0) -> None:
        _lib.soap_set_tuning(self.ctx, _lib.soap_tuning(gap_fused, gap_slices, prep_block, cell_split, gap_tile))

    def set_tuning_cache(self, path: str | None) -> None:
        """soap_set_tuning_cache: autotune() then answers from / stores into this file."""
        _lib.check(_lib.load().soap_set_tuning_cache(self.ctx, None if path is None else os.fsencode(path)),
                   self.ctx)

    @property
    def tuning_cache_hits(self) -> int:
        return int(_lib.load().soap_tuning_cache_hits(self.ctx))

    def tuning_key(self, n_atoms: int, M: int) -> _lib.soap_tuning_key:
        k = _lib.soap_tuning_key()
        _lib.check(_lib.load().soap_tuning_key_for(self.ctx, int(n_atoms), int(M), ctypes.byref(k)), self.ctx)
        return k

    def autotune_neighbors(self, positions: torch.Tensor, cells, pbc, nl: NeighbourList, struct_offsets=None,
                           repeats: int = 3) -> dict:
        """soap_autotune_neighbors: times the build for cell_split 1, 2, 3, installs the
        fastest and leaves nl built with it."""
        pos = positions.contiguous()
        assert pos.dtype == torch.float64 and pos.is_cuda and pos.shape[0] == nl.n_atoms
        cells = np.ascontiguousarray(np.asarray(cells, dtype=np.float64).reshape(-1, 9))
        pbc = np.ascontiguousarray(np.asarray(pbc, dtype=np.int32).reshape(-1, 3))
        so = None if struct_offsets is None else np.ascontiguousarray(np.asarray(struct_offsets, dtype=np.int32))
        c = nl.c_struct()
        t = _lib.soap_tuning()
        _lib.check(_lib.load().soap_autotune_neighbors(self.ctx, nl.n_atoms, pos.data_ptr(), cells.ctypes.data,
                                                       pbc.ctypes.data, None if so is None else so.ctypes.data,
                                                       cells.shape[0], ctypes.byref(c), int(repeats),
                                                       ctypes.byref(t), _stream()), self.ctx)
        nl.n_pairs = int(c.n_pairs)
        nl.n_structures = cells.shape[0]
        return t.as_dict()

    def autotune(self, nl: NeighbourList, species: torch.Tensor, q_sparse: torch.Tensor, alpha: torch.Tensor,
                 zeta: int, repeats: int = 3) -> dict:
        """soap_autotune on these inputs; installs and returns the fastest setting (from the
        attached cache when it holds one for these inputs)."""
        qs = q_sparse.to(torch.float64).contiguous()
        al = alpha.to(torch.float64).contiguous()
        sp = species.to(torch.int32).contiguous()
        t = _lib.soap_autotune(self.ctx, nl.c_struct(), sp.data_ptr(), qs.data_ptr(), al.data_ptr(), qs.shape[0],
                               int(zeta), int(repeats), _stream())
        return t.as_dict()
