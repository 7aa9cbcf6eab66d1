"""ctypes binding of libsoap.so: the C ABI of include/soap.h, same names, argument
marshalling only.  Every step of the computation runs in the HIP library; if
the library is missing or cannot be loaded this module raises instead of
falling back to anything else."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsoap.so")
# an alternative build of the same library (e.g. other compile-time tuning) can be named here
LIB_PATH = os.environ.get("SOAP_LIBRARY", LIB_PATH)

SOAP_OK, SOAP_EINVAL, SOAP_ENOMEM, SOAP_EOVERFLOW, SOAP_EHIP, SOAP_ENOTSUP = 0, -1, -2, -3, -4, -5
SOAP_FP64, SOAP_MIXED_F32, SOAP_MIXED_BF16, SOAP_MIXED_BF16X3, SOAP_MIXED_BF16_PS = 0, 1, 2, 3, 4
SOAP_RADIAL_AUTO, SOAP_RADIAL_FP64, SOAP_RADIAL_DD = 0, 1, 2
SOAP_PAIRS_DEFERRED = -1

# every function include/soap.h declares
EXPORTED = (
    "soap_create", "soap_destroy", "soap_descriptor_dim", "soap_status_string", "soap_last_error",
    "soap_build_neighbors", "soap_descriptor", "soap_descriptor_grad", "gap_energy_forces",
    "soap_radial_basis_table", "soap_workspace_bytes", "soap_profile", "soap_profile_read", "soap_stage_name",
    "soap_get_tuning", "soap_set_tuning", "soap_autotune", "soap_profile_stages",
    "soap_build_neighbors_async", "soap_neighbors_check", "soap_descriptor_jacobian", "soap_set_neighbor_skin",
    "soap_update_pair_vectors", "soap_workspace_generation", "soap_descriptor_noalloc",
    "soap_autotune_neighbors", "soap_tuning_key_for", "soap_tuning_cache_lookup", "soap_tuning_cache_store",
    "soap_set_tuning_cache", "soap_tuning_cache_hits",
)
SOAP_TUNING_CACHE_VERSION = 1
SOAP_NOALLOC_SCRATCH_BYTES = 128 << 20
STAGES = ("neighbors", "descriptor", "gap_scores", "gap_qbar", "pair_adjoint", "force_gather", "gap_fused",
          "pair_prep", "cbar", "pair_angular")


class soap_params(ctypes.Structure):
    _fields_ = [
        ("n_max", ctypes.c_int), ("l_max", ctypes.c_int), ("n_species", ctypes.c_int),
        ("r_cut", ctypes.c_double), ("r_soft", ctypes.c_double), ("n_f", ctypes.c_double),
        ("sigma0_r", ctypes.c_double), ("sigma0_perp", ctypes.c_double),
        ("alpha_r", ctypes.c_double), ("alpha_perp", ctypes.c_double), ("a", ctypes.c_double),
        ("central_weight", ctypes.c_double), ("l_weight", ctypes.c_int), ("precision", ctypes.c_int),
        ("radial_precision", ctypes.c_int),
    ]


class soap_tuning(ctypes.Structure):
    _fields_ = [("gap_fused", ctypes.c_int), ("gap_slices", ctypes.c_int), ("prep_block", ctypes.c_int),
                ("cell_split", ctypes.c_int), ("gap_tile", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class soap_tuning_key(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int), ("n_channels", ctypes.c_int), ("l_max", ctypes.c_int),
                ("K", ctypes.c_int), ("M", ctypes.c_int), ("precision", ctypes.c_int), ("radial_dd", ctypes.c_int),
                ("size_class", ctypes.c_int), ("arch", ctypes.c_char * 32)]


class soap_nlist(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int), ("n_structures", ctypes.c_int),
        ("n_pairs", ctypes.c_longlong), ("capacity", ctypes.c_longlong),
        ("offsets", ctypes.c_void_p), ("j", ctypes.c_void_p), ("img", ctypes.c_void_p),
        ("rev", ctypes.c_void_p), ("center", ctypes.c_void_p),
        ("dx", ctypes.c_void_p), ("dy", ctypes.c_void_p), ("dz", ctypes.c_void_p),
    ]


class SoapError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libsoap.so once and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is not built; run __graft_entry__.build() or "
                          f"python -m paper_1905_02142_amd.build")
    lib = ctypes.CDLL(path)
    vp, i, d, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    P = ctypes.POINTER
    lib.soap_create.argtypes = [P(soap_params), P(vp)]
    lib.soap_create.restype = i
    lib.soap_destroy.argtypes = [vp]
    lib.soap_destroy.restype = None
    lib.soap_descriptor_dim.argtypes = [vp]
    lib.soap_descriptor_dim.restype = i
    lib.soap_status_string.argtypes = [i]
    lib.soap_status_string.restype = ctypes.c_char_p
    lib.soap_last_error.argtypes = [vp]
    lib.soap_last_error.restype = ctypes.c_char_p
    lib.soap_workspace_bytes.argtypes = [vp]
    lib.soap_workspace_bytes.restype = ll
    lib.soap_workspace_generation.argtypes = [vp]
    lib.soap_workspace_generation.restype = ll
    lib.soap_build_neighbors.argtypes = [vp, i, vp, vp, vp, vp, i, P(soap_nlist), P(ll), vp]
    lib.soap_build_neighbors.restype = i
    lib.soap_build_neighbors_async.argtypes = [vp, i, vp, vp, vp, vp, i, P(soap_nlist), vp]
    lib.soap_build_neighbors_async.restype = i
    lib.soap_neighbors_check.argtypes = [vp, P(soap_nlist), P(ll), vp]
    lib.soap_neighbors_check.restype = i
    lib.soap_descriptor.argtypes = [vp, P(soap_nlist), vp, vp, vp, vp]
    lib.soap_descriptor.restype = i
    lib.soap_descriptor_noalloc.argtypes = [vp, P(soap_nlist), vp, vp, vp, vp]
    lib.soap_descriptor_noalloc.restype = i
    lib.soap_descriptor_grad.argtypes = [vp, P(soap_nlist), vp, vp, vp, vp]
    lib.soap_descriptor_grad.restype = i
    lib.soap_update_pair_vectors.argtypes = [vp, P(soap_nlist), vp, vp]
    lib.soap_update_pair_vectors.restype = i
    lib.soap_set_neighbor_skin.argtypes = [vp, d]
    lib.soap_set_neighbor_skin.restype = i
    lib.soap_descriptor_jacobian.argtypes = [vp, P(soap_nlist), vp, i, i, vp, vp]
    lib.soap_descriptor_jacobian.restype = i
    lib.gap_energy_forces.argtypes = [vp, P(soap_nlist), vp, vp, vp, i, i, vp, vp, vp, vp]
    lib.gap_energy_forces.restype = i
    lib.soap_radial_basis_table.argtypes = [i, d, d, vp, vp]
    lib.soap_radial_basis_table.restype = i
    lib.soap_profile.argtypes = [vp, i]
    lib.soap_profile.restype = i
    lib.soap_profile_read.argtypes = [vp, vp, vp]
    lib.soap_profile_read.restype = i
    lib.soap_stage_name.argtypes = [i]
    lib.soap_stage_name.restype = ctypes.c_char_p
    lib.soap_profile_stages.argtypes = [vp, ctypes.c_uint]
    lib.soap_profile_stages.restype = i
    lib.soap_get_tuning.argtypes = [vp, P(soap_tuning)]
    lib.soap_get_tuning.restype = i
    lib.soap_set_tuning.argtypes = [vp, P(soap_tuning)]
    lib.soap_set_tuning.restype = i
    lib.soap_autotune.argtypes = [vp, P(soap_nlist), vp, vp, vp, i, i, i, P(soap_tuning), vp]
    lib.soap_autotune.restype = i
    lib.soap_autotune_neighbors.argtypes = [vp, i, vp, vp, vp, vp, i, P(soap_nlist), i, P(soap_tuning), vp]
    lib.soap_autotune_neighbors.restype = i
    lib.soap_tuning_key_for.argtypes = [vp, i, i, P(soap_tuning_key)]
    lib.soap_tuning_key_for.restype = i
    lib.soap_tuning_cache_lookup.argtypes = [ctypes.c_char_p, P(soap_tuning_key), P(soap_tuning), P(i)]
    lib.soap_tuning_cache_lookup.restype = i
    lib.soap_tuning_cache_store.argtypes = [ctypes.c_char_p, P(soap_tuning_key), P(soap_tuning)]
    lib.soap_tuning_cache_store.restype = i
    lib.soap_set_tuning_cache.argtypes = [vp, ctypes.c_char_p]
    lib.soap_set_tuning_cache.restype = i
    lib.soap_tuning_cache_hits.argtypes = [vp]
    lib.soap_tuning_cache_hits.restype = ll
    _lib = lib
    return lib


def check(status: int, ctx=None) -> None:
    if status != SOAP_OK:
        lib = load()
        msg = lib.soap_status_string(status).decode()
        if ctx:
            detail = lib.soap_last_error(ctx).decode()
            if detail:
                msg = f"{msg}: {detail}"
        raise SoapError(status, msg)


# Thin wrappers with the C names.  Pointers are ints (device addresses, e.g.
# tensor.data_ptr()) or ctypes objects; streams are hipStream_t handles as ints.

def soap_create(params: soap_params) -> int:
    ctx = ctypes.c_void_p()
    check(load().soap_create(ctypes.byref(params), ctypes.byref(ctx)))
    return ctx.value


def soap_destroy(ctx: int) -> None:
    load().soap_destroy(ctx)


def soap_descriptor_dim(ctx: int) -> int:
    return load().soap_descriptor_dim(ctx)


def soap_workspace_bytes(ctx: int) -> int:
    return load().soap_workspace_bytes(ctx)


def soap_workspace_generation(ctx: int) -> int:
    return load().soap_workspace_generation(ctx)


def soap_build_neighbors(ctx, n_atoms, pos, cells, pbc, struct_offsets, n_structures, nl: soap_nlist,
                         stream) -> int:
    """Returns the status (SOAP_OK or SOAP_EOVERFLOW); other failures raise. nl.n_pairs holds the count."""
    req = ctypes.c_longlong(0)
    st = load().soap_build_neighbors(ctx, n_atoms, pos, cells, pbc, struct_offsets, n_structures,
                                     ctypes.byref(nl), ctypes.byref(req), stream)
    if st == SOAP_EOVERFLOW:
        nl.n_pairs = req.value
        return st
    check(st, ctx)
    return st


def soap_build_neighbors_async(ctx, n_atoms, pos, cells, pbc, struct_offsets, n_structures, nl: soap_nlist,
                               stream) -> None:
    """Enqueues the build; nl.n_pairs becomes SOAP_PAIRS_DEFERRED."""
    check(load().soap_build_neighbors_async(ctx, n_atoms, pos, cells, pbc, struct_offsets, n_structures,
                                            ctypes.byref(nl), stream), ctx)


def soap_neighbors_check(ctx, nl: soap_nlist, stream) -> tuple[int, int]:
    """(status, pair count) of the last build: SOAP_OK or SOAP_EOVERFLOW; other failures raise."""
    n = ctypes.c_longlong(0)
    st = load().soap_neighbors_check(ctx, ctypes.byref(nl), ctypes.byref(n), stream)
    if st != SOAP_EOVERFLOW:
        check(st, ctx)
    return st, n.value


def soap_descriptor(ctx, nl: soap_nlist, species, q, p_norm, stream) -> None:
    check(load().soap_descriptor(ctx, ctypes.byref(nl), species, q, p_norm, stream), ctx)


def soap_descriptor_noalloc(ctx, nl: soap_nlist, species, q, p_norm, stream) -> None:
    check(load().soap_descriptor_noalloc(ctx, ctypes.byref(nl), species, q, p_norm, stream), ctx)


def soap_descriptor_grad(ctx, nl: soap_nlist, species, q_bar, pos_grad, stream) -> None:
    check(load().soap_descriptor_grad(ctx, ctypes.byref(nl), species, q_bar, pos_grad, stream), ctx)


def soap_update_pair_vectors(ctx, nl: soap_nlist, pos, stream) -> None:
    check(load().soap_update_pair_vectors(ctx, ctypes.byref(nl), pos, stream), ctx)


def soap_set_neighbor_skin(ctx, skin: float) -> None:
    check(load().soap_set_neighbor_skin(ctx, float(skin)), ctx)


def soap_descriptor_jacobian(ctx, nl: soap_nlist, species, k0, k1, jac, stream) -> None:
    check(load().soap_descriptor_jacobian(ctx, ctypes.byref(nl), species, k0, k1, jac, stream), ctx)


def gap_energy_forces(ctx, nl: soap_nlist, species, q_sparse, alpha, M, zeta, e_atom, forces, alpha_grad,
                      stream) -> None:
    check(load().gap_energy_forces(ctx, ctypes.byref(nl), species, q_sparse, alpha, M, zeta, e_atom, forces,
                                   alpha_grad, stream), ctx)


def soap_radial_basis_table(n_max: int, r_cut: float, sigma0_r: float, W, lam) -> None:
    check(load().soap_radial_basis_table(n_max, r_cut, sigma0_r, W, lam))


def soap_profile(ctx, enable: bool) -> None:
    check(load().soap_profile(ctx, 1 if enable else 0), ctx)


def soap_profile_stages(ctx, names) -> None:
    """Record events only around the named stages."""
    mask = 0
    for n in names:
        mask |= 1 << STAGES.index(n)
    check(load().soap_profile_stages(ctx, mask), ctx)


def soap_profile_read(ctx) -> dict:
    """{stage name: (milliseconds, launches)} accumulated since the last read."""
    import numpy as np

    ms = np.zeros(len(STAGES))
    n = np.zeros(len(STAGES), dtype=np.int64)
    check(load().soap_profile_read(ctx, ms.ctypes.data, n.ctypes.data), ctx)
    return {STAGES[k]: (float(ms[k]), int(n[k])) for k in range(len(STAGES))}


def soap_get_tuning(ctx) -> soap_tuning:
    t = soap_tuning()
    check(load().soap_get_tuning(ctx, ctypes.byref(t)), ctx)
    return t


def soap_set_tuning(ctx, t: soap_tuning) -> None:
    check(load().soap_set_tuning(ctx, ctypes.byref(t)), ctx)


def soap_autotune(ctx, nl: soap_nlist, species, q_sparse, alpha, M, zeta, repeats, stream) -> soap_tuning:
    t = soap_tuning()
    check(load().soap_autotune(ctx, ctypes.byref(nl), species, q_sparse, alpha, M, zeta, repeats, ctypes.byref(t),
                               stream), ctx)
    return t


def soap_tuning_cache_lookup(path: str, key: soap_tuning_key):
    """(setting, found) for key in the cache file at path (host only)."""
    t = soap_tuning()
    found = ctypes.c_int(0)
    check(load().soap_tuning_cache_lookup(os.fsencode(path), ctypes.byref(key), ctypes.byref(t), ctypes.byref(found)))
    return t, bool(found.value)


def soap_tuning_cache_store(path: str, key: soap_tuning_key, t: soap_tuning) -> None:
    check(load().soap_tuning_cache_store(os.fsencode(path), ctypes.byref(key), ctypes.byref(t)))
