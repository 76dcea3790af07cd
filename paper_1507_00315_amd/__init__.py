"""Exact and approximate counting of Skolem, Langford and hooked Skolem pairings
on AMD Instinct MI355X (gfx950), after arXiv 1507.00315.

Thin ctypes binding over the C ABI in ``include/skolem.h``: argument
marshalling only.  Every step of the computation runs in ``libskolem.so``
(host planning and CRT in C++, the sums in HIP kernels).  There is no
fallback: if the library is missing this module raises on import of the
binding (``lib()``), and if no GPU is present the calls report a device error.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Callable, Dict, Iterable, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libskolem.so")

SKOLEM, LANGFORD, HOOKED = 0, 1, 2
VARIANTS = {"skolem": SKOLEM, "langford": LANGFORD, "hooked": HOOKED}

ORDERED, NO_SHORTCUT, VERIFY, NO_SYMMETRY = 0x1, 0x2, 0x4, 0x8

STATUS = {0: "SK_OK", -1: "SK_EINVAL", -2: "SK_ERANGE", -3: "SK_EDEVICE", -4: "SK_ECHECK",
          -5: "SK_ENOMEM", -6: "SK_EABORTED", -7: "SK_ENOLIB"}


class SkolemError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        self.status = status
        msg = f"{what}: {STATUS.get(status, status)}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


class U128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]

    def value(self) -> int:
        return (int(self.hi) << 64) | int(self.lo)


class Tuning(ctypes.Structure):
    _fields_ = [("log2_chunk_terms", ctypes.c_int), ("waves_per_launch", ctypes.c_int),
                ("primes", ctypes.c_int), ("kernel", ctypes.c_int), ("primes_per_item", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("wall_ms", ctypes.c_double),
                ("terms", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("chunks", ctypes.c_uint64), ("nprimes", ctypes.c_int), ("passes", ctypes.c_int),
                ("log2_chunk_terms", ctypes.c_int), ("kernel_variant", ctypes.c_int),
                ("ms_per_launch_avg", ctypes.c_double), ("primes", ctypes.c_uint64 * 8),
                ("symmetry_halved", ctypes.c_int), ("reversal_quads", ctypes.c_int)]

    def as_dict(self) -> Dict:
        d = {name: getattr(self, name) for name, _ in self._fields_ if name != "primes"}
        d["primes"] = [int(x) for x in self.primes if x]
        return d


class Instance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("variant", ctypes.c_int), ("flags", ctypes.c_uint)]


class PlanDesc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("n_lane", ctypes.c_int), ("n_walk", ctypes.c_int),
                ("n_job", ctypes.c_int), ("quads", ctypes.c_int), ("groups", ctypes.c_int),
                ("halved", ctypes.c_int), ("primes", ctypes.c_int), ("slot_factor", ctypes.c_int * 32),
                ("symmetric", ctypes.c_int), ("reversal_quads", ctypes.c_int)]


class LearnedParams(ctypes.Structure):
    _fields_ = [("hidden1", ctypes.c_int), ("hidden2", ctypes.c_int), ("first_level", ctypes.c_int),
                ("plain_per_learned", ctypes.c_uint64), ("train_iterations", ctypes.c_uint64),
                ("snapshots", ctypes.c_int), ("train_steps", ctypes.c_int), ("minibatch", ctypes.c_int),
                ("lr", ctypes.c_double), ("init_seed", ctypes.c_uint64), ("params", ctypes.POINTER(ctypes.c_float))]


class PtParams(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("beta", ctypes.POINTER(ctypes.c_double)), ("ladders", ctypes.c_int),
                ("iterations", ctypes.c_uint64), ("seed", ctypes.c_uint64), ("proposal", ctypes.c_int),
                ("flags", ctypes.c_uint), ("segment", ctypes.c_uint64), ("burn_in", ctypes.c_uint64),
                ("learned", ctypes.POINTER(LearnedParams))]


class PtStats(ctypes.Structure):
    _fields_ = [("mean_energy", ctypes.c_double * 64), ("move_accept", ctypes.c_double * 64),
                ("swap_accept", ctypes.c_double * 64), ("ratio", ctypes.c_double * 64),
                ("gpu_ms", ctypes.c_double), ("wall_ms", ctypes.c_double), ("moves", ctypes.c_uint64),
                ("levels", ctypes.c_int), ("ladders", ctypes.c_int), ("learned_accept", ctypes.c_double * 64),
                ("learned_moves", ctypes.c_uint64), ("train_ms", ctypes.c_double), ("train_loss", ctypes.c_double),
                ("estimate_half", ctypes.c_double * 2), ("std_error_half", ctypes.c_double * 2),
                ("half_z", ctypes.c_double)]

    def as_dict(self) -> Dict:
        M = self.levels
        return {"mean_energy": list(self.mean_energy[:M]), "move_accept": list(self.move_accept[:M]),
                "swap_accept": list(self.swap_accept[:M]), "ratio": list(self.ratio[:M]),
                "gpu_ms": self.gpu_ms, "wall_ms": self.wall_ms, "moves": int(self.moves),
                "levels": M, "ladders": self.ladders, "learned_accept": list(self.learned_accept[:M]),
                "learned_moves": int(self.learned_moves), "train_ms": self.train_ms,
                "train_loss": self.train_loss, "estimate_half": list(self.estimate_half),
                "std_error_half": list(self.std_error_half), "half_z": self.half_z}


PROGRESS_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64)

_lib = None


def lib() -> ctypes.CDLL:
    """Loads libskolem.so (built by ``paper_1507_00315_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_1507_00315_amd.build` "
                           "(there is no CPU fallback)")
    # torch (the device-memory and stream plumbing) ships its own HIP runtime
    # under the same soname; loading it first makes the library bind to that
    # copy, so a process that uses both holds one HIP runtime, not two.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    c_int, c_uint, c_size, vp = ctypes.c_int, ctypes.c_uint, ctypes.c_size_t, ctypes.c_void_p
    u64p = ctypes.POINTER(ctypes.c_uint64)
    L.sk_set_device.argtypes = [c_int]
    L.sk_count.argtypes = [c_int, c_int, c_uint, ctypes.POINTER(U128)]
    L.sk_count_ex.argtypes = [c_int, c_int, c_uint, ctypes.POINTER(Tuning), vp, c_size, vp, PROGRESS_FN, vp,
                              ctypes.POINTER(Stats), ctypes.POINTER(U128)]
    L.sk_sign_sum_residues.argtypes = [c_int, c_int, u64p, c_int, ctypes.POINTER(Tuning), vp, u64p]
    L.sk_partial_chunks.argtypes = [c_int, c_int, c_int, u64p, c_size, u64p, c_int, ctypes.POINTER(Tuning), vp,
                                    c_size, vp, u64p]
    L.sk_max_chunk_bits.argtypes = [c_int, c_int]
    L.sk_last_stats.argtypes = [ctypes.POINTER(Stats)]
    L.sk_count_part.argtypes = [c_int, c_int, c_uint, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(Tuning), vp,
                                c_size, vp, PROGRESS_FN, vp, ctypes.POINTER(Stats), u64p]
    L.sk_count_combine.argtypes = [c_int, c_int, c_uint, u64p, ctypes.c_uint64, ctypes.POINTER(U128)]
    L.sk_describe.argtypes = [c_int, c_int, ctypes.POINTER(PlanDesc)]
    L.sk_describe_larsen.argtypes = [c_int, c_int, ctypes.POINTER(PlanDesc)]
    L.sk_pt_bins.argtypes = [c_int, c_int]
    L.sk_pt_run.argtypes = [c_int, c_int, ctypes.POINTER(PtParams), vp, u64p, u64p, u64p,
                            ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32)]
    L.sk_pt_tune_ladder.argtypes = [c_int, c_int, ctypes.c_double, ctypes.c_double, c_int, c_int, ctypes.c_uint64,
                                    ctypes.c_uint64, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(c_int),
                                    ctypes.POINTER(ctypes.c_double)]
    L.sk_approx.argtypes = [c_int, c_int, ctypes.POINTER(PtParams), vp, ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(PtStats)]
    L.sk_count_batch.argtypes = [ctypes.POINTER(Instance), c_size, ctypes.POINTER(Tuning), vp, c_size, vp,
                                 ctypes.POINTER(Stats), ctypes.POINTER(U128)]
    L.sk_count_larsen.argtypes = [c_int, c_int, c_uint, ctypes.POINTER(Tuning), vp, c_size, vp,
                                  ctypes.POINTER(Stats), ctypes.POINTER(U128)]
    L.sk_count_batch_noalloc.argtypes = [ctypes.POINTER(Instance), c_size, ctypes.POINTER(Tuning), vp,
                                         ctypes.POINTER(Stats), ctypes.POINTER(U128)]
    L.sk_workspace_bytes.argtypes = [ctypes.POINTER(Instance), c_size, ctypes.POINTER(Tuning)]
    L.sk_workspace_bytes.restype = c_size
    L.sk_partial_workspace_bytes.argtypes = [c_int, c_int, c_size, c_int, ctypes.POINTER(Tuning)]
    L.sk_partial_workspace_bytes.restype = c_size
    L.sk_autotune_batch.argtypes = [ctypes.POINTER(Instance), c_size, vp, ctypes.POINTER(Tuning),
                                    ctypes.POINTER(ctypes.c_double)]
    fp = ctypes.POINTER(ctypes.c_float)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    dp = ctypes.POINTER(ctypes.c_double)
    L.sk_mlp_param_count.argtypes = [c_int, c_int, c_int, c_int]
    L.sk_mlp_param_count.restype = c_size
    L.sk_mlp_init.argtypes = [c_int, c_int, c_int, c_int, ctypes.c_uint64, ctypes.c_double, fp]
    L.sk_mlp_forward.argtypes = [c_int, c_int, c_int, c_int, fp, u8p, dp, c_int, vp, fp]
    L.sk_mlp_loss_grad.argtypes = [c_int, c_int, c_int, c_int, fp, u8p, dp, c_int, vp, dp, fp]
    L.sk_mlp_train.argtypes = [c_int, c_int, c_int, c_int, fp, u8p, dp, c_int, c_int, c_int, ctypes.c_double, vp,
                               dp]
    L.sk_mlp_mh_step.argtypes = [c_int, c_int, c_int, c_int, fp, u8p, dp, u32p, u32p, c_int, vp, u8p, u8p, u8p, fp,
                                 fp]
    L.sk_strerror.argtypes = [c_int]
    L.sk_strerror.restype = ctypes.c_char_p
    L.sk_last_error.restype = ctypes.c_char_p
    L.sk_kernel_name.argtypes = [c_int]
    L.sk_kernel_name.restype = ctypes.c_char_p
    for fn in ("sk_set_device", "sk_count", "sk_count_ex", "sk_sign_sum_residues", "sk_partial_chunks", "sk_count_batch_noalloc",
               "sk_count_larsen", "sk_describe_larsen", "sk_pt_tune_ladder",
               "sk_max_chunk_bits", "sk_describe", "sk_count_batch", "sk_autotune_batch", "sk_pt_bins",
               "sk_pt_run", "sk_approx", "sk_last_stats", "sk_count_part", "sk_count_combine", "sk_mlp_init", "sk_mlp_forward", "sk_mlp_loss_grad", "sk_mlp_train",
               "sk_mlp_mh_step"):
        getattr(L, fn).restype = c_int
    _lib = L
    return L


EXPORTED = ["sk_set_device", "sk_count", "sk_count_ex", "sk_count_batch", "sk_autotune_batch", "sk_pt_bins",
            "sk_workspace_bytes", "sk_partial_workspace_bytes", "sk_count_batch_noalloc", "sk_count_larsen", "sk_describe_larsen", "sk_pt_tune_ladder",
            "sk_pt_run", "sk_approx", "sk_sign_sum_residues", "sk_partial_chunks",
            "sk_max_chunk_bits", "sk_describe", "sk_strerror", "sk_last_error", "sk_u128_to_decimal", "sk_kernel_name",
            "sk_last_stats", "sk_count_part", "sk_count_combine", "sk_mlp_param_count", "sk_mlp_init", "sk_mlp_forward", "sk_mlp_loss_grad", "sk_mlp_train",
            "sk_mlp_mh_step"]


def _variant(v) -> int:
    if isinstance(v, str):
        return VARIANTS[v.lower()]
    return int(v)


def _check(status: int, what: str) -> None:
    if status != 0:
        detail = lib().sk_last_error().decode(errors="replace")
        raise SkolemError(status, what, detail)


def _workspace(workspace):
    """(device pointer, bytes) of a workspace: None, a torch tensor on the
    GPU (its storage), or a (pointer, bytes) pair."""
    if workspace is None:
        return None, 0
    if hasattr(workspace, "data_ptr"):
        return int(workspace.data_ptr()), int(workspace.numel() * workspace.element_size())
    ptr, nbytes = workspace
    return int(ptr), int(nbytes)


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):  # torch.cuda.Stream
        return int(stream.cuda_stream)
    return int(stream)


def _tuning(tuning: Optional[Dict]) -> Optional[Tuning]:
    if not tuning:
        return None
    return Tuning(int(tuning.get("log2_chunk_terms", 0)), int(tuning.get("waves_per_launch", 0)),
                  int(tuning.get("primes", 0)), int(tuning.get("kernel", 0)), int(tuning.get("primes_per_item", 0)))


def set_device(device: int) -> None:
    _check(lib().sk_set_device(device), "sk_set_device")


@dataclass
class CountResult:
    count: int
    stats: Dict


def _flags(ordered, verify, no_shortcut, no_symmetry) -> int:
    return ((ORDERED if ordered else 0) | (VERIFY if verify else 0) | (NO_SHORTCUT if no_shortcut else 0)
            | (NO_SYMMETRY if no_symmetry else 0))


def count_ex(n: int, variant="skolem", ordered: bool = False, verify: bool = False,
             no_shortcut: bool = False, tuning: Optional[Dict] = None, stream=None,
             progress: Optional[Callable[[int, int], Optional[bool]]] = None,
             no_symmetry: bool = False, workspace=None) -> CountResult:
    """Exact count (reflections counted once unless ``ordered``) with launch
    statistics.  ``workspace``: device memory for the call (a torch tensor of
    at least workspace_bytes() bytes), or None for the library's own."""
    wp, wb = _workspace(workspace)
    flags = _flags(ordered, verify, no_shortcut, no_symmetry)
    out = U128()
    st = Stats()
    t = _tuning(tuning)

    def _cb(_ctx, done, total):
        if progress is None:
            return 0
        return 1 if progress(int(done), int(total)) else 0

    cb = PROGRESS_FN(_cb)
    status = lib().sk_count_ex(n, _variant(variant), flags, ctypes.byref(t) if t else None, wp, wb,
                               _stream_handle(stream), cb, None, ctypes.byref(st), ctypes.byref(out))
    _check(status, f"sk_count_ex(n={n}, variant={variant})")
    return CountResult(out.value(), st.as_dict())


def count_larsen(n: int, variant="skolem", ordered: bool = False, verify: bool = False,
                 no_shortcut: bool = False, tuning: Optional[Dict] = None, stream=None,
                 workspace=None) -> CountResult:
    """Exact count by inclusion-exclusion over the empty positions (the third
    approach of Sec. 2), with launch statistics (sk_count_larsen)."""
    flags = _flags(ordered, verify, no_shortcut, False)
    out = U128()
    st = Stats()
    t = _tuning(tuning)
    wp, wb = _workspace(workspace)
    _check(lib().sk_count_larsen(n, _variant(variant), flags, ctypes.byref(t) if t else None, wp, wb,
                                 _stream_handle(stream), ctypes.byref(st), ctypes.byref(out)),
           f"sk_count_larsen(n={n}, variant={variant})")
    return CountResult(out.value(), st.as_dict())


def count(n: int, variant="skolem", ordered: bool = False, verify: bool = False,
          no_shortcut: bool = False, no_symmetry: bool = False) -> int:
    """Exact number of pairings (Sec. 2).  ``ordered`` counts reflections as distinct."""
    flags = _flags(ordered, verify, no_shortcut, no_symmetry)
    out = U128()
    _check(lib().sk_count(n, _variant(variant), flags, ctypes.byref(out)), f"sk_count(n={n})")
    return out.value()


def count_part(n: int, variant, part: int, parts: int, ordered: bool = False, no_shortcut: bool = False,
               no_symmetry: bool = False, tuning: Optional[Dict] = None, stream=None,
               progress: Optional[Callable[[int, int], Optional[bool]]] = None, workspace=None):
    """Residues of the part-th of `parts` shares of an exact count (sk_count_part):
    (residues, stats)."""
    flags = _flags(ordered, False, no_shortcut, no_symmetry)
    k = describe(n, variant)["primes"]
    out = (ctypes.c_uint64 * k)()
    st = Stats()
    t = _tuning(tuning)

    def _cb(_ctx, done, total):
        if progress is None:
            return 0
        return 1 if progress(int(done), int(total)) else 0

    cb = PROGRESS_FN(_cb)
    wp, wb = _workspace(workspace)
    _check(lib().sk_count_part(n, _variant(variant), flags, part, parts, ctypes.byref(t) if t else None, wp, wb,
                               _stream_handle(stream), cb, None, ctypes.byref(st), out),
           f"sk_count_part(n={n}, part={part}/{parts})")
    return [int(x) for x in out], st.as_dict()


def count_combine(n: int, variant, rows: Sequence[Sequence[int]], ordered: bool = False,
                  no_shortcut: bool = False, no_symmetry: bool = False) -> int:
    """The count from every part's residues (sk_count_combine, host only)."""
    flags = _flags(ordered, False, no_shortcut, no_symmetry)
    flat = [int(x) for row in rows for x in row]
    arr = _u64_array(flat)
    out = U128()
    _check(lib().sk_count_combine(n, _variant(variant), flags, arr, len(rows), ctypes.byref(out)),
           "sk_count_combine")
    return out.value()


def _instances(instances) -> "ctypes.Array":
    arr = (Instance * len(instances))()
    for i, it in enumerate(instances):
        n, v = it[0], it[1]
        fl = it[2] if len(it) > 2 else 0
        arr[i] = Instance(int(n), _variant(v), int(fl))
    return arr


def count_batch(instances, tuning: Optional[Dict] = None, stream=None, workspace=None):
    """Exact counts of several instances [(n, variant[, flags]), ...] in one
    persistent launch; returns (counts, stats).  ``workspace`` as in count_ex."""
    arr = _instances(instances)
    out = (U128 * len(instances))()
    st = Stats()
    t = _tuning(tuning)
    wp, wb = _workspace(workspace)
    _check(lib().sk_count_batch(arr, len(instances), ctypes.byref(t) if t else None, wp, wb,
                                _stream_handle(stream), ctypes.byref(st), out), "sk_count_batch")
    return [o.value() for o in out], st.as_dict()


def count_batch_noalloc(instances, tuning: Optional[Dict] = None, stream=None):
    """count_batch on the library's fixed per-device workspace: the call
    allocates no device memory (sk_count_batch_noalloc)."""
    arr = _instances(instances)
    out = (U128 * len(instances))()
    st = Stats()
    t = _tuning(tuning)
    _check(lib().sk_count_batch_noalloc(arr, len(instances), ctypes.byref(t) if t else None,
                                        _stream_handle(stream), ctypes.byref(st), out), "sk_count_batch_noalloc")
    return [o.value() for o in out], st.as_dict()


def workspace_bytes(instances, tuning: Optional[Dict] = None) -> int:
    """Device workspace bytes count_ex / count_part / count_batch need for these
    instances [(n, variant[, flags]), ...] (sk_workspace_bytes)."""
    arr = _instances(instances)
    t = _tuning(tuning)
    return int(lib().sk_workspace_bytes(arr, len(instances), ctypes.byref(t) if t else None))


def partial_workspace_bytes(n: int, variant, nchunks: int, nprimes: int, tuning: Optional[Dict] = None) -> int:
    """Device workspace bytes partial_chunks needs (sk_partial_workspace_bytes)."""
    t = _tuning(tuning)
    return int(lib().sk_partial_workspace_bytes(n, _variant(variant), nchunks, nprimes,
                                                ctypes.byref(t) if t else None))


def autotune_batch(instances, stream=None):
    """Finds and caches the launch shape of count_batch for this instance set."""
    arr = _instances(instances)
    best = Tuning()
    rate = ctypes.c_double()
    _check(lib().sk_autotune_batch(arr, len(instances), _stream_handle(stream), ctypes.byref(best),
                                   ctypes.byref(rate)), "sk_autotune_batch")
    return {"log2_chunk_terms": best.log2_chunk_terms, "waves_per_launch": best.waves_per_launch,
            "primes_per_item": best.primes_per_item}, rate.value


def _u64_array(values: Sequence[int]):
    arr = (ctypes.c_uint64 * len(values))()
    for i, v in enumerate(values):
        arr[i] = int(v)
    return arr


def sign_sum_residues(n: int, variant, primes: Sequence[int], tuning: Optional[Dict] = None,
                      stream=None) -> List[int]:
    """H mod p for each prime: H = sum over x with x_1 = +1 of (prod x) prod_k f_k(x)."""
    ps = _u64_array(primes)
    out = (ctypes.c_uint64 * len(primes))()
    t = _tuning(tuning)
    _check(lib().sk_sign_sum_residues(n, _variant(variant), ps, len(primes), ctypes.byref(t) if t else None,
                                      _stream_handle(stream), out), "sk_sign_sum_residues")
    return [int(x) for x in out]


def partial_chunks(n: int, variant, log2_chunks: int, chunk_ids: Sequence[int], primes,
                   tuning: Optional[Dict] = None, stream=None, with_stats: bool = False, workspace=None):
    """Per-chunk residues (see the chunk definition in include/skolem.h).
    primes: a list of primes, or an int k for the library's k default primes.
    With with_stats, returns (rows, stats of the call)."""
    ids = _u64_array(chunk_ids)
    if isinstance(primes, int):
        k, ps = primes, None
    else:
        k, ps = len(primes), _u64_array(primes)
    out = (ctypes.c_uint64 * (len(chunk_ids) * k))()
    t = _tuning(tuning)
    wp, wb = _workspace(workspace)
    _check(lib().sk_partial_chunks(n, _variant(variant), log2_chunks, ids, len(chunk_ids), ps, k,
                                   ctypes.byref(t) if t else None, wp, wb, _stream_handle(stream), out),
           "sk_partial_chunks")
    rows = [[int(out[c * k + i]) for i in range(k)] for c in range(len(chunk_ids))]
    if with_stats:
        return rows, last_stats()
    return rows


def last_stats() -> Dict:
    """Totals of this thread's last exact-sum call (sk_last_stats)."""
    st = Stats()
    _check(lib().sk_last_stats(ctypes.byref(st)), "sk_last_stats")
    return st.as_dict()


def max_chunk_bits(n: int, variant) -> int:
    return int(lib().sk_max_chunk_bits(n, _variant(variant)))


def describe(n: int, variant, larsen: bool = False) -> Dict:
    """Variable split and product grouping the library uses for (n, variant):
    of the sign sum, or with larsen of the inclusion-exclusion sum."""
    d = PlanDesc()
    fn = lib().sk_describe_larsen if larsen else lib().sk_describe
    _check(fn(n, _variant(variant), ctypes.byref(d)), "sk_describe")
    out = {name: getattr(d, name) for name, _ in d._fields_ if name != "slot_factor"}
    out["slot_factor"] = [int(x) for x in d.slot_factor[: 4 * d.quads]]
    return out


PROPOSAL_UNIFORM, PROPOSAL_LEARNED = 0, 1


def _learned_params(learned: Optional[Dict]):
    """sk_learned_params from a dict (keys as in the C struct); params, if
    given, is a float32 numpy array that receives the trained network."""
    if learned is None:
        return None, None
    params = learned.get("params")
    ptr = None
    if params is not None:
        if not (isinstance(params, np.ndarray) and params.dtype == np.float32 and params.flags.c_contiguous):
            raise TypeError("learned['params'] must be a contiguous float32 numpy array")
        ptr = params.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    lp = LearnedParams(int(learned.get("hidden1", 0)), int(learned.get("hidden2", 0)),
                       int(learned.get("first_level", 0)), int(learned.get("plain_per_learned", 1)),
                       int(learned.get("train_iterations", 0)), int(learned.get("snapshots", 1)),
                       int(learned.get("train_steps", 0)), int(learned.get("minibatch", 256)),
                       float(learned.get("lr", 1e-3)), int(learned.get("init_seed", 0)), ptr)
    return lp, params


def _pt_params(betas, ladders, iterations, seed, proposal, ordered, segment, burn_in=0, learned=None):
    arr = (ctypes.c_double * len(betas))(*[float(x) for x in betas])
    lp, params = _learned_params(learned)
    p = PtParams(len(betas), arr, int(ladders), int(iterations), int(seed), int(proposal),
                 ORDERED if ordered else 0, int(segment), int(burn_in),
                 ctypes.pointer(lp) if lp is not None else None)
    return p, (arr, lp, params)


def pt_bins(n: int, variant) -> int:
    return int(lib().sk_pt_bins(n, _variant(variant)))


def pt_run(n: int, variant, betas: Sequence[float], ladders: int, iterations: int, seed: int,
           proposal: int = PROPOSAL_UNIFORM, segment: int = 0, stream=None, burn_in: int = 0,
           learned: Optional[Dict] = None) -> Dict:
    """Runs the tempering ladders (Sec. 3) and returns raw chain statistics:
    hist[ladder][level][E], move/exchange acceptance counts, final states."""
    M = len(betas)
    H = pt_bins(n, variant)
    if H < 0:
        raise SkolemError(-1, "sk_pt_bins")
    p, keep = _pt_params(betas, ladders, iterations, seed, proposal, False, segment, burn_in, learned)
    hist = (ctypes.c_uint64 * (ladders * M * H))()
    ma = (ctypes.c_uint64 * (ladders * M))()
    sw = (ctypes.c_uint64 * (ladders * M))()
    state = (ctypes.c_uint8 * (ladders * M * n))()
    energy = (ctypes.c_int32 * (ladders * M))()
    _check(lib().sk_pt_run(n, _variant(variant), ctypes.byref(p), _stream_handle(stream), hist, ma, sw, state,
                           energy), "sk_pt_run")
    return {"hist": [[[int(hist[(l * M + j) * H + e]) for e in range(H)] for j in range(M)] for l in range(ladders)],
            "move_accept": [[int(ma[l * M + j]) for j in range(M)] for l in range(ladders)],
            "swap_accept": [[int(sw[l * M + j]) for j in range(M)] for l in range(ladders)],
            "state": [[[int(state[(l * M + j) * n + k]) for k in range(n)] for j in range(M)] for l in range(ladders)],
            "energy": [[int(energy[l * M + j]) for j in range(M)] for l in range(ladders)]}


def pt_tune_ladder(n: int, variant, beta_max: float, target: float = 0.5, max_levels: int = 64, ladders: int = 256,
                   pilot_iterations: int = 1 << 14, seed: int = 1, stream=None):
    """Inverse temperatures from 0 to beta_max with every neighbouring
    exchange accepted at least `target` of the time (Sec. 3): (betas, the last
    pilot's exchange acceptances)."""
    b = (ctypes.c_double * max_levels)()
    acc = (ctypes.c_double * max_levels)()
    m = ctypes.c_int()
    _check(lib().sk_pt_tune_ladder(n, _variant(variant), beta_max, target, max_levels, ladders, pilot_iterations, seed,
                                   _stream_handle(stream), b, ctypes.byref(m), acc), "sk_pt_tune_ladder")
    return [b[j] for j in range(m.value)], [acc[j] for j in range(m.value - 1)]


def approx(n: int, variant, betas: Sequence[float], ladders: int, iterations: int, seed: int,
           proposal: int = PROPOSAL_UNIFORM, ordered: bool = False, segment: int = 0, stream=None,
           burn_in: int = 0, learned: Optional[Dict] = None):
    """Approximate count by parallel tempering: (estimate, standard error, stats).
    With proposal=PROPOSAL_LEARNED, ``learned`` holds the sk_learned_params
    fields (see include/skolem.h)."""
    p, keep = _pt_params(betas, ladders, iterations, seed, proposal, ordered, segment, burn_in, learned)
    est = ctypes.c_double()
    se = ctypes.c_double()
    st = PtStats()
    _check(lib().sk_approx(n, _variant(variant), ctypes.byref(p), _stream_handle(stream), ctypes.byref(est),
                           ctypes.byref(se), ctypes.byref(st)), "sk_approx")
    return est.value, se.value, st.as_dict()


# ---------------------------------------------------------------- network


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _states(states, n: int) -> np.ndarray:
    s = np.ascontiguousarray(states, dtype=np.uint8)
    if s.ndim != 2 or s.shape[1] != n:
        raise ValueError(f"states must be (batch, {n})")
    return s


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def mlp_param_count(n: int, variant, h1: int = 0, h2: int = 0) -> int:
    return int(lib().sk_mlp_param_count(n, _variant(variant), h1, h2))


def mlp_init(n: int, variant, h1: int = 0, h2: int = 0, seed: int = 0, scale: float = 1.0) -> np.ndarray:
    P = np.zeros(mlp_param_count(n, variant, h1, h2), dtype=np.float32)
    _check(lib().sk_mlp_init(n, _variant(variant), h1, h2, seed, scale, _ptr(P, ctypes.c_float)), "sk_mlp_init")
    return P


def mlp_forward(n: int, variant, params, states, betas, h1: int = 0, h2: int = 0, stream=None) -> np.ndarray:
    """Logits (batch, n * T) of the proposal network on the GPU."""
    P, S = _f32(params), _states(states, n)
    b = np.ascontiguousarray(betas, dtype=np.float64)
    B = S.shape[0]
    T = pt_bins(n, variant) - 1
    out = np.zeros((B, n * T), dtype=np.float32)
    _check(lib().sk_mlp_forward(n, _variant(variant), h1, h2, _ptr(P, ctypes.c_float), _ptr(S, ctypes.c_uint8),
                                _ptr(b, ctypes.c_double), B, _stream_handle(stream), _ptr(out, ctypes.c_float)),
           "sk_mlp_forward")
    return out


def mlp_loss_grad(n: int, variant, params, states, betas, h1: int = 0, h2: int = 0, stream=None):
    """(mean cross-entropy, gradient in parameter layout) on the GPU."""
    P, S = _f32(params), _states(states, n)
    b = np.ascontiguousarray(betas, dtype=np.float64)
    g = np.zeros_like(P)
    loss = ctypes.c_double()
    _check(lib().sk_mlp_loss_grad(n, _variant(variant), h1, h2, _ptr(P, ctypes.c_float), _ptr(S, ctypes.c_uint8),
                                  _ptr(b, ctypes.c_double), S.shape[0], _stream_handle(stream), ctypes.byref(loss),
                                  _ptr(g, ctypes.c_float)), "sk_mlp_loss_grad")
    return loss.value, g


def mlp_train(n: int, variant, params, states, betas, steps: int, minibatch: int, lr: float, h1: int = 0,
              h2: int = 0, stream=None):
    """Adam on the GPU; returns (trained params, last minibatch loss)."""
    P, S = _f32(params).copy(), _states(states, n)
    b = np.ascontiguousarray(betas, dtype=np.float64)
    loss = ctypes.c_double()
    _check(lib().sk_mlp_train(n, _variant(variant), h1, h2, _ptr(P, ctypes.c_float), _ptr(S, ctypes.c_uint8),
                              _ptr(b, ctypes.c_double), S.shape[0], steps, minibatch, lr, _stream_handle(stream),
                              ctypes.byref(loss)), "sk_mlp_train")
    return P, loss.value


def mlp_mh_step(n: int, variant, params, states, betas, w_pick, w_acc, h1: int = 0, h2: int = 0,
                stream=None) -> Dict:
    """One learned Metropolis-Hastings move per state on the GPU."""
    P, S = _f32(params), _states(states, n)
    B = S.shape[0]
    b = np.ascontiguousarray(betas, dtype=np.float64)
    wp = np.ascontiguousarray(w_pick, dtype=np.uint32)
    wa = np.ascontiguousarray(w_acc, dtype=np.uint32)
    if b.shape != (B,) or wp.shape != (B,) or wa.shape != (B,):
        raise ValueError("betas, w_pick and w_acc need one entry per state")
    out = np.zeros_like(S)
    acc = np.zeros(B, dtype=np.uint8)
    prop = np.zeros_like(S)
    lf = np.zeros(B, dtype=np.float32)
    lr = np.zeros(B, dtype=np.float32)
    _check(lib().sk_mlp_mh_step(n, _variant(variant), h1, h2, _ptr(P, ctypes.c_float), _ptr(S, ctypes.c_uint8),
                                _ptr(b, ctypes.c_double), _ptr(wp, ctypes.c_uint32), _ptr(wa, ctypes.c_uint32), B,
                                _stream_handle(stream), _ptr(out, ctypes.c_uint8), _ptr(acc, ctypes.c_uint8),
                                _ptr(prop, ctypes.c_uint8), _ptr(lf, ctypes.c_float), _ptr(lr, ctypes.c_float)),
           "sk_mlp_mh_step")
    return {"states": out, "accepted": acc.astype(bool), "proposed": prop, "logq_forward": lf, "logq_reverse": lr}


def kernel_name(kv: int) -> str:
    return lib().sk_kernel_name(kv).decode()


def last_stats_dict(st: Stats) -> Dict:
    return st.as_dict()


__all__ = ["pt_tune_ladder", "count", "count_ex", "count_larsen", "count_batch", "count_batch_noalloc", "workspace_bytes", "partial_workspace_bytes", "autotune_batch", "pt_run", "approx", "pt_bins", "sign_sum_residues",
           "partial_chunks", "last_stats", "count_part", "count_combine", "max_chunk_bits", "set_device", "mlp_param_count", "mlp_init", "mlp_forward",
           "mlp_loss_grad", "mlp_train", "mlp_mh_step", "PROPOSAL_UNIFORM", "PROPOSAL_LEARNED",
           "SkolemError", "SKOLEM", "LANGFORD", "HOOKED", "lib", "EXPORTED"]
