"""Python binding of libg3 (ctypes): argument marshalling only.

Every function mirrors one entry point of ``include/g3.h`` (same name without
the ``g3_`` prefix).  Device buffers are torch tensors on the current HIP
device, passed as raw pointers with torch's current stream; all the work runs
in the HIP library.  If ``libg3.so`` has not been built this module raises on
first use -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libg3.so")

HALF, FULL = 0, 1
STAGE_TRIPLET, STAGE_NEIGHBOURS, STAGE_CELLS = 0, 1, 2
OK, EINVAL, EDOMAIN, ENOMEM, EDEVICE, EBUSY = range(6)
MAX_NBINS = 160
MAX_RMAX = 46340.0


class G3Error(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = int(status)
        msg = _strerror(self.status)
        super().__init__(f"{what}: {msg} (status {self.status})" if what else msg)


class System(C.Structure):
    _fields_ = [("frames", C.c_void_p), ("n_frames", C.c_int32), ("n_atoms", C.c_int32),
                ("box", C.c_int32 * 3), ("rmax", C.c_double), ("nbins", C.c_int32),
                ("layout", C.c_int32), ("hist", C.c_void_p),
                ("pair_hist", C.c_void_p), ("nbins_third", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("lds_hist_bins", C.c_int32),
                ("centres_per_item", C.c_int32), ("wg_per_cu", C.c_int32),
                ("per_centre", C.c_int32), ("slot_limit", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libg3.so (raises if it is missing: the product has no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1708_08619_amd.build` "
                           "(or __graft_entry__.build()) first")
    # torch ships its own HIP runtime.  Loading it first makes libg3's
    # libamdhip64.so.7 / libhsa-runtime64.so.1 resolve (by soname) to the
    # copies torch already loaded, so the process has exactly one runtime and
    # torch's device pointers and streams are valid inside libg3.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "g3_plan_create": ([C.POINTER(P), P], I32),
        "g3_plan_destroy": ([P], None),
        "g3_accumulate": ([P, P, I32, I32, P, D, I32, I32, P, P], I32),
        "g3_accumulate_batch": ([P, P, I32], I32),
        "g3_accumulate_system": ([P, P], I32),
        "g3_accumulate_noalloc": ([P, P], I32),
        "g3_hist_len3": ([I32, I32, I32], C.c_size_t),
        "g3_normalize3": ([P, I32, I32, I32, D, I64, I32, P, P], I32),
        "g3_sync": ([P], I32),
        "g3_query": ([P], I32),
        "g3_last_ticket": ([P, C.POINTER(C.c_uint64)], I32),
        "g3_ticket_query": ([P, C.c_uint64, C.POINTER(I32)], I32),
        "g3_hist_len": ([I32, I32], C.c_size_t),
        "g3_check_args": ([I32, P, D, I32, I32], I32),
        "g3_thresholds": ([D, I32, P], I32),
        "g3_normalize": ([P, I32, I32, D, I64, I32, P, P], I32),
        "g3_ideal_volume": ([I32, D, P], I32),
        "g3_normalize_pairs": ([P, I32, D, I64, I32, P, P], I32),
        "g3_superposition": ([P, I32, I32, P, P], I32),
        "g3_isosceles": ([P, I32, I32, I32, P, P], I32),
        "g3_set_tuning": ([P, P], I32),
        "g3_get_tuning": ([P, P], I32),
        "g3_autotune": ([P, P, I32, P], I32),
        "g3_kernel_time": ([P, C.POINTER(D), C.POINTER(I64)], I32),
        "g3_kernel_time_reset": ([P, I32], I32),
        "g3_stage_time": ([P, I32, C.POINTER(D), C.POINTER(I64)], I32),
        "g3_build_counts": ([P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)], I32),
        "g3_candidates": ([P, C.POINTER(C.c_uint64)], I32),
        "g3_strerror": ([I32], C.c_char_p),
        "g3_lds_rate": ([I32, I32, C.POINTER(D)], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _strerror(status: int) -> str:
    try:
        return lib().g3_strerror(int(status)).decode()
    except Exception:  # library missing while formatting an error
        return f"status {status}"


def _check(status: int, what: str):
    if status != OK:
        raise G3Error(status, what)


def _box(box) -> C.Array:
    b = [int(x) for x in box]
    if len(b) != 3:
        raise ValueError("box needs 3 edges")
    return (C.c_int32 * 3)(*b)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------------ host helpers
def hist_len(nbins: int, layout: int, nbins_third: int | None = None) -> int:
    """Bins of the histogram; nbins_third third-side bins (default nbins)."""
    return int(lib().g3_hist_len3(int(nbins), int(nbins_third or nbins), int(layout)))


def check_args(n_atoms: int, box, rmax: float, nbins: int, layout: int) -> int:
    return int(lib().g3_check_args(int(n_atoms), _box(box), float(rmax), int(nbins), int(layout)))


def thresholds(rmax: float, nbins: int) -> np.ndarray:
    thr = np.zeros(int(nbins) + 1, dtype=np.uint32)
    _check(lib().g3_thresholds(float(rmax), int(nbins), _np_ptr(thr)), "g3_thresholds")
    return thr


def ideal_volume(nbins: int, rmax: float) -> np.ndarray:
    W = np.zeros(int(nbins) ** 3, dtype=np.float64)
    _check(lib().g3_ideal_volume(int(nbins), float(rmax), _np_ptr(W)), "g3_ideal_volume")
    return W.reshape((int(nbins),) * 3)


def normalize(hist: np.ndarray, layout: int, nbins: int, rmax: float, n_frames: int,
              n_atoms: int, box, nbins_third: int | None = None) -> np.ndarray:
    nc = int(nbins_third or nbins)
    h = np.ascontiguousarray(hist, dtype=np.uint64).reshape(-1)
    if h.shape[0] != hist_len(nbins, layout, nc):
        raise ValueError("histogram length does not match nbins/layout")
    out = np.zeros(h.shape[0], dtype=np.float64)
    _check(lib().g3_normalize3(_np_ptr(h), int(layout), int(nbins), nc, float(rmax),
                               int(n_frames), int(n_atoms), _box(box), _np_ptr(out)),
           "g3_normalize3")
    return out


def normalize_pairs(pair_hist: np.ndarray, nbins: int, rmax: float, n_frames: int,
                    n_atoms: int, box) -> np.ndarray:
    """g2 from the pair histogram (ordered pairs), fp64 on the host."""
    h = np.ascontiguousarray(pair_hist, dtype=np.uint64).reshape(-1)
    if h.shape[0] != int(nbins):
        raise ValueError("pair histogram length does not match nbins")
    out = np.zeros(h.shape[0], dtype=np.float64)
    _check(lib().g3_normalize_pairs(_np_ptr(h), int(nbins), float(rmax), int(n_frames),
                                    int(n_atoms), _box(box), _np_ptr(out)), "g3_normalize_pairs")
    return out


def superposition(g3: np.ndarray, layout: int, nbins: int, g2: np.ndarray) -> np.ndarray:
    """g3 / (g2 g2 g2) bin by bin (0 where the product is 0), host fp64."""
    x = np.ascontiguousarray(g3, dtype=np.float64).reshape(-1)
    y = np.ascontiguousarray(g2, dtype=np.float64).reshape(-1)
    if x.shape[0] != hist_len(nbins, layout) or y.shape[0] != int(nbins):
        raise ValueError("array lengths do not match nbins/layout")
    out = np.zeros_like(x)
    _check(lib().g3_superposition(_np_ptr(x), int(layout), int(nbins), _np_ptr(y), _np_ptr(out)),
           "g3_superposition")
    return out


def isosceles(g3: np.ndarray, layout: int, nbins: int, a: int):
    """(theta, g3(a, a, c)) for c = 0..nbins-1; theta -1 where no triangle."""
    x = np.ascontiguousarray(g3, dtype=np.float64).reshape(-1)
    if x.shape[0] != hist_len(nbins, layout):
        raise ValueError("array length does not match nbins/layout")
    th = np.zeros(int(nbins))
    val = np.zeros(int(nbins))
    _check(lib().g3_isosceles(_np_ptr(x), int(layout), int(nbins), int(a), _np_ptr(th),
                              _np_ptr(val)), "g3_isosceles")
    return th, val


def strerror(status: int) -> str:
    return _strerror(status)


LDS_ADD_LANE, LDS_ADD_RANDOM, LDS_READ_RANDOM, LDS_READ_ADD = range(4)


def lds_rate(pattern: int, words: int) -> float:
    """Measured LDS lane operations per second of the current device
    (g3_lds_rate)."""
    v = C.c_double()
    _check(lib().g3_lds_rate(int(pattern), int(words), C.byref(v)), "g3_lds_rate")
    return float(v.value)


# ------------------------------------------------------------------ device plan
def _stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_ptr(t, dtype_name: str, what: str) -> int:
    import torch
    want = {"int32": torch.int32, "uint64": torch.uint64}[dtype_name]
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a torch tensor on the GPU")
    if t.dtype != want or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous {dtype_name} tensor")
    return int(t.data_ptr())


class Plan:
    """Owns a ``g3_plan`` bound to one HIP stream (torch's current stream by
    default)."""

    def __init__(self, stream=None):
        self._h = C.c_void_p()
        self.stream = stream
        _check(lib().g3_plan_create(C.byref(self._h), C.c_void_p(_stream_handle(stream))),
               "g3_plan_create")

    def close(self):
        if self._h:
            lib().g3_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- g3_accumulate: the plain per-frame form
    def accumulate(self, frames, box, rmax: float, nbins: int, layout: int, hist,
                   pair_hist=None, nbins_third: int | None = None):
        arr = self._systems([dict(frames=frames, box=box, rmax=rmax, nbins=nbins, layout=layout,
                                  hist=hist, pair_hist=pair_hist, nbins_third=nbins_third)])
        _check(lib().g3_accumulate_system(self._h, arr), "g3_accumulate_system")

    # -- g3_accumulate_noalloc: the plain form on the library's static scratch
    def accumulate_noalloc(self, frames, box, rmax: float, nbins: int, layout: int, hist,
                           pair_hist=None, nbins_third: int | None = None):
        arr = self._systems([dict(frames=frames, box=box, rmax=rmax, nbins=nbins, layout=layout,
                                  hist=hist, pair_hist=pair_hist, nbins_third=nbins_third)])
        _check(lib().g3_accumulate_noalloc(self._h, arr), "g3_accumulate_noalloc")

    @staticmethod
    def _systems(systems: Sequence[dict]):
        arr = (System * len(systems))()
        for i, s in enumerate(systems):
            fr, h = s["frames"], s["hist"]
            F, three, N = (int(x) for x in fr.shape)
            if three != 3:
                raise ValueError("frames must be [n_frames, 3, n_atoms]")
            nc = int(s.get("nbins_third") or 0)
            if h.numel() != hist_len(s["nbins"], s["layout"], nc or None):
                raise ValueError("hist has the wrong length")
            arr[i].frames = _dev_ptr(fr, "int32", "frames")
            arr[i].n_frames = F
            arr[i].n_atoms = N
            arr[i].box = _box(s["box"])
            arr[i].rmax = float(s["rmax"])
            arr[i].nbins = int(s["nbins"])
            arr[i].layout = int(s["layout"])
            arr[i].hist = _dev_ptr(h, "uint64", "hist")
            arr[i].pair_hist = _pair_ptr(s.get("pair_hist"), s["nbins"])
            arr[i].nbins_third = nc
        return arr

    # -- g3_accumulate_batch: one graph launch for many systems
    def accumulate_batch(self, systems: Sequence[dict]):
        arr = self._systems(systems)
        _check(lib().g3_accumulate_batch(self._h, arr, len(systems)), "g3_accumulate_batch")

    # -- g3_autotune: pick (and keep) the fastest tuning for these systems
    def autotune(self, systems: Sequence[dict]) -> dict:
        arr = self._systems(systems)
        t = Tuning()
        _check(lib().g3_autotune(self._h, arr, len(systems), C.byref(t)), "g3_autotune")
        return t.as_dict()

    def sync(self):
        _check(lib().g3_sync(self._h), "g3_sync")

    def query(self) -> bool:
        """True if all queued work has finished (non-blocking)."""
        st = int(lib().g3_query(self._h))
        if st == EBUSY:
            return False
        _check(st, "g3_query")
        return True

    def last_ticket(self) -> int:
        """Ticket of the latest accumulate call (g3_last_ticket)."""
        t = C.c_uint64()
        _check(lib().g3_last_ticket(self._h, C.byref(t)), "g3_last_ticket")
        return int(t.value)

    def ticket_query(self, ticket: int):
        """None while the call runs; then True if its histograms are final,
        False if g3_sync must run first (g3_ticket_query)."""
        fin = C.c_int32()
        st = int(lib().g3_ticket_query(self._h, C.c_uint64(int(ticket)), C.byref(fin)))
        if st == EBUSY:
            return None
        _check(st, "g3_ticket_query")
        return bool(fin.value)

    def sync_status(self) -> int:
        return int(lib().g3_sync(self._h))

    def set_tuning(self, **kw):
        t = Tuning(**{k: int(v) for k, v in kw.items()})
        _check(lib().g3_set_tuning(self._h, C.byref(t)), "g3_set_tuning")

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(lib().g3_get_tuning(self._h, C.byref(t)), "g3_get_tuning")
        return t.as_dict()

    def kernel_time_reset(self, enable: bool = True):
        _check(lib().g3_kernel_time_reset(self._h, int(bool(enable))), "g3_kernel_time_reset")

    def candidates(self) -> int:
        n = C.c_uint64()
        _check(lib().g3_candidates(self._h, C.byref(n)), "g3_candidates")
        return int(n.value)

    def stage_time(self, stage: int) -> tuple[float, int]:
        """(ms per launch, launches) of one stage since the last reset."""
        ms, n = C.c_double(), C.c_int64()
        _check(lib().g3_stage_time(self._h, int(stage), C.byref(ms), C.byref(n)), "g3_stage_time")
        return float(ms.value), int(n.value)

    def build_counts(self) -> tuple[int, int]:
        """(candidates tested, neighbours accepted) by the neighbour builds."""
        a, b = C.c_uint64(), C.c_uint64()
        _check(lib().g3_build_counts(self._h, C.byref(a), C.byref(b)), "g3_build_counts")
        return int(a.value), int(b.value)

    def kernel_time(self) -> tuple[float, int]:
        ms, n = C.c_double(), C.c_int64()
        _check(lib().g3_kernel_time(self._h, C.byref(ms), C.byref(n)), "g3_kernel_time")
        return float(ms.value), int(n.value)


def _pair_ptr(pair_hist, nbins: int):
    if pair_hist is None:
        return None
    if pair_hist.numel() != int(nbins):
        raise ValueError("pair_hist must hold nbins entries")
    return _dev_ptr(pair_hist, "uint64", "pair_hist")


def new_pair_hist(nbins: int, device="cuda"):
    import torch
    return torch.zeros(int(nbins), dtype=torch.uint64, device=device)


def new_hist(nbins: int, layout: int, device="cuda", nbins_third: int | None = None):
    import torch
    return torch.zeros(hist_len(nbins, layout, nbins_third), dtype=torch.uint64, device=device)
