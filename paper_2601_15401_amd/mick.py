"""Python binding of libmick (ctypes).  Argument marshalling only: every step
of the multiply runs in the library's HIP kernels.  PyTorch provides device
memory (uint32 data held in int32 tensors) and the current HIP stream.

The library must be built (``python -m paper_2601_15401_amd.build``); when it
is missing every call raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np
import torch  # loads the HIP runtime that libmick then shares

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmick.so")

OP_RELIN, OP_RESCALE, OP_MUL_RELIN_RESCALE = 1, 2, 3

_c_u32p = ctypes.POINTER(ctypes.c_uint32)
_c_i64p = ctypes.POINTER(ctypes.c_int64)
_c_dblp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p

# name: (restype, argtypes)
_SIGS = {
    "mick_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "mick_last_error": (ctypes.c_char_p, []),
    "mick_params_create": (ctypes.c_int, [ctypes.c_int] * 4 + [ctypes.POINTER(_vp)]),
    "mick_params_destroy": (None, [_vp]),
    "mick_params_moduli": (ctypes.c_int, [_vp, _c_u32p, _c_u32p]),
    "mick_params_shape": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int)]),
    "mick_keygen": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "mick_keys_destroy": (None, [_vp]),
    "mick_keys_kmax": (ctypes.c_int, [_vp]),
    "mick_keys_export": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp]),
    "mick_encode": (ctypes.c_int, [_vp, _c_dblp, _c_dblp, ctypes.c_size_t, ctypes.c_double, _c_i64p]),
    "mick_decode": (ctypes.c_int, [_vp, _c_i64p, ctypes.c_double, _c_dblp, _c_dblp, ctypes.c_size_t]),
    "mick_encrypt": (ctypes.c_int, [_vp, _vp, _c_i64p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, _vp, _vp]),
    "mick_decrypt_residues": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _c_u32p, _vp]),
    "mick_decrypt": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _c_i64p, _vp]),
    "mick_workspace_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "mick_mul_k": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp, _vp]),
    "mick_relin_k": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_size_t, _vp]),
    "mick_rescale_multi": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_size_t, _vp]),
    "mick_mul_relin_rescale": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp, _vp,
                                              ctypes.c_size_t, _vp]),
    "mick_mul_relin_rescale_noalloc": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int,
                                                      _vp, _vp]),
    "mick_batch_workspace_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "mick_mul_relin_rescale_batch": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp,
                                                    _vp, ctypes.c_size_t, _vp]),
    "mick_ntt": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "mick_bconv": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _vp]),
    "mick_jobs_workspace_bytes": (ctypes.c_size_t, [_vp, _vp, ctypes.c_int]),
    "mick_mul_relin_rescale_jobs": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp, ctypes.c_size_t, _vp]),
    "mick_jobs_plan": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp, ctypes.c_size_t, _vp,
                                      ctypes.POINTER(_vp)]),
    "mick_plan_execute": (ctypes.c_int, [_vp, _vp]),
    "mick_plan_destroy": (None, [_vp]),
    "mick_tree_plan": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "mick_tree_shape": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "mick_tree_workspace_bytes": (ctypes.c_size_t, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int]),
    "mick_mul_tree": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                     ctypes.c_int, _vp, _vp, ctypes.c_size_t, _vp]),
    "mick_queue_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_size_t,
                                         ctypes.POINTER(_vp)]),
    "mick_queue_job_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "mick_queue_push": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "mick_queue_run": (ctypes.c_int, [_vp, _vp]),
    "mick_queue_poll": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]),
    "mick_queue_drain": (ctypes.c_int, [_vp, _vp]),
    "mick_queue_info": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_size_t)]),
    "mick_queue_cancel": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "mick_queue_destroy": (None, [_vp]),
    "mick_output_scale": (ctypes.c_int, [_vp, _c_dblp, ctypes.c_int, ctypes.c_int, _c_dblp]),
    "mick_autotune": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "mick_params_set_schedule": (ctypes.c_int, [_vp, ctypes.c_int]),
    "mick_params_schedule": (ctypes.c_int, [_vp]),
    "mick_params_set_tensor_method": (ctypes.c_int, [_vp, ctypes.c_int]),
    "mick_params_set_modup_targets": (ctypes.c_int, [_vp, ctypes.c_int]),
    "mick_params_modup_targets": (ctypes.c_int, [_vp]),
    "mick_autotune_report": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _c_dblp]),
    "mick_params_tensor_method": (ctypes.c_int, [_vp]),
    "mick_set_allocator": (ctypes.c_int, [_vp, _vp, _vp]),
    "mick_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "mick_profile_select": (ctypes.c_int, [ctypes.c_char_p]),
    "mick_profile_collect": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]),
}

_lib = None


class Job(ctypes.Structure):
    """mick_job: one multiply of a heterogeneous batch."""
    _fields_ = [("k", ctypes.c_int), ("level", ctypes.c_int), ("cts", ctypes.c_void_p * 12),
                ("out", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class QJob(ctypes.Structure):
    """mick_qjob: one multiply pushed to a queue."""
    _fields_ = [("id", ctypes.c_uint64), ("set", ctypes.c_int), ("k", ctypes.c_int), ("level", ctypes.c_int),
                ("cts", ctypes.c_void_p * 12), ("out", ctypes.c_void_p), ("status", ctypes.c_void_p)]

OK, E_ARG, E_LEVEL, E_KEY, E_NOMEM, E_HIP, E_RANGE, E_WS, E_BUSY, E_CANCELLED = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
PENDING = 1


class MickError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        lib = load()
        msg = "%s: %s (%s)" % (where, lib.mick_strerror(status).decode(), lib.mick_last_error().decode())
        super().__init__(msg)


def load():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmick.so is not built (run python -m paper_2601_15401_amd.build)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(status: int, where: str):
    if status != 0:
        raise MickError(status, where)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor, n: int = 0, what: str = "buffer"):
    """Device address of a contiguous int32 CUDA tensor.  n > 0: the number of
    words the library reads or writes there (the C ABI takes bare pointers, so
    a buffer of another size is refused here rather than overrun on the GPU).
    n <= 0 leaves the size to the library's own argument checks, which reject
    such shapes before touching memory."""
    if not t.is_cuda or not t.is_contiguous() or t.dtype != torch.int32:
        raise ValueError("%s: expected a contiguous int32 CUDA tensor" % what)
    if n > 0 and t.numel() != n:
        raise ValueError("%s: expected %d int32 words, got %d" % (what, n, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


def _dev_empty(*shape):
    return torch.empty(*shape, dtype=torch.int32, device="cuda")


def to_numpy_u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def from_numpy_u32(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


class Params:
    def __init__(self, log_n: int, L: int, K: int, dnum: int):
        lib = load()
        h = _vp()
        _check(lib.mick_params_create(log_n, L, K, dnum, ctypes.byref(h)), "mick_params_create")
        self._h = h
        self.log_n, self.L, self.K, self.dnum = log_n, L, K, dnum
        self.N = 1 << log_n
        q = (ctypes.c_uint32 * L)()
        p = (ctypes.c_uint32 * K)()
        _check(lib.mick_params_moduli(h, q, p), "mick_params_moduli")
        self.q, self.p = list(q), list(p)
        shape = (ctypes.c_int * 5)()
        _check(lib.mick_params_shape(h, shape), "mick_params_shape")
        self.alpha = shape[4]

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mick_params_destroy(self._h)
            self._h = None

    def workspace_bytes(self, op: int, k: int, level: int) -> int:
        return load().mick_workspace_bytes(self._h, op, k, level)


class Keys:
    def __init__(self, prm: Params, seed: int, k_max: int):
        h = _vp()
        _check(load().mick_keygen(prm.handle, seed, k_max, _stream(), ctypes.byref(h)), "mick_keygen")
        self._h, self.prm, self.k_max, self.seed = h, prm, k_max, seed

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            torch.cuda.synchronize()
            _lib.mick_keys_destroy(self._h)
            self._h = None

    def export_secret(self) -> np.ndarray:
        out = np.empty(self.prm.N, dtype=np.int64)
        _check(load().mick_keys_export(self._h, 0, 0, 0, out.ctypes.data_as(_vp), _stream()), "export")
        return out

    def export_pk(self) -> np.ndarray:
        out = np.empty((2, self.prm.L, self.prm.N), dtype=np.uint32)
        _check(load().mick_keys_export(self._h, 1, 0, 0, out.ctypes.data_as(_vp), _stream()), "export")
        return out

    def export_evk(self, t: int, b: int) -> np.ndarray:
        out = np.empty((2, self.prm.L + self.prm.K, self.prm.N), dtype=np.uint32)
        _check(load().mick_keys_export(self._h, 2, t, b, out.ctypes.data_as(_vp), _stream()), "export")
        return out


def encode(prm: Params, re: np.ndarray, im: np.ndarray, scale: float) -> np.ndarray:
    re = np.ascontiguousarray(re, dtype=np.float64)
    im = np.ascontiguousarray(im, dtype=np.float64)
    out = np.empty(prm.N, dtype=np.int64)
    _check(load().mick_encode(prm.handle, re.ctypes.data_as(_c_dblp), im.ctypes.data_as(_c_dblp), re.size, scale,
                              out.ctypes.data_as(_c_i64p)), "mick_encode")
    return out


def decode(prm: Params, m: np.ndarray, scale: float):
    m = np.ascontiguousarray(m, dtype=np.int64)
    re = np.empty(prm.N // 2)
    im = np.empty(prm.N // 2)
    _check(load().mick_decode(prm.handle, m.ctypes.data_as(_c_i64p), scale, re.ctypes.data_as(_c_dblp),
                              im.ctypes.data_as(_c_dblp), re.size), "mick_decode")
    return re, im


def encrypt(prm: Params, keys: Keys, m: np.ndarray, level: int, seed: int, ct_id: int, out=None) -> torch.Tensor:
    m = np.ascontiguousarray(m, dtype=np.int64)
    if out is None:
        out = _dev_empty(2, level, prm.N)
    _check(load().mick_encrypt(prm.handle, keys.handle, m.ctypes.data_as(_c_i64p), level, seed, ct_id, _ptr(out, 2 * level * prm.N, "out"),
                               _stream()), "mick_encrypt")
    return out


def decrypt_residues(prm: Params, keys: Keys, ct: torch.Tensor, level: int) -> np.ndarray:
    out = np.empty((level, prm.N), dtype=np.uint32)
    _check(load().mick_decrypt_residues(prm.handle, keys.handle, _ptr(ct, 2 * level * prm.N, "ct"), level, out.ctypes.data_as(_c_u32p),
                                        _stream()), "mick_decrypt_residues")
    return out


def decrypt(prm: Params, keys: Keys, ct: torch.Tensor, level: int) -> np.ndarray:
    out = np.empty(prm.N, dtype=np.int64)
    _check(load().mick_decrypt(prm.handle, keys.handle, _ptr(ct, 2 * level * prm.N, "ct"), level, out.ctypes.data_as(_c_i64p), _stream()),
           "mick_decrypt")
    return out


def workspace(prm: Params, op: int, k: int, level: int) -> torch.Tensor:
    nbytes = prm.workspace_bytes(op, k, level)
    if nbytes == 0:
        raise ValueError("invalid (op, k, level)")
    return _dev_empty(nbytes // 4)


def mul_k(prm: Params, cts: Sequence[torch.Tensor], level: int, out=None) -> torch.Tensor:
    k = len(cts)
    if out is None:
        out = _dev_empty(k + 1, level, prm.N)
    arr = (_vp * k)(*[_ptr(c, 2 * level * prm.N, "ct").value for c in cts])
    _check(load().mick_mul_k(prm.handle, arr, k, level, _ptr(out, (k + 1) * level * prm.N, "out"), _stream()),
           "mick_mul_k")
    return out


def relin_k(prm: Params, keys: Keys, d: torch.Tensor, k: int, level: int, out=None, ws=None) -> torch.Tensor:
    if out is None:
        out = _dev_empty(2, level, prm.N)
    if ws is None:
        ws = workspace(prm, OP_RELIN, k, level)
    _check(load().mick_relin_k(prm.handle, keys.handle, _ptr(d, (k + 1) * level * prm.N, "d"), k, level,
                               _ptr(out, 2 * level * prm.N, "out"), _ptr(ws), ws.numel() * 4,
                               _stream()), "mick_relin_k")
    return out


def rescale_multi(prm: Params, ct: torch.Tensor, level: int, mu: int, out=None, ws=None) -> torch.Tensor:
    if out is None:
        out = _dev_empty(2, level - mu, prm.N)
    if ws is None:
        ws = workspace(prm, OP_RESCALE, mu, level)
    _check(load().mick_rescale_multi(prm.handle, _ptr(ct, 2 * level * prm.N, "ct"), level, mu,
                                     _ptr(out, 2 * (level - mu) * prm.N, "out"), _ptr(ws), ws.numel() * 4,
                                     _stream()), "mick_rescale_multi")
    return out


def mul_relin_rescale(prm: Params, keys: Keys, cts: Sequence[torch.Tensor], level: int, out=None,
                      ws=None) -> torch.Tensor:
    k = len(cts)
    if out is None:
        out = _dev_empty(2, level - k + 1, prm.N)
    if ws is None:
        ws = workspace(prm, OP_MUL_RELIN_RESCALE, k, level)
    arr = (_vp * k)(*[_ptr(c, 2 * level * prm.N, "ct").value for c in cts])
    _check(load().mick_mul_relin_rescale(prm.handle, keys.handle, arr, k, level,
                                         _ptr(out, 2 * (level - k + 1) * prm.N, "out"), _ptr(ws),
                                         ws.numel() * 4, _stream()), "mick_mul_relin_rescale")
    return out


def mul_relin_rescale_noalloc(prm: Params, keys: Keys, cts: Sequence[torch.Tensor], level: int, out=None):
    """The multiply on the library's static workspace (no allocation inside)."""
    k = len(cts)
    if out is None:
        out = _dev_empty(2, level - k + 1, prm.N)
    arr = (_vp * k)(*[_ptr(c, 2 * level * prm.N, "ct").value for c in cts])
    _check(load().mick_mul_relin_rescale_noalloc(prm.handle, keys.handle, arr, k, level,
                                                 _ptr(out, 2 * (level - k + 1) * prm.N, "out"), _stream()),
           "mick_mul_relin_rescale_noalloc")
    return out


def batch_workspace(prm: Params, n_jobs: int, k: int, level: int) -> torch.Tensor:
    nbytes = load().mick_batch_workspace_bytes(prm.handle, n_jobs, k, level)
    if nbytes == 0:
        raise ValueError("invalid (n_jobs, k, level)")
    return _dev_empty(nbytes // 4)


def mul_relin_rescale_batch(prm: Params, keys: Keys, cts: torch.Tensor, level: int, out=None,
                            ws=None) -> torch.Tensor:
    """cts: [n_jobs, k, 2, level, N] int32 device tensor."""
    n_jobs, k = cts.shape[0], cts.shape[1]
    if tuple(cts.shape[2:]) != (2, level, prm.N):
        raise ValueError("cts must be [n_jobs, k, 2, level, N]")
    if out is None:
        out = _dev_empty(n_jobs, 2, level - k + 1, prm.N)
    if ws is None:
        ws = batch_workspace(prm, n_jobs, k, level)
    _check(load().mick_mul_relin_rescale_batch(prm.handle, keys.handle, _ptr(cts), n_jobs, k, level,
                                               _ptr(out, n_jobs * 2 * (level - k + 1) * prm.N, "out"),
                                               _ptr(ws), ws.numel() * 4, _stream()), "mick_mul_relin_rescale_batch")
    return out


def make_jobs(prm: Params, specs, status=None):
    """specs: list of (cts, level, out) with cts a list of [2, level, N] tensors
    (None entries pass a NULL pointer) and out a [2, level - k + 1, N] tensor or
    None.  status: optional ctypes int array, one status word per job (a job
    whose shape is out of range then gets a one-word placeholder output, left
    untouched by the library, which refuses the job).  Returns (ctypes array,
    outputs)."""
    arr = (Job * len(specs))()
    outs = []
    for i, (cts, level, out) in enumerate(specs):
        k = len(cts)
        valid = 2 <= k <= 12 and k <= level <= prm.L
        if out is None:
            if not valid and status is None:
                raise ValueError("job %d: k=%d, level=%d out of range" % (i, k, level))
            out = _dev_empty(2, level - k + 1, prm.N) if valid else _dev_empty(1)
        arr[i].k, arr[i].level = k, level
        for u, c in enumerate(cts):
            arr[i].cts[u] = None if c is None else _ptr(c, 2 * level * prm.N if valid else 0, "ct").value
        arr[i].out = _ptr(out, 2 * (level - k + 1) * prm.N if valid else 0, "out").value
        if status is not None:
            arr[i].status = ctypes.addressof(status) + i * ctypes.sizeof(ctypes.c_int)
        outs.append(out)
    return arr, outs


def jobs_workspace_bytes(prm: Params, shapes) -> int:
    """Workspace of a job table holding jobs of the given (k, level) shapes
    (pointers are not needed to size it)."""
    arr = (Job * len(shapes))()
    for i, (k, level) in enumerate(shapes):
        arr[i].k, arr[i].level = k, level
    nbytes = load().mick_jobs_workspace_bytes(prm.handle, ctypes.cast(arr, _vp), len(arr))
    if nbytes == 0:
        raise ValueError("invalid job shapes")
    return nbytes


def jobs_workspace(prm: Params, arr) -> torch.Tensor:
    nbytes = load().mick_jobs_workspace_bytes(prm.handle, ctypes.cast(arr, _vp), len(arr))
    if nbytes == 0:
        raise ValueError("invalid jobs")
    return _dev_empty((nbytes + 3) // 4)


def mul_relin_rescale_jobs(prm: Params, keys: Keys, specs, ws=None, isolate: bool = False):
    """Heterogeneous batch: every job (k, level may differ) in one launch per stage.
    isolate: give every job a status word, so an invalid job is refused alone;
    returns (outputs, statuses) then."""
    st = (ctypes.c_int * len(specs))(*([E_HIP] * len(specs))) if isolate else None
    arr, outs = make_jobs(prm, specs, st)
    if ws is None:
        ws = jobs_workspace(prm, arr)
    _check(load().mick_mul_relin_rescale_jobs(prm.handle, keys.handle, ctypes.cast(arr, _vp), len(arr), _ptr(ws),
                                              ws.numel() * 4, _stream()), "mick_mul_relin_rescale_jobs")
    return (outs, list(st)) if isolate else outs


def output_scale(prm: Params, scales, level: int) -> float:
    """The scale of a k-input multiply's output at `level` (k = len(scales))."""
    arr = (ctypes.c_double * len(scales))(*scales)
    out = ctypes.c_double()
    _check(load().mick_output_scale(prm.handle, arr, len(scales), level, ctypes.byref(out)), "mick_output_scale")
    return out.value


class Plan:
    """A heterogeneous batch whose job table has been written to `ws`.  run()
    only launches kernels, so it can be captured into a CUDA/HIP graph."""

    def __init__(self, prm: Params, keys: Keys, specs, ws=None):
        self.arr, self.outs = make_jobs(prm, specs)
        self.ws = jobs_workspace(prm, self.arr) if ws is None else ws
        self.prm, self.keys, self.specs = prm, keys, specs  # keep the buffers alive
        h = _vp()
        _check(load().mick_jobs_plan(prm.handle, keys.handle, ctypes.cast(self.arr, _vp), len(self.arr),
                                     _ptr(self.ws), self.ws.numel() * 4, _stream(), ctypes.byref(h)), "mick_jobs_plan")
        self._h = h

    def run(self):
        _check(load().mick_plan_execute(self._h, _stream()), "mick_plan_execute")
        return self.outs

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mick_plan_destroy(self._h)
            self._h = None


def ntt(prm: Params, data: torch.Tensor, first_prime: int, inverse: bool = False) -> torch.Tensor:
    """In-place transform of data [n_limbs, N]; limb i uses prime index first_prime + i."""
    if data.dim() != 2 or data.shape[1] != prm.N:
        raise ValueError("data must be [n_limbs, N]")
    _check(load().mick_ntt(prm.handle, _ptr(data), data.shape[0], first_prime, int(inverse), _stream()), "mick_ntt")
    return data


BCONV_VALU, BCONV_MFMA = 0, 1


def bconv(prm: Params, src: torch.Tensor, level: int, digit: int, method: int = BCONV_VALU, out=None):
    """Fast basis conversion of digit `digit` at `level` for src [n_polys, na, N]
    (coefficient domain); returns [n_polys, level + K - na, N]."""
    if src.dim() != 3 or src.shape[2] != prm.N:
        raise ValueError("src must be [n_polys, na, N]")
    lo = digit * prm.alpha
    na = max(0, min(prm.alpha, level - lo))
    n_polys = src.shape[0]
    if src.shape[1] != na:
        raise ValueError("src holds %d limbs; digit %d at level %d has %d" % (src.shape[1], digit, level, na))
    T = level + prm.K - na
    if out is None:
        out = _dev_empty(n_polys, T, prm.N)
    _check(load().mick_bconv(prm.handle, _ptr(src, n_polys * na * prm.N, "src"), n_polys, level, digit,
                             _ptr(out, n_polys * T * prm.N, "out"), method, _stream()), "mick_bconv")
    return out


def profile_enable(on: bool = True):
    """Bracket every library kernel launch with HIP events on its stream."""
    _check(load().mick_profile_enable(int(on)), "mick_profile_enable")


def profile_select(sites=None):
    """Record only the named sites while profiling is on (None: every site)."""
    arg = None if not sites else ",".join(sites).encode()
    _check(load().mick_profile_select(arg), "mick_profile_select")


def profile_collect():
    """{site: (total_ms, launches)} for the launches recorded since the last collect."""
    n_max = 32
    names = (ctypes.c_char_p * n_max)()
    ms = (ctypes.c_double * n_max)()
    cnt = (ctypes.c_int * n_max)()
    n = load().mick_profile_collect(n_max, names, ms, cnt)
    if n < 0:
        raise MickError(n, "mick_profile_collect")
    return {names[i].decode(): (ms[i], cnt[i]) for i in range(n)}


# ---------------------------------------------------------------- queue

class Queue:
    """mick_queue over several parameter sets (with their keys) and a device
    workspace arena of `capacity` bytes.  push() keeps the input and output
    tensors of each job alive until poll() or drain() reports it done."""

    def __init__(self, sets: Sequence[tuple], capacity: int):
        self.sets = list(sets)  # [(Params, Keys)], kept alive
        n = len(self.sets)
        prms = (_vp * n)(*[p.handle.value for p, _ in self.sets])
        keys = (_vp * n)(*[k.handle.value for _, k in self.sets])
        h = _vp()
        _check(load().mick_queue_create(prms, keys, n, capacity, ctypes.byref(h)), "mick_queue_create")
        self._h = h
        self._live = {}  # id -> tensors (and status words) of the job
        self._status = {}  # id -> (status array, index)

    def job_bytes(self, set_index: int, k: int, level: int) -> int:
        return load().mick_queue_job_bytes(self._h, set_index, k, level)

    def push(self, jobs, isolate: bool = False):
        """jobs: iterable of (id, set_index, cts, level, out) with cts k tensors
        [2, level, N] and out a [2, level - k + 1, N] tensor.  isolate: every job
        gets a status word (status(id)), so an invalid job is refused alone."""
        jobs = list(jobs)
        arr = (QJob * len(jobs))()
        st_arr = (ctypes.c_int * len(jobs))(*([E_HIP] * len(jobs))) if isolate else None
        for i, (jid, st, cts, level, out) in enumerate(jobs):
            arr[i].id, arr[i].set, arr[i].k, arr[i].level = jid, st, len(cts), level
            # an unknown set index or shape is the library's to reject
            N = self.sets[st][0].N if 0 <= st < len(self.sets) else 0
            ok_shape = 2 <= len(cts) <= 12 and len(cts) <= level and N > 0
            for u, c in enumerate(cts):
                arr[i].cts[u] = None if c is None else _ptr(c, 2 * level * N if ok_shape else 0, "ct").value
            arr[i].out = _ptr(out, 2 * (level - len(cts) + 1) * N if ok_shape else 0, "out").value
            if isolate:
                arr[i].status = ctypes.addressof(st_arr) + i * ctypes.sizeof(ctypes.c_int)
        _check(load().mick_queue_push(self._h, ctypes.cast(arr, _vp), len(jobs)), "mick_queue_push")
        for i, (jid, _st, cts, _lv, out) in enumerate(jobs):
            # the status words stay alive while the queue may write them
            self._live.setdefault(jid, []).append((cts, out, st_arr))
            if isolate:
                self._status[jid] = (st_arr, i)

    def status(self, jid):
        """The status word of a job pushed with isolate=True."""
        arr, i = self._status[jid]
        return arr[i]

    def cancel(self, jid):
        """Removes the pending jobs with this id; MickError(E_BUSY) if it already runs."""
        _check(load().mick_queue_cancel(self._h, jid), "mick_queue_cancel")

    def run(self) -> int:
        n = load().mick_queue_run(self._h, _stream())
        if n < 0:
            raise MickError(n, "mick_queue_run")
        return n

    def poll(self, max_ids: int = 4096):
        buf = (ctypes.c_uint64 * max_ids)()
        n = load().mick_queue_poll(self._h, buf, max_ids)
        if n < 0:
            raise MickError(n, "mick_queue_poll")
        ids = [buf[i] for i in range(n)]
        for i in ids:
            self._live.pop(i, None)
        return ids

    def drain(self):
        _check(load().mick_queue_drain(self._h, _stream()), "mick_queue_drain")
        self._live.clear()

    def info(self):
        p, r, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        _check(load().mick_queue_info(self._h, ctypes.byref(p), ctypes.byref(r), ctypes.byref(b)), "mick_queue_info")
        return p.value, r.value, b.value

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mick_queue_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        self.close()


# ---------------------------------------------------------------- schedule, allocator

def autotune(prm: Params, cache_path: str | None = None) -> int:
    """Chooses the transform schedule of `prm` by timing (or from the cache
    file); returns the first-pass log size now in use."""
    _check(load().mick_autotune(prm.handle, cache_path.encode() if cache_path else None), "mick_autotune")
    return schedule(prm)


def set_schedule(prm: Params, first_pass_log: int):
    _check(load().mick_params_set_schedule(prm.handle, first_pass_log), "mick_params_set_schedule")


TENSOR_CHAIN, TENSOR_TREE, TENSOR_FILTER = 0, 1, 2


def set_tensor_method(prm: Params, method: int):
    _check(load().mick_params_set_tensor_method(prm.handle, method), "mick_params_set_tensor_method")


def set_modup_targets(prm: Params, targets: int):
    _check(load().mick_params_set_modup_targets(prm.handle, targets), "mick_params_set_modup_targets")


def modup_targets(prm: Params) -> int:
    m = load().mick_params_modup_targets(prm.handle)
    if m < 0:
        raise MickError(m, "mick_params_modup_targets")
    return m


def autotune_report(prm: Params):
    """[((first-pass log, tensor method, ModUp targets), us per multiply)] of the
    last timing run of mick_autotune on these parameters."""
    n = 64
    cfg = (ctypes.c_int * (3 * n))()
    us = (ctypes.c_double * n)()
    m = load().mick_autotune_report(prm.handle, n, cfg, us)
    if m < 0:
        raise MickError(m, "mick_autotune_report")
    return [((cfg[3 * i], cfg[3 * i + 1], cfg[3 * i + 2]), us[i]) for i in range(min(m, n))]


def tensor_method(prm: Params) -> int:
    m = load().mick_params_tensor_method(prm.handle)
    if m < 0:
        raise MickError(m, "mick_params_tensor_method")
    return m


def schedule(prm: Params) -> int:
    v = load().mick_params_schedule(prm.handle)
    if v < 0:
        raise MickError(v, "mick_params_schedule")
    return v


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocator_refs = None  # keeps the registered callbacks alive


def use_torch_allocator(on: bool = True):
    """Routes the library's own device allocations (tables, keys, queue
    arenas) through PyTorch's caching allocator (on=True) or back to
    hipMalloc (on=False).  Objects keep the allocator they were created
    with."""
    global _allocator_refs
    if not on:
        _check(load().mick_set_allocator(None, None, None), "mick_set_allocator")
        return

    def _alloc(nbytes, _ctx):
        try:
            return torch.cuda.caching_allocator_alloc(max(int(nbytes), 1))
        except Exception:  # out of memory: the library reports MICK_E_NOMEM
            return None

    def _free(ptr, _ctx):
        torch.cuda.caching_allocator_delete(ptr)

    refs = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _check(load().mick_set_allocator(ctypes.cast(refs[0], _vp), ctypes.cast(refs[1], _vp), None),
           "mick_set_allocator")
    # earlier callbacks stay referenced: objects created with them still free through them
    _allocator_refs = (refs, _allocator_refs)


# ---------------------------------------------------------------- tree multiply

def tree_tokens(tree) -> list:
    """Nested tuples (an int: a group of that many inputs; a tuple: a node)
    to the library's prefix tokens."""
    if isinstance(tree, int):
        return [tree]
    out = [-len(tree)]
    for c in tree:
        out += tree_tokens(c)
    return out


def tree_from_tokens(tok) -> object:
    def rec(i):
        v = tok[i]
        if v > 0:
            return v, i + 1
        kids, j = [], i + 1
        for _ in range(-v):
            c, j = rec(j)
            kids.append(c)
        return tuple(kids), j
    t, end = rec(0)
    if end != len(tok):
        raise ValueError("tokens left over")
    return t


def _tok_array(tree):
    tok = tree_tokens(tree)
    return (ctypes.c_int * len(tok))(*tok), len(tok)


def tree_plan(n: int):
    """The partition of n inputs with the fewest rescale units at depth
    ceil(log2 n), as nested tuples."""
    buf = (ctypes.c_int * 64)()
    k = load().mick_tree_plan(n, buf, 64)
    if k < 0:
        raise MickError(k, "mick_tree_plan")
    return tree_from_tokens(list(buf[:k]))


def tree_shape(tree):
    """(inputs, depth, rescale units before relinearisation)."""
    arr, k = _tok_array(tree)
    n, d, u = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load().mick_tree_shape(arr, k, ctypes.byref(n), ctypes.byref(d), ctypes.byref(u)), "mick_tree_shape")
    return n.value, d.value, u.value


def _tree_depth(t) -> int:
    if isinstance(t, int):
        return t - 1
    return max(_tree_depth(c) for c in t) + len(t) - 1


def tree_rescales(tree, level: int):
    """[(product level, mu)] of every rescale the tree performs on inputs at
    `level` (every subtree runs at the level at which it enters its parent);
    the output scale is Delta^n over the product of the primes q_j with
    product level - mu <= j < product level over all entries."""
    out = []

    def walk(t, end):
        mu = (t if isinstance(t, int) else len(t)) - 1
        prod = end + mu
        if not isinstance(t, int):
            for c in t:
                walk(c, prod)
        if mu > 0:
            out.append((prod, mu))
    walk(tree, level - _tree_depth(tree))
    return out


def tree_workspace(prm: Params, tree, level: int) -> torch.Tensor:
    arr, k = _tok_array(tree)
    nbytes = load().mick_tree_workspace_bytes(prm.handle, arr, k, level)
    if nbytes == 0:
        raise ValueError("invalid tree or level")
    return _dev_empty((nbytes + 3) // 4)


def mul_tree(prm: Params, keys: Keys, cts: Sequence[torch.Tensor], level: int, tree, out=None, ws=None):
    """Tree-structured multiply; returns the [2, level - depth, N] output."""
    arr, k = _tok_array(tree)
    n, depth, _ = tree_shape(tree)
    if len(cts) != n:
        raise ValueError("the tree takes %d inputs" % n)
    if out is None:
        out = _dev_empty(2, level - depth, prm.N)
    if ws is None:
        ws = tree_workspace(prm, tree, level)
    ptrs = (_vp * n)(*[_ptr(c, 2 * level * prm.N, "ct").value for c in cts])
    _check(load().mick_mul_tree(prm.handle, keys.handle, ptrs, level, arr, k,
                                _ptr(out, 2 * (level - depth) * prm.N, "out"), _ptr(ws), ws.numel() * 4,
                                _stream()), "mick_mul_tree")
    return out
