"""Thin Python binding of libcc3.so (C ABI in include/cc3.h).

Argument marshalling only: every step of the residual runs in the library's
HIP kernels.  Arrays are torch CUDA tensors (float64, contiguous); torch
supplies device memory and the stream, nothing else.  There is no fallback:
if the library is missing or fails to load, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("CC3_LIB", os.path.join(_HERE, "libcc3.so"))

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libcc3.so not found at {LIB_PATH}; build it with "
                      "`python -m paper_2007_01088_amd.csrc.build` (or __graft_entry__.build())")
_lib = ctypes.CDLL(LIB_PATH)

OK, E_INVAL, E_NOMEM, E_DEVICE, E_PRECOND, E_NOTFOUND, E_BUSY, E_TIMEOUT, E_CANCELLED = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
FP64, FP32, BF16X3, BF16X6 = 0, 1, 2, 3
ACCUMULATE, CHECK, ONE_STREAM, LOWP_CONTRACT, DETERMINISTIC = 1, 2, 4, 8, 16

_c_int, _c_size, _vp, _dp = ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double)]


def _sig(name, args, res=_c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_create = _sig("cc3_create", [ctypes.POINTER(_vp), _c_int])
_destroy = _sig("cc3_destroy", [_vp])
_last_error = _sig("cc3_last_error", [], ctypes.c_char_p)
_ws_size = _sig("cc3_workspace_size", [_c_int, _c_int, _c_int, _c_int, ctypes.c_uint,
                                       ctypes.POINTER(_c_size)])
_residual = _sig("cc3_triples_residual", [_vp, _c_int, _c_int, _c_int, _dp, _dp, _dp, _dp, _dp,
                                          _dp, _c_int, ctypes.c_uint, _vp, _c_size, _vp])
_residual_blocks = _sig("cc3_triples_residual_blocks",
                        [_vp, _c_int, _c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                         _c_int, ctypes.c_uint, _vp, _c_size, _vp])
_residual_subset = _sig("cc3_triples_residual_subset",
                        [_vp, _c_int, _c_int, _c_int, _dp, _dp, _dp, _dp, _vp, _c_int, _dp, _dp,
                         _c_int, ctypes.c_uint, _vp, _c_size, _vp])
_residual_subset_blocks = _sig("cc3_triples_residual_subset_blocks",
                               [_vp, _c_int, _c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _vp,
                                _c_int, _dp, _dp, _c_int, ctypes.c_uint, _vp, _c_size, _vp])
_t3_block_blocks = _sig("cc3_t3_block_blocks",
                        [_vp, _c_int, _c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _c_int,
                         _c_int, _c_int, _dp, _c_int, _vp, _c_size, _vp])
_t3_block = _sig("cc3_t3_block", [_vp, _c_int, _c_int, _c_int, _dp, _dp, _dp, _dp, _c_int, _c_int,
                                  _c_int, _dp, _c_int, _vp, _c_size, _vp])
_jprep = _sig("cc3_jacobian_prep", [_vp, _c_int, _c_int, _c_int, _dp, _dp, _dp, _dp, _dp, _dp,
                                     _c_int, ctypes.c_uint, _vp, _c_size, _vp])
_residual_noalloc = _sig("cc3_triples_residual_noalloc",
                         [_vp, _c_int, _c_int, _c_int, _dp, _dp, _dp, _dp, _dp, _dp, _c_int,
                          ctypes.c_uint, _vp])
_td_ws = _sig("cc3_transition_density_workspace_size",
               [_c_int, _c_int, _c_int, ctypes.POINTER(_c_size)])
_td = _sig("cc3_transition_density",
           [_vp, _c_int, _c_int, _c_int, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_double, _dp, _dp,
            _dp, _dp, _dp, ctypes.c_uint, _vp, _c_size, _vp])
_batch_plan = _sig("cc3_batch_plan", [_c_int, _c_int, _c_int, _c_int, ctypes.c_uint,
                                      ctypes.POINTER(_c_int), ctypes.POINTER(_c_int)])
_flops = _sig("cc3_flops", [_c_int, _c_int, ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_double)])
_cvs = _sig("cc3_cvs_triples", [_c_int, ctypes.POINTER(ctypes.c_int32), _c_int,
                                ctypes.POINTER(ctypes.c_int32), _c_int, ctypes.POINTER(ctypes.c_int)])
_prof_enable = _sig("cc3_profile_enable", [_vp, _c_int])
_prof_get = _sig("cc3_profile_get", [_vp, ctypes.POINTER(KernelStat), _c_int,
                                     ctypes.POINTER(_c_int)])



class Timing(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("finish_s", ctypes.c_double),
                ("device_ms", ctypes.c_double), ("slot", _c_int), ("rebuilt", _c_int)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("queued", _c_int), ("inflight", _c_int), ("max_inflight_seen", _c_int),
                ("molecules", _c_int), ("arena_bytes", _c_size), ("arena_used", _c_size),
                ("arena_peak", _c_size), ("packed", ctypes.c_int64), ("packs", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_u64 = ctypes.c_uint64
_srv_create = _sig("cc3_server_create", [ctypes.POINTER(_vp), _c_int, _vp, _c_size, _c_int])
_srv_destroy = _sig("cc3_server_destroy", [_vp])
_srv_footprint = _sig("cc3_server_footprint", [_vp, _c_int, _c_int, _c_int, _c_int,
                                               ctypes.POINTER(_c_size), ctypes.POINTER(_c_size)])
_mol_register = _sig("cc3_molecule_register", [_vp, _c_int, _c_int, _c_int, _dp, _dp, _dp,
                                               ctypes.POINTER(_u64)])
_mol_release = _sig("cc3_molecule_release", [_vp, _u64])
_submit = _sig("cc3_submit", [_vp, _u64, _dp, _dp, _c_int, ctypes.c_uint, ctypes.POINTER(_u64)])
_poll = _sig("cc3_poll", [_vp, _u64, ctypes.POINTER(_c_int)])
_wait = _sig("cc3_wait", [_vp, _u64, _dp, _dp, ctypes.POINTER(Timing)])
_cancel = _sig("cc3_cancel", [_vp, _u64])
_srv_stats = _sig("cc3_server_get_stats", [_vp, ctypes.POINTER(ServerStats)])
_srv_packing = _sig("cc3_server_set_packing", [_vp, _c_int, ctypes.c_double])

EXPORTED = ["cc3_create", "cc3_destroy", "cc3_last_error", "cc3_workspace_size",
            "cc3_triples_residual", "cc3_triples_residual_blocks", "cc3_triples_residual_subset",
            "cc3_t3_block", "cc3_triples_residual_subset_blocks", "cc3_t3_block_blocks",
            "cc3_flops", "cc3_batch_plan", "cc3_triples_residual_noalloc",
            "cc3_transition_density_workspace_size", "cc3_transition_density", "cc3_cvs_triples", "cc3_profile_enable", "cc3_profile_get",
            "cc3_jacobian_prep", "cc3_server_create", "cc3_server_destroy", "cc3_server_footprint",
            "cc3_molecule_register", "cc3_molecule_release", "cc3_submit", "cc3_poll",
            "cc3_wait", "cc3_cancel", "cc3_server_get_stats", "cc3_server_set_packing"]


class CC3Error(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _last_error().decode(errors="replace")
        super().__init__(f"{where} failed ({code}): {msg}")


def _check(rc: int, where: str) -> None:
    if rc != OK:
        raise CC3Error(rc, where)


def last_error() -> str:
    return _last_error().decode(errors="replace")


def _ptr(t: torch.Tensor | None, name: str, dtype=torch.float64) -> int:
    if t is None:
        return 0
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA tensor of dtype {dtype}")
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def workspace_size(no: int, nv: int, nchol: int, prec: int = FP64, flags: int = 0) -> int:
    n = _c_size(0)
    _check(_ws_size(no, nv, nchol, prec, flags, ctypes.byref(n)), "cc3_workspace_size")
    return n.value


def cvs_triples(no: int, core) -> np.ndarray:
    """The restricted-loop triples (int32 [n][3], lexicographic) containing at least one
    of the core orbital indices `core` (cc3_cvs_triples)."""
    import numpy as np
    c = np.ascontiguousarray(np.asarray(core, dtype=np.int32).reshape(-1))
    cp = c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if c.size else None
    n = ctypes.c_int(0)
    _check(_cvs(no, cp, int(c.size), None, 0, ctypes.byref(n)), "cc3_cvs_triples")
    out = np.zeros((n.value, 3), dtype=np.int32)
    if n.value:
        _check(_cvs(no, cp, int(c.size), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    n.value, ctypes.byref(n)), "cc3_cvs_triples")
    return out


def batch_plan(no: int, nv: int, nchol: int, prec: int = FP64, flags: int = 0) -> tuple[int, int]:
    """(triples per batch, number of batches) of the one-shot calls' triple loop."""
    b, n = _c_int(0), _c_int(0)
    _check(_batch_plan(no, nv, nchol, prec, flags, ctypes.byref(b), ctypes.byref(n)),
           "cc3_batch_plan")
    return b.value, n.value


def batch_triples(no: int, nbatches: int, b: int):
    """The unordered triples of batch b (int32 [n][3]): loop positions b, b + nbatches, ..."""
    import numpy as np
    allt = [(i, j, k) for i in range(no) for j in range(i + 1) for k in range(j + 1)
            if not (i == j == k)]
    return np.array(allt[b::nbatches], dtype=np.int32).reshape(-1, 3)


def flops(no: int, nv: int) -> tuple[float, float]:
    a, b = ctypes.c_double(0), ctypes.c_double(0)
    _check(_flops(no, nv, ctypes.byref(a), ctypes.byref(b)), "cc3_flops")
    return a.value, b.value


class Context:
    """A libcc3 context on one device, with a cached workspace tensor."""

    def __init__(self, device: int = 0):
        h = _vp()
        _check(_create(ctypes.byref(h), device), "cc3_create")
        self._h = h
        self.device = device
        self._ws = None

    def close(self) -> None:
        if self._h:
            _destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, nbytes: int) -> torch.Tensor:
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8,
                                   device=f"cuda:{self.device}")
        return self._ws

    # ---- residual calls ------------------------------------------------
    def triples_residual(self, eps, L, t1, t2, omega1=None, omega2=None, prec=FP64, flags=0,
                         stream=None):
        no, nv = t1.shape
        nchol = L.shape[0]
        if omega1 is None:
            omega1 = torch.empty((no, nv), dtype=torch.float64, device=t2.device)
        if omega2 is None:
            omega2 = torch.empty((no, no, nv, nv), dtype=torch.float64, device=t2.device)
        nbytes = workspace_size(no, nv, nchol, prec, flags)
        ws = self.workspace(nbytes)
        _check(_residual(self._h, no, nv, nchol, _any_ptr(eps, "eps"), _any_ptr(L, "L"),
                         _any_ptr(t1, "t1"), _any_ptr(t2, "t2"), _any_ptr(omega1, "omega1"),
                         _any_ptr(omega2, "omega2"), prec, flags, ws.data_ptr(), ws.numel(),
                         _stream(stream)),
               "cc3_triples_residual")
        return omega1, omega2

    def triples_residual_noalloc(self, eps, L, t1, t2, omega1, omega2, prec=FP64, flags=0,
                                 stream=None):
        """cc3_triples_residual_noalloc: no workspace argument, no device allocation (the
        library's static scratch array); device tensors only, outputs given by the caller."""
        no, nv = t1.shape
        _check(_residual_noalloc(self._h, no, nv, L.shape[0], _ptr(eps, "eps"), _ptr(L, "L"),
                                 _ptr(t1, "t1"), _ptr(t2, "t2"), _ptr(omega1, "omega1"),
                                 _ptr(omega2, "omega2"), prec, flags, _stream(stream)),
               "cc3_triples_residual_noalloc")
        return omega1, omega2

    def triples_residual_blocks(self, eps, g_vvvo, g_oovo, g_ovov, g_ooov, g_vvov, F_ov, t2,
                                omega1=None, omega2=None, prec=FP64, flags=0, stream=None):
        no, nv = F_ov.shape
        if omega1 is None:
            omega1 = torch.empty((no, nv), dtype=torch.float64, device=t2.device)
        if omega2 is None:
            omega2 = torch.empty((no, no, nv, nv), dtype=torch.float64, device=t2.device)
        nbytes = workspace_size(no, nv, 0, prec, flags)
        ws = self.workspace(nbytes)
        _check(_residual_blocks(self._h, no, nv, _any_ptr(eps, "eps"), _any_ptr(g_vvvo, "g_vvvo"),
                                _any_ptr(g_oovo, "g_oovo"), _any_ptr(g_ovov, "g_ovov"),
                                _any_ptr(g_ooov, "g_ooov"), _any_ptr(g_vvov, "g_vvov"),
                                _any_ptr(F_ov, "F_ov"), _any_ptr(t2, "t2"),
                                _any_ptr(omega1, "omega1"), _any_ptr(omega2, "omega2"), prec,
                                flags, ws.data_ptr(), ws.numel(), _stream(stream)),
               "cc3_triples_residual_blocks")
        return omega1, omega2

    def triples_residual_subset(self, eps, L, t1, t2, triples, prec=FP64, flags=0, stream=None):
        """Contravariant (Ot1, Ot2) from the listed unordered triples (host int32 [n][3])."""
        import numpy as np
        no, nv = t1.shape
        nchol = L.shape[0]
        tri = np.ascontiguousarray(np.asarray(triples, dtype=np.int32).reshape(-1, 3))
        o1 = torch.empty((no, nv), dtype=torch.float64, device=t2.device)
        o2 = torch.empty((no, no, nv, nv), dtype=torch.float64, device=t2.device)
        nbytes = workspace_size(no, nv, nchol, prec, flags)
        ws = self.workspace(nbytes)
        _check(_residual_subset(self._h, no, nv, nchol, _any_ptr(eps, "eps"), _any_ptr(L, "L"),
                                _any_ptr(t1, "t1"), _any_ptr(t2, "t2"),
                                tri.ctypes.data_as(ctypes.c_void_p), int(tri.shape[0]),
                                _any_ptr(o1, "o1"), _any_ptr(o2, "o2"), prec, flags, ws.data_ptr(),
                                ws.numel(), _stream(stream)), "cc3_triples_residual_subset")
        return o1, o2

    def t3_block(self, eps, L, t1, t2, i, j, k, prec=FP64, stream=None):
        no, nv = t1.shape
        nchol = L.shape[0]
        tau = torch.empty((nv, nv, nv), dtype=torch.float64, device=t2.device)
        nbytes = workspace_size(no, nv, nchol, prec, 0)
        ws = self.workspace(nbytes)
        _check(_t3_block(self._h, no, nv, nchol, _any_ptr(eps, "eps"), _any_ptr(L, "L"),
                         _any_ptr(t1, "t1"), _any_ptr(t2, "t2"), i, j, k, _any_ptr(tau, "tau"),
                         prec, ws.data_ptr(), ws.numel(), _stream(stream)), "cc3_t3_block")
        return tau

    def triples_residual_subset_blocks(self, eps, g_vvvo, g_oovo, g_ovov, g_ooov, g_vvov, F_ov,
                                       t2, triples, prec=FP64, flags=0, stream=None):
        """Contravariant (Ot1, Ot2) of the listed triples from integral blocks."""
        import numpy as np
        no, nv = F_ov.shape
        tri = np.ascontiguousarray(np.asarray(triples, dtype=np.int32).reshape(-1, 3))
        o1 = torch.empty((no, nv), dtype=torch.float64, device=t2.device)
        o2 = torch.empty((no, no, nv, nv), dtype=torch.float64, device=t2.device)
        nbytes = workspace_size(no, nv, 0, prec, flags)
        ws = self.workspace(nbytes)
        _check(_residual_subset_blocks(
            self._h, no, nv, _any_ptr(eps, "eps"), _any_ptr(g_vvvo, "g_vvvo"),
            _any_ptr(g_oovo, "g_oovo"), _any_ptr(g_ovov, "g_ovov"), _any_ptr(g_ooov, "g_ooov"),
            _any_ptr(g_vvov, "g_vvov"), _any_ptr(F_ov, "F_ov"), _any_ptr(t2, "t2"),
            tri.ctypes.data_as(ctypes.c_void_p), int(tri.shape[0]), _any_ptr(o1, "o1"),
            _any_ptr(o2, "o2"), prec, flags, ws.data_ptr(), ws.numel(), _stream(stream)),
            "cc3_triples_residual_subset_blocks")
        return o1, o2

    def t3_block_blocks(self, eps, g_vvvo, g_oovo, g_ovov, g_ooov, g_vvov, F_ov, t2, i, j, k,
                        prec=FP64, stream=None):
        no, nv = F_ov.shape
        tau = torch.empty((nv, nv, nv), dtype=torch.float64, device=t2.device)
        nbytes = workspace_size(no, nv, 0, prec, 0)
        ws = self.workspace(nbytes)
        _check(_t3_block_blocks(
            self._h, no, nv, _any_ptr(eps, "eps"), _any_ptr(g_vvvo, "g_vvvo"),
            _any_ptr(g_oovo, "g_oovo"), _any_ptr(g_ovov, "g_ovov"), _any_ptr(g_ooov, "g_ooov"),
            _any_ptr(g_vvov, "g_vvov"), _any_ptr(F_ov, "F_ov"), _any_ptr(t2, "t2"), i, j, k,
            _any_ptr(tau, "tau"), prec, ws.data_ptr(), ws.numel(), _stream(stream)),
            "cc3_t3_block_blocks")
        return tau

    def jacobian_prep(self, eps, L, t1, t2, zv=None, zo=None, prec=FP64, flags=0, stream=None):
        """Algorithm 2 intermediates: zv[a][b][i][d] = Z~v_{abid}, zo[a][j][i][l] = Z~o_{ajil}."""
        no, nv = t1.shape
        nchol = L.shape[0]
        if zv is None:
            zv = torch.empty((nv, nv, no, nv), dtype=torch.float64, device=t2.device)
        if zo is None:
            zo = torch.empty((nv, no, no, no), dtype=torch.float64, device=t2.device)
        nbytes = workspace_size(no, nv, nchol, prec, flags)
        ws = self.workspace(nbytes)
        _check(_jprep(self._h, no, nv, nchol, _ptr(eps, "eps"), _ptr(L, "L"), _ptr(t1, "t1"),
                      _ptr(t2, "t2"), _ptr(zv, "zv"), _ptr(zo, "zo"), prec, flags, ws.data_ptr(),
                      ws.numel(), _stream(stream)), "cc3_jacobian_prep")
        return zv, zo

    def transition_density(self, eps, L, t1, t2, l1, l2, omega, flags=0, want_yo=False,
                           out=None, stream=None):
        """Algorithm 3: (D_cd, D_kc, D_ld, D_lk[, Yo]) for the left state (l1, l2, omega)."""
        no, nv = t1.shape
        nchol = L.shape[0]
        dev = t2.device
        if out is None:
            out = (torch.empty((nv, nv), dtype=torch.float64, device=dev),
                   torch.empty((no, nv), dtype=torch.float64, device=dev),
                   torch.empty((no, nv), dtype=torch.float64, device=dev),
                   torch.empty((no, no), dtype=torch.float64, device=dev),
                   torch.empty((nv, no, no, no), dtype=torch.float64, device=dev)
                   if want_yo else None)
        n = _c_size(0)
        _check(_td_ws(no, nv, nchol, ctypes.byref(n)), "cc3_transition_density_workspace_size")
        ws = self.workspace(n.value)
        dcd, dkc, dld, dlk, yo = out
        _check(_td(self._h, no, nv, nchol, _ptr(eps, "eps"), _ptr(L, "L"), _ptr(t1, "t1"),
                   _ptr(t2, "t2"), _ptr(l1, "l1"), _ptr(l2, "l2"), float(omega),
                   _ptr(dcd, "D_cd"), _ptr(dkc, "D_kc"), _ptr(dld, "D_ld"), _ptr(dlk, "D_lk"),
                   _ptr(yo, "Yo"), flags, ws.data_ptr(), ws.numel(), _stream(stream)),
               "cc3_transition_density")
        return out if want_yo else out[:4]

    # ---- kernel timing ---------------------------------------------------
    def profile_enable(self, on: bool = True) -> None:
        _check(_prof_enable(self._h, 1 if on else 0), "cc3_profile_enable")

    def profile_get(self) -> dict:
        arr = (KernelStat * 16)()
        n = _c_int(0)
        _check(_prof_get(self._h, arr, 16, ctypes.byref(n)), "cc3_profile_get")
        return {arr[i].name.decode(): {"launches": arr[i].launches, "total_ms": arr[i].total_ms,
                                       "flops": arr[i].flops, "bytes": arr[i].bytes}
                for i in range(n.value)}


class Server:
    """A libcc3 serving loop over one arena tensor (uint8, on the server's GPU).

    Inputs may be CUDA tensors or host (CPU) tensors; they are copied before
    each call returns.  Results are copied out by `wait`.
    """

    def __init__(self, arena: torch.Tensor, max_inflight: int = 4, device: int = 0):
        if not arena.is_cuda or arena.dtype != torch.uint8 or not arena.is_contiguous():
            raise ValueError("arena must be a contiguous uint8 CUDA tensor")
        h = _vp()
        _check(_srv_create(ctypes.byref(h), device, arena.data_ptr(), arena.numel(),
                           max_inflight), "cc3_server_create")
        self._h = h
        self._arena = arena  # kept alive as long as the server
        self.device = device
        self._shape = {}

    def close(self) -> None:
        if self._h:
            _srv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def footprint(self, no: int, nv: int, nchol: int, prec: int = FP64) -> tuple[int, int]:
        r, t = _c_size(0), _c_size(0)
        _check(_srv_footprint(self._h, no, nv, nchol, prec, ctypes.byref(r), ctypes.byref(t)),
               "cc3_server_footprint")
        return r.value, t.value

    @staticmethod
    def _ready(*ts) -> None:
        # the server copies on a stream of its own: work queued on torch's
        # current stream that produces these inputs must be complete first
        if any(t is not None and t.is_cuda for t in ts):
            torch.cuda.current_stream().synchronize()

    def register(self, no: int, nv: int, eps, L, t1=None) -> int:
        """Copy a molecule's eps, L (and t1; None = zero) into the arena; returns its id."""
        self._ready(eps, L, t1)
        nchol = L.shape[0]
        mol = _u64(0)
        _check(_mol_register(self._h, no, nv, nchol, _any_ptr(eps, "eps"), _any_ptr(L, "L"),
                             _any_ptr(t1, "t1"), ctypes.byref(mol)), "cc3_molecule_register")
        self._shape[mol.value] = (no, nv)
        return mol.value

    def release(self, mol: int) -> None:
        _check(_mol_release(self._h, mol), "cc3_molecule_release")
        self._shape.pop(mol, None)

    def submit(self, mol: int, t2, t1=None, prec: int = FP64, flags: int = 0) -> int:
        self._ready(t2, t1)
        tk = _u64(0)
        _check(_submit(self._h, mol, _any_ptr(t1, "t1"), _any_ptr(t2, "t2"), prec, flags,
                       ctypes.byref(tk)), "cc3_submit")
        return tk.value

    def try_submit(self, mol: int, t2, t1=None, prec: int = FP64, flags: int = 0):
        """(ticket, 0) or (None, error code) without raising."""
        self._ready(t2, t1)
        tk = _u64(0)
        rc = _submit(self._h, mol, _any_ptr(t1, "t1"), _any_ptr(t2, "t2"), prec, flags,
                     ctypes.byref(tk))
        return (tk.value, 0) if rc == OK else (None, rc)

    def poll(self, ticket: int) -> bool:
        d = _c_int(0)
        _check(_poll(self._h, ticket, ctypes.byref(d)), "cc3_poll")
        return bool(d.value)

    def wait(self, ticket: int, omega1=None, omega2=None, mol: int | None = None,
             want_result: bool = True):
        """Block for `ticket`; returns (omega1, omega2, timing dict).  With
        want_result and no output tensors given, device tensors are allocated
        (the molecule id is needed for their shapes)."""
        if want_result and omega1 is None and omega2 is None:
            if mol is None:
                raise ValueError("give output tensors or the molecule id")
            no, nv = self._shape[mol]
            dev = f"cuda:{self.device}"
            omega1 = torch.empty((no, nv), dtype=torch.float64, device=dev)
            omega2 = torch.empty((no, no, nv, nv), dtype=torch.float64, device=dev)
        self._ready(omega1, omega2)  # CC3_ACCUMULATE adds into their current contents
        tm = Timing()
        _check(_wait(self._h, ticket, _any_ptr(omega1, "omega1"), _any_ptr(omega2, "omega2"),
                     ctypes.byref(tm)), "cc3_wait")
        return omega1, omega2, tm.as_dict()

    def wait_status(self, ticket: int) -> int:
        """Collect a ticket without its result; returns the request's status code."""
        return _wait(self._h, ticket, 0, 0, None)

    def cancel(self, ticket: int) -> None:
        _check(_cancel(self._h, ticket), "cc3_cancel")

    def set_packing(self, max_pack: int = 8, max_request_flops: float = 2e12) -> None:
        """Group small requests into shared launches (max_pack 1: off)."""
        _check(_srv_packing(self._h, max_pack, float(max_request_flops)),
               "cc3_server_set_packing")

    def stats(self) -> dict:
        st = ServerStats()
        _check(_srv_stats(self._h, ctypes.byref(st)), "cc3_server_get_stats")
        return st.as_dict()


def _any_ptr(t, name: str) -> int:
    """Pointer of a contiguous float64 tensor on the GPU or the host (None -> NULL)."""
    if t is None:
        return 0
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 tensor")
    return t.data_ptr()
