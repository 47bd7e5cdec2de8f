"""Python binding of libebv.so (argument marshalling only).

Every function hands device pointers of torch tensors, the sizes, and the
current HIP stream to the C ABI declared in ``include/ebv.h``; all arithmetic
runs in the library's HIP kernels.  PyTorch provides device memory and the
stream.  The library must be built (``paper_1907_05767_amd/build.py``); a
missing library raises immediately, there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libebv.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "ebv.h")

F64, F32 = 0, 1
(OP_FACTOR, OP_SOLVE, OP_BATCHED, OP_ADJOINT, OP_MIXED, OP_BAND, OP_BATCHED_MIXED, OP_FACTOR_SOLVE,
 OP_BAND_SOLVE, OP_INVERSE) = range(10)
ORDER_EBV, ORDER_INDEX, ORDER_LONGEST_FIRST = 0, 1, 2
ORDER_NAMES = {"ebv": ORDER_EBV, "index": ORDER_INDEX, "longest": ORDER_LONGEST_FIRST}
# the autotuner's table for this GPU, loaded into the default handle when present
TUNING_PATH = os.path.join(_HERE, "tuning", "mi355x.txt")

_lib = None
_handle = None


class EbvError(RuntimeError):
    """A libebv entry point returned a nonzero status."""


def _declare(lib):
    i64, i32, vp, sz, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_double
    ci = ctypes.c_int
    pi = ctypes.POINTER(ci)
    sig = {
        "ebv_version": ([], ci),
        "ebv_status_string": ([ci], ctypes.c_char_p),
        "ebv_init": ([], ci),
        "ebv_create": ([ctypes.POINTER(vp)], ci),
        "ebv_destroy": ([vp], ci),
        "ebv_load_tuning": ([vp, ctypes.c_char_p], ci),
        "ebv_workspace_status_offset": ([], sz),
        "ebv_workspace_size": ([ci, ci, i64, i64, i64], sz),
        "ebv_set_dense_tuning": ([vp, ci, ci, ci, ci], ci),
        "ebv_set_batched_tuning": ([vp, ci, ci, ci, ci], ci),
        "ebv_get_batched_tuning": ([vp, ci, ci, pi, pi], ci),
        "ebv_set_wait_limit": ([vp, i64], ci),
        "ebv_profile_update_enable": ([vp, ci], ci),
        "ebv_profile_update_read": ([vp, ctypes.POINTER(dbl), ctypes.POINTER(i64), ctypes.POINTER(dbl)], ci),
        "ebv_lu_factor": ([vp, ci, i64, vp, i64, i64, i64, vp, vp, sz, vp], ci),
        "ebv_lu_solve": ([vp, ci, i64, i64, vp, i64, vp, i64, i64, i64, i64, vp, vp, sz, vp], ci),
        "ebv_lu_factor_solve": ([vp, ci, i64, i64, vp, i64, vp, i64, vp, vp, sz, vp], ci),
        "ebv_pipeline_factor_solve": ([vp, ci, i64, i64, i64, vp, vp, vp, vp, vp, vp, sz, vp, vp, vp], ci),
        "ebv_skyline_workspace_size": ([i64, vp, vp], sz),
        "ebv_lu_factor_skyline": ([vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp], ci),
        "ebv_lu_solve_skyline": ([vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, vp, sz, vp], ci),
        "ebv_lu_inverse": ([vp, ci, i64, vp, i64, vp, i64, vp, sz, vp], ci),
        "ebv_lu_factor_solve_noalloc": ([vp, ci, i64, i64, vp, i64, vp, i64, vp, vp], ci),
        "ebv_noalloc_scratch_bytes": ([], sz),
        "ebv_noalloc_max_n": ([], i64),
        "ebv_lu_factor_band": ([vp, i64, i64, i64, vp, i64, vp, vp, sz, vp], ci),
        "ebv_lu_solve_band": ([vp, i64, i64, i64, i64, vp, i64, vp, i64, vp, vp, sz, vp], ci),
        "ebv_lu_factor_batched": ([vp, ci, i64, vp, vp, vp, i64, vp, vp, i64, vp, vp, ci, i32, dbl, vp, i32, vp, sz,
                                   vp], ci),
        "ebv_batched_order": ([ci, i64, vp, vp], ci),
        "ebv_lu_solve_adjoint": ([vp, ci, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, i64, i64, i64, i64, i64, vp,
                                  vp, sz, vp], ci),
        "ebv_lu_solve_mixed": ([vp, i64, i64, vp, i64, vp, i64, vp, i64, i32, dbl, vp, vp, vp, vp, sz, vp], ci),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


def lib():
    """The loaded libebv.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise EbvError(f"{LIB_PATH} is missing: build it with paper_1907_05767_amd/build.py")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def handle():
    """The process's default library handle (created on first use; the
    autotuner's table for this GPU is loaded into it when present)."""
    global _handle
    if _handle is None:
        h = ctypes.c_void_p()
        _check(lib().ebv_create(ctypes.byref(h)), "ebv_create")
        if os.path.exists(TUNING_PATH) and not os.environ.get("EBV_TUNING_FILE"):
            _check(lib().ebv_load_tuning(h, TUNING_PATH.encode()), "ebv_load_tuning")
        _handle = h
    return _handle


def header_symbols():
    """Names of the functions declared in include/ebv.h."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ebv_\w+)\s*\(", text)))


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().ebv_status_string(rc).decode()
        raise EbvError(f"{what} failed: status {rc} ({msg})")


def _dt(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need_gpu(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("tensors must be contiguous and on the GPU")


def workspace(op: int, dtype: int, n: int, nrhs: int = 0, batch: int = 1, device=None) -> Optional[torch.Tensor]:
    """Device workspace for an operation (None when it needs none)."""
    nbytes = lib().ebv_workspace_size(op, dtype, n, nrhs, batch)
    if nbytes == 0:
        return None
    return torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")


def _ws_args(ws: Optional[torch.Tensor]):
    if ws is None:
        return None, 0
    base = ws.data_ptr()
    pad = (-base) % 256
    return ctypes.c_void_p(base + pad), ws.numel() - pad


def workspace_status(ws: Optional[torch.Tensor]) -> int:
    """Device-side error word of a workspace (synchronizes)."""
    if ws is None:
        return 0
    base = ws.data_ptr()
    pad = (-base) % 256
    return int(ws[pad:pad + 4].view(torch.int32).item())


def set_dense_tuning(small_update_below: int = 0, lookahead: bool = True, defer_group: int = 3,
                     defer_above: int = 1024):
    """Tuning of the single-system factor on the default handle (see ebv_set_dense_tuning)."""
    _check(lib().ebv_set_dense_tuning(handle(), int(small_update_below), int(bool(lookahead)), int(defer_group),
                                      int(defer_above)), "ebv_set_dense_tuning")


def set_batched_tuning(dtype: int, mixed: bool, wg_per_cu: int, order: int):
    _check(lib().ebv_set_batched_tuning(handle(), int(dtype), int(bool(mixed)), int(wg_per_cu), int(order)),
           "ebv_set_batched_tuning")


def get_batched_tuning(dtype: int, mixed: bool):
    """(workgroups per compute unit, order policy) of the default handle for one batch form."""
    w, o = ctypes.c_int(), ctypes.c_int()
    _check(lib().ebv_get_batched_tuning(handle(), int(dtype), int(bool(mixed)), ctypes.byref(w), ctypes.byref(o)),
           "ebv_get_batched_tuning")
    return w.value, o.value


def set_wait_limit(spins: int = 0):
    """Bounded-wait budget of the default handle (0 = the defaults; see ebv_set_wait_limit)."""
    _check(lib().ebv_set_wait_limit(handle(), int(spins)), "ebv_set_wait_limit")


def profile_update_enable(max_launches: int):
    """Bracket the next single-system block-step launches with HIP events (0 = off)."""
    _check(lib().ebv_profile_update_enable(handle(), int(max_launches)), "ebv_profile_update_enable")


def profile_update_read():
    """(summed ms, launches, summed algorithmic flops) of the bracketed block-step launches."""
    ms, n, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    _check(lib().ebv_profile_update_read(handle(), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl)),
           "ebv_profile_update_read")
    return ms.value, n.value, fl.value


def check_info(info: torch.Tensor, what: str):
    """Raise on a nonzero device info (synchronizes): k > 0 a zero pivot at
    step k, negative a bounded wait that gave up (-status)."""
    v = info.detach().to("cpu").reshape(-1)
    bad = torch.nonzero(v).reshape(-1)
    if bad.numel():
        k = int(bad[0])
        code = int(v[k])
        if code < 0:
            raise EbvError(f"{what}: a bounded wait gave up (status {-code}) in system {k}; results are invalid")
        raise EbvError(f"{what}: zero pivot at elimination step {code} in system {k}")


# ----------------------------------------------------------------- dense ---
def lu_factor_(A: torch.Tensor, info: Optional[torch.Tensor] = None,
               ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """In-place Doolittle LU of A (n x n, or batch x n x n). Returns info (int32[batch])."""
    _need_gpu(A)
    batched = A.dim() == 3
    batch = A.shape[0] if batched else 1
    n = A.shape[-1]
    assert A.shape[-2] == n
    if info is None:
        info = torch.zeros(batch, dtype=torch.int32, device=A.device)
    if ws is None:
        ws = workspace(OP_FACTOR, _dt(A), n, 0, batch, A.device)
    w, wb = _ws_args(ws)
    rc = lib().ebv_lu_factor(handle(), _dt(A), n, _p(A), n, batch, n * n, _p(info), w, wb, _stream())
    _check(rc, "ebv_lu_factor")
    return info


def lu_factor(A: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
    LU = A.clone()
    info = lu_factor_(LU)
    return LU, info


def lu_solve_(LU: torch.Tensor, B: torch.Tensor, ws: Optional[torch.Tensor] = None,
              info: Optional[torch.Tensor] = None) -> torch.Tensor:
    """In-place solve: B (n x nrhs, or batch x n x nrhs) <- A^{-1} B from the packed factor.
    info (int32[batch], optional) receives 0 or -status."""
    _need_gpu(LU, B)
    batched = LU.dim() == 3
    batch = LU.shape[0] if batched else 1
    n = LU.shape[-1]
    nrhs = B.shape[-1]
    if ws is None:
        ws = workspace(OP_SOLVE, _dt(LU), n, nrhs, batch, LU.device)
    w, wb = _ws_args(ws)
    rc = lib().ebv_lu_solve(handle(), _dt(LU), n, nrhs, _p(LU), n, _p(B), nrhs, batch, n * n, n * nrhs, _p(info),
                            w, wb, _stream())
    _check(rc, "ebv_lu_solve")
    return B


def lu_solve(LU: torch.Tensor, B: torch.Tensor, check: bool = True) -> torch.Tensor:
    """X = A^{-1} B from the packed factor; check: raise if a bounded wait gave up (synchronizes)."""
    batch = LU.shape[0] if LU.dim() == 3 else 1
    info = torch.zeros(batch, dtype=torch.int32, device=LU.device) if check else None
    X = lu_solve_(LU, B.clone(), info=info)
    if check:
        check_info(info, "ebv_lu_solve")
    return X


def lu_factor_solve_(A: torch.Tensor, B: torch.Tensor, info: Optional[torch.Tensor] = None,
                     ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """In place: A (n x n) <- L\\U and B (n x nrhs) <- A^{-1} B, the forward
    substitution carried inside the factorization. Returns info (int32[1])."""
    _need_gpu(A, B)
    n, nrhs = A.shape[0], B.shape[-1]
    assert A.dim() == 2 and A.shape[1] == n and B.shape[0] == n
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    if ws is None:
        ws = workspace(OP_FACTOR_SOLVE, _dt(A), n, nrhs, 1, A.device)
    w, wb = _ws_args(ws)
    rc = lib().ebv_lu_factor_solve(handle(), _dt(A), n, nrhs, _p(A), n, _p(B), nrhs, _p(info), w, wb, _stream())
    _check(rc, "ebv_lu_factor_solve")
    return info


# --------------------------------------------------------------- skyline ---
class Skyline:
    """A skyline (profile) system on the device (layout of inputs.skyline):
    the profile arrays f, g on the host and the device, the offsets rp, cp,
    and the values AL (lower, by rows) and AU (upper with the diagonal, by
    columns) as device tensors; factor_() and solve() run in the library."""

    def __init__(self, f, rp, AL, g, cp, AU, device="cuda"):
        self.f_host = np.ascontiguousarray(f, dtype=np.int32)
        self.g_host = np.ascontiguousarray(g, dtype=np.int32)
        self.n = len(self.f_host)
        self.f = torch.from_numpy(self.f_host).to(device)
        self.g = torch.from_numpy(self.g_host).to(device)
        self.rp = torch.from_numpy(np.ascontiguousarray(rp, dtype=np.int64)).to(device)
        self.cp = torch.from_numpy(np.ascontiguousarray(cp, dtype=np.int64)).to(device)
        self.AL = AL if torch.is_tensor(AL) else torch.from_numpy(np.ascontiguousarray(AL)).to(device)
        self.AU = AU if torch.is_tensor(AU) else torch.from_numpy(np.ascontiguousarray(AU)).to(device)
        hp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self._fh, self._gh = hp(self.f_host), hp(self.g_host)
        nb = lib().ebv_skyline_workspace_size(self.n, self._fh, self._gh)
        self.ws = torch.empty(nb + 256, dtype=torch.uint8, device=device) if nb else None

    def factor_(self, info: Optional[torch.Tensor] = None) -> torch.Tensor:
        """In place: AL <- L, AU <- U. Returns info (int32[1])."""
        if info is None:
            info = torch.zeros(1, dtype=torch.int32, device=self.AL.device)
        w, wb = _ws_args(self.ws)
        _check(lib().ebv_lu_factor_skyline(handle(), self.n, self._fh, self._gh, _p(self.f), _p(self.rp),
                                           _p(self.AL), _p(self.g), _p(self.cp), _p(self.AU), _p(info), w, wb,
                                           _stream()), "ebv_lu_factor_skyline")
        return info

    def solve_(self, B: torch.Tensor) -> torch.Tensor:
        """In place: B (n x nrhs) <- X, with the factors from factor_()."""
        _need_gpu(B)
        w, wb = _ws_args(self.ws)
        _check(lib().ebv_lu_solve_skyline(handle(), self.n, B.shape[1], self._fh, self._gh, _p(self.f),
                                          _p(self.rp), _p(self.AL), _p(self.g), _p(self.cp), _p(self.AU), _p(B),
                                          B.stride(0), w, wb, _stream()), "ebv_lu_solve_skyline")
        return B


# -------------------------------------------------------------- inverse ---
def lu_inverse(LU: torch.Tensor, out: Optional[torch.Tensor] = None,
               ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Explicit inverse A^{-1} from the factors of lu_factor (the product form
    of Eq. 4-c)."""
    _need_gpu(LU)
    n = LU.shape[0]
    assert LU.dim() == 2 and LU.shape[1] == n
    if out is None:
        out = torch.empty_like(LU)
    if ws is None:
        ws = workspace(OP_INVERSE, _dt(LU), n, 0, 1, LU.device)
    w, wb = _ws_args(ws)
    _check(lib().ebv_lu_inverse(handle(), _dt(LU), n, _p(LU), LU.stride(0), _p(out), out.stride(0), w, wb, _stream()),
           "ebv_lu_inverse")
    return out


def inverse(A: torch.Tensor) -> torch.Tensor:
    """A^{-1} of a dense system: factor a copy, then the explicit inverse."""
    LU = A.clone()
    info = lu_factor_(LU)
    check_info(info, "inverse")
    return lu_inverse(LU)


# ------------------------------------------------------ transfer pipeline ---
class Pipeline:
    """Factor + solve of host-resident systems with the transfers overlapped
    (ebv_pipeline_factor_solve): two device slots and three streams of its
    own (default priority).  run() only enqueues; synchronize() waits.
    The overlap needs the three streams on distinct hardware queues: HIP
    assigns queues to streams round-robin (four per process by default), so
    create the Pipeline before other streams where the overlap matters."""

    def __init__(self, n: int, nrhs: int, dtype=torch.float64, device="cuda"):
        self.n, self.nrhs, self.dtype = n, nrhs, dtype
        self.dA = [torch.empty((n, n), dtype=dtype, device=device) for _ in range(2)]
        self.dB = [torch.empty((n, max(nrhs, 1)), dtype=dtype, device=device) for _ in range(2)]
        self.ws = workspace(OP_FACTOR_SOLVE, _dt(self.dA[0]), n, nrhs, 1, device)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(3)]

    def run(self, A_host, B_host, info: Optional[torch.Tensor] = None):
        """A_host, B_host: lists of pinned CPU tensors (n x n, n x nrhs);
        B_host[s] receives X_s (A_host[s] the factors when nrhs = 0)."""
        count = len(A_host)
        for a in A_host:
            assert a.dtype == self.dtype and a.shape == (self.n, self.n) and a.is_contiguous() and not a.is_cuda
        arr = lambda ts: (ctypes.c_void_p * max(len(ts), 1))(*[t.data_ptr() for t in ts])
        ah = arr(A_host)
        bh = arr(B_host) if self.nrhs > 0 else None
        da = (ctypes.c_void_p * 2)(*[t.data_ptr() for t in self.dA])
        db = (ctypes.c_void_p * 2)(*[t.data_ptr() for t in self.dB])
        w, wb = _ws_args(self.ws)
        cs, ci, co = (s.cuda_stream for s in self.streams)
        # the slots and the workspace follow the caller's earlier work
        for s in self.streams:
            s.wait_stream(torch.cuda.current_stream())
        rc = lib().ebv_pipeline_factor_solve(handle(), _dt(self.dA[0]), count, self.n, self.nrhs, ah, bh, da, db,
                                             _p(info), w, wb, cs, ci, co)
        _check(rc, "ebv_pipeline_factor_solve")
        for s in self.streams:
            torch.cuda.current_stream().wait_stream(s)

    def synchronize(self):
        for s in self.streams:
            s.synchronize()


# ------------------------------------------------------------------ band ---
def lu_factor_band_(AB: torch.Tensor, kl: int, ku: int, info: Optional[torch.Tensor] = None,
                    ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """In-place band LU of row-wise band storage AB[i, j - i + kl] (n x (kl+ku+1), float64)."""
    _need_gpu(AB)
    n, wd = AB.shape
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=AB.device)
    if ws is None:
        ws = workspace(OP_BAND, F64, n, 0, 1, AB.device)
    w, wb = _ws_args(ws)
    _check(lib().ebv_lu_factor_band(handle(), n, kl, ku, _p(AB), wd, _p(info), w, wb, _stream()),
           "ebv_lu_factor_band")
    return info


def lu_solve_band_(LUB: torch.Tensor, kl: int, ku: int, B: torch.Tensor, info: Optional[torch.Tensor] = None,
                   ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    _need_gpu(LUB, B)
    n, wd = LUB.shape
    nrhs = B.shape[-1]
    if ws is None:
        ws = workspace(OP_BAND_SOLVE, F64, n, nrhs, 1, LUB.device)
    w, wb = _ws_args(ws)
    _check(lib().ebv_lu_solve_band(handle(), n, kl, ku, nrhs, _p(LUB), wd, _p(B), nrhs, _p(info), w, wb, _stream()),
           "ebv_lu_solve_band")
    return B


# --------------------------------------------------------------- batched ---
def batched_order(ns, policy: int = ORDER_EBV) -> np.ndarray:
    """Batch schedule (host) for an order policy; ORDER_EBV: costliest system
    first, then the cheapest, ..."""
    ns = np.ascontiguousarray(ns, dtype=np.int32)
    order = np.empty_like(ns)
    _check(lib().ebv_batched_order(int(policy), len(ns), ns.ctypes.data_as(ctypes.c_void_p),
                                   order.ctypes.data_as(ctypes.c_void_p)), "ebv_batched_order")
    return order


class RaggedBatch:
    """Device-side description of a packed ragged batch (sizes, offsets, order).
    ebv_order: True takes the EbV order, False index order; policy (ORDER_*)
    overrides both."""

    def __init__(self, ns, offA, offB, device="cuda", ebv_order: bool = True, policy: Optional[int] = None):
        ns = np.ascontiguousarray(ns, dtype=np.int32)
        self.count = len(ns)
        self.ns_host = ns
        self.n = torch.from_numpy(ns).to(device)
        self.offA = torch.from_numpy(np.ascontiguousarray(offA, dtype=np.int64)).to(device)
        self.offB = torch.from_numpy(np.ascontiguousarray(offB, dtype=np.int64)).to(device)
        self.totA = int((np.asarray(offA, dtype=np.int64) + ns.astype(np.int64) ** 2).max()) if self.count else 0
        self.totB = int((np.asarray(offB, dtype=np.int64) + ns.astype(np.int64)).max()) if self.count else 0
        if policy is None:
            policy = ORDER_EBV if ebv_order else ORDER_INDEX
        self.policy = policy
        self.order = None if policy == ORDER_INDEX else torch.from_numpy(batched_order(ns, policy)).to(device)
        self.device = device


def uniform_ragged(batch: int, n: int, device="cuda") -> RaggedBatch:
    """A batch of `batch` n x n systems stored back to back (n*n and n elements
    apart, one right-hand side each) described as a packed ragged batch, so
    that factor_solve_batched_ runs it (equal sizes: index order)."""
    ns = np.full(batch, n, dtype=np.int32)
    k = np.arange(batch, dtype=np.int64)
    return RaggedBatch(ns, k * n * n, k * n, device=device, policy=ORDER_INDEX)


def factor_solve_batched_(rb: RaggedBatch, A: torch.Tensor, B: Optional[torch.Tensor], mixed: bool = False,
                          max_iter: int = 10, tol: float = 1e-12, info: Optional[torch.Tensor] = None,
                          iters: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                          wg_per_cu: int = 0):
    """Factor + solve every system of a packed ragged batch in one persistent launch.
    Plain: A <- LU and B <- X in A's dtype.  mixed: float factor of each system
    in the workspace, A unchanged, B <- X refined in double."""
    _need_gpu(A, B)
    dt = _dt(A)
    if info is None:
        info = torch.zeros(rb.count, dtype=torch.int32, device=A.device)
    if mixed and iters is None:
        iters = torch.zeros(rb.count, dtype=torch.int32, device=A.device)
    if ws is None:
        ws = workspace(OP_BATCHED_MIXED if mixed else OP_BATCHED, dt, rb.totA, rb.totB, rb.count, A.device)
    w, wb = _ws_args(ws)
    rc = lib().ebv_lu_factor_batched(handle(), dt, rb.count, _p(rb.n), _p(rb.offA), _p(A), A.numel(), _p(rb.offB), _p(B),
                                     0 if B is None else B.numel(), _p(rb.order), _p(info), int(mixed),
                                     int(max_iter), float(tol), _p(iters), int(wg_per_cu), w, wb, _stream())
    _check(rc, "ebv_lu_factor_batched")
    return info, iters


# --------------------------------------------------------------- adjoint ---
def lu_solve_adjoint(LU: torch.Tensor, X: torch.Tensor, Xbar: torch.Tensor, want_abar: bool = True,
                     ws: Optional[torch.Tensor] = None, info: Optional[torch.Tensor] = None):
    """Reverse-mode of X = A^{-1} B: returns (Bbar, Abar) = (A^{-T} Xbar, -Bbar X^T).
    info (int32[batch], optional) receives 0 or -status."""
    _need_gpu(LU, X, Xbar)
    batched = LU.dim() == 3
    batch = LU.shape[0] if batched else 1
    n = LU.shape[-1]
    nrhs = Xbar.shape[-1]
    Bbar = Xbar.clone()
    Abar = torch.empty_like(LU) if want_abar else None
    if ws is None:
        ws = workspace(OP_ADJOINT, _dt(LU), n, nrhs, batch, LU.device)
    w, wb = _ws_args(ws)
    rc = lib().ebv_lu_solve_adjoint(handle(), _dt(LU), n, nrhs, _p(LU), n, _p(X), nrhs, _p(Bbar), nrhs, _p(Abar), n,
                                    batch, n * n, n * nrhs, n * nrhs, n * n, _p(info), w, wb, _stream())
    _check(rc, "ebv_lu_solve_adjoint")
    return Bbar, Abar


class EbvSolve(torch.autograd.Function):
    """X = A^{-1} B with the EbV factor; backward reuses the factor (U^T and L^T
    solves, Abar = -Bbar X^T) through the library's adjoint entry point.
    Both directions check the device info (a synchronization) and raise on a
    zero pivot or a bounded wait that gave up."""

    @staticmethod
    def forward(ctx, A, B):
        LU = A.detach().contiguous().clone()
        X = B.detach().contiguous().clone()
        if LU.dim() == 2:
            info = lu_factor_solve_(LU, X)
        elif X.dim() == 3 and X.shape[-1] == 1:
            # one right-hand side per system: the persistent batched launch,
            # the forward substitution fused into each factorization
            info, _ = factor_solve_batched_(uniform_ragged(LU.shape[0], LU.shape[-1], LU.device), LU.view(-1),
                                            X.view(-1))
        else:
            info = lu_factor_(LU)
            info2 = torch.zeros_like(info)
            lu_solve_(LU, X, info=info2)
            info = torch.where(info2 != 0, info2, info)
        check_info(info, "EbvSolve.forward")
        ctx.save_for_backward(LU, X)
        return X

    @staticmethod
    def backward(ctx, Xbar):
        LU, X = ctx.saved_tensors
        batch = LU.shape[0] if LU.dim() == 3 else 1
        info = torch.zeros(batch, dtype=torch.int32, device=LU.device)
        Bbar, Abar = lu_solve_adjoint(LU, X, Xbar.contiguous(), want_abar=ctx.needs_input_grad[0], info=info)
        check_info(info, "EbvSolve.backward")
        return Abar, Bbar


def solve(A: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
    """Differentiable X = A^{-1} B (A: n x n or batch x n x n)."""
    return EbvSolve.apply(A, B)


# ------------------------------------------------------- mixed precision ---
def solve_mixed(A: torch.Tensor, B: torch.Tensor, tol: float = 1e-12, max_iter: int = 10,
                ws: Optional[torch.Tensor] = None):
    """Float factor + double refinement to the forward-error bound tol.
    Returns (X, iters, ferr, info) as device tensors (ferr: the bound per column)."""
    _need_gpu(A, B)
    n = A.shape[0]
    nrhs = B.shape[-1]
    X = torch.empty_like(B)
    iters = torch.empty(nrhs, dtype=torch.int32, device=A.device)
    ferr = torch.empty(nrhs, dtype=torch.float64, device=A.device)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    if ws is None:
        ws = workspace(OP_MIXED, F64, n, nrhs, 1, A.device)
    w, wb = _ws_args(ws)
    rc = lib().ebv_lu_solve_mixed(handle(), n, nrhs, _p(A), n, _p(B), nrhs, _p(X), nrhs, int(max_iter), float(tol),
                                  _p(iters), _p(ferr), _p(info), w, wb, _stream())
    _check(rc, "ebv_lu_solve_mixed")
    return X, iters, ferr, info
