"""Multi-scale low-rank decomposition on MI355X: Python binding of libmsld.so.

Argument marshalling only: every step of the ADMM / block-wise SVT iteration runs
in the library's HIP kernels. PyTorch supplies device memory and the stream.
There is no CPU fallback: without the built library (``python -m
paper_1507_08751_amd.build``) every call raises.

A solver runs each scale on a HIP stream of its own (a batch: each shape class, a
server: each active class). Streams only run side by side on hardware queues of their
own, so set ``GPU_MAX_HW_QUEUES`` (HIP's default is 4 per process) to 16 or so before
HIP initialises, i.e. before torch is imported.
"""
from __future__ import annotations

import ctypes
import math
import os

__all__ = ["load", "Solver", "Batch", "Server", "solve", "bsvt", "cycle_shift", "default_lambda",
           "MAX_SCALES", "TIERS", "MsldError", "KIND_BLOCK", "KIND_NOISE"]

MAX_SCALES = 16
TIERS = {0: "1x1", 1: "register", 2: "lds", 3: "panel", 4: "lowrank", 5: "lowrank_small",
         6: "noise"}
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmsld.so")

_lib = None


class MsldError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = int(status)
        msg = _lib.msld_status_string(self.status).decode() if _lib else str(status)
        super().__init__(f"{what}: {msg}" if what else msg)


class Params(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("N", ctypes.c_int32), ("L", ctypes.c_int32),
                ("block_m", ctypes.c_int32 * MAX_SCALES),
                ("block_n", ctypes.c_int32 * MAX_SCALES),
                ("lambda_", ctypes.c_float * MAX_SCALES),
                ("rho", ctypes.c_float), ("max_iters", ctypes.c_int32),
                ("tol", ctypes.c_float), ("check_every", ctypes.c_int32),
                ("cycle_spin", ctypes.c_int32), ("lowrank_min", ctypes.c_int32),
                ("shift_seed", ctypes.c_uint64), ("kind", ctypes.c_int32 * MAX_SCALES),
                ("spin_count", ctypes.c_int32), ("image_w", ctypes.c_int32),
                ("patch_w", ctypes.c_int32 * MAX_SCALES), ("fork_mode", ctypes.c_int32)]

KIND_BLOCK = 0
KIND_NOISE = 1
KIND_SPATIAL = 2


class TuneResult(ctypes.Structure):
    _fields_ = [("tier", ctypes.c_int32), ("lds_cap", ctypes.c_int32),
                ("lrs_wide", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("us_per_block", ctypes.c_float), ("us_default", ctypes.c_float)]


class Result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("primal_resid", ctypes.c_double), ("dual_resid", ctypes.c_double),
                ("live", ctypes.c_uint64 * MAX_SCALES),
                ("sweeps", ctypes.c_uint64 * MAX_SCALES),
                ("rank", ctypes.c_uint64 * MAX_SCALES),
                ("certified", ctypes.c_uint64 * MAX_SCALES),
                ("fail_coupling", ctypes.c_uint64 * MAX_SCALES),
                ("fail_bound", ctypes.c_uint64 * MAX_SCALES),
                ("polar", ctypes.c_uint64 * MAX_SCALES),
                ("polar_steps", ctypes.c_uint64 * MAX_SCALES),
                ("undecided", ctypes.c_uint64 * MAX_SCALES),
                ("cw_certified", ctypes.c_uint64 * MAX_SCALES),
                ("gram_certified", ctypes.c_uint64 * MAX_SCALES)]


EXPORTS = {
    "msld_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_void_p)]),
    "msld_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_void_p, ctypes.POINTER(Result)]),
    "msld_bsvt": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_float, ctypes.c_int32,
                                 ctypes.c_int32]),
    "msld_free": (None, [ctypes.c_void_p]),
    "msld_bsvt_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_float, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p]),
    "msld_set_mask": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "msld_set_graph": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "msld_autotune": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_void_p]),
    "msld_autotune_clear": (None, []),
    "msld_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Params)]),
    "msld_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "msld_default_lambda": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]),
    "msld_cycle_shift": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "msld_device_shifts": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32)]),
    "msld_scale_tier": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "msld_reset": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "msld_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                 ctypes.c_void_p, ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_double)]),
    "msld_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Result)]),
    "msld_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(Params), ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "msld_batch_classes": (ctypes.c_int32, [ctypes.c_void_p]),
    "msld_batch_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Result)]),
    "msld_batch_free": (None, [ctypes.c_void_p]),
    "msld_server_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_size_t, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "msld_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Params),
                                          ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_int64]),
    "msld_server_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "msld_server_free": (None, [ctypes.c_void_p]),
    "msld_server_class_bytes": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_size_t)]),
    "msld_profile_begin": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "msld_profile_end": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int32)]),
}


def load(path: str | None = None):
    """Load libmsld.so (built in-tree). Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing; build it with "
                           "`python -m paper_1507_08751_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status, what):
    if status != 0:
        raise MsldError(status, what)


def default_lambda(M, N, m, n) -> float:
    lib = load()
    out = ctypes.c_float()
    _check(lib.msld_default_lambda(M, N, m, n, ctypes.byref(out)), "msld_default_lambda")
    return float(out.value)


def cycle_shift(seed, k, i, m, n):
    lib = load()
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(lib.msld_cycle_shift(seed, k, i, m, n, ctypes.byref(a), ctypes.byref(b)),
           "msld_cycle_shift")
    return a.value, b.value


def make_params(M, N, ladder, lam=None, rho=1.0, iters=100, tol=0.0, check_every=1,
                cycle_spin=False, seed=0, lowrank_min=0, kinds=None, spin_count=0,
                image_w=0, patch_w=None, fork_mode=0) -> Params:
    if len(ladder) < 1 or len(ladder) > MAX_SCALES:
        raise ValueError("ladder must have 1..16 scales")
    p = Params()
    p.M, p.N, p.L = int(M), int(N), len(ladder)
    for i, (m, n) in enumerate(ladder):
        p.block_m[i], p.block_n[i] = int(m), int(n)
        p.lambda_[i] = float(lam[i]) if lam is not None else 0.0
    p.rho = float(rho)
    p.max_iters = int(iters)
    p.tol = float(tol)
    p.check_every = int(check_every)
    p.cycle_spin = 1 if cycle_spin else 0
    p.shift_seed = int(seed) & ((1 << 64) - 1)
    p.lowrank_min = int(lowrank_min)
    for i in range(len(ladder)):
        p.kind[i] = int(kinds[i]) if kinds is not None else KIND_BLOCK
    p.spin_count = int(spin_count)
    p.image_w = int(image_w)
    for i in range(len(ladder)):
        p.patch_w[i] = int(patch_w[i]) if patch_w is not None else 0
    p.fork_mode = int(fork_mode)
    return p


def workspace_bytes(M, N, ladder, **kw) -> int:
    lib = load()
    p = make_params(M, N, ladder, **kw)
    return int(lib.msld_workspace_bytes(ctypes.byref(p)))


def _stream_ptr(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Solver:
    """One planned decomposition problem (msld_create). Reusable across solves."""

    def __init__(self, M, N, ladder, lam=None, rho=1.0, iters=100, tol=0.0, check_every=1,
                 cycle_spin=False, seed=0, device=None, lowrank_min=0, kinds=None,
                 spin_count=0, image_w=0, patch_w=None, fork_mode=0):
        import torch
        self._torch = torch
        lib = load()
        self.M, self.N = int(M), int(N)
        self.ladder = [(int(m), int(n)) for (m, n) in ladder]
        self.L = len(self.ladder)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.params = make_params(M, N, ladder, lam, rho, iters, tol, check_every,
                                  cycle_spin, seed, lowrank_min, kinds, spin_count, image_w,
                                  patch_w, fork_mode)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.msld_create(ctypes.byref(self.params), _stream_ptr(torch, self.device),
                                 ctypes.byref(h))
        _check(st, "msld_create")
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.msld_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tier(self, i) -> int:
        return int(self._lib.msld_scale_tier(self._h, i))

    def solve(self, Y, out=None, info=True):
        """Run the ADMM on Y (M x N float32 device tensor); returns (Z [L,M,N], info)."""
        torch = self._torch
        if Y.dtype != torch.float32 or not Y.is_cuda or Y.dim() != 2:
            raise ValueError("Y must be a 2-D float32 device tensor")
        if tuple(Y.shape) != (self.M, self.N) or Y.stride(1) != 1:
            raise ValueError("Y has the wrong shape or a non-unit column stride")
        if out is None:
            out = torch.empty((self.L, self.M, self.N), dtype=torch.float32, device=Y.device)
        if out.shape != (self.L, self.M, self.N) or not out.is_contiguous():
            raise ValueError("out must be a contiguous (L, M, N) float32 tensor")
        res = Result()
        with torch.cuda.device(Y.device):
            st = self._lib.msld_solve(self._h, ctypes.c_void_p(Y.data_ptr()),
                                      ctypes.c_int64(Y.stride(0)),
                                      ctypes.c_void_p(out.data_ptr()),
                                      ctypes.byref(res) if info else None)
        _check(st, "msld_solve")
        if not info:
            return out, None
        return out, {"iters": res.iters, "primal_resid": res.primal_resid,
                     "dual_resid": res.dual_resid,
                     "live": list(res.live)[:self.L], "sweeps": list(res.sweeps)[:self.L],
                     "rank": list(res.rank)[:self.L],
                     "certified": list(res.certified)[:self.L],
                     "fail_coupling": list(res.fail_coupling)[:self.L],
                     "fail_bound": list(res.fail_bound)[:self.L],
                "polar": list(res.polar)[:self.L],
                "polar_steps": list(res.polar_steps)[:self.L],
                "undecided": list(res.undecided)[:self.L],
                "cw_certified": list(res.cw_certified)[:self.L],
                "gram_certified": list(res.gram_certified)[:self.L]}

    def _check_yz(self, Y, Z):
        torch = self._torch
        if Y.dtype != torch.float32 or not Y.is_cuda or tuple(Y.shape) != (self.M, self.N) \
                or Y.stride(1) != 1:
            raise ValueError("Y must be an (M, N) float32 device tensor with unit column stride")
        if Z.dtype != torch.float32 or tuple(Z.shape) != (self.L, self.M, self.N) \
                or not Z.is_contiguous():
            raise ValueError("Z must be a contiguous (L, M, N) float32 device tensor")

    def reset(self, Z):
        with self._torch.cuda.device(Z.device):
            _check(self._lib.msld_reset(self._h, ctypes.c_void_p(Z.data_ptr())), "msld_reset")

    def step(self, Y, Z, count=1, resid=False):
        """Run `count` more iterations on the iterate Z; returns r of the last one or None."""
        self._check_yz(Y, Z)
        r = ctypes.c_double(-1.0)
        with self._torch.cuda.device(Y.device):
            st = self._lib.msld_step(self._h, ctypes.c_void_p(Y.data_ptr()),
                                     ctypes.c_int64(Y.stride(0)), ctypes.c_void_p(Z.data_ptr()),
                                     int(count), ctypes.byref(r) if resid else None)
        _check(st, "msld_step")
        return r.value if resid else None

    def stats(self):
        res = Result()
        with self._torch.cuda.device(self.device):
            _check(self._lib.msld_stats(self._h, ctypes.byref(res)), "msld_stats")
        return {"iters": res.iters, "live": list(res.live)[:self.L],
                "sweeps": list(res.sweeps)[:self.L], "rank": list(res.rank)[:self.L],
                "certified": list(res.certified)[:self.L],
                "fail_coupling": list(res.fail_coupling)[:self.L],
                "fail_bound": list(res.fail_bound)[:self.L],
                "polar": list(res.polar)[:self.L],
                "polar_steps": list(res.polar_steps)[:self.L],
                "undecided": list(res.undecided)[:self.L],
                "cw_certified": list(res.cw_certified)[:self.L],
                "gram_certified": list(res.gram_certified)[:self.L]}

    def set_graph(self, enable=True):
        """Allow (default) or forbid replaying iterations from captured HIP graphs;
        returns whether iterations will be replayed from graphs (msld_set_graph)."""
        with self._torch.cuda.device(self.device):
            r = int(self._lib.msld_set_graph(self._h, 1 if enable else 0))
        if r < 0:
            _check(r, "msld_set_graph")
        return r == 1

    def set_mask(self, mask):
        """Observed-entry mask (M x N bool / uint8 device tensor, kept alive by the
        solver) for the masked data consistency of Sec. 10; None clears it."""
        torch = self._torch
        if mask is None:
            self._mask = None
            _check(self._lib.msld_set_mask(self._h, None, 0), "msld_set_mask")
            return
        if tuple(mask.shape) != (self.M, self.N) or not mask.is_cuda:
            raise ValueError("mask must be an (M, N) device tensor")
        m = mask.to(torch.uint8).contiguous()
        self._mask = m
        _check(self._lib.msld_set_mask(self._h, m.data_ptr(), self.N), "msld_set_mask")

    def profile_begin(self, max_iters):
        _check(self._lib.msld_profile_begin(self._h, int(max_iters)), "msld_profile_begin")

    def profile_end(self):
        ms = (ctypes.c_double * (4 * (self.L + 1) + self.L))()
        rl = (ctypes.c_int64 * self.L)()
        n = ctypes.c_int32()
        with self._torch.cuda.device(self.device):
            _check(self._lib.msld_profile_end(self._h, ms, rl, ctypes.byref(n)),
                   "msld_profile_end")
        per = [list(ms[4 * i:4 * i + 4]) for i in range(self.L)]
        return {"scale_ms": per, "consensus_ms": ms[4 * self.L],
                "stream_ms": ms[4 * self.L + 1], "round_launches": list(rl), "iters": n.value,
                "gram_ms": list(ms[4 * (self.L + 1):4 * (self.L + 1) + self.L])}

    def bsvt(self, scale, V, tau, shift=(0, 0), out=None):
        """Z = Shift_{-s}(BSVT_tau(Shift_s(V))) with scale `scale`'s block shape."""
        torch = self._torch
        if V.dtype != torch.float32 or not V.is_cuda or tuple(V.shape) != (self.M, self.N) \
                or not V.is_contiguous():
            raise ValueError("V must be a contiguous (M, N) float32 device tensor")
        if out is None:
            out = torch.empty_like(V)
        with torch.cuda.device(V.device):
            st = self._lib.msld_bsvt(self._h, int(scale), ctypes.c_void_p(V.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), float(tau),
                                     int(shift[0]), int(shift[1]))
        _check(st, "msld_bsvt")
        return out

    def device_shifts(self, k0, count):
        buf = (ctypes.c_int32 * (2 * self.L * count))()
        with self._torch.cuda.device(self.device):
            _check(self._lib.msld_device_shifts(self._h, k0, count, buf), "msld_device_shifts")
        import numpy as np
        return np.array(buf, dtype=np.int64).reshape(count, self.L, 2)


class Batch:
    """Many independent decompositions solved together (msld_batch_*). `problems` is a
    list of dicts with keys M, N, ladder and optional lam, rho, iters, tol,
    check_every, cycle_spin, seed, lowrank_min, kinds, spin_count, image_w, patch_w."""

    def __init__(self, problems, device=None):
        import torch
        self._torch = torch
        self._lib = load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        n = len(problems)
        arr = (Params * n)()
        self.shapes = []
        for i, pr in enumerate(problems):
            arr[i] = make_params(pr["M"], pr["N"], pr["ladder"], pr.get("lam"),
                                 pr.get("rho", 1.0), pr.get("iters", 100), pr.get("tol", 0.0),
                                 pr.get("check_every", 1), pr.get("cycle_spin", False),
                                 pr.get("seed", 0), pr.get("lowrank_min", 0),
                                 pr.get("kinds"), pr.get("spin_count", 0),
                                 pr.get("image_w", 0), pr.get("patch_w"))
            self.shapes.append((len(pr["ladder"]), pr["M"], pr["N"]))
        self.n = n
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self._lib.msld_batch_create(n, arr, _stream_ptr(torch, self.device),
                                               ctypes.byref(h)), "msld_batch_create")
        self._h = h

    @property
    def classes(self):
        return int(self._lib.msld_batch_classes(self._h))

    def solve(self, Ys, outs=None, info=True):
        torch = self._torch
        n = self.n
        if outs is None:
            outs = [torch.empty(sh, dtype=torch.float32, device=self.device) for sh in self.shapes]
        ys = (ctypes.c_void_p * n)(*[y.data_ptr() for y in Ys])
        lds = (ctypes.c_int64 * n)(*[y.stride(0) for y in Ys])
        zs = (ctypes.c_void_p * n)(*[z.data_ptr() for z in outs])
        res = (Result * n)() if info else None
        with torch.cuda.device(self.device):
            _check(self._lib.msld_batch_solve(self._h, ys, lds, zs, res), "msld_batch_solve")
        infos = None
        if info:
            infos = [{"iters": r.iters, "primal_resid": r.primal_resid, "status": r.status}
                     for r in res]
        return outs, infos

    def close(self):
        if getattr(self, "_h", None):
            self._lib.msld_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop of the library (msld_server_*).

    submit() queues a decomposition of a device tensor Y into a caller-provided (or
    new) Z tensor; step() admits, advances every active request by one iteration and
    returns the requests that finished: [(id, iters, resid, status)]."""

    def __init__(self, max_active=16, hbm_budget=64 << 30, num_streams=8, device=None):
        import torch
        self._torch = torch
        self._lib = load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self._lib.msld_server_create(int(max_active), int(hbm_budget),
                                                int(num_streams), ctypes.byref(h)),
                   "msld_server_create")
        self._h = h
        self._keep = {}
        self._cap = 256
        self._ids = (ctypes.c_int64 * self._cap)()
        self._its = (ctypes.c_int32 * self._cap)()
        self._res = (ctypes.c_double * self._cap)()
        self._sts = (ctypes.c_int32 * self._cap)()

    def submit(self, request_id, Y, ladder, lam=None, rho=1.0, iters=300, tol=1e-4,
               check_every=1, cycle_spin=False, seed=0, lowrank_min=0, out=None):
        torch = self._torch
        M, N = Y.shape
        if out is None:
            out = torch.empty((len(ladder), M, N), dtype=torch.float32, device=Y.device)
        p = make_params(M, N, ladder, lam, rho, iters, tol, check_every, cycle_spin, seed,
                        lowrank_min)
        with torch.cuda.device(self.device):
            _check(self._lib.msld_server_submit(self._h, ctypes.byref(p),
                                                ctypes.c_void_p(Y.data_ptr()),
                                                ctypes.c_int64(Y.stride(0)),
                                                ctypes.c_void_p(out.data_ptr()),
                                                ctypes.c_int64(int(request_id))),
                   "msld_server_submit")
        self._keep[int(request_id)] = (Y, out)
        return out

    def step(self):
        nd, na, nq = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        with self._torch.cuda.device(self.device):
            _check(self._lib.msld_server_step(self._h, self._ids, self._its, self._res,
                                              self._sts, self._cap, ctypes.byref(nd),
                                              ctypes.byref(na), ctypes.byref(nq)),
                   "msld_server_step")
        out = []
        for k in range(nd.value):
            rid = int(self._ids[k])
            Y, Z = self._keep.pop(rid, (None, None))
            out.append((rid, int(self._its[k]), float(self._res[k]), int(self._sts[k]), Z))
        self.active, self.queued = na.value, nq.value
        return out

    @staticmethod
    def class_bytes(M, N, ladder, max_active, lam=None, rho=1.0, iters=300, tol=1e-4,
                    check_every=1, cycle_spin=False, seed=0, lowrank_min=0):
        """HBM bytes a server with this max_active charges its budget for the class of
        an M x N problem with this ladder (msld_server_class_bytes)."""
        p = make_params(M, N, ladder, lam, rho, iters, tol, check_every, cycle_spin, seed,
                        lowrank_min)
        out = ctypes.c_size_t()
        _check(load().msld_server_class_bytes(ctypes.byref(p), int(max_active),
                                              ctypes.byref(out)), "msld_server_class_bytes")
        return int(out.value)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.msld_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(Y, ladder, lam=None, rho=1.0, iters=100, tol=0.0, check_every=1,
          cycle_spin=False, seed=0, lowrank_min=0, fork_mode=0):
    """One-shot decomposition: returns (Z [L, M, N] device tensor, info dict)."""
    s = Solver(Y.shape[0], Y.shape[1], ladder, lam, rho, iters, tol, check_every,
               cycle_spin, seed, device=Y.device, lowrank_min=lowrank_min,
               fork_mode=fork_mode)
    try:
        return s.solve(Y)
    finally:
        s.close()


def bsvt(V, m, n, tau, shift=(0, 0), lowrank_min=0):
    """One block-wise SVT call on V with m x n blocks and shift s (Sec. 7 and 9)."""
    s = Solver(V.shape[0], V.shape[1], [(m, n)], iters=1, device=V.device,
               lowrank_min=lowrank_min)
    try:
        return s.bsvt(0, V.contiguous(), tau, shift)
    finally:
        s.close()


def bsvt_noalloc(V, m, n, tau, shift=(0, 0), out=None):
    """msld_bsvt_noalloc: the same block-wise SVT without a handle and without any
    device allocation by the library (its fixed device workspace is shared by every call
    on a device: do not overlap calls). Enqueued on torch's current stream."""
    import torch
    lib = load()
    if V.dtype != torch.float32 or not V.is_cuda or V.dim() != 2 or not V.is_contiguous():
        raise ValueError("V must be a contiguous 2-D float32 CUDA tensor")
    if out is None:
        out = torch.empty_like(V)
    with torch.cuda.device(V.device):
        st = lib.msld_bsvt_noalloc(V.shape[0], V.shape[1], int(m), int(n),
                                   ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   float(tau), int(shift[0]), int(shift[1]),
                                   _stream_ptr(torch, V.device))
    _check(st, "msld_bsvt_noalloc")
    return out


def autotune(m, n, device=None):
    """Time the BlockSVT launch choices for m x n blocks on the device and record the
    fastest for later plans (msld_autotune); returns the choice as a dict."""
    import torch
    lib = load()
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None \
        else torch.device(device)
    r = TuneResult()
    with torch.cuda.device(dev):
        _check(lib.msld_autotune(int(m), int(n), _stream_ptr(torch, dev), ctypes.byref(r)),
               "msld_autotune")
    return {"tier": TIERS.get(r.tier, str(r.tier)), "lds_cap": r.lds_cap,
            "lrs_wide": bool(r.lrs_wide), "candidates": r.candidates,
            "us_per_block": r.us_per_block, "us_default": r.us_default}


def autotune_clear():
    """Forget every autotuned choice (msld_autotune_clear)."""
    load().msld_autotune_clear()
