"""MI355X (gfx950) flat-window voting sparse FFT.

Thin Python binding of the C ABI declared in ``include/sfft.h``: argument
marshalling only. Every step of the transform runs in the HIP kernels of
``libsfft_mi355x.so``; torch supplies device memory and streams. There is no
CPU fallback: if the library has not been built, every call raises.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _capi
from ._capi import (SFFT_FLAG_FOLD_GATHER, SFFT_FLAG_FOLD_STRIP, SFFT_FLAG_XCD_ORDER, SFFT_FLAG_NO_RESIDUAL,  # noqa: F401,E501
                    SFFT_FLAG_MEAN_ESTIMATE, SFFT_FLAG_ITERATE, SFFT_FLAG_PHASE_LOCATION, SFFT_FLAG_FFT_TWO_PASS,
                    SFFT_FLAG_VOTE_BY_LOOP, SFFT_FLAG_VOTE_BY_PAIR, SFFT_FLAG_FUSED,
                    SfftError, check,
                    load)

__all__ = ["PlanParams", "Plan", "Batch", "Server", "host_tables", "params_describe", "load", "SfftError",
           "SFFT_FLAG_FOLD_GATHER", "SFFT_FLAG_FOLD_STRIP", "SFFT_FLAG_XCD_ORDER", "SFFT_FLAG_NO_RESIDUAL",
           "SFFT_FLAG_MEAN_ESTIMATE", "SFFT_FLAG_ITERATE", "SFFT_FLAG_PHASE_LOCATION",
           "SFFT_FLAG_FFT_TWO_PASS", "SFFT_FLAG_VOTE_BY_LOOP", "SFFT_FLAG_VOTE_BY_PAIR", "SFFT_FLAG_FUSED"]


@dataclass
class PlanParams:
    N: int
    K: int
    B: int
    L: int
    w: int
    seed: int = 0
    d: int = 2
    vote_threshold: int = 0
    n_resid: int = 0
    gauss_c: float = 0.0
    flags: int = 0
    strip_cols: int = 0
    sigma: np.ndarray | None = None
    tau: np.ndarray | None = None
    comb_b: int = 0
    comb_loops: int = 0
    comb_keep: int = 0
    est_loops: int = 0
    est_B: int = 0
    est_w: int = 0

    def to_c(self):
        """Return (Params struct, keep-alive list)."""
        lib = load()
        p = _capi.Params()
        check(lib.sfft_params_init(C.byref(p), self.N, self.K, self.B, self.L, self.w), "sfft_params_init")
        p.seed = self.seed & ((1 << 64) - 1)
        p.d = self.d
        p.vote_threshold = self.vote_threshold
        p.n_resid = self.n_resid
        p.gauss_c = self.gauss_c
        p.flags = self.flags
        p.strip_cols = self.strip_cols
        p.comb_b = self.comb_b
        p.comb_loops = self.comb_loops
        p.comb_keep = self.comb_keep
        p.est_loops = self.est_loops
        p.est_B = self.est_B
        p.est_w = self.est_w
        keep = []
        if self.sigma is not None:
            s = np.ascontiguousarray(self.sigma, dtype=np.uint32)
            t = np.ascontiguousarray(self.tau, dtype=np.uint32)
            keep += [s, t]
            p.sigma = s.ctypes.data_as(C.POINTER(C.c_uint32))
            p.tau = t.ctypes.data_as(C.POINTER(C.c_uint32))
        return p, keep


def _ptr(a) -> int:
    return 0 if a is None else int(a.data_ptr())


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _desc_dict(d) -> dict:
    """A plan description as a dict; the loop pairs of the vote as a list of (first, second)."""
    out = {f: getattr(d, f) for f, _ in _capi.PlanDesc._fields_ if f != "vote_pair"}
    out["vote_pair"] = [(v & 255, v >> 8) for v in list(d.vote_pair)[:d.vote_pairs]]
    return out


def params_describe(params: PlanParams) -> dict:
    """The description sfft_plan_ex would give these parameters, without a device."""
    p, keep = params.to_c()
    d = _capi.PlanDesc()
    check(load().sfft_params_describe(C.byref(p), C.byref(d)), "sfft_params_describe")
    del keep
    return _desc_dict(d)


def host_tables(params: PlanParams) -> dict:
    """FP64 host tables of a plan, built without a device (sfft_host_tables)."""
    lib = load()
    p, keep = params.to_c()
    L, w, M = params.L + params.est_loops, params.w, params.N // params.B
    S = 0 if params.flags & SFFT_FLAG_NO_RESIDUAL else (params.n_resid or 4096)
    out = dict(sigma=np.zeros(L, np.uint32), sigma_inv=np.zeros(L, np.uint32), tau=np.zeros(L, np.uint32),
               tpos=np.zeros(max(S, 1), np.uint32), window=np.zeros(w, np.float64),
               gain=np.zeros(2 * M, np.float64))
    check(lib.sfft_host_tables(C.byref(p), *(out[k].ctypes.data for k in
                                             ("sigma", "sigma_inv", "tau", "tpos", "window", "gain"))),
          "sfft_host_tables")
    out["tpos"] = out["tpos"][:S]
    out["gain"] = out["gain"][0::2] + 1j * out["gain"][1::2]
    del keep
    return out


class Plan:
    """A resident plan: device tables + one workspace on the current device."""

    def __init__(self, N: int, K: int, B: int, L: int, w: int, **kw):
        self.params = PlanParams(N, K, B, L, w, **kw)
        lib = load()
        p, keep = self.params.to_c()
        h = C.c_void_p()
        check(lib.sfft_plan_ex(C.byref(h), C.byref(p)), "sfft_plan_ex")
        self._h = h
        del keep
        self.desc = self.describe()

    @classmethod
    def from_params(cls, params: PlanParams) -> "Plan":
        kw = {k: getattr(params, k) for k in ("seed", "d", "vote_threshold", "n_resid", "gauss_c", "flags",
                                               "strip_cols", "sigma", "tau", "comb_b", "comb_loops", "comb_keep",
                                               "est_loops", "est_B", "est_w")}
        return cls(params.N, params.K, params.B, params.L, params.w, **kw)

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    def describe(self) -> dict:
        d = _capi.PlanDesc()
        check(load().sfft_plan_describe(self._h, C.byref(d)), "sfft_plan_describe")
        return _desc_dict(d)

    def perms(self):
        """sigma, sigma^{-1}, tau of every loop (the estimation-only loops last)."""
        L = self.params.L + self.params.est_loops
        s, si, t = (np.zeros(L, np.uint32) for _ in range(3))
        check(load().sfft_plan_get_perms(self._h, s.ctypes.data, si.ctypes.data, t.ctypes.data),
              "sfft_plan_get_perms")
        return s, si, t

    def outputs(self, device=None):
        import torch
        K = self.params.K
        idx = torch.empty(K, dtype=torch.int64, device=device or "cuda")
        val = torch.empty(K, dtype=torch.complex64, device=device or "cuda")
        res = torch.empty(2, dtype=torch.float64, device=device or "cuda")
        return idx, val, res

    def execute(self, x, out_idx, out_val, out_resid=None, stream=None) -> None:
        """Asynchronous execution on `stream` (default: torch's current stream)."""
        import torch
        if x.dtype != torch.complex64 or not x.is_cuda or x.numel() != self.params.N or not x.is_contiguous():
            raise ValueError("x must be a contiguous complex64 CUDA tensor of length N")
        check(load().sfft_execute_ex(self._h, _ptr(x), _ptr(out_idx), _ptr(out_val), _ptr(out_resid),
                                     _stream_handle(stream)), "sfft_execute_ex")

    def __call__(self, x, stream=None, residual: bool = False):
        idx, val, res = self.outputs(x.device)
        self.execute(x, idx, val, res, stream)
        return (idx, val, res) if residual else (idx, val)

    def trace(self) -> dict:
        """Host copies of the last execution's intermediates (synchronous)."""
        d = self.desc
        L, B, dK, cap = d["L"], d["B"], d["d"] * d["K"], d["cand_cap"]
        wpl = (B + 31) // 32
        uh = np.zeros(2 * L * B, np.float32)
        jb = np.zeros(L * wpl, np.uint32)
        jl = np.zeros(L * dK, np.uint32)
        cd = np.zeros(max(cap, 1), np.uint32)
        nc, cb = self.params.comb_loops, self.params.comb_b
        cw = max(1, cb // 32) if nc else 1
        cbits = np.zeros(max(nc, 1) * cw, np.uint32)
        K = d["K"]
        ri = np.zeros(K, np.uint32)
        rv = np.zeros(2 * K, np.float32)
        t = _capi.Trace(uh.ctypes.data_as(C.POINTER(C.c_float)), jb.ctypes.data_as(C.POINTER(C.c_uint32)),
                        jl.ctypes.data_as(C.POINTER(C.c_uint32)), cd.ctypes.data_as(C.POINTER(C.c_uint32)), 0,
                        cbits.ctypes.data_as(C.POINTER(C.c_uint32)), ri.ctypes.data_as(C.POINTER(C.c_uint32)),
                        rv.ctypes.data_as(C.POINTER(C.c_float)), 0)
        check(load().sfft_plan_read_trace(self._h, C.byref(t)), "sfft_plan_read_trace")
        uhat = (uh[0::2] + 1j * uh[1::2]).reshape(L, B)
        out = dict(uhat=uhat, jbits=jb.reshape(L, wpl), jlist=jl.reshape(L, dK), cand=cd[:t.cand_count].copy())
        if self.params.flags & SFFT_FLAG_ITERATE:
            # first-round outputs (the trace arrays above are the second round's)
            n1 = int(t.rec_count)
            out["rec_idx"] = ri[:n1].astype(np.int64)
            out["rec_val"] = (rv[0::2] + 1j * rv[1::2])[:n1]
        if nc:
            rows = cbits.reshape(nc, cw)
            out["comb_rows"] = np.array([[(rows[c, i >> 5] >> (i & 31)) & 1 for i in range(cb)] for c in range(nc)],
                                        dtype=bool)
        return out

    def close(self) -> None:
        if getattr(self, "_h", None):
            check(load().sfft_destroy(self._h), "sfft_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr_array(vals):
    arr = (C.c_void_p * len(vals))()
    for i, v in enumerate(vals):
        arr[i] = v
    return arr


class Batch:
    """Uneven batch of signals run as one HIP graph of batched launches."""

    def __init__(self, plans, branches: int = 1):
        self.plans = list(plans)
        hs = _ptr_array([p.handle.value for p in self.plans])
        h = C.c_void_p()
        check(load().sfft_batch_create_ex(C.byref(h), hs, len(self.plans), branches), "sfft_batch_create_ex")
        self._h = h

    def run(self, xs, idxs, vals, resids=None, stream=None) -> None:
        n = len(self.plans)
        if not (len(xs) == len(idxs) == len(vals) == n):
            raise ValueError("one x, idx and val per plan")
        xa = _ptr_array([_ptr(x) for x in xs])
        ia = _ptr_array([_ptr(i) for i in idxs])
        va = _ptr_array([_ptr(v) for v in vals])
        ra = _ptr_array([_ptr(r) for r in resids]) if resids is not None else None
        check(load().sfft_batch_run(self._h, xa, ia, va, ra, _stream_handle(stream)), "sfft_batch_run")

    def bind(self, xs, idxs, vals, resids=None) -> None:
        """Marshal the buffers' device pointers once for run_bound (which then skips the
        per-call pointer arrays); the tensors are kept alive while bound."""
        n = len(self.plans)
        if not (len(xs) == len(idxs) == len(vals) == n):
            raise ValueError("one x, idx and val per plan")
        arrays = tuple(_ptr_array([_ptr(t) for t in ts]) if ts is not None else None
                       for ts in (xs, idxs, vals, resids))
        self._bound = (arrays, (list(xs), list(idxs), list(vals), list(resids) if resids is not None else None))

    def run_bound(self, stream=None) -> None:
        """run() on the buffers given to bind()."""
        xa, ia, va, ra = self._bound[0]
        check(load().sfft_batch_run(self._h, xa, ia, va, ra, _stream_handle(stream)), "sfft_batch_run")

    def run_timed(self, xs, idxs, vals, resids, ev_begin, ev_end, stream=None) -> None:
        """As run(); records HipEvent ev_begin / ev_end around the bucketization."""
        xa = _ptr_array([_ptr(x) for x in xs])
        ia = _ptr_array([_ptr(i) for i in idxs])
        va = _ptr_array([_ptr(v) for v in vals])
        ra = _ptr_array([_ptr(r) for r in resids]) if resids is not None else None
        check(load().sfft_batch_run_timed(self._h, xa, ia, va, ra, _stream_handle(stream),
                                          ev_begin.handle, ev_end.handle), "sfft_batch_run_timed")

    def close(self) -> None:
        if getattr(self, "_h", None):
            check(load().sfft_batch_destroy(self._h), "sfft_batch_destroy")
            self._h = None
        self._bound = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop over the C ABI (continuous batching, HBM admission)."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 64, n_streams: int = 2):
        h = C.c_void_p()
        check(load().sfft_server_create(C.byref(h), hbm_budget_bytes, max_inflight, n_streams),
              "sfft_server_create")
        self._h = h

    def prepare(self, params: PlanParams):
        """Build and cache the plan of `params`; returns a handle `submit` accepts."""
        p, keep = params.to_c()
        check(load().sfft_server_prepare(self._h, C.byref(p)), "sfft_server_prepare")
        return (p, keep)

    def submit(self, params, x, out_idx, out_val, out_resid=None) -> int:
        """Queue one request; `params` is a PlanParams or a handle from `prepare`."""
        p, keep = params if isinstance(params, tuple) else params.to_c()
        t = C.c_uint64()
        check(load().sfft_server_submit(self._h, C.byref(p), _ptr(x), _ptr(out_idx), _ptr(out_val),
                                        _ptr(out_resid), C.byref(t)), "sfft_server_submit")
        del keep
        return t.value

    def submit_many(self, params, xs, idxs, vals, resids=None) -> list:
        """Queue one request per signal of `xs` with one parameter set (all or none);
        returns their tickets in order."""
        p, keep = params if isinstance(params, tuple) else params.to_c()
        n = len(xs)
        if not (len(idxs) == len(vals) == n) or (resids is not None and len(resids) != n):
            raise ValueError("one x, idx and val (and resid) per request")
        t = (C.c_uint64 * max(n, 1))()
        xa = _ptr_array([_ptr(x) for x in xs])
        ia = _ptr_array([_ptr(i) for i in idxs])
        va = _ptr_array([_ptr(v) for v in vals])
        ra = _ptr_array([_ptr(r) for r in resids]) if resids is not None else None
        check(load().sfft_server_submit_batch(self._h, C.byref(p), n, xa, ia, va, ra, t), "sfft_server_submit_batch")
        del keep
        return list(t[:n])

    def poll(self, ticket: int):
        done, lat, st = C.c_int32(), C.c_double(), C.c_int32()
        check(load().sfft_server_poll(self._h, ticket, C.byref(done), C.byref(lat), C.byref(st)),
              "sfft_server_poll")
        return bool(done.value), lat.value, st.value

    def wait(self, ticket: int):
        lat, st = C.c_double(), C.c_int32()
        check(load().sfft_server_wait(self._h, ticket, C.byref(lat), C.byref(st)), "sfft_server_wait")
        return lat.value, st.value

    def stats(self) -> dict:
        s = _capi.ServerStats()
        check(load().sfft_server_stats_get(self._h, C.byref(s)), "sfft_server_stats_get")
        return {f: getattr(s, f) for f, _ in _capi.ServerStats._fields_}

    def close(self) -> None:
        if getattr(self, "_h", None):
            check(load().sfft_server_destroy(self._h), "sfft_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
