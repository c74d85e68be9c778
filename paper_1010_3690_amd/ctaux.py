"""Python binding of libctaux_hip.so (the C ABI of include/ctaux.h).

Marshalling only: every step of the Monte Carlo path runs in the HIP
kernels of the library.  PyTorch provides the device workspace and the HIP
stream.  Importing works without a GPU; creating a batch needs the built
library and a GPU and raises otherwise (there is no CPU fallback).
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libctaux_hip.so")

CTAUX_OK, CTAUX_EINVAL, CTAUX_ENOMEM, CTAUX_EDEVICE, CTAUX_ENUMERIC, CTAUX_ECAPACITY = 0, -1, -2, -3, -4, -5
CTAUX_FP64, CTAUX_FP32, CTAUX_BF16X3 = 0, 1, 2
OBS_HEADER = 8
# order of the per-kernel timing entries (ctaux_get_timing)
TIMED_KERNELS = ["block_begin", "interp", "prep", "propose", "assemble", "rankk", "block_end", "measure",
                 "refine"]

EXPORTED = [
    "ctaux_workspace_bytes", "ctaux_create", "ctaux_run", "ctaux_recompute", "ctaux_obs_len", "ctaux_get_obs_kw",
    "ctaux_get_obs", "ctaux_reset_obs", "ctaux_get_stats", "ctaux_get_config", "ctaux_get_N",
    "ctaux_get_decisions", "ctaux_set_timing", "ctaux_set_timing_every", "ctaux_get_timing",
    "ctaux_set_graph", "ctaux_graph_launches",
    "ctaux_checkpoint", "ctaux_restore", "ctaux_recompute_from_scratch",
    "ctaux_build_N_workspace_bytes", "ctaux_build_N", "ctaux_build_N_noalloc",
    "ctaux_last_error", "ctaux_destroy",
]


class _Model(C.Structure):
    _fields_ = [("beta", C.c_double), ("U", C.c_double), ("K", C.c_double), ("n_sites", C.c_int32),
                ("n_tau", C.c_int32), ("n_disp", C.c_int32), ("site_disp", C.c_void_p),
                ("g0_up", C.c_void_p), ("g0_dn", C.c_void_p), ("site_pos", C.c_void_p), ("kvecs", C.c_void_p),
                ("n_k", C.c_int32)]


class _Opts(C.Structure):
    _fields_ = [("k_max", C.c_int32), ("k_cap", C.c_int32), ("p_flip", C.c_double),
                ("recompute_every", C.c_int32), ("precision", C.c_int32), ("meas_every", C.c_int32),
                ("n_therm", C.c_int64), ("n_tau_out", C.c_int32), ("n_cap", C.c_int32),
                ("seed", C.c_uint64), ("log_cap", C.c_int64), ("gamma_tol", C.c_double),
                ("drift_tol", C.c_double), ("rankk_tile", C.c_int32), ("drift_target", C.c_double),
                ("n_matsubara", C.c_int32), ("recompute_mode", C.c_int32),
                ("p_pair", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("proposals", C.c_int64), ("accepted", C.c_int64), ("blocks", C.c_int64),
                ("sum_ka", C.c_int64), ("next_id", C.c_int64), ("order", C.c_int32),
                ("status", C.c_int32), ("sign", C.c_double), ("max_drift", C.c_double),
                ("rankk_flops", C.c_double), ("rankk_bytes", C.c_double), ("sum_order", C.c_double),
                ("gj_fallbacks", C.c_int64), ("prep_flops", C.c_double), ("prep_bytes", C.c_double),
                ("meas_flops", C.c_double), ("meas_bytes", C.c_double), ("scratch_recomputes", C.c_int64),
                ("refine_interval", C.c_int32)]


class _Vertex(C.Structure):
    _fields_ = [("id", C.c_int64), ("tau", C.c_double), ("site", C.c_int32), ("s", C.c_int32)]


class CtauxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ctaux error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: the library must bind to the HIP runtime torch already loaded
    # (loading it first would bring a second runtime into the process)
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1010_3690_amd.build`")
    lib = C.CDLL(path)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.ctaux_workspace_bytes.restype = C.c_size_t
    lib.ctaux_workspace_bytes.argtypes = [vp, i32, vp]
    lib.ctaux_create.argtypes = [vp, i32, vp, vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.ctaux_run.argtypes = [vp, i64]
    lib.ctaux_recompute.argtypes = [vp, C.POINTER(d)]
    lib.ctaux_recompute_from_scratch.argtypes = [vp, C.POINTER(d)]
    lib.ctaux_build_N_workspace_bytes.restype = C.c_size_t
    lib.ctaux_build_N_workspace_bytes.argtypes = [vp, i32]
    lib.ctaux_build_N.argtypes = [vp, vp, i32, i32, vp, i32, vp, C.c_size_t, vp]
    lib.ctaux_build_N_noalloc.argtypes = [vp, vp, i32, i32, vp, i32, vp]
    lib.ctaux_obs_len.restype = i32
    lib.ctaux_obs_len.argtypes = [vp]
    lib.ctaux_get_obs.argtypes = [vp, i32, vp, i32]
    lib.ctaux_get_obs_kw.argtypes = [vp, i32, vp, vp, i32]
    lib.ctaux_reset_obs.argtypes = [vp]
    lib.ctaux_get_stats.argtypes = [vp, i32, C.POINTER(_Stats)]
    lib.ctaux_get_config.argtypes = [vp, i32, i32, vp, C.POINTER(i32)]
    lib.ctaux_get_N.argtypes = [vp, i32, i32, vp, i32, C.POINTER(i32)]
    lib.ctaux_get_decisions.argtypes = [vp, i32, i64, i64, vp, vp]
    lib.ctaux_set_timing.argtypes = [vp, i32]
    lib.ctaux_set_timing_every.argtypes = [vp, i32]
    lib.ctaux_set_graph.argtypes = [vp, i32]
    lib.ctaux_graph_launches.restype = i64
    lib.ctaux_graph_launches.argtypes = [vp]
    lib.ctaux_get_timing.restype = i32
    lib.ctaux_get_timing.argtypes = [vp, vp, vp, vp, i32]
    lib.ctaux_checkpoint.argtypes = [vp, i32, vp, C.POINTER(C.c_size_t)]
    lib.ctaux_restore.argtypes = [vp, i32, vp, C.c_size_t]
    lib.ctaux_last_error.restype = C.c_char_p
    lib.ctaux_last_error.argtypes = [vp]
    lib.ctaux_destroy.argtypes = [vp]
    _lib = lib
    return lib


@dataclass
class Options:
    k_max: int = 64
    k_cap: int = 64
    p_flip: float = 0.2
    recompute_every: int = 64
    precision: int = CTAUX_FP64
    meas_every: int = 64
    n_therm: int = 0
    n_tau_out: int = 16
    n_cap: int = 1024
    seed: int = 0
    log_cap: int = 0
    gamma_tol: float = 1e-8
    drift_tol: float = 1e-2
    rankk_tile: int = 64
    drift_target: float = 0.0
    n_matsubara: int = 0
    recompute_mode: int = 0
    p_pair: float = 0.0

    def _c(self) -> _Opts:
        return _Opts(self.k_max, self.k_cap, self.p_flip, self.recompute_every, self.precision,
                     self.meas_every, self.n_therm, self.n_tau_out, self.n_cap, self.seed, self.log_cap,
                     self.gamma_tol, self.drift_tol, self.rankk_tile, self.drift_target, self.n_matsubara,
                     self.recompute_mode, self.p_pair)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class CtauxBatch:
    """A batch of independent chains on one GPU (one chain is a batch of one)."""

    def __init__(self, workloads, opts: Options, device: str = "cuda:0", stream=None):
        import torch

        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("CtauxBatch needs a GPU; there is no CPU path")
        if not isinstance(workloads, (list, tuple)):
            workloads = [workloads]
        self.workloads = list(workloads)
        self.opts = opts
        self.device = torch.device(device)
        self._arrays = []
        models = (_Model * len(workloads))()
        for i, w in enumerate(workloads):
            models[i], keep = _model_of(w)
            self._arrays += list(keep)
        self._models = models
        self._copts = opts._c()
        nbytes = self.lib.ctaux_workspace_bytes(C.byref(models), len(workloads), C.byref(self._copts))
        if nbytes == 0:
            raise CtauxError(CTAUX_EINVAL, self.lib.ctaux_last_error(None).decode())
        self.workspace_bytes = int(nbytes)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = self.lib.ctaux_create(C.byref(models), len(workloads), C.byref(self._copts),
                                   C.c_void_p(self.workspace.data_ptr()), nbytes,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != 0:
            raise CtauxError(rc, self.lib.ctaux_last_error(None).decode())
        self.h = h
        self.n_chains = len(workloads)

    def close(self):
        if getattr(self, "h", None):
            self.lib.ctaux_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc != 0:
            raise CtauxError(rc, self.lib.ctaux_last_error(self.h).decode())

    def run(self, n_proposals: int):
        self._check(self.lib.ctaux_run(self.h, int(n_proposals)))

    def recompute(self) -> float:
        d = C.c_double()
        self._check(self.lib.ctaux_recompute(self.h, C.byref(d)))
        return d.value

    def recompute_from_scratch(self) -> float:
        d = C.c_double()
        self._check(self.lib.ctaux_recompute_from_scratch(self.h, C.byref(d)))
        return d.value

    def obs(self, chain: int = 0) -> np.ndarray:
        n = self.lib.ctaux_obs_len(self.h)
        out = np.zeros(n)
        self._check(self.lib.ctaux_get_obs(self.h, chain, _ptr(out), n))
        w = self.workloads[chain]
        return out[: OBS_HEADER + 2 * w.n_disp * self.opts.n_tau_out]

    def obs_kw(self, chain: int = 0):
        """(accumulated sign * S(K, w_n), G0(K, i w_n)), complex [2, n_k, n_matsubara] each."""
        w = self.workloads[chain]
        nk, nm = w.kvecs.shape[0], self.opts.n_matsubara
        s = np.zeros(4 * nk * nm)
        g = np.zeros(4 * nk * nm)
        self._check(self.lib.ctaux_get_obs_kw(self.h, chain, _ptr(s), _ptr(g), len(s)))
        s = s.reshape(2, nk, nm, 2)
        g = g.reshape(2, nk, nm, 2)
        return s[..., 0] + 1j * s[..., 1], g[..., 0] + 1j * g[..., 1]

    def reset_obs(self):
        self._check(self.lib.ctaux_reset_obs(self.h))

    def stats(self, chain: int = 0) -> dict:
        s = _Stats()
        self._check(self.lib.ctaux_get_stats(self.h, chain, C.byref(s)))
        return {f: getattr(s, f) for f, _ in _Stats._fields_}

    def config(self, chain: int = 0):
        n = C.c_int32()
        self._check(self.lib.ctaux_get_config(self.h, chain, 0, None, C.byref(n)))
        buf = (_Vertex * max(n.value, 1))()
        self._check(self.lib.ctaux_get_config(self.h, chain, n.value, buf, C.byref(n)))
        m = n.value
        return (np.array([buf[i].id for i in range(m)], np.int64),
                np.array([buf[i].tau for i in range(m)]),
                np.array([buf[i].site for i in range(m)], np.int32),
                np.array([buf[i].s for i in range(m)], np.int32))

    def N(self, chain: int = 0, sector: int = 0) -> np.ndarray:
        n = C.c_int32()
        self._check(self.lib.ctaux_get_N(self.h, chain, sector, None, 0, C.byref(n)))
        out = np.zeros((n.value, n.value))
        if n.value:
            self._check(self.lib.ctaux_get_N(self.h, chain, sector, _ptr(out), n.value, C.byref(n)))
        return out

    def decisions(self, chain: int, first: int, count: int):
        acc = np.zeros(count, np.uint8)
        R = np.zeros(count)
        self._check(self.lib.ctaux_get_decisions(self.h, chain, first, count, _ptr(acc), _ptr(R)))
        return acc, R

    def checkpoint(self, chain: int = 0) -> bytes:
        n = C.c_size_t(0)
        self._check(self.lib.ctaux_checkpoint(self.h, chain, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(self.lib.ctaux_checkpoint(self.h, chain, buf, C.byref(n)))
        return buf.raw[: n.value]

    def restore(self, blob: bytes, chain: int = 0):
        self._check(self.lib.ctaux_restore(self.h, chain, C.c_char_p(blob), len(blob)))

    def set_graph(self, blocks: int):
        """Replay windows of `blocks` blocks from a captured HIP graph (0: off)."""
        self._check(self.lib.ctaux_set_graph(self.h, int(blocks)))

    @property
    def graph_launches(self) -> int:
        return int(self.lib.ctaux_graph_launches(self.h))

    def set_timing(self, enable, kernels=None, every=1):
        """Time every kernel (enable True), none (False), or only the named ones,
        one launch in `every`."""
        self._check(self.lib.ctaux_set_timing_every(self.h, int(every)))
        mask = 0
        if kernels is not None:
            names = TIMED_KERNELS
            for k in kernels:
                mask |= 1 << names.index(k)
        elif enable:
            mask = -1
        self._check(self.lib.ctaux_set_timing(self.h, mask))

    def timing(self) -> dict:
        cap = 32
        names = (C.c_char_p * cap)()
        ms = np.zeros(cap)
        cnt = np.zeros(cap, np.int64)
        k = self.lib.ctaux_get_timing(self.h, names, _ptr(ms), _ptr(cnt), cap)
        return {names[i].decode(): (float(ms[i]), int(cnt[i])) for i in range(k)}


def _model_of(w):
    """ctaux_model of a workload and the arrays it points to (kept alive by the caller)."""
    sd = np.ascontiguousarray(w.site_disp, np.int32)
    gu = np.ascontiguousarray(w.g0_up, np.float64)
    gd = np.ascontiguousarray(w.g0_dn, np.float64)
    keep = [sd, gu, gd]
    pos = kv = None
    n_k = 0
    if getattr(w, "site_pos", None) is not None:
        pos = np.ascontiguousarray(w.site_pos, np.float64)
        kv = np.ascontiguousarray(w.kvecs, np.float64)
        n_k = kv.shape[0]
        keep += [pos, kv]
    m = _Model(w.beta, w.U, w.K, w.n_sites, w.n_tau, w.n_disp, _ptr(sd), _ptr(gu), _ptr(gd),
               _ptr(pos) if pos is not None else None, _ptr(kv) if kv is not None else None, n_k)
    return m, keep


def _vertices(tau, site, s):
    n = len(tau)
    buf = (_Vertex * max(n, 1))()
    for i in range(n):
        buf[i] = _Vertex(i, float(tau[i]), int(site[i]), int(s[i]))
    return buf


def build_N(w, tau, site, s, sector: int, device: str = "cuda:0") -> np.ndarray:
    """N of one sector of a configuration from its definition, computed on the
    GPU by ctaux_build_N (M from the tables, pivoted elimination)."""
    import torch
    lib = load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("build_N needs a GPU; there is no CPU path")
    model, keep = _model_of(w)
    n = len(tau)
    verts = _vertices(tau, site, s)
    nbytes = lib.ctaux_build_N_workspace_bytes(C.byref(model), n)
    if nbytes == 0:
        raise CtauxError(CTAUX_EINVAL, lib.ctaux_last_error(None).decode())
    dev = torch.device(device)
    with torch.cuda.device(dev):
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        out = torch.empty((max(n, 1), max(n, 1)), dtype=torch.float64, device=dev)
        stream = torch.cuda.current_stream(dev)
        rc = lib.ctaux_build_N(C.byref(model), verts, n, sector, C.c_void_p(out.data_ptr()), max(n, 1),
                               C.c_void_p(ws.data_ptr()), nbytes, C.c_void_p(stream.cuda_stream))
    if rc != 0:
        raise CtauxError(rc, lib.ctaux_last_error(None).decode())
    return out[:n, :n].cpu().numpy()


def build_N_noalloc(w, tau, site, s, sector: int, out=None, device: str = "cuda:0"):
    """As build_N, through the allocation-free entry point ctaux_build_N_noalloc.
    out: an optional float64 device tensor of at least n x n (row-major); the
    result is written there and returned as a numpy copy."""
    import torch
    lib = load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("build_N_noalloc needs a GPU; there is no CPU path")
    model, keep = _model_of(w)
    n = len(tau)
    verts = _vertices(tau, site, s)
    dev = torch.device(device)
    with torch.cuda.device(dev):
        if out is None:
            out = torch.empty((max(n, 1), max(n, 1)), dtype=torch.float64, device=dev)
        ld = out.shape[1]
        stream = torch.cuda.current_stream(dev)
        rc = lib.ctaux_build_N_noalloc(C.byref(model), verts, n, sector, C.c_void_p(out.data_ptr()), ld,
                                       C.c_void_p(stream.cuda_stream))
    if rc != 0:
        raise CtauxError(rc, lib.ctaux_last_error(None).decode())
    return out[:n, :n].cpu().numpy()
