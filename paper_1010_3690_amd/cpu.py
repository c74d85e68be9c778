"""Python binding of libctaux_cpu.so (include/ctaux_cpu.h): the submatrix
update on the host CPU, one chain per object.  Marshalling only."""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .ctaux import CtauxError, Options, _Vertex, _model_of, _ptr

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libctaux_cpu.so")
EXPORTED = ["ctaux_cpu_create", "ctaux_cpu_run", "ctaux_cpu_get_state", "ctaux_cpu_get_config", "ctaux_cpu_get_N",
            "ctaux_cpu_get_decisions", "ctaux_cpu_get_obs", "ctaux_cpu_set_config", "ctaux_cpu_set_growth",
            "ctaux_cpu_last_error", "ctaux_cpu_destroy"]

_lib = None


def load_cpu_library(path: str = LIB_PATH):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1010_3690_amd.build`")
    lib = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.ctaux_cpu_create.argtypes = [vp, vp, i32, C.POINTER(vp)]
    lib.ctaux_cpu_run.argtypes = [vp, i64]
    lib.ctaux_cpu_get_state.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.ctaux_cpu_get_config.argtypes = [vp, i32, vp, vp]
    lib.ctaux_cpu_get_N.argtypes = [vp, i32, vp, i32]
    lib.ctaux_cpu_get_decisions.argtypes = [vp, i64, i64, vp, vp]
    lib.ctaux_cpu_get_obs.argtypes = [vp, vp, i32]
    lib.ctaux_cpu_set_config.argtypes = [vp, i32, vp, i64, i64, C.c_double]
    lib.ctaux_cpu_last_error.restype = C.c_char_p
    lib.ctaux_cpu_last_error.argtypes = [vp]
    lib.ctaux_cpu_set_growth.argtypes = [vp, i32]
    lib.ctaux_cpu_destroy.argtypes = [vp]
    _lib = lib
    return lib


class CpuChain:
    """One chain of the host submatrix implementation."""

    def __init__(self, w, opts: Options, chain_id: int = 0):
        self.lib = load_cpu_library()
        self.w = w
        self.opts = opts
        self._model, self._keep = _model_of(w)
        self._copts = opts._c()
        h = C.c_void_p()
        rc = self.lib.ctaux_cpu_create(C.byref(self._model), C.byref(self._copts), chain_id, C.byref(h))
        if rc != 0:
            raise CtauxError(rc, "ctaux_cpu_create rejected its arguments")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.ctaux_cpu_destroy(self.h)
            self.h = None

    def _check(self, rc):
        if rc != 0:
            raise CtauxError(rc, self.lib.ctaux_cpu_last_error(self.h).decode())

    def set_growth(self, mode: int):
        """0: Gamma's inverse grown by partitioning; 1: Gamma's LU factors grown."""
        self._check(self.lib.ctaux_cpu_set_growth(self.h, int(mode)))

    def run(self, n_proposals: int):
        self._check(self.lib.ctaux_cpu_run(self.h, int(n_proposals)))

    def state(self) -> dict:
        p, a, b = C.c_int64(), C.c_int64(), C.c_int64()
        o, s = C.c_int32(), C.c_double()
        self._check(self.lib.ctaux_cpu_get_state(self.h, C.byref(p), C.byref(a), C.byref(b), C.byref(o), C.byref(s)))
        return {"proposals": p.value, "accepted": a.value, "blocks": b.value, "order": o.value, "sign": s.value}

    def config(self):
        n = C.c_int32()
        self._check(self.lib.ctaux_cpu_get_config(self.h, 0, None, C.byref(n)))
        buf = (_Vertex * max(n.value, 1))()
        self._check(self.lib.ctaux_cpu_get_config(self.h, n.value, buf, C.byref(n)))
        m = n.value
        return (np.array([buf[i].id for i in range(m)], np.int64), np.array([buf[i].tau for i in range(m)]),
                np.array([buf[i].site for i in range(m)], np.int32), np.array([buf[i].s for i in range(m)], np.int32))

    def N(self, sector: int) -> np.ndarray:
        n = self.state()["order"]
        out = np.zeros((n, n))
        if n:
            self._check(self.lib.ctaux_cpu_get_N(self.h, sector, _ptr(out), n))
        return out

    def decisions(self, first: int, count: int):
        acc = np.zeros(count, np.uint8)
        R = np.zeros(count)
        self._check(self.lib.ctaux_cpu_get_decisions(self.h, first, count, _ptr(acc), _ptr(R)))
        return acc, R

    def obs(self) -> np.ndarray:
        out = np.zeros(8 + 2 * self.w.n_disp * self.opts.n_tau_out)
        self._check(self.lib.ctaux_cpu_get_obs(self.h, _ptr(out), len(out)))
        return out

    def set_config(self, ids, tau, site, s, proposals_done=0, next_id=None, sign=1.0):
        n = len(tau)
        buf = (_Vertex * max(n, 1))()
        for i in range(n):
            buf[i] = _Vertex(int(ids[i]), float(tau[i]), int(site[i]), int(s[i]))
        nid = int(ids[-1]) + 1 if (next_id is None and n) else (next_id or 0)
        self._check(self.lib.ctaux_cpu_set_config(self.h, n, buf, int(proposals_done), nid, float(sign)))
