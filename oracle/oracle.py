"""ctypes wrapper of the CT-AUX oracle (TEST INFRASTRUCTURE ONLY)."""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ctaux_oracle.c")
_LIB = os.path.join(_HERE, "libctaux_oracle.so")

OC_OBS_HEADER = 8


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
            os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "ctaux_oracle.h"))):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-o", tmp,
                               _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build_oracle()
    lib = C.CDLL(_LIB)
    P = C.POINTER
    d, i32, i64, u64, u32 = C.c_double, C.c_int32, C.c_int64, C.c_uint64, C.c_uint32
    vp = C.c_void_p
    lib.oc_create.restype = vp
    lib.oc_create.argtypes = [d, d, d, i32, i32, i32, vp, vp, vp, u64, u32, d, i32, i64, i32, i32]
    lib.oc_destroy.argtypes = [vp]
    lib.oc_error.restype = C.c_char_p
    lib.oc_error.argtypes = [vp]
    lib.oc_run.argtypes = [vp, i64]
    lib.oc_set_log.argtypes = [vp, i64]
    lib.oc_get_log.argtypes = [vp, i64, i64, vp, vp]
    lib.oc_order.restype = i32
    lib.oc_order.argtypes = [vp]
    lib.oc_proposals_done.restype = i64
    lib.oc_proposals_done.argtypes = [vp]
    lib.oc_sign.restype = d
    lib.oc_sign.argtypes = [vp]
    lib.oc_gamma_value.restype = d
    lib.oc_gamma_value.argtypes = [vp]
    lib.oc_get_config.argtypes = [vp, vp, vp, vp, vp]
    lib.oc_get_N.argtypes = [vp, i32, vp]
    lib.oc_build_Minv.argtypes = [vp, i32, vp]
    lib.oc_build_M_of.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    lib.oc_set_config.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    lib.oc_get_state.argtypes = [vp, P(i64), P(i64), P(d)]
    lib.oc_set_state.argtypes = [vp, i64, i64, d]
    lib.oc_last_proposal.argtypes = [vp, P(i32), P(i32), P(d), P(i32), P(i32), P(d), P(i32)]
    lib.oc_last_pair.argtypes = [vp, P(i32), P(d), P(i32), P(i32)]
    lib.oc_set_pair.argtypes = [vp, d]
    lib.oc_pair_draws.argtypes = [u64, u32, u64, vp]
    lib.oc_obs_len.restype = i32
    lib.oc_obs_len.argtypes = [vp]
    lib.oc_get_obs.argtypes = [vp, vp]
    lib.oc_reset_obs.argtypes = [vp]
    lib.oc_estimate_G.argtypes = [vp, i32, i32, i32, d, P(d)]
    lib.oc_g0_lookup.restype = d
    lib.oc_g0_lookup.argtypes = [vp, i32, i32, i32, d]
    lib.oc_set_momentum.argtypes = [vp, i32, vp, vp, i32]
    lib.oc_get_obs_kw.argtypes = [vp, vp]
    lib.oc_g0_matsubara.argtypes = [vp, i32, i32, i32, vp]
    lib.oc_philox4x32_10.argtypes = [vp, vp, vp]
    lib.oc_draws.argtypes = [u64, u32, u64, vp]
    lib.oc_gamma_of.restype = d
    lib.oc_gamma_of.argtypes = [d, d, d, i32]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def philox4x32_10(ctr, key) -> np.ndarray:
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.oc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def draws(seed: int, chain: int, index: int) -> np.ndarray:
    lib = _load()
    out = np.zeros(5)
    lib.oc_draws(seed, chain, index, _ptr(out))
    return out


def pair_draws(seed: int, chain: int, index: int) -> np.ndarray:
    """u_spin2, u_tau2, u_pick2 of a pair proposal."""
    lib = _load()
    out = np.zeros(3)
    lib.oc_pair_draws(seed, chain, index, _ptr(out))
    return out


def gamma_of(beta, U, K, n_sites) -> float:
    return _load().oc_gamma_of(beta, U, K, n_sites)


class OracleError(RuntimeError):
    pass


class OracleChain:
    """One Markov chain of the oracle."""

    def __init__(self, w, seed=0, chain_id=0, p_flip=0.2, meas_every=16, n_therm=0,
                 n_tau_out=16, n_cap=4096, p_pair=0.0):
        self.lib = _load()
        self.w = w
        self._keep = (np.ascontiguousarray(w.site_disp, np.int32),
                      np.ascontiguousarray(w.g0_up, np.float64),
                      np.ascontiguousarray(w.g0_dn, np.float64))
        sd, gu, gd = self._keep
        self.h = self.lib.oc_create(w.beta, w.U, w.K, w.n_sites, w.n_tau, w.n_disp, _ptr(sd),
                                    _ptr(gu), _ptr(gd), seed, chain_id, p_flip, meas_every,
                                    n_therm, n_tau_out, n_cap)
        if not self.h:
            raise OracleError("oc_create rejected its arguments")
        self.n_tau_out = n_tau_out
        if p_pair:
            self._check(self.lib.oc_set_pair(self.h, p_pair))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.oc_destroy(h)
            self.h = None

    def _check(self, rc):
        if rc != 0:
            raise OracleError(f"oracle error {rc}: {self.lib.oc_error(self.h).decode()}")

    def run(self, n_proposals: int):
        self._check(self.lib.oc_run(self.h, n_proposals))

    def set_log(self, cap: int):
        self._check(self.lib.oc_set_log(self.h, cap))

    def get_log(self, first: int, count: int):
        acc = np.zeros(count, np.uint8)
        R = np.zeros(count)
        self._check(self.lib.oc_get_log(self.h, first, count, _ptr(acc), _ptr(R)))
        return acc, R

    @property
    def order(self) -> int:
        return self.lib.oc_order(self.h)

    @property
    def proposals_done(self) -> int:
        return self.lib.oc_proposals_done(self.h)

    @property
    def sign(self) -> float:
        return self.lib.oc_sign(self.h)

    @property
    def gamma(self) -> float:
        return self.lib.oc_gamma_value(self.h)

    def config(self):
        n = self.order
        ids = np.zeros(n, np.int64)
        tau = np.zeros(n)
        site = np.zeros(n, np.int32)
        s = np.zeros(n, np.int32)
        self._check(self.lib.oc_get_config(self.h, _ptr(ids), _ptr(tau), _ptr(site), _ptr(s)))
        return ids, tau, site, s

    def N(self, sector: int) -> np.ndarray:
        n = self.order
        out = np.zeros((n, n))
        self._check(self.lib.oc_get_N(self.h, sector, _ptr(out)))
        return out

    def Minv(self, sector: int) -> np.ndarray:
        n = self.order
        out = np.zeros((n, n))
        self._check(self.lib.oc_build_Minv(self.h, sector, _ptr(out)))
        return out

    def M_of(self, sector: int, tau, site, s) -> np.ndarray:
        """N^{-1} = e^V - G0 (e^V - 1) of a given configuration, from its definition."""
        tau = np.ascontiguousarray(tau, np.float64)
        site = np.ascontiguousarray(site, np.int32)
        s = np.ascontiguousarray(s, np.int32)
        n = len(tau)
        out = np.zeros((n, n))
        self._check(self.lib.oc_build_M_of(self.h, sector, n, _ptr(tau), _ptr(site), _ptr(s), _ptr(out)))
        return out

    def set_config(self, ids, tau, site, s):
        ids = np.ascontiguousarray(ids, np.int64)
        tau = np.ascontiguousarray(tau, np.float64)
        site = np.ascontiguousarray(site, np.int32)
        s = np.ascontiguousarray(s, np.int32)
        lad = np.zeros(2)
        sg = np.zeros(2)
        self._check(self.lib.oc_set_config(self.h, len(tau), _ptr(ids), _ptr(tau), _ptr(site),
                                           _ptr(s), _ptr(lad), _ptr(sg)))
        return lad, sg

    def get_state(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_double()
        self._check(self.lib.oc_get_state(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def set_state(self, done, next_id, sign):
        self._check(self.lib.oc_set_state(self.h, done, next_id, sign))

    def last_proposal(self):
        t, p, site, s, acc = (C.c_int32() for _ in range(5))
        tau, R = C.c_double(), C.c_double()
        self._check(self.lib.oc_last_proposal(self.h, C.byref(t), C.byref(p), C.byref(tau),
                                              C.byref(site), C.byref(s), C.byref(R),
                                              C.byref(acc)))
        p2, site2, s2 = C.c_int32(), C.c_int32(), C.c_int32()
        tau2 = C.c_double()
        self._check(self.lib.oc_last_pair(self.h, C.byref(p2), C.byref(tau2), C.byref(site2), C.byref(s2)))
        return dict(type=t.value, p=p.value, tau=tau.value, site=site.value, s_new=s.value,
                    R=R.value, acc=acc.value, p2=p2.value, tau2=tau2.value, site2=site2.value,
                    s2=s2.value)

    def obs(self) -> np.ndarray:
        out = np.zeros(self.lib.oc_obs_len(self.h))
        self._check(self.lib.oc_get_obs(self.h, _ptr(out)))
        return out

    def reset_obs(self):
        self._check(self.lib.oc_reset_obs(self.h))

    def set_momentum(self, kvecs, site_pos, n_matsubara):
        k = np.ascontiguousarray(np.asarray(kvecs, np.float64).reshape(-1, 3))
        r = np.ascontiguousarray(np.asarray(site_pos, np.float64).reshape(-1, 3))
        self._kw = (k, r, int(n_matsubara))
        self._check(self.lib.oc_set_momentum(self.h, len(k), _ptr(k), _ptr(r), int(n_matsubara)))

    def obs_kw(self) -> np.ndarray:
        """Accumulated sign * S_sigma(K, w_n) as complex [2, n_k, n_matsubara]."""
        k, r, nm = self._kw
        out = np.zeros(2 * len(k) * nm * 2)
        self._check(self.lib.oc_get_obs_kw(self.h, _ptr(out)))
        out = out.reshape(2, len(k), nm, 2)
        return out[..., 0] + 1j * out[..., 1]

    def g0_matsubara(self, sector, k, n) -> complex:
        out = np.zeros(2)
        self._check(self.lib.oc_g0_matsubara(self.h, sector, k, n, _ptr(out)))
        return complex(out[0], out[1])

    def estimate_G(self, sector, x, y, tau) -> float:
        out = C.c_double()
        self._check(self.lib.oc_estimate_G(self.h, sector, x, y, tau, C.byref(out)))
        return out.value

    def g0(self, sector, x, y, dtau) -> float:
        return self.lib.oc_g0_lookup(self.h, sector, x, y, dtau)


def split_obs(obs: np.ndarray, n_disp: int, n_tau_out: int) -> dict:
    """Normalised observables of an accumulator vector (sign-weighted means)."""
    cnt, ssum = obs[0], obs[1]
    h = OC_OBS_HEADER
    g = obs[h:].reshape(2, n_disp, n_tau_out)
    return dict(count=cnt, sign=ssum / cnt, order=obs[2] / ssum, order2=obs[3] / ssum,
                p0=obs[4] / ssum, D=obs[5] / ssum, n_up=obs[6] / ssum, n_dn=obs[7] / ssum,
                G=g / ssum)
