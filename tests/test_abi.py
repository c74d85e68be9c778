"""The C-ABI library loads, exports what include/ctaux.h declares and
validates arguments on the host (no GPU needed, no compute call made)."""

import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from ctaux_inputs import dca_square

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1010_3690_amd import ctaux
    if not os.path.exists(ctaux.LIB_PATH):
        from paper_1010_3690_amd.build import build
        build()
    return ctaux.load_library()


def _declared():
    src = open(os.path.join(ROOT, "include", "ctaux.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ctaux_\w+)\s*\(", src)))


def test_every_declared_symbol_is_exported(lib):
    from paper_1010_3690_amd import ctaux
    out = subprocess.run(["nm", "-D", "--defined-only", ctaux.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (ctaux_\w+)", out))
    declared = _declared()
    assert len(declared) >= 15
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    assert set(ctaux.EXPORTED) == set(declared)


def _model_and_opts(ctaux, **over):
    w = dca_square(L=2, beta=2.0, U=4.0, n_tau=256, n_fine=8)
    sd = np.ascontiguousarray(w.site_disp, np.int32)
    g = np.ascontiguousarray(w.g0_up)
    m = ctaux._Model(w.beta, w.U, w.K, w.n_sites, w.n_tau, w.n_disp, sd.ctypes.data, g.ctypes.data,
                     g.ctypes.data)
    o = ctaux.Options(**over)._c()
    return m, o, (sd, g)


def test_workspace_bytes_and_validation(lib):
    from paper_1010_3690_amd import ctaux
    m, o, keep = _model_and_opts(ctaux, n_cap=256)
    nb = lib.ctaux_workspace_bytes(C.byref(m), 1, C.byref(o))
    assert nb > 4 * 256 * 256 * 8          # four FP64 N buffers at least
    m2, o2, keep2 = _model_and_opts(ctaux, n_cap=256, precision=ctaux.CTAUX_FP32)
    assert lib.ctaux_workspace_bytes(C.byref(m2), 1, C.byref(o2)) < nb
    for bad in (dict(k_max=0), dict(k_max=129), dict(k_cap=65), dict(k_cap=8, k_max=4), dict(p_flip=1.5),
                dict(precision=7), dict(n_cap=0), dict(meas_every=0), dict(rankk_tile=16),
                dict(gamma_tol=float("nan")),
                # 2 (n_tau_out + 1) n_sites n_cap >= 2^31 (32-bit table indices): 2 * 4097 * 4 * 65536
                dict(n_tau_out=4096, n_cap=65536),
                # the proposal kernel's LDS (Gamma^-1 of both sectors plus two bytes per
                # vertex of the augmented configuration) exceeds 160 KB
                dict(n_cap=45000), dict(drift_target=-1.0), dict(recompute_mode=2),
                # pair updates: p_flip + p_pair <= 1, and room for a pair in a block
                dict(p_pair=0.9), dict(p_pair=-0.1), dict(p_pair=0.1, k_cap=1),
                dict(p_pair=0.1, k_max=1, k_cap=1)):
        mb, ob, kb = _model_and_opts(ctaux, **bad)
        assert lib.ctaux_workspace_bytes(C.byref(mb), 1, C.byref(ob)) == 0, bad
    # a non-finite table entry is rejected
    g = keep[1].copy()
    g[0, 3] = np.inf
    m.g0_up = g.ctypes.data
    assert lib.ctaux_workspace_bytes(C.byref(m), 1, C.byref(o)) == 0
    assert b"non-finite" in lib.ctaux_last_error(None)


def test_create_rejects_small_workspace(lib):
    from paper_1010_3690_amd import ctaux
    m, o, keep = _model_and_opts(ctaux, n_cap=64)
    h = C.c_void_p()
    rc = lib.ctaux_create(C.byref(m), 1, C.byref(o), None, 0, None, C.byref(h))
    assert rc == ctaux.CTAUX_ENOMEM
    assert not h.value
    assert b"workspace" in lib.ctaux_last_error(None)


def test_lds_bound_is_the_boundary(lib):
    """The largest n_cap accepted at k_cap = 64 leaves the proposal kernel within
    the 160 KB of LDS of a workgroup; one more vertex of capacity does not."""
    from paper_1010_3690_amd import ctaux
    ok, bad = [], []
    # 8 (2 * 64 * 65 + 12 * 64) + 4 * 64 + 2 (n_cap + 64) + 16 + 8192 <= 163840  <=>  n_cap <= 41272
    for n_cap in (16384, 41272, 41273, 49152):
        m, o, keep = _model_and_opts(ctaux, n_cap=n_cap)
        (ok if lib.ctaux_workspace_bytes(C.byref(m), 1, C.byref(o)) > 0 else bad).append(n_cap)
    assert ok == [16384, 41272] and bad == [41273, 49152], (ok, bad)
    assert b"LDS" in lib.ctaux_last_error(None)


def test_build_N_validation_without_gpu(lib):
    from paper_1010_3690_amd import ctaux
    m, o, keep = _model_and_opts(ctaux)
    assert lib.ctaux_build_N_workspace_bytes(C.byref(m), -1) == 0
    assert lib.ctaux_build_N_workspace_bytes(C.byref(m), 40000) == 0
    nb = lib.ctaux_build_N_workspace_bytes(C.byref(m), 100)
    assert nb > 100 * 100 * 8
    verts = (ctaux._Vertex * 2)(ctaux._Vertex(0, 0.5, 0, 1), ctaux._Vertex(1, 0.7, 9, 1))   # site 9 >= n_sites
    rc = lib.ctaux_build_N(C.byref(m), verts, 2, 0, None, 2, None, 0, None)
    assert rc == ctaux.CTAUX_EINVAL and b"vertex 1" in lib.ctaux_last_error(None)
    verts[1] = ctaux._Vertex(1, 0.7, 1, 1)
    out = C.c_void_p(256)   # never dereferenced: the workspace check fails first
    rc = lib.ctaux_build_N(C.byref(m), verts, 2, 0, out, 2, None, 0, None)
    assert rc == ctaux.CTAUX_ENOMEM
    assert lib.ctaux_build_N(C.byref(m), verts, 0, 0, None, 0, None, 0, None) == 0   # n = 0: nothing to do
