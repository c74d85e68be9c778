"""The allocation-free entry point ctaux_build_N_noalloc against ctaux_build_N
(the same kernels on a caller workspace), through the C ABI: identical
results on two calls in a row, the second smaller than the first (the shared
device scratch keeps the first call's contents), no device allocation during
the call, and the documented limits refused with EINVAL."""

import numpy as np
import pytest

from ctaux_inputs import dca_square
from ctaux_inputs.workloads import Workload
from oracle import OracleChain

pytestmark = pytest.mark.gpu


def _ctaux():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1010_3690_amd import ctaux
    return ctaux


def test_noalloc_matches_build_N_on_two_calls():
    import torch
    ctaux = _ctaux()
    w = dca_square(L=4, beta=3.0, U=4.0, K=20.0, n_tau=4096, n_fine=16, density=0.9)
    rng = np.random.default_rng(0)
    oc = OracleChain(w, n_cap=1024)
    for n in (700, 300):
        tau = rng.uniform(0.0, w.beta, n)
        site = rng.integers(0, w.n_sites, n).astype(np.int32)
        s = rng.choice([-1, 1], n).astype(np.int32)
        for sec in (0, 1):
            print(f"[noalloc] n={n} sector={sec}", flush=True)
            ref = ctaux.build_N(w, tau, site, s, sec)
            out = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            before = torch.cuda.memory_allocated()
            got = ctaux.build_N_noalloc(w, tau, site, s, sec, out=out)
            assert torch.cuda.memory_allocated() == before
            assert np.array_equal(got, ref)
            exact = np.linalg.inv(oc.M_of(sec, tau, site, s))
            assert np.linalg.norm(got - exact) / np.linalg.norm(exact) < 1e-10


def test_noalloc_limits():
    ctaux = _ctaux()
    w = dca_square(L=2, beta=3.0, U=4.0, K=5.0, n_tau=1024, n_fine=8)
    n = 1025
    tau = np.linspace(0.0, 2.9, n)
    site = np.zeros(n, np.int32)
    s = np.ones(n, np.int32)
    with pytest.raises(ctaux.CtauxError) as e:
        ctaux.build_N_noalloc(w, tau, site, s, 0)
    assert e.value.code == ctaux.CTAUX_EINVAL and "1024" in str(e.value)
    # tables of one sector beyond the scratch: 100 tables of 40000 points (32 MB)
    nc = 10
    g = np.full((nc * nc, 40000), 0.5)
    big = Workload("big", 3.0, 4.0, 5.0, nc, np.arange(nc * nc, dtype=np.int32), g, g)
    with pytest.raises(ctaux.CtauxError) as e:
        ctaux.build_N_noalloc(big, tau[:10], site[:10], s[:10], 0)
    assert e.value.code == ctaux.CTAUX_EINVAL and "scratch" in str(e.value)
