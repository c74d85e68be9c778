"""Pair updates (two vertices inserted or removed at once; Gamma grows by two
rows and columns, Sec. IV B) on the GPU against the CPU oracle, through the C
ABI.

The oracle takes a pair's ratio from the 2x2 Schur complement of the enlarged
N^{-1} (insertion) or the complementary 2x2 minor of N (removal); the GPU
applies the two changes one after the other to Gamma~^{-1} in LDS (new slots
by partitioning, vertices already in P by the repeated-change formulas) and
multiplies the two sector ratios.  Decisions must be identical, ratios agree
to R_TOL, configurations exactly and N to 1e-10.  The cases cover pairs that
overfill Gamma (the block ends before them), blocks cut because a pair
insertion's two candidates would exceed k_max, pair removals of vertices
changed earlier in the same block, U = 0 (no Gamma) and a batch of chains.
"""

import numpy as np
import pytest

from ctaux_inputs import anderson_semicircle, dca_square, hubbard_atom, hubbard_dimer
from oracle import OracleChain
from test_gpu_parity import _compare, _compare_obs, _ctaux

pytestmark = pytest.mark.gpu


def _plaquette(**kw):
    a = dict(beta=4.0, U=4.0, K=1.0, n_tau=4096, n_fine=16, superlattice=[[2, 0], [0, 2]])
    a.update(kw)
    return dca_square(**a)


def _cluster16(**kw):
    a = dict(L=4, beta=3.0, U=4.0, K=20.0, n_tau=4096, n_fine=16, density=0.9)
    a.update(kw)
    return dca_square(**a)


def _oracle(w, opts, chain_id=0):
    oc = OracleChain(w, seed=opts.seed, chain_id=chain_id, p_flip=opts.p_flip, meas_every=opts.meas_every,
                     n_therm=opts.n_therm, n_tau_out=opts.n_tau_out, n_cap=opts.n_cap, p_pair=opts.p_pair)
    oc.set_log(opts.log_cap)
    return oc


def _opts(ctaux, n_prop, **kw):
    a = dict(k_max=64, k_cap=64, n_cap=2048, log_cap=n_prop, meas_every=64, n_tau_out=8, recompute_every=0,
             seed=5, p_pair=0.3)
    a.update(kw)
    return ctaux.Options(**a)


@pytest.mark.parametrize("name,make,n_prop,kw", [
    ("plaquette", _plaquette, 6000, dict()),
    ("cluster16_cap32", _cluster16, 6000, dict(k_cap=32)),
    # small Gamma: pairs often do not fit and end the block before them
    ("semicircle_k16_cap4", lambda: anderson_semicircle(n_tau=4096), 6000, dict(k_max=16, k_cap=4, meas_every=16,
                                                                                 p_pair=0.6)),
    # k_max = 3, k_cap = 2: pair insertions cut blocks at their candidates
    ("dimer_k3_cap2", lambda: hubbard_dimer(beta=2.0, U=2.0, n_tau=2001), 4000, dict(k_max=3, k_cap=2,
                                                                                     meas_every=3, p_pair=0.7,
                                                                                     p_flip=0.1)),
    # mostly pair moves on a long block: removals of vertices inserted earlier in the block
    ("plaquette_pairs_only", _plaquette, 6000, dict(p_pair=0.8, p_flip=0.2)),
])
def test_pair_decisions_and_N_match_oracle(name, make, n_prop, kw):
    ctaux = _ctaux()
    w = make()
    opts = _opts(ctaux, n_prop, **kw)
    print(f"[pairs] {name} k_max={opts.k_max} k_cap={opts.k_cap} p_pair={opts.p_pair}", flush=True)
    gb = ctaux.CtauxBatch([w], opts)
    oc = _oracle(w, opts)
    for _ in range(2):
        gb.run(n_prop // 2)
        oc.run(n_prop // 2)
    st = _compare(gb, oc, n_prop, seed=opts.seed)
    assert st["accepted"] > 50
    _compare_obs(gb.obs(0), oc.obs())


def test_pair_chain_does_not_depend_on_blocking():
    """The same chain with k = 64 / Gamma 64 and k = 24 / Gamma 8: identical
    decisions, configuration and N (block boundaries move, the chain does not)."""
    ctaux = _ctaux()
    w = _plaquette()
    n_prop = 4800
    runs = []
    for k, cap in ((64, 64), (24, 8)):
        opts = _opts(ctaux, n_prop, k_max=k, k_cap=cap, meas_every=48, p_pair=0.5)
        print(f"[pairs] blocking k_max={k} k_cap={cap}", flush=True)
        gb = ctaux.CtauxBatch([w], opts)
        gb.run(n_prop)
        runs.append(gb)
    a, b = runs
    acc_a, R_a = a.decisions(0, 0, n_prop)
    acc_b, R_b = b.decisions(0, 0, n_prop)
    assert np.array_equal(acc_a, acc_b)
    np.testing.assert_allclose(R_a, R_b, rtol=1e-6, atol=1e-300)
    for x, y in zip(a.config(0), b.config(0)):
        assert np.array_equal(x, y)
    for sec in (0, 1):
        Na, Nb = a.N(0, sec), b.N(0, sec)
        assert np.linalg.norm(Na - Nb) / np.linalg.norm(Na) < 1e-10
    assert b.stats(0)["blocks"] > a.stats(0)["blocks"]


def test_pair_u_zero():
    """U = 0: every determinant ratio is 1, R = K^2/((n+1)(n+2)) or n(n-1)/K^2;
    no Gamma is kept (the bookkeeping alone decides the block)."""
    ctaux = _ctaux()
    w = hubbard_atom(beta=2.0, U=0.0, K=3.0)
    n_prop = 6000
    opts = _opts(ctaux, n_prop, k_max=32, k_cap=16, meas_every=32, p_pair=0.5)
    gb = ctaux.CtauxBatch([w], opts)
    oc = _oracle(w, opts)
    gb.run(n_prop)
    oc.run(n_prop)
    _compare(gb, oc, n_prop, check_n=False)


def test_pair_batch_of_chains():
    """Eight chains of different models in one batch, each against the oracle
    with its own chain id."""
    ctaux = _ctaux()
    ws = [_plaquette(U=3.0 + 0.5 * c) if c % 2 == 0 else _cluster16(beta=2.0 + 0.25 * c) for c in range(8)]
    n_prop = 3200
    opts = _opts(ctaux, n_prop, k_cap=32, p_pair=0.4, recompute_every=16)
    gb = ctaux.CtauxBatch(ws, opts)
    ocs = [_oracle(w, opts, chain_id=c) for c, w in enumerate(ws)]
    gb.run(n_prop)
    for c, oc in enumerate(ocs):
        print(f"[pairs] batch chain {c}", flush=True)
        oc.run(n_prop)
        _compare(gb, oc, n_prop, chain=c)
        _compare_obs(gb.obs(c), oc.obs())


def test_pair_fp32_storage():
    """Pairs with N stored in FP32 (the float instantiation of the pair path):
    the first 1200 decisions equal the oracle's (ratios to FP32 rounding), and
    after 4000 proposals N is within 1e-4 of the FP64 inverse of the chain's
    own configuration; a refinement restores it to FP32 rounding."""
    ctaux = _ctaux()
    w = _cluster16()
    n_first = 1200
    opts = _opts(ctaux, 4000, k_cap=48, n_cap=1024, precision=ctaux.CTAUX_FP32, p_pair=0.4)
    gb = ctaux.CtauxBatch([w], opts)
    oc = _oracle(w, opts)
    gb.run(n_first)
    oc.run(n_first)
    acc_g, R_g = gb.decisions(0, 0, n_first)
    acc_o, R_o = oc.get_log(0, n_first)
    assert np.array_equal(acc_g, acc_o)
    np.testing.assert_allclose(R_g, R_o, rtol=1e-3, atol=1e-300)
    gb.run(4000 - n_first)
    ids, tau, site, s = gb.config(0)
    ref_chain = OracleChain(w, n_cap=1024)
    ref_chain.set_config(ids, tau, site, s)
    errs = []
    for sec in (0, 1):
        ref = np.linalg.inv(ref_chain.Minv(sec))
        errs.append(np.linalg.norm(gb.N(0, sec) - ref) / np.linalg.norm(ref))
    assert max(errs) < 1e-4, errs
    gb.recompute()
    for sec in (0, 1):
        ref = np.linalg.inv(ref_chain.Minv(sec))
        assert np.linalg.norm(gb.N(0, sec) - ref) / np.linalg.norm(ref) < 1e-6
