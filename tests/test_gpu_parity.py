"""GPU submatrix path vs the CPU rank-1 oracle, through the C ABI.

Both sides draw the same proposals from their own Philox4x32-10
implementations, so the chains must take identical accept/reject decisions;
N must agree to 1e-10 (normwise, FP64) and observables to rounding.  Sizes
span several 64-wide tiles with a ragged tail; block lengths and Gamma
capacities are varied to show the chain does not depend on the blocking.
"""

import math

import numpy as np
import pytest

from ctaux_inputs import anderson_semicircle, dca_square, hubbard_atom, hubbard_dimer, hubbard_plaquette
from oracle import OracleChain, draws

pytestmark = pytest.mark.gpu

N_TOL = 1e-10          # ||N_gpu - N_oracle||_F / ||N_oracle||_F, FP64
# Per-proposal ratios: the GPU takes them from Gamma~^{-1} grown by partitioning
# (unpivoted), the oracle from rank-1 updated N; a ratio that is small because
# its Schur complement cancels carries a relative error of eps times that
# cancellation on both sides.  Decisions are compared exactly.
R_TOL = 1e-6


def _ctaux():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1010_3690_amd import ctaux
    return ctaux


def _plaquette(**kw):
    a = dict(beta=4.0, U=4.0, K=1.0, n_tau=4096, n_fine=16, superlattice=[[2, 0], [0, 2]])
    a.update(kw)
    return dca_square(**a)


def _cluster16(**kw):
    a = dict(L=4, beta=3.0, U=4.0, K=20.0, n_tau=4096, n_fine=16, density=0.9)
    a.update(kw)
    return dca_square(**a)


def _run_pair(ctaux, w, n_prop, opts, chain_id=0, steps=1):
    print(f"[parity] workload={w.name} nc={w.n_sites} K={w.K} n_prop={n_prop} k_max={opts.k_max} "
          f"k_cap={opts.k_cap} prec={opts.precision}", flush=True)
    gb = ctaux.CtauxBatch([w], opts)
    oc = OracleChain(w, seed=opts.seed, chain_id=chain_id, p_flip=opts.p_flip, meas_every=opts.meas_every,
                     n_therm=opts.n_therm, n_tau_out=opts.n_tau_out, n_cap=opts.n_cap)
    oc.set_log(opts.log_cap)
    per = n_prop // steps
    for _ in range(steps):
        gb.run(per)
        oc.run(per)
    return gb, oc


def near_ties(seed, chain, R, rel=1e-9):
    """Proposals whose uniform lies within rel |R| of |R| (where the two sides'
    roundings could decide differently; the tie rule is u < |R|)."""
    u = np.array([draws(seed, chain, i)[1] for i in range(len(R))])
    return int(np.sum(np.abs(u - np.abs(R)) < rel * np.abs(R)))


def _compare(gb, oc, n_prop, chain=0, n_tol=N_TOL, check_n=True, seed=None):
    acc_g, R_g = gb.decisions(chain, 0, n_prop)
    acc_o, R_o = oc.get_log(0, n_prop)
    if seed is not None:
        print(f"[parity] chain {chain}: {near_ties(seed, chain, R_o)} near ties in {n_prop} proposals", flush=True)
    first_bad = np.nonzero(acc_g != acc_o)[0]
    assert first_bad.size == 0, f"decisions diverge at proposal {first_bad[:5]}"
    np.testing.assert_allclose(R_g, R_o, rtol=R_TOL, atol=1e-300)
    st = gb.stats(chain)
    assert st["proposals"] == oc.proposals_done
    assert st["order"] == oc.order
    assert st["sign"] == oc.sign
    ids_g, tau_g, site_g, s_g = gb.config(chain)
    ids_o, tau_o, site_o, s_o = oc.config()
    assert np.array_equal(ids_g, ids_o)
    assert np.array_equal(tau_g, tau_o)
    assert np.array_equal(site_g, site_o)
    assert np.array_equal(s_g, s_o)
    if check_n and oc.order > 0:
        for sec in (0, 1):
            Ng, No = gb.N(chain, sec), oc.N(sec)
            err = np.linalg.norm(Ng - No) / np.linalg.norm(No)
            assert err <= n_tol, f"sector {sec}: N relative error {err:.3e}"
    return st


def _compare_obs(og, oo):
    """Observables measured on identical configurations: per-measurement averages
    agree to the rounding of the estimator (N agrees to 1e-10; the G(tau)
    estimator sums O(n) terms with cancellation)."""
    assert og[0] == oo[0] and og[0] > 0
    np.testing.assert_allclose(og / og[0], oo / oo[0], rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("name,make,n_prop,kmax,kcap,gamma_tol", [
    ("plaquette", _plaquette, 6000, 64, 64, 1e-8),
    # isolated doped plaquette with diagonal hopping: <sign> ~ 0.5
    ("plaquette_sign", hubbard_plaquette, 6000, 64, 64, 1e-8),
    ("semicircle_k16", lambda: anderson_semicircle(n_tau=4096), 8000, 16, 16, 1e-8),
    ("dimer_k7_cap3", lambda: hubbard_dimer(beta=2.0, U=2.0, n_tau=2001), 4000, 7, 3, 1e-8),
    ("cluster16", _cluster16, 6000, 64, 32, 1e-8),
    # Gamma^{-1} always from the pivoted Gauss-Jordan elimination
    ("plaquette_gj", _plaquette, 6000, 64, 64, -1.0),
    ("cluster16_gj", _cluster16, 6000, 64, 32, -1.0),
    # rank-k update on 32x32 output tiles
    ("cluster16_tile32", _cluster16, 6000, 64, 32, 1e-8),
])
def test_decisions_and_N_match_oracle(name, make, n_prop, kmax, kcap, gamma_tol):
    ctaux = _ctaux()
    w = make()
    opts = ctaux.Options(k_max=kmax, k_cap=kcap, n_cap=2048, log_cap=n_prop, meas_every=kmax,
                         n_tau_out=8, recompute_every=0, seed=3, gamma_tol=gamma_tol,
                         rankk_tile=32 if name.endswith("tile32") else 64)
    gb, oc = _run_pair(ctaux, w, n_prop, opts, steps=2)
    st = _compare(gb, oc, n_prop, seed=opts.seed)
    assert st["accepted"] > 50
    if name == "plaquette_sign":   # both signs occurred
        assert gb.stats(0)["sign"] in (1.0, -1.0) and 0 < gb.obs(0)[1] < gb.obs(0)[0]
    if gamma_tol < 0:   # every sector-block with changes took the elimination
        assert 0 < st["gj_fallbacks"] <= 2 * st["blocks"]
    _compare_obs(gb.obs(0), oc.obs())


def test_block_independence():
    """k_max = 1 (rank-1 in disguise), odd k and a tiny Gamma give one chain."""
    ctaux = _ctaux()
    w = _plaquette()
    n_prop = 3000
    logs = []
    for kmax, kcap in ((1, 1), (13, 2), (64, 64), (128, 5)):
        opts = ctaux.Options(k_max=kmax, k_cap=kcap, n_cap=512, log_cap=n_prop, meas_every=16,
                             recompute_every=0, seed=8)
        gb = ctaux.CtauxBatch([w], opts)
        gb.run(n_prop)
        logs.append(gb.decisions(0, 0, n_prop)[0])
        gb.close()
    for l in logs[1:]:
        assert np.array_equal(l, logs[0])


def test_thermalisation_and_meas_cadence_match_oracle():
    """n_therm > 0 and a measurement interval that is not a multiple of k_max:
    blocks are cut at the measurement points past n_therm; decisions, N and the
    accumulated observables (same count) equal the oracle's."""
    ctaux = _ctaux()
    w = _cluster16()
    n_prop = 5000
    opts = ctaux.Options(k_max=64, k_cap=48, n_cap=1024, log_cap=n_prop, meas_every=48, n_therm=1000,
                         n_tau_out=8, recompute_every=0, seed=9)
    gb, oc = _run_pair(ctaux, w, n_prop, opts, steps=2)
    _compare(gb, oc, n_prop, seed=opts.seed)
    og, oo = gb.obs(0), oc.obs()
    assert og[0] == oo[0] == (n_prop // 48 - 1000 // 48)
    _compare_obs(og, oo)


def test_momentum_matsubara_measurement_matches_oracle():
    """Measurement in cluster momenta and Matsubara frequencies: three chains of
    different Nc (4x4 DCA cluster, the sign-problem plaquette, the dimer) in one
    batch, with no G(tau) bins (n_tau_out = 0).  The sign-weighted S(K, w_n)
    accumulators equal the oracle's (element by element; the same
    configurations are measured) and G0(K, i w_n) equals the oracle's transform
    of the interpolated tables."""
    ctaux = _ctaux()
    ws = [_cluster16(), hubbard_plaquette(), hubbard_dimer(beta=2.0, U=2.0, n_tau=2001)]
    n_prop, nm = 3000, 6
    opts = ctaux.Options(k_max=64, k_cap=48, n_cap=1024, log_cap=n_prop, meas_every=64, n_tau_out=0,
                         n_matsubara=nm, recompute_every=16, seed=4)
    gb = ctaux.CtauxBatch(ws, opts)
    gb.run(n_prop)
    for c, w in enumerate(ws):
        oc = OracleChain(w, seed=4, chain_id=c, meas_every=64, n_tau_out=2, n_cap=1024)
        oc.set_momentum(w.kvecs, w.site_pos, nm)
        oc.set_log(n_prop)
        oc.run(n_prop)
        _compare(gb, oc, n_prop, chain=c)
        og, oo = gb.obs(c), oc.obs()
        assert og[0] == oo[0] > 0
        np.testing.assert_allclose(og[:8] / og[0], oo[:8] / oo[0], rtol=1e-7, atol=1e-9)
        S_g, G0_g = gb.obs_kw(c)
        S_o = oc.obs_kw()
        scale = np.abs(S_o).max()
        print(f"[kw] chain {c} nc={w.n_sites}: max |S| {scale:.3e}, max diff {np.abs(S_g - S_o).max():.3e}",
              flush=True)
        np.testing.assert_allclose(S_g, S_o, rtol=1e-8, atol=1e-10 * scale)
        for sec in (0, 1):
            for q in range(len(w.kvecs)):
                for n in range(nm):
                    go = oc.g0_matsubara(sec, q, n)
                    assert abs(G0_g[sec, q, n] - go) <= 1e-10 * abs(go) + 1e-13, (sec, q, n)


def test_batched_chains_match_their_oracles():
    ctaux = _ctaux()
    ws = [_plaquette(), hubbard_dimer(beta=2.0, U=2.0, n_tau=2001), _plaquette(beta=2.0, U=6.0),
          _cluster16(K=5.0), anderson_semicircle(n_tau=4096)]
    n_prop = 3000
    # ~94 blocks per chain with the FP64 refinement schedule of production runs
    opts = ctaux.Options(k_max=32, k_cap=24, n_cap=1024, log_cap=n_prop, meas_every=32, n_tau_out=8,
                         recompute_every=16, seed=11)
    gb = ctaux.CtauxBatch(ws, opts)
    gb.run(n_prop)
    for c, w in enumerate(ws):
        oc = OracleChain(w, seed=opts.seed, chain_id=c, p_flip=opts.p_flip, meas_every=opts.meas_every,
                         n_tau_out=opts.n_tau_out, n_cap=opts.n_cap)
        oc.set_log(n_prop)
        oc.run(n_prop)
        _compare(gb, oc, n_prop, chain=c)
        _compare_obs(gb.obs(c), oc.obs())


def test_many_chains_match_their_oracles():
    """Nine chains: the many-chain launch shapes (chain grids with all
    workgroups of a chain on one XCD, Bc as a persistent product of its own,
    one wave per skinny item) against the oracle, chain by chain."""
    ctaux = _ctaux()
    ws = [_plaquette(beta=3.0 + 0.5 * c, U=3.0 + c, K=5.0 + 3 * c) for c in range(4)]
    ws += [_cluster16(K=10.0 * (c + 1)) for c in range(3)]   # orders ~90: two 64-wide tiles, ragged
    ws += [hubbard_dimer(beta=2.0, U=2.0, n_tau=2001), anderson_semicircle(n_tau=4096)]
    n_prop = 4000
    opts = ctaux.Options(k_max=32, k_cap=24, n_cap=1024, log_cap=n_prop, meas_every=32, n_tau_out=8,
                         recompute_every=16, seed=5)
    print(f"[parity] {len(ws)} chains, n_prop={n_prop}", flush=True)
    gb = ctaux.CtauxBatch(ws, opts)
    gb.run(n_prop)
    for c, w in enumerate(ws):
        oc = OracleChain(w, seed=opts.seed, chain_id=c, p_flip=opts.p_flip, meas_every=opts.meas_every,
                         n_tau_out=opts.n_tau_out, n_cap=opts.n_cap)
        oc.set_log(n_prop)
        oc.run(n_prop)
        _compare(gb, oc, n_prop, chain=c)
        _compare_obs(gb.obs(c), oc.obs())


@pytest.mark.parametrize("tile", [64, 32])
def test_config4_shape_chains_match_their_oracles(tile):
    """The batched workload at full shape: 512 chains of the mix (Nc in
    {4, 8, 16, 32}, beta in [4, 12], U in [4, 8], K = 1) with the options of the
    batched bench (k = 64, Gamma capacity 64, the FP64 refinement schedule, both
    rank-k tile sizes).  Eight chains, two of each Nc and four of them above
    index 256 (the per-chain tile prefixes carry across 256-chain chunks), take
    the oracle's decisions and ratios and end with its configuration, N (1e-10)
    and observables."""
    import torch
    from ctaux_inputs import batched_mix
    ctaux = _ctaux()
    ws = batched_mix(n_chains=512, seed=0, n_tau=2048, n_fine=16)
    n_prop = 64 * 40
    opts = ctaux.Options(k_max=64, k_cap=64, recompute_every=64, meas_every=64, n_tau_out=8, n_cap=2048, seed=0,
                         log_cap=n_prop, rankk_tile=tile)
    print(f"[config4] 512 chains, tile {tile}", flush=True)
    gb = ctaux.CtauxBatch(ws, opts)
    gb.run(n_prop)
    for c in (5, 508, 3, 511, 1, 502, 0, 507):
        w = ws[c]
        oc = OracleChain(w, seed=0, chain_id=c, meas_every=64, n_tau_out=8, n_cap=2048)
        oc.set_log(n_prop)
        oc.run(n_prop)
        print(f"[config4] chain {c} nc={w.n_sites} order {oc.order}", flush=True)
        _compare(gb, oc, n_prop, chain=c, seed=0)
        _compare_obs(gb.obs(c), oc.obs())
    gb.close()
    del gb
    torch.cuda.empty_cache()


def test_refinement_keeps_fp64_N():
    ctaux = _ctaux()
    w = _cluster16()
    n_prop = 4000
    opts = ctaux.Options(k_max=64, k_cap=48, n_cap=1024, log_cap=n_prop, recompute_every=4, seed=5)
    gb, oc = _run_pair(ctaux, w, n_prop, opts)
    _compare(gb, oc, n_prop)
    drift = gb.recompute()
    assert drift < 1e-11
    assert gb.stats(0)["max_drift"] < 1e-11
    _compare(gb, oc, n_prop)


def test_fp32_storage_error_and_refinement():
    """FP32 N: error against the FP64 inverse of the same configuration."""
    ctaux = _ctaux()
    w = _cluster16()
    opts = ctaux.Options(k_max=64, k_cap=48, n_cap=1024, recompute_every=0, precision=ctaux.CTAUX_FP32,
                         seed=5)
    gb = ctaux.CtauxBatch([w], opts)
    gb.run(4000)
    ids, tau, site, s = gb.config(0)
    oc = OracleChain(w, n_cap=1024)
    oc.set_config(ids, tau, site, s)
    errs = []
    for sec in (0, 1):
        ref = np.linalg.inv(oc.Minv(sec))
        errs.append(np.linalg.norm(gb.N(0, sec) - ref) / np.linalg.norm(ref))
    assert max(errs) < 1e-4, errs
    drift = gb.recompute()
    assert drift == pytest.approx(max(errs), rel=0.5)
    for sec in (0, 1):
        ref = np.linalg.inv(oc.Minv(sec))
        # after the FP64 Newton step N is the FP32 rounding of the FP64 inverse
        assert np.linalg.norm(gb.N(0, sec) - ref) / np.linalg.norm(ref) < 1e-6


def test_bf16x3_storage_error_and_refinement():
    """Split-BF16x3 rank-k update (FP32 storage): N against the FP64 inverse of
    the same configuration, beside FP32 MFMA on the same chain; a refinement
    restores the FP32 rounding of the FP64 inverse."""
    ctaux = _ctaux()
    w = _cluster16()
    errs = {}
    for prec in (ctaux.CTAUX_FP32, ctaux.CTAUX_BF16X3):
        opts = ctaux.Options(k_max=64, k_cap=48, n_cap=1024, recompute_every=0, precision=prec, seed=5,
                             log_cap=4000)
        gb = ctaux.CtauxBatch([w], opts)
        gb.run(4000)
        ids, tau, site, s = gb.config(0)
        oc = OracleChain(w, n_cap=1024)
        e = []
        for sec in (0, 1):
            ref = np.linalg.inv(oc.M_of(sec, tau, site, s))
            e.append(np.linalg.norm(gb.N(0, sec) - ref) / np.linalg.norm(ref))
        errs[prec] = max(e)
        gb.recompute()
        for sec in (0, 1):
            ref = np.linalg.inv(oc.M_of(sec, tau, site, s))
            assert np.linalg.norm(gb.N(0, sec) - ref) / np.linalg.norm(ref) < 1e-6
        if prec == ctaux.CTAUX_BF16X3:
            # the first decisions (before N carries enough error to flip one) are the oracle's
            oc2 = OracleChain(w, seed=5, n_cap=1024)
            oc2.set_log(1000)
            oc2.run(1000)
            assert np.array_equal(gb.decisions(0, 0, 1000)[0], oc2.get_log(0, 1000)[0])
    print(f"[bf16x3] N error after 4000 proposals: FP32 {errs[ctaux.CTAUX_FP32]:.2e}, "
          f"BF16x3 {errs[ctaux.CTAUX_BF16X3]:.2e}", flush=True)
    assert errs[ctaux.CTAUX_BF16X3] < 1e-2


def test_u_zero_walk():
    ctaux = _ctaux()
    w = hubbard_atom(beta=2.0, U=0.0, K=3.0)
    n_prop = 4000
    opts = ctaux.Options(k_max=32, k_cap=8, n_cap=256, log_cap=n_prop, meas_every=32, n_tau_out=4,
                         recompute_every=0, seed=2)
    gb, oc = _run_pair(ctaux, w, n_prop, opts)
    _compare(gb, oc, n_prop)


def test_capacity_error_matches_oracle():
    ctaux = _ctaux()
    w = _plaquette()
    opts = ctaux.Options(k_max=64, k_cap=64, n_cap=12, log_cap=4000, recompute_every=0, seed=1)
    gb = ctaux.CtauxBatch([w], opts)
    with pytest.raises(ctaux.CtauxError) as e:
        gb.run(4000)
    assert e.value.code == ctaux.CTAUX_ECAPACITY
    oc = OracleChain(w, seed=1, n_cap=12)
    oc.set_log(4000)
    with pytest.raises(Exception):
        oc.run(4000)
    done = oc.proposals_done
    st = gb.stats(0)
    assert st["proposals"] == done and st["order"] == oc.order == 12
    _compare(gb, oc, done)


def test_drift_tol_stops_the_chains():
    """A refinement whose drift exceeds drift_tol stops the chain with
    CTAUX_ENUMERIC.  A tolerance below any FP64 drift forces it at the first
    refinement (after block 1: a chain's refinement interval starts at one
    block): both chains of the batch stop there, although the next block's
    start has already been launched, their decisions up to there equal the
    oracle's, and a further run reports the same error."""
    ctaux = _ctaux()
    w = _plaquette()
    n_prop = 64 * 12
    opts = ctaux.Options(k_max=64, k_cap=64, n_cap=512, log_cap=n_prop, recompute_every=4, seed=3,
                         drift_tol=1e-300)
    gb = ctaux.CtauxBatch([w, w], opts)
    with pytest.raises(ctaux.CtauxError) as e:
        gb.run(n_prop)
    assert e.value.code == ctaux.CTAUX_ENUMERIC and "drift_tol" in str(e.value)
    for c in range(2):
        st = gb.stats(c)
        assert st["status"] == ctaux.CTAUX_ENUMERIC
        # the first refinement follows block 1; nothing runs after it
        assert st["proposals"] == 64, st["proposals"]
        oc = OracleChain(w, seed=3, chain_id=c, n_cap=512)
        oc.set_log(st["proposals"])
        oc.run(st["proposals"])
        acc_g, _ = gb.decisions(c, 0, st["proposals"])
        acc_o, _ = oc.get_log(0, st["proposals"])
        assert np.array_equal(acc_g, acc_o)
    with pytest.raises(ctaux.CtauxError) as e2:
        gb.run(64)
    assert e2.value.code == ctaux.CTAUX_ENUMERIC


def test_full_size_cluster_N_is_inverse_of_definition():
    """4x4 cluster at order ~1000 (k = 64): N equals the FP64 inverse of its definition."""
    ctaux = _ctaux()
    w = dca_square(L=4, beta=8.0, U=8.0, K=620.0, density=0.9, n_tau=8192)
    opts = ctaux.Options(k_max=64, k_cap=64, n_cap=2048, recompute_every=64, seed=0, log_cap=4000)
    gb = ctaux.CtauxBatch([w], opts)
    gb.run(64 * 200)
    st = gb.stats(0)
    assert 700 < st["order"] < 1600, st
    ids, tau, site, s = gb.config(0)
    oc = OracleChain(w, n_cap=2048)
    oc.set_config(ids, tau, site, s)
    rng = np.random.default_rng(0)
    for sec in (0, 1):
        Minv = oc.Minv(sec)
        N = gb.N(0, sec)
        # sampled rows of N Minv = I
        rows = rng.choice(st["order"], 16, replace=False)
        P = N[rows] @ Minv
        E = np.zeros_like(P)
        E[np.arange(16), rows] = 1.0
        assert np.linalg.norm(P - E) / math.sqrt(16) < 1e-9
    # the first 4000 decisions agree with the oracle
    oc2 = OracleChain(w, seed=0, n_cap=2048)
    oc2.set_log(4000)
    oc2.run(4000)
    acc_g, R_g = gb.decisions(0, 0, 4000)
    acc_o, R_o = oc2.get_log(0, 4000)
    assert np.array_equal(acc_g, acc_o)
    np.testing.assert_allclose(R_g, R_o, rtol=R_TOL)


def test_checkpoint_restore_continues_the_chain():
    """A chain restored into a fresh batch takes the decisions of the
    uninterrupted chain and ends with the same configuration and N (both sides
    run the same kernels on the same data, so bit for bit)."""
    ctaux = _ctaux()
    w = _cluster16()
    n1, n2 = 2000, 3000
    opts = ctaux.Options(k_max=64, k_cap=32, n_cap=1024, log_cap=n1 + n2, meas_every=64,
                         n_tau_out=8, recompute_every=8, seed=5)
    a = ctaux.CtauxBatch([w], opts)
    a.run(n1)
    blob = a.checkpoint(0)
    b = ctaux.CtauxBatch([w], opts)
    b.restore(blob, 0)
    assert b.stats(0)["proposals"] == n1 and b.stats(0)["order"] == a.stats(0)["order"]
    a.run(n2)
    b.run(n2)
    acc_a, R_a = a.decisions(0, n1, n2)
    acc_b, R_b = b.decisions(0, n1, n2)
    assert np.array_equal(acc_a, acc_b) and np.array_equal(R_a, R_b)
    for x, y in zip(a.config(0), b.config(0)):
        assert np.array_equal(x, y)
    for sec in (0, 1):
        assert np.array_equal(a.N(0, sec), b.N(0, sec))
    assert np.array_equal(a.obs(0), b.obs(0))
    # a blob of another model is refused
    other = ctaux.CtauxBatch([_plaquette()], opts)
    with pytest.raises(ctaux.CtauxError) as e:
        other.restore(blob, 0)
    assert e.value.code == ctaux.CTAUX_EINVAL


def _n_vs_definition(ctaux, gb, oc, chain, tol):
    """||N - (e^V - G0(e^V - 1))^{-1}||_F / ||.||_F for both sectors; the
    definition is built by the oracle, inverted by LAPACK."""
    ids, tau, site, s = gb.config(chain)
    errs = []
    for sec in (0, 1):
        M = oc.M_of(sec, tau, site, s)
        Nref = np.linalg.inv(M)
        N = gb.N(chain, sec)
        errs.append(np.linalg.norm(N - Nref) / np.linalg.norm(Nref))
    assert max(errs) < tol, errs
    return errs


def test_config3_6x6_mixed_precision():
    """6x6 cluster, beta = 10, order ~3000, N stored in FP32 with the rank-k
    update on FP32 MFMA, FP64 recompute every 64 blocks.  The drift before a
    recompute is the N error of the mixed form; after it N is the FP64 inverse
    of its definition rounded to FP32."""
    ctaux = _ctaux()
    w = dca_square(L=6, beta=10.0, U=8.0, K=1800.0, density=0.9, n_tau=8192)
    opts = ctaux.Options(k_max=128, k_cap=64, n_cap=4096, precision=ctaux.CTAUX_FP32,
                         recompute_every=64, seed=0, log_cap=4000)
    print(f"[config3] nc={w.n_sites} K={w.K}", flush=True)
    gb = ctaux.CtauxBatch([w], opts)
    gb.run(128 * 280)
    st = gb.stats(0)
    print(f"[config3] order {st['order']} blocks {st['blocks']} max drift {st['max_drift']:.3e}", flush=True)
    assert 2000 < st["order"] < 4096, st
    assert st["max_drift"] < 1e-2
    drift = gb.recompute()
    oc = OracleChain(w, n_cap=4096)
    errs = _n_vs_definition(ctaux, gb, oc, 0, 1e-6)
    print(f"[config3] drift before recompute {drift:.3e}, N error after {max(errs):.3e}", flush=True)
    # the chain's first decisions are the oracle's
    oc2 = OracleChain(w, seed=0, n_cap=4096)
    oc2.set_log(4000)
    oc2.run(4000)
    acc_g, _ = gb.decisions(0, 0, 4000)
    acc_o, _ = oc2.get_log(0, 4000)
    assert np.array_equal(acc_g, acc_o)


def test_config5_cubic_nc100_eight_chains():
    """3D cluster Nc = 100 (bipartite periodic), beta = 6, half filling, eight
    chains batched.  FP64: every chain's first 4000 proposals take the
    oracle's decisions and ratios (oracles replayed in a process pool) and
    measure its observables.  Mixed form (FP32 storage, FP64 refresh every <= 32
    blocks), thermalised to order ~5000-6000: N after a refresh is the FP64
    inverse of its definition rounded to FP32."""
    import torch
    from ctaux_inputs import dca_cubic
    from oracle_pool import replay_many
    ctaux = _ctaux()
    w = dca_cubic(beta=6.0, U=8.0, K=4300.0, n_tau=8192)
    n_prop = 4000
    opts = ctaux.Options(k_max=128, k_cap=64, n_cap=8192, recompute_every=32, seed=0, meas_every=128,
                         n_tau_out=8, log_cap=n_prop)
    print(f"[config5] nc={w.n_sites} K={w.K}: FP64 parity over {n_prop} proposals", flush=True)
    gb = ctaux.CtauxBatch([w] * 8, opts)
    gb.run(n_prop)
    ref = replay_many([(w, 0, c, n_prop, 128, 8, 8192) for c in range(8)])
    for c in range(8):
        acc_g, R_g = gb.decisions(c, 0, n_prop)
        print(f"[config5] chain {c}: order {ref[c]['order']}, {near_ties(0, c, ref[c]['R'])} near ties",
              flush=True)
        assert np.array_equal(acc_g, ref[c]["acc"]), np.nonzero(acc_g != ref[c]["acc"])[0][:5]
        np.testing.assert_allclose(R_g, ref[c]["R"], rtol=R_TOL, atol=1e-300)
        assert gb.stats(c)["order"] == ref[c]["order"] and gb.stats(c)["sign"] == ref[c]["sign"]
        for x, y in zip(gb.config(c), ref[c]["config"]):
            assert np.array_equal(x, y)
        _compare_obs(gb.obs(c), ref[c]["obs"])
    gb.close()
    del gb
    torch.cuda.empty_cache()
    opts = ctaux.Options(k_max=128, k_cap=64, n_cap=8192, precision=ctaux.CTAUX_FP32,
                         recompute_every=32, seed=0, meas_every=128, n_tau_out=8)
    gb = ctaux.CtauxBatch([w] * 8, opts)
    gb.run(128 * 300)
    orders = [gb.stats(c)["order"] for c in range(8)]
    print(f"[config5] FP32 storage: orders {orders}, max drift {max(gb.stats(c)['max_drift'] for c in range(8)):.2e}",
          flush=True)
    assert all(4500 < o < 8192 for o in orders), orders
    assert len(set(orders)) > 1   # independent streams per chain
    gb.recompute()
    oc = OracleChain(w, n_cap=8192)
    errs = _n_vs_definition(ctaux, gb, oc, 3, 1e-6)
    print(f"[config5] chain 3 N error after recompute {max(errs):.3e}", flush=True)


def test_strongly_coupled_chain_holds_fp64_without_refinement():
    """Nc = 32, beta = 7.08, U = 7.13, K = 1 (gamma ~ 7.4, N^{-1} conditioned
    ~1e5): 60 blocks of 64 proposals without any refinement keep N within 1e-9
    of the inverse of its definition (repeated changes of a vertex update its
    slot of Gamma instead of adding a nearly equal column), and one
    refinement brings it to FP64 rounding."""
    from ctaux_inputs.workloads import _MIX_LATTICES
    ctaux = _ctaux()
    w = dca_square(beta=7.0812185938101795, U=7.13460658748971, K=1.0, n_tau=2048, n_fine=16,
                   superlattice=_MIX_LATTICES[32])
    opts = ctaux.Options(k_max=64, k_cap=64, n_cap=2048, recompute_every=0, seed=0, drift_tol=0.0,
                         meas_every=64, n_tau_out=8, log_cap=4000)
    print(f"[strong] nc={w.n_sites} K={w.K}", flush=True)
    gb = ctaux.CtauxBatch([w], opts)
    gb.run(64 * 60)
    oc = OracleChain(w, n_cap=2048)
    errs = _n_vs_definition(ctaux, gb, oc, 0, 1e-9)
    d1 = gb.recompute()
    d2 = gb.recompute()
    print(f"[strong] order {gb.stats(0)['order']} N error {max(errs):.3e} drift {d1:.3e} then {d2:.3e}",
          flush=True)
    assert d1 < 1e-9 and d2 < 1e-12
    # the LAPACK inverse that serves as reference carries cond(M) eps ~ 1e-11 itself
    _n_vs_definition(ctaux, gb, oc, 0, 1e-10)
    oc2 = OracleChain(w, seed=0, n_cap=2048)
    oc2.set_log(64 * 60)
    oc2.run(64 * 60)
    acc_g, R_g = gb.decisions(0, 0, 64 * 60)
    acc_o, R_o = oc2.get_log(0, 64 * 60)
    assert np.array_equal(acc_g, acc_o)
    np.testing.assert_allclose(R_g, R_o, rtol=R_TOL)


def test_autotune_keeps_the_chain():
    """The autotuner's candidates continue the same thermalised chains; the
    chosen options are one of the timed candidates, each timed three times
    (median and spread reported), and a candidate with k_max > meas_every is
    skipped."""
    ctaux = _ctaux()
    from paper_1010_3690_amd.autotune import autotune
    ws = [_plaquette(beta=3.0 + 0.25 * i) for i in range(6)]
    opts = ctaux.Options(k_max=64, k_cap=64, n_cap=512, recompute_every=16, seed=2, meas_every=64)
    best, results = autotune(ws, opts, candidates=((16, 32), (32, 64), (64, 32), (128, 64)),
                             warmup_proposals=64 * 20, trial_proposals=64 * 8)
    timed = [r for r in results if "updates_per_s" in r]
    assert len(results) == 4 and len(timed) == 3
    assert results[3].get("skipped") and results[3]["k_max"] == 128
    for r in timed:
        assert r["trials"] == 3 and 0 < r["min_updates_per_s"] <= r["updates_per_s"] <= r["max_updates_per_s"]
    assert (best.k_max, best.rankk_tile) in ((16, 32), (32, 64), (64, 32))
