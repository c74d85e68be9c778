"""Pins of the oracle's pair updates (two vertices inserted or removed at once,
Gamma enlarged by two rows and columns, Sec. IV B) against facts its code does
not compute: the Philox words the extra draws are defined from, numpy
determinants of N^{-1} built from its definition (Eq. Nmatrix) before and
after each proposal, exact diagonalisation, and the Poisson law of the U = 0
walk, which detailed balance keeps whatever the proposal mix.
"""

import math

import numpy as np
import pytest

from ctaux_inputs import anderson_bath, dca_square, hubbard_atom, hubbard_dimer
from ed import ED
from oracle import OracleChain, draws, philox4x32_10
from oracle.oracle import OracleError, pair_draws, split_obs


def _u53(hi, lo):
    return float(((int(hi) << 32) | int(lo)) >> 11) * 2.0 ** -53


def test_pair_draws_are_the_defined_philox_words():
    """u_spin2 = second word pair of tag 2, (u_tau2, u_pick2) = tag 3, counter
    (index lo, index hi, chain, tag), key = seed; the five single draws are
    unchanged."""
    seed, chain = (5 << 32) | 77, 9
    key = [seed & 0xffffffff, seed >> 32]
    for index in (0, 1, 1000, (3 << 32) + 17):
        ctr = [index & 0xffffffff, index >> 32, chain]
        x2 = philox4x32_10(ctr + [2], key)
        x3 = philox4x32_10(ctr + [3], key)
        v = pair_draws(seed, chain, index)
        assert v[0] == _u53(x2[2], x2[3])
        assert v[1] == _u53(x3[0], x3[1])
        assert v[2] == _u53(x3[2], x3[3])
        assert draws(seed, chain, index)[4] == _u53(x2[0], x2[1])


def _slogdets(c, tau, site, s):
    out = []
    for sec in (0, 1):
        if len(tau) == 0:
            out.append((1.0, 0.0))
        else:
            out.append(np.linalg.slogdet(c.M_of(sec, tau, site, s)))
    return out


def _after(cfg, lp):
    ids, tau, site, s = (np.array(a) for a in cfg)
    t = lp["type"]
    if t == 0:
        return np.append(tau, lp["tau"]), np.append(site, lp["site"]), np.append(s, lp["s_new"])
    if t == 3:
        return (np.append(tau, [lp["tau"], lp["tau2"]]), np.append(site, [lp["site"], lp["site2"]]),
                np.append(s, [lp["s_new"], lp["s2"]]))
    if t in (1, 4):
        drop = {lp["p"]} | ({lp["p2"]} if t == 4 else set())
        keep = np.array([i not in drop for i in range(len(tau))], dtype=bool)
        return tau[keep], site[keep], s[keep]
    s = s.copy()
    s[lp["p"]] = lp["s_new"]
    return tau, site, s


def _plaquette():
    return dca_square(beta=4.0, U=4.0, K=1.0, n_tau=4096, n_fine=16, superlattice=[[2, 0], [0, 2]])


@pytest.mark.parametrize("make,seed", [(_plaquette, 1), (lambda: anderson_bath(beta=4.0, U=3.0, n_tau=2048), 2)])
def test_pair_ratios_match_determinants(make, seed):
    """Every ratio of a walk with pair moves equals its prefactor times
    prod_sigma det N'^{-1} / det N^{-1} from numpy: K^2/((n+1)(n+2)) for a pair
    insertion, n(n-1)/K^2 for a pair removal (and the single-move factors)."""
    w = make()
    c = OracleChain(w, seed=seed, p_pair=0.4)
    c.run(400)
    seen = [0] * 5
    for _ in range(700):
        cfg = c.config()
        n = len(cfg[0])
        before = _slogdets(c, cfg[1], cfg[2], cfg[3])
        c.run(1)
        lp = c.last_proposal()
        t = lp["type"]
        if (t in (1, 2) and n == 0) or (t == 4 and n < 2):
            assert lp["R"] == 0.0 and lp["acc"] == 0
            continue
        seen[t] += 1
        if t == 4:
            assert lp["p"] != lp["p2"] and 0 <= lp["p"] < n and 0 <= lp["p2"] < n
        after = _slogdets(c, *_after(cfg, lp))
        ratio = 1.0
        for (s0, l0), (s1, l1) in zip(before, after):
            ratio *= s0 * s1 * math.exp(l1 - l0)
        K = w.K
        factor = {0: K / (n + 1), 1: n / K, 2: 1.0, 3: K * K / ((n + 1) * (n + 2)),
                  4: n * (n - 1) / (K * K)}[t]
        assert lp["R"] == pytest.approx(factor * ratio, rel=1e-8), (t, n)
        if lp["acc"]:
            # the chain's N is the inverse of its configuration's N^{-1}
            for sec in (0, 1):
                Mi = c.Minv(sec)
                if len(Mi):
                    assert np.abs(Mi @ c.N(sec) - np.eye(len(Mi))).max() < 1e-9
    assert min(seen) > 25, seen


def test_pair_proposal_mix_and_ranks():
    """The type thresholds (1 - p_flip - p_pair)/2, twice that, + p_pair/2,
    + p_pair, and the second removal rank skipping the first."""
    w = _plaquette()
    pf, pp = 0.2, 0.3
    c = OracleChain(w, seed=4, p_flip=pf, p_pair=pp)
    c.run(300)
    for _ in range(300):
        idx = c.proposals_done
        n = c.order
        c.run(1)
        lp = c.last_proposal()
        u = draws(4, 0, idx)
        a = 0.5 * (1.0 - pf - pp)
        want = 0 if u[0] < a else 1 if u[0] < 2 * a else 3 if u[0] < 2 * a + 0.5 * pp else \
            4 if u[0] < 2 * a + pp else 2
        assert lp["type"] == want
        if want == 4 and n >= 2:
            v = pair_draws(4, 0, idx)
            r1 = min(int(math.floor(n * u[3])), n - 1)
            r2 = min(int(math.floor((n - 1) * v[2])), n - 2)
            assert lp["p"] == r1 and lp["p2"] == (r2 + 1 if r2 >= r1 else r2)
        if want == 3:
            v = pair_draws(4, 0, idx)
            assert lp["tau"] == w.beta * u[2] and lp["tau2"] == w.beta * v[1]
            assert lp["s_new"] == (-1 if u[4] < 0.5 else 1) and lp["s2"] == (-1 if v[0] < 0.5 else 1)


def test_pair_options_are_checked():
    w = _plaquette()
    with pytest.raises(OracleError, match="p_pair"):
        OracleChain(w, p_flip=0.5, p_pair=0.6)
    with pytest.raises(OracleError, match="p_pair"):
        OracleChain(w, p_pair=-0.1)
    # capacity: a pair insertion at order n_cap - 1 stops the walk
    c = OracleChain(w, seed=1, n_cap=3, p_pair=0.9, p_flip=0.0)
    with pytest.raises(OracleError, match="n_cap"):
        c.run(10000)


def _bins(make_chain, w, n_chains, bins_per_chain, per_bin, n_therm, nto):
    out = []
    for seed in range(n_chains):
        c = make_chain(seed)
        c.run(n_therm)
        for _ in range(bins_per_chain):
            c.reset_obs()
            c.run(per_bin)
            out.append(split_obs(c.obs(), w.n_disp, nto))
    return out


def _mean_err(vals):
    v = np.asarray(vals, dtype=np.float64)
    return v.mean(axis=0), v.std(axis=0, ddof=1) / np.sqrt(len(v))


def _within(mean, err, exact, nsig=3.0):
    return np.all(np.abs(mean - exact) <= nsig * err + 1e-12)


@pytest.mark.parametrize("make", [lambda: hubbard_dimer(beta=2.0, U=2.0, n_tau=2001),
                                  lambda: anderson_bath(beta=4.0, U=3.0, n_tau=2048)])
def test_pair_walk_against_exact_diagonalisation(make):
    """With half of the insertions and removals made in pairs the walk still
    samples the CT-AUX weights: D, <n> and <k> = K - beta <V> of exact
    diagonalisation within 3 sigma."""
    w = make()
    nto = 4
    B = _bins(lambda sd: OracleChain(w, seed=sd, meas_every=4, n_tau_out=nto, p_pair=0.4),
              w, 4, 8, 15000, 4000, nto)
    sites = list(range(w.n_sites))
    ed = ED(w.meta["h1"], w.U, w.beta, sites)
    m, e = _mean_err([b["D"] for b in B])
    assert _within(m, e, np.mean([ed.double_occ(x) for x in sites]))
    m, e = _mean_err([b["order"] for b in B])
    assert _within(m, e, w.K - w.beta * ed.potential())
    m, e = _mean_err([b["n_up"] for b in B])
    assert _within(m, e, np.mean([ed.density(x, 0) for x in sites]))


def test_pair_walk_u_zero_is_poisson():
    """At U = 0 every determinant ratio is 1; with pair moves (pair insert
    K^2/((n+1)(n+2)), pair removal n(n-1)/K^2) the order is still Poisson(K)."""
    K = 3.0
    w = hubbard_atom(beta=2.0, U=0.0, K=K)
    B = _bins(lambda sd: OracleChain(w, seed=sd, meas_every=2, p_pair=0.5), w, 4, 10, 10000, 2000, 16)
    for key, exact in (("order", K), ("order2", K + K * K), ("p0", math.exp(-K))):
        m, e = _mean_err([b[key] for b in B])
        assert _within(m, e, exact), (key, m, e, exact)
