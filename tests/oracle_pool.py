"""Oracle replays in worker processes (test infrastructure).

Replaying several long chains with the rank-1 oracle is CPU-bound and
independent per chain; the parity tests run them in a pool of spawned
processes (fresh interpreters: they never touch the GPU)."""

from __future__ import annotations

import multiprocessing as mp

from oracle import OracleChain


def replay(args):
    """(workload, seed, chain, n_prop, meas_every, n_tau_out, n_cap) -> the
    oracle's decision log, observables, configuration, sign and order."""
    w, seed, chain, n_prop, meas_every, n_tau_out, n_cap = args
    oc = OracleChain(w, seed=seed, chain_id=chain, meas_every=meas_every, n_tau_out=n_tau_out, n_cap=n_cap)
    oc.set_log(n_prop)
    oc.run(n_prop)
    acc, R = oc.get_log(0, n_prop)
    return {"acc": acc, "R": R, "obs": oc.obs(), "config": oc.config(), "sign": oc.sign, "order": oc.order}


def replay_many(jobs, processes=8):
    ctx = mp.get_context("spawn")
    with ctx.Pool(processes=min(processes, len(jobs))) as pool:
        return pool.map(replay, jobs)
