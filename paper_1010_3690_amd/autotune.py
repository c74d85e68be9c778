"""Autotuner for a batch: proposals per block (k_max, with the Gamma capacity
k_cap = min(k_max, 64)) and the rank-k output tile.

The Markov chain does not depend on the blocking (the same seed gives the same
decisions for every k), so all candidates continue the same thermalised
chains: the batch is thermalised once with the given options, every chain is
checkpointed, and each candidate restores the checkpoints into a batch of its
own and is timed on the same number of proposals.  The measurement cadence
(meas_every) and the refinement interval are left as given: they are choices
of the simulation, not of the implementation.
"""

from __future__ import annotations

import time
from dataclasses import replace

DEFAULT_CANDIDATES = tuple((k, tile) for k in (16, 32, 64, 96, 128) for tile in (64, 32))


def autotune(workloads, opts, candidates=DEFAULT_CANDIDATES, warmup_proposals=None,
             trial_proposals=None, repeats=3, device="cuda:0"):
    """Returns (best options, list of per-candidate results).

    warmup_proposals defaults to 200 blocks of opts.k_max proposals per chain,
    trial_proposals to 64 blocks of 64.  Every candidate is timed `repeats`
    times, each trial restoring the same checkpoints (so the trials run the
    same proposals); the median rate decides and the spread is reported.  A
    block ends at the next measurement, so candidates with k_max > meas_every
    run the same blocks as k_max = meas_every: they are reported as skipped.
    """
    import torch

    from . import ctaux

    workloads = list(workloads)
    warmup = warmup_proposals if warmup_proposals is not None else 200 * opts.k_max
    trial = trial_proposals if trial_proposals is not None else 64 * 64
    base = ctaux.CtauxBatch(workloads, opts, device)
    base.run(warmup)
    blobs = [base.checkpoint(c) for c in range(len(workloads))]
    base.close()
    del base
    results = []
    for k, tile in candidates:
        o = replace(opts, k_max=int(k), k_cap=min(int(k), 64), rankk_tile=int(tile))
        entry = {"k_max": o.k_max, "k_cap": o.k_cap, "rankk_tile": o.rankk_tile}
        if o.k_max > opts.meas_every:
            entry["skipped"] = f"k_max > meas_every = {opts.meas_every}"
            results.append(entry)
            continue
        gb = ctaux.CtauxBatch(workloads, o, device)
        rates = []
        for _ in range(max(int(repeats), 1)):
            for c, blob in enumerate(blobs):
                gb.restore(blob, c)
            p0 = sum(gb.stats(c)["proposals"] for c in range(len(workloads)))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gb.run(trial)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            p1 = sum(gb.stats(c)["proposals"] for c in range(len(workloads)))
            rates.append((p1 - p0) / dt)
        rates.sort()
        entry.update({"updates_per_s": rates[len(rates) // 2], "min_updates_per_s": rates[0],
                      "max_updates_per_s": rates[-1], "spread": (rates[-1] - rates[0]) / rates[len(rates) // 2],
                      "trials": len(rates)})
        results.append(entry)
        gb.close()
        del gb
    timed = [r for r in results if "updates_per_s" in r]
    if not timed:
        raise ValueError("no autotuner candidate has k_max <= meas_every")
    best = max(timed, key=lambda r: r["updates_per_s"])
    return replace(opts, k_max=best["k_max"], k_cap=best["k_cap"], rankk_tile=best["rankk_tile"]), results
