#!/usr/bin/env python
"""Throughput of the CT-AUX submatrix path on one MI355X.

Workload (step = one block: k_max = 64 proposals, the Gamma inner loop, the
rank-k update of N in both spin sectors, the measurement, and every 64 blocks
the FP64 refinement of N): 2D Hubbard DCA cluster 4x4 (Nc = 16), t = 1, U = 8,
beta = 8, <n> = 0.9, cluster G0(tau) from the coarse-grained square-lattice
dispersion on 8192 points, one chain, FP64 plain submatrix, K = 600 so that
the mean order is ~1000.  Inputs are synthetic and resident in HBM before the
timed region.

Prints one JSON line: vertex updates/s (proposals processed, accepted or not),
the rank-k TFLOP/s, the roofline of the dominant kernel (per-launch device
time from HIP events on the library's stream over the timed region), and the
CPU oracle timed on a bounded sample of the same workload.

Extra legs (--legs): "mixed" runs the same chain with FP32 storage and the FP32
MFMA rank-k update; "batched" runs 512 independent chains of mixed clusters
(Nc in {4, 8, 16, 32}, beta in [4, 12], U in [4, 8]) in FP64; "batched32" the
same with FP32 storage, which stops with an error when a chain's refinement
drift shows that FP32 cannot hold its N.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
FP32_PEAK_TFS = 157.3

METRIC = "vertex updates/s + rank-k TFLOP/s, mixed/batched vs plain FP64, same GPU"


def cfg2_workload():
    from ctaux_inputs import dca_square
    return dca_square(L=4, beta=8.0, U=8.0, K=600.0, density=0.9, n_tau=8192, t=1.0, n_fine=64)


def _opts(ctaux, precision, n_cap=2048, k=64):
    return ctaux.Options(k_max=k, k_cap=k, p_flip=0.2, recompute_every=64, precision=precision,
                         meas_every=k, n_therm=0, n_tau_out=16, n_cap=n_cap, seed=0)


STAT_KEYS = ("proposals", "accepted", "blocks", "sum_ka", "rankk_flops", "rankk_bytes", "sum_order",
             "prep_flops", "prep_bytes", "meas_flops", "meas_bytes")


def _delta(gb, s0, n_chains):
    s1 = [gb.stats(c) for c in range(n_chains)]
    d = {key: sum(s1[c][key] - s0[c][key] for c in range(n_chains)) for key in STAT_KEYS}
    return d, s1


def timed_run(gb, steps, k, n_chains=1, profile_blocks=40):
    """Per-kernel shares from a short run with HIP events around every kernel,
    then `steps` blocks with events around the dominant kernel only (each event
    pair adds device time), timed on the host between synchronisations."""
    import torch
    s0 = [gb.stats(c) for c in range(n_chains)]
    gb.set_timing(True)
    gb.run(profile_blocks * k)
    prof = gb.timing()
    dprof, _ = _delta(gb, s0, n_chains)
    # the kernel with the largest device time per block; the periodic
    # refinement does not run every block and is excluded
    dominant = max((n for n in prof if n != "refine"), key=lambda name: prof[name][0])
    # one launch in four carries the events: their device time stays out of the rest
    gb.set_timing(False, kernels=[dominant], every=4)
    s0 = [gb.stats(c) for c in range(n_chains)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gb.run(steps * k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = gb.timing()
    gb.set_timing(False)
    d, s1 = _delta(gb, s0, n_chains)
    d["seconds"] = t1 - t0
    d["dominant"] = dominant
    d["timing"] = timing
    d["profile"] = {"blocks": dprof["blocks"], "timing": prof, "stats": dprof}
    d["order_now"] = [s1[c]["order"] for c in range(n_chains)]
    d["max_drift"] = max(s1[c]["max_drift"] for c in range(n_chains))
    return d


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel's source has changed since the counters
    were taken (the summary records the source's SHA-256)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_bytes_per_launch.txt")
    src = {"propose": "k_propose.hip", "rankk": "k_update.hip"}.get(kernel)
    if src is None or not os.path.exists(path):
        return None
    with open(os.path.join(ROOT, "paper_1010_3690_amd", "csrc", src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    for line in open(path):
        parts = line.split()
        if len(parts) == 3 and not line.startswith("#") and parts[0] == kernel and parts[2] == sha:
            return float(parts[1])
    return None


def roofline(d, precision):
    """Roofline of the dominant kernel of the timed region: its algorithmic work
    per launch over its average launch duration (HIP events on the library's
    stream around each launch of that kernel)."""
    name = d["dominant"]
    ms, timed = d["timing"][name]
    if timed == 0 or ms <= 0.0:
        return {"kernel": name, "error": "no timed launch"}
    avg_s = ms / 1e3 / timed
    # one launch of each per-block kernel per block of the batch
    launches = d["blocks"] / d.get("n_chains", 1)
    prof = d["profile"]["timing"]
    out = {"kernel": name, "share": prof[name][0] / sum(v[0] for v in prof.values()),
           "launches": launches, "timed_launches": timed, "avg_launch_us": avg_s * 1e6}
    if name in ("rankk", "prep", "measure"):
        key = {"rankk": "rankk_bytes", "prep": "prep_bytes", "measure": "meas_bytes"}[name]
        achieved = d[key] / max(launches, 1) / avg_s / 1e9
        out.update({"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": None})
    else:
        # The proposal loop is one workgroup per chain running k dependent
        # proposals; its work per launch is the O(k_a^2) Gamma^{-1} arithmetic
        # (per proposal and sector two matrix-vector products with Gamma^{-1},
        # 4 k_a^2 flops, and for an accepted proposal the growth, 2 k_a^2),
        # reported against the FP64 vector peak of the compute units it
        # occupies (one per chain).
        ka = d["sum_ka"] / max(d["blocks"], 1)
        k = d["proposals"] / max(d["blocks"], 1)
        acc_frac = ka / max(k, 1)
        flops_launch = d["proposals"] / max(launches, 1) * 2 * (4 * ka * ka / 4 + acc_frac * 2 * ka * ka / 4)
        achieved = flops_launch / avg_s / 1e12
        n_chains = d.get("n_chains", 1)
        peak = FP64_PEAK_TFS * min(n_chains, 256) / 256.0
        out.update({"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                    "frac": achieved / peak, "traffic": measured_traffic(name) if n_chains == 1 else None})
    return out


def cpu_baseline(w, config, budget_s=15.0):
    """The oracle (rank-1 CT-AUX, one core) on a bounded sample of the workload:
    it starts from the GPU chain's thermalised configuration and runs
    proposals until about budget_s seconds have elapsed."""
    from oracle import OracleChain
    ids, tau, site, s = config
    oc = OracleChain(w, seed=12345, meas_every=64, n_tau_out=16, n_cap=4096)
    oc.set_config(ids, tau, site, s)
    oc.set_state(0, int(ids.max()) + 1 if len(ids) else 0, 1.0)
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        oc.run(16)
        done += 16
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "vertex updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} proposals of the same chain from a thermalised order-{len(ids)} "
                      f"configuration, {el:.1f} s on one host core"}


def leg_plain(args, precision):
    import torch
    from paper_1010_3690_amd import ctaux
    w = cfg2_workload()
    gb = ctaux.CtauxBatch([w], _opts(ctaux, precision))
    gb.run(args.warmup * 64)
    torch.cuda.synchronize()
    d = timed_run(gb, args.steps, 64)
    return w, gb, d


def leg_batched(args, precision):
    """512 chains; with --autotune the block length and rank-k tile come from
    paper_1010_3690_amd.autotune (trials continue the same thermalised chains)."""
    import torch
    from ctaux_inputs import batched_mix
    from paper_1010_3690_amd import ctaux
    ws = batched_mix(n_chains=args.batch_chains, seed=0, n_tau=2048, n_fine=16)
    opts = ctaux.Options(k_max=64, k_cap=64, recompute_every=64, precision=precision, meas_every=64,
                         n_tau_out=8, n_cap=2048, seed=0)
    tuning = None
    if args.autotune:
        from paper_1010_3690_amd.autotune import autotune
        print("[bench] autotuning the batched form", file=sys.stderr, flush=True)
        opts, tuning = autotune(ws, opts, warmup_proposals=args.batch_warmup * 64, trial_proposals=32 * 64)
        print(f"[bench] autotuned: k_max={opts.k_max} k_cap={opts.k_cap} rankk_tile={opts.rankk_tile}",
              file=sys.stderr, flush=True)
    gb = ctaux.CtauxBatch(ws, opts)
    gb.run(args.batch_warmup * 64)
    torch.cuda.synchronize()
    d = timed_run(gb, args.batch_steps, 64, n_chains=len(ws), profile_blocks=4)
    d["n_chains"] = len(ws)
    d["options"] = {"k_max": opts.k_max, "k_cap": opts.k_cap, "rankk_tile": opts.rankk_tile}
    d["tuning"] = tuning
    return d


def summary(d):
    prof = d["profile"]
    pb = max(prof["blocks"], 1)
    rk = prof["timing"].get("rankk")
    return {
        "updates_per_s": d["proposals"] / d["seconds"],
        "accepted_per_s": d["accepted"] / d["seconds"],
        # rank-k TFLOP/s of the update kernel alone (operand assembly reported in kernel_us)
        "rankk_tflops": (prof["stats"]["rankk_flops"] / (rk[0] / 1e3) / 1e12) if rk and rk[0] > 0 else None,
        "mean_order": d["sum_order"] / max(d["blocks"], 1),
        "mean_ka": d["sum_ka"] / max(d["blocks"], 1),
        "ms_per_block": d["seconds"] * 1e3 / max(d["blocks"], 1),
        "kernel_us_per_block": {k: round(v[0] * 1e3 / pb, 2) for k, v in prof["timing"].items()},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--legs", default="plain,mixed,batched",
                    help="comma list of plain (FP64, one chain), mixed (FP32 storage, one chain), "
                         "batched (FP64, many chains), batched32 (FP32 storage, many chains)")
    ap.add_argument("--batch-chains", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=64)
    ap.add_argument("--batch-warmup", type=int, default=60)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action=argparse.BooleanOptionalAction, default=True,
                    help="choose k and the rank-k tile of the batched legs with the autotuner")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run 10 device copies of 1 GiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: independent Markov chains shard across GPUs with no "
              "communication on the hot path, and this build measures one GPU's share.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(10):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 1 << 30, "launches": 10}))
        return
    from paper_1010_3690_amd import ctaux

    legs = [x.strip() for x in args.legs.split(",") if x.strip()]
    print(f"[bench] plain FP64 leg: warmup {args.warmup} blocks, timed {args.steps} blocks", file=sys.stderr,
          flush=True)
    w, gb, d = leg_plain(args, ctaux.CTAUX_FP64)
    s = summary(d)
    roof = roofline(d, ctaux.CTAUX_FP64)
    out = {
        "metric": METRIC,
        "value": s["updates_per_s"],
        "unit": "vertex updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": s["ms_per_block"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D Hubbard DCA 4x4 cluster (Nc=16), t=1, U=8, beta=8, <n>=0.9, "
                               "coarse-grained G0 on 8192 tau points, K=600, one chain, FP64 plain "
                               "submatrix, k=64, step = one block of 64 proposals",
                   "k": 64, "mean_order": s["mean_order"], "mean_accepted_per_block": s["mean_ka"]},
        "rankk_tflops": s["rankk_tflops"],
        "accepted_per_s": s["accepted_per_s"],
        "kernel_us_per_block": s["kernel_us_per_block"],
        "roofline": roof,
    }
    forms = {"plain_fp64": {k: s[k] for k in ("updates_per_s", "rankk_tflops", "mean_order", "mean_ka")}}
    forms["plain_fp64"]["max_refinement_drift"] = d["max_drift"]
    if "mixed" in legs:
        print("[bench] mixed leg: FP32 storage, same chain", file=sys.stderr, flush=True)
        _, gbm, dm = leg_plain(args, ctaux.CTAUX_FP32)
        sm = summary(dm)
        forms["mixed_fp32"] = {k: sm[k] for k in ("updates_per_s", "rankk_tflops", "mean_order", "mean_ka")}
        forms["mixed_fp32"]["max_refinement_drift"] = dm["max_drift"]
        forms["mixed_fp32"]["kernel_us_per_block"] = sm["kernel_us_per_block"]
        gbm.close()
    for leg, name, prec in (("batched", "batched_fp64", ctaux.CTAUX_FP64),
                            ("batched32", "batched_fp32", ctaux.CTAUX_FP32)):
        if leg not in legs:
            continue
        print(f"[bench] {name} leg: {args.batch_chains} chains", file=sys.stderr, flush=True)
        try:
            db = leg_batched(args, prec)
        except ctaux.CtauxError as e:   # FP32 storage cannot hold every chain of the mix
            forms[name] = {"error": str(e)}
            continue
        sb = summary(db)
        forms[name] = {k: sb[k] for k in ("updates_per_s", "rankk_tflops", "mean_order", "mean_ka")}
        forms[name]["n_chains"] = args.batch_chains
        forms[name]["max_refinement_drift"] = db["max_drift"]
        forms[name]["roofline"] = roofline(db, prec)
        forms[name]["kernel_us_per_block"] = sb["kernel_us_per_block"]
        forms[name]["options"] = db["options"]
        if db["tuning"]:
            forms[name]["autotune"] = [{k: (round(v, 1) if isinstance(v, float) else v) for k, v in r.items()}
                                       for r in db["tuning"]]
    out["forms"] = forms
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, gb.config(0), args.cpu_budget)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
