#!/usr/bin/env python
"""Throughput of the CT-AUX submatrix path on one MI355X.

Headline workload (step = one block: k_max = 64 proposals, the Gamma inner
loop, the rank-k update of N in both spin sectors, the measurement, and the
FP64 refinement of N on its schedule): 2D Hubbard DCA cluster 4x4 (Nc = 16),
t = 1, U = 8, beta = 8, <n> = 0.9, cluster G0(tau) from the coarse-grained
square-lattice dispersion on 8192 points, one chain, FP64 plain submatrix,
K = 600 so that the mean order is ~1000.  The chain is thermalised until its
mean order is stable (whatever --warmup asks for beyond that), then exactly
--steps blocks are timed.  Inputs are synthetic and resident in HBM before
the timed region.

Prints one JSON line: vertex updates/s (proposals processed, accepted or not),
the rank-k TFLOP/s, the roofline of the dominant kernel (per-launch device
time from HIP events on the library's stream over the timed region), the CPU
oracle timed on a bounded sample of the same workload, and further forms:
  mixed       the same chain with N in FP32 (FP32 MFMA rank-k update), at the
              default drift target and at an N error target of 1e-6, and with
              the split-BF16x3 rank-k update;
  cfg2x128    128 independent chains of the headline workload, FP64 and FP32
              storage (mixed/batched vs plain on one workload);
  batched     512 chains of mixed clusters (Nc in {4, 8, 16, 32}, beta in
              [4, 12], U in [4, 8], K = 1), FP64, k and tile autotuned, with the
              real-space G(tau) measurement and again measuring in cluster
              momenta and Matsubara frequencies;
  config3     6x6 cluster, beta = 10, order ~3000, FP32 storage (FP32 MFMA and
              split-BF16x3 rank-k) with FP64 refresh every <= 64 blocks, and the
              same in FP64;
  config5     3D Nc = 100 cluster, beta = 6, order ~5000, 8 chains, FP32
              storage with FP64 refresh every <= 32 blocks;
  graph       windows of 16 blocks replayed from a captured HIP graph against
              blocks launched one by one (headline chain; one-site chain);
  cpu         the host FP64 submatrix form on one core, on the oracle's
              sample, with and without the measurement, beside the oracle.
Each form reports its N error: the largest refinement drift of the run
(||N - N_refined|| / ||N_refined|| before each refinement) and the drift of a
refinement taken at the end of the timed region.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
FP32_PEAK_TFS = 157.3
N_CU = 256

METRIC = "vertex updates/s + rank-k TFLOP/s, mixed/batched vs plain FP64, same GPU"
ALL_LEGS = "plain,mixed,pairs,cfg2x128,batched,config3,config5,graph,cpu"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cfg2_workload():
    from ctaux_inputs import dca_square
    return dca_square(L=4, beta=8.0, U=8.0, K=600.0, density=0.9, n_tau=8192, t=1.0, n_fine=64)


def _opts(ctaux, precision, n_cap=2048, k=64, **kw):
    o = dict(k_max=k, k_cap=min(k, 64), p_flip=0.2, recompute_every=64, precision=precision,
             meas_every=k, n_therm=0, n_tau_out=16, n_cap=n_cap, seed=0)
    o.update(kw)
    return ctaux.Options(**o)


STAT_KEYS = ("proposals", "accepted", "blocks", "sum_ka", "rankk_flops", "rankk_bytes", "sum_order",
             "prep_flops", "prep_bytes", "meas_flops", "meas_bytes")


def _stats(gb, n_chains):
    return [gb.stats(c) for c in range(n_chains)]


def _delta(gb, s0, n_chains):
    s1 = _stats(gb, n_chains)
    d = {key: sum(s1[c][key] - s0[c][key] for c in range(n_chains)) for key in STAT_KEYS}
    return d, s1


def thermalise(gb, k, n_chains, min_blocks, chunk, tol=0.02, max_chunks=40):
    """Runs min_blocks blocks, then chunks of `chunk` blocks until the mean order
    over a chunk differs from the previous chunk's by less than tol (relative)."""
    gb.run(min_blocks * k)
    prev, total, mean = None, min_blocks, 0.0
    for _ in range(max_chunks):
        s0 = _stats(gb, n_chains)
        gb.run(chunk * k)
        total += chunk
        d, _ = _delta(gb, s0, n_chains)
        mean = d["sum_order"] / max(d["blocks"], 1)
        if prev is not None and abs(mean - prev) <= tol * prev:
            break
        prev = mean
    return {"blocks": total, "mean_order": mean}


def timed_run(gb, steps, k, n_chains=1, profile_blocks=40):
    """Per-kernel shares from a short run with HIP events around every kernel,
    then `steps` blocks with events around the dominant kernel only (each event
    pair adds device time), timed on the host between synchronisations."""
    import torch
    s0 = _stats(gb, n_chains)
    gb.set_timing(True)
    gb.run(profile_blocks * k)
    prof = gb.timing()
    dprof, _ = _delta(gb, s0, n_chains)
    # the kernel with the largest device time per block; the periodic
    # refinement does not run every block and is excluded
    dominant = max((n for n in prof if n != "refine"), key=lambda name: prof[name][0])
    # one launch in four carries the events: their device time stays out of the rest
    gb.set_timing(False, kernels=[dominant], every=4)
    s0 = _stats(gb, n_chains)
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
    d["n_chains"] = n_chains
    return d


def measured_traffic(kernel, n_chains):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary: the proposal loop and the rank-k update on the headline chain, the
    measurement kernels (gR, W, G, accumulation) on the 512-chain batch.  None
    when no entry exists for that case or the kernel's sources have changed since
    the counters were taken (the summary records their SHA-256)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_bytes_per_launch.txt")
    key, srcs = {("propose", 1): ("propose", ["k_propose.hip"]),
                 ("rankk", 1): ("rankk", ["k_update.hip"]),
                 ("measure", 512): ("measure_batched512", ["k_measure.hip", "k_skinny.hip"])}.get(
                     (kernel, n_chains), (None, None))
    if key is None or not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for src in srcs:
        with open(os.path.join(ROOT, "paper_1010_3690_amd", "csrc", src), "rb") as f:
            h.update(f.read())
    sha = h.hexdigest()
    for line in open(path):
        parts = line.split()
        if len(parts) == 3 and not line.startswith("#") and parts[0] == key and parts[2] == sha:
            return float(parts[1])
    return None


def roofline(d):
    """Roofline of the dominant kernel of the timed region: its algorithmic work
    per launch over its average launch duration (HIP events on the library's
    stream around each launch of that kernel), against the chip's published peak."""
    name = d["dominant"]
    ms, timed = d["timing"][name]
    if timed == 0 or ms <= 0.0:
        return {"kernel": name, "error": "no timed launch"}
    avg_s = ms / 1e3 / timed
    n_chains = d.get("n_chains", 1)
    launches = d["blocks"] / n_chains   # one launch of each per-block kernel serves every chain
    prof = d["profile"]["timing"]
    out = {"kernel": name, "share": prof[name][0] / sum(v[0] for v in prof.values()),
           "launches": launches, "timed_launches": timed, "avg_launch_us": avg_s * 1e6}
    if name in ("rankk", "prep", "measure"):
        key = {"rankk": "rankk_bytes", "prep": "prep_bytes", "measure": "meas_bytes"}[name]
        achieved = d[key] / max(launches, 1) / avg_s / 1e9
        out.update({"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(name, n_chains)})
    else:
        # The proposal loop is one workgroup per chain running k dependent
        # proposals; its work per launch is the O(k_a^2) Gamma^{-1} arithmetic
        # (per proposal and sector two matrix-vector products with Gamma^{-1},
        # 4 k_a^2 flops, and for an accepted proposal the growth, 2 k_a^2).  It is
        # latency-bound: the figure that matters is the time per proposal.
        ka = d["sum_ka"] / max(d["blocks"], 1)
        k = d["proposals"] / max(d["blocks"], 1)
        acc_frac = ka / max(k, 1)
        flops_launch = d["proposals"] / max(launches, 1) * 2 * (4 * ka * ka / 4 + acc_frac * 2 * ka * ka / 4)
        achieved = flops_launch / avg_s / 1e12
        per_chain_props = d["proposals"] / max(launches, 1) / n_chains
        cu_peak = FP64_PEAK_TFS * min(n_chains, N_CU) / N_CU
        out.update({"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                    "frac": achieved / FP64_PEAK_TFS, "traffic": measured_traffic(name, n_chains),
                    "frac_of_occupied_cus": achieved / cu_peak,
                    "us_per_proposal": avg_s * 1e6 / max(per_chain_props, 1e-9),
                    "proposals_per_s_per_chain": per_chain_props / avg_s})
    return out


def host_info():
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu": model, "nproc": avail, "cpu_count": os.cpu_count()}


def cpu_baseline(w, config, therm_blocks, budget_s=15.0):
    """The oracle (rank-1 CT-AUX, one core) on a bounded sample of the workload:
    it starts from the configuration the GPU chain reached after thermalisation
    and runs proposals until about budget_s seconds have elapsed, measuring
    every 64 proposals like the GPU chain; then a third as long with the
    measurement off (the update rate alone, compared with the host submatrix
    form)."""
    from oracle import OracleChain
    ids, tau, site, s = config

    def sample(meas_every, seconds):
        oc = OracleChain(w, seed=12345, meas_every=meas_every, n_tau_out=16, n_cap=4096)
        oc.set_config(ids, tau, site, s)
        oc.set_state(0, int(ids.max()) + 1 if len(ids) else 0, 1.0)
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            oc.run(16)
            done += 16
        return done, time.perf_counter() - t0

    done, el = sample(64, budget_s)
    done_nm, el_nm = sample(1 << 30, budget_s / 3)
    out = {"value": done / el, "unit": "vertex updates/s", "cores": 1, "kind": "oracle",
           "sample": f"{done} proposals of the headline chain from the order-{len(ids)} configuration the GPU "
                     f"chain reached after {therm_blocks} blocks of thermalisation, measuring every 64 proposals, "
                     f"{el:.1f} s on one host core (the oracle is single-threaded)",
           "no_measurement": {"value": done_nm / el_nm, "proposals": done_nm, "seconds": el_nm}}
    out.update({"host_" + k: v for k, v in host_info().items()})
    return out


def leg_graph(ctaux):
    """Blocks launched one by one against windows of 16 blocks replayed from a
    captured HIP graph: the headline chain (k = 64, order ~1000) and the
    one-site chain of a semicircular bath (beta = 10, U = 4, K = 1, order ~20,
    k = 16), whose kernels are short enough for launch costs to show."""
    import torch
    from ctaux_inputs import anderson_semicircle
    out = {}
    cases = (("headline_4x4", cfg2_workload(), 64, 300, 200),
             ("semicircle_nc1", anderson_semicircle(beta=10.0, U=4.0, K=1.0, n_tau=4096), 16, 4000, 2000))
    for name, w, k, steps, warm in cases:
        res = {}
        for g in (0, 16):
            gb = ctaux.CtauxBatch([w], _opts(ctaux, ctaux.CTAUX_FP64, k=k))
            gb.set_graph(g)
            gb.run(warm * k)
            torch.cuda.synchronize()
            best = None
            for _ in range(3):
                s0 = gb.stats(0)
                t0 = time.perf_counter()
                gb.run(steps * k)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                s1 = gb.stats(0)
                rate = (s1["proposals"] - s0["proposals"]) / el
                best = rate if best is None else max(best, rate)
            res[f"graph_{g}"] = {"updates_per_s": best, "us_per_block": k / best * 1e6,
                                 "mean_order_end": gb.stats(0)["order"], "graph_launches": gb.graph_launches}
            gb.close()
        res["speedup"] = res["graph_16"]["updates_per_s"] / res["graph_0"]["updates_per_s"]
        out[name] = res
    return out


def leg_cpu_submatrix(w, config, oracle, budget_s=10.0):
    """The host FP64 submatrix form (one core, k = 64, AVX2 register tiles) on the
    oracle's sample: the same starting configuration, measuring every 64
    proposals, then with the measurement off, Gamma grown by partitioning and
    then as LU factors; each rate beside the oracle's under the same settings
    (the paper compares the two update rates on one core)."""
    from paper_1010_3690_amd import ctaux
    from paper_1010_3690_amd.cpu import CpuChain
    ids, tau, site, s = config
    out = {"cores": 1, "k": 64, "host_cpu": host_info()["cpu"]}
    for name, meas, growth in (("measuring", 64, 0), ("no_measurement", 1 << 30, 0),
                               ("no_measurement_lu_growth", 1 << 30, 1)):
        ch = CpuChain(w, ctaux.Options(k_max=64, k_cap=64, p_flip=0.2, meas_every=meas, n_tau_out=16,
                                       n_cap=4096, seed=12345))
        ch.set_growth(growth)
        ch.set_config(ids, tau, site, s)
        ch.run(64 * 4)   # first blocks: buffers sized
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s / 2:
            ch.run(64 * 4)
            done += 64 * 4
        el = time.perf_counter() - t0
        rate = done / el
        ref = oracle["value"] if name == "measuring" else oracle["no_measurement"]["value"]
        out[name] = {"updates_per_s": rate, "proposals": done, "seconds": el, "mean_order_end": ch.state()["order"],
                     "oracle_updates_per_s": ref, "vs_oracle": rate / ref}
    return out


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
        "ms_per_block": d["seconds"] * 1e3 / max(d["blocks"] / d.get("n_chains", 1), 1),
        "kernel_us_per_block": {k: round(v[0] * 1e3 / max(pb / d.get("n_chains", 1), 1), 2)
                                for k, v in prof["timing"].items()},
    }


def form(gb, d, therm, extra=None):
    """Summary of a timed form plus its N error: the largest refinement drift of
    the run and the drift of one refinement at the end."""
    s = summary(d)
    out = {k: s[k] for k in ("updates_per_s", "accepted_per_s", "rankk_tflops", "mean_order", "mean_ka",
                             "ms_per_block", "kernel_us_per_block")}
    out["n_chains"] = d.get("n_chains", 1)
    out["thermalisation_blocks"] = therm["blocks"]
    out["max_refinement_drift"] = d["max_drift"]
    out["n_error_at_end"] = gb.recompute()
    out["roofline"] = roofline(d)
    if extra:
        out.update(extra)
    return out


def single_chain(ctaux, w, precision, steps, warmup, k=64, n_cap=2048, chunk=50, **kw):
    gb = ctaux.CtauxBatch([w], _opts(ctaux, precision, n_cap=n_cap, k=k, **kw))
    therm = thermalise(gb, k, 1, max(warmup, 100), chunk)
    d = timed_run(gb, steps, k)
    return gb, d, therm


def many_chains(ctaux, ws, opts, steps, min_blocks, chunk, profile_blocks=4):
    gb = ctaux.CtauxBatch(ws, opts)
    therm = thermalise(gb, opts.k_max, len(ws), min_blocks, chunk)
    d = timed_run(gb, steps, opts.k_max, n_chains=len(ws), profile_blocks=profile_blocks)
    return gb, d, therm


def leg_batched(ctaux, args):
    """512 chains of the config-4 mix in FP64; k and the rank-k tile from the
    autotuner (its trials continue the same thermalised chains)."""
    from ctaux_inputs import batched_mix
    ws = batched_mix(n_chains=args.batch_chains, seed=0, n_tau=2048, n_fine=16)
    opts = ctaux.Options(k_max=64, k_cap=64, recompute_every=64, precision=ctaux.CTAUX_FP64, meas_every=64,
                         n_tau_out=8, n_cap=2048, seed=0)
    tuning = None
    if args.autotune:
        from paper_1010_3690_amd.autotune import autotune
        log("autotuning the batched form")
        opts, tuning = autotune(ws, opts, warmup_proposals=60 * 64, trial_proposals=32 * 64)
        log(f"autotuned: k_max={opts.k_max} k_cap={opts.k_cap} rankk_tile={opts.rankk_tile}")
    gb, d, therm = many_chains(ctaux, ws, opts, args.batch_steps, 60, 20)
    extra = {"options": {"k_max": opts.k_max, "k_cap": opts.k_cap, "rankk_tile": opts.rankk_tile}}
    if tuning:
        extra["autotune"] = [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()} for r in tuning]
    out = form(gb, d, therm, extra)
    gb.close()
    return out


def leg_batched_kw(ctaux, args, opts_like):
    """The same 512 chains measuring G in cluster momenta and 8 Matsubara
    frequencies instead of the real-space G(tau) bins (densities and double
    occupancy still from the equal-time G)."""
    from dataclasses import replace
    from ctaux_inputs import batched_mix
    ws = batched_mix(n_chains=args.batch_chains, seed=0, n_tau=2048, n_fine=16)
    opts = replace(opts_like, n_tau_out=0, n_matsubara=8)
    gb, d, therm = many_chains(ctaux, ws, opts, args.batch_steps, 60, 20)
    out = form(gb, d, therm, {"options": {"k_max": opts.k_max, "k_cap": opts.k_cap, "rankk_tile": opts.rankk_tile,
                                          "n_tau_out": 0, "n_matsubara": 8}})
    gb.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400, help="timed blocks of the headline chain")
    ap.add_argument("--warmup", type=int, default=200,
                    help="least blocks before timing; thermalisation continues until the mean order is stable")
    ap.add_argument("--legs", default=ALL_LEGS, help=f"comma list of extra forms: {ALL_LEGS}")
    ap.add_argument("--batch-chains", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=32)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action=argparse.BooleanOptionalAction, default=True,
                    help="choose k and the rank-k tile of the batched leg with the autotuner")
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
    log(f"plain FP64 leg: thermalise (>= {max(args.warmup, 100)} blocks), time {args.steps} blocks")
    w = cfg2_workload()
    gb, d, therm = single_chain(ctaux, w, ctaux.CTAUX_FP64, args.steps, args.warmup)
    s = summary(d)
    roof = roofline(d)
    plain = form(gb, d, therm)
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
                   "k": 64, "mean_order": s["mean_order"], "mean_accepted_per_block": s["mean_ka"],
                   "thermalisation_blocks": therm["blocks"]},
        "rankk_tflops": s["rankk_tflops"],
        "accepted_per_s": s["accepted_per_s"],
        "kernel_us_per_block": s["kernel_us_per_block"],
        "roofline": roof,
    }
    forms = {"plain_fp64": plain}
    config0 = gb.config(0)
    gb.close()

    def leg(name, fn):
        """Runs one extra form; a form that fails is recorded with its error and
        the run goes on (the headline above is measured already)."""
        try:
            fn()
        except Exception as e:   # noqa: BLE001 - any failure of an extra form is reported, not fatal
            log(f"{name} failed: {e}")
            forms[name] = {"error": str(e)}
            import gc
            gc.collect()
            torch.cuda.empty_cache()

    # Mixed forms (FP32 storage) run with drift_tol = 1: a chain whose N drifted past
    # the Newton step's basin is recomputed from scratch rather than stopped, and the
    # largest drift of the run is reported.
    mixed_tol = 1.0

    def mixed():
        log("mixed leg: FP32 storage, same chain (default drift target, then 1e-6)")
        g2, d2, t2 = single_chain(ctaux, w, ctaux.CTAUX_FP32, args.steps, args.warmup, drift_tol=mixed_tol)
        forms["mixed_fp32"] = form(g2, d2, t2)
        g2.close()
        g2, d2, t2 = single_chain(ctaux, w, ctaux.CTAUX_FP32, args.steps, args.warmup, drift_target=1e-6,
                                  drift_tol=mixed_tol)
        forms["mixed_fp32_target_1e-6"] = form(g2, d2, t2, {"drift_target": 1e-6})
        g2.close()
        g2, d2, t2 = single_chain(ctaux, w, ctaux.CTAUX_BF16X3, args.steps, args.warmup, drift_tol=mixed_tol)
        forms["mixed_bf16x3"] = form(g2, d2, t2)
        g2.close()

    def pairs():
        log("pairs_fp64 leg: the same workload with pair insertions and removals (p_pair = 0.2)")
        g2, d2, t2 = single_chain(ctaux, w, ctaux.CTAUX_FP64, args.steps, args.warmup, p_pair=0.2)
        forms["pairs_fp64"] = form(g2, d2, t2, {"p_pair": 0.2, "p_flip": 0.2})
        g2.close()

    def cfg2x128(name, prec):
        def run():
            log(f"{name}: 128 chains of the headline workload")
            opts = _opts(ctaux, prec, drift_tol=mixed_tol if prec != ctaux.CTAUX_FP64 else 1e-2)
            g2, d2, t2 = many_chains(ctaux, [w] * 128, opts, 32, 150, 20)
            forms[name] = form(g2, d2, t2)
            g2.close()
        return run

    def batched():
        log(f"batched_fp64 leg: {args.batch_chains} chains")
        forms["batched_fp64"] = leg_batched(ctaux, args)
        o = forms["batched_fp64"]["options"]
        log("batched_fp64_kw: the same chains measuring in cluster momenta / Matsubara frequencies")
        forms["batched_fp64_kw"] = leg_batched_kw(
            ctaux, args, ctaux.Options(k_max=o["k_max"], k_cap=o["k_cap"], rankk_tile=o["rankk_tile"],
                                       recompute_every=64, meas_every=64, n_tau_out=8, n_cap=2048, seed=0))

    def config3(name, prec):
        def run():
            from ctaux_inputs import dca_square
            w3 = dca_square(L=6, beta=10.0, U=8.0, K=1800.0, density=0.9, n_tau=8192)
            log(f"{name}: 6x6 cluster, order ~3000")
            g3, d3, t3 = single_chain(ctaux, w3, prec, 100, 200, k=128, n_cap=4096, chunk=40, n_tau_out=8,
                                      drift_tol=mixed_tol if prec != ctaux.CTAUX_FP64 else 1e-2)
            forms[name] = form(g3, d3, t3)
            g3.close()
        return run

    def graph():
        log("graph: block windows replayed from a HIP graph vs launched one by one")
        forms["graph_windows"] = leg_graph(ctaux)

    def config5():
        from ctaux_inputs import dca_cubic
        w5 = dca_cubic(beta=6.0, U=8.0, K=4300.0, n_tau=8192)
        log("config5_fp32: 3D Nc = 100, 8 chains, order ~5000-6000")
        opts = _opts(ctaux, ctaux.CTAUX_FP32, n_cap=8192, k=128, recompute_every=32, n_tau_out=8,
                     drift_tol=mixed_tol)
        g5, d5, t5 = many_chains(ctaux, [w5] * 8, opts, 16, 200, 20)
        forms["config5_fp32"] = form(g5, d5, t5)
        g5.close()

    if "mixed" in legs:
        leg("mixed_fp32", mixed)
    if "pairs" in legs:
        leg("pairs_fp64", pairs)
    if "cfg2x128" in legs:
        leg("cfg2x128_fp64", cfg2x128("cfg2x128_fp64", ctaux.CTAUX_FP64))
        leg("cfg2x128_fp32", cfg2x128("cfg2x128_fp32", ctaux.CTAUX_FP32))
    if "batched" in legs:
        leg("batched_fp64", batched)
    if "config3" in legs:
        for name, prec in (("config3_fp32", ctaux.CTAUX_FP32), ("config3_bf16x3", ctaux.CTAUX_BF16X3),
                           ("config3_fp64", ctaux.CTAUX_FP64)):
            leg(name, config3(name, prec))
    if "graph" in legs:
        leg("graph_windows", graph)
    if "config5" in legs:
        leg("config5_fp32", config5)
    out["forms"] = forms
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(w, config0, therm["blocks"], args.cpu_budget)
        if "cpu" in legs:
            def cpu_leg():
                log("cpu_submatrix_fp64: host submatrix form on the oracle's sample")
                forms["cpu_submatrix_fp64"] = leg_cpu_submatrix(w, config0, out["cpu_baseline"])
            leg("cpu_submatrix_fp64", cpu_leg)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
