"""Benchmark of the TDA-risp hot path on one MI355X.

Default workload: the 1000-atom chain-and-ring molecule (600 C + 400 H; nao 7400, nocc 1500,
nvir 5900, 2400 Coulomb and 600 exchange auxiliary functions, 40 eV window). A step is one sigma
block of 30 trial vectors (risp_sigma: diagonal, Coulomb and windowed exchange, BF16 MFMA products
with FP32 accumulation and per-slice power-of-two scales) on the BF16 factors, which are built once
before the timed steps; `value` is its sigma-build throughput (algorithmic flops of the block / its
time) and `ms_per_step` its time. Beside the steps, each path runs once end to end from the inputs
to 15 converged states (factor build + Davidson, with the FP32 correction pass on the BF16 path):
`time_to_15_states_s` for BF16 and plain FP32, with the phase breakdown, and one FP32 sigma block.
The FP32 measurements run first, in a child process; the CPU oracle baseline follows, then the BF16
measurements in this process: device memory freed by one run is cleared by the driver in the
background, and an allocation that arrives before that is done waits for it inside the timed build.

Prints one JSON line. Inputs are generated on the host before any timed region; the factor build
takes the MO coefficients from host memory (their PCIe copy is inside the time-to-15-states).
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"bf16": 2516.6, "fp32": 157.3, "fp64": 78.6}  # dense MFMA TFLOP/s (MI355X datasheet)
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chainring1000")
    ap.add_argument("--m", type=int, default=30, help="trial vectors per timed sigma block")
    ap.add_argument("--no-t2s", action="store_true", help="skip the end-to-end time-to-15-states runs")
    ap.add_argument("--nstates", type=int, default=15)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--no-fp32", action="store_true", help="skip the plain FP32 comparison steps")
    ap.add_argument("--no-bf16", action="store_true", help="time only the plain FP32 path (long workloads)")
    ap.add_argument("--verbose", action="store_true", help="one stderr line per Davidson iteration")
    ap.add_argument("--olsen", action="store_true", help="Olsen's correction vectors in the Davidson solves")
    ap.add_argument("--part", choices=["bf16", "fp32"], default=None,
                    help=argparse.SUPPRESS)  # internal: one precision's measurements in a child process
    ap.add_argument("--bf16-coulomb-fp32", action="store_true",
                    help="BF16 path: Coulomb term of every sigma from the FP32 copy of T_ia")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ao", action="store_true", help="also time one AO-density Coulomb route sigma block")
    ap.add_argument("--cpu-sample-aux", type=int, default=0,
                    help="exchange auxiliary slices in the CPU sample (0: sized for about 15 s on 16 cores)")
    ap.add_argument("--no-serving", action="store_true", help="skip the 64-job serving stream (the default)")
    ap.add_argument("--serving", action="store_true",
                    help="also run the 64-job serving stream (off by default: its run ended in a host "
                         "segmentation fault after the thick-restart change, cause not found yet)")
    ap.add_argument("--serving-jobs", type=int, default=64)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (the reference kernel for scaling "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def cpu_baseline(mol, nsample_k=0, m=30, gpu_flops=None, target_flops=1.5e13):
    """The FP64 oracle's sigma product on a bounded sample of the same workload.

    The sample keeps the full orbital dimensions (nocc, nvir, window) and m trial vectors and takes
    the first nsample_k exchange and 4 * nsample_k Coulomb auxiliary slices (random factor values:
    the oracle's cost does not depend on them); nsample_k = 0 sizes it for target_flops (about 15 s
    on 16 host cores). Reported as sigma-build TFLOP/s in the same flop convention as the GPU value,
    with the oracle's full sigma block extrapolated from it.
    """
    import numpy as np
    from oracle import risp as R
    rng = np.random.default_rng(7)
    nocc, nvir = mol.nocc, mol.nvir
    occK, virK = R.window_sets(mol.mo_energy, nocc, 40.0)
    ov, nok, nvk = nocc * nvir, len(occK), len(virK)
    per_k = 4.0 * ov * 4 * m + 2.0 * nok * nvk * m * (nok + nvk)  # one exchange + four Coulomb slices
    if nsample_k <= 0:
        nsample_k = int(max(1, min(600, target_flops // per_k)))
    nj = 4 * nsample_k
    F = R.Factors(nocc=nocc, nvir=nvir, de=(mol.mo_energy[None, nocc:] - mol.mo_energy[:nocc, None]),
                  B_ia=rng.standard_normal((nj, nocc, nvir)) * 1e-2,
                  Bx_ij=rng.standard_normal((nsample_k, nok, nok)) * 1e-2,
                  Bx_ab=rng.standard_normal((nsample_k, nvk, nvk)) * 1e-2, occK=occK, virK=virK)
    X = rng.standard_normal((m, nocc, nvir))
    t0 = time.perf_counter()
    R.sigma(F, X)
    dt = time.perf_counter() - t0
    flops = 4.0 * ov * nj * m + 2.0 * nsample_k * nok * nvk * m * (nok + nvk) + ov * m
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    out = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
           "sample": f"one FP64 sigma block (m={m}) with {nsample_k} of the exchange and {nj} of the Coulomb "
                     f"auxiliary slices at full nocc/nvir/window, {dt:.1f} s",
           "seconds": dt, "flops": flops}
    if gpu_flops:
        out["full_sigma_block_s_extrapolated"] = gpu_flops / (flops / dt)
    return out


def _gen_k(item):
    k, (n, seed) = item
    sys.path.insert(0, ROOT)
    import synth
    return k, synth.make_chain_ring(int(n), int(seed))


def serving_jobs(n_jobs=64, seed=2603, mean_gap=0.5, workers=8):
    """The serving stream: sizes U{50..400} atoms (C:H = 3:2), nstates U{5..15}, FP32/BF16 half and
    half in a seeded order, exponential inter-arrival gaps (Poisson arrivals); job k's molecule uses
    seed 2603 * 1000 + k."""
    import multiprocessing as mp

    import numpy as np
    rng = np.random.default_rng(seed)
    sizes = rng.integers(50, 401, n_jobs)
    nstates = rng.integers(5, 16, n_jobs)
    prec = rng.permutation(np.arange(n_jobs) % 2)
    gaps = rng.exponential(mean_gap, n_jobs)
    arrivals = np.cumsum(gaps) - gaps[0]
    # fresh worker interpreters (forking a process whose BLAS threads are running can deadlock),
    # two BLAS threads each
    saved = os.environ.get("OPENBLAS_NUM_THREADS")
    os.environ["OPENBLAS_NUM_THREADS"] = "2"
    mols = [None] * n_jobs
    try:
        with mp.get_context("spawn").Pool(workers) as pool:
            args = [(int(n), seed * 1000 + k) for k, n in enumerate(sizes)]
            for done, (k, m) in enumerate(pool.imap_unordered(_gen_k, list(enumerate(args)))):
                mols[k] = m
                if done % 8 == 7:
                    print(f"# serving molecules {done + 1}/{n_jobs}", file=sys.stderr, flush=True)
    finally:
        if saved is None:
            os.environ.pop("OPENBLAS_NUM_THREADS", None)
        else:
            os.environ["OPENBLAS_NUM_THREADS"] = saved
    return [dict(mol=m, nstates=int(ns), prec=("fp32", "bf16")[int(p)], arrival=float(a))
            for m, ns, p, a in zip(mols, nstates, prec, arrivals)]


def serving_bench(jobs, tol=1e-5, max_active=8):
    """Submit the jobs at their arrival times, poll until all are done; latency = done - submit."""
    import numpy as np

    import paper_2603_29257_amd as P
    ctx = P.Context(0)
    ctx.serve_config(0, max_active=max_active, use_graphs=True)
    systems = [P.System(j["mol"]) for j in jobs]
    ids, pending = [], {}
    t0 = time.perf_counter()
    k = 0
    results = {}
    while len(results) < len(jobs):
        now = time.perf_counter() - t0
        while k < len(jobs) and jobs[k]["arrival"] <= now:
            jid = ctx.submit(systems[k], P.Params(precision=P.PRECISIONS[jobs[k]["prec"]]), jobs[k]["nstates"], tol=tol)
            ids.append(jid)
            pending[jid] = k
            k += 1
        for jid in list(pending):
            r = ctx.poll(jid, jobs[pending[jid]]["nstates"])
            if r is not None:
                results[pending.pop(jid)] = r
                if len(results) % 8 == 0:
                    print(f"# serving {len(results)}/{len(jobs)} done at {time.perf_counter() - t0:.1f} s",
                          file=sys.stderr, flush=True)
        time.sleep(0.005)
    stats = ctx.serve_stats()
    ctx.close()
    lat = np.array([results[i]["t_done"] - results[i]["t_submit"] for i in range(len(jobs))])
    makespan = max(r["t_done"] for r in results.values()) - min(r["t_submit"] for r in results.values())
    ok = all(r["status"] == 0 for r in results.values())
    return {"jobs": len(jobs), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "makespan_s": float(makespan), "jobs_per_hour": len(jobs) / makespan * 3600,
            "all_converged": ok, "graph_ticks": stats["graph_ticks"], "ticks": stats["ticks"],
            "max_active": max_active, "mean_gap_s": 0.5}


def sigma_block_flops(d, m):
    """Algorithmic flops of one sigma block of m vectors (stored-factor Coulomb route): diagonal
    ov*m, Coulomb 4*ov*naux_J*m (two passes over T_ia), exchange 2*nK*noK*nvK*m*(noK + nvK)."""
    ov = d.nocc * d.nvir
    return (ov * m + 4.0 * ov * d.naux_j * m +
            2.0 * d.naux_k * d.nocc_k * d.nvir_k * m * (d.nocc_k + d.nvir_k))


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"exchange_m_{workload}_traffic.json")


def _source_digest():
    """Digest of the exchange kernel's sources (its file and the tile header it includes)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("gemm_bf16.hip", "gemm_tile.hpp"):
        with open(os.path.join(ROOT, "paper_2603_29257_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload, m):
    """HBM bytes per launch of the exchange kernel from the committed counter runs for this workload
    and block size, or None when there are none or the kernel source changed since they were taken."""
    path = traffic_file(workload)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256_16") != _source_digest() or rec.get("m", m) != m:
        return None
    return rec.get("bytes_per_launch")


def copy_calibration(mib):
    import torch
    n = (mib << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "launches": 5}))


def ao_route_block(ctx, P, sysc, torch, m=30):
    """One sigma block of m vectors with the AO-density Coulomb route (no stored T_ia; (mu nu|P)
    regenerated twice per block; BF16 exchange), against the stored-factor route on the same input."""
    out = {}
    for name, jm in (("ao", P.J_AO_DIRECT), ("mo", P.J_MO)):
        F = ctx.build_factors(sysc, P.Params(precision=P.BF16, j_mode=jm))
        d = F.desc
        X = torch.randn(m, d.nocc, d.nvir, device=ctx.device, dtype=torch.float32)
        ctx.sigma(F, X)
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.sigma(F, X)
        torch.cuda.synchronize()
        out[name] = {"sigma_block_s": time.perf_counter() - t, "factor_bytes": d.bytes}
        F.free()
    ov, nao = d.nocc * d.nvir, d.nao
    # the D and back-transform products, both integral contractions and the metric (FP64)
    out["ao_coulomb_flops"] = 4.0 * m * (ov * nao + d.nocc * nao * nao + d.naux_j * nao * nao + d.naux_j ** 2)
    out["m"] = m
    return out


def sigma_rows_check(ctx, F, P, torch, workload, m):
    """Max error of this GPU's sigma at the oracle's sampled rows (tests/golden/<workload>_sigma_rows.json,
    written by the FP64 oracle alone), relative to the largest sampled element; None without the file."""
    import numpy as np

    import synth
    gold = os.path.join(ROOT, "tests", "golden", f"{workload}_sigma_rows.json")
    if not os.path.exists(gold):
        return None
    g = json.load(open(gold))
    d = F.desc
    X = torch.tensor(synth.random_trial_vectors(len(g["sigma"]), d.nocc, d.nvir, g["seed"]), dtype=torch.float32,
                     device=ctx.device)
    S = ctx.sigma(F, X).reshape(X.shape[0], -1)[:, torch.tensor(g["rows"], device=ctx.device)].cpu().numpy()
    want = np.array(g["sigma"])
    return float(np.abs(S - want).max() / np.abs(want).max())


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; multi-GPU sharding over the "
                                   "auxiliary index is a design note, not an implemented path", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2603_29257_amd as P
    import synth

    def log(msg):
        print(f"# {msg}", file=sys.stderr, flush=True)

    t_gen = time.perf_counter()
    mol = synth.config_system(args.workload)
    jobs = serving_jobs(args.serving_jobs) if (args.serving and not args.no_serving and not args.part) else None
    t_gen = time.perf_counter() - t_gen
    log(f"{args.workload}: nao {mol.nao}, nocc {mol.nocc}, nvir {mol.nvir}; generated in {t_gen:.1f} s")
    precs = ([] if args.no_bf16 else ["bf16"]) + ([] if args.no_fp32 else ["fp32"])
    if args.part:
        precs = [args.part]
    if not precs:
        sys.exit("nothing to time: --no-bf16 and --no-fp32 together")
    mp_ = precs[0]  # the path the value and the roofline describe
    # Device memory that a finished run freed is cleared by the driver in the background before it
    # can be handed out again; an allocation that comes first waits for it (seconds at this size,
    # inside the time-to-15-states). So the other precisions run first, each in a child process, and
    # this process then does its CPU work (the oracle baseline) before it touches the GPU: each path
    # starts on cleared memory.
    child = {}
    if not args.part and not args.no_t2s:
        for prec in precs[1:]:
            cmd = [sys.executable, os.path.abspath(__file__), "--part", prec, "--workload", args.workload,
                   "--m", str(args.m), "--nstates", str(args.nstates), "--tol", str(args.tol)]
            cmd += [f for f, on in (("--olsen", args.olsen), ("--bf16-coulomb-fp32", args.bf16_coulomb_fp32),
                                    ("--verbose", args.verbose)) if on]
            r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True)
            if r.returncode != 0:
                sys.exit(f"{prec} measurements failed in their child process (exit status {r.returncode})")
            child[prec] = json.loads(r.stdout.strip().splitlines()[-1])
    t_child_end = time.perf_counter()
    cpu_base = None
    if child and not args.no_cpu_baseline:
        flops_block = next(iter(child.values()))["flops"]  # the same workload in every precision
        cpu_base = cpu_baseline(mol, args.cpu_sample_aux, m=args.m, gpu_flops=flops_block)
    if child:
        # give the driver time to clear the memory the child process used (untimed)
        time.sleep(max(0.0, 12.0 - (time.perf_counter() - t_child_end)))
    ctx = P.Context(0)
    sysc = P.System(mol)
    m = args.m

    def params(prec):
        return P.Params(precision=P.PRECISIONS[prec], bf16_coulomb_fp32=args.bf16_coulomb_fp32)

    def t2s(prec):
        """Inputs on the host -> factors -> Davidson to nstates converged states; the factors stay."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = ctx.build_factors(sysc, params(prec))
        e, _, info = ctx.davidson(F, args.nstates, tol=args.tol, want_vectors=False, allow_notconv=True,
                                  verbose=args.verbose, olsen=args.olsen)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        log(f"{prec} time-to-{args.nstates}-states {dt:.2f} s (build {info.t_build:.2f} s, "
            f"{info.iters}+{info.correction_iters} iterations, converged={info.converged})")
        return F, dict(t2s=dt, energies=[float(x) for x in e], iters=info.iters,
                       correction_iters=info.correction_iters, converged=bool(info.converged),
                       resid_hist=[float(x) for x in info.resid_hist],
                       breakdown={"build": info.t_build, "sigma": info.t_sigma, "subspace": info.t_subspace,
                                  "correction": info.t_correct},
                       sigma_tflops=info.sigma_flops / info.t_sigma / 1e12 if info.t_sigma > 0 else None,
                       sigma_tflops_correction=(info.sigma_flops_correct / info.t_sigma_correct / 1e12
                                                if info.t_sigma_correct > 0 else None))

    def sigma_blocks(F, n, warm):
        """n timed sigma blocks of m vectors (after `warm` untimed ones); returns seconds per block."""
        d = F.desc
        X = torch.tensor(synth.random_trial_vectors(m, d.nocc, d.nvir, 2603), dtype=torch.float32,
                         device=ctx.device)
        out = torch.empty_like(X)
        for _ in range(warm):
            ctx.sigma(F, X, out=out)
        torch.cuda.synchronize()
        times = []
        for k in range(n):
            t0 = time.perf_counter()
            ctx.sigma(F, X, out=out)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        return times

    res, t2s_res = {}, {}
    for prec, c in child.items():
        t2s_res[prec] = c["t2s"]
        res[prec] = dict(times=c["times"], flops=c["flops"], prof=None, desc=None, sigma_rows_err=c["sigma_rows_err"])
    for prec in precs:
        if prec in child:
            continue
        if args.no_t2s:
            F = ctx.build_factors(sysc, params(prec))
        else:
            F, t2s_res[prec] = t2s(prec)
        d = F.desc
        flops = sigma_block_flops(F.desc, m)
        if prec == mp_ and not args.part:
            for k in range(args.warmup):
                sigma_blocks(F, 1, 0)
                log(f"warmup {k}")
            ctx.profile(True, True)
            times = []
            for k in range(args.steps):
                times += sigma_blocks(F, 1, 0)
                log(f"{prec} step {k}: {times[-1] * 1e3:.1f} ms, {flops / times[-1] / 1e12:.0f} TFLOP/s")
            prof = ctx.profile(False, True)
        else:
            times = sigma_blocks(F, 1, 1)
            prof = None
            log(f"{prec} sigma block: {times[-1] * 1e3:.1f} ms, {flops / times[-1] / 1e12:.0f} TFLOP/s")
        res[prec] = dict(times=times, flops=flops, prof=prof, desc=d,
                         sigma_rows_err=sigma_rows_check(ctx, F, P, torch, args.workload, m))
        F.free()
    if args.part:
        r = res[args.part]
        print(json.dumps({"t2s": t2s_res[args.part], "times": r["times"], "flops": r["flops"],
                          "sigma_rows_err": r["sigma_rows_err"]}))
        ctx.close()
        return

    b = res[mp_]
    t_step = float(np.mean(b["times"]))
    # dominant kernel of the step: the exchange product M = T_ab X (one launch per auxiliary chunk)
    ph = b["prof"][mp_]["exchange_m"]
    per_launch_ms = ph["ms"] / max(ph["launches"], 1)
    per_launch_flops = ph["flops"] / max(ph["launches"], 1)
    achieved = per_launch_flops / (per_launch_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma",
                "kernel": ("exchange M^P = T_ab^P X (BF16 MFMA, FP32 accumulate)" if mp_ == "bf16"
                           else "exchange M^P = T_ab^P X (FP32 MFMA)"),
                "achieved": achieved, "peak": PEAK[mp_], "unit": "TFLOP/s", "frac": achieved / PEAK[mp_],
                "traffic": recorded_traffic(args.workload, m) if mp_ == "bf16" else None,
                "launches": ph["launches"], "avg_launch_ms": per_launch_ms, "flops_per_launch": per_launch_flops}

    def phase_table(pr):
        return {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                    "tflops": (v["flops"] / (v["ms"] * 1e-3) / 1e12) if v["ms"] > 0 else 0.0,
                    "gbs": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else 0.0}
                for k, v in pr.items() if v["launches"] > 0}
    d = b["desc"]
    nsh = len(mol.shells)
    out = {
        "metric": "time-to-15-states & sigma-build TFLOP/s, BF16 vs plain FP32; p50/p99 latency",
        "value": b["flops"] / t_step / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_step * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": mp_, "data": "synthetic",
        "config": {"workload": args.workload, "atoms": int(mol.natm), "nao": d.nao, "nocc": d.nocc, "nvir": d.nvir,
                   "naux_j": d.naux_j, "naux_k": d.naux_k, "nocc_k": d.nocc_k, "nvir_k": d.nvir_k,
                   "npair": d.npair, "shell_pairs": nsh * (nsh + 1) // 2,
                   "pair_survival_pct": 100.0 * d.npair / (nsh * (nsh + 1) // 2),
                   "cond_S": float(mol.cond_S), "step": f"one sigma block of {m} trial vectors on prebuilt factors",
                   "m": m, "nstates": args.nstates, "tol": args.tol, "window_ev": 40.0, "c_x": 0.22, "beta": 0.78,
                   "omega": 0.2},
        "sigma_block_s": {p: float(np.mean(res[p]["times"])) for p in res},
        "sigma_tflops": {p: res[p]["flops"] / float(np.mean(res[p]["times"])) / 1e12 for p in res},
        "sigma_block_flops": b["flops"],
        "sigma_rows_vs_oracle_rel_err": {p: res[p]["sigma_rows_err"] for p in res},
        f"phases_{mp_}": phase_table(b["prof"][mp_]),
        "roofline": roofline,
        "latency": None if jobs is None else serving_bench(jobs, tol=args.tol),
        "generator_s": t_gen,
    }
    if t2s_res:
        out["time_to_15_states_s"] = {p: t2s_res[p]["t2s"] for p in t2s_res}
        out["t2s_detail"] = t2s_res
        if "bf16" in t2s_res and "fp32" in t2s_res:
            out["t2s_bf16_over_fp32"] = t2s_res["bf16"]["t2s"] / t2s_res["fp32"]["t2s"]
            out["max_abs_dE_bf16_vs_fp32_ha"] = float(np.max(np.abs(np.array(t2s_res["bf16"]["energies"]) -
                                                                   np.array(t2s_res["fp32"]["energies"]))))
        gold = os.path.join(ROOT, "tests", "golden", f"{args.workload}_oracle.json")
        if os.path.exists(gold):
            ref = np.array(json.load(open(gold))["energies_ha"])[:args.nstates]
            out["max_abs_dE_vs_oracle_ha"] = {p: float(np.max(np.abs(np.array(t2s_res[p]["energies"]) - ref)))
                                              for p in t2s_res}
    if args.ao:
        out["ao_route"] = ao_route_block(ctx, P, sysc, torch, m=m)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_base or cpu_baseline(mol, args.cpu_sample_aux, m=m, gpu_flops=b["flops"])
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
