"""Benchmark of the two-site DMRG hot path on one MI355X.

Default workload (the configuration the headline metric is quoted on: DMRG at
chi = 2048): spin-1/2 Heisenberg chain, J = 1, open ends, d = 2, MPO bond
dimension 5, every bond held at chi = min(2048, the rank the chain allows),
20 H_eff applications per Lanczos (the fixed-profile throughput mode), FP64
Lanczos and Jacobi SVD.  A step is one bond visit at a centre bond with
chi_l = chi_r = 2048: theta formation, 20 H_eff matvecs with CGS2, the SVD of
the 4096 x 4096 two-site matrix, entropy and controller, truncation to 2048,
gauge move and environment growth.  The visits run on the centre bond of an
N = 24 chain (the shortest open chain whose centre bond and both neighbours
reach 2048), alternating direction, which repeats the same-shape step with
unchanged environments.  The sweep rate of the N = 100 chain at fixed
chi = 2048 is derived from the measured step: its sweep has 154 visits of
exactly this shape (bonds 11..87, both directions) and 44 edge visits whose
shapes are those of the N = 24 sweep minus its two centre visits, timed one
by one in the warm-up sweep:
    sweeps/s = 1 / (sum of the 44 edge visit times + 154 x mean step time).
W warm-up steps, then K timed steps.  Also reported: the G1 form (FP32 H_eff)
of the same visit with its energy difference from FP64, sampled H_eff
elements at the run's own chi = 2048 environments against the oracle,
isolated 4096 x 4096 FP64 SVDs against their closed-form spectrum, the
N = 100 PID run of the adaptive configuration (first sweep against the
oracle, then its sweep rate), the roofline of the dominant kernel from HIP
events over the timed region, and the oracle's time on a bounded sample.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64_tflops": 78.6, "f32_tflops": 157.3, "hbm_gbs": 8000.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=100)
    ap.add_argument("--svd-n", type=int, default=4096)
    ap.add_argument("--svd-reps", type=int, default=2)
    ap.add_argument("--no-svd", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--prec", choices=["f64", "f32"], default="f64")
    ap.add_argument("--roofline-kernel", default="", help="kernel-name prefix to time (default: auto)")
    ap.add_argument("--workload", choices=["chi2048", "heisenberg100", "xxz_batch", "svd", "fixed_chi", "scheduler",
                                           "rules", "circuit"], default="chi2048")
    ap.add_argument("--qubits", type=int, default=64, help="circuit: number of qubits")
    ap.add_argument("--layers", type=int, default=24, help="circuit: ansatz layers (two gate layers each)")
    ap.add_argument("--no-f32", action="store_true", help="chi2048: skip the FP32-H_eff companion run")
    ap.add_argument("--no-pid", action="store_true", help="chi2048: skip the N=100 PID parity and rate")
    ap.add_argument("--chi", type=int, default=256, help="fixed_chi: bond dimension")
    ap.add_argument("--matvecs", type=int, default=20, help="fixed_chi: H_eff applications per visit")
    ap.add_argument("--chains", type=int, default=64)
    ap.add_argument("--sites", type=int, default=200, help="scheduler: chain length")
    ap.add_argument("--chi-max", type=int, default=1024, help="scheduler: upper bond dimension")
    ap.add_argument("--compare-serial", action="store_true", help="xxz_batch: also run the chains one by one")
    ap.add_argument("--svd-batch", type=int, default=1)
    ap.add_argument("--svd-dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--svd-tau", type=float, default=64.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with three 1 GiB device-to-device copies (a known-size reference for HBM counters)")
    return ap.parse_args()


def copy_probe():
    """Three copies of 2^27 doubles (1 GiB read + 1 GiB written each) on the current stream."""
    import torch
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each": 2 * a.numel() * 8, "copies": 3}), file=sys.stderr)


# HBM traffic per launch measured with rocprofv3 (FETCH_SIZE and WRITE_SIZE, each scaled by
# what the counter reads for a 1 GiB device copy); valid only while the kernel's source file
# is unchanged since the counters were taken (sha256 recorded next to the figure)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
# the H_eff products' kernel is in gemm.hip, their launch shapes (problem lists) in batch.cpp
_HEFF_SRC = ["paper_2604_03960_amd/csrc/gemm.hip", "paper_2604_03960_amd/csrc/batch.cpp"]
KERNEL_SOURCE = {"lz.small": ["paper_2604_03960_amd/csrc/batch.hip"], "svd.fused": ["paper_2604_03960_amd/csrc/svd.hip"],
                 "heff.f64": _HEFF_SRC, "heff.f32": _HEFF_SRC,
                 "svd.apply": ["paper_2604_03960_amd/csrc/svd.hip"], "svd.eigen": ["paper_2604_03960_amd/csrc/svd.hip"]}


def source_sha256(kernel):
    """sha256 over the concatenated sources a kernel family's traffic figure depends on"""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCE[kernel]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_for(kernel):
    try:
        with open(TRAFFIC_FILE) as f:
            table = json.load(f)
        ent = table[kernel]
        if source_sha256(kernel) != ent["source_sha256"]:
            return None
        return ent["bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def progress(msg):
    if os.environ.get("TNA_BENCH_PROGRESS"):
        print(msg, file=sys.stderr, flush=True)


def roofline_from(stats, dominant, with_traffic=True):
    """Roofline of the kernel (or kernel family: every timer name that starts with `dominant`) from HIP
    events: algorithmic flops or bytes per launch over the mean launch time.  The measured HBM traffic
    per launch (profiles/hbm_traffic.json) belongs to the headline's launch shape: runs whose launches
    of the same kernel have other shapes pass with_traffic=False and report it as null."""
    fam = [r for r in stats if r["name"].startswith(dominant) and r["count"] > 0]
    if len(fam) > 1:
        agg = {"name": dominant, "count": sum(r["count"] for r in fam), "ms": sum(r["ms"] for r in fam),
               "flops": sum(r["flops"] for r in fam), "bytes": sum(r["bytes"] for r in fam)}
        stats = [agg]
    for r in stats:
        if r["name"] == dominant and r["count"] > 0:
            avg_ms = r["ms"] / r["count"]
            fl, by = r["flops"] / r["count"], r["bytes"] / r["count"]
            if fl > 0 and fl / max(by, 1.0) > 10.0:
                peak = PEAK["f32_tflops"] if ".f32." in dominant else PEAK["f64_tflops"]
                ach = fl / (avg_ms * 1e-3) / 1e12
                roof = {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak}
            else:
                ach = by / (avg_ms * 1e-3) / 1e9
                roof = {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                        "frac": ach / PEAK["hbm_gbs"]}
            roof.update({"kernel": dominant, "launches": r["count"], "avg_us": 1e3 * avg_ms,
                         "flops_per_launch": fl, "bytes_per_launch": by,
                         "traffic": traffic_for(dominant) if with_traffic else None})
            return roof
    return None


def run_batch(a):
    """64 XXZ chains (Delta ~ U[0,2], N from {32,48,64,96,128}) swept together, FP32 H_eff."""
    import numpy as np
    import torch

    import paper_2604_03960_amd as tna
    import synth
    ctx = tna.Context(0)
    chains = synth.xxz_chain_set(a.chains, 0)
    Ws = [tna.mpo_build(tna.MODEL_XXZ, N, [1.0, dlt, 0.0]) for dlt, N in chains]
    As, chis = [], []
    for i, (dlt, N) in enumerate(chains):
        A, chi, _ = synth.random_mps(N, 2, 8, seed=i)
        As.append(A)
        chis.append(chi)
    pid = tna.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 8, 256)
    prec = tna.HEFF_F32  # the batched-chain configuration runs the H_eff contractions in FP32
    bt = tna.DmrgBatch(ctx, Ws, As, chis, pid, heff_prec=prec)
    for _ in range(a.warmup):
        bt.sweep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for _ in range(a.steps):
        E, per, stats, st = bt.sweep()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Ns = np.array([N for _, N in chains])
    serial = None
    if a.compare_serial:
        # the same chains, one at a time through the single-chain driver, same sweeps
        t_ser, dE = 0.0, []
        for i, (dlt, N) in enumerate(chains):
            dm = tna.Dmrg(ctx, Ws[i], As[i], chis[i], pid, heff_prec=prec)
            for _ in range(a.warmup):
                dm.sweep()
            torch.cuda.synchronize()
            ts = time.perf_counter()
            for _ in range(a.steps):
                Es, _, _ = dm.sweep()
            torch.cuda.synchronize()
            t_ser += time.perf_counter() - ts
            dE.append(abs(Es - E[i]) / N)
            dm.close()
            progress(f"serial chain {i + 1}/{len(chains)} done")
        serial = {"chain_sweeps_per_s": a.chains * a.steps / t_ser, "speedup_batched": (t_ser / (t1 - t0)),
                  "max_dE_per_site_vs_batched": float(max(dE)), "note": "Delta > 1 chains may settle on a "
                  "different quasi-degenerate Neel state; compare energies"}
    out = {"metric": "chain-sweeps/s (64 XXZ chains swept together)", "value": a.chains * a.steps / (t1 - t0),
           "unit": "chain-sweeps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": 1e3 * (t1 - t0) / a.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32-heff+f64", "data": "synthetic",
           "config": {"workload": f"xxz_batch{a.chains}_N32-128_chi8-256", "chains": a.chains,
                      "N_total_sites": int(Ns.sum())},
           "batch_stats": stats, "E_per_site": (E / Ns).tolist()[:8], "serial": serial}
    print(json.dumps(out))


def run_fixed_chi(a):
    """Throughput mode: chi_min = chi_max = chi (capped by the rank each bond allows), a fixed number
    of matvecs per visit; reports sweeps/s and the H_eff GEMM rate."""
    import numpy as np
    import torch

    import paper_2604_03960_amd as tna
    import synth
    ctx = tna.Context(0)
    N = a.N
    W = tna.mpo_build(tna.MODEL_XXZ, N, [1.0, 1.0, 0.0])
    A, chi, _ = synth.random_mps(N, 2, a.chi, seed=0)
    prec = tna.HEFF_F64 if a.prec == "f64" else tna.HEFF_F32
    dm = tna.Dmrg(ctx, W, A, chi, tna.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 16, a.chi), heff_prec=prec,
                  fixed_iters=a.matvecs, fixed_chi=a.chi)
    def sweep(tag):
        """one sweep as its bond visits in sweep order (the engine step of a sweep), with progress lines"""
        recs, E = [], None
        for h in (0, 1):
            for i in range(N - 1):
                b = i if h == 0 else N - 2 - i
                E, rec, _ = dm.visit(b, h)
                recs.append(rec)
                if i % 10 == 9:
                    progress(f"{tag}: half {h}, {i + 1} of {N - 1} visits")
        return E, recs

    for w in range(a.warmup):
        sweep(f"warm-up sweep {w + 1}")
    gname = "heff." + ("f64" if a.prec == "f64" else "f32")  # the H_eff products (both GEMM forms)
    ctx.set_timing(True, gname)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        E, recs = sweep(f"timed sweep {i + 1}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = ctx.kernel_stats(reset=True)
    ctx.set_timing(False)
    fl = sum(r["flops"] for r in stats)
    ms = sum(r["ms"] for r in stats)
    dom = gname if stats else ""
    chis = np.array([r["k"] for r in recs])
    out = {"metric": f"DMRG sweeps/s at fixed chi={a.chi}", "value": a.steps / (t1 - t0), "unit": "sweeps/s",
           "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * (t1 - t0) / a.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": a.prec, "data": "synthetic",
           "config": {"workload": f"heisenberg_obc_N{N}_fixed_chi{a.chi}_{a.matvecs}matvecs", "N": N, "chi": a.chi,
                      "matvecs_per_visit": a.matvecs, "heff_prec": a.prec},
           "E_per_site": E / N, "k_max": int(chis.max()), "k_mean": float(chis.mean()),
           "heff_gemm_tflops": fl / (ms * 1e-3) / 1e12 if ms > 0 else None,
           "roofline": roofline_from(stats, dom, with_traffic=False) if dom else None,
           "phase_ms": {"lanczos": sum(r["ms_lanczos"] for r in recs), "svd": sum(r["ms_svd"] for r in recs)}}
    print(json.dumps(out))


def run_scheduler(a):
    """Learned bond-dimension scheduler vs the PID alone (J1-J2, J2 = 0.241, N = 200, D = 8, chi 16..1024,
    target 1e-8, 10 sweeps).  The network is trained on the per-visit records of PID-only Heisenberg and XXZ
    runs (the method's own sweeps), on the device."""
    import numpy as np
    import torch

    import paper_2604_03960_amd as tna
    from paper_2604_03960_amd import scheduler
    import synth
    ctx = tna.Context(0)
    chi_min, chi_max, eps_t = 16, a.chi_max, 1e-8
    pid = tna.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, chi_min, chi_max)

    def run(model, params, N, sweeps, net=None, cmin=chi_min):
        W = tna.mpo_build(model, N, params)
        A, chi, _ = synth.random_mps(N, 2, chi_min, seed=N + 7 * model)
        pp = pid if cmin == chi_min else tna.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, cmin, chi_max)
        dm = tna.Dmrg(ctx, W, A, chi, pp, eps_target=eps_t)
        if net is not None:
            dm.set_scheduler(net)
        recs, E = [], None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(sweeps):
            E, r, _ = dm.sweep()
            recs += r
            progress(f"model {model} N {N} sweep {i + 1}/{sweeps}")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        dm.close()
        return E, recs, dt

    train_runs = []
    for model, params, N in [(tna.MODEL_XXZ, [1.0, 1.0, 0.0], 40), (tna.MODEL_XXZ, [1.0, 0.5, 0.0], 40),
                             (tna.MODEL_XXZ, [1.0, 1.5, 0.0], 40), (tna.MODEL_XXZ, [1.0, 0.8, 0.0], 60)]:
        train_runs.append(run(model, params, N, 6)[1])
    X, T = scheduler.build_dataset(train_runs, chi_min, chi_max)
    t0 = time.perf_counter()
    net, losses = scheduler.train(ctx, X, T, epochs=150, batch=128, lr=2e-3, seed=1)
    t_train = time.perf_counter() - t0
    N = a.sites
    E_pid, r_pid, t_pid = run(tna.MODEL_J1J2, [1.0, 0.241], N, a.steps)
    E_ml, r_ml, t_ml = run(tna.MODEL_J1J2, [1.0, 0.241], N, a.steps, net=net)
    last = 2 * (N - 1)
    s_pid, s_ml = scheduler.summarize(r_pid[-last:], eps_t), scheduler.summarize(r_ml[-last:], eps_t)
    # the PID alone at matched cost: chi_min raised to the cube root of the learned run's mean k^3 over
    # its last sweep, so that both spend about the same sum of k^3
    k3 = np.mean([float(r["k"]) ** 3 for r in r_ml[-last:]])
    c_match = int(min(max(round(k3 ** (1.0 / 3.0)), chi_min), chi_max))
    E_pm, r_pm, t_pm = run(tna.MODEL_J1J2, [1.0, 0.241], N, a.steps, cmin=c_match)
    s_pm = scheduler.summarize(r_pm[-last:], eps_t)
    out = {"metric": f"sweeps/s, J1-J2 N={N} with the learned scheduler (PID fallback)", "value": a.steps / t_ml,
           "unit": "sweeps/s", "n_gpus": 1, "steps": a.steps, "warmup": 0, "ms_per_step": 1e3 * t_ml / a.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32-mlp",
           "data": "synthetic", "config": {"workload": f"j1j2_N{N}_J2_0.241_chi{chi_min}-{chi_max}_eps1e-8_learned_vs_pid",
                                           "train_samples": int(X.shape[0]), "epochs": 150},
           "pid_only": {"sweeps_per_s": a.steps / t_pid, "E_per_site": E_pid / N, **s_pid},
           "learned": {"sweeps_per_s": a.steps / t_ml, "E_per_site": E_ml / N, **s_ml},
           "pid_matched_cost": {"chi_min": c_match, "sweeps_per_s": a.steps / t_pm, "E_per_site": E_pm / N, **s_pm},
           "dE_per_site_learned_minus_pid": (E_ml - E_pid) / N, "train_s": t_train,
           "loss_first_last": [float(losses[0]), float(losses[-1])]}
    print(json.dumps(out))


def run_rules(a):
    """The rank rules side by side (the paper's ablation, Sec. 13): Heisenberg chain, chi_max = 64,
    5 sweeps from the same initial MPS under fixed chi, the PID (Algorithm 2), the threshold rule
    (eps_trunc = 1e-10) and Algorithm 1 (gamma = 1.5).  Wall time per run, E/N, mean and max kept chi."""
    import numpy as np
    import torch

    import paper_2604_03960_amd as tna
    import synth
    ctx = tna.Context(0)
    out_runs = {}
    for N in (20, a.N):
        W = tna.mpo_build(tna.MODEL_XXZ, N, [1.0, 1.0, 0.0])
        A, chi, _ = synth.random_mps(N, 2, 4, seed=1)
        rules = {"fixed_chi64": dict(fixed_chi=64), "pid": dict(),
                 "threshold_1e-10": dict(chi_rule=tna.CHI_THRESHOLD, rule_param=1e-10),
                 "alg1_gamma1.5": dict(chi_rule=tna.CHI_ENTROPY, rule_param=1.5),
                 "pid_gains_x0.5": dict(gain_scale=0.5), "pid_gains_x1.5": dict(gain_scale=1.5)}
        for name, kw in rules.items():
            g = kw.pop("gain_scale", 1.0)  # the paper's +-50% robustness check scales all three gains
            pp = tna.pid_params(2.0 * g, 0.1 * g, 0.5 * g, 0.5, 0.3, 4, 64)
            dm = tna.Dmrg(ctx, W, A, chi, pp, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Es = []
            for i in range(5):
                E, recs, st = dm.sweep()
                Es.append(E / N)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ks = np.array([r["k"] for r in recs[-(N - 1):]])
            out_runs[f"N{N}_{name}"] = {"s": dt, "E_per_site": E / N, "chi_mean": float(ks.mean()),
                                        "chi_max": int(ks.max()), "E_per_site_by_sweep": Es}
            dm.close()
            progress(f"N {N} {name} done")
    base = {N: out_runs[f"N{N}_fixed_chi64"]["s"] for N in (20, a.N)}
    for k, v in out_runs.items():
        v["speedup_vs_fixed"] = base[int(k.split("_")[0][1:])] / v["s"]
    out = {"metric": "5-sweep wall time per rank rule (fixed chi 64 = 1.0x)", "value": out_runs["N20_pid"]["speedup_vs_fixed"],
           "unit": "x vs fixed chi (N=20 PID)", "n_gpus": 1, "steps": 5, "warmup": 0, "ms_per_step": None,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"heisenberg_rules_N20_N{a.N}_chimax64"}, "runs": out_runs}
    print(json.dumps(out))


def run_svd(a):
    """Isolated truncated SVDs of n x n matrices with spectrum exp(-k/tau), keep n/2."""
    import numpy as np
    import torch

    import paper_2604_03960_amd as tna
    import synth
    ctx = tna.Context(0)
    n, B = a.svd_n, a.svd_batch
    dt = torch.float64 if a.svd_dtype == "f64" else torch.float32
    mats = []
    for i in range(B):
        mats.append(torch.from_numpy(synth.svd_test_matrix(n, a.svd_tau, seed=0, index=i)))
        progress(f"input matrix {i + 1}/{B} generated")
    A = torch.stack(mats)
    A = A.to(dt).cuda().contiguous()
    sig = torch.from_numpy(synth.svd_test_spectrum(n, a.svd_tau)).cuda()
    run = (lambda: ctx.svd_truncate(A[0], n // 2)) if B == 1 else (lambda: ctx.svd_truncate_batched(A, n // 2))
    res = run()
    torch.cuda.synchronize()
    ctx.set_timing(True, "svd.apply")
    t0 = time.perf_counter()
    for _ in range(a.svd_reps):
        res = run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = ctx.kernel_stats(reset=True)
    ctx.set_timing(False)
    S = res[0]
    err = (S.reshape(B, -1) - sig[None, :]).abs().max().item()
    sweeps = res[5] if B == 1 else res[4]
    # one more call with every svd kernel timed, for the per-kernel breakdown
    ctx.set_timing(True, "svd.")
    run()
    torch.cuda.synchronize()
    brk = sorted(ctx.kernel_stats(reset=True), key=lambda r: -r["ms"])
    ctx.set_timing(False)
    breakdown = {r["name"]: {"ms": r["ms"], "launches": r["count"], "avg_us": 1e3 * r["ms"] / max(r["count"], 1)}
                 for r in brk}
    value = B * a.svd_reps / (t1 - t0)
    nominal = 22.0 * n ** 3  # Golub-Reinsch count with thin U and V
    out = {"metric": f"SVD/s at chi={n // 2} ({n}x{n}, {a.svd_dtype}, batch {B})", "value": value,
           "unit": "SVD/s", "n_gpus": 1, "steps": a.svd_reps, "warmup": 1,
           "ms_per_step": 1e3 * (t1 - t0) / a.svd_reps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": a.svd_dtype, "data": "synthetic",
           "config": {"workload": f"svd_{n}x{n}_tau{a.svd_tau:g}_batch{B}", "n": n, "tau": a.svd_tau, "batch": B},
           "max_abs_sigma_err": err, "nominal_tflops": value * nominal / 1e12, "jacobi_sweeps": sweeps,
           "breakdown_one_call": breakdown,
           "roofline": roofline_from(stats, "svd.apply")}
    print(json.dumps(out))


CHI_HEAD = 2048   # bond dimension of the headline configuration
N_VISIT = 24      # shortest open chain whose centre bond and both neighbours reach chi = 2048
N_SWEEP = 100     # chain whose sweep rate is derived
N_FULL = 154      # visits of the N = 100 sweep with chi_l = chi_r = 2048 (bonds 11..87, both directions)


def _visit(dm, b, h):
    t = time.perf_counter()
    E, rec, st = dm.visit(b, h)  # synchronises
    return E, rec, time.perf_counter() - t


def cpu_baseline_leg(a, gpu):
    """The oracle on the host: a bounded sample of the headline step, plus the oracle's side of the parity
    figures the bench reports (sampled H_eff elements at the run's own chi = 2048 environments, and the
    first sweep of the N = 100 PID run)."""
    import numpy as np

    import oracle
    import synth
    out = {}
    # sample: one visit at the same bond shape scaled down to chi = 256 (20 Lanczos matvecs, Jacobi SVD of
    # the 512 x 512 two-site matrix, one environment growth), seeded environments
    cs = 192
    W = oracle.mpo(oracle.MODEL_XXZ, 4, [1.0, 1.0, 0.0])
    D = W.shape[1]
    L = synth.normal(101, cs * D * cs).reshape(cs, D, cs)
    R = synth.normal(102, cs * D * cs).reshape(cs, D, cs)
    L, R = 0.5 * (L + L.transpose(2, 1, 0)), 0.5 * (R + R.transpose(2, 1, 0))
    th = synth.normal(103, cs * 4 * cs).reshape(cs, 2, 2, cs)
    t0 = time.perf_counter()
    E, th1, it, rc = oracle.lanczos_heff(L, W[1], W[2], R, th, fixed_iters=a.matvecs)
    S, U, V, sw, rc = oracle.svd(th1.reshape(2 * cs, 2 * cs))
    Aleft = U[:, :cs].reshape(cs, 2, cs)
    oracle.env_left(L, W[1], Aleft)
    t_sample = time.perf_counter() - t0
    scale = (CHI_HEAD / cs) ** 3
    t_full = t_sample * scale
    ratio = gpu["edge_s"] / gpu["step_s"]  # the N = 100 sweep's edge visits in units of one full visit
    out["cpu_baseline"] = {
        "value": 1.0 / (t_full * (N_FULL + ratio)), "unit": "sweeps/s", "cores": 1, "kind": "oracle",
        "sample": f"one oracle bond visit at chi = {cs} ({a.matvecs} H_eff matvecs, Jacobi SVD of the "
                  f"{2 * cs}x{2 * cs} two-site matrix, one environment growth; single-threaded C, "
                  f"{t_sample:.1f} s), scaled by chi^3 ({scale:.0f}x) to the chi = 2048 visit and by the GPU's "
                  f"edge-to-centre time ratio to the N = 100 sweep",
        "sample_s": t_sample, "visit_s_extrapolated": t_full}
    # H_eff elements at the run's own environments against the element-wise oracle
    if gpu.get("heff_sample") is not None:
        hs = gpu["heff_sample"]
        ref = np.array([oracle.heff_element(hs["L"], hs["W1"], hs["W2"], hs["R"], hs["theta"], ix)
                        for ix in hs["idx"]])
        scale_out = hs["out_absmax"]
        out["heff_chi2048_sampled"] = {
            "elements": len(hs["idx"]),
            "max_abs_err_rel_to_max_out_f64": float(np.max(np.abs(hs["gpu_f64"] - ref)) / scale_out),
            "max_abs_err_rel_to_max_out_f32": float(np.max(np.abs(hs["gpu_f32"] - ref)) / scale_out)}
    # the adaptive N = 100 configuration: the oracle's first sweep from the same initial MPS
    if gpu.get("pid") is not None:
        p = gpu["pid"]
        Wo = oracle.mpo(oracle.MODEL_XXZ, N_SWEEP, [1.0, 1.0, 0.0])
        pp = oracle.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 16, 1024)
        t4 = time.perf_counter()
        ro = oracle.dmrg_run(Wo, p["A"], p["chi"], pp, 1, eps_target=1e-8)
        t5 = time.perf_counter()
        chi_ref = [int(r["chi_ctrl"]) for r in ro["log"]]
        E_ref = [float(r["E"]) for r in ro["log"]]
        out["pid_N100_first_sweep"] = {
            "dE_per_site": abs(p["E_first"] - float(ro["E"][0])) / N_SWEEP,
            "max_visit_dE_per_site": float(np.max(np.abs(np.array(p["E_visits"]) - np.array(E_ref)))) / N_SWEEP,
            "chi_decisions_equal": p["chi_ctrl"] == chi_ref, "visits": len(chi_ref),
            "oracle_sweeps_per_s_1core": 1.0 / (t5 - t4), "E_oracle": float(ro["E"][0]), "E_gpu": p["E_first"]}
    return out


def run_chi2048(a):
    """Headline: DMRG at fixed chi = 2048, one centre-bond visit per step (see the module docstring)."""
    import numpy as np
    import torch

    import paper_2604_03960_amd as tna
    import synth

    torch.cuda.init()
    ctx = tna.Context(0)
    chi, Nv = CHI_HEAD, N_VISIT
    c = Nv // 2 - 1  # centre bond: theta is (chi d) x (d chi)
    W = tna.mpo_build(tna.MODEL_XXZ, Nv, [1.0, 1.0, 0.0])
    A, chi0, _ = synth.random_mps(Nv, 2, chi, seed=0)
    pid = tna.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 16, chi)

    def prepare(prec, tag):
        """create, one sweep with every visit timed, then left-to-right visits up to the centre bond"""
        dm = tna.Dmrg(ctx, W, A, chi0, pid, heff_prec=prec, fixed_iters=a.matvecs, fixed_chi=chi)
        times, E_sweep = {}, None
        for h in (0, 1):
            for step in range(Nv - 1):
                b = step if h == 0 else Nv - 2 - step
                E_sweep, _, dt = _visit(dm, b, h)
                times[(b, h)] = dt
            progress(f"{tag}: warm-up half sweep {h} done")
        for b in range(c):
            _visit(dm, b, 0)
        return dm, times, E_sweep

    dm, times, E_sweep64 = prepare(tna.HEFF_F64, "f64")
    edge_s = sum(t for (b, h), t in times.items() if b != c)
    # warm-up steps at the centre bond; the first one also ranks the kernels (every launch timed)
    dirn = 0
    ctx.set_timing(True, "")
    E_first64, rec, _ = _visit(dm, c, dirn)
    dirn ^= 1
    ranking = ctx.kernel_stats(reset=True)
    ctx.set_timing(False)
    for _ in range(max(a.warmup, 1) - 1):
        _visit(dm, c, dirn)
        dirn ^= 1
    # dominant kernel family (timer names up to the tile suffix: the H_eff GEMMs' NN and NT forms are one
    # kernel template, gemm_grouped_kernel) by time in the ranking visit
    fams = {}
    for r in ranking:
        f = ".".join(r["name"].split(".")[:2])
        fams[f] = fams.get(f, 0.0) + r["ms"]
    dominant = a.roofline_kernel or (max(fams, key=fams.get) if fams else "")
    if dominant:
        ctx.set_timing(True, dominant)
    st0 = dm.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for i in range(a.steps):
        E, rec, st = dm.visit(c, dirn)
        dirn ^= 1
        recs.append(rec)
        progress(f"step {i + 1}/{a.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = ctx.kernel_stats(reset=True) if dominant else []
    ctx.set_timing(False)
    st1 = dm.stats()
    svd_rows_swept = (st1["svd_rows_swept"] - st0["svd_rows_swept"]) / a.steps
    step_s = (t1 - t0) / a.steps
    roof = roofline_from(stats, dominant) if dominant else None
    # H_eff at the run's own environments (stand-alone entry point, FP64 and FP32) for the oracle check
    hs = None
    if not a.no_cpu_baseline:
        L, R = dm.env(0, c), dm.env(1, c + 1)
        th = torch.from_numpy(synth.normal(11, chi * 4 * chi).reshape(chi, 2, 2, chi)).cuda()
        W1, W2 = torch.from_numpy(W[c]).cuda(), torch.from_numpy(W[c + 1]).cuda()
        o64 = ctx.heff_apply(L, W1, W2, R, th, prec=tna.HEFF_F64)
        o32 = ctx.heff_apply(L, W1, W2, R, th, prec=tna.HEFF_F32)
        u = synth.uniform53(12, 0, 4 * 8)
        idx = [(int(u[4 * i] * chi), int(u[4 * i + 1] * 2), int(u[4 * i + 2] * 2), int(u[4 * i + 3] * chi))
               for i in range(8)]
        pick = lambda o: np.array([o[ix].item() for ix in idx])
        hs = {"L": L.cpu().numpy(), "R": R.cpu().numpy(), "W1": W[c], "W2": W[c + 1], "theta": th.cpu().numpy(),
              "idx": idx, "gpu_f64": pick(o64), "gpu_f32": pick(o32), "out_absmax": o64.abs().max().item()}
        del L, R, th, o64, o32
    ks = [r["k"] for r in recs]
    phase = {k: float(np.mean([r[k] for r in recs])) for k in ("ms_lanczos", "ms_svd", "ms_other")}
    svd_sweeps = [r["svd_sweeps"] for r in recs]
    dm.close()
    torch.cuda.empty_cache()
    # G1: the same sequence with the H_eff contractions in FP32
    g1 = None
    if not a.no_f32:
        dm32, t32, E_sweep32 = prepare(tna.HEFF_F32, "f32")
        E_first32, _, _ = _visit(dm32, c, 0)
        k32 = 4  # two visits in each direction, like the timed steps
        tt = 0.0
        dd = 1
        ph32 = []
        for _ in range(k32):
            _, r32, dt = _visit(dm32, c, dd)
            dd ^= 1
            tt += dt
            ph32.append(r32)
        g1 = {"ms_per_step": 1e3 * tt / k32, "steps": k32,
              "phase_ms_per_step": {k: float(np.mean([r[k] for r in ph32])) for k in ("ms_lanczos", "ms_svd", "ms_other")},
              "sweeps_per_s_N100": 1.0 / (sum(t for (b, h), t in t32.items() if b != c) + N_FULL * tt / k32),
              "dE_per_site_vs_f64_first_centre_visit": abs(E_first32 - E_first64) / Nv,
              "dE_per_site_vs_f64_after_warmup_sweep": abs(E_sweep32 - E_sweep64) / Nv}
        dm32.close()
        torch.cuda.empty_cache()
    # isolated SVD at chi = 2048 (4096 x 4096, FP64) against the closed-form spectrum
    svd = None
    if not a.no_svd:
        n = a.svd_n
        Ad = torch.from_numpy(synth.svd_test_matrix(n, 64.0, seed=0)).cuda()
        sig = torch.from_numpy(synth.svd_test_spectrum(n, 64.0)).cuda()
        S, U, Vt, spec, k, sw, st = ctx.svd_truncate(Ad, n // 2)  # warm-up
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        sweeps = []
        for _ in range(a.svd_reps):
            S, U, Vt, spec, k, sw, st = ctx.svd_truncate(Ad, n // 2)
            sweeps.append(sw)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        err = (S - sig).abs().max().item()
        svd = {"n": n, "chi": n // 2, "svd_per_s": a.svd_reps / (t3 - t2), "ms_per_svd": 1e3 * (t3 - t2) / a.svd_reps,
               "jacobi_sweeps": sweeps, "max_abs_sigma_err": err, "entropy": spec[1].item(),
               "nominal_22n3_tflops": 22.0 * n ** 3 * a.svd_reps / (t3 - t2) / 1e12}
        del Ad, U, Vt
    # the adaptive configuration (N = 100, PID, chi 16..1024): first sweep for the oracle comparison,
    # then its sweep rate
    pid100 = None
    pid_in = None
    if not a.no_pid:
        Wp = tna.mpo_build(tna.MODEL_XXZ, N_SWEEP, [1.0, 1.0, 0.0])
        Ap, chip, _ = synth.random_mps(N_SWEEP, 2, 16, seed=0)
        dmp = tna.Dmrg(ctx, Wp, Ap, chip, tna.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 16, 1024), eps_target=1e-8)
        E1, r1, _ = dmp.sweep()
        pid_in = {"A": Ap, "chi": chip, "E_first": E1, "chi_ctrl": [r["chi_ctrl"] for r in r1],
                  "E_visits": [r["E"] for r in r1]}
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for _ in range(4):
            Ep, _, _ = dmp.sweep()
        torch.cuda.synchronize()
        pid100 = {"sweeps_per_s": 4 / (time.perf_counter() - tp), "sweeps_timed": 4, "E_per_site_after_5": Ep / N_SWEEP,
                  "chi_max_final": int(np.max(dmp.state()[0]))}
        dmp.close()
    gpu = {"edge_s": edge_s, "step_s": step_s, "heff_sample": hs, "pid": pid_in}
    cpu = cpu_baseline_leg(a, gpu) if not a.no_cpu_baseline else {}
    if pid100 is not None and "pid_N100_first_sweep" in cpu:
        pid100["vs_oracle_first_sweep"] = cpu.pop("pid_N100_first_sweep")
    value = 1.0 / (edge_s + N_FULL * step_s)
    out = {
        "metric": "DMRG sweeps/s & SVD/s at chi=2048 vs FP64 plain, same dE/N vs oracle",
        "value": value, "unit": "sweeps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1e3 * step_s, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "heisenberg_obc_fixed_chi2048_centre_visit_N100_sweep_rate", "chi": chi,
                   "N_sweep": N_SWEEP, "N_visit_chain": Nv, "centre_bond": c, "d": 2, "D": 5,
                   "matvecs_per_visit": a.matvecs, "theta": f"{2 * chi}x{2 * chi}", "heff_prec": "f64",
                   "step": "one centre-bond visit (theta, Lanczos, SVD, controller, truncation, environment)",
                   "derivation": "sweeps/s = 1 / (edge visits of the N=24 warm-up sweep + 154 x step time)"},
        "centre_visits_per_s": 1.0 / step_s, "edge_visits_s": edge_s, "kept_rank": ks[:4],
        "phase_ms_per_step": phase, "svd_jacobi_sweeps_per_step": svd_sweeps[:4],
        "svd_rows_swept_per_step": svd_rows_swept,
        "E_per_site_warmup_sweep_N24": E_sweep64 / Nv,
        "roofline": roof, "svd_chi2048": svd, "g1_f32_heff": g1, "pid_N100": pid100,
        "heff_chi2048_vs_oracle": cpu.get("heff_chi2048_sampled"),
        "cpu_baseline": cpu.get("cpu_baseline"),
        "kernel_ranking_one_step": sorted(ranking, key=lambda r: -r["ms"])[:16],
    }
    print(json.dumps(out))


def run_circuit(a):
    """Circuit simulation with adaptive bond dimensions (the circuit-level bond-dimension map): a
    hardware-efficient ansatz (RY rotations and CNOT brickwork) of N qubits and L layers, the PID
    choosing each gate bond's dimension (chi in [chi_min, chi_max]); every gate layer's SVDs as one
    group, against the same gates one at a time."""
    import numpy as np
    import torch

    import paper_2604_03960_amd as tna
    import synth
    ctx = tna.Context(0)
    N, L = a.qubits, a.layers
    par, g, _ = synth.hea_circuit(N, L, seed=0)
    pid = tna.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 4, a.chi_max)
    out_runs = {}
    for name, one in (("batched", False), ("one_at_a_time", True)):
        circ = tna.Circuit(ctx, N, pid, one_at_a_time=one)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cmap, recs = circ.run(par, g)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out_runs[name] = {"s": dt, "gates_per_s": len(recs) / dt, "layers_per_s": L / dt,
                          "chi_max_reached": int(cmap.max()), "chi_mean_last": float(cmap[-1].mean()),
                          "trunc_err_sum": float(sum(r["eps"] for r in recs))}
        if name == "batched":
            chi_map = cmap
        circ.close()
        progress(f"circuit {name} done")
    b, s = out_runs["batched"], out_runs["one_at_a_time"]
    out = {"metric": f"gate layers/s, {N}-qubit hardware-efficient ansatz with adaptive chi", "value": b["layers_per_s"],
           "unit": "layers/s", "n_gpus": 1, "steps": L, "warmup": 0, "ms_per_step": 1e3 * b["s"] / L,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"hea_N{N}_L{L}_pid_chi4-{a.chi_max}", "qubits": N, "ansatz_layers": L,
                      "gate_layers": 2 * L},
           "runs": out_runs, "speedup_batched_vs_one_at_a_time": s["s"] / b["s"],
           "chi_map_every_4th_layer": chi_map[::8].tolist()}
    print(json.dumps(out))


def run_pid100(a):
    """The adaptive configuration: N = 100, PID with chi in [16, 1024], Lanczos tol 1e-12, 10 sweeps."""
    import numpy as np
    import torch

    import paper_2604_03960_amd as tna
    import synth

    torch.cuda.init()
    N, d, chi0 = a.N, 2, 16
    W = tna.mpo_build(tna.MODEL_XXZ, N, [1.0, 1.0, 0.0])
    A, chi, _ = synth.random_mps(N, d, chi0, seed=0)
    pid = tna.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 16, 1024)
    ctx = tna.Context(0)
    prec = tna.HEFF_F64 if a.prec == "f64" else tna.HEFF_F32
    dm = tna.Dmrg(ctx, W, A, chi, pid, lanczos_tol=1e-12, heff_prec=prec, eps_target=1e-8)

    # warm-up sweeps; the first one also ranks kernels by total time (all launches timed)
    ctx.set_timing(True, "")
    for _ in range(max(a.warmup, 1) if a.warmup > 0 else 0):
        dm.sweep()
    warm_stats = ctx.kernel_stats(reset=True)
    ctx.set_timing(False)
    dominant = a.roofline_kernel
    if not dominant and warm_stats:
        dominant = max(warm_stats, key=lambda r: r["ms"])["name"]

    # timed region: only the dominant kernel carries events
    if dominant:
        ctx.set_timing(True, dominant)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Es, logs = [], []
    for i in range(a.steps):
        E, recs, st = dm.sweep()
        Es.append(E)
        logs += recs
        progress(f"sweep {i + 1}/{a.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = ctx.kernel_stats(reset=True)
    ctx.set_timing(False)
    ms_step = 1e3 * (t1 - t0) / a.steps
    chi_fin, _ = dm.state()

    roof = roofline_from(stats, dominant, with_traffic=False) if dominant else None

    # isolated SVD at chi = 2048 (4096 x 4096, FP64)
    svd = None
    if not a.no_svd:
        n = a.svd_n
        Ad = torch.from_numpy(synth.svd_test_matrix(n, 64.0, seed=0)).cuda()
        sig = torch.from_numpy(synth.svd_test_spectrum(n, 64.0)).cuda()
        S, U, Vt, spec, k, sw, st = ctx.svd_truncate(Ad, n // 2)  # warm-up
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        sweeps = []
        for _ in range(a.svd_reps):
            S, U, Vt, spec, k, sw, st = ctx.svd_truncate(Ad, n // 2)
            sweeps.append(sw)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        err = (S - sig).abs().max().item()
        svd = {"n": n, "chi": n // 2, "svd_per_s": a.svd_reps / (t3 - t2), "ms_per_svd": 1e3 * (t3 - t2) / a.svd_reps,
               "jacobi_sweeps": sweeps, "max_abs_sigma_err": err, "entropy": spec[1].item()}

    # CPU baseline: the oracle on a bounded sample of the same workload
    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        Wo = oracle.mpo(oracle.MODEL_XXZ, N, [1.0, 1.0, 0.0])
        pp = oracle.pid_params(2.0, 0.1, 0.5, 1.0, 0.3, 16, 1024)
        t4 = time.perf_counter()
        ro = oracle.dmrg_run(Wo, A, chi, pp, 1)
        t5 = time.perf_counter()
        cpu = {"value": 1.0 / (t5 - t4), "unit": "sweeps/s", "cores": 1, "kind": "oracle",
               "sample": f"first sweep of the same N={N} run from the same initial MPS (single-threaded C, "
                         f"{t5 - t4:.1f} s)", "E_first_sweep": float(ro["E"][0])}

    out = {
        "metric": "DMRG sweeps/s, adaptive PID run (chi 16..1024)",
        "value": a.steps / (t1 - t0), "unit": "sweeps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if a.prec == "f64" else "f32-heff+f64", "data": "synthetic",
        "config": {"workload": f"heisenberg_obc_N{N}_pid_chi16-1024_two_site_dmrg", "N": N, "d": d, "D": 5,
                   "chi_min": 16, "chi_max": 1024, "alpha": 0.3, "gains": [2.0, 0.1, 0.5], "s_target": 1.0,
                   "lanczos_tol": 1e-12, "heff_prec": a.prec},
        "E_per_site_last": Es[-1] / N if Es else None,
        "chi_final_mean": float(np.mean(chi_fin)), "chi_final_max": int(np.max(chi_fin)),
        "roofline": roof, "svd_chi2048": svd, "cpu_baseline": cpu,
        "kernel_ranking_warmup": sorted(warm_stats, key=lambda r: -r["ms"])[:8],
    }
    print(json.dumps(out))


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (no multi-GPU path)"}))
        sys.exit(2)
    runs = {"chi2048": run_chi2048, "heisenberg100": run_pid100, "xxz_batch": run_batch, "svd": run_svd,
            "fixed_chi": run_fixed_chi, "scheduler": run_scheduler, "rules": run_rules, "circuit": run_circuit}
    return runs[a.workload](a)


if __name__ == "__main__":
    args = parse()
    main()
    if args.copy_probe:
        copy_probe()
