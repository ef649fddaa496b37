#!/usr/bin/env python3
"""Throughput of the batched peridynamic Monte-Carlo solve on one MI355X.

Workload (default): the level-1 notched concrete beam (70 x 20 x 20 = 28,000
nodes, 1,490,324 unique bonds after the notch cut), a batch of 64 samples
whose per-node limit stretch is a lognormal field (mean s0, CoV 0.2) from a
50-mode Karhunen-Loeve expansion of a squared-exponential Gaussian field
(length scale 20 mm, seed 1), 8000 damped velocity-Verlet steps under the
literal displacement control (5e-8 mm per step scaled to dx), FP32 bond work
with compensated accumulation and an FP64 reaction.  One benchmark "step" is
one whole batch solve (every sample, every time step) with the inputs already
resident in device memory.

value = unique bond updates per second (bonds x time steps x samples / s).
Alongside: samples/s, the plain per-sample FP64 solve of the same beam, the
cracking-load variant, the three-level MLMC hierarchy (MLMC samples/s), the
step kernel's roofline (algorithmic bytes against the HBM peak, beside the
counter-measured traffic), and the FP64 CPU oracle on a bounded sample of the
same workload, on one host thread and on all of them.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Roofline of the step kernel (the hot path is bound by HBM bandwidth: no
# dense contraction, ~40 flop per ~8 algorithmic bytes).  Algorithmic bytes
# per unique bond-update of the batched FP32 path: the bond's history word
# (4 B), its neighbour identity shared by the samples of a mesh, and the node
# state (u, v, their compensation terms, two fields: ~104 B per node-step)
# amortised over the 46-57 bonds of a node: 7.8 B.
ALG_BYTES_PER_BOND_UPDATE_F32 = 7.8
PEAK_HBM_GBPS = 8000.0
# Algorithmic floating-point operations per bond direction of the FP32 path
# (a labelled extra beside the HBM roofline):
# e = u_j - u_i (3), v.e (5), e.e (5), 2 v.e + e.e (2), |v|^2 + num (1),
# |y| = y2 rsqrt(y2) (2), |v|(|y| + |v|) (2), s = num / den (1),
# w = s / |y| (1), existence weight (1), y = v + e (3), G += w y (6),
# compensated accumulation of the pair sums (12 per pair = 6 per direction).
FLOPS_PER_BOND_DIR_F32 = 38
# Vector FP32 peak of the chip: 256 CUs x 4 SIMDs x 32 lanes x 2 (FMA) x
# 2.4 GHz = 157.3 TFLOP/s.
PEAK_TFLOPS_F32 = 256 * 4 * 32 * 2 * 2.4e9 / 1e12
# step-kernel instantiation per launch shape (FP32, compensated, no c field)
SHAPE_NAMES = ["lds 16x4x4", "lds 8x8x4", "lds 12x4x4", "global 256"]
SHAPE_KERNELS = ["step_kernel<float, true, false, true, Brick<16, 4, 4, 2>>",
                 "step_kernel<float, true, false, true, Brick<8, 8, 4>>",
                 "step_kernel<float, true, false, true, Brick<12, 4, 4>>",
                 "step_kernel<float, true, false, false, Brick<256, 1, 1>>"]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("step_kernels.h", "pd_internal.h"):
        with open(os.path.join(ROOT, "paper_2212_04415_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel):
    """HBM bytes per step-kernel launch from the committed rocprofv3 PMC
    summary, or None when it is missing, was taken on other kernel source, or
    covers another launch shape than the one this run uses."""
    path = os.path.join(ROOT, "profiles", "step_kernel_L1x64_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("kernel") != "pdmi::" + kernel:
        return None
    return d.get("hbm_bytes_per_launch")


def finite_json(x):
    """The bench line with every non-finite float replaced by null (strict
    JSON has no NaN or infinity)."""
    if isinstance(x, dict):
        return {k: finite_json(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [finite_json(v) for v in x]
    if isinstance(x, float) and not math.isfinite(x):
        return None
    return x


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def host_threads():
    """Threads the oracle may use: OMP_NUM_THREADS if set, else the CPUs this
    process may run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.strip().isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(seconds_each=8.0):
    """The FP64 oracle on the host: one sample of the same beam and field,
    timed over a bounded number of its steps, once on one thread and once on
    every host thread (its force loop runs in OpenMP over fixed bond chunks)."""
    import numpy as np
    import workloads as W
    from oracle import geometry as OG
    from oracle import kl as OKL
    from oracle import solver as OS
    OS.build(force=False)
    lv = W.level(1)
    ob = OKL.Basis3D((lv.beam.length, lv.beam.thickness, lv.beam.depth), W.FIELD_CORR_LEN, W.FIELD_MODES, 256)
    pos = OG.node_positions(lv.shape, lv.dx)
    xi = W.kl_coefficients(1, 1)
    s0 = OKL.lognormal_field(ob, pos, xi, W.S0_MEAN, W.FIELD_COV)[0]
    out = {}
    for threads in (1, host_threads()):
        used = OS.set_threads(threads)
        probe = OS.beam_problem(lv, s0=s0, n_steps=10)
        t = time.perf_counter()
        probe.run(want_state=False)
        per_step = (time.perf_counter() - t) / 10
        n = max(10, int(seconds_each / per_step))
        prob = OS.beam_problem(lv, s0=s0, n_steps=n)
        t = time.perf_counter()
        prob.run(want_state=False)
        dt = time.perf_counter() - t
        out[used] = (prob.n_bonds * n / dt, n, dt)
    OS.set_threads(host_threads())
    cores = max(out)
    rate, n, dt = out[cores]
    one_rate, one_n, one_dt = out[1]
    return {"value": rate, "unit": "bond-updates/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "single_thread": {"value": one_rate, "steps": one_n, "seconds": one_dt},
            "sample": f"1 sample of the level-1 beam (seed-1 KL field), first {n} of {lv.n_steps} steps on "
                      f"{cores} threads ({dt:.1f} s) and {one_n} steps on 1 thread ({one_dt:.1f} s); "
                      f"C at -O2, OpenMP over fixed bond chunks"}


def mlmc_leg(fracture=True, field_model="lognormal"):
    """The three-level MLMC batch (dx = 5 / 2.5 / 1.25 mm; 1024 / 128 / 16
    samples, each level-l>0 sample paired with a coarse solve on the same KL
    coefficients: 1152 / 144 / 16 solves) in one batched call."""
    import workloads as W
    from paper_2212_04415_amd import mlmc
    levels = [W.level(l, fracture=fracture) for l in range(3)]
    out = mlmc.coupled_batch(levels, [1024, 128, 16], seed=2, precision="f32", corr_len=W.FIELD_CORR_LEN,
                             n_modes=W.FIELD_MODES, mean=W.S0_MEAN, cov=W.FIELD_COV,
                             kl_coefficients=W.kl_coefficients, field_model=field_model)
    bu = sum(b * n * st for b, n, st in zip(out["bonds"], out["solves"], out["steps"]))
    import torch
    samples = [1024, 128, 16]
    fine = [torch.tensor(out["Q"][l][:samples[l]], device="cuda") for l in range(3)]
    coarse = [None] + [torch.tensor(out["Q"][l - 1][samples[l - 1]:samples[l - 1] + samples[l]], device="cuda")
                       for l in (1, 2)]
    u = [0.05, 0.5, 0.95]
    quant = mlmc.cdf(fine, coarse, u)
    return {"wall_s": out["wall_s"], "bond_updates_per_s": bu / out["wall_s"],
            "multilevel_quantiles_N": {str(k): float(v) for k, v in zip(u, quant)},
            "mlmc_samples_per_s": (1024 + 128 + 16) / out["wall_s"],
            "solves_per_level": out["solves"], "estimate_N": out["estimate"],
            "sampling_std_N": max(out["sampling_variance"], 0.0) ** 0.5,
            "level_mean_var": [[m, v] for m, v, _ in out["levels"]],
            "load_per_step_mm_L0": levels[0].du * 1e3}


def adaptive_leg(eps=80.0, n_warm=100):
    """Algorithm 1 (adaptive MLMC) on the three cracking-load levels, with the
    paper's 100 warm-up samples, fitted alpha and RMSE target eps (N)."""
    import workloads as W
    from paper_2212_04415_amd import mlmc
    levels = [W.level(l, fracture=True) for l in range(3)]
    run, costs, dofs = mlmc.solver_sampler(levels, seed=2, precision="f32", corr_len=W.FIELD_CORR_LEN,
                                           n_modes=W.FIELD_MODES, mean=W.S0_MEAN, cov=W.FIELD_COV,
                                           kl_coefficients=W.kl_coefficients)
    out = mlmc.adaptive(run, eps, costs, dofs, n_warm=n_warm, alpha=None, alpha_default=0.5)
    return {"eps_N": eps, "levels_used": out["L"] + 1, "converged": out["converged"], "N": out["N"],
            "estimate_N": out["estimate"], "sampling_std_N": max(out["sampling_variance"], 0.0) ** 0.5,
            "bias_estimate_N": out["bias"], "alpha_fitted": out["history"][-1]["alpha"],
            "wall_s": out["wall_s"], "bond_updates_per_s": out["cost"] / out["wall_s"],
            "mlmc_samples_per_s": sum(out["N"]) / out["wall_s"]}


def sweep_leg(steps=1000):
    """The size-sweep beams (D = 50 / 100 / 200 / 400 mm, dx = 2.5 mm, 32
    samples each, seed 4): batched FP32 throughput over the first `steps`
    time steps of each (the full runs take 8000 D / 50 steps)."""
    import dataclasses
    import torch
    import workloads as W
    from paper_2212_04415_amd import beam as B
    sweep = [c for c in W.configs() if c.name == "size_sweep"][0]
    out = []
    for i, lv in enumerate(sweep.levels):
        mesh = B.Mesh.for_level(lv)
        kl = B.KL(mesh, W.FIELD_CORR_LEN, W.FIELD_MODES, 256)
        S = sweep.samples[i]
        xi = torch.tensor(W.kl_coefficients(sweep.seed, S, stream=i))
        s0 = kl.lognormal(xi, W.S0_MEAN, W.FIELD_COV, dtype=torch.float32)
        tune = B.autotune(mesh, B.make_params(lv), S)
        lvs = dataclasses.replace(lv, n_steps=min(steps, lv.n_steps))
        item = B.BatchItem(mesh, B.make_params(lvs), S, s0)
        B.run_batch([dataclasses.replace(item, params=B.make_params(lvs, n_steps=64))])
        torch.cuda.synchronize()
        t = time.perf_counter()
        B.run_batch([item])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        out.append({"depth_mm": round(lv.beam.depth * 1e3), "nodes": mesh.n_nodes, "bonds": mesh.n_bonds,
                    "samples": S, "steps_timed": lvs.n_steps, "bond_updates_per_s": mesh.n_bonds * lvs.n_steps * S / dt,
                    "us_per_step": dt / lvs.n_steps * 1e6, "launch_shape": SHAPE_NAMES[tune["shape"]]})
        del item, s0, kl, mesh
        torch.cuda.empty_cache()
    return out


def size_effect_leg(sizes=(50, 100, 200, 400), samples=32):
    """The statistical size-effect sweep to full length: geometrically similar
    notched beams of depth D = 50 / 100 / 200 / 400 mm (span 3 D, length
    3.5 D, thickness 50 mm, notch 0.2 D, dx = 2.5 mm), the cracking load at the
    level-1 rate for 8000 D / 50 steps (the load-pad displacement at the end
    grows with D), 32 lognormal-field samples per size (seed 4, stream = size
    index), batched FP32.  Per size: the mean and coefficient of variation of
    the nominal strength sigma_N = 3 P S / (2 b D^2) (the modulus of rupture of
    the peak load P; S span, b thickness).  The largest beam runs its samples
    in groups of 8 (bit-identical per sample), each group a progress line."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2212_04415_amd import beam as B
    sweep = [c for c in W.configs(fracture=True) if c.name == "size_sweep"][0]
    out = []
    for i, lv in enumerate(sweep.levels):
        D_mm = round(lv.beam.depth * 1e3)
        if D_mm not in sizes:
            continue
        mesh = B.Mesh.for_level(lv)
        kl = B.KL(mesh, W.FIELD_CORR_LEN, W.FIELD_MODES, 256)
        xi = torch.tensor(W.kl_coefficients(sweep.seed, samples, stream=i))
        group = samples if D_mm <= 200 else 8
        Q, ns, wall = [], [], 0.0
        for g0 in range(0, samples, group):
            s0 = kl.lognormal(xi[g0:g0 + group], W.S0_MEAN, W.FIELD_COV, dtype=torch.float32)
            torch.cuda.synchronize()
            t = time.perf_counter()
            q, n, st = B.run_batch([B.BatchItem(mesh, B.make_params(lv), group, s0)])[0]
            torch.cuda.synchronize()
            wall += time.perf_counter() - t
            assert int(st.abs().sum()) == 0
            Q.append(q.cpu().numpy())
            ns.append(n.cpu().numpy())
            print(f"[bench] size effect D = {D_mm} mm: samples {g0}..{g0 + group - 1} done ({wall:.1f} s)",
                  file=sys.stderr, flush=True)
            del s0
        Q, ns = np.concatenate(Q), np.concatenate(ns)
        b, D, S = lv.beam.thickness, lv.beam.depth, lv.beam.span
        sig = 3.0 * Q * S / (2.0 * b * D * D) / 1e6
        out.append({"depth_mm": D_mm, "nodes": mesh.n_nodes, "bonds": mesh.n_bonds, "samples": samples,
                    "time_steps": lv.n_steps, "load_per_step_mm": lv.du * 1e3, "wall_s": wall,
                    "bond_updates_per_s": mesh.n_bonds * lv.n_steps * samples / wall,
                    "peak_load_mean_N": float(Q.mean()),
                    "sigma_N_mean_MPa": float(sig.mean()), "sigma_N_cov": float(sig.std(ddof=1) / sig.mean()),
                    "peak_step_mean": float(ns.mean()), "peak_step_min": int(ns.min()), "peak_step_max": int(ns.max())})
        del kl, mesh
        torch.cuda.empty_cache()
    return out


def plane_leg(samples=(2152, 567, 204, 67, 18), notched=True, eps_s=10.0):
    """The paper's own case: the plane-stress Specimen 3 (350 x 100 mm,
    t = 50 mm, half-notched) on the five levels of its Table discretisation
    (350 ... 89,600 nodes), the paper's material model (exponential
    covariance on the plane, Weibull strength, fib relations), every level-l
    sample paired with a coarse solve on the same coefficients, one batched
    FP32 call.  The sample counts are the paper's allocation for this
    specimen at a sampling tolerance of 10 N (section 6.2).  notched=False:
    the unnotched specimen of case study 2 (section 6.3)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2212_04415_amd import mlmc
    levels = [W.level2d(l, notched=notched) for l in range(len(samples))]
    out = mlmc.coupled_batch(levels, list(samples), seed=5, precision="f32", corr_len=20e-3,
                             n_modes=W.FIELD_MODES, mean=W.S0_MEAN, cov=W.FIELD_COV,
                             kl_coefficients=W.kl_coefficients, field_model="paper")
    bu = sum(b * n * st for b, n, st in zip(out["bonds"], out["solves"], out["steps"]))
    L = len(samples)
    fine = [torch.tensor(out["Q"][l][:samples[l]], device="cuda") for l in range(L)]
    coarse = [None] + [torch.tensor(out["Q"][l - 1][samples[l - 1]:samples[l - 1] + samples[l]], device="cuda")
                       for l in range(1, L)]
    u = [0.05, 0.5, 0.95]
    quant = mlmc.cdf(fine, coarse, u)
    # standard Monte Carlo at the same sampling tolerance (Eq. MC_num_samples):
    # N = V[Q_L] / eps_s^2 solves of the finest level, V from its fine samples
    qL = np.asarray(out["Q"][L - 1][:samples[L - 1]])
    n_mc = float(np.var(qL, ddof=1)) / eps_s ** 2
    mc_cost = n_mc * out["bonds"][L - 1] * out["steps"][L - 1]
    return {"workload": "specimen3_plane_stress_paper_material" + ("" if notched else "_unnotched"),
            "nodes": out["nodes"], "bonds": out["bonds"], "solves_per_level_fine": list(samples),
            "mc_equivalent": {"eps_s_N": eps_s, "N": n_mc, "bond_updates": mc_cost,
                              "mlmc_bond_updates": bu, "cost_ratio_mc_over_mlmc": mc_cost / bu},
            "steps": out["steps"], "solves_per_level": out["solves"], "wall_s": out["wall_s"],
            "bond_updates_per_s": bu / out["wall_s"], "mlmc_samples_per_s": sum(samples) / out["wall_s"],
            "estimate_N": out["estimate"], "sampling_std_N": max(out["sampling_variance"], 0.0) ** 0.5,
            "level_mean_var": [[m, v] for m, v, _ in out["levels"]],
            "multilevel_quantiles_N": {str(k): float(v) for k, v in zip(u, quant)}}


def plane_adaptive_leg(eps=50.0, n_warm=100):
    """Algorithm 1 on the plane-stress Specimen 3 (five levels, the paper's
    material model, 100 warm-up samples per level as in the paper, refinement
    ratio 4 between 2D levels, fitted alpha) at RMSE target eps (N)."""
    import workloads as W
    from paper_2212_04415_amd import mlmc
    levels = [W.level2d(l) for l in range(5)]
    run, costs, dofs = mlmc.solver_sampler(levels, seed=6, precision="f32", corr_len=20e-3, n_modes=W.FIELD_MODES,
                                           mean=W.S0_MEAN, cov=W.FIELD_COV, kl_coefficients=W.kl_coefficients,
                                           field_model="paper")
    out = mlmc.adaptive(run, eps, costs, dofs, n_warm=n_warm, alpha=None, alpha_default=0.5, refinement=4.0)
    return {"eps_N": eps, "levels_used": out["L"] + 1, "converged": out["converged"], "N": out["N"],
            "estimate_N": out["estimate"], "sampling_std_N": max(out["sampling_variance"], 0.0) ** 0.5,
            "bias_estimate_N": out["bias"], "alpha_fitted": out["history"][-1]["alpha"],
            "level_means_N": [m for m, _, _ in out["levels"]],
            "wall_s": out["wall_s"], "bond_updates_per_s": out["cost"] / out["wall_s"],
            "mlmc_samples_per_s": sum(out["N"]) / out["wall_s"]}


def adjoint_leg(oracle_steps=400):
    """The gradient workload: level 1, one lognormal-field sample (seed 3),
    the cracking load with the exponential-linear law, 8000 steps,
    checkpoints every 200.  Wall time of pd_qoi_grad (peak, dQ/ds0 and dQ/dc)
    in FP64 and FP32 beside the forward solve alone (pd_run), and the
    oracle's discrete adjoint (C, all host threads) over the first
    oracle_steps steps of the same sample, with its per-step time scaled to
    the full run (labelled as such)."""
    import numpy as np
    import torch
    import workloads as W
    from oracle import solver as S
    from paper_2212_04415_amd import beam as B
    from paper_2212_04415_amd import pd
    lv = W.level(1, fracture=True, law=W.LAW_EXPLIN)
    mesh = B.Mesh.for_level(lv)
    kl = B.KL(mesh, W.FIELD_CORR_LEN, W.FIELD_MODES, 256)
    s0 = kl.lognormal(torch.tensor(W.kl_coefficients(3, 1)), W.S0_MEAN, W.FIELD_COV, dtype=torch.float64)[0]
    out = {"workload": "level-1 beam, 1 sample, 8000 steps, checkpoints every 200", "steps": lv.n_steps}
    for prec in ("f64", "f32"):
        p = B.make_params(lv, precision=prec, checkpoint_every=200)
        mesh.set_field(pd.PD_FIELD_S0, s0.cpu().numpy())
        B.run(mesh, B.make_params(lv, precision=prec, n_steps=64))      # tunes the launch shape
        torch.cuda.synchronize()
        t = time.perf_counter()
        fwd = B.run(mesh, p)
        forward_s = time.perf_counter() - t
        mesh.set_field(pd.PD_FIELD_S0, None)
        t = time.perf_counter()
        g = B.qoi_grad(mesh, p, s0=s0, as_tensors=True)
        torch.cuda.synchronize()
        grad_s = time.perf_counter() - t
        out[prec] = {"grad_s": grad_s, "forward_s": forward_s, "grad_over_forward": grad_s / forward_s,
                     "peak_N": g["Q"], "nstar": g["nstar"], "forward_peak_N": fwd["Q"],
                     "dQ_ds0_norm": float(torch.linalg.vector_norm(g["dQ_ds0"])),
                     "dQ_dc_norm": float(torch.linalg.vector_norm(g["dQ_dc"]))}
    threads = host_threads()
    S.set_threads(threads)
    prob = S.beam_problem(lv, s0=s0.cpu().numpy(), n_steps=oracle_steps)
    t = time.perf_counter()
    prob.run(want_state=False)
    fwd_s = time.perf_counter() - t
    t = time.perf_counter()
    a = prob.adjoint()
    adj_s = time.perf_counter() - t
    # the oracle's adjoint is one forward sweep over every step (trajectory
    # kept) and one backward sweep from the peak step down to step 0
    back_per_step = max(adj_s - fwd_s, 0.0) / max(a["nstar"], 1)
    nstar = out["f64"]["nstar"]
    out["oracle"] = {"steps": oracle_steps, "threads": threads, "cpu_model": cpu_model(),
                     "forward_s": fwd_s, "adjoint_s": adj_s, "adjoint_nstar": a["nstar"],
                     "estimated_full_s": fwd_s / oracle_steps * lv.n_steps + back_per_step * nstar,
                     "note": f"estimate: forward and backward per-step times of the first {oracle_steps} (elastic) "
                             f"steps, times {lv.n_steps} forward and {nstar} backward steps"}
    out["f64"]["speedup_vs_oracle_estimate"] = out["oracle"]["estimated_full_s"] / out["f64"]["grad_s"]
    return out


def cost_curve_leg(eps_list=(100.0, 50.0, 25.0, 10.0 * 2 ** 0.5), n_warm=100):
    """Cost of the adaptive estimator against the RMSE target (the last one
    splits into the paper's 10 N sampling tolerance) on the plane-stress
    Specimen 3 (paper's material model, five levels), in bond
    updates and seconds, beside the cost standard MC would need at the same
    sampling tolerance: N = V[Q] / eps_s^2 finest-level solves (Eq.
    MC_num_samples), with V[Q] taken as the level-0 variance.  The slopes
    are least-squares fits of log cost against log eps."""
    import numpy as np
    import workloads as W
    from paper_2212_04415_amd import mlmc
    levels = [W.level2d(l) for l in range(5)]
    run, costs, dofs = mlmc.solver_sampler(levels, seed=6, precision="f32", corr_len=20e-3, n_modes=W.FIELD_MODES,
                                           mean=W.S0_MEAN, cov=W.FIELD_COV, kl_coefficients=W.kl_coefficients,
                                           field_model="paper")
    fine_cost = costs[-1] - costs[-2]          # one finest-level solve alone
    rows = []
    for eps in eps_list:
        out = mlmc.adaptive(run, eps, costs, dofs, n_warm=n_warm, alpha=None, alpha_default=0.5, refinement=4.0)
        v0 = out["levels"][0][1]
        n_mc = v0 / out["eps_s"] ** 2
        rows.append({"eps_N": eps, "levels_used": out["L"] + 1, "converged": out["converged"], "N": out["N"],
                     "mlmc_bond_updates": out["cost"], "mlmc_wall_s": out["wall_s"],
                     "mc_solves": n_mc, "mc_bond_updates": n_mc * fine_cost,
                     "estimate_N": out["estimate"], "bias_estimate_N": out["bias"]})
    le = np.log([r["eps_N"] for r in rows])
    slope = lambda key: float(np.polyfit(le, np.log([r[key] for r in rows]), 1)[0])
    return {"rows": rows, "mlmc_cost_exponent": slope("mlmc_bond_updates"),
            "mc_cost_exponent": slope("mc_bond_updates")}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed batch solves")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the plain FP64 and cracking-load legs")
    ap.add_argument("--no-mlmc", action="store_true",
                    help="skip the three-level MLMC hierarchy (1024/128/16 samples + coupled partners), "
                         "which the default run times")
    ap.add_argument("--mlmc-literal", action="store_true",
                    help="also run the MLMC hierarchy on the literal (elastic) load")
    ap.add_argument("--mlmc-paper", action="store_true",
                    help="also run the MLMC hierarchy with the paper's material model (exponential covariance, "
                         "Weibull strength, fib relations)")
    ap.add_argument("--adaptive", action="store_true",
                    help="also run the adaptive MLMC algorithm on the three levels (RMSE target 80 N)")
    ap.add_argument("--sweep", action="store_true",
                    help="also time the size-sweep beams (D = 50..400 mm, 32 samples, first 1000 steps)")
    ap.add_argument("--size-effect", action="store_true",
                    help="also run the size-effect sweep to full length (D = 50..400 mm, cracking load, 32 samples "
                         "each; about 10 minutes) and report the mean and CoV of the nominal strength per size")
    ap.add_argument("--sizes", default="50,100,200,400", help="depths (mm) of the size-effect sweep")
    ap.add_argument("--plane", action="store_true",
                    help="also run the plane-stress Specimen-3 MLMC hierarchy (five levels, paper material model)")
    ap.add_argument("--plane-unnotched", action="store_true",
                    help="also run the unnotched Specimen-3 hierarchy (case study 2) with the paper's allocation at a "
                         "50 N sampling tolerance (1624/479/230/63/22 samples)")
    ap.add_argument("--plane-adaptive", action="store_true",
                    help="also run the adaptive MLMC algorithm on the plane-stress Specimen 3 (RMSE target 50 N)")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time the gradient (pd_qoi_grad, FP64 and FP32) on the level-1 sample beside the "
                         "forward solve and the oracle's adjoint")
    ap.add_argument("--cost-curve", action="store_true",
                    help="also run the adaptive MLMC on the plane-stress Specimen 3 at eps = 100 / 50 / 25 / 14.1 N "
                         "(the last: a 10 N sampling tolerance, as in the paper's allocation table)")
    ap.add_argument("--time-steps", type=int, default=None,
                    help="profiling only: time steps per batch solve (default: the workload's 8000)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="profiling only: run a plain 1 GiB device copy (for scaling HBM counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the batched solve runs on a single MI355X and this build "
              "has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    from paper_2212_04415_amd import beam as B
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")     # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4}))
        return

    S = 64
    lv = W.level(1)
    if args.time_steps:
        import dataclasses
        lv = dataclasses.replace(lv, n_steps=args.time_steps)
    mesh = B.Mesh.for_level(lv)
    kl = B.KL(mesh, W.FIELD_CORR_LEN, W.FIELD_MODES, 256)
    xi = torch.tensor(W.kl_coefficients(1, S), dtype=torch.float64)
    s0 = kl.lognormal(xi, W.S0_MEAN, W.FIELD_COV, dtype=torch.float32)
    params = B.make_params(lv, precision="f32", accumulate="kahan")
    item = B.BatchItem(mesh, params, S, s0)
    tune = B.autotune(mesh, params, S)       # the choice run_batch then uses

    for _ in range(args.warmup):
        B.run_batch([item])
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        outs = B.run_batch([item], stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    Q = outs[0][0].cpu().numpy()
    assert np.all(np.isfinite(Q)) and int(outs[0][2].abs().sum()) == 0

    bond_updates = mesh.n_bonds * lv.n_steps * S
    value = bond_updates * args.steps / wall
    launches = lv.n_steps * args.steps
    avg_launch_s = gpu_s / launches
    alg_bytes_per_launch = ALG_BYTES_PER_BOND_UPDATE_F32 * mesh.n_bonds * S
    achieved_gbps = alg_bytes_per_launch / avg_launch_s / 1e9
    flops_per_launch = 2 * mesh.n_bonds * S * FLOPS_PER_BOND_DIR_F32
    achieved_tflops = flops_per_launch / avg_launch_s / 1e12
    kernel = SHAPE_KERNELS[tune["shape"]]
    traffic = traffic_from_profiles(kernel)

    line = {
        "metric": "bond-updates/s and MLMC samples/s on 1 MI355X, batched FP32 vs plain FP64 at equal QoI error",
        "value": value,
        "unit": "bond-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched_fp32_L1x64", "nodes": mesh.n_nodes, "bonds": mesh.n_bonds,
                   "samples": S, "time_steps": lv.n_steps, "dx_mm": lv.dx * 1e3,
                   "field": "lognormal KL, 50 modes, l=20 mm, CoV 0.2, seed 1",
                   "load_per_step_mm": lv.du * 1e3, "accumulation": "kahan", "reaction": "f64"},
        "samples_per_s": S * args.steps / wall,
        "time_step_us": avg_launch_s * 1e6,
        "roofline": {"bound": "hbm", "achieved": achieved_gbps, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": achieved_gbps / PEAK_HBM_GBPS, "traffic": traffic, "kernel": kernel,
                     "avg_launch_us": avg_launch_s * 1e6,
                     "algorithmic_bytes_per_bond_update": ALG_BYTES_PER_BOND_UPDATE_F32,
                     "algorithmic_bytes_per_launch": alg_bytes_per_launch,
                     "bond_updates_per_launch": mesh.n_bonds * S,
                     "measured_hbm": None if traffic is None else {
                         "bytes_per_launch": traffic, "GBps": traffic / avg_launch_s / 1e9,
                         "frac_of_peak": traffic / avg_launch_s / 1e9 / PEAK_HBM_GBPS},
                     "valu_extra": {"flops_per_launch": flops_per_launch, "TFLOPs": achieved_tflops,
                                    "peak_fp32_vector_TFLOPs": PEAK_TFLOPS_F32,
                                    "frac": achieved_tflops / PEAK_TFLOPS_F32}},
        "launch_shape": {"chosen": SHAPE_NAMES[tune["shape"]],
                         "autotune_us_per_step": {n: float(t) for n, t in zip(SHAPE_NAMES, tune["us_per_step"])}},
    }

    if not args.no_extras:
        # plain per-sample FP64 solve of sample 0's field
        p64 = B.make_params(lv, precision="f64")
        mesh.set_field(0, s0[0].double().cpu().numpy())
        B.run(mesh, B.make_params(lv, precision="f64", n_steps=64))
        torch.cuda.synchronize()
        t = time.perf_counter()
        r64 = B.run(mesh, p64)
        dt64 = time.perf_counter() - t
        mesh.set_field(0, None)
        line["plain_fp64"] = {"samples_per_s": 1.0 / dt64, "bond_updates_per_s": mesh.n_bonds * lv.n_steps / dt64,
                              "peak_rel_diff_vs_batched_sample0": abs(r64["Q"] - float(Q[0])) / abs(r64["Q"])}
        line["speedup_vs_plain_fp64"] = line["samples_per_s"] / line["plain_fp64"]["samples_per_s"]
        # the same 64 samples batched in FP64: splits the speed-up into the gain
        # of batching and the gain of FP32 with compensation
        s064 = s0.double()
        B.run_batch([B.BatchItem(mesh, B.make_params(lv, precision="f64", n_steps=64), S, s064)])
        torch.cuda.synchronize()
        t = time.perf_counter()
        o64 = B.run_batch([B.BatchItem(mesh, p64, S, s064)])
        torch.cuda.synchronize()
        dtb = time.perf_counter() - t
        q64 = o64[0][0].cpu().numpy()
        line["batched_fp64"] = {"samples_per_s": S / dtb, "bond_updates_per_s": mesh.n_bonds * lv.n_steps * S / dtb,
                                "peak_max_rel_diff_vs_batched_fp32": float(np.max(np.abs(q64 - Q) / np.abs(q64)))}
        # cracking-load variant (400x the literal increment): damage localises
        lvf = W.level(1, fracture=True)
        itf = B.BatchItem(mesh, B.make_params(lvf), S, s0)
        B.run_batch([itf])
        torch.cuda.synchronize()
        t = time.perf_counter()
        of = B.run_batch([itf])
        torch.cuda.synchronize()
        dtf = time.perf_counter() - t
        qf = of[0][0].cpu().numpy()
        line["fracture_variant"] = {"bond_updates_per_s": mesh.n_bonds * lvf.n_steps * S / dtf,
                                    "samples_per_s": S / dtf, "peak_mean_N": float(qf.mean()),
                                    "peak_cov": float(qf.std() / qf.mean()),
                                    "load_per_step_mm": lvf.du * 1e3}

    def leg(key, fn, *fargs, **fkw):
        t = time.perf_counter()
        line[key] = fn(*fargs, **fkw)
        print(f"[bench] {key} done in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)

    print("[bench] headline done", file=sys.stderr, flush=True)
    if not args.no_mlmc:
        leg("mlmc_hierarchy", mlmc_leg, fracture=True)
        line["mlmc_samples_per_s"] = line["mlmc_hierarchy"]["mlmc_samples_per_s"]
    if args.mlmc_literal:
        leg("mlmc_hierarchy_literal", mlmc_leg, fracture=False)
    if args.mlmc_paper:
        leg("mlmc_hierarchy_paper_material", mlmc_leg, fracture=True, field_model="paper")
    if args.adaptive:
        leg("mlmc_adaptive", adaptive_leg)
    if args.sweep:
        leg("size_sweep", sweep_leg)
    if args.size_effect:
        leg("size_effect", size_effect_leg, sizes=tuple(int(x) for x in args.sizes.split(",")))
    if args.plane:
        leg("plane_stress_mlmc", plane_leg)
    if args.plane_unnotched:
        leg("plane_stress_mlmc_unnotched", plane_leg, samples=(1624, 479, 230, 63, 22), notched=False, eps_s=50.0)
    if args.plane_adaptive:
        leg("plane_stress_mlmc_adaptive", plane_adaptive_leg)
    if args.cost_curve:
        leg("plane_stress_cost_curve", cost_curve_leg)
    if args.adjoint:
        leg("adjoint", adjoint_leg)

    if not args.no_cpu_baseline:
        leg("cpu_baseline", cpu_baseline)

    print(json.dumps(finite_json(line)), flush=True)


if __name__ == "__main__":
    main()
