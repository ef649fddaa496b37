"""MLMC drivers (paper section 4): a fixed hierarchy in one batched solve,
and the adaptive algorithm (section 4.3, Algorithm 1).

Fixed hierarchy (section 4.2).

Level l contributes Y_0 = Q_0 and Y_l = Q_l - Q_{l-1} for l > 0, where both
terms of a difference are evaluated on the same random input (the same KL
coefficients, evaluated at each level's node centres).  All samples of all
levels — the level-l samples and the coarse partners of level l+1's pairs,
which live on the level-l mesh — run in a single pd_run_batch call (one
launch per time tick over every active work item), and the FP64 level sums
and the estimator come from pd_level_stats / pd_mlmc_estimate.  Argument
marshalling only."""
from __future__ import annotations

import ctypes as C
import dataclasses
import json
import os
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import beam as B
from . import pd


class SampleFailure(RuntimeError):
    """Samples that failed (PD_ENONFINITE / PD_EUNSTABLE) and failed again
    when re-run; .failed lists (item, sample, status) triples."""

    def __init__(self, failed):
        super().__init__("samples failed after re-running in FP64: " +
                         ", ".join(f"item {i} sample {k} (status {st})" for i, k, st in failed))
        self.failed = failed


def run_batch_requeue(items: Sequence, stream=None, run=None):
    """B.run_batch with per-sample failure handling.  The samples are
    independent, so a sample whose status is not PD_OK is simply run again:
    every failed sample of every item goes into one more batch, with its own
    field rows and the item's parameters at FP64 precision, and its peak,
    step and status replace the failed ones.  Returns (outs, requeued) with
    requeued a list of (item, sample) pairs; raises SampleFailure if a
    re-run sample fails too.  run(items, stream) defaults to B.run_batch."""
    run = B.run_batch if run is None else run
    outs = run(items, stream=stream)
    bad = [(i, (o[2] != 0).nonzero().flatten()) for i, o in enumerate(outs)]
    bad = [(i, idx) for i, idx in bad if idx.numel() > 0]
    if not bad:
        return outs, []
    retry = []
    for i, idx in bad:
        it = items[i]
        p = pd.pd_params()
        C.memmove(C.byref(p), C.byref(it.params), C.sizeof(p))
        p.precision = pd.PD_FP64
        rows = {f: (None if getattr(it, f) is None else getattr(it, f)[idx].contiguous()) for f in ("s0", "c", "gf")}
        retry.append(dataclasses.replace(it, params=p, n_samples=int(idx.numel()), **rows))
    again = run(retry, stream=stream)
    failed = []
    for (i, idx), o in zip(bad, again):
        for k in range(len(outs[i])):
            outs[i][k][idx] = o[k].to(outs[i][k].dtype)
        for j, st in zip(idx.tolist(), o[2].tolist()):
            if st != 0:
                failed.append((i, j, st))
    if failed:
        raise SampleFailure(failed)
    return outs, [(i, j) for i, idx in bad for j in idx.tolist()]


def coupled_batch(levels: Sequence, samples: Sequence[int], seed: int, *, precision: str = "f32",
                  corr_len: float, n_modes: int, mean: float, cov: float, kl_coefficients,
                  n_quad: int = 256, stream=None, field_model: str = "lognormal"):
    """Runs the hierarchy.  kl_coefficients(seed, n, n_modes, stream) supplies
    the seeded standard normals; level l uses stream l.  field_model
    "lognormal": lognormal limit stretch (mean, cov) from the separable
    squared-exponential KL basis of each level; "paper": the exponential-
    covariance basis of the level-0 mesh extended to every level, mapped to
    per-node s0, c and fracture energy by the Weibull / fib model (mean and
    cov unused).  Returns a dict with per-level Y and Q arrays, the estimate,
    sampling variance, per-level (mean, var, var_unbiased), and the batch's
    wall time."""
    import torch
    L = len(levels)
    meshes = [B.Mesh.for_level(lv) for lv in levels]
    if field_model == "lognormal":
        kls = [B.KL(m, corr_len, n_modes, n_quad) for m in meshes]
    elif field_model == "paper":
        base = B.KL.exponential(meshes[0], corr_len, n_modes)
        kls = [base] + [base.extend(m) for m in meshes[1:]]
        n_modes = base.n_modes
    else:
        raise ValueError(f"unknown field model {field_model!r}")
    xi = [torch.tensor(kl_coefficients(seed, samples[l], n_modes, stream=l)) for l in range(L)]
    dtype = torch.float32 if precision == "f32" else torch.float64
    items, params = [], []
    for l in range(L):
        rows = xi[l] if l + 1 == L else torch.cat([xi[l], xi[l + 1]])
        p = B.make_params(levels[l], precision=precision)
        params.append(p)
        if field_model == "lognormal":
            s0 = kls[l].lognormal(rows, mean, cov, dtype=dtype, stream=stream)
            items.append(B.BatchItem(meshes[l], p, rows.shape[0], s0))
        else:
            s0, c, gf = B.fib_fields(meshes[l], kls[l].gaussian(rows, stream=stream), dtype=dtype, stream=stream)
            items.append(B.BatchItem(meshes[l], p, rows.shape[0], s0, c, gf))
    torch.cuda.synchronize()
    t = time.perf_counter()
    outs, requeued = run_batch_requeue(items, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    Ys, sums = [], []
    for l in range(L):
        qf = outs[l][0][: samples[l]]
        qc = None if l == 0 else outs[l - 1][0][samples[l - 1]: samples[l - 1] + samples[l]]
        sums.append(B.level_stats(qf.contiguous(), None if qc is None else qc.contiguous(), stream=stream))
        Ys.append((qf - qc) if qc is not None else qf.clone())
    est = B.mlmc_estimate(sums, stream=stream)
    return dict(Q=[o[0].cpu().numpy() for o in outs], Y=[y.cpu().numpy() for y in Ys],
                sums=[s.cpu().numpy() for s in sums], estimate=est["estimate"],
                sampling_variance=est["sampling_variance"], levels=est["levels"], wall_s=wall,
                bonds=[m.n_bonds for m in meshes], nodes=[m.n_nodes for m in meshes],
                solves=[o[0].numel() for o in outs], steps=[lv.n_steps for lv in levels], requeued=requeued)


# ---------------------------------------------------------------- adaptive MLMC
def allocation(V, costs, eps_s):
    """pd_mlmc_allocation: (real N_l, N_l rounded down)."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    Cs = np.ascontiguousarray(costs, dtype=np.float64)
    real = np.zeros(V.size)
    n = np.zeros(V.size, dtype=np.int64)
    pd.pd_mlmc_allocation(V.ctypes.data, Cs.ctypes.data, V.size, float(eps_s), real.ctypes.data, n.ctypes.data)
    return real, n


def bias(y_last_mean, alpha, refinement=8.0, r=1.0):
    out = C.c_double()
    pd.pd_mlmc_bias(float(y_last_mean), float(alpha), float(refinement), float(r), C.byref(out))
    return out.value


def fit_rate(x, y):
    """pd_mlmc_fit_rate: (slope, intercept) of log|y| against log x."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    b, a = C.c_double(), C.c_double()
    pd.pd_mlmc_fit_rate(x.ctypes.data, y.ctypes.data, x.size, C.byref(b), C.byref(a))
    return b.value, a.value


def solver_sampler(levels: Sequence, seed: int, *, precision: str = "f32", corr_len: float, n_modes: int,
                   mean: float, cov: float, kl_coefficients, n_quad: int = 256, stream=None,
                   field_model: str = "lognormal"):
    """A sampler for `adaptive` backed by the batched solver: run(requests)
    with requests {level: (start, count)} runs, in one pd_run_batch call, the
    level-l samples start .. start+count-1 (KL coefficients of stream l) and,
    for l > 0, their coarse partners on the level l-1 mesh with the same
    coefficients, and returns {level: (q_fine, q_coarse or None)} as device
    FP64 tensors.  Also returns the per-sample costs (bond updates, fine plus
    coarse) and the node counts.  field_model as in coupled_batch."""
    import torch
    meshes = [B.Mesh.for_level(lv) for lv in levels]
    if field_model == "lognormal":
        kls = [B.KL(m, corr_len, n_modes, n_quad) for m in meshes]
    elif field_model == "paper":
        base = B.KL.exponential(meshes[0], corr_len, n_modes)
        kls = [base] + [base.extend(m) for m in meshes[1:]]
        n_modes = base.n_modes
    else:
        raise ValueError(f"unknown field model {field_model!r}")
    dtype = torch.float32 if precision == "f32" else torch.float64
    params = [B.make_params(lv, precision=precision) for lv in levels]
    work = [m.n_bonds * lv.n_steps for m, lv in zip(meshes, levels)]
    costs = [work[l] + (work[l - 1] if l > 0 else 0) for l in range(len(levels))]
    dofs = [3 * m.n_nodes for m in meshes]

    def item(l, xi, count):
        if field_model == "lognormal":
            return B.BatchItem(meshes[l], params[l], count, kls[l].lognormal(xi, mean, cov, dtype=dtype, stream=stream))
        s0, c, gf = B.fib_fields(meshes[l], kls[l].gaussian(xi, stream=stream), dtype=dtype, stream=stream)
        return B.BatchItem(meshes[l], params[l], count, s0, c, gf)

    def run(requests: Dict[int, Tuple[int, int]]):
        items, owners = [], []
        for l, (start, count) in sorted(requests.items()):
            xi = torch.tensor(kl_coefficients(seed, start + count, n_modes, stream=l)[start:])
            items.append(item(l, xi, count))
            owners.append((l, "fine"))
            if l > 0:
                items.append(item(l - 1, xi, count))
                owners.append((l, "coarse"))
        outs, requeued = run_batch_requeue(items, stream=stream)
        for i, j in requeued:
            l, kind = owners[i]
            run.requeued.append((l, kind, requests[l][0] + j))
        res: Dict[int, list] = {}
        for (l, kind), (Q, ns, st) in zip(owners, outs):
            res.setdefault(l, [None, None])[0 if kind == "fine" else 1] = Q
        return {l: (v[0], v[1]) for l, v in res.items()}

    run.requeued = []    # (level, "fine" | "coarse", sample index) of every re-run sample

    return run, costs, dofs


def adaptive(run: Callable, eps: float, costs: Sequence[float], dofs: Sequence[float], *, n_warm: int = 100,
             alpha=None, alpha_default: float = 0.5, refinement: float = 8.0, r: float = 1.0, max_levels=None,
             stream=None, journal: Optional[str] = None, journal_tag=None):
    """Adaptive MLMC, Algorithm 1.  run({level: (start, count)}) returns
    {level: (q_fine, q_coarse or None)} device FP64 tensors (see
    solver_sampler); costs[l] is the cost of one level-l sample and dofs[l]
    its degrees of freedom.  The RMSE budget eps is split evenly between the
    sampling error (eps_s = eps / sqrt 2, Eq. sampling_error) and the bias
    (eps_b = eps / sqrt 2, Eq. bias_error).  Per iteration: warm-up samples
    on the new finest level, level variances (Eq. sample_variance) from the
    FP64 level sums, the optimal allocation (Eq. sample_allocation, rounded
    down), the additional samples of every level in one run() call, and the
    bias estimate of the finest level, with alpha fitted from |Y_hat_l|,
    l >= 1, when alpha is None and two such levels exist.  Stops when the
    bias estimate is below eps_b, or at the last level (converged False).

    journal: path of an append-only JSONL record of every sample (a header
    with journal_tag, costs, dofs, eps and n_warm, then one line per sample:
    level, index, Q_f, Q_c, cost).  Samples already in it are read back
    instead of being run, so a run restarted after an interruption replays
    the same decisions and ends with the same level sums and estimate,
    bit for bit, running only the samples the journal lacks.  A journal
    written for another configuration is refused."""
    import torch
    eps_s = eps_b = eps / np.sqrt(2.0)
    last = len(costs) - 1 if max_levels is None else max_levels - 1
    N: List[int] = []
    sums: List[np.ndarray] = []
    history = []
    wall = 0.0
    header = dict(kind="header", tag=journal_tag, costs=[float(c) for c in costs], dofs=[float(d) for d in dofs],
                  eps=float(eps), n_warm=int(n_warm))
    known = _read_journal(journal, header) if journal else {}
    sink = open(journal, "a") if journal else None
    if sink is not None and not known and sink.tell() == 0:
        _append(sink, [header])
    replayed = 0

    def take(requests):
        nonlocal wall, replayed
        torch.cuda.synchronize()
        t = time.perf_counter()
        # per level: the journal's prefix of the requested range, the rest run
        first = {}
        for l, c in requests.items():
            k = 0
            while k < c and (l, N[l] + k) in known:
                k += 1
            first[l] = k
        todo = {l: (N[l] + first[l], c - first[l]) for l, c in requests.items() if first[l] < c}
        got = run(todo) if todo else {}
        records = []
        for l, c in requests.items():
            old = [known[(l, N[l] + k)] for k in range(first[l])]
            replayed += len(old)
            qf = torch.tensor([r[0] for r in old], dtype=torch.float64, device="cuda")
            qc = torch.tensor([r[1] for r in old], dtype=torch.float64, device="cuda") if l > 0 else None
            if l in got:
                nf, nc = got[l]
                qf = torch.cat([qf, nf.to(torch.float64)])
                if l > 0:
                    qc = torch.cat([qc, nc.to(torch.float64)])
                hf = nf.cpu().tolist()
                hc = nc.cpu().tolist() if l > 0 else [None] * len(hf)
                for k, (a, b) in enumerate(zip(hf, hc)):
                    i = N[l] + first[l] + k
                    if (l, i) not in known:
                        known[(l, i)] = (a, b)
                        records.append(dict(level=l, i=i, q_f=a, q_c=b, cost=float(costs[l])))
            s = B.level_stats(qf.contiguous(), None if qc is None else qc.contiguous(), stream=stream)
            sums[l] += s.cpu().numpy()
            N[l] += c
        if sink is not None and records:
            _append(sink, records)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t

    def moments():
        dev = torch.tensor(np.stack(sums), dtype=torch.float64, device="cuda")
        return B.mlmc_estimate(list(dev), stream=stream)

    try:
        L = 0
        converged = False
        while True:
            N.append(0)
            sums.append(np.zeros(3))
            take({L: n_warm})
            est = moments()
            V = [max(lv[1], 0.0) for lv in est["levels"]]   # rounding can push Eq. sample_variance below 0
            _, n_hat = allocation(V, costs[:L + 1], eps_s)
            extra = {l: int(n_hat[l]) - N[l] for l in range(L + 1) if int(n_hat[l]) > N[l]}
            if extra:
                take(extra)
                est = moments()
            means = [lv[0] for lv in est["levels"]]
            if alpha is not None:
                a = alpha
            elif L >= 2:
                a = -fit_rate(dofs[1:L + 1], means[1:L + 1])[0]
            else:
                a = alpha_default
            # Eq. bias_error needs a positive rate; corrections that do not decay
            # (fitted alpha <= 0) leave the bias unbounded
            b = bias(means[L], a, refinement, r) if r * refinement ** a > 1.0 else float("inf")
            history.append(dict(L=L, V=list(V), n_hat=[int(v) for v in n_hat], N=list(N), alpha=a, bias=b))
            if b < eps_b:
                converged = True
                break
            if L == last:
                break
            L += 1
        est = moments()
    finally:
        if sink is not None:
            sink.close()
    return dict(L=L, N=N, sums=[tuple(x) for x in sums], estimate=est["estimate"],
                sampling_variance=est["sampling_variance"], levels=est["levels"], bias=history[-1]["bias"],
                converged=converged, history=history, eps_s=eps_s, eps_b=eps_b, wall_s=wall,
                cost=float(sum(n * c for n, c in zip(N, costs))), replayed=replayed)


def _append(f, records):
    """Appends JSON lines and forces them to disk (a record is either
    whole in the file or absent, up to a torn last line)."""
    f.write("".join(json.dumps(r) + "\n" for r in records))
    f.flush()
    os.fsync(f.fileno())


def _read_journal(path, header):
    """{(level, index): (q_f, q_c)} from a journal; a torn last line (an
    interrupted write) is dropped and cut from the file so that appends
    start on a fresh line.  Raises ValueError if the header differs."""
    if not os.path.exists(path):
        return {}
    with open(path, "rb") as f:
        data = f.read()
    lines = data.split(b"\n")
    keep = len(data)
    if lines[-1] != b"":          # no newline after the last line: torn
        keep -= len(lines[-1])
    lines = lines[:-1]
    out = {}
    for n, raw in enumerate(lines):
        try:
            rec = json.loads(raw)
        except ValueError:
            if n == len(lines) - 1:
                keep -= len(raw) + 1
                break
            raise ValueError(f"{path}: line {n + 1} is not JSON")
        if n == 0:
            if rec != json.loads(json.dumps(header)):
                raise ValueError(f"{path} was written for another configuration: {rec} != {header}")
            continue
        out[(int(rec["level"]), int(rec["i"]))] = (rec["q_f"], rec["q_c"])
    if keep < len(data):
        with open(path, "r+b") as f:
            f.truncate(keep)
    return out


# ---------------------------------------------------------------- multilevel CDF
def cdf(q_fine: Sequence, q_coarse: Sequence, u, x=None, stream=None):
    """pd_mlmc_cdf: multilevel inverse CDF at u (in (0, 1]) and, when x is
    given, the empirical CDF of those quantiles at x.  q_fine[l] / q_coarse[l]:
    device FP64 tensors of the level-l fine samples and their coarse partners
    (q_coarse[0] is ignored)."""
    L = len(q_fine)
    fine = (C.c_void_p * L)(*[q.data_ptr() for q in q_fine])
    coarse = (C.c_void_p * L)(*[None if l == 0 else q_coarse[l].data_ptr() for l in range(L)])
    n = np.array([q.numel() for q in q_fine], dtype=np.int64)
    for l in range(1, L):
        assert q_coarse[l].numel() == n[l]
    u = np.ascontiguousarray(u, dtype=np.float64)
    qs = np.zeros(u.size)
    xs = None if x is None else np.ascontiguousarray(x, dtype=np.float64)
    cs = None if x is None else np.zeros(xs.size)
    pd.pd_mlmc_cdf(fine, coarse, n.ctypes.data, L, u.ctypes.data, u.size, qs.ctypes.data,
                   None if xs is None else xs.ctypes.data, 0 if xs is None else xs.size,
                   None if cs is None else cs.ctypes.data, B._stream_ptr(stream))
    return (qs, cs) if x is not None else qs
