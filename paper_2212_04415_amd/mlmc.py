"""MLMC hierarchy in one batched solve (paper section 4.2).

Level l contributes Y_0 = Q_0 and Y_l = Q_l - Q_{l-1} for l > 0, where both
terms of a difference are evaluated on the same random input (the same KL
coefficients, evaluated at each level's node centres).  All samples of all
levels — the level-l samples and the coarse partners of level l+1's pairs,
which live on the level-l mesh — run in a single pd_run_batch call (one
launch per time tick over every active work item), and the FP64 level sums
and the estimator come from pd_level_stats / pd_mlmc_estimate.  Argument
marshalling only."""
from __future__ import annotations

import time
from typing import List, Sequence

import numpy as np

from . import beam as B


def coupled_batch(levels: Sequence, samples: Sequence[int], seed: int, *, precision: str = "f32",
                  corr_len: float, n_modes: int, mean: float, cov: float, kl_coefficients,
                  n_quad: int = 256, stream=None):
    """Runs the hierarchy.  kl_coefficients(seed, n, n_modes, stream) supplies
    the seeded standard normals; level l uses stream l.  Returns a dict with
    per-level Y and Q arrays, the estimate, sampling variance, per-level
    (mean, var, var_unbiased), and the batch's wall time."""
    import torch
    L = len(levels)
    meshes = [B.Mesh.for_level(lv) for lv in levels]
    kls = [B.KL(m, corr_len, n_modes, n_quad) for m in meshes]
    xi = [torch.tensor(kl_coefficients(seed, samples[l], n_modes, stream=l)) for l in range(L)]
    dtype = torch.float32 if precision == "f32" else torch.float64
    items, params = [], []
    for l in range(L):
        rows = xi[l] if l + 1 == L else torch.cat([xi[l], xi[l + 1]])
        s0 = kls[l].lognormal(rows, mean, cov, dtype=dtype, stream=stream)
        p = B.make_params(levels[l], precision=precision)
        params.append(p)
        items.append(B.BatchItem(meshes[l], p, rows.shape[0], s0))
    torch.cuda.synchronize()
    t = time.perf_counter()
    outs = B.run_batch(items, stream=stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    for Q, ns, st in outs:
        if int(st.abs().sum()) != 0:
            raise RuntimeError("a sample went non-finite")
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
                solves=[o[0].numel() for o in outs], steps=[lv.n_steps for lv in levels])
