"""The batched MLMC hierarchy on the GPU: coupled pairs, FP64 level sums and
the estimator, against the oracle's solves and statistics."""
import concurrent.futures as cf

import numpy as np
import pytest

import workloads as W
from oracle import geometry as G
from oracle import kl as OKL
from oracle import mlmc as OM
from oracle import solver as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def run():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2212_04415_amd import mlmc
    levels = [W.level(0, fracture=True, steps_scale=0.25), W.level(1, fracture=True, steps_scale=0.25)]
    samples = [6, 3]
    out = mlmc.coupled_batch(levels, samples, seed=2, precision="f32", corr_len=W.FIELD_CORR_LEN,
                             n_modes=W.FIELD_MODES, mean=W.S0_MEAN, cov=W.FIELD_COV,
                             kl_coefficients=W.kl_coefficients)
    return levels, samples, out


def test_every_solve_matches_the_oracle(run):
    """Each fine sample and its coarse partner are re-solved by the oracle on
    the same KL coefficients (level 0: 6 samples + 3 partners, level 1: 3)."""
    levels, samples, out = run
    jobs = []
    for l, lv in enumerate(levels):
        ob = OKL.Basis3D((lv.beam.length, lv.beam.thickness, lv.beam.depth), W.FIELD_CORR_LEN, W.FIELD_MODES, 256)
        pos = G.node_positions(lv.shape, lv.dx)
        xi = W.kl_coefficients(2, samples[l], stream=l)
        if l + 1 < len(levels):
            xi = np.concatenate([xi, W.kl_coefficients(2, samples[l + 1], stream=l + 1)])
        fields = OKL.lognormal_field(ob, pos, xi, W.S0_MEAN, W.FIELD_COV)
        jobs += [(l, k, S.beam_problem(lv, s0=fields[k])) for k in range(xi.shape[0])]
    with cf.ThreadPoolExecutor(8) as ex:
        refs = list(ex.map(lambda j: j[2].run(want_state=False)["Q"], jobs))
    for (l, k, _), q in zip(jobs, refs):
        assert out["Q"][l][k] == pytest.approx(q, rel=5e-3), (l, k)


def test_level_statistics_and_estimator(run):
    levels, samples, out = run
    Y0 = out["Q"][0][:6]
    Y1 = out["Q"][1][:3] - out["Q"][0][6:9]
    assert np.array_equal(out["Y"][0], Y0) and np.allclose(out["Y"][1], Y1, rtol=0, atol=1e-12)
    est, var, per = OM.mlmc_estimate([Y0, Y1])
    assert out["estimate"] == pytest.approx(est, rel=1e-12)
    assert out["sampling_variance"] == pytest.approx(var, rel=1e-9)
    for (n, m, v), (gm, gv, gvu) in zip(per, out["levels"]):
        assert gm == pytest.approx(m, rel=1e-12)
        assert gv == pytest.approx(v, rel=1e-9, abs=1e-9)
        assert gvu == pytest.approx(v * n / (n - 1), rel=1e-9, abs=1e-9)
