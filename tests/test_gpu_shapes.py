"""GPU: launch shapes and the autotuner.

Every launch shape of the step kernel maps the same per-node arithmetic onto
the GPU differently (brick of nodes per block, LDS tile or not), so a solve
must give bit-identical peak loads, displacements and damage histories
whichever shape runs it, and whatever the autotuner picks.  Parity of the
default shape with the oracle is in test_gpu_parity.py."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return t


@pytest.fixture(scope="module")
def B(torch):
    from paper_2212_04415_amd import beam
    return beam


@pytest.fixture(scope="module")
def pd(torch):
    from paper_2212_04415_amd import pd as p
    return p


def fields(M, S, seed):
    rng = np.random.default_rng(seed)
    return W.S0_MEAN * np.exp(0.2 * rng.standard_normal((S, M)))


@pytest.mark.parametrize("ell,steps_scale", [(0, 0.5), (1, 0.125)])
def test_every_shape_gives_identical_batch_results(B, pd, torch, ell, steps_scale):
    lv = W.level(ell, fracture=True, steps_scale=steps_scale)
    mesh = B.Mesh.for_level(lv)
    S = 5
    f = torch.tensor(fields(mesh.n_nodes, S, 11 + ell), device="cuda", dtype=torch.float32)
    p = B.make_params(lv)
    ref = None
    for shape in range(pd.PD_N_SHAPES):
        mesh.set_launch_shape(shape)
        Q, ns, st = B.run_batch([B.BatchItem(mesh, p, S, f)])[0]
        assert torch.all(st == 0)
        got = (Q.cpu().numpy(), ns.cpu().numpy())
        if ref is None:
            ref = got
            assert np.all(np.isfinite(ref[0]))
        else:
            assert np.array_equal(got[0], ref[0]), shape
            assert np.array_equal(got[1], ref[1]), shape
    mesh.set_launch_shape(pd.PD_SHAPE_AUTO)


def test_every_shape_gives_identical_state(B, pd):
    """Final displacements and the damage history of a cracked level-0 run."""
    lv = W.level(0, fracture=True, steps_scale=0.6)
    mesh = B.Mesh.for_level(lv)
    mesh.set_field(pd.PD_FIELD_S0, fields(mesh.n_nodes, 1, 3)[0])
    p = B.make_params(lv)
    ref = None
    for shape in range(pd.PD_N_SHAPES):
        mesh.set_launch_shape(shape)
        out = B.run(mesh, p, want_state=True)
        if ref is None:
            ref = out
            assert np.count_nonzero(out["kappa"]) > 100     # the run has damaged bonds
        else:
            assert out["Q"] == ref["Q"] and out["nstar"] == ref["nstar"], shape
            assert np.array_equal(out["u"], ref["u"]), shape
            assert np.array_equal(out["kappa"], ref["kappa"]), shape


def test_autotune_reports_every_usable_shape(B, pd):
    lv = W.level(1)
    mesh = B.Mesh.for_level(lv)
    r = B.autotune(mesh, B.make_params(lv), 8)
    us = r["us_per_step"]
    assert 0 <= r["shape"] < pd.PD_N_SHAPES
    assert np.all(us > 0)                       # FP32 + compensation can use every shape
    assert us[r["shape"]] == us.min()
    r64 = B.autotune(mesh, B.make_params(lv, precision="f64"), 1)
    assert r64["shape"] == pd.PD_SHAPE_GLOBAL_256
    assert r64["us_per_step"][pd.PD_SHAPE_GLOBAL_256] > 0
    assert np.all(np.delete(r64["us_per_step"], pd.PD_SHAPE_GLOBAL_256) == -1)


def test_unusable_pinned_shape_falls_back(B, pd, torch):
    """Uncompensated accumulation (the ablation) has the default brick and the
    global shape only; pinning another shape runs the default brick, with
    identical results."""
    lv = W.level(0, fracture=True, steps_scale=0.25)
    mesh = B.Mesh.for_level(lv)
    S = 3
    s0 = torch.tensor(fields(mesh.n_nodes, S, 7), device="cuda")
    p = B.make_params(lv, accumulate="plain")
    outs = []
    for shape in (pd.PD_SHAPE_LDS_16x4x4, pd.PD_SHAPE_LDS_8x8x4, pd.PD_SHAPE_GLOBAL_256):
        mesh.set_launch_shape(shape)
        Q, ns, st = B.run_batch([B.BatchItem(mesh, p, S, s0)])[0]
        assert torch.all(st == 0)
        outs.append(Q.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_every_shape_agrees_with_a_micromodulus_field(B, pd, torch):
    """With per-node s0 and c every launch shape gives the same peaks."""
    lv = W.level(0, fracture=True, steps_scale=0.25)
    mesh = B.Mesh.for_level(lv)
    S = 3
    rng = np.random.default_rng(5)
    s0 = torch.tensor(fields(mesh.n_nodes, S, 7), device="cuda")
    c = torch.tensor(np.exp(0.1 * rng.standard_normal((S, mesh.n_nodes))), device="cuda")
    p = B.make_params(lv)
    outs = []
    for shape in range(pd.PD_N_SHAPES):
        mesh.set_launch_shape(shape)
        Q, ns, st = B.run_batch([B.BatchItem(mesh, p, S, s0, c)])[0]
        assert torch.all(st == 0)
        outs.append((Q.cpu().numpy(), ns.cpu().numpy()))
    for q, n in outs[1:]:
        assert np.array_equal(q, outs[0][0]) and np.array_equal(n, outs[0][1])
