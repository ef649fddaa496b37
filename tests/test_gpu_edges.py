"""Degenerate and ragged cases of the time loop on the GPU against the
oracle: no time step at all, step counts that are not a multiple of the
captured chunk (1, 63, 65, 130), and a batch of single samples on two levels
whose step counts do not fill the batch graph's hyper-period."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import solver as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2212_04415_amd import beam as B
    return torch, B


def test_no_time_step_gives_no_peak(env):
    """With zero steps there is no reaction: the peak is -inf at step 0 on
    both sides (the maximum over an empty set)."""
    torch, B = env
    lv = dataclasses.replace(W.level(0), n_steps=0)
    ref = S.beam_problem(lv).run(want_state=False)
    assert ref["Q"] == -np.inf and ref["nstar"] == 0
    mesh = B.Mesh.for_level(lv)
    out = B.run(mesh, B.make_params(lv, precision="f64"))
    assert out["Q"] == -np.inf and out["nstar"] == 0
    (Q, ns, st), = B.run_batch([B.BatchItem(mesh, B.make_params(lv), 3)])
    assert torch.all(st == 0) and torch.all(torch.isneginf(Q)) and torch.all(ns == 0)


@pytest.mark.parametrize("n", [1, 63, 65, 130])
def test_ragged_step_counts_match_the_oracle(env, n):
    """Cracking-rate loading (fast enough that the reaction is non-zero from
    the first steps) for n steps: the FP64 reaction history, peak and step."""
    torch, B = env
    lv = dataclasses.replace(W.level(0, fracture=True), n_steps=n, du=2e-7)
    ref = S.beam_problem(lv).run(want_state=False)
    out = B.run(B.Mesh.for_level(lv), B.make_params(lv, precision="f64", record_history=True))
    assert np.allclose(out["R"], ref["R"], rtol=1e-9, atol=1e-9 * np.max(np.abs(ref["R"])))
    assert out["Q"] == pytest.approx(ref["Q"], rel=1e-9) and out["nstar"] == ref["nstar"]


def test_uneven_batch_of_single_samples(env):
    """One sample on level 0 (37 steps) and one on level 1 (23 steps, half
    the time step) in one batch: each equals its own single run bit for bit,
    although neither step count fills the batch graph's replay period."""
    torch, B = env
    l0 = dataclasses.replace(W.level(0, fracture=True), n_steps=37, du=2e-7)
    l1 = dataclasses.replace(W.level(1, fracture=True), n_steps=23, du=1e-7)
    m0, m1 = B.Mesh.for_level(l0), B.Mesh.for_level(l1)
    p0, p1 = B.make_params(l0), B.make_params(l1)
    outs = B.run_batch([B.BatchItem(m0, p0, 1), B.BatchItem(m1, p1, 1)])
    for mesh, p, (Q, ns, st) in ((m0, p0, outs[0]), (m1, p1, outs[1])):
        assert int(st[0]) == 0
        single = B.run(mesh, p)
        assert Q[0].item() == single["Q"] and ns[0].item() == single["nstar"]
    for lv, (Q, ns, st) in ((l0, outs[0]), (l1, outs[1])):
        ref = S.beam_problem(lv).run(want_state=False)
        assert Q[0].item() == pytest.approx(ref["Q"], rel=5e-3)


def test_batch_beyond_one_launch_is_refused(env):
    """65535 samples of the level-2 mesh would need 1.5e10 work-items in one
    step launch (more than a dispatch can count): refused with a message
    before anything is allocated; the library stays usable."""
    torch, B = env
    from paper_2212_04415_amd import pd
    lv = dataclasses.replace(W.level(2), n_steps=1)
    mesh = B.Mesh.for_level(lv)
    with pytest.raises(pd.PdError, match="exceed one launch"):
        B.run_batch([B.BatchItem(mesh, B.make_params(lv), 65535)])
    (Q, ns, st), = B.run_batch([B.BatchItem(mesh, B.make_params(lv), 2)])
    assert torch.all(st == 0)


def test_tick_schedule_equals_the_branch_schedule(env, monkeypatch):
    """A three-level batch (dt ratios 4 : 2 : 1, uneven step counts, lognormal
    limit-stretch fields) run with one launch per tick over all levels gives
    the graph-branch schedule's peaks, steps and final displacements bit
    for bit; so does a pair of levels with a micromodulus field."""
    torch, B = env
    lvs = [dataclasses.replace(W.level(l, fracture=True), n_steps=n, du=2e-7 / 2 ** l)
           for l, n in ((0, 90), (1, 170), (2, 333))]
    meshes = [B.Mesh.for_level(lv) for lv in lvs]
    g = torch.Generator("cuda").manual_seed(4)

    def field(mesh, S, scale):
        return scale * (1.0 + 0.1 * torch.randn((S, mesh.n_nodes), dtype=torch.float64, device="cuda",
                                                generator=g)).abs()

    s0 = [field(m, S, W.S0_MEAN) for m, S in zip(meshes, (5, 3, 2))]
    items = [B.BatchItem(m, B.make_params(lv), f.shape[0], f, want_u=True) for m, lv, f in zip(meshes, lvs, s0)]
    c = [field(m, 2, S.micromodulus(W.E_MODULUS, 3.14 * lv.dx)) for m, lv in zip(meshes[:2], lvs[:2])]
    items_c = [B.BatchItem(m, B.make_params(lv), 2, f[:2].contiguous(), cc)
               for m, lv, f, cc in zip(meshes[:2], lvs[:2], s0[:2], c)]
    ref = B.run_batch(items)
    ref_c = B.run_batch(items_c)
    monkeypatch.setenv("PD_BATCH_SCHEDULE", "tick")
    got = B.run_batch(items)
    got_c = B.run_batch(items_c)
    for a, b in zip(ref + ref_c, got + got_c):
        assert torch.all(a[2] == 0)
        for x, y in zip(a, b):
            assert torch.equal(x, y)


def test_runs_are_deterministic(env):
    """Run to run, the batched FP32 path (damage developing: 32 level-1
    samples on the cracking load for 3000 steps) repeats its peaks, peak
    steps and final displacements bit for bit, and the FP64 single-sample
    path its displacements and per-bond damage history: there are no atomics
    or scheduling-dependent sums anywhere in the step."""
    torch, B = env
    lv = dataclasses.replace(W.level(1, fracture=True), n_steps=3000)
    mesh = B.Mesh.for_level(lv)
    g = torch.Generator("cuda").manual_seed(12)
    s0 = W.S0_MEAN * (1.0 + 0.2 * torch.randn((32, mesh.n_nodes), dtype=torch.float64, device="cuda",
                                              generator=g)).abs()
    item = B.BatchItem(mesh, B.make_params(lv), 32, s0, want_u=True)
    runs = [B.run_batch([item])[0] for _ in range(3)]
    assert torch.all(runs[0][2] == 0)
    for other in runs[1:]:
        for x, y in zip(runs[0], other):
            assert torch.equal(x, y)
    l0 = dataclasses.replace(W.level(0, fracture=True), n_steps=2500)
    m0 = B.Mesh.for_level(l0)
    p = B.make_params(l0, precision="f64")
    a, b = (B.run(m0, p, want_state=True) for _ in range(2))
    assert np.count_nonzero(a["kappa"]) > 0
    assert np.array_equal(a["u"], b["u"]) and np.array_equal(a["kappa"], b["kappa"]) and a["Q"] == b["Q"]
