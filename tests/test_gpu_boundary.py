"""Contract of the C ABI at its edges, on the GPU: material fields are
checked when they are set (and a rejected field leaves the old one in
place), a micromodulus field too stiff for the time step is refused by the
single-sample and gradient entry points and marks only its own sample in a
batch, a sample that goes non-finite away from the supports is flagged
although its reaction stays finite, and pd_run_batch returns before the
solve has finished (outputs in stream order, pd_batch_sync to wait)."""
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
    from paper_2212_04415_amd import pd
    return torch, B, pd


def c_ref(lv):
    return S.micromodulus(W.E_MODULUS, 3.14 * lv.dx)


def mid_top_node(mesh, lv):
    """A node at mid-span near the top face (far from both supports)."""
    nx, ny, nz = lv.shape
    return (nx // 2) + nx * (ny // 2 + ny * (nz - 2))


def test_rejected_field_keeps_the_old_one(env):
    """A micromodulus field with a NaN, a zero, a negative or an infinite
    value is refused with PD_EINVAL (host and device values); the field set
    before stays in force and the run reproduces its result bit for bit.
    FP32 device values pass the same check, and clearing the field brings
    back the homogeneous result."""
    torch, B, pd = env
    lv = dataclasses.replace(W.level(0, fracture=True), n_steps=200)
    mesh = B.Mesh.for_level(lv)
    rng = np.random.default_rng(5)
    good = c_ref(lv) * (0.9 + 0.2 * rng.random(mesh.n_nodes))
    p = B.make_params(lv, precision="f64")
    plain = B.run(mesh, p)
    mesh.set_field(pd.PD_FIELD_C, good)
    ref = B.run(mesh, p)
    assert ref["Q"] != plain["Q"]
    for bad_value in (np.nan, -1e-4, 0.0, np.inf):
        bad = good.copy()
        bad[17] = bad_value
        with pytest.raises(pd.PdError, match="positive and finite") as ei:
            mesh.set_field(pd.PD_FIELD_C, bad)
        assert ei.value.code == pd.PD_EINVAL
        dev = torch.tensor(bad[None, :], device="cuda")
        with pytest.raises(pd.PdError, match="positive and finite"):
            pd.pd_set_material_field(mesh.h, pd.PD_FIELD_C, 1, dev.data_ptr(), 1, pd.PD_DTYPE_F64, None)
        out = B.run(mesh, p)
        assert out["Q"] == ref["Q"] and out["nstar"] == ref["nstar"]
    dev32 = torch.tensor(good[None, :], dtype=torch.float32, device="cuda")
    pd.pd_set_material_field(mesh.h, pd.PD_FIELD_C, 1, dev32.data_ptr(), 1, pd.PD_DTYPE_F32, None)
    assert B.run(mesh, p)["Q"] == pytest.approx(ref["Q"], rel=1e-6)
    mesh.set_field(pd.PD_FIELD_C, None)
    assert B.run(mesh, p)["Q"] == plain["Q"]


def test_too_stiff_micromodulus_is_refused(env):
    """A micromodulus field 1e4 times c_ref at one node needs a time step
    100 times smaller: pd_run and pd_qoi_grad refuse it with PD_EUNSTABLE,
    while the same field scaled to c_ref runs."""
    torch, B, pd = env
    lv = dataclasses.replace(W.level(0, fracture=True), n_steps=40)
    mesh = B.Mesh.for_level(lv)
    c = np.full(mesh.n_nodes, c_ref(lv))
    p = B.make_params(lv, precision="f64")
    mesh.set_field(pd.PD_FIELD_C, c)
    ok = B.run(mesh, p)
    assert np.isfinite(ok["Q"])
    c[mid_top_node(mesh, lv)] *= 1e4
    mesh.set_field(pd.PD_FIELD_C, c)
    with pytest.raises(pd.PdError) as ei:
        B.run(mesh, p)
    assert ei.value.code == pd.PD_EUNSTABLE
    mesh.set_field(pd.PD_FIELD_C, None)
    c_dev = torch.tensor(c, device="cuda")
    with pytest.raises(pd.PdError, match="micromodulus") as ei:
        B.qoi_grad(mesh, p, c=c_dev)
    assert ei.value.code == pd.PD_EUNSTABLE
    assert np.isfinite(B.run(mesh, p)["Q"])


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_batch_marks_only_the_unstable_sample(env, precision):
    """In a batch of three samples the one whose micromodulus field is too
    stiff for dt gets PD_EUNSTABLE; the others run to the results they have
    in a batch without it, bit for bit."""
    torch, B, pd = env
    lv = dataclasses.replace(W.level(0, fracture=True), n_steps=48)
    mesh = B.Mesh.for_level(lv)
    p = B.make_params(lv, precision=precision)
    c = torch.full((3, mesh.n_nodes), c_ref(lv), dtype=torch.float64, device="cuda")
    c[1] *= 1.0 + 0.2 * torch.rand(mesh.n_nodes, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    (Qa, na, sa), = B.run_batch([B.BatchItem(mesh, p, 2, None, c[:2].contiguous())])
    c[2, mid_top_node(mesh, lv)] *= 1e4
    (Q, ns, st), = B.run_batch([B.BatchItem(mesh, p, 3, None, c)])
    assert st.tolist() == [pd.PD_OK, pd.PD_OK, pd.PD_EUNSTABLE]
    assert torch.equal(Q[:2], Qa) and torch.equal(ns[:2], na) and torch.all(sa == 0)


def test_non_finite_state_away_from_the_supports_is_flagged(env):
    """A NaN micromodulus at one mid-span node of one sample: the forces
    of step n are NaN within 3 (n + 1) cells of it, so after 4 steps the
    reaction at the supports (17 cells away) is still finite, yet the sample
    is flagged PD_ENONFINITE from its node states; the other sample is
    untouched."""
    torch, B, pd = env
    lv = dataclasses.replace(W.level(0, fracture=True), n_steps=4)
    mesh = B.Mesh.for_level(lv)
    nx, ny, _ = lv.shape

    def cell(n):
        n = np.asarray(n)
        return np.stack([n % nx, (n // nx) % ny, n // (nx * ny)], axis=-1)

    node = mid_top_node(mesh, lv)
    dist = np.linalg.norm(cell(mesh.support) - cell(node), axis=-1)
    assert np.min(dist) > 3 * (lv.n_steps + 1)
    p = B.make_params(lv, precision="f64")
    c = torch.full((2, mesh.n_nodes), c_ref(lv), dtype=torch.float64, device="cuda")
    (Q0, n0, s0), = B.run_batch([B.BatchItem(mesh, p, 1, None, c[:1].contiguous())])
    c[1, node] = float("nan")
    (Q, ns, st), = B.run_batch([B.BatchItem(mesh, p, 2, None, c)])
    assert st.tolist() == [pd.PD_OK, pd.PD_ENONFINITE]
    assert torch.isfinite(Q[1])
    assert Q[0] == Q0[0] and ns[0] == n0[0]


def test_batch_returns_before_the_solve_ends(env):
    """pd_run_batch enqueues the solve and returns: on a side stream the
    outputs equal those of a run on the current stream, bit for bit, once
    the current stream (joined by run_batch) has caught up; the inputs may
    be dropped right after the call; two batches in flight and
    pd_batch_sync give the same results again."""
    torch, B, pd = env
    lv = dataclasses.replace(W.level(1, fracture=True), n_steps=600)
    mesh = B.Mesh.for_level(lv)
    p = B.make_params(lv)
    g = torch.Generator("cuda").manual_seed(11)

    def field():
        return W.S0_MEAN * (1.0 + 0.1 * torch.randn((4, mesh.n_nodes), dtype=torch.float64, device="cuda",
                                                    generator=g)).abs()

    s0 = field()
    (Qr, nr, sr), = B.run_batch([B.BatchItem(mesh, p, 4, s0.clone())])
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    x = s0.clone()
    torch.cuda.current_stream().synchronize()
    t0 = __import__("time").perf_counter()
    (Q, ns, st), = B.run_batch([B.BatchItem(mesh, p, 4, x)], stream=side)
    t_call = __import__("time").perf_counter() - t0
    del x
    junk = torch.full((4, mesh.n_nodes), -1.0, dtype=torch.float64, device="cuda")   # may reuse x's memory
    assert torch.equal(Q, Qr) and torch.equal(ns, nr) and torch.all(st == 0)
    side.synchronize()
    t_all = __import__("time").perf_counter() - t0
    assert t_call < t_all
    outs = [B.run_batch([B.BatchItem(mesh, p, 4, s0.clone())]) for _ in range(2)]
    pd.pd_batch_sync(C_stream(torch))
    for (Qk, nk, sk), in outs:
        assert torch.equal(Qk, Qr) and torch.equal(nk, nr)
    del junk


def C_stream(torch):
    import ctypes
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_batch_flags_a_non_positive_micromodulus(env):
    """A batch sample whose micromodulus field has a zero or a negative value
    gets PD_EINVAL (the kernels keep c / c_ref in the flag word, where 0
    marks a ghost cell); its neighbours in the batch are unaffected."""
    torch, B, pd = env
    lv = dataclasses.replace(W.level(0, fracture=True), n_steps=32)
    mesh = B.Mesh.for_level(lv)
    p = B.make_params(lv)
    c = torch.full((3, mesh.n_nodes), c_ref(lv), dtype=torch.float64, device="cuda")
    (Qa, na, sa), = B.run_batch([B.BatchItem(mesh, p, 1, None, c[:1].contiguous())])
    c[1, 100] = 0.0
    c[2, 7] = -c_ref(lv)
    (Q, ns, st), = B.run_batch([B.BatchItem(mesh, p, 3, None, c)])
    assert st.tolist() == [pd.PD_OK, pd.PD_EINVAL, pd.PD_EINVAL]
    assert Q[0] == Qa[0] and ns[0] == na[0]
