"""GPU parity on the size-sweep beams (geometrically similar notched beams,
D = 50 / 100 / 200 / 400 mm at dx = 2.5 mm: up to 1.79M nodes and 102M
bonds), at full size with the sweep's 32 samples per launch.

A solve of these beams is out of the oracle's reach (the D = 400 beam costs
the oracle about 2 s per time step, and the support reaction stays exactly
zero until the stress wave reaches the supports after about D / 2 mm steps),
so the check is one force evaluation of the step kernel on 32 frozen smooth
fields with per-node limit stretches, compared with the oracle's force at
sampled nodes: every node next to the notch tip, the pad nodes' corners,
the box corners and random interior and surface nodes, each evaluated by the
oracle over that node's own bonds (neighbourhood, notch cut and all)."""
import numpy as np
import pytest

import workloads as W
from oracle import geometry as G
from oracle import solver as S

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_2212_04415_amd import beam
    return beam


def sweep_level(D):
    return [lv for lv in [c for c in W.configs() if c.name == "size_sweep"][0].levels
            if abs(lv.beam.depth - D * 1e-3) < 1e-9][0]


def sampled_nodes(shape, dx, beam, rng, n_random=96):
    nx, ny, nz = shape
    ix = lambda i, j, k: i + nx * (j + ny * k)
    xn = int(round(0.5 * beam.length / dx))           # first node column right of the notch plane
    tip = int(round(beam.notch_depth / dx))
    picks = [ix(i, j, k) for i in range(xn - 3, xn + 3) for j in (0, ny // 2, ny - 1)
             for k in range(max(tip - 3, 0), min(tip + 3, nz))]
    sup, load = G.beam_pads(shape, dx, beam)
    picks += [int(sup[0]), int(sup[-1]), int(load[0]), int(load[-1])]
    picks += [ix(i, j, k) for i in (0, nx - 1) for j in (0, ny - 1) for k in (0, nz - 1)]
    picks += list(rng.integers(0, nx * ny * nz, n_random))
    return np.unique(np.array(picks, dtype=np.int64))


def local_problem(lv, shape, node, s0):
    """The oracle problem of one node's bonds, renumbered: local node 0 is
    the node, 1.. its neighbours.  Returns the problem and the global ids."""
    nx, ny, nz = shape
    i, j, k = node % nx, (node // nx) % ny, node // (nx * ny)
    st = G.stencil(W.M_RATIO)
    i2, j2, k2 = i + st[:, 0], j + st[:, 1], k + st[:, 2]
    ok = (i2 >= 0) & (i2 < nx) & (j2 >= 0) & (j2 < ny) & (k2 >= 0) & (k2 < nz)
    nb = (i2 + nx * (j2 + ny * k2))[ok]
    v = st[ok]
    cut = G.notch_cut_mask(shape, lv.dx, np.minimum(nb, node), np.maximum(nb, node), 0.5 * lv.beam.length,
                           lv.beam.notch_depth)
    nb, v = nb[~cut], v[~cut]
    ids = np.concatenate([[node], nb]).astype(np.int64)
    n = ids.size
    delta = W.M_RATIO * lv.dx
    prob = S.Problem(shape=(n, 1, 1), dx=lv.dx, bond_i=np.zeros(n - 1, dtype=np.int64),
                     bond_j=np.arange(1, n, dtype=np.int64), xi=v.astype(np.float64) * lv.dx,
                     support=np.zeros(0, dtype=np.int64), load=np.zeros(0, dtype=np.int64), s0=s0[ids],
                     c=np.full(n, S.micromodulus(W.E_MODULUS, delta)), rho=W.DENSITY, damping=W.DAMPING,
                     dt=lv.dt, du=0.0, n_steps=0, law=lv.law, k=W.SOFT_K, alpha=W.SOFT_ALPHA,
                     GF=W.FRACTURE_ENERGY, delta=delta)
    return prob, ids


@pytest.mark.parametrize("D", [50, 100, 200, 400])
def test_size_sweep_force_at_full_size(B, D):
    lv = sweep_level(D)
    mesh = B.Mesh.for_level(lv)
    M, shape = mesh.n_nodes, mesh.shape
    n_samples = 32
    rng = np.random.default_rng(4000 + D)
    s0 = W.S0_MEAN * np.exp(0.2 * rng.standard_normal((n_samples, M)))
    amp = 3e-6                                        # strains up to a few 1e-4 across the 50 mm thickness
    u = np.stack([W.smooth_displacement(shape, lv.dx, amp, seed=40 + k) for k in (0, n_samples - 1)])
    u_all = np.empty((n_samples, M, 3))
    u_all[:] = u[0]
    u_all[-1] = u[1]
    u_all = (u_all / lv.dx).astype(np.float32).astype(np.float64) * lv.dx     # as the FP32 state holds it
    mesh.set_field(0, s0)
    L = B.force_eval(mesh, B.make_params(lv, precision="f32"), u_all)
    mesh.set_field(0, None)
    nodes = sampled_nodes(shape, lv.dx, lv.beam, rng)
    damaged = 0
    worst = 0.0
    for smp in (0, n_samples - 1):
        for node in nodes:
            prob, ids = local_problem(lv, shape, int(node), s0[smp])
            ul = u_all[smp][ids]
            ref = prob.force(ul)[0]
            s = prob.stretch(ul)
            sig = np.sum(np.abs(prob.c[0] * s)) * prob.volume
            damaged += int(np.sum(s > 0.5 * (prob.s0[0] + prob.s0[1:])))
            err = np.max(np.abs(L[smp, node] - ref))
            worst = max(worst, err / (64 * EPS32 * sig))
            assert err <= 64 * EPS32 * sig, (D, smp, int(node), err, sig)
    print(f"D = {D} mm: {len(nodes)} nodes x 2 samples, {damaged} bonds past s0, max err / bound = {worst:.3f}")
    assert damaged > 0


@pytest.mark.slow
def test_size_effect_beam_full_length_matches_oracle():
    """The D = 50 mm beam of the size-effect sweep to full length in the
    sweep's launch configuration (32 samples, seed 4, cracking load, 8000
    steps, FP32 with compensation): sample 0's peak load and peak step
    against the oracle on the same KL coefficients."""
    import torch
    from oracle import kl as OKL
    from paper_2212_04415_amd import beam as B
    lv = [lv for lv in [c for c in W.configs(fracture=True) if c.name == "size_sweep"][0].levels
          if abs(lv.beam.depth - 50e-3) < 1e-9][0]
    mesh = B.Mesh.for_level(lv)
    kl = B.KL(mesh, W.FIELD_CORR_LEN, W.FIELD_MODES, 256)
    xi = W.kl_coefficients(4, 32, stream=0)
    s0 = kl.lognormal(torch.tensor(xi), W.S0_MEAN, W.FIELD_COV, dtype=torch.float32)
    (Q, ns, st), = B.run_batch([B.BatchItem(mesh, B.make_params(lv), 32, s0)])
    assert torch.all(st == 0)
    ob = OKL.Basis3D((lv.beam.length, lv.beam.thickness, lv.beam.depth), W.FIELD_CORR_LEN, W.FIELD_MODES, 256)
    pos = G.node_positions(mesh.shape, lv.dx)
    ref = S.beam_problem(lv, s0=OKL.lognormal_field(ob, pos, xi[:1], W.S0_MEAN, W.FIELD_COV)[0]).run(
        want_state=False)
    print(f"D = 50 mm sample 0: peak {Q[0].item():.4f} N at step {ns[0].item()}, oracle {ref['Q']:.4f} N at "
          f"step {ref['nstar']}")
    assert 0.1 * lv.n_steps < ref["nstar"] < lv.n_steps
    assert Q[0].item() == pytest.approx(ref["Q"], rel=5e-3)
    assert abs(ns[0].item() - ref["nstar"]) <= 0.02 * lv.n_steps


@pytest.mark.parametrize("depth_mm", [100, 200])
def test_size_effect_beams_fp32_batch_matches_fp64(depth_mm):
    """Equal QoI error beyond the oracle's reach: the D = 100 and 200 mm
    beams of the size-effect sweep to full length (16,000 / 32,000 steps,
    cracking load) on the sweep's first two KL fields, batched FP32 with
    compensation against the FP64 solve of the same fields (itself pinned to
    the oracle to 1e-9 on smaller meshes): peaks within 0.5%, peak steps
    within 2% of the run."""
    import torch
    from paper_2212_04415_amd import beam as B
    sweep = [c for c in W.configs(fracture=True) if c.name == "size_sweep"][0]
    i, lv = [(k, lv) for k, lv in enumerate(sweep.levels) if abs(lv.beam.depth - depth_mm * 1e-3) < 1e-9][0]
    mesh = B.Mesh.for_level(lv)
    kl = B.KL(mesh, W.FIELD_CORR_LEN, W.FIELD_MODES, 256)
    xi = torch.tensor(W.kl_coefficients(sweep.seed, 2, stream=i))
    s32 = kl.lognormal(xi, W.S0_MEAN, W.FIELD_COV, dtype=torch.float32)
    s64 = kl.lognormal(xi, W.S0_MEAN, W.FIELD_COV, dtype=torch.float64)
    (q32, n32, st32), = B.run_batch([B.BatchItem(mesh, B.make_params(lv), 2, s32)])
    (q64, n64, st64), = B.run_batch([B.BatchItem(mesh, B.make_params(lv, precision="f64"), 2, s64)])
    assert torch.all(st32 == 0) and torch.all(st64 == 0)
    for k in range(2):
        print(f"D = {depth_mm} mm sample {k}: FP32 {q32[k].item():.4f} N at {n32[k].item()}, "
              f"FP64 {q64[k].item():.4f} N at {n64[k].item()}")
        assert 0.1 * lv.n_steps < n64[k].item() < lv.n_steps
        assert q32[k].item() == pytest.approx(q64[k].item(), rel=5e-3)
        assert abs(n32[k].item() - n64[k].item()) <= 0.02 * lv.n_steps
