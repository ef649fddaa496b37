"""Pins of the oracle's discrete adjoint (dQ/ds0, dQ/dc of the peak reaction):

* exactly zero sensitivity to the limit stretch while every bond is elastic;
* the complex-step derivative of an independent, vectorised complex-valued
  re-evaluation of the same time loop, along random directions, on a small
  notched beam that cracks before its peak: a complex step i*h in the fields
  carries the exact directional derivative of the branch the real trajectory
  follows (every max, threshold and law segment is decided on real parts), to
  rounding, with no subtractive cancellation;
* central finite differences on the level-0 beam with the smooth
  exponential-linear law (loose: finite differences straddle damage-onset
  events)."""
import numpy as np
import pytest

import workloads as W
from oracle import solver as S

SMALL_BEAM = W.Beam(length=50e-3, thickness=10e-3, depth=15e-3, span=40e-3, notch_depth=5e-3, pad_width=5e-3)


def complex_peak(p, s0, c):
    """The time loop of the oracle (R11 of the design notes) in complex
    arithmetic over the unique bonds, vectorised with NumPy."""
    bi, bj, xi = p.bond_i, p.bond_j, p.xi
    M, V, h = p.n_nodes, p.volume, p.dt / (2 * p.rho)
    c_b = 0.5 * (c[bi] + c[bj])
    s0_b = 0.5 * (s0[bi] + s0[bj])
    d5 = p.delta ** 5
    if p.law == S.LAW_EXPLIN:
        ek = np.exp(p.k)
        P = 2 * p.k - 2 * ek + p.alpha * p.k - p.alpha * p.k * ek + 2
        sc_b = s0_b - p.GF * 10 * p.k * (ek - 1) * (1 + p.alpha) / (np.pi * c_b * s0_b * d5 * P)
    else:
        sc_b = s0_b + p.GF * 5 / (np.pi * d5 * 0.2 * c_b * s0_b)
    fixed = np.zeros(M, dtype=bool)
    fixed[p.support] = True
    fixed[p.load] = True
    free = np.ones((M, 3), dtype=bool)
    free[fixed, 2] = False
    u = np.zeros((M, 3), dtype=complex)
    v = np.zeros((M, 3), dtype=complex)
    L = np.zeros((M, 3), dtype=complex)
    kap = np.full(bi.size, -np.inf + 0j)
    xl = np.linalg.norm(xi, axis=1)
    best, bestR = -np.inf, None
    with np.errstate(divide="ignore", invalid="ignore"):
        return _loop(p, bi, bj, xi, M, V, h, c_b, s0_b, sc_b, free, u, v, L, kap, xl, best, bestR)


def _loop(p, bi, bj, xi, M, V, h, c_b, s0_b, sc_b, free, u, v, L, kap, xl, best, bestR):
    for n in range(p.n_steps):
        v = np.where(free, v + h * (L - p.damping * v), v)
        u = u + p.dt * v
        u[p.support, 2] = 0
        v[p.support, 2] = 0
        u[p.load, 2] = -(n + 1) * p.du
        v[p.load, 2] = -p.du / p.dt
        y = xi + u[bj] - u[bi]
        l = np.sqrt(np.sum(y * y, axis=1))
        s = (l - xl) / xl
        kap = np.where(s.real > kap.real, s, kap)
        t = (kap - s0_b) / (sc_b - s0_b)
        if p.law == S.LAW_EXPLIN:
            br = 1 - (1 - np.exp(-p.k * t)) / (1 - np.exp(-p.k)) + p.alpha * (1 - t)
            keep = (s0_b / kap) * br / (1 + p.alpha)
        else:
            g = np.where(t.real <= 0.2, s0_b * (1 - 4 * t), 0.25 * s0_b * (1 - t))
            keep = g / kap
        keep = np.where(kap.real <= s0_b.real, 1.0 + 0j, np.where(kap.real >= sc_b.real, 0j, keep))
        f = (c_b * keep * s * V / l)[:, None] * y
        L = np.zeros((M, 3), dtype=complex)
        for d in range(3):
            L[:, d] += np.bincount(bi, weights=f[:, d].real, minlength=M) + \
                1j * np.bincount(bi, weights=f[:, d].imag, minlength=M)
            L[:, d] -= np.bincount(bj, weights=f[:, d].real, minlength=M) + \
                1j * np.bincount(bj, weights=f[:, d].imag, minlength=M)
        v = np.where(free, (v + h * L) / (1 + p.damping * h), v)
        R = -np.sum(L[p.support, 2]) * V
        if R.real > best:
            best, bestR = R.real, R
    return bestR


@pytest.mark.parametrize("law", [S.LAW_EXPLIN, S.LAW_TRILINEAR])
def test_adjoint_matches_complex_step(law):
    lv = W.Level(beam=SMALL_BEAM, dx=2.5e-3, dt=5e-7, n_steps=600, du=4e-8, law=law)
    rng = np.random.default_rng(4)
    p = S.beam_problem(lv)
    p.s0 = W.S0_MEAN * np.exp(0.1 * rng.standard_normal(p.n_nodes))
    p.c = p.c * np.exp(0.05 * rng.standard_normal(p.n_nodes))
    a = p.adjoint()
    assert 0.2 * lv.n_steps < a["nstar"] < 0.9 * lv.n_steps
    assert np.count_nonzero(a["dQ_ds0"]) > 50              # damage before the peak
    h = 1e-20
    for field in ("s0", "c"):
        dirn = rng.standard_normal(p.n_nodes)
        base = p.s0 if field == "s0" else p.c
        pert = base * (1 + 1j * h * dirn)
        Rc = complex_peak(p, pert if field == "s0" else p.s0.astype(complex),
                          p.c.astype(complex) if field == "s0" else pert)
        assert Rc.real == pytest.approx(a["Q"], rel=1e-12)
        cs = Rc.imag / h
        adj = np.dot(a["dQ_ds0"] if field == "s0" else a["dQ_dc"], base * dirn)
        assert adj == pytest.approx(cs, rel=1e-8), field


def test_elastic_limit_stretch_has_no_influence():
    lv = W.level(0)
    p = S.beam_problem(lv, n_steps=400)
    a = p.adjoint()
    assert np.all(a["dQ_ds0"] == 0.0)
    assert np.max(np.abs(a["dQ_dc"])) > 0


@pytest.mark.slow
def test_adjoint_against_central_differences_level0():
    lv = W.level(0, fracture=True, law=W.LAW_EXPLIN)
    rng = np.random.default_rng(0)
    M = int(np.prod(lv.shape))
    s0 = W.S0_MEAN * np.exp(0.1 * rng.standard_normal(M))
    p = S.beam_problem(lv, s0=s0, du=4e-8, n_steps=1000)
    a = p.adjoint()
    dirn = rng.standard_normal(M)
    h = 1e-4
    for field, g in (("s0", a["dQ_ds0"]), ("c", a["dQ_dc"])):
        base = s0 if field == "s0" else p.c
        qs = []
        for sgn in (1, -1):
            kw = dict(s0=s0 + sgn * h * base * dirn) if field == "s0" else dict(s0=s0, c=p.c + sgn * h * base * dirn)
            qs.append(S.beam_problem(lv, du=4e-8, n_steps=1000, **kw).run(want_state=False)["Q"])
        fd = (qs[0] - qs[1]) / 2
        assert np.dot(g, h * base * dirn) == pytest.approx(fd, rel=5e-3)


def test_keep_derivatives_match_differences():
    for law in (S.LAW_EXPLIN, S.LAW_TRILINEAR):
        s0, sc = 1e-4, 5e-3
        for kap in (1.5e-4, 6e-4, 2e-3, 4.5e-3):
            k0, dk, ds0, dsc = S.keep_derivs(law, kap, s0, sc, W.SOFT_K, W.SOFT_ALPHA)
            e = 1e-7
            def keep(kk, a, b):
                return S.keep_derivs(law, kk, a, b, W.SOFT_K, W.SOFT_ALPHA)[0]
            assert k0 == pytest.approx(1 - S.damage(law, kap, s0, sc, W.SOFT_K, W.SOFT_ALPHA), rel=1e-13)
            assert dk == pytest.approx((keep(kap * (1 + e), s0, sc) - keep(kap * (1 - e), s0, sc)) / (2 * e * kap), rel=1e-5)
            assert ds0 == pytest.approx((keep(kap, s0 * (1 + e), sc) - keep(kap, s0 * (1 - e), sc)) / (2 * e * s0), rel=1e-5)
            assert dsc == pytest.approx((keep(kap, s0, sc * (1 + e)) - keep(kap, s0, sc * (1 - e))) / (2 * e * sc), rel=1e-5)
