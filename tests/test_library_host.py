"""CPU checks of libpdmi.so: it loads, exports every entry point declared in
include/pd.h, and its host-side lattice, notch cut and pads agree exactly with
the oracle's.  No compute call is made (there is no GPU here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import geometry as G
from paper_2212_04415_amd import pd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "pd.h")).read()
    return sorted(set(re.findall(r"PD_API\s+[\w\s\*]+?\b(pd_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = pd.lib()
    names = declared_symbols()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(pd.SIGNATURES)
    # and the binding has a Python function of the same name for each
    for n in names:
        assert callable(getattr(pd, n)), n


def build(beam, dx, m_ratio=W.M_RATIO, extent_y=None, thickness=0.0, plane_strain=0):
    desc = pd.pd_mesh_desc((C.c_double * 3)(beam.length, beam.thickness if extent_y is None else extent_y,
                                            beam.depth), dx, m_ratio, beam.span, beam.notch_depth, beam.pad_width,
                           thickness, plane_strain)
    h = C.c_void_p()
    rc = pd.lib().pd_build_mesh(C.byref(desc), C.byref(h))
    return rc, h


@pytest.mark.parametrize("ell", [0, 1])
def test_host_geometry_matches_oracle(ell):
    lv = W.level(ell)
    rc, h = build(lv.beam, lv.dx)
    assert rc == 0, pd.pd_last_error()
    try:
        nb = C.c_int64()
        assert pd.lib().pd_build_bonds(h, C.byref(nb)) == 0, pd.pd_last_error()
        info = pd.pd_mesh_info_t()
        pd.pd_mesh_get_info(h, C.byref(info))
        shape = lv.shape
        bi, bj, _ = G.unique_bonds(shape, W.M_RATIO)
        cut = G.notch_cut_mask(shape, lv.dx, bi, bj, 0.5 * lv.beam.length, lv.beam.notch_depth)
        assert (info.nx, info.ny, info.nz) == shape
        assert info.n_nodes == np.prod(shape)
        assert nb.value == info.n_bonds == bi.size - cut.sum()
        assert info.n_cut == cut.sum()
        assert info.n_stencil == 122
        sup = np.zeros(info.n_support, dtype=np.int32)
        ld = np.zeros(info.n_load, dtype=np.int32)
        pd.pd_mesh_get_pads(h, sup.ctypes.data, ld.ctypes.data)
        osup, old = G.beam_pads(shape, lv.dx, lv.beam)
        assert np.array_equal(np.sort(sup), osup) and np.array_equal(np.sort(ld), old)
    finally:
        pd.pd_free_mesh(h)


def test_host_geometry_size_sweep_beam():
    beam = W.Beam.similar(100e-3)
    rc, h = build(beam, 2.5e-3)
    assert rc == 0, pd.pd_last_error()
    try:
        nb = C.c_int64()
        pd.pd_build_bonds(h, C.byref(nb))
        shape = G.grid_shape((beam.length, beam.thickness, beam.depth), 2.5e-3)
        bi, bj, _ = G.unique_bonds(shape, W.M_RATIO)
        cut = G.notch_cut_mask(shape, 2.5e-3, bi, bj, 0.5 * beam.length, beam.notch_depth)
        assert nb.value == bi.size - cut.sum()
    finally:
        pd.pd_free_mesh(h)


@pytest.mark.parametrize("bad", ["extent", "m_ratio", "pad_face", "notch"])
def test_host_rejects_bad_geometry(bad):
    beam, dx, m = W.Beam(), 5e-3, W.M_RATIO
    if bad == "extent":
        beam = W.Beam(length=176e-3)
    elif bad == "m_ratio":
        m = 2.5
    elif bad == "pad_face":
        beam = W.Beam(pad_width=10e-3, span=145e-3)      # pad faces through node centres
    elif bad == "notch":
        beam = W.Beam(notch_depth=3.3e-3)
    rc, h = build(beam, dx, m)
    assert rc == pd.PD_EINVAL
    assert pd.pd_last_error()


def test_null_arguments_are_rejected():
    assert pd.lib().pd_build_mesh(None, None) == pd.PD_EINVAL
    assert pd.lib().pd_run(None, None, None, None) == pd.PD_EINVAL
    assert pd.lib().pd_level_stats(None, None, 0, None, None) == pd.PD_EINVAL


def test_launch_shape_pinning_is_validated():
    rc, h = build(W.level(0).beam, W.level(0).dx)
    assert rc == pd.PD_OK
    try:
        for shape in (pd.PD_SHAPE_AUTO, pd.PD_SHAPE_LDS_16x4x4, pd.PD_SHAPE_GLOBAL_256, pd.PD_N_SHAPES - 1):
            assert pd.lib().pd_set_launch_shape(h, shape) == pd.PD_OK
        for bad in (-2, pd.PD_N_SHAPES, 99):
            assert pd.lib().pd_set_launch_shape(h, bad) == pd.PD_EINVAL
            assert "launch shape" in pd.pd_last_error()
        assert pd.lib().pd_set_launch_shape(None, 0) == pd.PD_EINVAL
        assert pd.lib().pd_autotune(None, None, 1, None, None, None) == pd.PD_EINVAL
    finally:
        pd.lib().pd_free_mesh(h)


@pytest.mark.parametrize("ell", [0, 2, 4])
def test_host_geometry_plane_specimen_matches_oracle(ell):
    """The plane-stress Specimen 3 (one node thick) at the paper's levels."""
    lv = W.level2d(ell)
    rc, h = build(lv.beam, lv.dx, extent_y=lv.dx, thickness=lv.beam.thickness)
    assert rc == 0, pd.pd_last_error()
    try:
        nb = C.c_int64()
        assert pd.lib().pd_build_bonds(h, C.byref(nb)) == 0, pd.pd_last_error()
        info = pd.pd_mesh_info_t()
        pd.pd_mesh_get_info(h, C.byref(info))
        shape = lv.shape
        assert (info.nx, info.ny, info.nz) == shape and shape[1] == 1
        bi, bj, _ = G.unique_bonds(shape, W.M_RATIO)
        cut = G.notch_cut_mask(shape, lv.dx, bi, bj, 0.5 * lv.beam.length, lv.beam.notch_depth)
        assert nb.value == info.n_bonds == bi.size - cut.sum()
        sup = np.zeros(info.n_support, dtype=np.int32)
        ld = np.zeros(info.n_load, dtype=np.int32)
        pd.pd_mesh_get_pads(h, sup.ctypes.data, ld.ctypes.data)
        osup, old = G.beam_pads(shape, lv.dx, lv.beam)
        assert np.array_equal(np.sort(sup), osup) and np.array_equal(np.sort(ld), old)
    finally:
        pd.pd_free_mesh(h)


@pytest.mark.parametrize("extent_y,thickness,strain", [(2 * 10e-3, 50e-3, 0), (10e-3, -1.0, 0), (10e-3, 0.0, 1),
                                                       (10e-3, 50e-3, 2)])
def test_plane_mesh_rejects_bad_thickness(extent_y, thickness, strain):
    """A plane body must be one node thick and its thickness non-negative;
    plane strain needs a plane body and is a 0/1 flag."""
    rc, h = build(W.SPECIMEN3, 10e-3, extent_y=extent_y, thickness=thickness, plane_strain=strain)
    assert rc == pd.PD_EINVAL and not h.value
    assert "thick" in pd.pd_last_error() or "plane_strain" in pd.pd_last_error()


def test_mesh_size_limit_is_the_kernels_addressing_limit():
    """A cube of 506 nodes per side has exactly 2^27 cells with its ghost
    layers and is accepted; one more node per side is refused with a message
    (the step kernels' per-lane byte offsets are 32-bit)."""
    dx = 1e-3
    for n, ok in ((506, True), (507, False)):
        beam = W.Beam(length=n * dx, thickness=n * dx, depth=n * dx, span=400e-3, notch_depth=100e-3,
                      pad_width=10e-3)
        rc, h = build(beam, dx)
        if ok:
            assert rc == pd.PD_OK, pd.pd_last_error()
            pd.lib().pd_free_mesh(h)
        else:
            assert rc == pd.PD_EINVAL
            assert "too large" in pd.pd_last_error()


def test_force_eval_sample_count_is_bounded():
    """Sample counts outside 1..65535 are refused before any device work."""
    from paper_2212_04415_amd import beam as B
    lv = W.level(0)
    rc, h = build(lv.beam, lv.dx)
    assert rc == pd.PD_OK
    try:
        p = B.make_params(lv)
        buf = (C.c_double * 3)()
        for n in (0, 65536):
            assert pd.lib().pd_force_eval(h, C.byref(p), n, buf, buf, None) == pd.PD_EINVAL
            assert "n_samples" in pd.pd_last_error()
    finally:
        pd.lib().pd_free_mesh(h)


def test_params_come_from_the_level_description():
    """make_params takes the material from the level it is given (the
    binding imports no workload module) and refuses to guess without one."""
    import ast
    import dataclasses
    from paper_2212_04415_amd import beam as B
    lv = W.level(1, fracture=True)
    p = B.make_params(lv, precision="f64")
    assert (p.E, p.rho, p.GF, p.s0, p.k, p.alpha, p.damping) == (
        W.E_MODULUS, W.DENSITY, W.FRACTURE_ENERGY, W.S0_MEAN, W.SOFT_K, W.SOFT_ALPHA, W.DAMPING)
    assert (p.dt, p.du, p.n_steps, p.law, p.precision) == (lv.dt, lv.du, lv.n_steps, lv.law, pd.PD_FP64)
    soft = dataclasses.replace(lv, material=dataclasses.replace(lv.material, E=30e9, damping=0.0))
    q = B.make_params(soft, GF=100.0)
    assert (q.E, q.damping, q.GF) == (30e9, 0.0, 100.0)
    with pytest.raises(ValueError, match="no value for E"):
        B.make_params(None, dt=1e-6, du=1e-9, n_steps=3)
    pkg = os.path.join(os.path.dirname(pd.__file__))
    for name in os.listdir(pkg):
        if name.endswith(".py"):
            tree = ast.parse(open(os.path.join(pkg, name)).read())
            for node in ast.walk(tree):
                if isinstance(node, ast.Import):
                    assert all(a.name != "workloads" for a in node.names), name
                if isinstance(node, ast.ImportFrom):
                    assert node.module != "workloads", name


def test_binding_constants_match_the_header():
    """Every enum constant of include/pd.h has the same value in the Python
    binding (a renamed or renumbered constant fails here, not on a GPU)."""
    text = open(os.path.join(ROOT, "include", "pd.h")).read()
    consts = {}
    for body in re.findall(r"enum\s*\{([^}]*)\}", text):
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        for name, value in re.findall(r"(PD_[A-Z0-9_x]+)\s*=\s*(-?\d+)", body):
            consts[name] = int(value)
    assert len(consts) >= 29
    for name, value in consts.items():
        assert getattr(pd, name) == value, name


def test_build_rejects_scratch_and_wide_step_kernels():
    """The build reads the compiler's resource remarks: an FP32 step kernel
    with scratch memory (spills, or a private array) or a default-brick FP32
    kernel past 128 VGPRs is named; FP64 kernels and the c-tile kernels
    above 128 VGPRs are not."""
    from paper_2212_04415_amd import build as BD
    fast = "_ZN4pdmi11step_kernelIfLb1ELb0ELb1ENS_5BrickILi16ELi4ELi4ELi2EEEEEvNS_10StepParamsIT_EE"
    ctile = "_ZN4pdmi11step_kernelIfLb1ELb1ELb1ENS_5BrickILi16ELi4ELi4ELi2EEEEEvNS_10StepParamsIT_EE"
    f64 = "_ZN4pdmi11step_kernelIdLb0ELb0ELb1ENS_5BrickILi16ELi4ELi4ELi2EEEEEvNS_10StepParamsIT_EE"

    def remarks(name, vgprs, scratch, spill):
        pre = "step_kernels.h:1:1: remark: "
        return (f"{pre}Function Name: {name} [-Rpass-analysis=kernel-resource-usage]\n"
                f"{pre}    VGPRs: {vgprs} [-Rpass-analysis=kernel-resource-usage]\n"
                f"{pre}    ScratchSize [bytes/lane]: {scratch} [-Rpass-analysis=kernel-resource-usage]\n"
                f"{pre}    VGPRs Spill: {spill} [-Rpass-analysis=kernel-resource-usage]\n")

    ok = BD.kernel_resources(remarks(fast, 121, 0, 0) + remarks(ctile, 140, 0, 0) + remarks(f64, 200, 64, 10))
    assert ok[fast] == {"VGPRs": 121, "ScratchSize": 0, "VGPRSpill": 0}
    assert BD.resource_problems(ok) == []
    for vgprs, scratch, spill, what in ((121, 32, 0, "scratch"), (121, 16, 4, "scratch"), (129, 0, 0, "128 VGPRs")):
        bad = BD.kernel_resources(remarks(fast, vgprs, scratch, spill))
        (msg,) = BD.resource_problems(bad)
        assert what in msg and fast in msg
