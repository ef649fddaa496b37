"""Convenience wrappers over the C ABI for beam workloads (argument
marshalling only; the solve runs in libpdmi's kernels)."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import pd


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class Mesh:
    """A built beam lattice (pd_build_mesh + pd_build_bonds)."""

    def __init__(self, beam, dx: float, m_ratio: float = 3.14):
        self.beam, self.dx = beam, dx
        plane = getattr(beam, "plane", False)
        desc = pd.pd_mesh_desc((C.c_double * 3)(beam.length, dx if plane else beam.thickness, beam.depth), dx,
                               m_ratio, beam.span, beam.notch_depth, beam.pad_width,
                               beam.thickness if plane else 0.0,
                               1 if plane and getattr(beam, "plane_strain", False) else 0)
        self.h = C.c_void_p()
        pd.pd_build_mesh(C.byref(desc), C.byref(self.h))
        nb = C.c_int64()
        pd.pd_build_bonds(self.h, C.byref(nb))
        info = pd.pd_mesh_info_t()
        pd.pd_mesh_get_info(self.h, C.byref(info))
        self.info = info
        self.shape = (info.nx, info.ny, info.nz)
        self.n_nodes = int(info.n_nodes)
        self.n_bonds = int(info.n_bonds)
        sup = np.zeros(info.n_support, dtype=np.int32)
        ld = np.zeros(info.n_load, dtype=np.int32)
        pd.pd_mesh_get_pads(self.h, sup.ctypes.data, ld.ctypes.data)
        self.support, self.load = sup, ld

    @classmethod
    def for_level(cls, level, m_ratio: float = 3.14):
        return cls(level.beam, level.dx, m_ratio)

    def set_field(self, field: int, values: Optional[np.ndarray]):
        if values is None:
            pd.pd_set_material_field(self.h, field, 0, None, 0, pd.PD_DTYPE_F64, None)
            return
        v = np.ascontiguousarray(values, dtype=np.float64)
        n = v.size // self.n_nodes
        pd.pd_set_material_field(self.h, field, n, v.ctypes.data, 0, pd.PD_DTYPE_F64, None)

    def set_launch_shape(self, shape: int):
        """Pin the step kernel's launch shape (pd.PD_SHAPE_*), or
        pd.PD_SHAPE_AUTO to let the autotuner choose."""
        pd.pd_set_launch_shape(self.h, shape)

    def close(self):
        if self.h:
            pd.pd_free_mesh(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params(level=None, *, precision="f32", accumulate="kahan", E=None, rho=None, GF=None, s0=None,
                k=None, alpha=None, law=None, damping=None, dt=None, du=None, n_steps=None,
                record_history=False, checkpoint_every=0) -> pd.pd_params:
    """pd_params from a level description (any object with dt, du, n_steps,
    law and a `material` record with E, rho, GF, s0, k, alpha, damping);
    keyword values override it.  Without a level every value must be given."""
    mat = getattr(level, "material", None)

    def pick(name, value, src):
        if value is not None:
            return value
        if src is None:
            raise ValueError(f"make_params: no value for {name} (pass it or a level that carries it)")
        return getattr(src, name)

    p = pd.pd_params()
    p.E = pick("E", E, mat)
    p.rho = pick("rho", rho, mat)
    p.GF = pick("GF", GF, mat)
    p.s0 = pick("s0", s0, mat)
    p.k = pick("k", k, mat)
    p.alpha = pick("alpha", alpha, mat)
    p.damping = pick("damping", damping, mat)
    p.law = law if law is not None else getattr(level, "law", pd.PD_LAW_TRILINEAR)
    p.dt = pick("dt", dt, level)
    p.du = pick("du", du, level)
    p.n_steps = pick("n_steps", n_steps, level)
    p.precision = {"f32": pd.PD_FP32, "f64": pd.PD_FP64}[precision]
    p.accumulate = {"kahan": pd.PD_ACC_KAHAN, "plain": pd.PD_ACC_PLAIN, "state_only": pd.PD_ACC_STATE_ONLY,
                    "forces_only": pd.PD_ACC_FORCES_ONLY}[accumulate]
    p.record_history = 1 if record_history else 0
    p.checkpoint_every = checkpoint_every
    return p


def force_eval(mesh: Mesh, params, u: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, mesh.n_nodes, 3)
    L = np.zeros_like(u)
    pd.pd_force_eval(mesh.h, C.byref(params), u.shape[0], u.ctypes.data, L.ctypes.data, None)
    return L


def run(mesh: Mesh, params, stream=None, want_state=False):
    """One sample (uses the mesh's single-sample fields).  Returns a dict with
    Q, nstar, R (when record_history) and u, kappa (when want_state)."""
    h = C.c_void_p()
    pd.pd_run(mesh.h, C.byref(params), _stream_ptr(stream) if stream is not None else None, C.byref(h))
    try:
        Q = C.c_double()
        ns = C.c_int64()
        R = np.zeros(max(params.n_steps, 1)) if params.record_history else None
        pd.pd_qoi(h, C.byref(Q), C.byref(ns), R.ctypes.data if R is not None else None)
        out = dict(Q=Q.value, nstar=ns.value, R=R)
        if want_state:
            u = np.zeros((mesh.n_nodes, 3))
            kap = np.zeros((122, mesh.n_nodes))
            pd.pd_run_state(h, u.ctypes.data, kap.ctypes.data)
            out["u"], out["kappa"] = u, kap
        return out
    finally:
        pd.pd_free_run(h)


@dataclass
class BatchItem:
    mesh: Mesh
    params: pd.pd_params
    n_samples: int
    s0: object = None          # torch tensor [S][M] on the device, or None
    c: object = None           # micromodulus (absolute), or None
    gf: object = None          # fracture energy (N/m), or None
    want_u: bool = False       # also return each sample's final displacement [S][M][3]


def run_batch(items: Sequence[BatchItem], stream=None, no_alloc=False):
    """Returns a list of (Q, nstar, status) torch tensors, one triple per item
    (a fourth tensor, the final displacements [S][M][3], for items with
    want_u).  no_alloc: through pd_run_batch_static (work buffers in the
    library's fixed device array; the outputs are still allocated here).
    The solve is enqueued on `stream` (default: torch's current stream) and
    this returns without waiting; the outputs are ready, in stream order, on
    torch's current stream (a different torch stream is joined into it)."""
    import torch
    dev = torch.device("cuda")
    arr = (pd.pd_batch_item * len(items))()
    outs, keep = [], []
    for i, it in enumerate(items):
        Q = torch.empty(it.n_samples, dtype=torch.float64, device=dev)
        ns = torch.empty(it.n_samples, dtype=torch.int64, device=dev)
        st = torch.empty(it.n_samples, dtype=torch.int32, device=dev)
        dtype = pd.PD_DTYPE_F64
        given = [f for f in (it.s0, it.c, it.gf) if f is not None]
        for f in given:
            assert f.is_cuda and f.is_contiguous() and f.shape == (it.n_samples, it.mesh.n_nodes)
            dtype = pd.PD_DTYPE_F32 if f.dtype == torch.float32 else pd.PD_DTYPE_F64
        assert all(f.dtype == given[0].dtype for f in given)
        keep.append(it.params)
        u = torch.empty((it.n_samples, it.mesh.n_nodes, 3), dtype=torch.float64, device=dev) if it.want_u else None
        arr[i] = pd.pd_batch_item(it.mesh.h, C.pointer(it.params), it.n_samples,
                                  it.s0.data_ptr() if it.s0 is not None else None,
                                  it.c.data_ptr() if it.c is not None else None,
                                  it.gf.data_ptr() if it.gf is not None else None, dtype,
                                  Q.data_ptr(), ns.data_ptr(), st.data_ptr(),
                                  u.data_ptr() if u is not None else None)
        outs.append((Q, ns, st) if u is None else (Q, ns, st, u))
    (pd.pd_run_batch_static if no_alloc else pd.pd_run_batch)(arr, len(items), _stream_ptr(stream))
    if isinstance(stream, torch.cuda.Stream) and stream != torch.cuda.current_stream():
        # the tensors are in use on `stream` until it reaches this point
        for it, o in zip(items, outs):
            for t in (it.s0, it.c, it.gf, *o):
                if t is not None:
                    t.record_stream(stream)
        torch.cuda.current_stream().wait_stream(stream)
    return outs


class KL:
    """Karhunen-Loeve basis of a mesh: squared-exponential (pd_kl_build), or
    exponential (KL.exponential / extend: pd_kl_build_exp, pd_kl_extend)."""

    def __init__(self, mesh: Mesh, corr_len: float = None, n_modes: int = 50, n_quad: int = 256, _handle=None):
        self.mesh = mesh
        self.h = C.c_void_p()
        if _handle is not None:
            self.h = _handle
        else:
            pd.pd_kl_build(mesh.h, corr_len, n_modes, n_quad, C.byref(self.h))
        n = C.c_int32()
        pd.pd_kl_n_modes(self.h, C.byref(n))
        self.n_modes = n.value

    @classmethod
    def exponential(cls, mesh: Mesh, corr_len: float, n_modes: int = 50):
        """Nystrom basis of exp(-|x - x'| / corr_len) on this (coarsest) mesh."""
        h = C.c_void_p()
        pd.pd_kl_build_exp(mesh.h, corr_len, n_modes, C.byref(h))
        return cls(mesh, _handle=h)

    def extend(self, target: Mesh):
        """This exponential basis evaluated at another mesh's nodes."""
        h = C.c_void_p()
        pd.pd_kl_extend(self.h, target.h, C.byref(h))
        return KL(target, _handle=h)

    def gaussian(self, xi, stream=None):
        """Unit-variance Gaussian field for xi [S][n_modes] (device FP64 out)."""
        import torch
        xi = xi.to(device="cuda", dtype=torch.float64).contiguous()
        out = torch.empty((xi.shape[0], self.mesh.n_nodes), dtype=torch.float64, device="cuda")
        pd.pd_kl_gaussian(self.h, xi.data_ptr(), xi.shape[0], out.data_ptr(), _stream_ptr(stream))
        return out

    def eigenvalues(self):
        lam = np.zeros(self.n_modes)
        pd.pd_kl_eigenvalues(self.h, lam.ctypes.data)
        return lam

    def lognormal(self, xi, mean: float, cov: float, dtype=None, stream=None):
        import torch
        dtype = torch.float64 if dtype is None else dtype
        xi = xi.to(device="cuda", dtype=torch.float64).contiguous()
        out = torch.empty((xi.shape[0], self.mesh.n_nodes), dtype=dtype, device="cuda")
        pd.pd_kl_field(self.h, xi.data_ptr(), xi.shape[0], mean, cov, out.data_ptr(),
                       pd.PD_DTYPE_F64 if dtype == torch.float64 else pd.PD_DTYPE_F32, _stream_ptr(stream))
        return out

    def close(self):
        if self.h:
            pd.pd_kl_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fib_fields(mesh: Mesh, g, fcm=42.3e6, weibull_m=3.0, alpha_E=1.0, delta_f=8.0e6, fck_min=1.0e6, dtype=None,
               stream=None):
    """pd_fib_fields: per-node (s0, c, G_F) device tensors from a Gaussian
    field g [S][n_nodes] (device FP64)."""
    import torch
    dtype = torch.float64 if dtype is None else dtype
    g = g.to(device="cuda", dtype=torch.float64).contiguous()
    outs = [torch.empty_like(g, dtype=dtype) for _ in range(3)]
    fp = pd.pd_fib_params(fcm, weibull_m, alpha_E, delta_f, fck_min)
    pd.pd_fib_fields(mesh.h, g.data_ptr(), g.shape[0], C.byref(fp), *[o.data_ptr() for o in outs],
                     pd.PD_DTYPE_F64 if dtype == torch.float64 else pd.PD_DTYPE_F32, _stream_ptr(stream))
    return tuple(outs)


def level_stats(q_fine, q_coarse=None, stream=None):
    """FP64 (N, sum Y, sum Y^2) of one MLMC level as a device tensor."""
    import torch
    sums = torch.empty(3, dtype=torch.float64, device="cuda")
    pd.pd_level_stats(q_fine.data_ptr(), q_coarse.data_ptr() if q_coarse is not None else None,
                      q_fine.numel(), sums.data_ptr(), _stream_ptr(stream))
    return sums


def autotune(mesh: Mesh, params, n_samples: int, stream=None):
    """pd_autotune: the fastest launch shape of this configuration and the
    time per step of every shape (-1 where the configuration cannot use it)."""
    shape = C.c_int32()
    us = np.zeros(pd.PD_N_SHAPES)
    pd.pd_autotune(mesh.h, C.byref(params), n_samples, _stream_ptr(stream), C.byref(shape), us.ctypes.data)
    return dict(shape=shape.value, us_per_step=us)


def qoi_grad(mesh: Mesh, params, s0=None, c=None, stream=None, as_tensors=False):
    """Peak reaction, its step, and dQ/ds0, dQ/dc per node (pd_qoi_grad).
    s0 / c: per-node fields (FP64 device tensors are passed as they are; other
    array-likes are uploaded once) or None for homogeneous.  The gradients come
    back as device tensors with as_tensors, else as NumPy arrays."""
    import torch
    dev = torch.device("cuda")

    def on_device(f):
        if f is None:
            return None
        if isinstance(f, torch.Tensor) and f.is_cuda and f.dtype == torch.float64:
            return f.detach().contiguous()
        return torch.as_tensor(np.asarray(f, dtype=np.float64), device=dev).contiguous()

    s0_t, c_t = on_device(s0), on_device(c)
    g0 = torch.empty(mesh.n_nodes, dtype=torch.float64, device=dev)
    gc = torch.empty(mesh.n_nodes, dtype=torch.float64, device=dev)
    Q = C.c_double()
    ns = C.c_int64()
    pd.pd_qoi_grad(mesh.h, C.byref(params), s0_t.data_ptr() if s0_t is not None else None,
                   c_t.data_ptr() if c_t is not None else None, g0.data_ptr(), gc.data_ptr(),
                   C.byref(Q), C.byref(ns), _stream_ptr(stream))
    if as_tensors:
        return dict(Q=Q.value, nstar=ns.value, dQ_ds0=g0, dQ_dc=gc)
    return dict(Q=Q.value, nstar=ns.value, dQ_ds0=g0.cpu().numpy(), dQ_dc=gc.cpu().numpy())


def mlmc_estimate(level_sums, stream=None):
    """Estimator from per-level (N, sum Y, sum Y^2) device tensors, via
    pd_mlmc_estimate.  Returns dict(estimate, sampling_variance, levels=[(mean,
    var, var_unbiased), ...])."""
    import torch
    sums = torch.stack(list(level_sums)).contiguous()
    L = sums.shape[0]
    out = np.zeros(2 + 3 * L)
    pd.pd_mlmc_estimate(sums.data_ptr(), L, out.ctypes.data, _stream_ptr(stream))
    return dict(estimate=out[0], sampling_variance=out[1],
                levels=[tuple(out[2 + 3 * l: 5 + 3 * l]) for l in range(L)])


def peak_load_function():
    """torch.autograd.Function: peak reaction of one sample as a function of
    its per-node s0 and c fields (FP64 device tensors [n_nodes]).  When a
    gradient is wanted the forward runs the hand-written adjoint
    (pd_qoi_grad: the forward solve, then the reverse sweep) and keeps
    dQ/ds0 and dQ/dc on the device for backward; otherwise it runs the
    forward solve alone (pd_run_batch).  The fields never leave the device."""
    import torch

    class PeakLoad(torch.autograd.Function):
        @staticmethod
        def forward(ctx, s0, c, mesh, params):
            if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
                out = qoi_grad(mesh, params, s0, c, as_tensors=True)
                ctx.save_for_backward(out["dQ_ds0"], out["dQ_dc"])
                return torch.tensor(out["Q"], dtype=torch.float64, device=s0.device)
            dtype = s0.dtype
            item = BatchItem(mesh, params, 1, s0.detach().reshape(1, -1).contiguous(),
                             c.detach().to(dtype).reshape(1, -1).contiguous())
            (Q, ns, st), = run_batch([item])
            return Q[0].clone()

        @staticmethod
        def backward(ctx, g):
            gs0, gc = ctx.saved_tensors
            return g * gs0, g * gc, None, None

    return PeakLoad
