"""Oracle problem assembly and the ctypes binding of the plain C time loop.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU
baseline).  Nothing in the product library imports this module.

Material constants (appendix A):
* micromodulus c = 12 E / (pi delta^4) in 3D, 9 E / (pi t delta^3) in plane
  stress and 48 E / (5 pi t delta^3) in plane strain
  (Eq. bond_stiffness_constant), nodal volume dx^3 or dx^2 t;
* per-bond values from per-node fields are endpoint means,
  c_b = (c_i + c_j)/2 and s0_b = (s0_i + s0_j)/2, so bond forces stay
  equal and opposite;
* critical stretch from the fracture-energy relation (computed in C).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import geometry as G

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LAW_EXPLIN = 0
LAW_TRILINEAR = 1


def build_sanitized(out: str) -> str:
    """The same source built with AddressSanitizer and UBSan (-O1, frame
    pointers kept) into `out`, for a host check of the oracle's memory
    accesses; load it with PD_ORACLE_LIB=<out> in a process that preloads
    sanitizer_runtime()."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", out,
                           _SRC, "-lm"])
    return out


def sanitizer_runtime() -> str:
    """gcc's AddressSanitizer runtime (to preload ahead of Python)."""
    return subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, no fast-math, OpenMP over the
    force loop's fixed bond chunks)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's force loop for calls made from this thread
    (n <= 0: unchanged); returns the count in use.  Results do not depend on
    it."""
    return int(lib().pdo_set_threads(int(n)))


class _Problem(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int64), ("n_bonds", C.c_int64),
        ("bond_i", C.c_void_p), ("bond_j", C.c_void_p), ("xi", C.c_void_p),
        ("s0_node", C.c_void_p), ("c_node", C.c_void_p),
        ("n_support", C.c_int64), ("support", C.c_void_p),
        ("n_load", C.c_int64), ("load", C.c_void_p),
        ("volume", C.c_double), ("rho", C.c_double), ("damping", C.c_double),
        ("dt", C.c_double), ("du", C.c_double), ("n_steps", C.c_int64),
        ("law", C.c_int32), ("k", C.c_double), ("alpha", C.c_double),
        ("GF", C.c_double), ("delta", C.c_double), ("load_offset", C.c_double), ("gf_node", C.c_void_p),
        ("thickness", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("PD_ORACLE_LIB")     # a sanitizer build of the same source
        if not path:
            path = _LIB
            if not os.path.exists(_LIB):
                build(force=False)
        L = C.CDLL(path)
        P = C.POINTER(_Problem)
        d, i64 = C.c_double, C.c_int64
        L.pdo_critical_stretch.restype = d
        L.pdo_critical_stretch.argtypes = [C.c_int32, d, d, d, d, d, d]
        L.pdo_critical_stretch_2d.restype = d
        L.pdo_critical_stretch_2d.argtypes = [C.c_int32, d, d, d, d, d, d, d]
        L.pdo_damage.restype = d
        L.pdo_damage.argtypes = [C.c_int32, d, d, d, d, d]
        L.pdo_force.restype = C.c_int
        L.pdo_force.argtypes = [P, C.c_void_p, C.c_void_p, C.c_void_p]
        L.pdo_stretch.restype = C.c_int
        L.pdo_stretch.argtypes = [P, C.c_void_p, C.c_void_p]
        L.pdo_keep_derivs.restype = None
        L.pdo_keep_derivs.argtypes = [C.c_int32, d, d, d, d, d, C.c_void_p]
        L.pdo_adjoint.restype = C.c_int
        L.pdo_adjoint.argtypes = [P, C.POINTER(d), C.POINTER(i64), C.c_void_p, C.c_void_p]
        L.pdo_set_threads.restype = C.c_int
        L.pdo_set_threads.argtypes = [C.c_int]
        L.pdo_run.restype = C.c_int
        L.pdo_run.argtypes = [P, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(d), C.POINTER(i64),
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def run_many(problems, fn=None, **kw):
    """Runs problems[k].run(**kw) (or fn(problems[k])) for every k, in order of
    the list.  Few large problems run one after the other, each on all of the
    host's cores; many run side by side in a thread pool whose workers use one
    core each (the C loop releases the GIL)."""
    import concurrent.futures as cf
    call = fn if fn is not None else (lambda p: p.run(**kw))
    cores = max(1, set_threads(0))
    if len(problems) < cores:
        return [call(p) for p in problems]

    def one(p):
        set_threads(1)
        return call(p)
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        return list(ex.map(one, problems))


def micromodulus(E, delta):
    """3D bond stiffness constant, appendix A Eq. bond_stiffness_constant."""
    return 12.0 * E / (np.pi * delta ** 4)


def critical_stretch(law, s0, c, GF, delta, k, alpha):
    return lib().pdo_critical_stretch(law, s0, c, GF, delta, k, alpha)


def critical_stretch_2d(law, s0, c, GF, delta, h, k, alpha):
    return lib().pdo_critical_stretch_2d(law, s0, c, GF, delta, h, k, alpha)


def micromodulus_plane_stress(E, delta, t):
    """Appendix A, Eq. bond_stiffness_constant (plane stress)."""
    return 9.0 * E / (np.pi * t * delta ** 3)


def micromodulus_plane_strain(E, delta, t):
    """Appendix A, Eq. bond_stiffness_constant (plane strain)."""
    return 48.0 * E / (5.0 * np.pi * t * delta ** 3)


def damage(law, kappa, s0, sc, k, alpha):
    return lib().pdo_damage(law, kappa, s0, sc, k, alpha)


def keep_derivs(law, kappa, s0, sc, k, alpha):
    """(keep, d/dkappa, d/ds0, d/dsc) of keep = 1 - damage."""
    out = np.zeros(4)
    lib().pdo_keep_derivs(law, kappa, s0, sc, k, alpha, out.ctypes.data)
    return out


def _ptr(a):
    return a.ctypes.data if a is not None else None


@dataclass
class Problem:
    """A beam discretisation with everything the time loop needs."""
    shape: tuple
    dx: float
    bond_i: np.ndarray
    bond_j: np.ndarray
    xi: np.ndarray
    support: np.ndarray
    load: np.ndarray
    s0: np.ndarray
    c: np.ndarray
    rho: float
    damping: float
    dt: float
    du: float
    n_steps: int
    law: int
    k: float
    alpha: float
    GF: float
    delta: float
    load_offset: float = 0.0
    gf: object = None          # per-node fracture energy (N/m), or None: GF everywhere
    thickness: float = 0.0     # 0: 3D body; > 0: plane stress of this thickness

    @property
    def n_nodes(self):
        return int(np.prod(self.shape))

    @property
    def n_bonds(self):
        return int(self.bond_i.size)

    @property
    def volume(self):
        return self.dx ** 3 if self.thickness == 0 else self.dx ** 2 * self.thickness

    def _struct(self):
        self._keep = [np.ascontiguousarray(a) for a in
                      (self.bond_i.astype(np.int32), self.bond_j.astype(np.int32),
                       self.xi.astype(np.float64), self.s0.astype(np.float64),
                       self.c.astype(np.float64), self.support.astype(np.int32),
                       self.load.astype(np.int32))]
        bi, bj, xi, s0, c, sup, ld = self._keep
        gf = None
        if self.gf is not None:
            gf = np.ascontiguousarray(np.asarray(self.gf, dtype=np.float64))
            self._keep.append(gf)
        return _Problem(self.n_nodes, self.n_bonds, _ptr(bi), _ptr(bj), _ptr(xi), _ptr(s0), _ptr(c),
                        sup.size, _ptr(sup), ld.size, _ptr(ld), self.volume, self.rho,
                        self.damping, self.dt, self.du, self.n_steps, self.law, self.k,
                        self.alpha, self.GF, self.delta, self.load_offset,
                        None if gf is None else gf.ctypes.data, self.thickness)

    def force(self, u, kappa=None):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.n_nodes, 3)
        L = np.zeros((self.n_nodes, 3))
        st = self._struct()
        if kappa is not None:
            assert kappa.dtype == np.float64 and kappa.flags.c_contiguous
        rc = lib().pdo_force(C.byref(st), _ptr(u), _ptr(kappa), _ptr(L))
        assert rc == 0
        return L

    def stretch(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.n_nodes, 3)
        s = np.zeros(self.n_bonds)
        st = self._struct()
        lib().pdo_stretch(C.byref(st), _ptr(u), _ptr(s))
        return s

    def adjoint(self):
        """Peak reaction, its step and dQ/ds0, dQ/dc per node (discrete
        adjoint of run(); starts from rest)."""
        Q = C.c_double(0.0); ns = C.c_int64(0)
        g0 = np.zeros(self.n_nodes); gc = np.zeros(self.n_nodes)
        st = self._struct()
        rc = lib().pdo_adjoint(C.byref(st), C.byref(Q), C.byref(ns), _ptr(g0), _ptr(gc))
        assert rc == 0, rc
        return dict(Q=Q.value, nstar=ns.value, dQ_ds0=g0, dQ_dc=gc)

    def run(self, u_init=None, v_init=None, kappa_init=None, want_state=True):
        """Returns dict(Q, nstar, R, u, v, kappa)."""
        M, nb = self.n_nodes, self.n_bonds
        Q = C.c_double(0.0); ns = C.c_int64(0)
        R = np.zeros(self.n_steps)
        u = np.zeros((M, 3)) if want_state else None
        v = np.zeros((M, 3)) if want_state else None
        kap = np.zeros(nb) if want_state else None
        ui = None if u_init is None else np.ascontiguousarray(u_init, dtype=np.float64)
        vi = None if v_init is None else np.ascontiguousarray(v_init, dtype=np.float64)
        ki = None if kappa_init is None else np.ascontiguousarray(kappa_init, dtype=np.float64)
        st = self._struct()
        rc = lib().pdo_run(C.byref(st), _ptr(ui), _ptr(vi), _ptr(ki), C.byref(Q), C.byref(ns), _ptr(R),
                           _ptr(u), _ptr(v), _ptr(kap))
        assert rc == 0, rc
        return dict(Q=Q.value, nstar=ns.value, R=R, u=u, v=v, kappa=kap)


def beam_problem(level, s0=None, c=None, *, E=None, rho=None, GF=None, damping=None,
                 k=None, alpha=None, m_ratio=None, n_steps=None, du=None, law=None, gf=None):
    """Assemble the oracle problem for a workloads.Level.  s0 / c are per-node
    fields (default: homogeneous values)."""
    import workloads as W
    E = W.E_MODULUS if E is None else E
    rho = W.DENSITY if rho is None else rho
    GF = W.FRACTURE_ENERGY if GF is None else GF
    damping = W.DAMPING if damping is None else damping
    k = W.SOFT_K if k is None else k
    alpha = W.SOFT_ALPHA if alpha is None else alpha
    m_ratio = W.M_RATIO if m_ratio is None else m_ratio
    beam, dx = level.beam, level.dx
    plane = getattr(beam, "plane", False)
    # a plane-stress body is one node thick; its physical thickness enters
    # the micromodulus, the nodal volume and the critical stretch
    shape = G.grid_shape((beam.length, dx if plane else beam.thickness, beam.depth), dx)
    bi, bj, v = G.unique_bonds(shape, m_ratio)
    cut = G.notch_cut_mask(shape, dx, bi, bj, 0.5 * beam.length, beam.notch_depth)
    bi, bj, v = bi[~cut], bj[~cut], v[~cut]
    sup, load = G.beam_pads(shape, dx, beam)
    M = int(np.prod(shape))
    delta = m_ratio * dx
    s0 = np.full(M, W.S0_MEAN) if s0 is None else np.asarray(s0, dtype=np.float64)
    if not plane:
        c_ref = micromodulus(E, delta)
    elif getattr(beam, "plane_strain", False):
        c_ref = micromodulus_plane_strain(E, delta, beam.thickness)
    else:
        c_ref = micromodulus_plane_stress(E, delta, beam.thickness)
    c = np.full(M, c_ref) if c is None else np.asarray(c, dtype=np.float64)
    return Problem(shape=shape, dx=dx, bond_i=bi, bond_j=bj, xi=v.astype(np.float64) * dx,
                   support=sup, load=load, s0=s0, c=c, rho=rho, damping=damping,
                   dt=level.dt, du=level.du if du is None else du,
                   n_steps=level.n_steps if n_steps is None else n_steps,
                   law=level.law if law is None else law, k=k, alpha=alpha, GF=GF, delta=delta,
                   gf=None if gf is None else np.asarray(gf, dtype=np.float64),
                   thickness=beam.thickness if plane else 0.0)
