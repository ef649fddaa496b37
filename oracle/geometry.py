"""Oracle geometry: lattice, horizon neighbourhoods, notch cut, pads.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU
baseline).  Plain NumPy, written for readability.

* Lattice: a regular cubic grid of cell-centred nodes, node (i, j, k) at
  ((i + 1/2) dx, (j + 1/2) dx, (k + 1/2) dx), x index fastest.  With this
  convention an L x D body at spacing dx has (L/dx)(D/dx) nodes, which is how
  the paper's level table counts nodes (section 6.2, Table discretisation).
* Horizon: x' is a neighbour of x when |x' - x| <= delta = m dx
  (section 2.1, Eq. PD_Horizon; m = 3.14, section 6.2).  On the lattice this is
  the set of integer offsets v != 0 with |v|^2 <= m^2.
* Notch: a zero-width cut in the plane x = x_n from the bottom face up to
  height a, through the whole thickness (section 6.2 set-up).  A bond is
  removed when its segment crosses that plane strictly below the notch tip;
  the crossing test is half-open in x (x_lo < x_n <= x_hi) so a node lying on
  the plane belongs to the right-hand side.
* Pads: nodes whose centre lies inside a support or load block.
"""
from __future__ import annotations

import numpy as np


def grid_shape(extent, dx):
    """Number of cells per axis; each extent must be a whole number of dx."""
    n = []
    for L in extent:
        r = L / dx
        k = int(round(r))
        if abs(r - k) > 1e-9 * max(1.0, r) or k < 1:
            raise ValueError(f"extent {L} is not a multiple of dx {dx}")
        n.append(k)
    return tuple(n)


def node_positions(shape, dx):
    nx, ny, nz = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([(i + 0.5) * dx, (j + 0.5) * dx, (k + 0.5) * dx], axis=-1)
    return pos.reshape(-1, 3)


def stencil(m_ratio):
    """Integer offsets inside the horizon, as an [n, 3] int array."""
    r = int(np.ceil(m_ratio))
    out = []
    for vz in range(-r, r + 1):
        for vy in range(-r, r + 1):
            for vx in range(-r, r + 1):
                n2 = vx * vx + vy * vy + vz * vz
                if 0 < n2 and n2 <= m_ratio * m_ratio:
                    out.append((vx, vy, vz))
    return np.array(out, dtype=np.int64)


def unique_bonds(shape, m_ratio):
    """All neighbour pairs (i, j), i < j, as two int64 arrays plus the integer
    offset v = (grid position of j) - (grid position of i)."""
    nx, ny, nz = shape
    ii, jj, vv = [], [], []
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    idx = i + nx * (j + ny * k)
    for v in stencil(m_ratio):
        i2, j2, k2 = i + v[0], j + v[1], k + v[2]
        ok = (i2 >= 0) & (i2 < nx) & (j2 >= 0) & (j2 < ny) & (k2 >= 0) & (k2 < nz)
        a = idx[ok]
        b = (i2 + nx * (j2 + ny * k2))[ok]
        keep = a < b
        ii.append(a[keep]); jj.append(b[keep])
        vv.append(np.broadcast_to(v, (int(keep.sum()), 3)))
    bi = np.concatenate(ii); bj = np.concatenate(jj); v = np.concatenate(vv)
    order = np.lexsort((bj, bi))
    return bi[order], bj[order], v[order]


def _half_units(value, dx, what):
    r = 2.0 * value / dx
    k = int(round(r))
    if abs(r - k) > 1e-9 * max(1.0, abs(r)):
        raise ValueError(f"{what} {value} is not a multiple of dx/2")
    return k


def notch_cut_mask(shape, dx, bi, bj, x_notch, notch_depth):
    """Boolean mask over bonds: True where the bond crosses the notch.

    Work in half-cell units, where node centres sit at odd integers: node i
    on an axis is at 2 i + 1.  The plane is X_n = 2 x_n / dx and the tip
    A = 2 a / dx; both must be integers.  For a bond with endpoints ordered so
    that X1 <= X2 the crossing height is Z1 + (X_n - X1)(Z2 - Z1)/(X2 - X1); the
    bond is cut when X1 < X_n <= X2 and that height is below A.  Multiplying
    through by X2 - X1 > 0 keeps the test in exact integers."""
    if notch_depth <= 0:
        return np.zeros(bi.shape, dtype=bool)
    nx, ny, _ = shape
    Xn = _half_units(x_notch, dx, "notch position")
    A = _half_units(notch_depth, dx, "notch depth")
    xa = 2 * (bi % nx) + 1; za = 2 * (bi // (nx * ny)) + 1
    xb = 2 * (bj % nx) + 1; zb = 2 * (bj // (nx * ny)) + 1
    swap = xa > xb
    X1 = np.where(swap, xb, xa); Z1 = np.where(swap, zb, za)
    X2 = np.where(swap, xa, xb); Z2 = np.where(swap, za, zb)
    crosses = (X1 < Xn) & (Xn <= X2)
    dX = X2 - X1
    below = Z1 * dX + (Xn - X1) * (Z2 - Z1) < A * dX
    return crosses & below


def box_nodes(shape, dx, x_range, z_range):
    """Nodes whose centre lies strictly inside x_range x [all y] x z_range.
    A centre lying on a box face is rejected as ambiguous."""
    pos = node_positions(shape, dx)
    eps = 1e-9 * dx
    for lo, hi, c in ((x_range[0], x_range[1], pos[:, 0]), (z_range[0], z_range[1], pos[:, 2])):
        if np.any(np.abs(c - lo) < eps) or np.any(np.abs(c - hi) < eps):
            raise ValueError("a node centre lies on a pad face")
    inside = ((pos[:, 0] > x_range[0]) & (pos[:, 0] < x_range[1]) &
              (pos[:, 2] > z_range[0]) & (pos[:, 2] < z_range[1]))
    return np.nonzero(inside)[0].astype(np.int64)


def beam_pads(shape, dx, beam):
    """Support pads (bottom, centred on x = L/2 -+ span/2) and the load pad
    (top, centred on x = L/2), each pad_width wide and pad_width tall."""
    L, D, w = beam.length, beam.depth, beam.pad_width
    xs = (0.5 * (L - beam.span), 0.5 * (L + beam.span))
    sup = np.concatenate([box_nodes(shape, dx, (x - 0.5 * w, x + 0.5 * w), (0.0, w)) for x in xs])
    load = box_nodes(shape, dx, (0.5 * L - 0.5 * w, 0.5 * L + 0.5 * w), (D - w, D))
    return np.sort(sup), np.sort(load)
