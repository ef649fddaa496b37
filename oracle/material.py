"""Oracle: the paper's material model (section 5 and section 6.2).

TEST INFRASTRUCTURE ONLY.  Plain NumPy / SciPy in FP64.

* Exponential covariance rho(x, x') = exp(-|x - x'| / l_c), unit variance,
  Euclidean distance (section 5, Eq. exponential_correlation_function).
* KL basis by Nystrom's method with the midpoint rule on a reference lattice
  (node centres, weight w = dx^3 each): the eigenpairs of w K, phi_k(x_j) =
  psi_kj / sqrt(w), so that sum_j w phi_k(x_j)^2 = 1; modes are evaluated
  anywhere by the Nystrom extension phi_k(x) = (1 / lambda_k) sum_j w
  rho(x, x_j) phi_k(x_j), which reproduces phi_k at the reference nodes, so
  every level sees the same continuous field.
* Modes whose eigenvalues agree to 1e-8 (relative) form a cluster; a cluster
  spans a unique subspace but has no unique basis, so it is replaced by the
  Gram-Schmidt orthonormalisation of the projections of fixed probe vectors
  r_j(i) = cos((i + 1)(j + 1) 0.6180339887498949), j = 0, 1, ...; for a
  single mode this fixes the sign (<phi, r_0> > 0).  The kept set is the
  largest n_modes eigenvalues, extended to the end of a cluster it would
  split.
* Weibull marginal through the Gaussian copula (section 5, material strength
  distribution): f_c = lambda (-ln(1 - Phi(g)))^(1/m), lambda = f_cm /
  Gamma(1 + 1/m), with 1 - Phi(g) = Phi(-g).
* fib Model Code 2010 relations (cited in section 6.2, not printed):
  E = alpha_E 21.5 GPa (f_c / 10 MPa)^(1/3); f_t = 0.3 MPa (f_ck / MPa)^(2/3)
  with f_ck = max(f_c - 8 MPa, f_ck_min); G_F = 73 N/m (f_c / MPa)^0.18;
  then s0 = f_t / E and c = 12 E / (pi delta^4) (plane stress of thickness
  t: c = 9 E / (pi t delta^3)).  fib_properties is parity unpinned: the
  paper prints none of these relations and nothing independent of them is
  available to check them against.
"""
from __future__ import annotations

import numpy as np
from scipy import special

PROBE_STEP = 0.6180339887498949
CLUSTER_RTOL = 1e-8


def exp_kernel(X, Y, corr_len):
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    d = np.sqrt(np.maximum(np.sum(X * X, 1)[:, None] + np.sum(Y * Y, 1)[None, :] - 2.0 * X @ Y.T, 0.0))
    return np.exp(-d / corr_len)


def exp_kernel_exact(X, Y, corr_len):
    """Same kernel with the distance formed from coordinate differences."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    diff = X[:, None, :] - Y[None, :, :]
    return np.exp(-np.sqrt(np.sum(diff * diff, axis=2)) / corr_len)


def probes(n, m):
    i = np.arange(n, dtype=np.float64)[:, None] + 1.0
    j = np.arange(m, dtype=np.float64)[None, :] + 1.0
    return np.cos(i * j * PROBE_STEP)


def canonical_basis(lam, vecs):
    """lam descending, vecs[:, k] orthonormal eigenvectors.  Returns the
    cluster-canonical basis (same subspaces)."""
    n, K = vecs.shape
    out = np.empty_like(vecs)
    k = 0
    while k < K:
        e = k + 1
        while e < K and abs(lam[e] - lam[k]) <= CLUSTER_RTOL * abs(lam[k]):
            e += 1
        V = vecs[:, k:e]
        R = probes(n, e - k)
        basis = []
        for j in range(e - k):
            v = V @ (V.T @ R[:, j])
            for b in basis:
                v = v - b * np.dot(b, v)
            v = v / np.linalg.norm(v)
            basis.append(v)
        out[:, k:e] = np.stack(basis, axis=1)
        k = e
    return out


class ExpBasis:
    """KL basis of the exponential covariance on reference points X (n, 3)
    with equal quadrature weights w."""

    def __init__(self, X, weight, corr_len, n_modes):
        self.X = np.asarray(X, dtype=np.float64)
        self.w = float(weight)
        self.corr_len = float(corr_len)
        A = self.w * exp_kernel_exact(self.X, self.X, corr_len)
        lam, vec = np.linalg.eigh(A)
        lam, vec = lam[::-1], vec[:, ::-1]
        K = n_modes
        while K < lam.size and abs(lam[K] - lam[K - 1]) <= CLUSTER_RTOL * abs(lam[K - 1]):
            K += 1
        # canonicalise with one extra eigenpair of look-ahead so a cluster at
        # the end is recognised whole
        take = min(K + 1, lam.size)
        vec_c = canonical_basis(lam[:take], vec[:, :take])
        self.lam = lam[:K].copy()
        self.psi = vec_c[:, :K].copy()
        self.phi_ref = self.psi / np.sqrt(self.w)        # phi_k(x_j), columns = modes
        self.all_lam = lam

    @property
    def n_modes(self):
        return self.lam.size

    def evaluate(self, Y, chunk=4096):
        """phi_k at points Y (m, 3), Nystrom extension; returns (m, K)."""
        Y = np.asarray(Y, dtype=np.float64)
        coef = self.w * self.phi_ref / self.lam[None, :]
        out = np.empty((Y.shape[0], self.n_modes))
        for a in range(0, Y.shape[0], chunk):
            out[a:a + chunk] = exp_kernel_exact(Y[a:a + chunk], self.X, self.corr_len) @ coef
        return out

    def gaussian(self, phi, xi):
        """g = sum_k sqrt(lambda_k) phi_k xi_k for xi (S, K) -> (S, m)."""
        xi = np.atleast_2d(np.asarray(xi, dtype=np.float64))[:, :self.n_modes]
        return (xi * np.sqrt(self.lam)[None, :]) @ phi.T


# ---------------------------------------------------------------- marginal and fib maps
def weibull_from_gaussian(g, fcm, m):
    """f_c with a Weibull(m) marginal of mean fcm from standard-normal g."""
    lam_w = fcm / special.gamma(1.0 + 1.0 / m)
    q = special.ndtr(-np.asarray(g, dtype=np.float64))       # 1 - Phi(g)
    return lam_w * (-np.log(q)) ** (1.0 / m)


def fib_properties(fc, alpha_E=1.0, delta_f=8.0e6, fck_min=1.0e6):
    """(E, f_t, G_F) in SI from compressive strength fc (Pa).  Parity
    unpinned (the relations are a reading of a cited, unprinted code)."""
    fc = np.asarray(fc, dtype=np.float64)
    E = alpha_E * 21.5e9 * (fc / 10.0e6) ** (1.0 / 3.0)
    fck = np.maximum(fc - delta_f, fck_min)
    ft = 0.3e6 * (fck / 1.0e6) ** (2.0 / 3.0)
    GF = 73.0 * (fc / 1.0e6) ** 0.18
    return E, ft, GF


def material_fields(g, delta, fcm=42.3e6, m=3.0, alpha_E=1.0, delta_f=8.0e6, fck_min=1.0e6, thickness=0.0,
                    plane_strain=False):
    """Per-node (s0, c, G_F) from a standard-normal Gaussian field g; c in
    the 3D form, or for a body of thickness t > 0 the plane-stress form
    9 E / (pi t delta^3) or plane-strain form 48 E / (5 pi t delta^3) of
    appendix A (Eq. bond_stiffness_constant)."""
    fc = weibull_from_gaussian(g, fcm, m)
    E, ft, GF = fib_properties(fc, alpha_E, delta_f, fck_min)
    if thickness > 0:
        c = (48.0 / 5.0 if plane_strain else 9.0) * E / (np.pi * thickness * delta ** 3)
    else:
        c = 12.0 * E / (np.pi * delta ** 4)
    return ft / E, c, GF


# ---------------------------------------------------------------- 1D closed form (pins)
def exp_kernel_1d_eigenvalues(corr_len, half_length, n):
    """The n largest eigenvalues of exp(-|x - y| / l) on [-a, a]:
    lambda = 2 c / (omega^2 + c^2), c = 1 / l, with omega the roots of
    c - omega tan(omega a) = 0 (even modes) and omega + c tan(omega a) = 0
    (odd modes), one root per branch interval of tan."""
    from scipy.optimize import brentq
    c, a = 1.0 / corr_len, half_length
    roots = []
    for i in range(n + 2):
        lo, hi = i * np.pi / a, (i + 0.5) * np.pi / a
        f = lambda w: c * np.cos(w * a) - w * np.sin(w * a)
        roots.append(brentq(f, lo + 1e-12, hi - 1e-12))
        lo, hi = (i + 0.5) * np.pi / a, (i + 1) * np.pi / a
        g = lambda w: w * np.cos(w * a) + c * np.sin(w * a)
        roots.append(brentq(g, lo + 1e-12, hi - 1e-12))
    lam = np.sort(2 * c / (np.array(roots) ** 2 + c * c))[::-1]
    return lam[:n]
