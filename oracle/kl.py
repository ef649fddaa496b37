"""Oracle Karhunen-Loeve random field (paper section 5, KL expansion).

TEST INFRASTRUCTURE ONLY.  Plain NumPy in FP64.

The per-node limit stretch is a lognormal field s0(x) = exp(mu + sigma g(x))
built from a zero-mean unit-variance Gaussian field g with squared-exponential
correlation rho(r) = exp(-r^2 / (2 l^2)), expanded in its leading KL modes:
g(x) = sum_m sqrt(lambda_m) phi_m(x) xi_m with independent standard normal
xi_m.  The mean and coefficient of variation of s0 fix
sigma^2 = ln(1 + CoV^2) and mu = ln(mean) - sigma^2 / 2.

The squared-exponential kernel on a box is a product of 1D kernels, so the
3D eigenpairs are products of 1D eigenpairs (lambda = lambda_x lambda_y
lambda_z, phi = phi_x phi_y phi_z).  Each 1D eigenproblem
int_0^L k(x, y) phi(y) dy = lambda phi(x) is solved by the Nystrom method on
an n-point Gauss-Legendre rule: with weights W the symmetric matrix
W^1/2 K W^1/2 has eigenvectors psi and phi(x_k) = psi_k / sqrt(w_k); phi at any
other point follows from the integral equation itself,
phi(x) = (1/lambda) sum_k w_k k(x, x_k) phi(x_k).

Conventions shared with the product (they are choices, not the paper's):
* sign: each 1D eigenfunction is positive at the left end of its interval;
* ranking: 3D modes by decreasing lambda; products equal to a relative 1e-9
  are ordered by their (a, b, c) 1D indices, lexicographically;
* the same continuous modes are evaluated at each level's node centres, so a
  coefficient vector xi gives the same field on every level.
"""
from __future__ import annotations

import numpy as np


def kernel(x, y, corr_len):
    d = np.subtract.outer(x, y)
    return np.exp(-d * d / (2.0 * corr_len * corr_len))


class Basis1D:
    def __init__(self, length, corr_len, n_quad):
        t, w = np.polynomial.legendre.leggauss(n_quad)
        self.x = 0.5 * length * (t + 1.0)
        self.w = 0.5 * length * w
        self.length, self.corr_len = length, corr_len
        sw = np.sqrt(self.w)
        A = sw[:, None] * kernel(self.x, self.x, corr_len) * sw[None, :]
        lam, psi = np.linalg.eigh(A)
        order = np.argsort(lam)[::-1]
        self.lam = lam[order]
        self.phi_nodes = psi[:, order] / sw[:, None]
        left = self.evaluate(np.array([0.0]), np.arange(len(self.lam)))[0]
        self.phi_nodes = self.phi_nodes * np.where(left < 0, -1.0, 1.0)[None, :]

    def evaluate(self, pts, modes):
        """phi_m(pts) for the given mode indices, [len(pts), len(modes)]."""
        Kx = kernel(np.asarray(pts, dtype=np.float64), self.x, self.corr_len)
        return (Kx * self.w[None, :]) @ self.phi_nodes[:, modes] / self.lam[modes][None, :]


def select_modes(lams, n_modes, tol=1e-9):
    """Top n_modes index triples of the separable spectrum."""
    lx, ly, lz = lams
    K = [min(n_modes, len(l)) for l in lams]
    cand = []
    for a in range(K[0]):
        for b in range(K[1]):
            for c in range(K[2]):
                cand.append((lx[a] * ly[b] * lz[c], a, b, c))
    cand.sort(key=lambda t: -t[0])
    groups, g = [], 0
    for i, t in enumerate(cand):
        if i > 0 and abs(cand[i - 1][0] - t[0]) > tol * abs(cand[i - 1][0]):
            g += 1
        groups.append(g)
    ranked = sorted(zip(groups, cand), key=lambda gt: (gt[0], gt[1][1], gt[1][2], gt[1][3]))
    return [(t[1], t[2], t[3], t[0]) for _, t in ranked[:n_modes]]


class Basis3D:
    def __init__(self, extent, corr_len, n_modes, n_quad=256):
        self.axes = [Basis1D(L, corr_len, n_quad) for L in extent]
        self.modes = select_modes([ax.lam for ax in self.axes], n_modes)
        self.lam = np.array([m[3] for m in self.modes])

    def eigenfunctions(self, positions):
        """[n_points, n_modes] values of the selected 3D eigenfunctions."""
        P = np.asarray(positions, dtype=np.float64)
        out = np.ones((P.shape[0], len(self.modes)))
        for d, ax in enumerate(self.axes):
            idx = np.array([m[d] for m in self.modes])
            out *= ax.evaluate(P[:, d], idx)
        return out

    def gaussian_field(self, positions, xi):
        """g = sum_m sqrt(lambda_m) phi_m xi_m; xi is [n_samples, n_modes]."""
        Phi = self.eigenfunctions(positions)
        return np.asarray(xi) @ (np.sqrt(self.lam)[:, None] * Phi.T)


def lognormal_params(mean, cov):
    sigma2 = np.log1p(cov * cov)
    return np.log(mean) - 0.5 * sigma2, np.sqrt(sigma2)


def lognormal_field(basis, positions, xi, mean, cov):
    mu, sigma = lognormal_params(mean, cov)
    return np.exp(mu + sigma * basis.gaussian_field(positions, xi))
