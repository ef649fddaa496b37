"""Oracle MC / MLMC estimators (paper section 4).

TEST INFRASTRUCTURE ONLY.  Plain NumPy in FP64.

* Y_l = Q_l - Q_{l-1} for l > 0 and Y_0 = Q_0, both evaluated on the same
  random input (section 4.2, telescoping sum);
* level mean Y_hat = (1/N) sum Y (Eq. MC_estimator);
* level variance s^2 = (1/N) sum Y^2 - Y_hat^2 (Eq. sample_variance), and the
  unbiased 1/(N-1) variant;
* MLMC estimate sum_l Y_hat_l (Eq. MLMC_estimator) and its sampling variance
  sum_l V_l / N_l (Eq. MLMC_error);
* optimal allocation N_l = eps^-2 (sum sqrt(V C)) sqrt(V_l / C_l)
  (Eq. sample_allocation), standard-MC count N = V / eps^2
  (Eq. MC_num_samples), both rounded down as in the paper's tables;
* cost growth exponents 2 + max(0, (gamma - beta)/alpha) for MLMC
  (Eq. MLMC_computational_cost) and 2 + gamma/alpha for standard MC;
* bias bound |Y_hat_L| / (r m^alpha - 1) (Eq. bias_error);
* convergence rates as least-squares slopes in log-log (section 4.2);
* the adaptive MLMC algorithm (section 4.3, Algorithm 1), with the garbled
  line read as "compute N_hat_l - N_l additional samples" and the RMSE budget
  split evenly: eps_s = eps_b = eps / sqrt(2) (section 4.3, error estimation);
* the multilevel inverse CDF and CDF (section 7): order statistics of each
  level's fine samples minus those of their coarse partners, at index
  ceil(N_l u), and the empirical CDF of those quantiles.
"""
from __future__ import annotations

import numpy as np


def level_sums(Y):
    Y = np.asarray(Y, dtype=np.float64)
    return Y.size, float(np.sum(Y)), float(np.sum(Y * Y))


def level_moments(n, s1, s2):
    """(mean, variance with 1/N, variance with 1/(N-1))."""
    mean = s1 / n
    var = s2 / n - mean * mean
    unbiased = var * n / (n - 1) if n > 1 else float("nan")
    return mean, var, unbiased


def differences(q_fine, q_coarse=None):
    """Y on a level from the coupled fine / coarse peak loads."""
    q_fine = np.asarray(q_fine, dtype=np.float64)
    if q_coarse is None:
        return q_fine.copy()
    return q_fine - np.asarray(q_coarse, dtype=np.float64)


def mlmc_estimate(levels):
    """levels: list of Y arrays, level 0 first.  Returns (estimate,
    sampling variance, per-level (N, mean, var))."""
    est, samp, per = 0.0, 0.0, []
    for Y in levels:
        n, s1, s2 = level_sums(Y)
        m, v, _ = level_moments(n, s1, s2)
        est += m
        samp += v / n
        per.append((n, m, v))
    return est, samp, per


def optimal_allocation(V, C, eps):
    V = np.asarray(V, dtype=np.float64); C = np.asarray(C, dtype=np.float64)
    real = eps ** -2 * np.sum(np.sqrt(V * C)) * np.sqrt(V / C)
    return real, np.floor(real).astype(np.int64)


def mc_samples(V, eps):
    real = V / eps ** 2
    return real, int(np.floor(real))


def cost_exponents(alpha, beta, gamma):
    return 2.0 + max(0.0, (gamma - beta) / alpha), 2.0 + gamma / alpha


def bias_bound(y_last, alpha, refinement, r=1.0):
    """Eq. bias_error.  It bounds the bias only for a positive rate
    (r m^alpha > 1); otherwise (a fitted rate at or below zero: the
    corrections do not decay) the bias is unbounded: +inf."""
    den = r * refinement ** alpha - 1.0
    return abs(y_last) / den if den > 0 else float("inf")


def fit_rate(x, y):
    """Slope and intercept of the least-squares line log|y| = a + b log x."""
    lx = np.log(np.asarray(x, dtype=np.float64))
    ly = np.log(np.abs(np.asarray(y, dtype=np.float64)))
    b, a = np.polyfit(lx, ly, 1)
    return float(b), float(a)


def adaptive(sampler, eps, costs, dofs, n_warm=100, alpha=None, alpha_default=0.5, refinement=8.0, r=1.0,
             max_levels=None):
    """Algorithm 1.  sampler(level, start, count) returns Y for samples
    start .. start+count-1 of that level (Y_0 = Q_0, Y_l = Q_l - Q_{l-1} on
    shared random inputs).  costs[l]: cost of one level-l sample; dofs[l]:
    degrees of freedom M_l (for fitting alpha).  alpha: weak rate for the bias
    estimate; None fits it from |Y_hat_l|, l >= 1, once two such levels exist,
    and uses alpha_default before.  Returns the per-level sample counts and
    sums, the estimate, its sampling variance, the bias estimate and the
    allocation history."""
    eps_s = eps_b = eps / np.sqrt(2.0)
    last = len(costs) - 1 if max_levels is None else max_levels - 1
    N, Y = [], []
    history = []
    L = 0
    converged = False
    while True:
        N.append(0)
        Y.append(np.zeros(0))
        # warm-up samples on the new level
        Y[L] = np.concatenate([Y[L], sampler(L, N[L], n_warm)])
        N[L] += n_warm
        # Eq. sample_variance can round below zero when Y barely varies
        V = [max(level_moments(*level_sums(Y[l]))[1], 0.0) for l in range(L + 1)]
        _, n_hat = optimal_allocation(V, costs[:L + 1], eps_s)
        for l in range(L + 1):
            extra = int(n_hat[l]) - N[l]
            if extra > 0:
                Y[l] = np.concatenate([Y[l], sampler(l, N[l], extra)])
                N[l] += extra
        means = [level_moments(*level_sums(Y[l]))[0] for l in range(L + 1)]
        if alpha is not None:
            a = alpha
        elif L >= 2:
            a = -fit_rate(dofs[1:L + 1], means[1:L + 1])[0]
        else:
            a = alpha_default
        bias = bias_bound(means[L], a, refinement, r)
        history.append(dict(L=L, V=list(V), n_hat=[int(v) for v in n_hat], N=list(N), alpha=a, bias=bias))
        if bias < eps_b:
            converged = True
            break
        if L == last:
            break
        L += 1
    est, samp, per = mlmc_estimate(Y)
    return dict(L=L, N=N, sums=[level_sums(y) for y in Y], estimate=est, sampling_variance=samp,
                bias=history[-1]["bias"], converged=converged, history=history, eps_s=eps_s, eps_b=eps_b)


def ml_inverse_cdf(fine, coarse, u):
    """F^-1(u) = R_0[ceil(N_0 u)] + sum_l (R_l[ceil(N_l u)] - Rc_l[ceil(N_l u)]);
    fine[l]: level-l samples, coarse[l]: their coarse partners (l >= 1)."""
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros(u.size)
    for l in range(len(fine)):
        f = np.sort(np.asarray(fine[l], dtype=np.float64))
        N = f.size
        idx = np.clip(np.ceil(N * u).astype(np.int64), 1, N) - 1
        out += f[idx]
        if l > 0:
            c = np.sort(np.asarray(coarse[l], dtype=np.float64))
            out -= c[idx]
    return out


def ecdf(values, x):
    """(1/n) #{values <= x} at each x."""
    v = np.sort(np.asarray(values, dtype=np.float64))
    return np.searchsorted(v, np.asarray(x, dtype=np.float64), side="right") / v.size
