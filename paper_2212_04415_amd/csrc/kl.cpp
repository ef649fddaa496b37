// Karhunen-Loeve basis of the squared-exponential Gaussian field on a box
// (paper section 5, KL expansion), built on the host in FP64.
//
// The kernel exp(-|x - y|^2 / (2 l^2)) factorises over the axes, so the
// eigenpairs on the box are products of 1D eigenpairs.  Each 1D integral
// eigenproblem int_0^L k(x, y) phi(y) dy = lambda phi(x) is discretised with an
// n-point Gauss-Legendre rule (Nystrom): B = W^1/2 K W^1/2 is symmetric, its
// eigenvectors psi give phi(x_q) = psi_q / sqrt(w_q), and phi anywhere else
// follows from the integral equation, phi(x) = sum_q w_q k(x, x_q) phi(x_q) /
// lambda.  B is diagonalised with cyclic Jacobi rotations.
#include <algorithm>
#include <cmath>
#include <vector>

#include "pd_internal.h"

namespace pdmi {

// Gauss-Legendre nodes / weights on [-1, 1] by Newton iteration on P_n.
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute the derivative at the converged root
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Cyclic Jacobi diagonalisation of the symmetric n x n matrix A (row-major,
// destroyed).  On return lam holds the eigenvalues and V (row-major) the
// eigenvectors as columns.
static void jacobi_eigen(std::vector<double> &A, int n, std::vector<double> &lam, std::vector<double> &V)
{
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    auto a = [&](int i, int j) -> double & { return A[(size_t)i * n + j]; };
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i) {
            diag += a(i, i) * a(i, i);
            for (int j = i + 1; j < n; ++j) off += a(i, j) * a(i, j);
        }
        if (off <= 1e-30 * diag) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = a(p, q);
                if (std::fabs(apq) < 1e-300) continue;
                double app = a(p, p), aqq = a(q, q);
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    double akp = a(k, p), akq = a(k, q);
                    a(k, p) = c * akp - s * akq;
                    a(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = a(p, k), aqk = a(q, k);
                    a(p, k) = c * apk - s * aqk;
                    a(q, k) = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = a(i, i);
}

struct Axis {
    double L, lc;
    std::vector<double> xq, wq;   // quadrature on [0, L]
    std::vector<double> lam;      // decreasing
    std::vector<double> phiq;     // [mode][q]: eigenfunction values at the quadrature points

    double eval(int mode, double x) const
    {
        double s = 0.0;
        for (size_t q = 0; q < xq.size(); ++q) {
            double d = x - xq[q];
            s += wq[q] * std::exp(-d * d / (2.0 * lc * lc)) * phiq[(size_t)mode * xq.size() + q];
        }
        return s / lam[mode];
    }
};

static void build_axis(Axis &ax, double L, double lc, int n)
{
    ax.L = L;
    ax.lc = lc;
    std::vector<double> t, w;
    gauss_legendre(n, t, w);
    ax.xq.resize(n);
    ax.wq.resize(n);
    for (int q = 0; q < n; ++q) {
        ax.xq[q] = 0.5 * L * (t[q] + 1.0);
        ax.wq[q] = 0.5 * L * w[q];
    }
    std::vector<double> B((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double d = ax.xq[i] - ax.xq[j];
            B[(size_t)i * n + j] = std::sqrt(ax.wq[i] * ax.wq[j]) * std::exp(-d * d / (2.0 * lc * lc));
        }
    std::vector<double> lam, V;
    jacobi_eigen(B, n, lam, V);
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return lam[a] > lam[b]; });
    ax.lam.resize(n);
    ax.phiq.assign((size_t)n * n, 0.0);
    for (int m = 0; m < n; ++m) {
        int c = order[m];
        ax.lam[m] = lam[c];
        for (int q = 0; q < n; ++q) ax.phiq[(size_t)m * n + q] = V[(size_t)q * n + c] / std::sqrt(ax.wq[q]);
    }
    // sign: each eigenfunction positive at the left end of the interval
    for (int m = 0; m < n; ++m) {
        if (!(ax.lam[m] > 0)) continue;
        if (ax.eval(m, 0.0) < 0)
            for (int q = 0; q < n; ++q) ax.phiq[(size_t)m * n + q] = -ax.phiq[(size_t)m * n + q];
    }
}

struct Mode3 {
    double lam;
    int a, b, c;
};

// The n_modes largest products lam_a lam_b lam_c; products equal to a
// relative 1e-9 are ordered by (a, b, c).
static std::vector<Mode3> select_modes(const Axis *ax, int n_modes)
{
    int K[3];
    for (int d = 0; d < 3; ++d) K[d] = std::min<int>(n_modes, (int)ax[d].lam.size());
    std::vector<Mode3> cand;
    for (int a = 0; a < K[0]; ++a)
        for (int b = 0; b < K[1]; ++b)
            for (int c = 0; c < K[2]; ++c) cand.push_back({ax[0].lam[a] * ax[1].lam[b] * ax[2].lam[c], a, b, c});
    std::stable_sort(cand.begin(), cand.end(), [](const Mode3 &x, const Mode3 &y) { return x.lam > y.lam; });
    std::vector<int> group(cand.size(), 0);
    for (size_t i = 1; i < cand.size(); ++i)
        group[i] = group[i - 1] + (std::fabs(cand[i - 1].lam - cand[i].lam) > 1e-9 * std::fabs(cand[i - 1].lam));
    std::vector<size_t> idx(cand.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
        if (group[x] != group[y]) return group[x] < group[y];
        const Mode3 &p = cand[x], &q = cand[y];
        if (p.a != q.a) return p.a < q.a;
        if (p.b != q.b) return p.b < q.b;
        return p.c < q.c;
    });
    std::vector<Mode3> out;
    for (int i = 0; i < n_modes && i < (int)idx.size(); ++i) out.push_back(cand[idx[i]]);
    return out;
}

int kl_basis(const pd_mesh_s *m, double corr_len, int n_modes, int n_quad, std::vector<double> &lam,
             std::vector<double> &phi)
{
    if (!(corr_len > 0)) return fail(PD_EINVAL, "corr_len must be positive");
    if (n_modes < 1 || n_quad < 2 || n_quad > 2048) return fail(PD_EINVAL, "bad n_modes or n_quad");
    if ((int64_t)n_modes > (int64_t)n_quad * n_quad * n_quad) return fail(PD_EINVAL, "n_modes too large for n_quad");
    Axis ax[3];
    for (int d = 0; d < 3; ++d) build_axis(ax[d], m->d.extent[d], corr_len, n_quad);
    std::vector<Mode3> modes = select_modes(ax, n_modes);
    int nm = (int)modes.size();
    lam.resize(nm);
    phi.assign((size_t)nm * m->M, 0.0);
    // 1D eigenfunctions at the node centres of each axis
    int n[3] = {m->nx, m->ny, m->nz};
    std::vector<std::vector<double>> tab(3);
    for (int d = 0; d < 3; ++d) {
        int used = 0;
        for (auto &md : modes) used = std::max(used, 1 + (d == 0 ? md.a : d == 1 ? md.b : md.c));
        tab[d].assign((size_t)used * n[d], 0.0);
        for (int k = 0; k < used; ++k)
            for (int i = 0; i < n[d]; ++i) tab[d][(size_t)k * n[d] + i] = ax[d].eval(k, (i + 0.5) * m->d.dx);
    }
    for (int q = 0; q < nm; ++q) {
        lam[q] = modes[q].lam;
        const double *fx = &tab[0][(size_t)modes[q].a * n[0]];
        const double *fy = &tab[1][(size_t)modes[q].b * n[1]];
        const double *fz = &tab[2][(size_t)modes[q].c * n[2]];
        double *out = &phi[(size_t)q * m->M];
        for (int k = 0; k < n[2]; ++k)
            for (int j = 0; j < n[1]; ++j)
                for (int i = 0; i < n[0]; ++i) out[i + (size_t)n[0] * (j + (size_t)n[1] * k)] = fx[i] * fy[j] * fz[k];
    }
    return PD_OK;
}

}  // namespace pdmi
