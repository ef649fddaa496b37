// Random material fields (paper section 5: KL expansion, lognormal marginal)
// and the FP64 MLMC level sums (section 4: Eq. MC_estimator, Eq.
// sample_variance).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "pd_internal.h"

namespace pdmi {
int kl_basis(const pd_mesh_s *m, double corr_len, int n_modes, int n_quad, std::vector<double> &lam,
             std::vector<double> &phi);

// out[s][i] = exp(mu + sigma * sum_m sqrt(lam_m) phi_m[i] xi[s][m]); one block
// row per sample so xi[s][*] is a uniform (scalar) load.
template <typename O>
__global__ void kl_field_kernel(const double *__restrict__ phi, const double *__restrict__ sqrt_lam,
                                const double *__restrict__ xi, int n_modes, int64_t M, double mu, double sigma,
                                O *__restrict__ out)
{
    const int64_t s = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const double *x = xi + s * n_modes;
    double g = 0.0;
    for (int m = 0; m < n_modes; ++m) g = fma(sqrt_lam[m] * x[m], phi[(int64_t)m * M + i], g);
    out[s * M + i] = (O)exp(fma(sigma, g, mu));
}

// sums = (N, sum Y, sum Y^2) in FP64: each thread adds a strided subset in
// index order, then a fixed-shape tree combines the 256 partials, so the
// result does not depend on scheduling.
__global__ __launch_bounds__(256) void level_sums_kernel(const double *qf, const double *qc, int64_t n, double *sums)
{
    __shared__ double p1[256], p2[256];
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        double y = qc ? qf[i] - qc[i] : qf[i];
        a += y;
        b = fma(y, y, b);
    }
    p1[threadIdx.x] = a;
    p2[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            p1[threadIdx.x] += p1[threadIdx.x + w];
            p2[threadIdx.x] += p2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sums[0] = (double)n;
        sums[1] = p1[0];
        sums[2] = p2[0];
    }
}

}  // namespace pdmi

using namespace pdmi;


namespace pdmi {

// ---------------------------------------------------------------- multilevel CDF
static unsigned cdf_blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

// Order statistics by exact ranking: rank(i) = #{j : q_j < q_i, or q_j = q_i
// and j < i}, so ties keep their input order and the result is deterministic.
__global__ void rank_sort_kernel(const double *q, int64_t n, double *sorted)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double qi = q[i];
    int64_t r = 0;
    for (int64_t j = 0; j < n; ++j) {
        const double qj = q[j];
        r += (qj < qi) || (qj == qi && j < i);
    }
    sorted[r] = qi;
}

struct CdfLevels {
    const double *fine[PD_MAX_CDF_LEVELS];
    const double *coarse[PD_MAX_CDF_LEVELS];
    int64_t n[PD_MAX_CDF_LEVELS];
    int n_levels;
};

// F^-1(u) = R_0[ceil(N_0 u)] + sum_l (R_l[ceil(N_l u)] - Rc_l[ceil(N_l u)]),
// R sorted fine samples, Rc the sorted coarse partners of level l (1-based
// order statistics, index clamped to 1..N_l).
__global__ void ml_quantile_kernel(CdfLevels lv, const double *u, int64_t nu, double *x)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nu) return;
    double v = 0.0;
    for (int l = 0; l < lv.n_levels; ++l) {
        const int64_t N = lv.n[l];
        int64_t idx = (int64_t)ceil((double)N * u[k]);
        idx = idx < 1 ? 1 : (idx > N ? N : idx);
        v += lv.fine[l][idx - 1];
        if (l > 0) v -= lv.coarse[l][idx - 1];
    }
    x[k] = v;
}

// Empirical CDF of the n values at the query points: #{values <= x} / n.
__global__ void ecdf_kernel(const double *values, int64_t n, const double *xq, int64_t nx, double *cdf)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nx) return;
    const double x = xq[m];
    int64_t c = 0;
    for (int64_t j = 0; j < n; ++j) c += values[j] <= x;
    cdf[m] = (double)c / (double)n;
}

}  // namespace pdmi

extern "C" {

int pd_kl_build(pd_mesh m, double corr_len, int32_t n_modes, int32_t n_quad, pd_kl *out)
{
    if (!m || !out) return fail(PD_EINVAL, "null argument");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(PD_EDEVICE, "no HIP device: the solver needs an MI355X (gfx950)");
    std::vector<double> lam, phi;
    int rc = kl_basis(m, corr_len, n_modes, n_quad, lam, phi);
    if (rc) return rc;
    pd_kl_s *k = new (std::nothrow) pd_kl_s();
    if (!k) return fail(PD_ENOMEM, "out of host memory");
    k->mesh = m;
    k->n_modes = (int)lam.size();
    k->lam = lam;
    std::vector<double> sl(lam.size());
    for (size_t i = 0; i < lam.size(); ++i) sl[i] = std::sqrt(std::fmax(lam[i], 0.0));
    hipError_t e = hipMalloc(&k->d_phi, 8 * phi.size());
    if (e == hipSuccess) e = hipMemcpy(k->d_phi, phi.data(), 8 * phi.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&k->d_sqrt_lam, 8 * sl.size());
    if (e == hipSuccess) e = hipMemcpy(k->d_sqrt_lam, sl.data(), 8 * sl.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (k->d_phi) (void)hipFree(k->d_phi);
        if (k->d_sqrt_lam) (void)hipFree(k->d_sqrt_lam);
        delete k;
        return hip_fail(e, "KL basis upload");
    }
    *out = k;
    return PD_OK;
}

int pd_kl_eigenvalues(pd_kl kl, double *lam_out)
{
    if (!kl || !lam_out) return fail(PD_EINVAL, "null argument");
    for (int i = 0; i < kl->n_modes; ++i) lam_out[i] = kl->lam[i];
    return PD_OK;
}

int pd_kl_field(pd_kl kl, const double *xi_dev, int64_t n_samples, double mean, double cov, void *out_dev,
                int32_t out_dtype, void *stream)
{
    if (!kl || !xi_dev || !out_dev) return fail(PD_EINVAL, "null argument");
    if (n_samples < 0 || n_samples > 65535) return fail(PD_EINVAL, "n_samples must be in [0, 65535]");
    if (!(mean > 0) || !(cov >= 0)) return fail(PD_EINVAL, "mean must be positive and cov non-negative");
    if (n_samples == 0) return PD_OK;
    double sigma2 = std::log1p(cov * cov);
    double mu = std::log(mean) - 0.5 * sigma2, sigma = std::sqrt(sigma2);
    int64_t M = kl->mesh->M;
    dim3 grid((unsigned)((M + 255) / 256), (unsigned)n_samples);
    hipStream_t st = (hipStream_t)stream;
    if (out_dtype == PD_DTYPE_F64)
        kl_field_kernel<double><<<grid, 256, 0, st>>>(kl->d_phi, kl->d_sqrt_lam, xi_dev, kl->n_modes, M, mu, sigma,
                                                      (double *)out_dev);
    else if (out_dtype == PD_DTYPE_F32)
        kl_field_kernel<float><<<grid, 256, 0, st>>>(kl->d_phi, kl->d_sqrt_lam, xi_dev, kl->n_modes, M, mu, sigma,
                                                     (float *)out_dev);
    else
        return fail(PD_EINVAL, "unknown dtype %d", out_dtype);
    PD_HIP(hipGetLastError());
    return PD_OK;
}

int pd_kl_free(pd_kl kl)
{
    if (!kl) return PD_OK;
    if (kl->d_phi) (void)hipFree(kl->d_phi);
    if (kl->d_sqrt_lam) (void)hipFree(kl->d_sqrt_lam);
    if (kl->d_qpos) (void)hipFree(kl->d_qpos);
    if (kl->d_ext) (void)hipFree(kl->d_ext);
    delete kl;
    return PD_OK;
}

int pd_level_stats(const double *q_fine_dev, const double *q_coarse_dev, int64_t n, double *sums_dev, void *stream)
{
    if (!q_fine_dev || !sums_dev) return fail(PD_EINVAL, "null argument");
    if (n < 1) return fail(PD_EINVAL, "n must be positive");
    level_sums_kernel<<<1, 256, 0, (hipStream_t)stream>>>(q_fine_dev, q_coarse_dev, n, sums_dev);
    PD_HIP(hipGetLastError());
    return PD_OK;
}

int pd_mlmc_estimate(const double *sums_dev, int32_t n_levels, double *out_host, void *stream)
{
    if (!sums_dev || !out_host || n_levels < 1) return fail(PD_EINVAL, "bad arguments");
    std::vector<double> sums(3 * (size_t)n_levels);
    PD_HIP(hipMemcpyAsync(sums.data(), sums_dev, 8 * sums.size(), hipMemcpyDeviceToHost, (hipStream_t)stream));
    PD_HIP(hipStreamSynchronize((hipStream_t)stream));
    double est = 0.0, var = 0.0;
    for (int l = 0; l < n_levels; ++l) {
        const double n = sums[3 * l], s1 = sums[3 * l + 1], s2 = sums[3 * l + 2];
        if (!(n >= 1)) return fail(PD_EINVAL, "level %d has no samples", l);
        const double mean = s1 / n;
        const double v = s2 / n - mean * mean;                // Eq. sample_variance
        const double vu = n > 1 ? v * n / (n - 1) : NAN;
        out_host[2 + 3 * l] = mean;
        out_host[3 + 3 * l] = v;
        out_host[4 + 3 * l] = vu;
        est += mean;                                          // Eq. MLMC_estimator
        var += v / n;                                         // sampling error of Eq. MLMC_error
    }
    out_host[0] = est;
    out_host[1] = var;
    return PD_OK;
}

int pd_mlmc_cdf(const double *const *q_fine_dev, const double *const *q_coarse_dev, const int64_t *n_samples,
                int32_t n_levels, const double *u_host, int64_t n_u, double *quantiles_host, const double *x_host,
                int64_t n_x, double *cdf_host, void *stream)
{
    if (!q_fine_dev || !n_samples || !u_host || !quantiles_host) return fail(PD_EINVAL, "null argument");
    if (n_levels < 1 || n_levels > PD_MAX_CDF_LEVELS) return fail(PD_EINVAL, "n_levels must be 1..%d", PD_MAX_CDF_LEVELS);
    if (n_u < 1) return fail(PD_EINVAL, "n_u must be positive");
    if (n_x < 0 || (n_x > 0 && (!x_host || !cdf_host))) return fail(PD_EINVAL, "bad CDF query");
    for (int l = 0; l < n_levels; ++l) {
        if (n_samples[l] < 1 || n_samples[l] > ((int64_t)1 << 24)) return fail(PD_EINVAL, "level %d: bad sample count", l);
        if (!q_fine_dev[l] || (l > 0 && (!q_coarse_dev || !q_coarse_dev[l])))
            return fail(PD_EINVAL, "level %d: missing samples", l);
    }
    for (int64_t k = 0; k < n_u; ++k)
        if (!(u_host[k] > 0.0 && u_host[k] <= 1.0)) return fail(PD_EINVAL, "u[%lld] must lie in (0, 1]", (long long)k);
    hipStream_t st = (hipStream_t)stream;
    int64_t total = 0;
    for (int l = 0; l < n_levels; ++l) total += (l > 0 ? 2 : 1) * n_samples[l];
    double *buf = nullptr;
    const size_t bytes = 8 * (size_t)(total + 2 * n_u + 2 * n_x);
    PD_HIP(hipMalloc(&buf, bytes));
    CdfLevels lv{};
    lv.n_levels = n_levels;
    double *p = buf;
    for (int l = 0; l < n_levels; ++l) {
        const int64_t N = n_samples[l];
        lv.n[l] = N;
        lv.fine[l] = p;
        rank_sort_kernel<<<cdf_blocks(N), 256, 0, st>>>(q_fine_dev[l], N, p);
        p += N;
        if (l > 0) {
            lv.coarse[l] = p;
            rank_sort_kernel<<<cdf_blocks(N), 256, 0, st>>>(q_coarse_dev[l], N, p);
            p += N;
        }
    }
    double *du = p, *dx = p + n_u, *dq = p + n_u + n_x, *dc = p + 2 * n_u + n_x;
    hipError_t e = hipMemcpyAsync(du, u_host, 8 * n_u, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && n_x) e = hipMemcpyAsync(dx, x_host, 8 * n_x, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        ml_quantile_kernel<<<cdf_blocks(n_u), 256, 0, st>>>(lv, du, n_u, dq);
        if (n_x) ecdf_kernel<<<cdf_blocks(n_x), 256, 0, st>>>(dq, n_u, dx, n_x, dc);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(quantiles_host, dq, 8 * n_u, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && n_x) e = hipMemcpyAsync(cdf_host, dc, 8 * n_x, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (e != hipSuccess) return hip_fail(e, "pd_mlmc_cdf");
    return PD_OK;
}

int pd_mlmc_allocation(const double *V, const double *C, int32_t n_levels, double eps_s, double *n_real_out,
                       int64_t *n_out)
{
    if (!V || !C || !n_out || n_levels < 1) return fail(PD_EINVAL, "bad arguments");
    if (!(eps_s > 0) || !std::isfinite(eps_s)) return fail(PD_EINVAL, "eps_s must be positive and finite");
    double sum = 0.0;
    for (int l = 0; l < n_levels; ++l) {
        if (!(V[l] >= 0) || !std::isfinite(V[l])) return fail(PD_EINVAL, "level %d: variance must be >= 0", l);
        if (!(C[l] > 0) || !std::isfinite(C[l])) return fail(PD_EINVAL, "level %d: cost must be > 0", l);
        sum += std::sqrt(V[l] * C[l]);
    }
    const double scale = sum / (eps_s * eps_s);
    for (int l = 0; l < n_levels; ++l) {
        const double real = scale * std::sqrt(V[l] / C[l]);          // Eq. sample_allocation
        if (real > 9.0e18) return fail(PD_EINVAL, "level %d: %g samples do not fit an int64", l, real);
        if (n_real_out) n_real_out[l] = real;
        n_out[l] = (int64_t)std::floor(real);
    }
    return PD_OK;
}

int pd_mlmc_bias(double y_last_mean, double alpha, double refinement, double r, double *bias_out)
{
    if (!bias_out) return fail(PD_EINVAL, "null output");
    const double den = r * std::pow(refinement, alpha) - 1.0;         // Eq. bias_error
    if (!(den > 0) || !std::isfinite(den)) return fail(PD_EINVAL, "r * refinement^alpha must exceed 1");
    *bias_out = std::fabs(y_last_mean) / den;
    return PD_OK;
}

int pd_mlmc_fit_rate(const double *x, const double *y, int32_t n, double *slope_out, double *intercept_out)
{
    if (!x || !y || !slope_out || n < 2) return fail(PD_EINVAL, "need at least two points");
    double sx = 0, sy = 0, sxx = 0, sxy = 0;
    for (int i = 0; i < n; ++i) {
        if (!(x[i] > 0) || !(std::fabs(y[i]) > 0)) return fail(PD_EINVAL, "point %d: x must be > 0 and y nonzero", i);
        const double lx = std::log(x[i]), ly = std::log(std::fabs(y[i]));
        sx += lx;
        sy += ly;
        sxx += lx * lx;
        sxy += lx * ly;
    }
    const double den = n * sxx - sx * sx;
    if (!(std::fabs(den) > 0)) return fail(PD_EINVAL, "x values must differ");
    const double b = (n * sxy - sx * sy) / den;
    *slope_out = b;
    if (intercept_out) *intercept_out = (sy - b * sx) / n;
    return PD_OK;
}

}  // extern "C"
