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

struct pd_kl_s {
    const pd_mesh_s *mesh = nullptr;
    int n_modes = 0;
    std::vector<double> lam;
    double *d_phi = nullptr;       // [n_modes][M]
    double *d_sqrt_lam = nullptr;  // [n_modes]
};

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
