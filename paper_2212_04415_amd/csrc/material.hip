// The paper's material model (section 5, section 6.2): exponential-covariance
// Karhunen-Loeve basis by Nystrom's method (dense symmetric eigensolver on
// the device), its Nystrom extension to other meshes, Gaussian field
// synthesis, and the Weibull-marginal / fib-relation map to per-node limit
// stretch, micromodulus and fracture energy.
#include <hip/hip_runtime.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "pd_internal.h"

namespace pdmi {

constexpr double kProbeStep = 0.6180339887498949;
constexpr double kClusterRtol = 1e-8;
constexpr int kMaxExpNodes = 20000;
constexpr int kModeChunk = 16;

// blocks for n elements along x, capped at 2^20 (kernels whose n can pass
// 2^28, the per-sample maps over several samples, loop with a grid stride)
static unsigned nblocks(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, int64_t(1) << 20); }

// node-centre positions of a mesh, [M][3]; a plane-stress body's nodes lie
// on the plane y = 0 whatever the spacing, so every level samples the field
// on the same plane
static std::vector<double> node_positions(const pd_mesh_s *m)
{
    std::vector<double> X(3 * (size_t)m->M);
    const double dx = m->d.dx;
    const bool plane = m->d.thickness > 0;
    for (int k = 0; k < m->nz; ++k)
        for (int j = 0; j < m->ny; ++j)
            for (int i = 0; i < m->nx; ++i) {
                const int64_t n = i + (int64_t)m->nx * (j + (int64_t)m->ny * k);
                X[3 * n] = (i + 0.5) * dx;
                X[3 * n + 1] = plane ? 0.0 : (j + 0.5) * dx;
                X[3 * n + 2] = (k + 0.5) * dx;
            }
    return X;
}

// A = w exp(-|x_i - x_j| / l), n x n (symmetric, so the storage order is moot)
__global__ void exp_matrix_kernel(const double *X, int64_t n, double w, double inv_l, double *A)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j = blockIdx.y;
    if (i >= n) return;
    const double dx = X[3 * i] - X[3 * j], dy = X[3 * i + 1] - X[3 * j + 1], dz = X[3 * i + 2] - X[3 * j + 2];
    A[i + n * j] = w * exp(-sqrt(dx * dx + dy * dy + dz * dz) * inv_l);
}

// phi_k(x_i) = sum_j rho(x_i, x_j) ext[k][j] for modes k0 .. k0 + 15 of this
// launch's chunk (blockIdx.y); ext[k][j] = w phi_k(x_j) / lambda_k.
__global__ void exp_extend_kernel(const double *Y, int64_t m, const double *X, int64_t n, const double *ext,
                                  int n_modes, double inv_l, double *phi)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k0 = blockIdx.y * kModeChunk;
    if (i >= m) return;
    const double yx = Y[3 * i], yy = Y[3 * i + 1], yz = Y[3 * i + 2];
    double acc[kModeChunk];
#pragma unroll
    for (int c = 0; c < kModeChunk; ++c) acc[c] = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        const double dx = yx - X[3 * j], dy = yy - X[3 * j + 1], dz = yz - X[3 * j + 2];
        const double r = exp(-sqrt(dx * dx + dy * dy + dz * dz) * inv_l);
#pragma unroll
        for (int c = 0; c < kModeChunk; ++c)
            if (k0 + c < n_modes) acc[c] = fma(r, ext[(int64_t)(k0 + c) * n + j], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < kModeChunk; ++c)
        if (k0 + c < n_modes) phi[(int64_t)(k0 + c) * m + i] = acc[c];
}

// g[s][i] = sum_k sqrt(lambda_k) phi_k[i] xi[s][k]
__global__ void gaussian_kernel(const double *phi, const double *sqrt_lam, const double *xi, int n_modes, int64_t M,
                                double *g)
{
    const int64_t s = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const double *x = xi + s * n_modes;
    double v = 0.0;
    for (int k = 0; k < n_modes; ++k) v = fma(sqrt_lam[k] * x[k], phi[(int64_t)k * M + i], v);
    g[s * M + i] = v;
}

struct FibConst {
    double lam_w, inv_m, alpha_E, delta_f, fck_min, c_scale;
};

template <typename O>
__global__ void fib_kernel(const double *g, int64_t n, FibConst f, O *s0, O *c, O *gf)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const double q = 0.5 * erfc(g[t] * 0.70710678118654752);     // 1 - Phi(g)
    const double fc = f.lam_w * pow(-log(q), f.inv_m);
    const double E = f.alpha_E * 21.5e9 * cbrt(fc / 10.0e6);
    const double fck = fmax(fc - f.delta_f, f.fck_min);
    const double ft = 0.3e6 * pow(fck / 1.0e6, 2.0 / 3.0);
    if (s0) s0[t] = (O)(ft / E);
    if (c) c[t] = (O)(f.c_scale * E);
    if (gf) gf[t] = (O)(73.0 * pow(fc / 1.0e6, 0.18));
    }
}

// Canonical basis of each cluster (eigenvalues equal to kClusterRtol): the
// Gram-Schmidt orthonormalisation of the projections of the probe vectors.
// vec: [K][n], mode k contiguous; lam descending.
static void canonicalise(const std::vector<double> &lam, std::vector<double> &vec, int64_t n, int K)
{
    std::vector<double> r(n), v(n), coef;
    int k = 0;
    while (k < K) {
        int e = k + 1;
        while (e < K && std::fabs(lam[e] - lam[k]) <= kClusterRtol * std::fabs(lam[k])) ++e;
        const int sz = e - k;
        std::vector<double> basis((size_t)sz * n);
        for (int j = 0; j < sz; ++j) {
            for (int64_t i = 0; i < n; ++i) r[i] = std::cos((double)(i + 1) * (double)(j + 1) * kProbeStep);
            coef.assign(sz, 0.0);
            for (int a = 0; a < sz; ++a) {
                const double *va = &vec[(size_t)(k + a) * n];
                double d = 0.0;
                for (int64_t i = 0; i < n; ++i) d += va[i] * r[i];
                coef[a] = d;
            }
            std::fill(v.begin(), v.end(), 0.0);
            for (int a = 0; a < sz; ++a) {
                const double *va = &vec[(size_t)(k + a) * n];
                for (int64_t i = 0; i < n; ++i) v[i] += coef[a] * va[i];
            }
            for (int b = 0; b < j; ++b) {
                const double *bb = &basis[(size_t)b * n];
                double d = 0.0;
                for (int64_t i = 0; i < n; ++i) d += bb[i] * v[i];
                for (int64_t i = 0; i < n; ++i) v[i] -= d * bb[i];
            }
            double nrm = 0.0;
            for (int64_t i = 0; i < n; ++i) nrm += v[i] * v[i];
            nrm = std::sqrt(nrm);
            for (int64_t i = 0; i < n; ++i) basis[(size_t)j * n + i] = v[i] / nrm;
        }
        std::copy(basis.begin(), basis.end(), vec.begin() + (size_t)k * n);
        k = e;
    }
}

struct DevMem {
    std::vector<void *> p;
    int get(void **q, size_t bytes)
    {
        hipError_t e = hipMalloc(q, bytes ? bytes : 16);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc");
        p.push_back(*q);
        return PD_OK;
    }
    void release(void *q)
    {
        auto it = std::find(p.begin(), p.end(), q);
        if (it != p.end()) p.erase(it);
    }
    ~DevMem()
    {
        for (void *q : p) (void)hipFree(q);
    }
};

// phi at the target's nodes from an exponential basis, into a new handle
static int extend_basis(const pd_kl_s *src, const pd_mesh_s *target, pd_kl_s **out)
{
    DevMem mem;
    const std::vector<double> Y = node_positions(target);
    const int64_t m = target->M;
    double *dY = nullptr, *dphi = nullptr, *dsl = nullptr;
    int rc;
    if ((rc = mem.get((void **)&dY, 8 * Y.size())) || (rc = mem.get((void **)&dphi, 8 * (size_t)src->n_modes * m)) ||
        (rc = mem.get((void **)&dsl, 8 * (size_t)src->n_modes)))
        return rc;
    PD_HIP(hipMemcpy(dY, Y.data(), 8 * Y.size(), hipMemcpyHostToDevice));
    PD_HIP(hipMemcpy(dsl, src->d_sqrt_lam, 8 * (size_t)src->n_modes, hipMemcpyDeviceToDevice));
    dim3 grid(nblocks(m), (unsigned)((src->n_modes + kModeChunk - 1) / kModeChunk));
    exp_extend_kernel<<<grid, 256>>>(dY, m, src->d_qpos, src->n_q, src->d_ext, src->n_modes, 1.0 / src->corr_len, dphi);
    PD_HIP(hipGetLastError());
    PD_HIP(hipDeviceSynchronize());
    pd_kl_s *k = new (std::nothrow) pd_kl_s();
    if (!k) return fail(PD_ENOMEM, "out of host memory");
    k->mesh = target;
    k->n_modes = src->n_modes;
    k->covariance = PD_COV_EXP;
    k->lam = src->lam;
    k->corr_len = src->corr_len;
    k->d_phi = dphi;
    k->d_sqrt_lam = dsl;
    // the quadrature stays with the source handle; a copy lets this one extend too
    k->n_q = src->n_q;
    if ((rc = mem.get((void **)&k->d_qpos, 24 * (size_t)src->n_q)) ||
        (rc = mem.get((void **)&k->d_ext, 8 * (size_t)src->n_modes * src->n_q))) {
        delete k;
        return rc;
    }
    PD_HIP(hipMemcpy(k->d_qpos, src->d_qpos, 24 * (size_t)src->n_q, hipMemcpyDeviceToDevice));
    PD_HIP(hipMemcpy(k->d_ext, src->d_ext, 8 * (size_t)src->n_modes * src->n_q, hipMemcpyDeviceToDevice));
    for (void *q : {(void *)dphi, (void *)dsl, (void *)k->d_qpos, (void *)k->d_ext}) mem.release(q);
    *out = k;
    return PD_OK;
}

}  // namespace pdmi

using namespace pdmi;

extern "C" {

int pd_kl_build_exp(pd_mesh m, double corr_len, int32_t n_modes, pd_kl *out)
{
    if (!m || !out) return fail(PD_EINVAL, "null argument");
    if (!(corr_len > 0) || n_modes < 1) return fail(PD_EINVAL, "corr_len and n_modes must be positive");
    if (m->M > kMaxExpNodes) return fail(PD_EINVAL, "%lld nodes: the dense Nystrom basis is limited to %d",
                                         (long long)m->M, kMaxExpNodes);
    if (n_modes > m->M) return fail(PD_EINVAL, "n_modes exceeds the number of nodes");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(PD_EDEVICE, "no HIP device: the solver needs an MI355X (gfx950)");
    const int64_t n = m->M;
    // midpoint weight: a cell's volume, or its area for a plane-stress body,
    // whose random field lives on the plane
    const double w = m->d.thickness > 0 ? m->d.dx * m->d.dx : m->d.dx * m->d.dx * m->d.dx;
    const std::vector<double> X = node_positions(m);
    DevMem mem;
    double *dX = nullptr, *dA = nullptr, *dD = nullptr, *dE = nullptr;
    rocblas_int *dinfo = nullptr;
    int rc;
    if ((rc = mem.get((void **)&dX, 8 * X.size())) || (rc = mem.get((void **)&dA, 8 * (size_t)n * n)) ||
        (rc = mem.get((void **)&dD, 8 * (size_t)n)) || (rc = mem.get((void **)&dE, 8 * (size_t)n)) ||
        (rc = mem.get((void **)&dinfo, sizeof(rocblas_int))))
        return rc;
    PD_HIP(hipMemcpy(dX, X.data(), 8 * X.size(), hipMemcpyHostToDevice));
    exp_matrix_kernel<<<dim3(nblocks(n), (unsigned)n), 256>>>(dX, n, w, 1.0 / corr_len, dA);
    PD_HIP(hipGetLastError());
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) return fail(PD_EDEVICE, "rocblas_create_handle failed");
    rocblas_status st = rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)n, dA,
                                         (rocblas_int)n, dD, dE, dinfo);
    hipError_t se = hipDeviceSynchronize();
    (void)rocblas_destroy_handle(h);
    if (st != rocblas_status_success) return fail(PD_EDEVICE, "rocsolver_dsyevd failed (status %d)", (int)st);
    PD_HIP(se);
    rocblas_int info = 0;
    PD_HIP(hipMemcpy(&info, dinfo, sizeof(info), hipMemcpyDeviceToHost));
    if (info != 0) return fail(PD_EDEVICE, "the eigensolver did not converge (info %d)", (int)info);
    std::vector<double> all(n);
    PD_HIP(hipMemcpy(all.data(), dD, 8 * (size_t)n, hipMemcpyDeviceToHost));
    std::vector<double> lam(n);
    for (int64_t k = 0; k < n; ++k) lam[k] = all[n - 1 - k];             // descending
    int K = n_modes;
    while (K < n && std::fabs(lam[K] - lam[K - 1]) <= kClusterRtol * std::fabs(lam[K - 1])) ++K;
    const int take = (int)std::min<int64_t>(K + 1, n);
    std::vector<double> vec((size_t)take * n);
    for (int k = 0; k < take; ++k)        // eigenvector of lam[k] is column n-1-k (column-major)
        PD_HIP(hipMemcpy(&vec[(size_t)k * n], dA + (size_t)(n - 1 - k) * n, 8 * (size_t)n, hipMemcpyDeviceToHost));
    canonicalise(lam, vec, n, take);
    lam.resize(K);
    vec.resize((size_t)K * n);
    const double isw = 1.0 / std::sqrt(w);
    std::vector<double> phi((size_t)K * n), ext((size_t)K * n), sl(K);
    for (int k = 0; k < K; ++k) {
        sl[k] = std::sqrt(std::fmax(lam[k], 0.0));
        for (int64_t j = 0; j < n; ++j) {
            phi[(size_t)k * n + j] = vec[(size_t)k * n + j] * isw;
            ext[(size_t)k * n + j] = w * phi[(size_t)k * n + j] / lam[k];
        }
    }
    pd_kl_s *kl = new (std::nothrow) pd_kl_s();
    if (!kl) return fail(PD_ENOMEM, "out of host memory");
    kl->mesh = m;
    kl->n_modes = K;
    kl->covariance = PD_COV_EXP;
    kl->lam = lam;
    kl->corr_len = corr_len;
    kl->n_q = n;
    if ((rc = mem.get((void **)&kl->d_phi, 8 * phi.size())) || (rc = mem.get((void **)&kl->d_sqrt_lam, 8 * sl.size())) ||
        (rc = mem.get((void **)&kl->d_qpos, 8 * X.size())) || (rc = mem.get((void **)&kl->d_ext, 8 * ext.size()))) {
        delete kl;
        return rc;
    }
    hipError_t e = hipMemcpy(kl->d_phi, phi.data(), 8 * phi.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(kl->d_sqrt_lam, sl.data(), 8 * sl.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(kl->d_qpos, X.data(), 8 * X.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(kl->d_ext, ext.data(), 8 * ext.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete kl;
        return hip_fail(e, "KL basis upload");
    }
    for (void *q : {(void *)kl->d_phi, (void *)kl->d_sqrt_lam, (void *)kl->d_qpos, (void *)kl->d_ext}) mem.release(q);
    *out = kl;
    return PD_OK;
}

int pd_kl_extend(pd_kl kl, pd_mesh target, pd_kl *out)
{
    if (!kl || !target || !out) return fail(PD_EINVAL, "null argument");
    if (kl->covariance != PD_COV_EXP || !kl->d_ext) return fail(PD_EINVAL, "only exponential bases can be extended");
    if ((kl->mesh->d.thickness > 0) != (target->d.thickness > 0))
        return fail(PD_EINVAL, "a plane-stress basis extends to plane-stress meshes only, a 3D one to 3D meshes");
    pd_kl_s *k = nullptr;
    int rc = extend_basis(kl, target, &k);
    if (rc) return rc;
    *out = k;
    return PD_OK;
}

int pd_kl_n_modes(pd_kl kl, int32_t *n_modes_out)
{
    if (!kl || !n_modes_out) return fail(PD_EINVAL, "null argument");
    *n_modes_out = kl->n_modes;
    return PD_OK;
}

int pd_kl_gaussian(pd_kl kl, const double *xi_dev, int64_t n_samples, double *g_dev, void *stream)
{
    if (!kl || !xi_dev || !g_dev) return fail(PD_EINVAL, "null argument");
    if (n_samples < 0 || n_samples > 65535) return fail(PD_EINVAL, "n_samples must be in [0, 65535]");
    if (n_samples == 0) return PD_OK;
    const int64_t M = kl->mesh->M;
    gaussian_kernel<<<dim3(nblocks(M), (unsigned)n_samples), 256, 0, (hipStream_t)stream>>>(
        kl->d_phi, kl->d_sqrt_lam, xi_dev, kl->n_modes, M, g_dev);
    PD_HIP(hipGetLastError());
    return PD_OK;
}

int pd_fib_fields(pd_mesh m, const double *g_dev, int64_t n_samples, const pd_fib_params *fp, void *s0_out,
                  void *c_out, void *gf_out, int32_t out_dtype, void *stream)
{
    if (!m || !g_dev || !fp) return fail(PD_EINVAL, "null argument");
    if (n_samples < 0) return fail(PD_EINVAL, "n_samples must be non-negative");
    if (!(fp->fcm > 0) || !(fp->weibull_m > 0) || !(fp->alpha_E > 0) || !(fp->fck_min > 0) || !(fp->delta_f >= 0))
        return fail(PD_EINVAL, "bad fib parameters");
    if (out_dtype != PD_DTYPE_F32 && out_dtype != PD_DTYPE_F64) return fail(PD_EINVAL, "unknown dtype %d", out_dtype);
    const int64_t n = n_samples * m->M;
    if (n == 0) return PD_OK;
    const double delta = m->d.m_ratio * m->d.dx;
    FibConst f;
    f.lam_w = fp->fcm / std::tgamma(1.0 + 1.0 / fp->weibull_m);
    f.inv_m = 1.0 / fp->weibull_m;
    f.alpha_E = fp->alpha_E;
    f.delta_f = fp->delta_f;
    f.fck_min = fp->fck_min;
    // micromodulus per unit E: the 3D, plane-stress or plane-strain form of the mesh
    const double t = m->d.thickness;
    const double k2 = m->d.plane_strain ? 48.0 / 5.0 : 9.0;
    f.c_scale = t > 0 ? k2 / (M_PI * t * delta * delta * delta) : 12.0 / (M_PI * delta * delta * delta * delta);
    hipStream_t st = (hipStream_t)stream;
    if (out_dtype == PD_DTYPE_F64)
        fib_kernel<double><<<nblocks(n), 256, 0, st>>>(g_dev, n, f, (double *)s0_out, (double *)c_out, (double *)gf_out);
    else
        fib_kernel<float><<<nblocks(n), 256, 0, st>>>(g_dev, n, f, (float *)s0_out, (float *)c_out, (float *)gf_out);
    PD_HIP(hipGetLastError());
    return PD_OK;
}

}  // extern "C"
