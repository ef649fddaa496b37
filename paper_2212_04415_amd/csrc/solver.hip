// Run management of the explicit peridynamic solve and the C entry points
// for meshes, single runs, force evaluations and batches.  The step kernel
// itself is in step_kernels.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <cstring>
#include <utility>
#include <vector>

#include "pd_internal.h"
#include "step_kernels.h"

namespace pdmi {

const char *last_error();

// ---------------------------------------------------------------- set-up kernels
template <typename T>
__global__ void init_state_kernel(typename Vec4<T>::t *u0, typename Vec4<T>::t *u1, int64_t P, int64_t S,
                                  int nx, int ny, int nz, int PX, int64_t PXY, const NodeInfo *info,
                                  double load0)
{
    // one thread per padded cell of every sample; real nodes get flag 1 and
    // the first prescribed load displacement, ghosts are all zero
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= P * S) return;
    int64_t q = g % P;
    int i = (int)(q % PX) - kHalo;
    int64_t rr = q / PX;
    int j = (int)(rr % (PXY / PX)) - kHalo;
    int k = (int)(rr / (PXY / PX)) - kHalo;
    using V4 = typename Vec4<T>::t;
    V4 v{};
    if (i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz) {
        int64_t node = i + (int64_t)nx * (j + (int64_t)ny * k);
        v.w = T(1);
        if (info[node].bc == -2) v.z = (T)load0;
    }
    u0[g] = v;
    u1[g] = v;
}

template <typename T, typename In>
__global__ void fields_kernel(T *s0pad, T *cpad, const In *s0, const In *c, double s0_const,
                              double inv_cref, int64_t P, int64_t M, int64_t S, int nx, int ny, int nz, int PX,
                              int64_t PXY, int64_t s0_stride, int64_t c_stride)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= P * S) return;
    int64_t sample = g / P, q = g % P;
    int i = (int)(q % PX) - kHalo;
    int64_t rr = q / PX;
    int j = (int)(rr % (PXY / PX)) - kHalo;
    int k = (int)(rr / (PXY / PX)) - kHalo;
    T sv = (T)INFINITY, cv = T(0);
    if (i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz) {
        int64_t node = i + (int64_t)nx * (j + (int64_t)ny * k);
        sv = (T)(s0 ? (double)s0[sample * s0_stride + node] : s0_const);
        cv = (T)(c ? (double)c[sample * c_stride + node] * inv_cref : 1.0);
    }
    s0pad[g] = sv;
    if (cpad) cpad[g] = cv;
}

template <typename T>
__global__ void threshold_kernel(T *thr, const T *s0pad, int64_t P, int64_t M, int64_t S, int nx, int ny, int PX,
                                 int64_t PXY)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= M * S) return;
    int64_t sample = g / M, node = g % M;
    int ix = (int)(node % nx);
    int64_t r = node / nx;
    int iy = (int)(r % ny), iz = (int)(r / ny);
    int64_t p = (int64_t)(ix + kHalo) + (int64_t)(iy + kHalo) * PX + (int64_t)(iz + kHalo) * PXY;
    const T *S0 = s0pad + sample * P;
    T mn = (T)INFINITY;
    for (int s = 0; s < kHalfStencil; ++s) {
        Off o = kHalf.v[s];
        int64_t off = (int64_t)o.x + (int64_t)o.y * PX + (int64_t)o.z * PXY;
        mn = fmin(mn, fmin(S0[p + off], S0[p - off]));
    }
    thr[g] = T(0.5) * (S0[p] + mn);
}

template <typename T>
__global__ void fill_kernel(T *x, int64_t n, T v)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) x[g] = v;
}

__global__ void init_qoi_kernel(double *Q, int64_t *nstar, int32_t *status, int64_t *step, int64_t S)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < S) {
        Q[g] = -INFINITY;
        nstar[g] = 0;
        status[g] = PD_OK;
        step[g] = 0;
    }
}

static unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------- run buffers
struct RunBuffers {
    int S = 0;
    bool f64 = false, kahan = true, has_c = false;
    void *u[2] = {nullptr, nullptr};
    void *vh = nullptr, *cu = nullptr, *cvh = nullptr;
    void *hist = nullptr, *s0pad = nullptr, *thr = nullptr, *cpad = nullptr;
    double *rf = nullptr, *Q = nullptr, *hist_R = nullptr;
    int64_t *nstar = nullptr, *step = nullptr;
    int32_t *status = nullptr;
    bool own_outputs = true;
    std::vector<void *> allocs;

    int alloc(void **p, size_t bytes)
    {
        hipError_t e = hipMalloc(p, bytes ? bytes : 16);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(run buffers)");
        allocs.push_back(*p);
        return PD_OK;
    }
    void release()
    {
        for (void *p : allocs) (void)hipFree(p);
        allocs.clear();
    }
};

static int alloc_run(const pd_mesh_s *m, int S, bool f64, bool kahan, bool has_c, bool want_hist_R, int64_t n_steps,
                     RunBuffers &b, bool outputs)
{
    b.S = S;
    b.f64 = f64;
    b.kahan = kahan && !f64;
    b.has_c = has_c;
    size_t ts = f64 ? 8 : 4, v4 = 4 * ts;
    int rc;
    for (int h = 0; h < 2; ++h)
        if ((rc = b.alloc(&b.u[h], v4 * m->P * S))) return rc;
    if ((rc = b.alloc(&b.vh, v4 * m->M * S))) return rc;
    if (b.kahan) {
        if ((rc = b.alloc(&b.cu, v4 * m->M * S))) return rc;
        if ((rc = b.alloc(&b.cvh, v4 * m->M * S))) return rc;
    }
    if ((rc = b.alloc(&b.hist, ts * kStencil * m->M * S))) return rc;
    if ((rc = b.alloc(&b.s0pad, ts * m->P * S))) return rc;
    if ((rc = b.alloc(&b.thr, ts * m->M * S))) return rc;
    if (has_c && (rc = b.alloc(&b.cpad, ts * m->P * S))) return rc;
    if ((rc = b.alloc((void **)&b.rf, 2 * 8 * m->support.size() * S))) return rc;
    if ((rc = b.alloc((void **)&b.step, 8 * S))) return rc;
    if (outputs) {
        if ((rc = b.alloc((void **)&b.Q, 8 * S))) return rc;
        if ((rc = b.alloc((void **)&b.nstar, 8 * S))) return rc;
        if ((rc = b.alloc((void **)&b.status, 4 * S))) return rc;
    }
    if (want_hist_R && (rc = b.alloc((void **)&b.hist_R, 8 * S * std::max<int64_t>(n_steps, 1)))) return rc;
    return PD_OK;
}

// Common state of one (mesh, params, samples) solve.
struct Solve {
    const pd_mesh_s *m;
    pd_params p;
    Material mat;
    RunBuffers b;
    int64_t n_steps;
};

// FP32 steps read neighbours from an LDS brick; FP64 (a single-sample,
// latency-bound solve) reads them through the caches.
#ifndef PD_FP32_LDS
#define PD_FP32_LDS 1
#endif
template <typename T>
constexpr bool use_lds() { return sizeof(T) == 4 && PD_FP32_LDS; }

template <typename T>
static StepParams<T> make_step_params(const Solve &s, int k_local)
{
    const int parity = k_local & 1;
    const pd_mesh_s *m = s.m;
    const RunBuffers &b = s.b;
    using V4 = typename Vec4<T>::t;
    StepParams<T> a{};
    a.u_cur = (const V4 *)b.u[parity];
    a.u_next = (V4 *)b.u[parity ^ 1];
    a.vh = (V4 *)b.vh;
    a.cu = (V4 *)b.cu;
    a.cvh = (V4 *)b.cvh;
    a.hist = (T *)b.hist;
    a.s0pad = (const T *)b.s0pad;
    a.thr = (const T *)b.thr;
    a.cpad = (const T *)b.cpad;
    a.info = m->d_info;
    a.cut = m->d_cut;
    a.rf = b.rf;
    a.rf_stride = (int64_t)b.S * (int64_t)m->support.size();
    a.L_out = nullptr;
    a.step_base = b.step;
    a.k_local = k_local;
    a.n_steps = s.n_steps;
    a.Q = b.Q;
    a.nstar = b.nstar;
    a.status = b.status;
    a.hist_R = b.hist_R;
    a.P = m->P;
    a.M = m->M;
    a.PXY = (int64_t)m->PX * m->PY;
    a.nbx = (m->nx + kBX - 1) / kBX;
    a.nby = (m->ny + kBY - 1) / kBY;
    const int64_t nbz = (m->nz + kBZ - 1) / kBZ;
    a.tiles = use_lds<T>() ? (int64_t)a.nbx * a.nby * nbz : (m->M + kBlock - 1) / kBlock;
    a.n_items = a.tiles * b.S;
    a.nz = m->nz;
    a.PY = m->PY;
    a.PZ = m->PZ;
    a.nx = m->nx;
    a.ny = m->ny;
    a.PX = m->PX;
    a.nsup = (int)m->support.size();
    a.force_only = 0;
    const pd_params &p = s.p;
    double dx = m->d.dx;
    double K = s.mat.c_ref * s.mat.volume / (p.rho * dx);   // acceleration per unit G, in dx/s^2
    double bcoef = 0.5 * p.dt * K;
    double g = 0.5 * p.dt * p.damping / p.rho;
    double D = 1.0 / (1.0 + g);
    a.two_d_b = (T)(2.0 * D * bcoef);
    a.two_d_g = (T)(2.0 * D * g);
    a.dt = (T)p.dt;
    a.vload = (T)(-p.du / (p.dt * dx));
    a.du_s = p.du / dx;
    a.gamma_rel = (T)(s.mat.gamma / s.mat.c_ref);
    a.k = (T)p.k;
    a.alpha = (T)p.alpha;
    a.inv1mek = (T)s.mat.inv_one_minus_ek;
    a.inv1pa = (T)s.mat.inv_one_plus_alpha;
    a.law = p.law;
    a.LV = s.mat.c_ref * s.mat.volume;
    a.Rscale = s.mat.c_ref * s.mat.volume * s.mat.volume;
    return a;
}

template <typename T>
static void launch_step(const Solve &s, int k_local, hipStream_t st, double *L_out = nullptr)
{
    StepParams<T> a = make_step_params<T>(s, k_local);
    if (L_out) {
        a.L_out = L_out;
        a.force_only = 1;
    }
    const int64_t items = a.n_items;
    dim3 grid((unsigned)((items + kXcds - 1) / kXcds * kXcds));
    if constexpr (std::is_same<T, float>::value) {
        if (s.b.kahan) {
            if (s.b.has_c) step_kernel<float, true, true, use_lds<T>()><<<grid, kBlock, 0, st>>>(a);
            else step_kernel<float, true, false, use_lds<T>()><<<grid, kBlock, 0, st>>>(a);
        } else {
            if (s.b.has_c) step_kernel<float, false, true, use_lds<T>()><<<grid, kBlock, 0, st>>>(a);
            else step_kernel<float, false, false, use_lds<T>()><<<grid, kBlock, 0, st>>>(a);
        }
    } else {
        if (s.b.has_c) step_kernel<double, false, true, false><<<grid, kBlock, 0, st>>>(a);
        else step_kernel<double, false, false, false><<<grid, kBlock, 0, st>>>(a);
    }
}

static void launch_advance(const Solve &s, int64_t by, hipStream_t st)
{
    advance_kernel<<<blocks_for(s.b.S), 256, 0, st>>>(s.b.step, s.b.S, by);
}

// s0 / c: device [S][M] fields of type In, or null (homogeneous)
template <typename T, typename In = double>
static int setup_solve(Solve &s, const In *s0, int64_t s0_stride, const In *c, int64_t c_stride,
                       hipStream_t st)
{
    const pd_mesh_s *m = s.m;
    int64_t S = s.b.S;
    unsigned nb = blocks_for(m->P * S);
    init_state_kernel<T><<<nb, 256, 0, st>>>((typename Vec4<T>::t *)s.b.u[0], (typename Vec4<T>::t *)s.b.u[1], m->P,
                                             S, m->nx, m->ny, m->nz, m->PX, (int64_t)m->PX * m->PY, m->d_info,
                                             -s.p.du / m->d.dx);
    int64_t nv = 4 * m->M * S;
    fill_kernel<T><<<blocks_for(nv), 256, 0, st>>>((T *)s.b.vh, nv, T(0));
    if (s.b.kahan) {
        fill_kernel<T><<<blocks_for(nv), 256, 0, st>>>((T *)s.b.cu, nv, T(0));
        fill_kernel<T><<<blocks_for(nv), 256, 0, st>>>((T *)s.b.cvh, nv, T(0));
    }
    int64_t nh = (int64_t)kStencil * m->M * S;
    fill_kernel<T><<<blocks_for(nh), 256, 0, st>>>((T *)s.b.hist, nh, T(0));
    fields_kernel<T, In><<<nb, 256, 0, st>>>((T *)s.b.s0pad, (T *)s.b.cpad, s0, c, s.p.s0, 1.0 / s.mat.c_ref, m->P, m->M,
                                         S, m->nx, m->ny, m->nz, m->PX, (int64_t)m->PX * m->PY, s0_stride, c_stride);
    threshold_kernel<T><<<blocks_for(m->M * S), 256, 0, st>>>((T *)s.b.thr, (const T *)s.b.s0pad, m->P, m->M, S,
                                                              m->nx, m->ny, m->PX, (int64_t)m->PX * m->PY);
    init_qoi_kernel<<<blocks_for(S), 256, 0, st>>>(s.b.Q, s.b.nstar, s.b.status, s.b.step, S);
    PD_HIP(hipGetLastError());
    return PD_OK;
}

static int check_params(const pd_mesh_s *m, const pd_params *p, Material *mat, double c_max_rel = 1.0)
{
    int rc = material_from_params(m, p, mat);
    if (rc) return rc;
    if (p->precision != PD_FP32 && p->precision != PD_FP64) return fail(PD_EINVAL, "unknown precision");
    if (p->accumulate != PD_ACC_KAHAN && p->accumulate != PD_ACC_PLAIN) return fail(PD_EINVAL, "unknown accumulate");
    double dtc = stability_limit(p->rho, mat->c_ref * c_max_rel, m->d.dx);
    if (p->dt > dtc)
        return fail(PD_EUNSTABLE, "dt %.6g s exceeds the explicit stability limit %.6g s", p->dt, dtc);
    return PD_OK;
}

static int upload_mesh(pd_mesh_s *m)
{
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(PD_EDEVICE, "no HIP device: the solver needs an MI355X (gfx950)");
    PD_HIP(hipGetDevice(&m->device));
    PD_HIP(hipMalloc(&m->d_info, sizeof(NodeInfo) * m->M));
    PD_HIP(hipMemcpy(m->d_info, m->info.data(), sizeof(NodeInfo) * m->M, hipMemcpyHostToDevice));
    size_t ncut = std::max<size_t>(m->cut_masks.size() / 4, 1);
    PD_HIP(hipMalloc(&m->d_cut, sizeof(uint4) * ncut));
    if (!m->cut_masks.empty())
        PD_HIP(hipMemcpy(m->d_cut, m->cut_masks.data(), 4 * m->cut_masks.size(), hipMemcpyHostToDevice));
    PD_HIP(hipMalloc(&m->d_support, sizeof(int32_t) * m->support.size()));
    PD_HIP(hipMemcpy(m->d_support, m->support.data(), 4 * m->support.size(), hipMemcpyHostToDevice));
    return PD_OK;
}

static int ensure_device(pd_mesh_s *m)
{
    if (!m->bonds_built) return fail(PD_ESTATE, "pd_build_bonds has not been called on this mesh");
    if (!m->d_info) {
        int rc = upload_mesh(m);
        if (rc) return rc;
    }
    int dev = -1;
    PD_HIP(hipGetDevice(&dev));
    if (dev != m->device) return fail(PD_EDEVICE, "mesh was uploaded to device %d, current device is %d", m->device, dev);
    return PD_OK;
}

// Capture `steps` (even) steps of a solve into an executable graph.
template <typename T>
static int capture_chunk(const Solve &s, int steps, hipStream_t cap, hipGraphExec_t *exec)
{
    hipGraph_t g = nullptr;
    PD_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < steps; ++k) launch_step<T>(s, k, cap);
    launch_advance(s, steps, cap);
    hipError_t e = hipStreamEndCapture(cap, &g);
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    return PD_OK;
}

static hipStream_t capture_stream()
{
    static thread_local hipStream_t s = nullptr;
    if (!s) (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    return s;
}

constexpr int kChunk = 64;  // steps per captured graph (even)

// Enqueue all steps of a solve on st: whole chunks from a graph, then the
// remainder.  A step's index is the per-sample chunk base (advanced on the
// device at the end of each chunk) plus its fixed offset in the chunk, so
// one captured chunk serves every replay; the chunk is even so the ping-pong
// parity of the displacement buffers repeats.
template <typename T>
static int enqueue_steps(const Solve &s, hipStream_t st, std::vector<hipGraphExec_t> &graphs)
{
    int64_t N = s.n_steps;
    int64_t full = N / kChunk;
    if (full > 0) {
        hipGraphExec_t ex = nullptr;
        int rc = capture_chunk<T>(s, kChunk, capture_stream(), &ex);
        if (rc) return rc;
        graphs.push_back(ex);
        for (int64_t c = 0; c < full; ++c) PD_HIP(hipGraphLaunch(ex, st));
    }
    // the remaining steps, then one launch at step N that only forms R^N
    for (int64_t k = full * kChunk; k <= N; ++k) launch_step<T>(s, (int)(k - full * kChunk), st);
    PD_HIP(hipGetLastError());
    return PD_OK;
}

}  // namespace pdmi

// ====================================================================== C ABI
using namespace pdmi;

struct pd_run_s {
    Solve s;
    hipStream_t stream = nullptr;
    std::vector<hipGraphExec_t> graphs;
};

extern "C" {

const char *pd_last_error(void) { return pdmi::last_error(); }

int pd_build_mesh(const pd_mesh_desc *desc, pd_mesh *out)
{
    if (!desc || !out) return fail(PD_EINVAL, "null argument");
    pd_mesh_s *m = new (std::nothrow) pd_mesh_s();
    if (!m) return fail(PD_ENOMEM, "out of host memory");
    int rc = build_mesh(desc, m);
    if (rc) {
        delete m;
        return rc;
    }
    *out = m;
    return PD_OK;
}

int pd_build_bonds(pd_mesh m, int64_t *n_bonds_out)
{
    if (!m) return fail(PD_EINVAL, "null mesh");
    if (!m->bonds_built) {
        int rc = build_cuts(m);
        if (rc) return rc;
        m->bonds_built = true;
        // upload now when a device is present; otherwise on first device use
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0 && (rc = upload_mesh(m))) return rc;
    }
    if (n_bonds_out) *n_bonds_out = m->n_bonds;
    return PD_OK;
}

int pd_mesh_get_info(pd_mesh m, pd_mesh_info_t *info)
{
    if (!m || !info) return fail(PD_EINVAL, "null argument");
    info->nx = m->nx;
    info->ny = m->ny;
    info->nz = m->nz;
    info->n_nodes = m->M;
    info->n_bonds = m->bonds_built ? m->n_bonds : 0;
    info->n_cut = m->bonds_built ? m->n_cut : 0;
    info->n_support = (int32_t)m->support.size();
    info->n_load = (int32_t)m->load.size();
    info->n_stencil = kStencil;
    info->delta = m->d.m_ratio * m->d.dx;
    return PD_OK;
}

int pd_mesh_get_pads(pd_mesh m, int32_t *support, int32_t *load)
{
    if (!m) return fail(PD_EINVAL, "null mesh");
    if (support) std::memcpy(support, m->support.data(), 4 * m->support.size());
    if (load) std::memcpy(load, m->load.data(), 4 * m->load.size());
    return PD_OK;
}

int pd_set_material_field(pd_mesh m, int32_t field, int64_t n_samples, const void *values, int32_t on_device,
                          int32_t dtype, void *stream)
{
    if (!m) return fail(PD_EINVAL, "null mesh");
    if (field != PD_FIELD_S0 && field != PD_FIELD_C) return fail(PD_EINVAL, "unknown field %d", field);
    if (dtype != PD_DTYPE_F32 && dtype != PD_DTYPE_F64) return fail(PD_EINVAL, "unknown dtype %d", dtype);
    double **dst = field == PD_FIELD_S0 ? &m->d_s0 : &m->d_c;
    int64_t *cnt = field == PD_FIELD_S0 ? &m->s0_samples : &m->c_samples;
    if (*dst) {
        (void)hipFree(*dst);
        *dst = nullptr;
        *cnt = 0;
    }
    if (!values) return PD_OK;
    if (n_samples < 1) return fail(PD_EINVAL, "n_samples must be positive");
    int64_t n = n_samples * m->M;
    std::vector<double> host(n);
    if (on_device) {
        std::vector<char> raw(n * (dtype == PD_DTYPE_F64 ? 8 : 4));
        PD_HIP(hipMemcpyAsync(raw.data(), values, raw.size(), hipMemcpyDeviceToHost, (hipStream_t)stream));
        PD_HIP(hipStreamSynchronize((hipStream_t)stream));
        for (int64_t i = 0; i < n; ++i)
            host[i] = dtype == PD_DTYPE_F64 ? ((const double *)raw.data())[i] : ((const float *)raw.data())[i];
    } else {
        for (int64_t i = 0; i < n; ++i)
            host[i] = dtype == PD_DTYPE_F64 ? ((const double *)values)[i] : ((const float *)values)[i];
    }
    for (int64_t i = 0; i < n; ++i)
        if (!(host[i] > 0) || !std::isfinite(host[i])) return fail(PD_EINVAL, "field values must be positive and finite");
    PD_HIP(hipMalloc(dst, 8 * n));
    PD_HIP(hipMemcpy(*dst, host.data(), 8 * n, hipMemcpyHostToDevice));
    *cnt = n_samples;
    return PD_OK;
}

int pd_free_mesh(pd_mesh m)
{
    if (!m) return PD_OK;
    if (m->d_info) (void)hipFree(m->d_info);
    if (m->d_cut) (void)hipFree(m->d_cut);
    if (m->d_support) (void)hipFree(m->d_support);
    if (m->d_s0) (void)hipFree(m->d_s0);
    if (m->d_c) (void)hipFree(m->d_c);
    delete m;
    return PD_OK;
}

int pd_force_eval(pd_mesh m, const pd_params *p, int64_t n_samples, const double *u_host, double *L_host,
                  void *stream)
{
    if (!m || !p || !u_host || !L_host) return fail(PD_EINVAL, "null argument");
    if (n_samples < 1) return fail(PD_EINVAL, "n_samples must be positive");
    int rc = ensure_device(m);
    if (rc) return rc;
    Solve s{};
    s.m = m;
    s.p = *p;
    if ((rc = material_from_params(m, p, &s.mat))) return rc;
    if (m->s0_samples && m->s0_samples != n_samples) return fail(PD_EINVAL, "s0 field has %lld samples", (long long)m->s0_samples);
    if (m->c_samples && m->c_samples != n_samples) return fail(PD_EINVAL, "c field has %lld samples", (long long)m->c_samples);
    s.n_steps = 0;
    bool f64 = p->precision == PD_FP64;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = alloc_run(m, (int)n_samples, f64, p->accumulate == PD_ACC_KAHAN, m->d_c != nullptr, false, 0, s.b, true))) {
        s.b.release();
        return rc;
    }
    double *dL = nullptr;
    std::vector<char> host;
    size_t ts = f64 ? 8 : 4;
    do {
        if (f64) rc = setup_solve<double>(s, m->d_s0, m->M, m->d_c, m->M, st);
        else rc = setup_solve<float>(s, m->d_s0, m->M, m->d_c, m->M, st);
        if (rc) break;
        // displacements into the padded grid (units of dx), flag 1
        host.assign(ts * 4 * m->P * n_samples, 0);
        for (int64_t smp = 0; smp < n_samples; ++smp)
            for (int k = 0; k < m->nz; ++k)
                for (int j = 0; j < m->ny; ++j)
                    for (int i = 0; i < m->nx; ++i) {
                        int64_t node = i + (int64_t)m->nx * (j + (int64_t)m->ny * k);
                        int64_t q = smp * m->P + m->padded(i, j, k);
                        const double *u = u_host + 3 * (smp * m->M + node);
                        for (int d = 0; d < 4; ++d) {
                            double v = d < 3 ? u[d] / m->d.dx : 1.0;
                            if (f64) ((double *)host.data())[4 * q + d] = v;
                            else ((float *)host.data())[4 * q + d] = (float)v;
                        }
                    }
        hipError_t e = hipMemcpyAsync(s.b.u[0], host.data(), host.size(), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) { rc = hip_fail(e, "upload u"); break; }
        e = hipMalloc(&dL, 8 * 3 * m->M * n_samples);
        if (e != hipSuccess) { rc = hip_fail(e, "hipMalloc(L)"); break; }
        if (f64) launch_step<double>(s, 0, st, dL);
        else launch_step<float>(s, 0, st, dL);
        e = hipGetLastError();
        if (e != hipSuccess) { rc = hip_fail(e, "force kernel"); break; }
        e = hipMemcpyAsync(L_host, dL, 8 * 3 * m->M * n_samples, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) { rc = hip_fail(e, "download L"); break; }
    } while (0);
    if (dL) (void)hipFree(dL);
    (void)hipStreamSynchronize(st);
    s.b.release();
    return rc;
}

int pd_run(pd_mesh m, const pd_params *p, void *stream, pd_run_h *out)
{
    if (!m || !p || !out) return fail(PD_EINVAL, "null argument");
    int rc = ensure_device(m);
    if (rc) return rc;
    if (m->s0_samples > 1 || m->c_samples > 1) return fail(PD_EINVAL, "pd_run takes single-sample fields");
    pd_run_s *r = new (std::nothrow) pd_run_s();
    if (!r) return fail(PD_ENOMEM, "out of host memory");
    r->s.m = m;
    r->s.p = *p;
    r->s.n_steps = p->n_steps;
    r->stream = (hipStream_t)stream;
    double cmax = 1.0;
    if ((rc = check_params(m, p, &r->s.mat, cmax))) {
        delete r;
        return rc;
    }
    bool f64 = p->precision == PD_FP64;
    rc = alloc_run(m, 1, f64, p->accumulate == PD_ACC_KAHAN, m->d_c != nullptr, p->record_history != 0, p->n_steps,
                   r->s.b, true);
    if (!rc) rc = f64 ? setup_solve<double>(r->s, m->d_s0, m->M, m->d_c, m->M, r->stream)
                      : setup_solve<float>(r->s, m->d_s0, m->M, m->d_c, m->M, r->stream);
    if (!rc) rc = f64 ? enqueue_steps<double>(r->s, r->stream, r->graphs) : enqueue_steps<float>(r->s, r->stream, r->graphs);
    if (rc) {
        (void)hipStreamSynchronize(r->stream);
        for (auto g : r->graphs) (void)hipGraphExecDestroy(g);
        r->s.b.release();
        delete r;
        return rc;
    }
    *out = r;
    return PD_OK;
}

int pd_qoi(pd_run_h r, double *peak, int64_t *peak_step, double *history)
{
    if (!r) return fail(PD_EINVAL, "null run");
    PD_HIP(hipStreamSynchronize(r->stream));
    double Q = 0;
    int64_t ns = 0;
    int32_t status = 0;
    PD_HIP(hipMemcpy(&Q, r->s.b.Q, 8, hipMemcpyDeviceToHost));
    PD_HIP(hipMemcpy(&ns, r->s.b.nstar, 8, hipMemcpyDeviceToHost));
    PD_HIP(hipMemcpy(&status, r->s.b.status, 4, hipMemcpyDeviceToHost));
    if (peak) *peak = Q;
    if (peak_step) *peak_step = ns;
    if (history) {
        if (!r->s.b.hist_R) return fail(PD_ESTATE, "run was started without record_history");
        PD_HIP(hipMemcpy(history, r->s.b.hist_R, 8 * r->s.n_steps, hipMemcpyDeviceToHost));
    }
    if (status != PD_OK) return fail(status, "the run produced a non-finite reaction");
    return PD_OK;
}

int pd_run_state(pd_run_h r, double *u_out, double *kappa_out)
{
    if (!r) return fail(PD_EINVAL, "null run");
    PD_HIP(hipStreamSynchronize(r->stream));
    const pd_mesh_s *m = r->s.m;
    bool f64 = r->s.b.f64;
    size_t ts = f64 ? 8 : 4;
    int64_t N = r->s.n_steps;
    int parity = N > 0 ? (int)((N - 1) & 1) : 0;
    if (u_out) {
        std::vector<char> h(ts * 4 * m->P);
        PD_HIP(hipMemcpy(h.data(), r->s.b.u[parity], h.size(), hipMemcpyDeviceToHost));
        for (int k = 0; k < m->nz; ++k)
            for (int j = 0; j < m->ny; ++j)
                for (int i = 0; i < m->nx; ++i) {
                    int64_t node = i + (int64_t)m->nx * (j + (int64_t)m->ny * k);
                    int64_t q = m->padded(i, j, k);
                    for (int d = 0; d < 3; ++d) {
                        double v = f64 ? ((double *)h.data())[4 * q + d] : ((float *)h.data())[4 * q + d];
                        u_out[3 * node + d] = v * m->d.dx;
                    }
                }
    }
    if (kappa_out) {
        std::vector<char> h(ts * kStencil * m->M);
        PD_HIP(hipMemcpy(h.data(), r->s.b.hist, h.size(), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < kStencil * m->M; ++i)
            kappa_out[i] = f64 ? ((double *)h.data())[i] : ((float *)h.data())[i];
    }
    return PD_OK;
}

int pd_free_run(pd_run_h r)
{
    if (!r) return PD_OK;
    (void)hipStreamSynchronize(r->stream);
    for (auto g : r->graphs) (void)hipGraphExecDestroy(g);
    r->s.b.release();
    delete r;
    return PD_OK;
}

static int64_t gcd64(int64_t a, int64_t b) { return b ? gcd64(b, a % b) : a; }

int pd_run_batch(const pd_batch_item *items, int32_t n_items, void *stream)
{
    if (!items || n_items < 1) return fail(PD_EINVAL, "empty batch");
    hipStream_t st = (hipStream_t)stream;
    std::vector<Solve> solves(n_items);
    double dt_min = INFINITY;
    int rc = PD_OK;
    for (int i = 0; i < n_items; ++i) {
        const pd_batch_item &it = items[i];
        if (!it.mesh || !it.params || !it.qoi) return fail(PD_EINVAL, "item %d: null mesh, params or qoi", i);
        if (it.n_samples < 1 || it.n_samples > 65535) return fail(PD_EINVAL, "item %d: n_samples out of range", i);
        if ((rc = ensure_device(it.mesh))) return rc;
        if (it.params->precision != items[0].params->precision || it.params->accumulate != items[0].params->accumulate)
            return fail(PD_EINVAL, "all batch items must share precision and accumulate");
        if (it.field_dtype != PD_DTYPE_F32 && it.field_dtype != PD_DTYPE_F64)
            return fail(PD_EINVAL, "item %d: unknown field dtype", i);
        Material mat;
        // the c field may stiffen bonds; the stability check uses its bound when given on the host side only
        if ((rc = check_params(it.mesh, it.params, &mat))) return rc;
        dt_min = std::min(dt_min, it.params->dt);
    }
    std::vector<int64_t> ratio(n_items);
    int64_t lcm = 1, ticks = 0;
    for (int i = 0; i < n_items; ++i) {
        double r = items[i].params->dt / dt_min;
        ratio[i] = llround(r);
        if (ratio[i] < 1 || std::fabs(r - (double)ratio[i]) > 1e-9 * r)
            return fail(PD_EINVAL, "item %d: dt is not an integer multiple of the finest dt", i);
        lcm = lcm / gcd64(lcm, ratio[i]) * ratio[i];
        if (lcm > 4096) return fail(PD_EINVAL, "dt ratios too irregular");
        ticks = std::max(ticks, items[i].params->n_steps * ratio[i]);
    }
    bool f64 = items[0].params->precision == PD_FP64;
    bool kahan = items[0].params->accumulate == PD_ACC_KAHAN;
    std::vector<void *> scratch;
    for (int i = 0; i < n_items && !rc; ++i) {
        const pd_batch_item &it = items[i];
        Solve &s = solves[i];
        s.m = it.mesh;
        s.p = *it.params;
        s.n_steps = it.params->n_steps;
        material_from_params(it.mesh, it.params, &s.mat);
        rc = alloc_run(it.mesh, (int)it.n_samples, f64, kahan, it.c != nullptr, false, s.n_steps, s.b, false);
        if (rc) break;
        s.b.Q = it.qoi;
        s.b.nstar = (int64_t *)it.nstar;
        s.b.status = it.status;
        if (!s.b.nstar) rc = s.b.alloc((void **)&s.b.nstar, 8 * it.n_samples);
        if (!rc && !s.b.status) rc = s.b.alloc((void **)&s.b.status, 4 * it.n_samples);
        if (rc) break;
        int64_t M = it.mesh->M;
        if (it.field_dtype == PD_DTYPE_F64)
            rc = f64 ? setup_solve<double, double>(s, (const double *)it.s0, M, (const double *)it.c, M, st)
                     : setup_solve<float, double>(s, (const double *)it.s0, M, (const double *)it.c, M, st);
        else
            rc = f64 ? setup_solve<double, float>(s, (const float *)it.s0, M, (const float *)it.c, M, st)
                     : setup_solve<float, float>(s, (const float *)it.s0, M, (const float *)it.c, M, st);
    }
    hipGraphExec_t exec = nullptr;
    if (!rc && ticks > 0) {
        // one hyper-period of 2 * lcm ticks: every item takes an even number
        // of steps in it, so the ping-pong parity of a replay is fixed
        int64_t H = 2 * lcm * std::max<int64_t>(1, 32 / lcm);
        hipStream_t cap = capture_stream();
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamBeginCapture");
        if (!rc) {
            for (int64_t t = 0; t < H; ++t)
                for (int i = 0; i < n_items; ++i) {
                    if (t % ratio[i]) continue;
                    int k_local = (int)(t / ratio[i]);
                    if (f64) launch_step<double>(solves[i], k_local, cap);
                    else launch_step<float>(solves[i], k_local, cap);
                }
            for (int i = 0; i < n_items; ++i) launch_advance(solves[i], H / ratio[i], cap);
            e = hipStreamEndCapture(cap, &g);
            if (e != hipSuccess) rc = hip_fail(e, "hipStreamEndCapture");
        }
        if (!rc) {
            e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) rc = hip_fail(e, "hipGraphInstantiate");
        }
        if (g) (void)hipGraphDestroy(g);
        for (int64_t done = 0; !rc && done < ticks; done += H) {
            e = hipGraphLaunch(exec, st);
            if (e != hipSuccess) rc = hip_fail(e, "hipGraphLaunch");
        }
        // a last launch per item forms the reaction of its final step (it is
        // a no-op for items whose overshooting replays already did)
        for (int i = 0; !rc && i < n_items; ++i) {
            if (f64) launch_step<double>(solves[i], 0, st);
            else launch_step<float>(solves[i], 0, st);
        }
    }
    hipError_t e = hipStreamSynchronize(st);
    if (!rc && e != hipSuccess) rc = hip_fail(e, "batch");
    if (exec) (void)hipGraphExecDestroy(exec);
    for (auto &s : solves) s.b.release();
    return rc;
}

}  // extern "C"

