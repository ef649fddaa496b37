// Host-side run management shared by the forward entry points and the
// adjoint: device buffers of a solve, set-up kernels, step launches and the
// captured-graph replay.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "pd_internal.h"
#include "step_kernels.h"

namespace pdmi {

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

static __global__ void init_qoi_kernel(double *Q, int64_t *nstar, int32_t *status, int64_t *step, int64_t S)
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
    void *hist = nullptr, *dmask = nullptr, *s0pad = nullptr, *thr = nullptr, *cpad = nullptr;
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
    if ((rc = b.alloc(&b.dmask, sizeof(uint4) * m->M * S))) return rc;
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
    a.dmask = (uint4 *)b.dmask;
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
    fill_kernel<uint32_t><<<blocks_for(4 * m->M * S), 256, 0, st>>>((uint32_t *)s.b.dmask, 4 * m->M * S, 0u);
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
