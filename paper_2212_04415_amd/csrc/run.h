// Host-side run management shared by the forward entry points and the
// adjoint: device buffers of a solve, set-up kernels, step launches and the
// captured-graph replay.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "pd_internal.h"
#include "step_kernels.h"

namespace pdmi {

// ---------------------------------------------------------------- set-up kernels
template <typename T>
__global__ void init_state_kernel(typename Vec4<T>::t *u0, typename Vec4<T>::t *u1, int64_t P, int64_t S,
                                  int nx, int ny, int nz, int PX, int64_t PXY, const NodeInfo *info,
                                  double load0, const T *cpad)
{
    // every padded cell of every sample (grid-stride); real nodes get the
    // flag word (1, or with a micromodulus field on a 3D body their c / c_ref,
    // which the step kernel reads from there; its sign later marks a node
    // that has had an exceptional bond) and the first prescribed load
    // displacement, ghosts are all zero
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < P * S;
         g += (int64_t)gridDim.x * blockDim.x) {
    int64_t q = g % P;
    int i = (int)(q % PX) - kHalo;
    int64_t rr = q / PX;
    int j = (int)(rr % (PXY / PX)) - kHalo;
    int k = (int)(rr / (PXY / PX)) - kHalo;
    using V4 = typename Vec4<T>::t;
    V4 v{};
    if (i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz) {
        int64_t node = i + (int64_t)nx * (j + (int64_t)ny * k);
        v.w = cpad ? cpad[g] : T(1);
        if (info[node].bc == -2) v.z = (T)load0;
    }
    u0[g] = v;
    u1[g] = v;
    }
}

// Flag words of displacement cells written from the host (1 for a real
// node, 0 for a ghost): a real node's word becomes its c / c_ref, as
// init_state_kernel sets it on a 3D body with a micromodulus field.
template <typename T>
__global__ void flag_from_c_kernel(typename Vec4<T>::t *u, const T *cpad, int64_t n)
{
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x)
        if (u[g].w != T(0)) u[g].w = cpad[g];
}

template <typename T, typename In>
__global__ void fields_kernel(T *s0pad, T *cpad, T *gpad, const In *s0, const In *c, const In *gf, double s0_const,
                              double inv_cref, double inv_gref, int64_t P, int64_t M, int64_t S, int nx, int ny,
                              int nz, int PX, int64_t PXY, int64_t s0_stride, int64_t c_stride, int64_t gf_stride)
{
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < P * S;
         g += (int64_t)gridDim.x * blockDim.x) {
    int64_t sample = g / P, q = g % P;
    int i = (int)(q % PX) - kHalo;
    int64_t rr = q / PX;
    int j = (int)(rr % (PXY / PX)) - kHalo;
    int k = (int)(rr / (PXY / PX)) - kHalo;
    T sv = (T)INFINITY, cv = T(0), gv = T(0);
    if (i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz) {
        int64_t node = i + (int64_t)nx * (j + (int64_t)ny * k);
        sv = (T)(s0 ? (double)s0[sample * s0_stride + node] : s0_const);
        cv = (T)(c ? (double)c[sample * c_stride + node] * inv_cref : 1.0);
        gv = (T)(gf ? (double)gf[sample * gf_stride + node] * inv_gref : 1.0);
    }
    s0pad[g] = sv;
    if (cpad) cpad[g] = cv;
    if (gpad) gpad[g] = gv;
    }
}

template <typename T>
__global__ void threshold_kernel(T *thr, const T *s0pad, int64_t P, int64_t M, int64_t S, int nx, int ny, int PX,
                                 int64_t PXY)
{
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < M * S;
         g += (int64_t)gridDim.x * blockDim.x) {
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
}

template <typename T>
__global__ void fill_kernel(T *x, int64_t n, T v)
{
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x)
        x[g] = v;
}

static __global__ void init_qoi_kernel(double *Q, int64_t *nstar, int32_t *status, int64_t *step, int64_t S)
{
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < S; g += (int64_t)gridDim.x * blockDim.x) {
        Q[g] = -INFINITY;
        nstar[g] = 0;
        status[g] = PD_OK;
        step[g] = 0;
    }
}

// Per-sample check of a micromodulus field [S][M] of type In: a sample
// with a value that is not positive gets PD_EINVAL in status (the step
// kernel keeps c / c_ref in the flag word, where 0 marks a ghost cell and
// the sign a node with an exceptional bond), else, when its largest value
// exceeds `limit`, `code` (the explicit step is unstable where the
// micromodulus exceeds the value its time step allows).  NaN passes, and the
// run then reports it as non-finite.  One block per sample.
template <typename In>
__global__ void field_limit_kernel(const In *f, int64_t M, double limit, int32_t code, int32_t *status)
{
    __shared__ double part[256];
    __shared__ int nonpos;
    if (threadIdx.x == 0) nonpos = 0;
    __syncthreads();
    const In *x = f + (int64_t)blockIdx.x * M;
    double mx = 0.0;
    bool bad = false;
    for (int64_t i = threadIdx.x; i < M; i += blockDim.x) {
        mx = fmax(mx, (double)x[i]);
        bad = bad || x[i] <= In(0);
    }
    part[threadIdx.x] = mx;
    if (bad) nonpos = 1;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] = fmax(part[threadIdx.x], part[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (nonpos) status[blockIdx.x] = PD_EINVAL;
        else if (part[0] > limit) status[blockIdx.x] = code;
    }
}

// FP64 copy of a device field with its largest value and a count of values
// that are not positive and finite (flags[0]: count, flags[1]: bits of the
// largest value; a positive double's bits order like its value).
template <typename In>
__global__ void field_copy_check_kernel(const In *src, int64_t n, double *dst, unsigned long long *flags)
{
    unsigned long long bad = 0, mx = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = (double)src[i];
        dst[i] = v;
        if (!(v > 0.0) || !isfinite(v)) ++bad;
        else mx = max(mx, (unsigned long long)__double_as_longlong(v));
    }
    if (bad) atomicAdd(flags, bad);
    if (mx) atomicMax(flags + 1, mx);
}

// Final displacement of every sample of a solve as FP64 [S][M][3] in metres
// (u in units of dx, from the padded ping-pong buffer that holds u^N).
template <typename T>
__global__ void export_u_kernel(const typename Vec4<T>::t *u, int64_t P, int64_t M, int64_t S, int nx, int ny,
                                int PX, int64_t PXY, double dx, double *out)
{
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < M * S;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t sample = g / M, node = g % M;
        const int ix = (int)(node % nx);
        const int64_t r = node / nx;
        const int iy = (int)(r % ny), iz = (int)(r / ny);
        const int64_t p = (int64_t)(ix + kHalo) + (int64_t)(iy + kHalo) * PX + (int64_t)(iz + kHalo) * PXY;
        const typename Vec4<T>::t v = u[sample * P + p];
        out[3 * g + 0] = (double)v.x * dx;
        out[3 * g + 1] = (double)v.y * dx;
        out[3 * g + 2] = (double)v.z * dx;
    }
}

// Blocks for one thread per element (kernels over one sample's nodes or
// cells, or over samples: at most 2^27 elements, far inside a dispatch's
// 32-bit work-item count).
static unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// Blocks for a grid-stride kernel over n elements: capped at 2^20 blocks
// (2^28 threads), since the arrays of a large batch (its damage history
// alone) can hold more than 2^32 values.
constexpr int64_t kMaxBlocks = int64_t(1) << 20;
static unsigned stride_blocks(int64_t n, int b = 256)
{
    return (unsigned)std::min<int64_t>((n + b - 1) / b, kMaxBlocks);
}

// ---------------------------------------------------------------- run buffers
struct RunBuffers {
    int S = 0;
    bool f64 = false, kahan = true, has_c = false, has_g = false;
    int acc_mode = PD_ACC_KAHAN;   // kahan: the production FP32 kernels (PD_ACC_KAHAN)
    bool comp_state = true;        // compensated u / vh updates (cu, cvh allocated)
    void *u[2] = {nullptr, nullptr};
    void *vh = nullptr, *cu = nullptr, *cvh = nullptr;
    void *hist = nullptr, *dmask = nullptr, *s0pad = nullptr, *thr = nullptr, *cpad = nullptr, *gpad = nullptr;
    double *rf = nullptr, *Q = nullptr, *hist_R = nullptr;
    int64_t *nstar = nullptr, *step = nullptr;
    int32_t *status = nullptr;
    bool own_outputs = true;
    std::vector<void *> allocs;
    // Arena mode: buffers are carved, 256-byte aligned, from a caller-given
    // device region instead of allocated; *arena_used counts the bytes taken
    // (shared by the solves of one call).  With a null arena only the count
    // advances (sizing pass).
    bool arena_mode = false;
    char *arena = nullptr;
    size_t *arena_used = nullptr;
    // Stream-ordered mode: buffers come from the stream-ordered allocator on
    // this stream and are released in stream order (no synchronisation).
    hipStream_t ordered = nullptr;
    bool use_ordered = false;

    int alloc(void **p, size_t bytes)
    {
        if (arena_mode) {
            const size_t off = (*arena_used + 255) & ~(size_t)255;
            *arena_used = off + (bytes ? bytes : 16);
            *p = arena ? arena + off : nullptr;
            return PD_OK;
        }
        hipError_t e = use_ordered ? hipMallocAsync(p, bytes ? bytes : 16, ordered) : hipMalloc(p, bytes ? bytes : 16);
        if (e != hipSuccess) return hip_fail(e, "allocating run buffers");
        allocs.push_back(*p);
        return PD_OK;
    }
    void release()
    {
        for (void *p : allocs) (void)(use_ordered ? hipFreeAsync(p, ordered) : hipFree(p));
        allocs.clear();
    }
};

static int check_launch_size(const pd_mesh_s *m, int64_t S);
static inline int vel_components(const pd_mesh_s *m);

// acc: the params' accumulate mode (ignored in FP64, which compensates nothing)
static int alloc_run(const pd_mesh_s *m, int S, bool f64, int acc, bool has_c, bool want_hist_R, int64_t n_steps,
                     RunBuffers &b, bool outputs, bool has_g = false)
{
    int rc = check_launch_size(m, S);
    if (rc) return rc;
    if (!f64 && has_c && (acc == PD_ACC_STATE_ONLY || acc == PD_ACC_FORCES_ONLY))
        return fail(PD_EINVAL, "the single-compensation ablations take no micromodulus field");
    b.S = S;
    b.f64 = f64;
    b.kahan = !f64 && acc == PD_ACC_KAHAN;
    b.acc_mode = f64 ? PD_ACC_PLAIN : acc;
    b.comp_state = !f64 && (acc == PD_ACC_KAHAN || acc == PD_ACC_STATE_ONLY);
    b.has_c = has_c;
    size_t ts = f64 ? 8 : 4, v4 = 4 * ts;
    for (int h = 0; h < 2; ++h)
        if ((rc = b.alloc(&b.u[h], v4 * m->P * S))) return rc;
    const size_t v3 = vel_components(m) * ts;   // vh, cu, cvh per node
    if ((rc = b.alloc(&b.vh, v3 * m->M * S))) return rc;
    if (b.comp_state) {
        if ((rc = b.alloc(&b.cu, v3 * m->M * S))) return rc;
        if ((rc = b.alloc(&b.cvh, v3 * m->M * S))) return rc;
    }
    if ((rc = b.alloc(&b.hist, ts * kStencil * m->M * S))) return rc;
    if ((rc = b.alloc(&b.dmask, sizeof(uint4) * m->M * S))) return rc;
    if ((rc = b.alloc(&b.s0pad, ts * m->P * S))) return rc;
    if ((rc = b.alloc(&b.thr, ts * m->M * S))) return rc;
    if (has_c && (rc = b.alloc(&b.cpad, ts * m->P * S))) return rc;
    b.has_g = has_g;
    if ((rc = b.alloc(&b.gpad, has_g ? ts * m->P * S : ts))) return rc;   // without a field: one 1
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

// Launch shapes of the step kernel (brick of nodes per block, LDS tile or
// not).  Every shape computes bit-identical results; the autotuner picks the
// fastest per configuration.  FP64 always uses the global shape.
struct LaunchShape {
    int bx, by, bz, threads;
    bool lds;
};
constexpr LaunchShape kShapes[PD_N_SHAPES] = {
    {16, 4, 4, 256, true},   // PD_SHAPE_LDS_16x4x4
    {8, 8, 4, 256, true},    // PD_SHAPE_LDS_8x8x4
    {12, 4, 4, 192, true},   // PD_SHAPE_LDS_12x4x4
    {256, 1, 1, 256, false}, // PD_SHAPE_GLOBAL_256
};
// the same shape indices on a body one node thick: planar patches
constexpr LaunchShape kPlaneShapes[PD_N_SHAPES] = {
    {64, 1, 4, 256, true},
    {32, 1, 8, 256, true},
    {32, 1, 4, 128, true},
    {256, 1, 1, 256, false},
};

// A body one node thick has neighbours in the x-z plane only; its step
// kernels visit the 28 in-plane offsets.
static inline bool plane_mesh(const pd_mesh_s *m) { return m->ny == 1; }

// Components per node of the velocity and compensation arrays: (x, z) in a
// body one node thick (its y components stay zero), else (x, y, z).
static inline int vel_components(const pd_mesh_s *m) { return plane_mesh(m) ? 2 : 3; }

// Blocks of one step launch: one per (sample, tile) work item, padded to a
// multiple of the XCD count.
static int64_t step_blocks(const pd_mesh_s *m, int64_t S, const LaunchShape &sh)
{
    const int64_t tiles = sh.lds ? (int64_t)((m->nx + sh.bx - 1) / sh.bx) * ((m->ny + sh.by - 1) / sh.by) *
                                       ((m->nz + sh.bz - 1) / sh.bz)
                                 : (m->M + sh.threads - 1) / sh.threads;
    return (tiles * S + kXcds - 1) / kXcds * kXcds;
}

// A step launch covers every (sample, tile) work item with one block; the
// dispatch counts its work-items in 32 bits, so every shape the solve might
// take (the autotuner tries them all) must stay below 2^32 work-items.
static int check_launch_size(const pd_mesh_s *m, int64_t S)
{
    for (const LaunchShape &sh : plane_mesh(m) ? kPlaneShapes : kShapes) {
        const int64_t blocks = step_blocks(m, S, sh);
        if (blocks * sh.threads > (int64_t)UINT32_MAX)
            return fail(PD_EINVAL, "%lld samples of this mesh exceed one launch (%lld work-items; at most 2^32 - 1)",
                        (long long)S, (long long)(blocks * sh.threads));
    }
    return PD_OK;
}

// Common state of one (mesh, params, samples) solve.
struct Solve {
    const pd_mesh_s *m;
    pd_params p;
    Material mat;
    RunBuffers b;
    int64_t n_steps;
    int shape = PD_SHAPE_LDS_16x4x4;
};

// The shape a solve can actually launch with: FP64 has the global shape
// only; uncompensated accumulation (an ablation) has the default brick and
// the global shape.
static int effective_shape(bool f64, bool kahan, bool has_c, int shape)
{
    (void)has_c;
    if (f64) return PD_SHAPE_GLOBAL_256;
    if (!kahan && shape != PD_SHAPE_GLOBAL_256) return PD_SHAPE_LDS_16x4x4;
    return shape;
}

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
    using V3 = typename Vec3<T>::t;
    a.vh = (V3 *)b.vh;
    a.cu = (V3 *)b.cu;
    a.cvh = (V3 *)b.cvh;
    a.acc_mode = b.acc_mode;
    a.hist = (T *)b.hist;
    a.dmask = (uint4 *)b.dmask;
    a.s0pad = (const T *)b.s0pad;
    a.thr = (const T *)b.thr;
    a.cpad = (const T *)b.cpad;
    a.gpad = (const T *)b.gpad;
    a.gstep = b.has_g ? 1 : 0;
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
    const LaunchShape &sh = (plane_mesh(m) ? kPlaneShapes : kShapes)[effective_shape(b.f64, b.kahan, b.has_c, s.shape)];
    a.nbx = (m->nx + sh.bx - 1) / sh.bx;
    a.nby = (m->ny + sh.by - 1) / sh.by;
    const int64_t nbz = (m->nz + sh.bz - 1) / sh.bz;
    a.tiles = sh.lds ? (int64_t)a.nbx * a.nby * nbz : (m->M + sh.threads - 1) / sh.threads;
    a.n_items = a.tiles * b.S;
    a.chunk = a.nby * (int)nbz;
    a.heavy_first = b.S % kXcds == 0;   // every XCD holds whole samples
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

// One step launch of a solve (defined with the kernel instantiations in
// solver.hip).  L_out != null: force-only evaluation into L_out.
void launch_step_f32(const Solve &s, int k_local, hipStream_t st, double *L_out);
void launch_step_f64(const Solve &s, int k_local, hipStream_t st, double *L_out);

template <typename T>
static inline void launch_step(const Solve &s, int k_local, hipStream_t st, double *L_out = nullptr)
{
    if constexpr (sizeof(T) == 4) launch_step_f32(s, k_local, st, L_out);
    else launch_step_f64(s, k_local, st, L_out);
}

static void launch_advance(const Solve &s, int64_t by, hipStream_t st)
{
    advance_kernel<<<blocks_for(s.b.S), 256, 0, st>>>(s.b.step, s.b.S, by);
}

// Copies a finished solve's displacement u^N (the input of its last step
// launch, in buffer (N - 1) & 1) to out, FP64 [S][M][3] in metres.
static void launch_export_u(const Solve &s, double *out, hipStream_t st)
{
    const pd_mesh_s *m = s.m;
    const int parity = s.n_steps > 0 ? (int)((s.n_steps - 1) & 1) : 0;
    const int64_t n = m->M * s.b.S;
    if (s.b.f64)
        export_u_kernel<double><<<stride_blocks(n), 256, 0, st>>>((const double4 *)s.b.u[parity], m->P, m->M, s.b.S,
                                                                  m->nx, m->ny, m->PX, (int64_t)m->PX * m->PY,
                                                                  m->d.dx, out);
    else
        export_u_kernel<float><<<stride_blocks(n), 256, 0, st>>>((const float4 *)s.b.u[parity], m->P, m->M, s.b.S,
                                                                 m->nx, m->ny, m->PX, (int64_t)m->PX * m->PY,
                                                                 m->d.dx, out);
}

// s0 / c: device [S][M] fields of type In, or null (homogeneous)
template <typename T, typename In = double>
static int setup_solve(Solve &s, const In *s0, int64_t s0_stride, const In *c, int64_t c_stride,
                       hipStream_t st, const In *gf = nullptr, int64_t gf_stride = 0)
{
    const pd_mesh_s *m = s.m;
    int64_t S = s.b.S;
    unsigned nb = stride_blocks(m->P * S);
    int64_t nv = vel_components(m) * m->M * S;
    fill_kernel<T><<<stride_blocks(nv), 256, 0, st>>>((T *)s.b.vh, nv, T(0));
    if (s.b.comp_state) {
        fill_kernel<T><<<stride_blocks(nv), 256, 0, st>>>((T *)s.b.cu, nv, T(0));
        fill_kernel<T><<<stride_blocks(nv), 256, 0, st>>>((T *)s.b.cvh, nv, T(0));
    }
    int64_t nh = (int64_t)kStencil * m->M * S;
    fill_kernel<T><<<stride_blocks(nh), 256, 0, st>>>((T *)s.b.hist, nh, T(0));
    fill_kernel<uint32_t><<<stride_blocks(4 * m->M * S), 256, 0, st>>>((uint32_t *)s.b.dmask, 4 * m->M * S, 0u);
    if (!s.b.has_g) fill_kernel<T><<<1, 256, 0, st>>>((T *)s.b.gpad, 1, T(1));
    fields_kernel<T, In><<<nb, 256, 0, st>>>((T *)s.b.s0pad, (T *)s.b.cpad, s.b.has_g ? (T *)s.b.gpad : nullptr, s0, c,
                                             s.b.has_g ? gf : nullptr, s.p.s0,
                                             1.0 / s.mat.c_ref, 1.0 / s.p.GF, m->P, m->M, S, m->nx, m->ny, m->nz,
                                             m->PX, (int64_t)m->PX * m->PY, s0_stride, c_stride, gf_stride);
    // after the fields: the flag words carry the padded c / c_ref
    init_state_kernel<T><<<nb, 256, 0, st>>>((typename Vec4<T>::t *)s.b.u[0], (typename Vec4<T>::t *)s.b.u[1], m->P,
                                             S, m->nx, m->ny, m->nz, m->PX, (int64_t)m->PX * m->PY, m->d_info,
                                             -s.p.du / m->d.dx,
                                             s.b.has_c && !plane_mesh(m) ? (const T *)s.b.cpad : nullptr);
    threshold_kernel<T><<<stride_blocks(m->M * S), 256, 0, st>>>((T *)s.b.thr, (const T *)s.b.s0pad, m->P, m->M, S,
                                                              m->nx, m->ny, m->PX, (int64_t)m->PX * m->PY);
    init_qoi_kernel<<<stride_blocks(S), 256, 0, st>>>(s.b.Q, s.b.nstar, s.b.status, s.b.step, S);
    if (c && s.n_steps > 0) {
        // the largest micromodulus a sample may have at this time step
        const double dtc = stability_limit(m, s.p.rho, s.mat.c_ref);
        const double c_limit = s.mat.c_ref * (dtc / s.p.dt) * (dtc / s.p.dt);
        field_limit_kernel<In><<<(unsigned)S, 256, 0, st>>>(c, c_stride, c_limit, PD_EUNSTABLE, s.b.status);
    }
    PD_HIP(hipGetLastError());
    return PD_OK;
}

static int check_params(const pd_mesh_s *m, const pd_params *p, Material *mat, double c_max_rel = 1.0)
{
    int rc = material_from_params(m, p, mat);
    if (rc) return rc;
    if (p->precision != PD_FP32 && p->precision != PD_FP64) return fail(PD_EINVAL, "unknown precision");
    if (p->accumulate < PD_ACC_KAHAN || p->accumulate > PD_ACC_FORCES_ONLY) return fail(PD_EINVAL, "unknown accumulate");
    double dtc = stability_limit(m, p->rho, mat->c_ref * c_max_rel);
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

// n streams (default priority) for the branches of a captured multi-item
// graph; the calling thread keeps them for later batches
static int branch_streams(int n, std::vector<hipStream_t> &out)
{
    static thread_local std::vector<hipStream_t> pool;
    while ((int)pool.size() < n) {
        hipStream_t x = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
        pool.push_back(x);
    }
    out.assign(pool.begin(), pool.begin() + n);
    return PD_OK;
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

// ---------------------------------------------------------------- autotuner
// Launch-shape choice per (grid dims, samples, precision, accumulation,
// micromodulus field), measured once per process and cached.
using TuneKey = std::tuple<int, int, int, int64_t, bool, bool, bool>;

struct TuneCache {
    std::mutex mu;
    std::map<TuneKey, int> best;
};

static TuneCache &tune_cache()
{
    static TuneCache c;
    return c;
}

static TuneKey tune_key(const Solve &s)
{
    return TuneKey{s.m->nx, s.m->ny, s.m->nz, (int64_t)s.b.S, s.b.f64, s.b.kahan, s.b.has_c};
}

// Times `reps` steps of every shape on the solve's buffers (after two
// warm-up steps each) and returns the fastest.  The solve's state advances:
// the caller re-initialises it afterwards.  Synchronises the stream.
template <typename T>
static int autotune_shapes(const Solve &s, hipStream_t st, int reps, int *best_out, double *us_out)
{
    Solve t = s;                  // same buffers; no history, no step limit
    t.n_steps = (int64_t)1 << 40;
    t.b.hist_R = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PD_HIP(hipEventCreate(&e0));
    PD_HIP(hipEventCreate(&e1));
    int best = -1;
    float best_ms = 0.f;
    int k = 0;
    int rc = PD_OK;
    for (int sh = 0; sh < PD_N_SHAPES && rc == PD_OK; ++sh) {
        if (us_out) us_out[sh] = -1.0;
        if (effective_shape(t.b.f64, t.b.kahan, t.b.has_c, sh) != sh) continue;
        t.shape = sh;
        for (int w = 0; w < 2; ++w) launch_step<T>(t, k++, st);
        hipError_t e = hipEventRecord(e0, st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) launch_step<T>(t, k++, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) {
            rc = hip_fail(e, "autotune");
            break;
        }
        if (us_out) us_out[sh] = 1000.0 * ms / reps;
        if (best < 0 || ms < best_ms) {
            best = sh;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == PD_OK && best_out) *best_out = best;
    return rc;
}

// The launch shape of a solve without measuring: the pinned one, else the
// cached choice, else the default brick.
static int known_shape(const Solve &s)
{
    if (s.m->shape_override >= 0) return effective_shape(s.b.f64, s.b.kahan, s.b.has_c, s.m->shape_override);
    if (s.b.f64) return PD_SHAPE_GLOBAL_256;
    std::lock_guard<std::mutex> g(tune_cache().mu);
    auto it = tune_cache().best.find(tune_key(s));
    return it != tune_cache().best.end() ? it->second : PD_SHAPE_LDS_16x4x4;
}

// Picks the launch shape of a set-up solve: the mesh's pinned shape, else the
// cached choice, else a fresh measurement (after which the solve is set up
// again from scratch, so the measurement leaves no trace in the results).
template <typename T, typename In>
static int choose_shape(Solve &s, const In *s0, int64_t s0_stride, const In *c, int64_t c_stride, hipStream_t st,
                        const In *gf = nullptr, int64_t gf_stride = 0)
{
    if (s.b.f64) {
        s.shape = PD_SHAPE_GLOBAL_256;
        return PD_OK;
    }
    if (s.m->shape_override >= 0) {
        s.shape = effective_shape(s.b.f64, s.b.kahan, s.b.has_c, s.m->shape_override);
        return PD_OK;
    }
    const TuneKey key = tune_key(s);
    {
        std::lock_guard<std::mutex> g(tune_cache().mu);
        auto it = tune_cache().best.find(key);
        if (it != tune_cache().best.end()) {
            s.shape = it->second;
            return PD_OK;
        }
    }
    int best = PD_SHAPE_LDS_16x4x4;
    int rc = autotune_shapes<T>(s, st, 8, &best, nullptr);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> g(tune_cache().mu);
        tune_cache().best[key] = best;
    }
    s.shape = best;
    return setup_solve<T, In>(s, s0, s0_stride, c, c_stride, st, gf, gf_stride);
}

}  // namespace pdmi
