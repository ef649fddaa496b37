// Discrete adjoint of the explicit solve: gradient of the peak reaction
// Q = R^{n*} (n* fixed by the forward run) with respect to the per-node
// limit-stretch field s0 and micromodulus field c.
//
// The forward map of step m, in the library's state variables (half-step
// velocity w, free degrees of freedom only; support and load z-components
// are prescribed and carry no sensitivity):
//   kappa^m = max(kappa^{m-1}, s(u^m))            (damage history)
//   L^m     = F(u^m, kappa^m; s0, c)              (bond forces, section 2.1;
//                                                  appendix A law)
//   w^m     = a1 w^{m-1} + a2 L^m,  a1 = A D, a2 = h (1 + A D)
//   u^{m+1} = u^m + dt w^m
//   R^m     = -V sum_supports L^m_z
// with h = dt / 2rho, A = 1 - damping h, D = 1 / (1 + damping h).
// The reverse sweep runs m = n* ... 1 carrying (ubar, wbar, kbar):
//   wbar += dt mask(ubar^{m+1});  Lbar = a2 wbar (+ seed at m = n*);
//   ubar^m = mask(ubar^{m+1}) - sum_bonds J^T (Lbar_i - Lbar_j)
//            - [kappa grew at m] kbar yhat / |xi|;
//   kbar  += V c keep'(kappa) s (yhat . Fbar);  theta-bar from the law;
//   wbar  <- a1 wbar.
// The forward pass stores a checkpoint (u, w and compensation terms, damage
// history) every K steps; each segment is recomputed from its checkpoint
// with the same step kernel, keeping u^m and kappa^m per step, and then swept
// backwards.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "pd_internal.h"
#include "run.h"

namespace pdmi {

// keep = 1 - d for the largest stretch kap, with its partial derivatives in
// (kap, s0, sc); constant (1 below s0, 0 above sc) outside the softening range.
__device__ __forceinline__ void keep_partials(int law, double kap, double s0, double sc, double k, double alpha,
                                              double &keep, double &dk, double &ds0, double &dsc)
{
    dk = ds0 = dsc = 0.0;
    if (!(kap > s0)) {
        keep = 1.0;
        return;
    }
    if (kap >= sc) {
        keep = 0.0;
        return;
    }
    const double w = sc - s0, t = (kap - s0) / w;
    const double t_k = 1.0 / w, t_s0 = (kap - sc) / (w * w), t_sc = -(kap - s0) / (w * w);
    double g, g_t, g_s0;   // keep = g(t, s0) / kap
    if (law == PD_LAW_EXPLIN) {
        const double om = -expm1(-k);
        const double et = exp(-k * t);
        const double br = 1.0 - (1.0 - et) / om + alpha * (1.0 - t);
        g = s0 * br / (1.0 + alpha);
        g_t = s0 * (-k * et / om - alpha) / (1.0 + alpha);
        g_s0 = br / (1.0 + alpha);
    } else if (t <= 0.2) {
        g = s0 * (1.0 - 4.0 * t);
        g_t = -4.0 * s0;
        g_s0 = 1.0 - 4.0 * t;
    } else {
        g = 0.25 * s0 * (1.0 - t);
        g_t = -0.25 * s0;
        g_s0 = 0.25 * (1.0 - t);
    }
    keep = g / kap;
    dk = g_t * t_k / kap - g / (kap * kap);
    ds0 = (g_s0 + g_t * t_s0) / kap;
    dsc = g_t * t_sc / kap;
}

struct AdjParams {
    int nx, ny, nz, PX;
    int64_t PXY, P, M;
    const NodeInfo *info;
    const uint4 *cut;
    const double *s0pad, *cpad;     // physical fields, padded
    const double *ub_next;          // [M][3]
    double *ub_out;                 // [M][3]
    double *wb;                     // [M][3]
    double4 *Lb;                    // padded [P]
    double *kb;                     // [122][M]
    double *gs0, *gc;               // [M]
    double dx, V, gamma, k, alpha, a1, a2, dt;
    int law;
    int seed;
};

__device__ __forceinline__ bool z_fixed(const NodeInfo &inf) { return inf.bc != -1; }

// wbar += dt mask(ubar^{m+1}); Lbar = a2 wbar (+ seed); wbar <- a1 wbar
__global__ void adj_elementwise(AdjParams a)
{
    const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= a.M) return;
    const NodeInfo inf = a.info[node];
    const uint32_t nd = (uint32_t)node, nx = (uint32_t)a.nx, ny = (uint32_t)a.ny;
    const uint32_t r = nd / nx;
    const int ix = (int)(nd - r * nx), iz = (int)(r / ny), iy = (int)(r - (uint32_t)iz * ny);
    const int64_t p = (int64_t)(ix + kHalo) + (int64_t)(iy + kHalo) * a.PX + (int64_t)(iz + kHalo) * a.PXY;
    double L[3];
    for (int d = 0; d < 3; ++d) {
        const bool fixed = d == 2 && z_fixed(inf);
        const double g = fixed ? 0.0 : a.ub_next[3 * node + d];
        const double wt = fixed ? 0.0 : a.wb[3 * node + d] + a.dt * g;
        L[d] = a.a2 * wt;
        a.wb[3 * node + d] = a.a1 * wt;
    }
    if (a.seed && inf.bc >= 0) L[2] += -a.V;
    a.Lb[p] = make_double4(L[0], L[1], L[2], 0.0);
}

// ubar^m = mask(ubar^{m+1}) - sum over bond directions of the force and
// damage-history adjoints; field gradients accumulate per node (each bond's
// share is computed by both of its nodes, half each).
template <typename T>
__global__ __launch_bounds__(256) void adj_gather(AdjParams a, const typename Vec4<T>::t *__restrict__ U,
                                                  const T *__restrict__ kap, const T *__restrict__ kap_prev)
{
    using V4 = typename Vec4<T>::t;
    const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= a.M) return;
    const NodeInfo inf = a.info[node];
    const uint32_t nd = (uint32_t)node, nx = (uint32_t)a.nx, ny = (uint32_t)a.ny;
    const uint32_t r = nd / nx;
    const int ix = (int)(nd - r * nx), iz = (int)(r / ny), iy = (int)(r - (uint32_t)iz * ny);
    const int64_t p = (int64_t)(ix + kHalo) + (int64_t)(iy + kHalo) * a.PX + (int64_t)(iz + kHalo) * a.PXY;
    const V4 ui = U[p];
    const double4 Li = a.Lb[p];
    const double s0i = a.s0pad[p], ci = a.cpad[p];
    const uint4 cm = inf.cut >= 0 ? a.cut[inf.cut] : make_uint4(0, 0, 0, 0);
    double acc[3];
    for (int d = 0; d < 3; ++d) acc[d] = (d == 2 && z_fixed(inf)) ? 0.0 : a.ub_next[3 * node + d];
    double g_s0 = 0.0, g_c = 0.0;
    for (int k = 0; k < kStencil; ++k) {
        const SlotEntry e = c_slots.e[k];
        const int64_t off = (int64_t)e.x + (int64_t)e.y * a.PX + (int64_t)e.z * a.PXY;
        const V4 uj = U[p + off];
        const uint32_t bits = k < 32 ? cm.x : k < 64 ? cm.y : k < 96 ? cm.z : cm.w;
        if (uj.w == T(0) || ((bits >> (k & 31)) & 1u)) continue;
        // bond geometry in units of dx: y = v + e
        const double ex = (double)uj.x - (double)ui.x, ey = (double)uj.y - (double)ui.y,
                     ez = (double)uj.z - (double)ui.z;
        const double yx = e.x + ex, yy = e.y + ey, yz = e.z + ez;
        const double num = ex * (2.0 * e.x + ex) + ey * (2.0 * e.y + ey) + ez * (2.0 * e.z + ez);
        const double vl = c_sqrt_int[e.len2];
        const double ls = sqrt(e.len2 + num);
        const double s = num / (vl * (ls + vl));
        const double yhx = yx / ls, yhy = yy / ls, yhz = yz / ls;
        const double l = a.dx * ls, x0 = a.dx * vl;
        const double4 Lj = a.Lb[p + off];
        const double Fx = Li.x - Lj.x, Fy = Li.y - Lj.y, Fz = Li.z - Lj.z;
        const double proj = yhx * Fx + yhy * Fy + yhz * Fz;
        const double s0b = 0.5 * (s0i + a.s0pad[p + off]);
        const double cb = 0.5 * (ci + a.cpad[p + off]);
        const double sc = s0b + a.gamma / (cb * s0b);
        const int64_t ks = (int64_t)k * a.M + node;
        const double kp = (double)kap[ks];
        double keep, dk, ds0, dsc;
        keep_partials(a.law, kp, s0b, sc, a.k, a.alpha, keep, dk, ds0, dsc);
        const double cJ = a.V * cb * keep;
        double bx = cJ * (yhx * proj / x0 + (s / l) * (Fx - yhx * proj));
        double by = cJ * (yhy * proj / x0 + (s / l) * (Fy - yhy * proj));
        double bz = cJ * (yhz * proj / x0 + (s / l) * (Fz - yhz * proj));
        double kbv = a.kb[ks] + a.V * cb * s * dk * proj;
        const double dsc_dc = -a.gamma / (cb * cb * s0b);
        const double dsc_ds0 = 1.0 - a.gamma / (cb * s0b * s0b);
        g_c += 0.5 * a.V * s * proj * (keep + cb * dsc * dsc_dc);
        g_s0 += 0.5 * a.V * cb * s * proj * (ds0 + dsc * dsc_ds0);
        if (kp != (double)kap_prev[ks]) {   // the history grew at this step
            bx += kbv * yhx / x0;
            by += kbv * yhy / x0;
            bz += kbv * yhz / x0;
            kbv = 0.0;
        }
        a.kb[ks] = kbv;
        acc[0] -= bx;
        acc[1] -= by;
        acc[2] -= bz;
    }
    for (int d = 0; d < 3; ++d) a.ub_out[3 * node + d] = acc[d];
    a.gs0[node] += g_s0;
    a.gc[node] += g_c;
}

template <typename T>
__global__ void pad_fields_kernel(double *s0pad, double *cpad, const double *s0, const double *c, double s0_const,
                                  double c_const, int64_t P, int nx, int ny, int nz, int PX, int64_t PXY)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P) return;
    const int i = (int)(q % PX) - kHalo;
    const int64_t rr = q / PX;
    const int j = (int)(rr % (PXY / PX)) - kHalo, kk = (int)(rr / (PXY / PX)) - kHalo;
    double sv = 1.0, cv = 0.0;
    if (i >= 0 && i < nx && j >= 0 && j < ny && kk >= 0 && kk < nz) {
        const int64_t node = i + (int64_t)nx * (j + (int64_t)ny * kk);
        sv = s0 ? s0[node] : s0_const;
        cv = c ? c[node] : c_const;
    }
    s0pad[q] = sv;
    cpad[q] = cv;
}

struct DevBuf {
    std::vector<void *> ptrs;
    int get(void **p, size_t bytes)
    {
        hipError_t e = hipMalloc(p, bytes ? bytes : 16);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(adjoint)");
        ptrs.push_back(*p);
        return PD_OK;
    }
    ~DevBuf()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
};

template <typename T>
static int qoi_grad(pd_mesh_s *m, const pd_params *p, const double *s0_dev, const double *c_dev, double *dq_ds0,
                    double *dq_dc, double *peak_out, int64_t *peak_step_out, hipStream_t st)
{
    using V4 = typename Vec4<T>::t;
    Solve s{};
    s.m = m;
    s.p = *p;
    s.n_steps = p->n_steps;
    int rc = check_params(m, p, &s.mat);
    if (rc) return rc;
    const int64_t N = p->n_steps;
    if (N < 1) return fail(PD_EINVAL, "n_steps must be positive for a gradient");
    const int64_t K = p->checkpoint_every > 0 ? p->checkpoint_every : 200;
    if ((rc = alloc_run(m, 1, sizeof(T) == 8, p->accumulate, c_dev != nullptr, false, N, s.b, true))) {
        s.b.release();
        return rc;
    }
    const bool kahan = s.b.comp_state;   // the forward carries compensation arrays to checkpoint
    struct Release {
        RunBuffers &b;
        ~Release() { b.release(); }
    } release{s.b};
    if ((rc = setup_solve<T>(s, s0_dev, m->M, c_dev, m->M, st))) return rc;
    s.shape = known_shape(s);

    const size_t ubytes = sizeof(V4) * m->P, vbytes = vel_components(m) * sizeof(T) * m->M, hbytes = sizeof(T) * kStencil * m->M;
    const size_t dbytes = sizeof(uint4) * m->M;
    const int64_t n_ck = (N + K - 1) / K;
    DevBuf mem;
    std::vector<void *> ck_u(n_ck), ck_vh(n_ck), ck_cu(n_ck), ck_cvh(n_ck), ck_h(n_ck), ck_d(n_ck);
    for (int64_t c = 0; c < n_ck; ++c) {
        if ((rc = mem.get(&ck_u[c], ubytes)) || (rc = mem.get(&ck_vh[c], vbytes)) || (rc = mem.get(&ck_h[c], hbytes)) ||
            (rc = mem.get(&ck_d[c], dbytes)))
            return rc;
        if (kahan && ((rc = mem.get(&ck_cu[c], vbytes)) || (rc = mem.get(&ck_cvh[c], vbytes)))) return rc;
    }
    auto d2d = [&](void *dst, const void *src, size_t n) { return hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, st); };
    // forward with checkpoints: before launch k the state is (u^{k+1}, w^k, kappa^k)
    // plus the damaged-bond bits of kappa^k
    for (int64_t k = 0; k < N; ++k) {
        if (k % K == 0) {
            const int64_t c = k / K;
            PD_HIP(d2d(ck_u[c], s.b.u[k & 1], ubytes));
            PD_HIP(d2d(ck_vh[c], s.b.vh, vbytes));
            PD_HIP(d2d(ck_h[c], s.b.hist, hbytes));
            PD_HIP(d2d(ck_d[c], s.b.dmask, dbytes));
            if (kahan) {
                PD_HIP(d2d(ck_cu[c], s.b.cu, vbytes));
                PD_HIP(d2d(ck_cvh[c], s.b.cvh, vbytes));
            }
        }
        launch_step<T>(s, (int)k, st);
    }
    launch_step<T>(s, (int)N, st);   // forms R^N
    PD_HIP(hipGetLastError());
    double Q = 0;
    int64_t nstar = 0;
    int32_t status = 0;
    PD_HIP(hipMemcpyAsync(&Q, s.b.Q, 8, hipMemcpyDeviceToHost, st));
    PD_HIP(hipMemcpyAsync(&nstar, s.b.nstar, 8, hipMemcpyDeviceToHost, st));
    PD_HIP(hipMemcpyAsync(&status, s.b.status, 4, hipMemcpyDeviceToHost, st));
    PD_HIP(hipStreamSynchronize(st));
    if (status == PD_EUNSTABLE) return fail(status, "the micromodulus field exceeds what dt allows");
    if (status != PD_OK) return fail(status, "the forward run went non-finite");
    if (peak_out) *peak_out = Q;
    if (peak_step_out) *peak_step_out = nstar;

    // adjoint state
    double *ub[2], *wb, *kb, *gs0, *gc, *s0pad, *cpad;
    double4 *Lb;
    if ((rc = mem.get((void **)&ub[0], 24 * m->M)) || (rc = mem.get((void **)&ub[1], 24 * m->M)) ||
        (rc = mem.get((void **)&wb, 24 * m->M)) || (rc = mem.get((void **)&kb, 8 * kStencil * m->M)) ||
        (rc = mem.get((void **)&gs0, 8 * m->M)) || (rc = mem.get((void **)&gc, 8 * m->M)) ||
        (rc = mem.get((void **)&s0pad, 8 * m->P)) || (rc = mem.get((void **)&cpad, 8 * m->P)) ||
        (rc = mem.get((void **)&Lb, sizeof(double4) * m->P)))
        return rc;
    PD_HIP(hipMemsetAsync(ub[0], 0, 24 * m->M, st));
    PD_HIP(hipMemsetAsync(wb, 0, 24 * m->M, st));
    PD_HIP(hipMemsetAsync(kb, 0, 8 * kStencil * m->M, st));
    PD_HIP(hipMemsetAsync(gs0, 0, 8 * m->M, st));
    PD_HIP(hipMemsetAsync(gc, 0, 8 * m->M, st));
    PD_HIP(hipMemsetAsync(Lb, 0, sizeof(double4) * m->P, st));
    pad_fields_kernel<T><<<blocks_for(m->P), 256, 0, st>>>(s0pad, cpad, s0_dev, c_dev, p->s0, s.mat.c_ref, m->P, m->nx,
                                                           m->ny, m->nz, m->PX, (int64_t)m->PX * m->PY);
    // segment storage: u^{cK+j} (j = 1..K) and kappa^{cK+j} (j = 0..K)
    void *useg = nullptr, *hseg = nullptr;
    if ((rc = mem.get(&useg, ubytes * (K + 1))) || (rc = mem.get(&hseg, hbytes * (K + 1)))) return rc;

    AdjParams a{};
    a.nx = m->nx;
    a.ny = m->ny;
    a.nz = m->nz;
    a.PX = m->PX;
    a.PXY = (int64_t)m->PX * m->PY;
    a.P = m->P;
    a.M = m->M;
    a.info = m->d_info;
    a.cut = m->d_cut;
    a.s0pad = s0pad;
    a.cpad = cpad;
    a.wb = wb;
    a.Lb = Lb;
    a.kb = kb;
    a.gs0 = gs0;
    a.gc = gc;
    a.dx = m->d.dx;
    a.V = s.mat.volume;
    a.gamma = s.mat.gamma;
    a.k = p->k;
    a.alpha = p->alpha;
    const double h = p->dt / (2.0 * p->rho), A = 1.0 - p->damping * h, D = 1.0 / (1.0 + p->damping * h);
    a.a1 = A * D;
    a.a2 = h * (1.0 + A * D);
    a.dt = p->dt;
    a.law = p->law;
    int cur = 0;
    for (int64_t c = (nstar - 1) / K; nstar >= 1 && c >= 0; --c) {
        const int64_t k0 = c * K, m_end = std::min<int64_t>(k0 + K, nstar);
        PD_HIP(d2d(s.b.u[k0 & 1], ck_u[c], ubytes));
        PD_HIP(d2d(s.b.vh, ck_vh[c], vbytes));
        PD_HIP(d2d(s.b.hist, ck_h[c], hbytes));
        PD_HIP(d2d(s.b.dmask, ck_d[c], dbytes));
        if (kahan) {
            PD_HIP(d2d(s.b.cu, ck_cu[c], vbytes));
            PD_HIP(d2d(s.b.cvh, ck_cvh[c], vbytes));
        }
        PD_HIP(d2d(hseg, s.b.hist, hbytes));
        for (int64_t k = k0; k < m_end; ++k) {
            const int64_t j = k - k0 + 1;
            PD_HIP(d2d((char *)useg + ubytes * j, s.b.u[k & 1], ubytes));
            launch_step<T>(s, (int)k, st);
            PD_HIP(d2d((char *)hseg + hbytes * j, s.b.hist, hbytes));
        }
        for (int64_t mm = m_end; mm > k0; --mm) {
            const int64_t j = mm - k0;
            a.ub_next = ub[cur];
            a.ub_out = ub[cur ^ 1];
            a.seed = mm == nstar;
            adj_elementwise<<<blocks_for(m->M), 256, 0, st>>>(a);
            adj_gather<T><<<blocks_for(m->M), 256, 0, st>>>(a, (const V4 *)((char *)useg + ubytes * j),
                                                            (const T *)((char *)hseg + hbytes * j),
                                                            (const T *)((char *)hseg + hbytes * (j - 1)));
            cur ^= 1;
        }
        PD_HIP(hipGetLastError());
    }
    if (dq_ds0) PD_HIP(hipMemcpyAsync(dq_ds0, gs0, 8 * m->M, hipMemcpyDeviceToDevice, st));
    if (dq_dc) PD_HIP(hipMemcpyAsync(dq_dc, gc, 8 * m->M, hipMemcpyDeviceToDevice, st));
    PD_HIP(hipStreamSynchronize(st));
    return PD_OK;
}

}  // namespace pdmi

using namespace pdmi;

extern "C" {

int pd_qoi_grad(pd_mesh m, const pd_params *p, const double *s0_dev, const double *c_dev, double *dq_ds0_dev,
                double *dq_dc_dev, double *peak_out, int64_t *peak_step_out, void *stream)
{
    if (!m || !p) return fail(PD_EINVAL, "null argument");
    if (p->n_steps > (int64_t)1 << 30) return fail(PD_EINVAL, "n_steps too large");
    int rc = ensure_device(m);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (p->precision == PD_FP64)
        return qoi_grad<double>(m, p, s0_dev, c_dev, dq_ds0_dev, dq_dc_dev, peak_out, peak_step_out, st);
    return qoi_grad<float>(m, p, s0_dev, c_dev, dq_ds0_dev, dq_dc_dev, peak_out, peak_step_out, st);
}

}  // extern "C"
