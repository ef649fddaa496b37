// Run management of the explicit peridynamic solve and the C entry points
// for meshes, single runs, force evaluations and batches.  The step kernel
// itself is in step_kernels.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "pd_internal.h"
#include "run.h"
#include "step_launch.h"

namespace pdmi {

const char *last_error();

template <typename T>
static void launch_step_impl(const Solve &s, int k_local, hipStream_t st, double *L_out)
{
    StepParams<T> a = make_step_params<T>(s, k_local);
    if (L_out) {
        a.L_out = L_out;
        a.force_only = 1;
    }
    const int shape = effective_shape(s.b.f64, s.b.kahan, s.b.has_c, s.shape);
    const bool plane = plane_mesh(s.m);
    dim3 grid((unsigned)step_blocks(s.m, s.b.S, (plane ? kPlaneShapes : kShapes)[shape]));
    if constexpr (sizeof(T) == 4) {
        if (s.b.kahan) {
            if (s.b.has_c) launch_f32_kahan_c(shape, plane, grid, st, a);
            else launch_f32_kahan(shape, plane, grid, st, a);
        } else {
            if (s.b.has_c) launch_f32_plain_c(shape, plane, grid, st, a);
            else launch_f32_plain(shape, plane, grid, st, a);
        }
    } else {
        if (s.b.has_c) launch_f64_c(shape, plane, grid, st, a);
        else launch_f64(shape, plane, grid, st, a);
    }
}

void launch_step_f32(const Solve &s, int k_local, hipStream_t st, double *L_out)
{
    launch_step_impl<float>(s, k_local, st, L_out);
}

void launch_step_f64(const Solve &s, int k_local, hipStream_t st, double *L_out)
{
    launch_step_impl<double>(s, k_local, st, L_out);
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
    if (field != PD_FIELD_S0 && field != PD_FIELD_C && field != PD_FIELD_GF)
        return fail(PD_EINVAL, "unknown field %d", field);
    if (dtype != PD_DTYPE_F32 && dtype != PD_DTYPE_F64) return fail(PD_EINVAL, "unknown dtype %d", dtype);
    double **dst = field == PD_FIELD_S0 ? &m->d_s0 : field == PD_FIELD_C ? &m->d_c : &m->d_gf;
    int64_t *cnt = field == PD_FIELD_S0 ? &m->s0_samples : field == PD_FIELD_C ? &m->c_samples : &m->gf_samples;
    auto clear = [&]() {
        if (*dst) (void)hipFree(*dst);
        *dst = nullptr;
        *cnt = 0;
        if (field == PD_FIELD_C) m->c_max = 0.0;
    };
    if (!values) {
        clear();
        return PD_OK;
    }
    if (n_samples < 1) return fail(PD_EINVAL, "n_samples must be positive");
    int rc = ensure_device(m);
    if (rc) return rc;
    const int64_t n = n_samples * m->M;
    hipStream_t st = (hipStream_t)stream;
    // checked and converted on the device into a new buffer (host values are
    // uploaded first); the old field is replaced only if every value passes
    void *src = const_cast<void *>(values);
    void *staged = nullptr;
    double *fresh = nullptr;
    unsigned long long flags[2] = {0, 0};
    unsigned long long *d_flags = nullptr;
    const size_t esz = dtype == PD_DTYPE_F64 ? 8 : 4;
    hipError_t e = hipMalloc(&fresh, 8 * n);
    if (e == hipSuccess) e = hipMalloc(&d_flags, sizeof(flags));
    if (e == hipSuccess) e = hipMemcpyAsync(d_flags, flags, sizeof(flags), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !on_device) {
        e = hipMalloc(&staged, esz * n);
        if (e == hipSuccess) e = hipMemcpyAsync(staged, values, esz * n, hipMemcpyHostToDevice, st);
        src = staged;
    }
    if (e == hipSuccess) {
        if (dtype == PD_DTYPE_F64)
            field_copy_check_kernel<double><<<stride_blocks(n), 256, 0, st>>>((const double *)src, n, fresh, d_flags);
        else
            field_copy_check_kernel<float><<<stride_blocks(n), 256, 0, st>>>((const float *)src, n, fresh, d_flags);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(flags, d_flags, sizeof(flags), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (staged) (void)hipFree(staged);
    if (d_flags) (void)hipFree(d_flags);
    if (e != hipSuccess) {
        if (fresh) (void)hipFree(fresh);
        return hip_fail(e, "pd_set_material_field");
    }
    if (flags[0] != 0) {
        (void)hipFree(fresh);
        return fail(PD_EINVAL, "field values must be positive and finite (%llu are not)", flags[0]);
    }
    clear();
    *dst = fresh;
    *cnt = n_samples;
    if (field == PD_FIELD_C) {
        double mx;
        std::memcpy(&mx, &flags[1], sizeof(mx));
        m->c_max = mx;
    }
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
    if (m->d_gf) (void)hipFree(m->d_gf);
    delete m;
    return PD_OK;
}

int pd_force_eval(pd_mesh m, const pd_params *p, int64_t n_samples, const double *u_host, double *L_host,
                  void *stream)
{
    if (!m || !p || !u_host || !L_host) return fail(PD_EINVAL, "null argument");
    if (n_samples < 1 || n_samples > 65535) return fail(PD_EINVAL, "n_samples out of range");
    int rc = ensure_device(m);
    if (rc) return rc;
    Solve s{};
    s.m = m;
    s.p = *p;
    if ((rc = material_from_params(m, p, &s.mat))) return rc;
    if (m->s0_samples && m->s0_samples != n_samples) return fail(PD_EINVAL, "s0 field has %lld samples", (long long)m->s0_samples);
    if (m->c_samples && m->c_samples != n_samples) return fail(PD_EINVAL, "c field has %lld samples", (long long)m->c_samples);
    if (m->gf_samples && m->gf_samples != n_samples)
        return fail(PD_EINVAL, "fracture-energy field has %lld samples", (long long)m->gf_samples);
    s.n_steps = 0;
    bool f64 = p->precision == PD_FP64;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = alloc_run(m, (int)n_samples, f64, p->accumulate, m->d_c != nullptr, false, 0, s.b, true,
                        m->d_gf != nullptr))) {
        s.b.release();
        return rc;
    }
    double *dL = nullptr;
    std::vector<char> host;
    size_t ts = f64 ? 8 : 4;
    do {
        if (f64) rc = setup_solve<double>(s, m->d_s0, m->M, m->d_c, m->M, st, m->d_gf, m->M);
        else rc = setup_solve<float>(s, m->d_s0, m->M, m->d_c, m->M, st, m->d_gf, m->M);
        if (rc) break;
        s.shape = known_shape(s);
        // displacements into the padded grid (units of dx), flag 1 (0 in ghosts)
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
        if (s.b.has_c && !plane_mesh(m)) {
            // a 3D body keeps each node's c / c_ref in its flag word
            const int64_t n = m->P * n_samples;
            if (f64) flag_from_c_kernel<double><<<stride_blocks(n), 256, 0, st>>>((double4 *)s.b.u[0], (const double *)s.b.cpad, n);
            else flag_from_c_kernel<float><<<stride_blocks(n), 256, 0, st>>>((float4 *)s.b.u[0], (const float *)s.b.cpad, n);
        }
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
    if (m->s0_samples > 1 || m->c_samples > 1 || m->gf_samples > 1)
        return fail(PD_EINVAL, "pd_run takes single-sample fields");
    pd_run_s *r = new (std::nothrow) pd_run_s();
    if (!r) return fail(PD_ENOMEM, "out of host memory");
    r->s.m = m;
    r->s.p = *p;
    r->s.n_steps = p->n_steps;
    r->stream = (hipStream_t)stream;
    Material mref;
    if ((rc = material_from_params(m, p, &mref))) {
        delete r;
        return rc;
    }
    // a micromodulus field stiffens bonds up to its largest value
    const double cmax = m->d_c ? std::max(1.0, m->c_max / mref.c_ref) : 1.0;
    if ((rc = check_params(m, p, &r->s.mat, cmax))) {
        delete r;
        return rc;
    }
    bool f64 = p->precision == PD_FP64;
    rc = alloc_run(m, 1, f64, p->accumulate, m->d_c != nullptr, p->record_history != 0, p->n_steps,
                   r->s.b, true, m->d_gf != nullptr);
    if (!rc) rc = f64 ? setup_solve<double>(r->s, m->d_s0, m->M, m->d_c, m->M, r->stream, m->d_gf, m->M)
                      : setup_solve<float>(r->s, m->d_s0, m->M, m->d_c, m->M, r->stream, m->d_gf, m->M);
    if (!rc) rc = f64 ? choose_shape<double, double>(r->s, m->d_s0, m->M, m->d_c, m->M, r->stream, m->d_gf, m->M)
                      : choose_shape<float, double>(r->s, m->d_s0, m->M, m->d_c, m->M, r->stream, m->d_gf, m->M);
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
    if (status == PD_EUNSTABLE) return fail(status, "the micromodulus field exceeds what dt allows");
    if (status != PD_OK) return fail(status, "the run went non-finite");
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

int pd_set_launch_shape(pd_mesh m, int32_t shape)
{
    if (!m) return fail(PD_EINVAL, "null mesh");
    if (shape < PD_SHAPE_AUTO || shape >= PD_N_SHAPES) return fail(PD_EINVAL, "unknown launch shape %d", shape);
    m->shape_override = shape;
    return PD_OK;
}

int pd_autotune(pd_mesh m, const pd_params *p, int64_t n_samples, void *stream, int32_t *shape_out,
                double *us_per_step_out)
{
    if (!m || !p) return fail(PD_EINVAL, "null argument");
    if (n_samples < 1 || n_samples > 65535) return fail(PD_EINVAL, "n_samples out of range");
    int rc = ensure_device(m);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    Solve s{};
    s.m = m;
    s.p = *p;
    s.n_steps = p->n_steps;
    if ((rc = check_params(m, p, &s.mat))) return rc;
    const bool f64 = p->precision == PD_FP64;
    rc = alloc_run(m, (int)n_samples, f64, p->accumulate, false, false, 0, s.b, true);
    int best = PD_SHAPE_GLOBAL_256;
    if (!rc) rc = f64 ? setup_solve<double>(s, (const double *)nullptr, 0, (const double *)nullptr, 0, st)
                      : setup_solve<float>(s, (const double *)nullptr, 0, (const double *)nullptr, 0, st);
    if (!rc) rc = f64 ? autotune_shapes<double>(s, st, 8, &best, us_per_step_out)
                      : autotune_shapes<float>(s, st, 8, &best, us_per_step_out);
    (void)hipStreamSynchronize(st);
    s.b.release();
    if (rc) return rc;
    if (!f64) {
        std::lock_guard<std::mutex> g(tune_cache().mu);
        tune_cache().best[tune_key(s)] = best;
    }
    if (shape_out) *shape_out = best;
    return PD_OK;
}

static int64_t gcd64(int64_t a, int64_t b) { return b ? gcd64(b, a % b) : a; }

// Executable graphs of batches still in flight, destroyed once the event
// recorded after their last launch has completed.
struct PendingGraph {
    hipStream_t stream;
    hipGraphExec_t exec;
    hipEvent_t done;
};

static std::mutex g_pending_mu;
static std::vector<PendingGraph> g_pending;

// Destroys the graphs whose batches have completed; with `wait`, first
// synchronises `stream` (every graph of that stream completes).
static void reap_graphs(bool wait, hipStream_t stream)
{
    std::lock_guard<std::mutex> g(g_pending_mu);
    std::vector<PendingGraph> keep;
    for (const PendingGraph &pg : g_pending) {
        const bool mine = wait && pg.stream == stream;
        if (mine || hipEventQuery(pg.done) == hipSuccess) {
            if (mine) (void)hipEventSynchronize(pg.done);
            (void)hipGraphExecDestroy(pg.exec);
            (void)hipEventDestroy(pg.done);
        } else {
            keep.push_back(pg);
        }
    }
    g_pending.swap(keep);
}

int pd_run_batch(const pd_batch_item *items, int32_t n_items, void *stream)
{
    if (!items || n_items < 1) return fail(PD_EINVAL, "empty batch");
    hipStream_t st = (hipStream_t)stream;
    reap_graphs(false, st);
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
        // a micromodulus field is checked per sample on the device (status
        // PD_EUNSTABLE for a sample whose field exceeds what dt allows)
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
    const int acc = items[0].params->accumulate;
    std::vector<void *> scratch;
    for (int i = 0; i < n_items && !rc; ++i) {
        const pd_batch_item &it = items[i];
        Solve &s = solves[i];
        s.m = it.mesh;
        s.p = *it.params;
        s.n_steps = it.params->n_steps;
        material_from_params(it.mesh, it.params, &s.mat);
        s.b.use_ordered = true;   // released in stream order: the call does not wait for the batch
        s.b.ordered = st;
        rc = alloc_run(it.mesh, (int)it.n_samples, f64, acc, it.c != nullptr, false, s.n_steps, s.b, false,
                       it.gf != nullptr);
        if (rc) break;
        s.b.Q = it.qoi;
        s.b.nstar = (int64_t *)it.nstar;
        s.b.status = it.status;
        if (!s.b.nstar) rc = s.b.alloc((void **)&s.b.nstar, 8 * it.n_samples);
        if (!rc && !s.b.status) rc = s.b.alloc((void **)&s.b.status, 4 * it.n_samples);
        if (rc) break;
        int64_t M = it.mesh->M;
        if (it.field_dtype == PD_DTYPE_F64) {
            const double *s0 = (const double *)it.s0, *c = (const double *)it.c, *gf = (const double *)it.gf;
            rc = f64 ? setup_solve<double, double>(s, s0, M, c, M, st, gf, M)
                     : setup_solve<float, double>(s, s0, M, c, M, st, gf, M);
            if (!rc) rc = f64 ? choose_shape<double, double>(s, s0, M, c, M, st, gf, M)
                              : choose_shape<float, double>(s, s0, M, c, M, st, gf, M);
        } else {
            const float *s0 = (const float *)it.s0, *c = (const float *)it.c, *gf = (const float *)it.gf;
            rc = f64 ? setup_solve<double, float>(s, s0, M, c, M, st, gf, M)
                     : setup_solve<float, float>(s, s0, M, c, M, st, gf, M);
            if (!rc) rc = f64 ? choose_shape<double, float>(s, s0, M, c, M, st, gf, M)
                              : choose_shape<float, float>(s, s0, M, c, M, st, gf, M);
        }
    }
    // Schedule: by default each item's chain of step launches is a branch
    // of the graph (below).  PD_BATCH_SCHEDULE=tick asks instead for one
    // launch per tick over the work items of every item stepping at that
    // tick (the tick kernel), which items can share when they are FP32
    // compensated 3D solves with the same micromodulus mode, at most
    // kMaxTickItems of them; they then take the launch shape of the item with
    // the most work per tick.  Both give the same results bit for bit; on
    // the three-level cracking hierarchy the branches are about 7% faster
    // (the tick launches cannot overlap one another's tails).
    const char *sched = getenv("PD_BATCH_SCHEDULE");
    bool tick = sched && !strcmp(sched, "tick") && !rc && n_items > 1 && n_items <= kMaxTickItems && !f64 &&
                acc == PD_ACC_KAHAN;
    for (int i = 0; tick && i < n_items; ++i)
        tick = !plane_mesh(items[i].mesh) && (items[i].c != nullptr) == (items[0].c != nullptr);
    if (tick) {
        int big = 0;
        for (int i = 1; i < n_items; ++i)
            if ((double)items[i].n_samples * items[i].mesh->M / ratio[i] >
                (double)items[big].n_samples * items[big].mesh->M / ratio[big])
                big = i;
        // one tick launch holds every item's work items: it too must stay
        // below 2^32 work-items, else the batch keeps the branches
        const int shape = solves[big].shape;
        const LaunchShape &sh = kShapes[effective_shape(false, true, items[0].c != nullptr, shape)];
        int64_t blocks = 0;
        for (int i = 0; i < n_items; ++i) blocks += step_blocks(items[i].mesh, items[i].n_samples, sh);
        if (blocks * sh.threads > (int64_t)UINT32_MAX) tick = false;
        for (int i = 0; tick && i < n_items; ++i) solves[i].shape = shape;
    }
    hipGraphExec_t exec = nullptr;
    if (!rc && ticks > 0 && tick) {
        const int64_t H = 2 * lcm * std::max<int64_t>(1, 32 / lcm);
        const int shape = effective_shape(false, true, items[0].c != nullptr, solves[0].shape);
        hipStream_t cap = capture_stream();
        hipGraph_t g = nullptr;
        // items with the most work per tick first in the work list
        std::vector<int> order(n_items);
        for (int i = 0; i < n_items; ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](int x, int y) {
            return (double)items[x].n_samples * items[x].mesh->M / ratio[x] <
                   (double)items[y].n_samples * items[y].mesh->M / ratio[y];
        });
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamBeginCapture");
        if (!rc) {
            for (int64_t t = 0; t < H; ++t) {
                TickParams<float> tp{};
                int n = 0;
                int64_t at = 0;
                for (int j = n_items - 1; j >= 0; --j) {
                    const int i = order[j];
                    if (t % ratio[i] != 0) continue;
                    tp.p[n] = make_step_params<float>(solves[i], (int)(t / ratio[i]));
                    tp.first[n] = at;
                    at += tp.p[n].n_items;
                    ++n;
                }
                tp.first[n] = at;
                tp.n = n;
                if (!n) continue;
                const dim3 grid((unsigned)((at + kXcds - 1) / kXcds * kXcds));
                if (items[0].c) launch_tick_f32_kahan_c(shape, grid, cap, tp);
                else launch_tick_f32_kahan(shape, grid, cap, tp);
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
        for (int i = 0; !rc && i < n_items; ++i) launch_step<float>(solves[i], 0, st);
    }
    if (!rc && ticks > 0 && !tick) {
        // one hyper-period of 2 * lcm ticks: every item takes an even number
        // of steps in it, so the ping-pong parity of a replay is fixed
        int64_t H = 2 * lcm * std::max<int64_t>(1, 32 / lcm);
        // The items share no mutable state, so each one's chain of steps is
        // a branch of its own in the graph (forked from and joined into the
        // capture stream): a small level's launches fill the CUs that a
        // large level's tail leaves idle.  Every branch runs its steps in
        // order, so the results do not depend on how the branches overlap.
        hipStream_t cap = capture_stream();
        std::vector<hipStream_t> br;
        std::vector<hipEvent_t> ev(n_items + 1, nullptr);
        hipGraph_t g = nullptr;
        rc = branch_streams(n_items, br);
        for (auto &x : ev) {
            if (rc) break;
            hipError_t ee = hipEventCreateWithFlags(&x, hipEventDisableTiming);
            if (ee != hipSuccess) rc = hip_fail(ee, "hipEventCreate");
        }
        hipError_t e = rc ? hipSuccess : hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamBeginCapture");
        if (!rc) {
            e = hipEventRecord(ev[n_items], cap);
            for (int i = 0; e == hipSuccess && i < n_items; ++i) {
                e = hipStreamWaitEvent(br[i], ev[n_items], 0);
                if (e != hipSuccess) break;
                for (int64_t k = 0; k < H / ratio[i]; ++k) {
                    if (f64) launch_step<double>(solves[i], (int)k, br[i]);
                    else launch_step<float>(solves[i], (int)k, br[i]);
                }
                launch_advance(solves[i], H / ratio[i], br[i]);
                e = hipEventRecord(ev[i], br[i]);
                if (e == hipSuccess) e = hipStreamWaitEvent(cap, ev[i], 0);
            }
            if (e != hipSuccess) rc = hip_fail(e, "graph branches");
            e = hipStreamEndCapture(cap, &g);
            if (e != hipSuccess && !rc) rc = hip_fail(e, "hipStreamEndCapture");
        }
        if (!rc) {
            e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) rc = hip_fail(e, "hipGraphInstantiate");
        }
        if (g) (void)hipGraphDestroy(g);
        for (auto x : ev)
            if (x) (void)hipEventDestroy(x);
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
    for (int i = 0; !rc && i < n_items; ++i)
        if (items[i].u_out) launch_export_u(solves[i], items[i].u_out, st);
    if (!rc) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) rc = hip_fail(e, "batch");
    }
    // buffers go back in stream order; the graph is destroyed once its last
    // launch has completed (on a later call or in pd_batch_sync)
    for (auto &s : solves) s.b.release();
    if (exec) {
        hipEvent_t done = nullptr;
        hipError_t e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(done, st);
        if (e == hipSuccess) {
            std::lock_guard<std::mutex> g(g_pending_mu);
            g_pending.push_back(PendingGraph{st, exec, done});
        } else {
            (void)hipStreamSynchronize(st);
            (void)hipGraphExecDestroy(exec);
            if (done) (void)hipEventDestroy(done);
            if (!rc) rc = hip_fail(e, "batch completion event");
        }
    }
    if (rc) (void)hipStreamSynchronize(st);
    return rc;
}

int pd_batch_sync(void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    PD_HIP(hipStreamSynchronize(st));
    reap_graphs(true, st);
    return PD_OK;
}

}  // extern "C"

