// pd_run_batch_static: the batched solve of pd_run_batch with every work
// buffer carved from one file-scope device array, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops).
//
// Each device that runs it holds its own copy of `scratch` for the life of
// the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (the array's name is a
// host-side stand-in, not a device address).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "pd_internal.h"
#include "run.h"

namespace pdmi {

constexpr size_t kStaticScratchBytes = size_t(256) << 20;   // 256 MiB
constexpr int kMaxStaticItems = 8;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
static int scratch_on_current_device(char **out)
{
    static std::mutex mu;
    static char *addr[kMaxDevices] = {};
    int dev = -1;
    PD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PD_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        addr[dev] = (char *)p;
    }
    *out = addr[dev];
    return PD_OK;
}

// Buffers of every item, sized (arena = null) or carved from the arena.
static int carve(const pd_batch_item *items, int n_items, bool f64, int acc, Solve *solves, char *arena,
                 size_t *used)
{
    *used = 0;
    for (int i = 0; i < n_items; ++i) {
        const pd_batch_item &it = items[i];
        Solve &s = solves[i];
        s = Solve{};
        s.m = it.mesh;
        s.p = *it.params;
        s.n_steps = it.params->n_steps;
        int rc = material_from_params(it.mesh, it.params, &s.mat);
        if (rc) return rc;
        s.b.arena_mode = true;
        s.b.arena = arena;
        s.b.arena_used = used;
        rc = alloc_run(it.mesh, (int)it.n_samples, f64, acc, it.c != nullptr, false, s.n_steps, s.b, false,
                       it.gf != nullptr);
        if (rc) return rc;
        s.b.Q = it.qoi;
        s.b.nstar = it.nstar;
        s.b.status = it.status;
        if (!s.b.nstar && (rc = s.b.alloc((void **)&s.b.nstar, 8 * it.n_samples))) return rc;
        if (!s.b.status && (rc = s.b.alloc((void **)&s.b.status, 4 * it.n_samples))) return rc;
    }
    return PD_OK;
}

// Set-up kernels of one item (fill kernels only: every buffer that must
// start at a fixed value is written, since the arena keeps the last call's
// contents), and its launch shape: pinned, else the autotuner's cached
// choice, else the default brick (no measurement: that would allocate).
template <typename T, typename In>
static int setup_item(Solve &s, const pd_batch_item &it, hipStream_t st)
{
    const int64_t M = it.mesh->M;
    const int rc = setup_solve<T, In>(s, (const In *)it.s0, M, (const In *)it.c, M, st, (const In *)it.gf, M);
    s.shape = known_shape(s);
    return rc;
}

}  // namespace pdmi

using namespace pdmi;

extern "C" int pd_run_batch_static(const pd_batch_item *items, int32_t n_items, void *stream)
{
    if (!items || n_items < 1) return fail(PD_EINVAL, "empty batch");
    if (n_items > kMaxStaticItems) return fail(PD_EINVAL, "at most %d items per call", kMaxStaticItems);
    hipStream_t st = (hipStream_t)stream;
    double dt_min = INFINITY;
    for (int i = 0; i < n_items; ++i) {
        const pd_batch_item &it = items[i];
        if (!it.mesh || !it.params || !it.qoi) return fail(PD_EINVAL, "item %d: null mesh, params or qoi", i);
        if (it.n_samples < 1 || it.n_samples > 65535) return fail(PD_EINVAL, "item %d: n_samples out of range", i);
        if (!it.mesh->bonds_built) return fail(PD_ESTATE, "item %d: pd_build_bonds has not been called", i);
        // the mesh tables must already be on the device (pd_build_bonds uploads them)
        if (!it.mesh->d_info) return fail(PD_ESTATE, "item %d: mesh tables are not on the device", i);
        int dev = -1;
        PD_HIP(hipGetDevice(&dev));
        if (dev != it.mesh->device) return fail(PD_EDEVICE, "item %d: mesh lives on device %d", i, it.mesh->device);
        if (it.params->precision != items[0].params->precision || it.params->accumulate != items[0].params->accumulate)
            return fail(PD_EINVAL, "all batch items must share precision and accumulate");
        if (it.field_dtype != PD_DTYPE_F32 && it.field_dtype != PD_DTYPE_F64)
            return fail(PD_EINVAL, "item %d: unknown field dtype", i);
        if (it.params->n_steps < 0 || it.params->n_steps > ((int64_t)1 << 30))
            return fail(PD_EINVAL, "item %d: n_steps out of range", i);
        Material mat;
        int rc = check_params(it.mesh, it.params, &mat);
        if (rc) return rc;
        dt_min = std::min(dt_min, it.params->dt);
    }
    int64_t ratio[kMaxStaticItems];
    int64_t ticks = 0;
    for (int i = 0; i < n_items; ++i) {
        const double r = items[i].params->dt / dt_min;
        ratio[i] = llround(r);
        if (ratio[i] < 1 || std::fabs(r - (double)ratio[i]) > 1e-9 * r)
            return fail(PD_EINVAL, "item %d: dt is not an integer multiple of the finest dt", i);
        ticks = std::max(ticks, items[i].params->n_steps * ratio[i]);
    }
    const bool f64 = items[0].params->precision == PD_FP64;
    const int acc = items[0].params->accumulate;
    Solve solves[kMaxStaticItems];
    size_t need = 0;
    int rc = carve(items, n_items, f64, acc, solves, nullptr, &need);
    if (rc) return rc;
    if (need > kStaticScratchBytes)
        return fail(PD_EINVAL, "the batch needs %zu bytes of work memory; pd_run_batch_static has %zu", need,
                    kStaticScratchBytes);
    char *arena = nullptr;
    if ((rc = scratch_on_current_device(&arena))) return rc;
    if ((rc = carve(items, n_items, f64, acc, solves, arena, &need))) return rc;
    for (int i = 0; i < n_items && !rc; ++i) {
        const pd_batch_item &it = items[i];
        if (it.field_dtype == PD_DTYPE_F64)
            rc = f64 ? setup_item<double, double>(solves[i], it, st) : setup_item<float, double>(solves[i], it, st);
        else
            rc = f64 ? setup_item<double, float>(solves[i], it, st) : setup_item<float, float>(solves[i], it, st);
    }
    if (rc) return rc;
    // one launch per item and step, items interleaved on their common clock;
    // then one launch per item at its step N, which forms R^N
    for (int64_t t = 0; t < ticks; ++t)
        for (int i = 0; i < n_items; ++i) {
            if (t % ratio[i] != 0 || t / ratio[i] >= solves[i].n_steps) continue;
            if (f64) launch_step<double>(solves[i], (int)(t / ratio[i]), st);
            else launch_step<float>(solves[i], (int)(t / ratio[i]), st);
        }
    for (int i = 0; i < n_items; ++i) {
        if (f64) launch_step<double>(solves[i], (int)solves[i].n_steps, st);
        else launch_step<float>(solves[i], (int)solves[i].n_steps, st);
        if (items[i].u_out) launch_export_u(solves[i], items[i].u_out, st);
    }
    PD_HIP(hipGetLastError());
    return PD_OK;
}
