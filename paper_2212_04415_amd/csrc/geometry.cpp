// Host-side mesh construction: lattice, pads, notch-cut bond masks and the
// material constants of a run.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "pd_internal.h"

namespace pdmi {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    set_error("HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
    return e == hipErrorOutOfMemory ? PD_ENOMEM : PD_EDEVICE;
}

const char *last_error() { return g_err; }

// a length as a whole number of `unit`, or -1
static long whole(double len, double unit)
{
    double r = len / unit;
    long k = lround(r);
    if (std::fabs(r - (double)k) > 1e-9 * std::fmax(1.0, std::fabs(r))) return -1;
    return k;
}

// sum over the horizon of 1/|v|; in_plane: the offsets with v_y = 0 only
double stencil_inv_len_sum(bool in_plane)
{
    double s = 0.0;
    for (int k = 0; k < kHalfStencil; ++k) {
        Off o = kHalf.v[k];
        if (in_plane && o.y != 0) continue;
        s += 2.0 / std::sqrt((double)(o.x * o.x + o.y * o.y + o.z * o.z));
    }
    return s;
}

// Explicit stability limit of an interior node (Silling and Askari's bound
// for bond-based peridynamics): dt_c = sqrt(2 rho / sum_j V c / |xi_j|).
double stability_limit(const pd_mesh_s *m, double rho, double c)
{
    const double dx = m->d.dx;
    const bool plane = m->d.thickness > 0;
    const double V = plane ? dx * dx * m->d.thickness : dx * dx * dx;
    return std::sqrt(2.0 * rho / (V * c * stencil_inv_len_sum(plane) / dx));
}

int build_mesh(const pd_mesh_desc *d, pd_mesh_s *m)
{
    if (!(d->dx > 0)) return fail(PD_EINVAL, "dx must be positive");
    if (!(d->m_ratio >= 3.0 && d->m_ratio * d->m_ratio < 10.0))
        return fail(PD_EINVAL, "m_ratio %g: the kernels are built for the 122-neighbour horizon (3 <= m < sqrt(10))",
                    d->m_ratio);
    long n[3];
    for (int a = 0; a < 3; ++a) {
        n[a] = whole(d->extent[a], d->dx);
        if (n[a] < 1) return fail(PD_EINVAL, "extent[%d] = %g is not a positive multiple of dx", a, d->extent[a]);
    }
    if ((double)n[0] * n[1] * n[2] > 2.0e9) return fail(PD_EINVAL, "mesh too large");
    if (!(d->thickness >= 0)) return fail(PD_EINVAL, "thickness must be >= 0");
    if (d->thickness > 0 && n[1] != 1)
        return fail(PD_EINVAL, "a plane body has one node through the thickness (extent[1] = dx)");
    if (d->plane_strain != 0 && d->plane_strain != 1) return fail(PD_EINVAL, "plane_strain must be 0 or 1");
    if (d->plane_strain && !(d->thickness > 0)) return fail(PD_EINVAL, "plane strain needs a thickness > 0");
    m->d = *d;
    m->nx = (int)n[0];
    m->ny = (int)n[1];
    m->nz = (int)n[2];
    m->M = (int64_t)n[0] * n[1] * n[2];
    m->PX = m->nx + 2 * kHalo;
    m->PY = m->ny + 2 * kHalo;
    m->PZ = m->nz + 2 * kHalo;
    m->P = (int64_t)m->PX * m->PY * m->PZ;
    // the step kernels form per-lane byte offsets of up to 32 bytes per cell in 32 bits
    if (m->P > (int64_t(1) << 27))
        return fail(PD_EINVAL, "mesh too large: %lld cells with ghost layers (at most 2^27)", (long long)m->P);

    // notch plane x = L/2 is at half-cell coordinate nx; its tip 2a/dx
    m->notch_X = m->nx;
    m->notch_A = 0;
    if (d->notch_depth > 0) {
        long A = whole(2.0 * d->notch_depth, d->dx);
        if (A < 1) return fail(PD_EINVAL, "notch depth %g is not a multiple of dx/2", d->notch_depth);
        m->notch_A = (int)A;
    }

    // pads: a node belongs to a block when its centre lies strictly inside;
    // a centre on a face is ambiguous and rejected.  Work in half-cell units
    // where centres are odd integers.
    double w = d->pad_width, L = d->extent[0], D = d->extent[2];
    if (!(w > 0)) return fail(PD_EINVAL, "pad_width must be positive");
    struct Box { double x0, x1, z0, z1; };
    Box sup[2] = {{0.5 * (L - d->span) - 0.5 * w, 0.5 * (L - d->span) + 0.5 * w, 0.0, w},
                  {0.5 * (L + d->span) - 0.5 * w, 0.5 * (L + d->span) + 0.5 * w, 0.0, w}};
    Box ld = {0.5 * L - 0.5 * w, 0.5 * L + 0.5 * w, D - w, D};
    auto on_face = [&](double c, double f) { return std::fabs(c - f) < 1e-9 * d->dx; };
    auto inside = [&](const Box &b, int i, int k, bool *ambiguous) {
        double xc = (i + 0.5) * d->dx, zc = (k + 0.5) * d->dx;
        if (on_face(xc, b.x0) || on_face(xc, b.x1) || on_face(zc, b.z0) || on_face(zc, b.z1)) *ambiguous = true;
        return xc > b.x0 && xc < b.x1 && zc > b.z0 && zc < b.z1;
    };
    m->info.assign(m->M, NodeInfo{-1, -1});
    m->support.clear();
    m->load.clear();
    bool amb = false;
    for (int k = 0; k < m->nz; ++k)
        for (int j = 0; j < m->ny; ++j)
            for (int i = 0; i < m->nx; ++i) {
                int64_t node = i + (int64_t)m->nx * (j + (int64_t)m->ny * k);
                bool s = inside(sup[0], i, k, &amb) || inside(sup[1], i, k, &amb);
                bool l = inside(ld, i, k, &amb);
                if (s && l) return fail(PD_EINVAL, "support and load pads overlap");
                if (s) m->support.push_back((int32_t)node);
                if (l) m->load.push_back((int32_t)node);
            }
    if (amb) return fail(PD_EINVAL, "a node centre lies on a pad face");
    if (m->support.empty() || m->load.empty()) return fail(PD_EINVAL, "empty support or load pad");
    for (size_t a = 0; a < m->support.size(); ++a) m->info[m->support[a]].bc = (int32_t)a;
    for (int32_t node : m->load) m->info[node].bc = -2;
    return PD_OK;
}

// Bond (p, q) crosses the notch when, ordering its ends so X1 <= X2 in
// half-cell units, X1 < Xn <= X2 and the crossing height
// Z1 + (Xn - X1)(Z2 - Z1)/(X2 - X1) lies below the tip A.
static bool crosses_notch(int X1, int Z1, int X2, int Z2, int Xn, int A)
{
    if (X1 > X2) {
        int t = X1; X1 = X2; X2 = t;
        t = Z1; Z1 = Z2; Z2 = t;
    }
    if (!(X1 < Xn && Xn <= X2)) return false;
    long dX = X2 - X1;
    return (long)Z1 * dX + (long)(Xn - X1) * (Z2 - Z1) < (long)A * dX;
}

int build_cuts(pd_mesh_s *m)
{
    m->cut_masks.clear();
    int64_t total = 0, cut = 0;
    for (int k = 0; k < m->nz; ++k)
        for (int j = 0; j < m->ny; ++j)
            for (int i = 0; i < m->nx; ++i) {
                int64_t node = i + (int64_t)m->nx * (j + (int64_t)m->ny * k);
                uint32_t mask[4] = {0, 0, 0, 0};
                bool any = false;
                for (int s = 0; s < kStencil; ++s) {
                    Off o = slot_offset(s);
                    int i2 = i + o.x, j2 = j + o.y, k2 = k + o.z;
                    if (i2 < 0 || i2 >= m->nx || j2 < 0 || j2 >= m->ny || k2 < 0 || k2 >= m->nz) continue;
                    bool c = m->notch_A > 0 &&
                             crosses_notch(2 * i + 1, 2 * k + 1, 2 * i2 + 1, 2 * k2 + 1, m->notch_X, m->notch_A);
                    if (s < kHalfStencil) {
                        ++total;
                        if (c) ++cut;
                    }
                    if (c) {
                        mask[s >> 5] |= 1u << (s & 31);
                        any = true;
                    }
                }
                if (any) {
                    m->info[node].cut = (int32_t)(m->cut_masks.size() / 4);
                    m->cut_masks.insert(m->cut_masks.end(), mask, mask + 4);
                } else {
                    m->info[node].cut = -1;
                }
            }
    m->n_cut = cut;
    m->n_bonds = total - cut;
    return PD_OK;
}

int material_from_params(const pd_mesh_s *m, const pd_params *p, Material *out)
{
    if (!(p->E > 0) || !(p->rho > 0) || !(p->GF > 0) || !(p->s0 > 0) || !(p->k > 0) || !(p->alpha >= 0))
        return fail(PD_EINVAL, "E, rho, GF, s0, k must be positive and alpha non-negative");
    if (p->law != PD_LAW_EXPLIN && p->law != PD_LAW_TRILINEAR) return fail(PD_EINVAL, "unknown law %d", p->law);
    if (!(p->damping >= 0) || !(p->dt > 0) || p->n_steps < 0) return fail(PD_EINVAL, "bad damping, dt or n_steps");
    if (!std::isfinite(p->du)) return fail(PD_EINVAL, "du must be finite");
    double dx = m->d.dx;
    const double t = m->d.thickness;
    out->delta = m->d.m_ratio * dx;
    // bond stiffness constant (appendix A, Eq. bond_stiffness_constant)
    if (t > 0) {
        out->c_ref = (m->d.plane_strain ? 48.0 / 5.0 : 9.0) * p->E / (M_PI * t * std::pow(out->delta, 3));
        out->volume = dx * dx * t;
    } else {
        out->c_ref = 12.0 * p->E / (M_PI * std::pow(out->delta, 4));      // 3D
        out->volume = dx * dx * dx;
    }
    // The appendix-A fracture energy is G_F = (pi delta^5 / 5) A for a 3D
    // body and (t delta^4 / 2) A in plane stress (the 2D integral of
    // Eq. exp_fracture_energy_2D), with A the area under the bond
    // force-stretch curve between s0 and sc.
    // EXPLIN: A = c s0 (sc - s0) I / (1 + alpha) with I = int_0^1 of the
    // normalised shape = 1/k - 1/(e^k - 1) + alpha / 2.
    // TRILINEAR: A = 0.2 c s0 (sc - s0).
    // Either way sc = s0 + gamma / (c s0).
    const double geo = t > 0 ? 0.5 * t * std::pow(out->delta, 4) : M_PI * std::pow(out->delta, 5) / 5.0;
    if (p->law == PD_LAW_EXPLIN) {
        double I = 1.0 / p->k - 1.0 / std::expm1(p->k) + 0.5 * p->alpha;
        out->gamma = p->GF * (1.0 + p->alpha) / (geo * I);
    } else {
        out->gamma = p->GF / (geo * 0.2);
    }
    out->k = p->k;
    out->alpha = p->alpha;
    out->inv_one_minus_ek = 1.0 / (-std::expm1(-p->k));
    out->inv_one_plus_alpha = 1.0 / (1.0 + p->alpha);
    out->law = p->law;
    return PD_OK;
}

}  // namespace pdmi
