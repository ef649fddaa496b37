// Internal declarations shared by the host and device sources of libpdmi.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "pd.h"

namespace pdmi {

// ---------------------------------------------------------------- stencil
// The horizon delta = m dx with 3 <= m < sqrt(10) contains exactly the
// integer offsets v with 0 < |v|^2 <= 9: 122 neighbours, 61 of them
// "positive" (first non-zero of (v_z, v_y, v_x) positive).  Slot k < 61 is the
// k-th positive offset and slot 61 + k its negation, so a bond seen from its
// two ends occupies slots k and 61 + k.
constexpr int kHalfStencil = 61;
constexpr int kStencil = 122;
constexpr int kHalo = 3;

struct Off {
    int x, y, z;
};

struct HalfTable {
    Off v[kHalfStencil];
};

constexpr HalfTable make_half_table()
{
    HalfTable t{};
    int n = 0;
    for (int z = 0; z <= 3; ++z)
        for (int y = -3; y <= 3; ++y)
            for (int x = -3; x <= 3; ++x) {
                int r2 = x * x + y * y + z * z;
                bool positive = z > 0 || (z == 0 && (y > 0 || (y == 0 && x > 0)));
                if (r2 > 0 && r2 <= 9 && positive) t.v[n++] = Off{x, y, z};
            }
    return t;
}

constexpr HalfTable kHalf = make_half_table();

constexpr int half_count()
{
    int n = 0;
    for (int z = 0; z <= 3; ++z)
        for (int y = -3; y <= 3; ++y)
            for (int x = -3; x <= 3; ++x) {
                int r2 = x * x + y * y + z * z;
                bool positive = z > 0 || (z == 0 && (y > 0 || (y == 0 && x > 0)));
                if (r2 > 0 && r2 <= 9 && positive) ++n;
            }
    return n;
}
static_assert(half_count() == kHalfStencil, "stencil size");

inline Off slot_offset(int slot)
{
    Off o = kHalf.v[slot % kHalfStencil];
    if (slot >= kHalfStencil) o = Off{-o.x, -o.y, -o.z};
    return o;
}

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);

#define PD_HIP(call)                                                   \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return ::pdmi::hip_fail(e_, #call);       \
    } while (0)

// ---------------------------------------------------------------- device tables
struct NodeInfo {
    int32_t bc;       // -1 free, -2 load pad, >= 0: index into the support list
    int32_t cut;      // -1 no cut bond, else row of the cut-mask table
};

}  // namespace pdmi

struct pd_mesh_s {
    pd_mesh_desc d{};
    int nx = 0, ny = 0, nz = 0;
    int64_t M = 0;
    int PX = 0, PY = 0, PZ = 0;    // padded grid (kHalo ghost layers per face)
    int64_t P = 0;
    int notch_X = 0, notch_A = 0;  // notch plane and tip in half-cell units (A = 0: none)
    std::vector<int32_t> support, load;
    std::vector<pdmi::NodeInfo> info;

    bool bonds_built = false;
    int64_t n_bonds = 0, n_cut = 0;
    std::vector<uint32_t> cut_masks;  // 4 words per row, bit s set = slot s cut

    // device copies (valid once bonds are built)
    int device = -1;
    pdmi::NodeInfo *d_info = nullptr;
    uint4 *d_cut = nullptr;
    int32_t *d_support = nullptr;

    // per-node fields for the single-sample entry points, device FP64 [S][M]
    double *d_s0 = nullptr;
    int64_t s0_samples = 0;
    double *d_c = nullptr;
    int64_t c_samples = 0;
    double *d_gf = nullptr;
    int64_t gf_samples = 0;

    int shape_override = -1;   // pinned launch shape (PD_SHAPE_*), -1 = tuned
    double c_max = 0.0;        // largest value of the micromodulus field (0: none set)

    int64_t padded(int i, int j, int k) const
    {
        return (int64_t)(i + pdmi::kHalo) + (int64_t)PX * ((j + pdmi::kHalo) + (int64_t)PY * (k + pdmi::kHalo));
    }
};

// Karhunen-Loeve basis evaluated at a mesh's node centres.  Exponential-
// covariance bases also keep their Nystrom quadrature (reference node
// positions and w phi_k(x_j) / lambda_k) so they can be evaluated on other
// meshes.
struct pd_kl_s {
    const pd_mesh_s *mesh = nullptr;
    int n_modes = 0;
    int covariance = 0;            // PD_COV_*
    std::vector<double> lam;
    double *d_phi = nullptr;       // [n_modes][M]
    double *d_sqrt_lam = nullptr;  // [n_modes]
    double corr_len = 0.0;
    int64_t n_q = 0;               // exponential: quadrature points
    double *d_qpos = nullptr;      // [n_q][3]
    double *d_ext = nullptr;       // [n_modes][n_q]
};

namespace pdmi {

// geometry.cpp
int build_mesh(const pd_mesh_desc *d, pd_mesh_s *m);
int build_cuts(pd_mesh_s *m);
double stencil_inv_len_sum(bool in_plane);   // sum of 1/|v| over the 122 (in plane: 28) offsets
double stability_limit(const pd_mesh_s *m, double rho, double c);

// material constants of a run, derived once on the host in FP64
struct Material {
    double delta, c_ref, volume;
    double gamma;        // sc_b = s0_b + gamma / (c_b s0_b)
    double k, alpha, inv_one_minus_ek, inv_one_plus_alpha;
    int law;
};
int material_from_params(const pd_mesh_s *m, const pd_params *p, Material *out);

}  // namespace pdmi
