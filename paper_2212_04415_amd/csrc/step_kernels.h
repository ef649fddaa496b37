// Device code of one explicit time step of the bond-based peridynamic solve.
//
// A step evaluates, for every node of every sample, the bond forces over its
// 122-point horizon (28 in-plane points on a body one node thick, the
// plane-stress model of appendix A) (paper section 2.1, Eq. PD_Force_Function and
// Eq. PD_EOM_Dynamic; appendix A, Eq. exp_scalar_force and
// Eq. exp_damage_parameter), sums them with compensated accumulation, closes
// the damped velocity-Verlet step and opens the next one.  The first block of
// each sample also forms the FP64 reaction of the previous step and keeps the
// running peak (section 4: the quantity of interest is the peak load).
//
// Layout (per sample; all arrays sample-major):
//   u     : padded grid of (u_x, u_y, u_z, flag) in units of dx, ping-pong.
//           kHalo ghost layers per face hold flag 0; flag +1 marks a node
//           whose bonds have all stayed inside the plain fast path, -1 a node
//           that has had a damaged, near-limit or strongly compressed bond.
//           |flag| is the neighbour-existence weight.
//   vh    : half-step velocity (dx/s), three components per node (two, x
//           and z, in a plane body, whose y components stay zero); in FP32
//           also the compensation terms of vh and u (cvh, cu), likewise;
//   hist  : largest stretch of each bond direction, [122][M], touched only
//           for damaged bonds (0 until the bond passes its limit);
//   dmask : per node, one bit per bond direction that has passed its limit;
//   s0pad : padded per-node limit stretch (+inf on ghosts); thr: per-node
//           lower bound of the limit stretches of its bonds.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "pd_internal.h"

#ifndef PD_PIPE_DEPTH
#define PD_PIPE_DEPTH 4
#endif

namespace pdmi {

constexpr int kXcds = 8;

// Brick of nodes owned by one block (one thread per node, x fastest) and, on
// the LDS path, its tile with the kHalo-wide halo, rows padded by PADX cells.
// The global path uses the thread count only (a tile is N consecutive nodes).
// A 128-bit LDS read serves lanes 0-7 together with lanes 16-23 (and so on),
// i.e. two rows of a 16-wide brick; a row pitch of 8 (mod 16) cells puts
// those two rows on disjoint banks.
template <int BX_, int BY_, int BZ_, int PADX = 0>
struct Brick {
    static constexpr bool PLANE = false;
    static constexpr int BX = BX_, BY = BY_, BZ = BZ_;
    static constexpr int N = BX * BY * BZ;
    static constexpr int LX = BX + 2 * kHalo + PADX, LY = BY + 2 * kHalo, LZ = BZ + 2 * kHalo;
    static constexpr int LXY = LX * LY;
    static constexpr int TILE = LX * LY * LZ;
    static_assert(N % 64 == 0, "a brick is whole wavefronts");
};

// The same for a body one node thick (every node at y = 0; its neighbours
// all lie in the x-z plane): a BX x BZ patch whose tile has no y halo, and
// the fast loop visits the 14 in-plane offset pairs only.  Rows of 32 or
// more cells fill whole 128-bit LDS phases, so no row padding is needed.
template <int BX_, int BZ_>
struct PlaneBrick {
    static constexpr bool PLANE = true;
    static constexpr int BX = BX_, BY = 1, BZ = BZ_;
    static constexpr int N = BX * BZ;
    static constexpr int LX = BX + 2 * kHalo, LY = 1, LZ = BZ + 2 * kHalo;
    static constexpr int LXY = LX;
    static constexpr int TILE = LX * LZ;
    static_assert(N % 64 == 0, "a brick is whole wavefronts");
};

// sqrt(n) for the squared lengths that occur in the stencil
constexpr double kSqrtInt[10] = {0.0, 1.0, 1.4142135623730951, 1.7320508075688772, 2.0,
                                 2.23606797749979, 2.449489742783178, 2.6457513110645907,
                                 2.8284271247461903, 3.0};

template <typename T> struct Vec4;
template <> struct Vec4<float> { using t = float4; };
template <> struct Vec4<double> { using t = double4; };
template <typename T> struct Vec3;
template <> struct Vec3<float> { using t = float3; };
template <> struct Vec3<double> { using t = double3; };
template <typename T> struct Vec2;
template <> struct Vec2<float> { using t = float2; };
template <> struct Vec2<double> { using t = double2; };

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double quot(double a, double b) { return a / b; }
__device__ __forceinline__ float expx(float x) { return __expf(x); }
__device__ __forceinline__ double expx(double x) { return exp(x); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
struct StepParams {
    using V4 = typename Vec4<T>::t;
    const V4 *u_cur;
    V4 *u_next;
    typename Vec3<T>::t *vh;
    typename Vec3<T>::t *cu;    // FP32 only: compensation of u
    typename Vec3<T>::t *cvh;   // FP32 only: compensation of vh
    T *hist;            // [S][122][M]
    uint4 *dmask;       // [S][M] damaged-bond bits, one per slot
    const T *s0pad;     // [S][P]
    const T *thr;       // [S][M]
    const T *cpad;      // [S][P] c / c_ref, or null
    const T *gpad;      // [S][P] fracture energy / its homogeneous value, or one 1 (gstep 0)
    int gstep;          // 1 with a fracture-energy field, else 0
    const NodeInfo *info;
    const uint4 *cut;
    double *rf;         // [2][S][nsup] support-node force sums, by step parity
    int64_t rf_stride;  // S * nsup
    double *L_out;      // force-only mode: [S][M][3]
    const int64_t *step_base;  // [S] first step of the current replay chunk
    int k_local;               // step within the chunk (fixed per launch)
    int64_t n_steps;
    double *Q;                 // [S] running peak reaction
    int64_t *nstar;            // [S] step of the peak (1-based)
    int32_t *status;           // [S]
    double *hist_R;            // [S][n_steps] or null
    double Rscale;             // R = -Rscale * sum of support-node G_z
    int64_t P, M, PXY;
    int64_t tiles, n_items;    // tiles per sample, samples * tiles
    int nx, ny, nz, PX, PY, PZ, nsup;
    int nbx, nby;              // bricks along x and y (LDS path)
    int chunk;                 // LDS path: bricks per x slab of one sample (nby * nbz)
    int heavy_first;           // LDS path: mid-span x slabs of each sample first
    int force_only;
    int acc_mode;              // FP32 without compensation: the ablation run (PD_ACC_*)
    T two_d_b, two_d_g, dt, vload;  // integrator in units of dx
    double du_s;                    // load increment in units of dx
    T gamma_rel, k, alpha, inv1mek, inv1pa;
    int law;
    double LV;                      // c_ref V: force density per unit G
};

template <typename T, bool KAHAN>
struct Acc3 {
    T x, y, z, cx, cy, cz;
    __device__ __forceinline__ void zero() { x = y = z = cx = cy = cz = T(0); }
    __device__ __forceinline__ void add(T px, T py, T pz)
    {
        if constexpr (KAHAN) {
            kahan(x, cx, px);
            kahan(y, cy, py);
            kahan(z, cz, pz);
        } else {
            x += px;
            y += py;
            z += pz;
        }
    }
    __device__ __forceinline__ void add_xz(T px, T pz)
    {
        if constexpr (KAHAN) {
            kahan(x, cx, px);
            kahan(z, cz, pz);
        } else {
            x += px;
            z += pz;
        }
    }
    __device__ __forceinline__ void add_if(bool on, T px, T py, T pz)
    {
        if constexpr (KAHAN) {
            T x1 = x, cx1 = cx, y1 = y, cy1 = cy, z1 = z, cz1 = cz;
            kahan(x1, cx1, px);
            kahan(y1, cy1, py);
            kahan(z1, cz1, pz);
            x = on ? x1 : x; cx = on ? cx1 : cx;
            y = on ? y1 : y; cy = on ? cy1 : cy;
            z = on ? z1 : z; cz = on ? cz1 : cz;
        } else {
            x = on ? x + px : x;
            y = on ? y + py : y;
            z = on ? z + pz : z;
        }
    }
    __device__ __forceinline__ static void kahan(T &s, T &c, T v)
    {
        T yv = v - c;
        T t = s + yv;
        c = (t - s) - yv;
        s = t;
    }
    __device__ __forceinline__ T gx() const { return KAHAN ? x - cx : x; }
    __device__ __forceinline__ T gy() const { return KAHAN ? y - cy : y; }
    __device__ __forceinline__ T gz() const { return KAHAN ? z - cz : z; }
};

// ---------------------------------------------------------------- stretch
// For a bond with lattice offset v (units of dx) and e = u_j - u_i,
// |v + e|^2 = |v|^2 + num with num = 2 v.e + e.e = sum_c e_c (2 v_c + e_c), and
// the stretch (|xi + eta| - |xi|)/|xi| equals num / (|v| (|v + e| + |v|)),
// which has no cancellation.  The operation sequence is spelled out (the
// library is built without floating-point contraction) so that the two ends
// of a bond, and the compile-time and run-time offset paths, produce
// bit-identical results: 2 v_c + e_c is exact up to its rounding, which is
// symmetric under (v, e) -> (-v, -e), and terms with v_c = 0 reduce to
// e_c * e_c on both paths.
template <int C, int SIGN, typename T>
__device__ __forceinline__ T term_c(T e)
{
    if constexpr (C == 0) return e;
    else return T(2 * SIGN * C) + e;
}

// PLANE: a body one node thick, whose y displacements are identically zero
// and whose bonds all lie in the x-z plane (VY = 0), so the y term of num is
// exactly zero and is left out.
template <typename T, int VX, int VY, int VZ, int SIGN, bool PLANE = false>
__device__ __forceinline__ T num_c(const typename Vec4<T>::t &ui, const typename Vec4<T>::t &uj, T &ex, T &ey,
                                   T &ez)
{
    static_assert(!PLANE || VY == 0, "in-plane offsets only");
    // (the statement order of the 3D form is kept as it is: it decides the
    // register allocation of the unrolled loop)
    ex = uj.x - ui.x;
    if constexpr (PLANE) ey = T(0);
    else ey = uj.y - ui.y;
    ez = uj.z - ui.z;
    T n = ex * term_c<VX, SIGN>(ex);
    if constexpr (!PLANE) n = fma_(ey, term_c<VY, SIGN>(ey), n);
    return fma_(ez, term_c<VZ, SIGN>(ez), n);
}

template <typename T>
__device__ __forceinline__ T num_rt(const typename Vec4<T>::t &ui, const typename Vec4<T>::t &uj, int vx, int vy,
                                    int vz, T &ex, T &ey, T &ez)
{
    ex = uj.x - ui.x;
    ey = uj.y - ui.y;
    ez = uj.z - ui.z;
    T n = ex * (vx == 0 ? ex : T(2 * vx) + ex);
    n = fma_(ey, vy == 0 ? ey : T(2 * vy) + ey, n);
    return fma_(ez, vz == 0 ? ez : T(2 * vz) + ez, n);
}

// closed-form stretch and 1/|v + e| from num
template <typename T>
__device__ __forceinline__ T stretch_from_num(T num, T V2, T VL, T &ry)
{
    T y2 = V2 + num;
    ry = rsq(y2);
    T den = fma_(VL, y2 * ry, V2);
    return quot(num, den);
}

// 1 - d for the largest stretch kap of a bond with limit s0 and critical sc
// (appendix A, Eq. exp_damage_parameter; piecewise-linear envelope otherwise)
template <typename T>
__device__ __forceinline__ T keep_fraction(const StepParams<T> &a, T kap, T s0, T sc)
{
    if (kap >= sc) return T(0);
    T t = quot(kap - s0, sc - s0);
    if (a.law == PD_LAW_EXPLIN) {
        T br = T(1) - (T(1) - expx(-a.k * t)) * a.inv1mek + a.alpha * (T(1) - t);
        return quot(s0, kap) * br * a.inv1pa;
    }
    // envelope c s0 at s0, 0.2 c s0 at s1 = s0 + 0.2 (sc - s0), 0 at sc
    T f = (t <= T(0.2)) ? s0 * (T(1) - T(4) * t) : s0 * (T(0.25) * (T(1) - t));
    return quot(f, kap);
}

// ---------------------------------------------------------------- neighbour sources
// element of a per-sample array at (lane base + uniform offset), addressed as a
// scalar base plus a 32-bit per-lane byte offset
template <typename E>
__device__ __forceinline__ E ld(const E *base, int64_t off, uint32_t lane_bytes)
{
    return *(const E *)((const char *)(base + off) + lane_bytes);
}

// displacement (get) and micromodulus ratio (getc) of the neighbour at
// lattice offset v, from the padded grids
template <typename T>
struct GlobalSrc {
    using V4 = typename Vec4<T>::t;
    static constexpr bool kLds = false;
    const V4 *U;
    uint32_t lb;
    int64_t PX, PXY;
    const T *Cp;          // padded c / c_ref of the sample, or null
    uint32_t lbc;
    template <int X, int Y, int Z> __device__ __forceinline__ V4 get() const
    {
        return ld(U, (int64_t)X + (int64_t)Y * PX + (int64_t)Z * PXY, lb);
    }
    __device__ __forceinline__ V4 get(int x, int y, int z) const
    {
        return ld(U, (int64_t)x + (int64_t)y * PX + (int64_t)z * PXY, lb);
    }
    template <int X, int Y, int Z> __device__ __forceinline__ T getc() const
    {
        return ld(Cp, (int64_t)X + (int64_t)Y * PX + (int64_t)Z * PXY, lbc);
    }
    __device__ __forceinline__ T getc(int x, int y, int z) const
    {
        return ld(Cp, (int64_t)x + (int64_t)y * PX + (int64_t)z * PXY, lbc);
    }
    // the node's position key, and the source seen from another node's key
    __device__ __forceinline__ uint32_t key() const { return lb; }
    __device__ __forceinline__ GlobalSrc rebased(uint32_t k) const
    {
        GlobalSrc r = *this;
        r.lb = k;
        r.lbc = k / (uint32_t)(sizeof(V4) / sizeof(T));
        return r;
    }
};

// ... from the block's LDS tiles (brick plus halo)
template <typename T, typename BR>
struct LdsSrc {
    using V4 = typename Vec4<T>::t;
    static constexpr bool kLds = true;
    const V4 *tile;
    const T *ctile;       // c / c_ref tile, or a dummy without a c field
    int c;
    template <int X, int Y, int Z> __device__ __forceinline__ V4 get() const
    {
        return tile[c + X + BR::LX * Y + BR::LXY * Z];
    }
    __device__ __forceinline__ V4 get(int x, int y, int z) const { return tile[c + x + BR::LX * y + BR::LXY * z]; }
    template <int X, int Y, int Z> __device__ __forceinline__ T getc() const
    {
        return ctile[c + X + BR::LX * Y + BR::LXY * Z];
    }
    __device__ __forceinline__ T getc(int x, int y, int z) const { return ctile[c + x + BR::LX * y + BR::LXY * z]; }
    __device__ __forceinline__ uint32_t key() const { return (uint32_t)c; }
    __device__ __forceinline__ LdsSrc rebased(uint32_t k) const
    {
        LdsSrc r = *this;
        r.c = (int)k;
        return r;
    }
};

// ---------------------------------------------------------------- pipelining
// The 61 offset pairs are unrolled with compile-time offsets.  Loads of pair
// K + D are issued before the arithmetic of pair K, and a scheduling fence
// every second pair keeps the compiler from hoisting all 122 neighbour loads
// (which would exhaust the register file) while letting it interleave the
// arithmetic of two neighbouring pairs (2% faster than a fence per pair).
template <int K, int N, int D, typename R, typename LoadF, typename CompF>
__device__ __forceinline__ void pipe_step(R (&ring)[D], LoadF &load, CompF &comp)
{
    if constexpr (K < N) {
        if constexpr (K % 2 == 0) __builtin_amdgcn_sched_barrier(0);
        R cur = ring[K % D];
        if constexpr (K + D < N) ring[K % D] = load(std::integral_constant<int, K + D>{});
        comp(std::integral_constant<int, K>{}, cur);
        pipe_step<K + 1, N, D>(ring, load, comp);
    }
}

template <int N, int D, typename R, typename LoadF, typename CompF, int... I>
__device__ __forceinline__ void pipeline(LoadF &load, CompF &comp, std::integer_sequence<int, I...>)
{
    R ring[D];
    ((ring[I] = load(std::integral_constant<int, I>{})), ...);
    pipe_step<0, N, D>(ring, load, comp);
}

// Order in which the fast loop visits the 61 offset pairs (the 14 with
// v_y = 0 on a plane body): by |v|^2, then by slot, so that bonds of one
// length are contiguous (their series coefficients and scaled thresholds are
// shared).  Slots keep their 3D numbering either way.
struct PairOrder {
    int k[kHalfStencil];
    int n;
};

constexpr int half_len2(int k) { return kHalf.v[k].x * kHalf.v[k].x + kHalf.v[k].y * kHalf.v[k].y + kHalf.v[k].z * kHalf.v[k].z; }

constexpr PairOrder make_pair_order(bool plane)
{
    PairOrder o{};
    o.n = 0;
    for (int l = 1; l <= 9; ++l)
        for (int k = 0; k < kHalfStencil; ++k)
            if (half_len2(k) == l && (!plane || kHalf.v[k].y == 0)) o.k[o.n++] = k;
    return o;
}

constexpr PairOrder kPairOrder = make_pair_order(false);
constexpr PairOrder kPairOrderPlane = make_pair_order(true);
static_assert(kPairOrder.n == kHalfStencil && kPairOrderPlane.n == 14, "stencil pair counts");

template <bool PLANE> struct Pairs {
    static constexpr const PairOrder &order = kPairOrder;
};
template <> struct Pairs<true> {
    static constexpr const PairOrder &order = kPairOrderPlane;
};

template <typename T> struct FastLoad {
    typename Vec4<T>::t a, b;
    T ca, cb;
};

// ---------------------------------------------------------------- fast path
// Every bond of the node is evaluated with compile-time offsets.
//
// Plain form (MASKED = false): all bonds of the node are known to be below
// their limit stretch (d = 0); flag is raised when a bond may have reached the
// node's lower bound of limit stretches (or leaves the series range), and the
// node is then redone in masked form.
//
// Masked form: bonds listed in `skip` (notch-cut or damaged) and bonds that
// reach the threshold or leave the series range contribute nothing here and
// are returned in `exc` (a superset of `skip`) for the exception pass.
//
// The two forms evaluate an in-range bond identically and flag exactly the
// bonds the other would except, so a node's result does not depend on which
// form its wavefront takes (nor, therefore, on the brick shape of the launch).
//
// In FP32 the stretch and the force weight w = s / |v + e| of an undamaged
// bond are evaluated without square root or division: with x = num / (2|v|^2),
// |v + e| = |v| sqrt(1 + 2x), so
//   s = sqrt(1 + 2x) - 1 <= x,
//   w = (1 - (1 + 2x)^(-1/2)) / |v| = (x / |v|)(1 - 3/2 x + 5/2 x^2 - 35/8 x^3 ...).
// Three terms are kept for |x| < 2^-10 (larger tensions are caught through
// s <= x by the threshold, which is clamped to 2^-10, larger compressions
// explicitly): relative error below 35/8 * 2^-30 = 4.1e-9, under FP32
// rounding (2^-24 = 6e-8).  FP64 and the exception pass use the closed form.
constexpr double kSeriesBound = 1.0 / 1024;

template <typename T, bool KAHAN, bool HAS_C, bool MASKED, bool PLANE, typename Src>
__device__ __forceinline__ void fast_loop(const StepParams<T> &a, const Src &src,
                                          const typename Vec4<T>::t &ui, T ci, T thr,
                                          Acc3<T, KAHAN> &acc, bool &flag, const uint32_t (&skip)[4],
                                          uint32_t (&exc)[4])
{
    using PO = Pairs<PLANE>;
    constexpr int NP = PO::order.n;
    // a 3D body keeps a node's c / c_ref in its flag word (a plane body, with
    // its small c tile, keeps the tile: its registers are the tighter limit)
    constexpr bool CW = HAS_C && !PLANE;
    auto load = [&](auto ic) {
        constexpr Off v = kHalf.v[PO::order.k[decltype(ic)::value]];
        FastLoad<T> r;
        r.a = src.template get<v.x, v.y, v.z>();
        r.b = src.template get<-v.x, -v.y, -v.z>();
        if constexpr (CW) {
            r.ca = fabs(r.a.w);
            r.cb = fabs(r.b.w);
        } else if constexpr (HAS_C) {
            r.ca = src.template getc<v.x, v.y, v.z>();
            r.cb = src.template getc<-v.x, -v.y, -v.z>();
        } else {
            r.ca = r.cb = T(1);
        }
        return r;
    };
    // Largest weighted series variable (FP32: num |w|, per bond length) or
    // stretch (FP64), and largest magnitude, for the plain form's flag.
    T hi = T(-1), ha = T(0);
    bool fl = false;
    T pend_x = T(0), pend_y = T(0), pend_z = T(0);   // partial sum of the current group of pairs
    auto comp_pair = [&](auto ic, const FastLoad<T> &r) {
        constexpr int I = decltype(ic)::value;
        constexpr int K = PO::order.k[I];
        constexpr Off v = kHalf.v[K];
        constexpr int V2 = v.x * v.x + v.y * v.y + v.z * v.z;
        T eax, eay, eaz, ebx, eby, ebz, wa, wb;
        const T na = num_c<T, v.x, v.y, v.z, 1, PLANE>(ui, r.a, eax, eay, eaz);
        const T nb = num_c<T, v.x, v.y, v.z, -1, PLANE>(ui, r.b, ebx, eby, ebz);
        bool exa = false, exb = false;
        if constexpr (sizeof(T) == 4) {
            // x = h num with h = 1/(2|v|^2), and w = (x/|v|)(1 - 3/2 x + 5/2 x^2)
            // = num (C1 + num (C2 + num C3)); tests on x compare num |w|
            // against the bound times 2|v|^2.
            constexpr double h = 0.5 / V2, L = kSqrtInt[V2];
            constexpr T C1 = T(h / L), C2 = T(-1.5 * h * h / L), C3 = T(2.5 * h * h * h / L);
            constexpr T S2 = T(2 * V2);
            // ghost neighbours (flag word 0) contribute nothing
            const T nwa = CW ? (r.a.w != T(0) ? na : T(0)) : na * fabs(r.a.w);
            const T nwb = CW ? (r.b.w != T(0) ? nb : T(0)) : nb * fabs(r.b.w);
            wa = nwa * fma_(na, fma_(na, C3, C2), C1);
            wb = nwb * fma_(nb, fma_(nb, C3, C2), C1);
            if constexpr (MASKED) {
                const T ts = thr * S2;
                exa = (nwa > ts) || (nwa < T(-kSeriesBound) * S2);
                exb = (nwb > ts) || (nwb < T(-kSeriesBound) * S2);
            } else {
                constexpr bool gfirst = I == 0 || half_len2(PO::order.k[I > 0 ? I - 1 : 0]) != V2;
                constexpr bool glast = I + 1 == NP || half_len2(PO::order.k[I + 1 < NP ? I + 1 : I]) != V2;
                if constexpr (gfirst) {
                    hi = fmax(nwa, nwb);
                    ha = fmax(fabs(nwa), fabs(nwb));
                } else {
                    hi = fmax(fmax(hi, nwa), nwb);
                    ha = fmax(fmax(ha, fabs(nwa)), fabs(nwb));
                }
                if constexpr (glast) fl = fl | (hi > thr * S2) | (ha > T(kSeriesBound) * S2);
            }
        } else {
            T rya, ryb;
            const T sa0 = stretch_from_num(na, T(V2), T(kSqrtInt[V2]), rya);
            const T sb0 = stretch_from_num(nb, T(V2), T(kSqrtInt[V2]), ryb);
            const T sa = CW ? (r.a.w != T(0) ? sa0 : T(0)) : sa0 * fabs(r.a.w);
            const T sb = CW ? (r.b.w != T(0) ? sb0 : T(0)) : sb0 * fabs(r.b.w);
            if constexpr (MASKED) {
                exa = sa > thr;
                exb = sb > thr;
            } else {
                hi = fmax(fmax(hi, sa), sb);
            }
            wa = sa * rya;
            wb = sb * ryb;
        }
        if constexpr (MASKED) {
            // slot K is the +v direction, slot K + 61 the -v direction
            constexpr int KB = K + kHalfStencil;
            constexpr uint32_t BA = 1u << (K % 32), BB = 1u << (KB % 32);
            exa = exa || (skip[K / 32] & BA) != 0u;
            exb = exb || (skip[KB / 32] & BB) != 0u;
            wa = exa ? T(0) : wa;
            wb = exb ? T(0) : wb;
            exc[K / 32] |= exa ? BA : 0u;
            exc[KB / 32] |= exb ? BB : 0u;
        }
        if constexpr (HAS_C) {
            wa = wa * (T(0.5) * (ci + r.ca));
            wb = wb * (T(0.5) * (ci + r.cb));
        }
        // wa (v + ea) + wb (-v + eb) = (wa - wb) v + wa ea + wb eb: the large
        // symmetric parts cancel exactly before they are scaled.  Pair sums
        // are chained into the group's partial sum, and each group of eight
        // pairs (sixteen bonds) enters the compensated accumulator once; the
        // 14-pair plane loop keeps groups of four, whose shorter chains it
        // needs to hide their latency.
        constexpr int G = PLANE ? 4 : 8;
        constexpr bool first = (I % G == 0);
        const T dw = wa - wb;
        auto part = [&](auto cc, T ea, T eb, T pend) {
            constexpr int C = decltype(cc)::value;
            const T base = first ? wb * eb : fma_(wb, eb, pend);
            if constexpr (C == 0) return fma_(wa, ea, base);
            else return fma_(wa, ea, fma_(dw, T(C), base));
        };
        pend_x = part(std::integral_constant<int, v.x>{}, eax, ebx, pend_x);
        if constexpr (!PLANE) pend_y = part(std::integral_constant<int, v.y>{}, eay, eby, pend_y);
        pend_z = part(std::integral_constant<int, v.z>{}, eaz, ebz, pend_z);
        if constexpr (I % G == G - 1 || I + 1 == NP) {
            // a plane body has no y force (its y sums would stay exactly zero)
            if constexpr (PLANE) acc.add_xz(pend_x, pend_z);
            else acc.add(pend_x, pend_y, pend_z);
        }
    };
    // neighbours read through the caches hold more registers in flight
    constexpr int D = (sizeof(T) == 4 && Src::kLds) ? PD_PIPE_DEPTH : 2;
    pipeline<NP, D, FastLoad<T>>(load, comp_pair, std::make_integer_sequence<int, D>{});
    if constexpr (MASKED) flag = false;
    // thr <= 2^-10, so this flags exactly the bonds the masked form excepts
    else if constexpr (sizeof(T) == 4) flag = fl;
    else flag = hi > thr;
}

// ---------------------------------------------------------------- exception pass
// Slot k of the stencil: k < 61 is +kHalf[k], k >= 61 is -kHalf[k - 61].
// Packed as (x + 3) | (y + 3) << 4 | (z + 3) << 8 | |v|^2 << 12; a block
// copies the table (and sqrt of the squared lengths) into LDS so that lanes
// can index it with their own slot.
constexpr uint32_t pack_slot(int k)
{
    const Off o = kHalf.v[k % kHalfStencil];
    const int sg = k < kHalfStencil ? 1 : -1;
    return (uint32_t)(sg * o.x + 3) | (uint32_t)(sg * o.y + 3) << 4 | (uint32_t)(sg * o.z + 3) << 8 |
           (uint32_t)(o.x * o.x + o.y * o.y + o.z * o.z) << 12;
}

struct SlotPack {
    uint32_t e[kStencil];
};

constexpr SlotPack make_slot_pack()
{
    SlotPack t{};
    for (int k = 0; k < kStencil; ++k) t.e[k] = pack_slot(k);
    return t;
}

static __constant__ SlotPack c_slot_pack = make_slot_pack();

// the same table unpacked, for loops where every lane takes the same slot
struct SlotEntry {
    int x, y, z, len2;
};

struct SlotTable {
    SlotEntry e[kStencil];
};

constexpr SlotTable make_slot_table()
{
    SlotTable t{};
    for (int k = 0; k < kStencil; ++k) {
        const uint32_t p = pack_slot(k);
        t.e[k] = SlotEntry{(int)(p & 15u) - 3, (int)((p >> 4) & 15u) - 3, (int)((p >> 8) & 15u) - 3, (int)(p >> 12)};
    }
    return t;
}

static __constant__ SlotTable c_slots = make_slot_table();
static __constant__ double c_sqrt_int[10] = {0.0, 1.0, 1.4142135623730951, 1.7320508075688772, 2.0,
                                             2.23606797749979, 2.449489742783178, 2.6457513110645907,
                                             2.8284271247461903, 3.0};

template <typename T>
struct SlotLds {
    uint32_t slot[kStencil];
    T len[10];
};

template <typename T>
__device__ __forceinline__ void fill_slot_lds(SlotLds<T> &t)
{
    if (threadIdx.x < kStencil) t.slot[threadIdx.x] = c_slot_pack.e[threadIdx.x];
    if (threadIdx.x < 10) t.len[threadIdx.x] = (T)c_sqrt_int[threadIdx.x];
}

// Cross-lane helpers of the pooled exception pass (wave64; every lane of the
// wave takes part).
__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ uint32_t shfl_u32(uint32_t v, uint32_t src)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)v);
}
__device__ __forceinline__ float shfl_t(float v, uint32_t src)
{
    return __builtin_bit_cast(float, shfl_u32(__builtin_bit_cast(uint32_t, v), src));
}
__device__ __forceinline__ double shfl_t(double v, uint32_t src)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = shfl_u32((uint32_t)b, src), hi = shfl_u32((uint32_t)(b >> 32), src);
    return __builtin_bit_cast(double, lo | (hi << 32));
}

// Bit k of a 128-bit mask held in four registers.  The helpers below are
// written as selects on values (range tests, no chains of equality tests,
// which the compiler turns into switches and then into branches): they run
// once per round of the exception pass on diverged lanes, where every branch
// costs exec-mask updates on the scalar unit.
__device__ __forceinline__ bool mask_bit(const uint32_t (&m)[4], int k)
{
    const uint32_t lo = k < 32 ? m[0] : m[1], hi = k < 96 ? m[2] : m[3];
    return ((k < 64 ? lo : hi) >> (k & 31)) & 1u;
}
// Sets bit k when on is true.
__device__ __forceinline__ void set_mask_bit(uint32_t (&m)[4], int k, bool on = true)
{
    const uint32_t b = on ? 1u << (k & 31) : 0u;
    m[0] |= k < 32 ? b : 0u;
    m[1] |= (k >= 32 && k < 64) ? b : 0u;
    m[2] |= (k >= 64 && k < 96) ? b : 0u;
    m[3] |= k >= 96 ? b : 0u;
}

// The lowest set bit of the 128-bit mask m (word order 0..3): its slot, or -1
// when m is empty.  Stored back into m with that bit cleared only when take
// is true, so lanes that sit a round out keep their mask.
__device__ __forceinline__ int pop_slot(uint32_t (&m)[4], bool take = true)
{
    const uint32_t m0 = m[0], m1 = m[1], m2 = m[2], m3 = m[3];
    const bool z0 = m0 == 0u, z01 = z0 && m1 == 0u, z012 = z01 && m2 == 0u;
    const uint32_t w = z0 ? (z01 ? (z012 ? m3 : m2) : m1) : m0;
    const int base = z0 ? (z01 ? (z012 ? 96 : 64) : 32) : 0;
    // clearing the lowest bit of an empty word leaves it empty, so each word
    // may take it unless an earlier word holds the bit
    m[0] = take ? m0 & (m0 - 1u) : m0;
    m[1] = take && z0 ? m1 & (m1 - 1u) : m1;
    m[2] = take && z01 ? m2 & (m2 - 1u) : m2;
    m[3] = take && z012 ? m3 & (m3 - 1u) : m3;
    return w != 0u ? base + __builtin_ctz(w) : -1;
}

// One exceptional bond (k) of the node whose values are given: closed-form
// stretch, damage history and damage law.  A bond's largest stretch is kept in
// hist once it passes the bond's limit stretch (never decreasing, so damage
// never heals); `was` says the bond had passed it before (its bit in the
// node's damage mask), and now is set when it passes it for the first time or
// its history grows.  The pass is bound by the latency of these reads, so they
// are split from the arithmetic: exc_fetch issues every read of a bond (ghost
// cells of the padded fields are valid addresses) and exc_finish uses them,
// letting a lane keep the reads of two bonds in flight.
template <typename T>
struct ExcFetch {
    typename Vec4<T>::t uj;
    T s0j, gj, cj, kap;
    int x, y, z, len2;
};

template <typename T, bool HAS_C, bool CW, typename Src>
__device__ __forceinline__ ExcFetch<T> exc_fetch(const StepParams<T> &a, const Src &src, const SlotLds<T> &tab,
                                                 const T *__restrict__ S0, const T *__restrict__ Hs,
                                                 const T *__restrict__ Gp, int gstep, uint32_t lb1, uint32_t lbh,
                                                 int k, bool was)
{
    ExcFetch<T> f;
    const uint32_t e = tab.slot[k];
    f.x = (int)(e & 15u) - 3;
    f.y = (int)((e >> 4) & 15u) - 3;
    f.z = (int)((e >> 8) & 15u) - 3;
    f.len2 = (int)(e >> 12);
    const int64_t off = (int64_t)f.x + (int64_t)f.y * a.PX + (int64_t)f.z * a.PXY;
    f.uj = src.get(f.x, f.y, f.z);
    f.s0j = ld(S0, off, lb1);
    f.gj = T(1);   // without a fracture-energy field its one word holds 1
    if (gstep != 0) f.gj = ld(Gp, off * gstep, lb1 * (uint32_t)gstep);
    f.cj = T(1);
    if constexpr (CW) f.cj = fabs(f.uj.w);
    else if constexpr (HAS_C) f.cj = src.getc(f.x, f.y, f.z);
    const T *H = (const T *)((const char *)(Hs + (int64_t)k * a.M) + lbh);
    f.kap = was ? *H : T(0);
    return f;
}

// Returns false for a ghost neighbour, which contributes nothing.
template <typename T, bool HAS_C>
__device__ __forceinline__ bool exc_finish(const StepParams<T> &a, const SlotLds<T> &tab, T *__restrict__ Hs,
                                           uint32_t lbh, const typename Vec4<T>::t &ui, T s0i, T ci, T gi, int k,
                                           const ExcFetch<T> &f, bool &now, T &fx, T &fy, T &fz)
{
    now = false;
    if (f.uj.w == T(0)) return false;
    T ex, ey, ez, ry;
    const T num = num_rt<T>(ui, f.uj, f.x, f.y, f.z, ex, ey, ez);
    const T s = stretch_from_num(num, T(f.len2), tab.len[f.len2], ry);
    const T s0b = T(0.5) * (s0i + f.s0j);
    T kap = f.kap;
    if (s > kap && s > s0b) {
        kap = s;
        *(T *)((char *)(Hs + (int64_t)k * a.M) + lbh) = s;
        now = true;
    }
    T cb = T(1);
    if constexpr (HAS_C) cb = T(0.5) * (ci + f.cj);
    T keep = T(1);
    if (kap > s0b) {
        // bond fracture energy: endpoint mean, as for s0 and c
        const T gb = T(0.5) * (gi + f.gj);
        const T sc = s0b + quot(a.gamma_rel * gb, cb * s0b);
        keep = keep_fraction(a, kap, s0b, sc);
    }
    const T w = keep * s * ry * cb;
    fx = w * (T(f.x) + ex);
    fy = w * (T(f.y) + ey);
    fz = w * (T(f.z) + ez);
    return true;
}

// The bonds the masked fast loop left out (todo = its exceptions minus the
// notch-cut bonds), for every node of the wavefront at once.  Nodes near a
// crack own many such bonds and their neighbours few; a walk of each lane
// over its own bonds would take as many rounds as the busiest lane, with most
// lanes idle.  Instead, round r takes the r-th bond (in slot order) of every
// node that has more than r, consecutive rounds are packed into a list of up
// to 128 bonds, and the list is evaluated two bonds per lane (their reads in
// flight together) with the owning node's values fetched across lanes.  Each
// owner then adds its results round by round, i.e. in slot order, so a
// node's force is bit-identical to a walk over its own bonds.  Called by
// every lane of the wave (lanes without a node pass todo = 0); list is this
// wave's 128-entry slice of block-shared memory.
template <typename T, bool KAHAN, bool HAS_C, bool CW, typename Src>
__device__ __forceinline__ void exc_pool(const StepParams<T> &a, const Src &src, const SlotLds<T> &tab,
                                         const T *__restrict__ S0, T *__restrict__ Hs, const T *__restrict__ Gp,
                                         int gstep, uint32_t p, uint32_t node, const typename Vec4<T>::t &ui,
                                         T s0i, T ci, T gi, const uint32_t (&todo)[4], uint32_t (&dm)[4],
                                         Acc3<T, KAHAN> &acc, uint16_t *list)
{
    using V4 = typename Vec4<T>::t;
    constexpr uint32_t kList = 128;
    const uint32_t lane = lane_id();
    const uint64_t below = (1ull << lane) - 1ull;
    const uint32_t cnt = __builtin_popcount(todo[0]) + __builtin_popcount(todo[1]) + __builtin_popcount(todo[2]) +
                         __builtin_popcount(todo[3]);
    uint32_t rem[4] = {todo[0], todo[1], todo[2], todo[3]};
    const uint32_t key = src.key();
    uint32_t r = 0;
    while (__any(cnt > r)) {
        // list rounds r0 .. r - 1 (at least one: a round has at most 64 bonds)
        const uint32_t r0 = r;
        uint32_t fill = 0;
        for (;;) {
            const uint64_t m = __ballot(cnt > r);
            const uint32_t n = (uint32_t)__popcll(m);
            if (n == 0 || fill + n > kList) break;
            const bool in = cnt > r;
            const int k = pop_slot(rem, in);
            const uint32_t at = fill + (uint32_t)__popcll(m & below);
            const uint32_t entry = lane << 8 | (mask_bit(dm, k) ? 128u : 0u) | (uint32_t)k;
            if (in) list[at] = (uint16_t)entry;
            fill += n;
            ++r;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // listed bonds lane and lane + 64
        const bool has0 = lane < fill, has1 = lane + 64u < fill;
        const uint32_t ent0 = has0 ? list[lane] : (lane << 8), ent1 = has1 ? list[lane + 64u] : (lane << 8);
        const uint32_t o0 = ent0 >> 8, o1 = ent1 >> 8;
        V4 u0, u1;
        u0.x = shfl_t(ui.x, o0);
        u0.y = shfl_t(ui.y, o0);
        u0.z = shfl_t(ui.z, o0);
        u0.w = T(1);
        u1.x = shfl_t(ui.x, o1);
        u1.y = shfl_t(ui.y, o1);
        u1.z = shfl_t(ui.z, o1);
        u1.w = T(1);
        const T s00 = shfl_t(s0i, o0), s01 = shfl_t(s0i, o1);
        const T c00 = HAS_C ? shfl_t(ci, o0) : T(1), c01 = HAS_C ? shfl_t(ci, o1) : T(1);
        T g00 = T(1), g01 = T(1);   // gi is 1 on every lane without a fracture-energy field
        if (gstep != 0) {
            g00 = shfl_t(gi, o0);
            g01 = shfl_t(gi, o1);
        }
        const uint32_t p0 = shfl_u32(p, o0), p1 = shfl_u32(p, o1);
        const uint32_t n0 = shfl_u32(node, o0), n1 = shfl_u32(node, o1);
        const uint32_t k0 = shfl_u32(key, o0), k1 = shfl_u32(key, o1);
        const uint32_t lh0 = n0 * (uint32_t)sizeof(T), lh1 = n1 * (uint32_t)sizeof(T);
        ExcFetch<T> f0, f1;
        if (has0)
            f0 = exc_fetch<T, HAS_C, CW>(a, src.rebased(k0), tab, S0, Hs, Gp, gstep, p0 * (uint32_t)sizeof(T), lh0,
                                     (int)(ent0 & 127u), (ent0 & 128u) != 0u);
        if (has1)
            f1 = exc_fetch<T, HAS_C, CW>(a, src.rebased(k1), tab, S0, Hs, Gp, gstep, p1 * (uint32_t)sizeof(T), lh1,
                                     (int)(ent1 & 127u), (ent1 & 128u) != 0u);
        T fx0 = T(0), fy0 = T(0), fz0 = T(0), fx1 = T(0), fy1 = T(0), fz1 = T(0);
        bool now0 = false, live0 = false, now1 = false, live1 = false;
        if (has0)
            live0 = exc_finish<T, HAS_C>(a, tab, Hs, lh0, u0, s00, c00, g00, (int)(ent0 & 127u), f0, now0, fx0, fy0,
                                         fz0);
        if (has1)
            live1 = exc_finish<T, HAS_C>(a, tab, Hs, lh1, u1, s01, c01, g01, (int)(ent1 & 127u), f1, now1, fx1, fy1,
                                         fz1);
        // per listed bond: live, first damage (its bit joins the node's
        // damage mask; a bond already in the mask only grows its history) and
        // its slot (9 bits; the second bond's from bit 16)
        const bool new0 = now0 && (ent0 & 128u) == 0u, new1 = now1 && (ent1 & 128u) == 0u;
        const uint32_t flags = (live0 ? 1u : 0u) | (new0 ? 2u : 0u) | (ent0 & 127u) << 2 |
                               ((live1 ? 1u : 0u) | (new1 ? 2u : 0u) | (ent1 & 127u) << 2) << 16;
        // owners add their results round by round
        uint32_t base = 0;
        for (uint32_t rr = r0; rr < r; ++rr) {
            const uint64_t m = __ballot(cnt > rr);
            const uint32_t n = (uint32_t)__popcll(m);
            const bool mi = cnt > rr;
            const uint32_t idx = mi ? base + (uint32_t)__popcll(m & below) : lane;
            // the round's results sit at list positions base .. base + n - 1
            // (n <= 64), so of the two a lane holds at most one is wanted:
            // entry lane + 64 when it lies in that range, else entry lane
            const bool up = lane + 64u >= base && lane + 64u < base + n;
            const T sx = up ? fx1 : fx0, sy = up ? fy1 : fy0, sz = up ? fz1 : fz0;
            const uint32_t srcl = idx & 63u;
            const T ax = shfl_t(sx, srcl), ay = shfl_t(sy, srcl), az = shfl_t(sz, srcl);
            const uint32_t fl = shfl_u32(up ? flags >> 16 : flags, srcl);
            if (mi && (fl & 2u)) set_mask_bit(dm, (int)((fl >> 2) & 127u), true);   // rare: a branch
            acc.add_if(mi && (fl & 1u), ax, ay, az);
            base += n;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------- integrator
template <typename T, bool KAHAN>
__device__ __forceinline__ void kick_drift(const StepParams<T> &a, T G, T &vh, T &cvh, T &u, T &cu)
{
    // vh^{n+1} = vh^n + 2D (b G - g vh^n);  u^{n+2} = u^{n+1} + dt vh^{n+1}
    T dv = fma_(a.two_d_b, G, -(a.two_d_g * vh));
    if constexpr (KAHAN) {
        Acc3<T, true>::kahan(vh, cvh, dv);
        Acc3<T, true>::kahan(u, cu, a.dt * vh);
    } else {
        vh += dv;
        u += a.dt * vh;
    }
}

// Reaction of step n-1, formed at the start of step n by the first block of
// each sample: the support-node forces of a step are written to one half of
// a double buffer and summed in FP64 by the next launch, so the kernel
// boundary orders the writes before the reads (no device-wide fences).  The
// sum runs in a fixed order (a strided pass over 64 lanes, then a fixed
// tree), so R depends neither on scheduling nor on the block size.
template <typename T, int NT>
__device__ __forceinline__ void reduce_previous(const StepParams<T> &a, int sample, int64_t n, double *part)
{
    const int64_t prev = n - 1;
    const double *rf = a.rf + ((int64_t)(prev & 1) * a.rf_stride) + (int64_t)sample * a.nsup;
    if (threadIdx.x < 64) {
        double sum = 0.0;
        for (int i = threadIdx.x; i < a.nsup; i += 64) sum += rf[i];
        part[threadIdx.x] = sum;
    }
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double R = -a.Rscale * part[0];
        if (!isfinite(R) && a.status[sample] == PD_OK) a.status[sample] = PD_ENONFINITE;
        if (R > a.Q[sample]) {
            a.Q[sample] = R;
            a.nstar[sample] = prev + 1;
        }
        if (a.hist_R) a.hist_R[(int64_t)sample * a.n_steps + prev] = R;
    }
}

// Forces and Verlet update of one node, given its neighbour source.  Every
// lane of the wavefront calls it (the exception pass works across lanes);
// lanes past the mesh edge pass valid = false and only help that pass.
// KF: compensated force sums; KS: compensated u / vh updates (both on in the
// production FP32 path; the ablation kernels take each one separately).
template <typename T, bool KF, bool KS, bool HAS_C, bool PLANE, typename Src>
__device__ __forceinline__ void node_step(const StepParams<T> &a, const Src &src, const SlotLds<T> &tab, int sample,
                                          int64_t n, int64_t node, int64_t p, const typename Vec4<T>::t &ui,
                                          bool valid, uint16_t *list)
{
    using V4 = typename Vec4<T>::t;
    const T *__restrict__ S0 = a.s0pad + (int64_t)sample * a.P;
    constexpr bool CW = HAS_C && !PLANE;   // c / c_ref in the flag word (3D)
    const T *__restrict__ Cp = HAS_C ? a.cpad + (int64_t)sample * a.P : nullptr;
    const int64_t sm = (int64_t)sample * a.M + node;
    const NodeInfo inf = valid ? a.info[node] : NodeInfo{-1, -1};
    const T ci = !(HAS_C && valid) ? T(1) : CW ? fabs(ui.w) : Cp[p];
    // without a fracture-energy field every bond reads the one unit value
    const int gstep = a.gstep;
    const T *__restrict__ Gp = a.gpad + (int64_t)sample * a.P * gstep;

    Acc3<T, KF> acc;
    acc.zero();
    // A node with a notch-cut bond, or one that has had an exceptional bond
    // (flag -1, kept from then on), runs the masked fast loop plus the
    // exception pass; so does every node of its wavefront, which then takes
    // one pass instead of two.  Other wavefronts run the plain fast loop, and
    // a node whose plain loop raises the flag is redone in masked form.
    // FP64 evaluates the closed form on both paths and always takes the
    // masked one.
    const bool is_cut = inf.cut >= 0;
    const bool sticky = valid && ui.w < T(0);
    bool masked = sizeof(T) == 8 || __any(is_cut || sticky) != 0;
    bool dirty = sticky;
    uint4 d0 = make_uint4(0u, 0u, 0u, 0u);
    uint32_t todo[4] = {0u, 0u, 0u, 0u};
    if (valid) {
        T thr = a.thr[sm];
        if constexpr (sizeof(T) == 4) thr = fmin(thr, T(kSeriesBound));
        if constexpr (sizeof(T) == 4) {
            if (!masked) {
                const uint32_t none[4] = {0u, 0u, 0u, 0u};
                uint32_t unused[4] = {0u, 0u, 0u, 0u};
                bool flag = false;
                fast_loop<T, KF, HAS_C, false, PLANE>(a, src, ui, ci, thr, acc, flag, none, unused);
                if (flag) {
                    acc.zero();
                    masked = true;
                }
            }
        }
        if (masked) {
            const uint4 cm = is_cut ? a.cut[inf.cut] : make_uint4(0u, 0u, 0u, 0u);
            if (sticky) d0 = a.dmask[sm];
            const uint32_t skip[4] = {cm.x | d0.x, cm.y | d0.y, cm.z | d0.z, cm.w | d0.w};
            uint32_t exc[4] = {0u, 0u, 0u, 0u};
            bool unused = false;
            fast_loop<T, KF, HAS_C, true, PLANE>(a, src, ui, ci, thr, acc, unused, skip, exc);
            todo[0] = exc[0] & ~cm.x;
            todo[1] = exc[1] & ~cm.y;
            todo[2] = exc[2] & ~cm.z;
            todo[3] = exc[3] & ~cm.w;
            dirty = dirty || ((exc[0] | exc[1] | exc[2] | exc[3]) != 0u);
        }
    }
    uint32_t dm[4] = {d0.x, d0.y, d0.z, d0.w};
    if (__any((todo[0] | todo[1] | todo[2] | todo[3]) != 0u)) {
        T *Hs = a.hist + (int64_t)sample * kStencil * a.M;
        const T s0i = valid ? S0[p] : T(1);
        const T gi = valid ? ld(Gp, p * gstep, 0u) : T(1);
        exc_pool<T, KF, HAS_C, CW>(a, src, tab, S0, Hs, Gp, gstep, (uint32_t)p, (uint32_t)node, ui, s0i, ci, gi, todo,
                                  dm, acc, list);
    }
    if (!valid) return;
    if (dm[0] != d0.x || dm[1] != d0.y || dm[2] != d0.z || dm[3] != d0.w)
        a.dmask[sm] = make_uint4(dm[0], dm[1], dm[2], dm[3]);
    if (a.force_only) {
        double *L = a.L_out + 3 * sm;
        L[0] = a.LV * ((double)acc.x - (KF ? (double)acc.cx : 0.0));
        L[1] = a.LV * ((double)acc.y - (KF ? (double)acc.cy : 0.0));
        L[2] = a.LV * ((double)acc.z - (KF ? (double)acc.cz : 0.0));
        return;
    }
    using V3 = typename Vec3<T>::t;
    using V2 = typename Vec2<T>::t;
    // a plane body stores (x, z) only: its y force, velocity and
    // displacement are zero throughout
    auto load3 = [&](const V3 *arr) {
        if constexpr (PLANE) {
            const V2 q = ((const V2 *)arr)[sm];
            return V3{q.x, T(0), q.y};
        } else {
            return arr[sm];
        }
    };
    auto store3 = [&](V3 *arr, const V3 &q) {
        if constexpr (PLANE) ((V2 *)arr)[sm] = V2{q.x, q.z};
        else arr[sm] = q;
    };
    V3 vh = load3(a.vh);
    V4 un = ui;
    V3 cu, cvh;
    if constexpr (KS) {
        cu = load3(a.cu);
        cvh = load3(a.cvh);
    } else {
        cu = V3{};
        cvh = V3{};
    }
    kick_drift<T, KS>(a, acc.gx(), vh.x, cvh.x, un.x, cu.x);
    if constexpr (!PLANE) kick_drift<T, KS>(a, acc.gy(), vh.y, cvh.y, un.y, cu.y);
    if (inf.bc == -1) {
        kick_drift<T, KS>(a, acc.gz(), vh.z, cvh.z, un.z, cu.z);
    } else if (inf.bc == -2) {
        vh.z = a.vload;
        un.z = (T)(-(double)(n + 2) * a.du_s);
        cu.z = T(0);
        cvh.z = T(0);
    } else {
        vh.z = T(0);
        un.z = T(0);
        cu.z = T(0);
        cvh.z = T(0);
        a.rf[(int64_t)(n & 1) * a.rf_stride + (int64_t)sample * a.nsup + inf.bc] =
            (double)acc.z - (KF ? (double)acc.cz : 0.0);
    }
    const T wn = CW ? ci : T(1);
    un.w = dirty ? -wn : wn;
    // every 64 steps (and at the last): a node whose state left the finite
    // numbers marks its sample (the reaction alone misses nodes away from
    // the supports); a status set earlier (an unstable field) is kept
    if (((n & 63) == 63 || n + 1 == a.n_steps) &&
        !(isfinite(un.x) && isfinite(un.y) && isfinite(un.z) && isfinite(vh.x) && isfinite(vh.y) && isfinite(vh.z)) &&
        a.status[sample] == PD_OK)
        a.status[sample] = PD_ENONFINITE;
    a.u_next[(int64_t)sample * a.P + p] = un;
    store3(a.vh, vh);
    if constexpr (KS) {
        store3(a.cu, cu);
        store3(a.cvh, cvh);
    }
}

// The node update a kernel runs: both compensations in the production
// kernels; in the FP32 kernels without them (the accuracy ablation) the
// launch's mode picks none, the force sums' only or the u / vh updates' only
// (the last two without a micromodulus field).
template <typename T, bool KAHAN, bool HAS_C, bool PLANE, typename Src>
__device__ __forceinline__ void node_step_mode(const StepParams<T> &a, const Src &src, const SlotLds<T> &tab,
                                               int sample, int64_t n, int64_t node, int64_t p,
                                               const typename Vec4<T>::t &ui, bool valid, uint16_t *list)
{
    if constexpr (KAHAN) {
        node_step<T, true, true, HAS_C, PLANE>(a, src, tab, sample, n, node, p, ui, valid, list);
    } else if constexpr (sizeof(T) == 8 || HAS_C) {
        node_step<T, false, false, HAS_C, PLANE>(a, src, tab, sample, n, node, p, ui, valid, list);
    } else {
        if (a.acc_mode == PD_ACC_STATE_ONLY)
            node_step<T, false, true, HAS_C, PLANE>(a, src, tab, sample, n, node, p, ui, valid, list);
        else if (a.acc_mode == PD_ACC_FORCES_ONLY)
            node_step<T, true, false, HAS_C, PLANE>(a, src, tab, sample, n, node, p, ui, valid, list);
        else
            node_step<T, false, false, HAS_C, PLANE>(a, src, tab, sample, n, node, p, ui, valid, list);
    }
}

// One time step for every (sample, tile) work item.
//   LDS = false: a tile is BR::N consecutive nodes; neighbours come from the
//                padded grid through the caches.
//   LDS = true : a tile is a BR::BX x BY x BZ brick; the block first copies
//                the brick and its kHalo-wide halo into LDS, then reads every
//                neighbour from there.
// Blocks are dealt round-robin to the 8 XCDs (block b runs on XCD b % 8); each
// XCD is given a contiguous range of work items so the halo a tile shares with
// its neighbours stays in that XCD's L2.  The grid is padded to a multiple of
// 8 and surplus blocks exit.
template <typename T, bool KAHAN, bool HAS_C, bool LDS, typename BR>
__device__ __forceinline__ void step_tile(const StepParams<T> &a, int64_t item)
{
    using V4 = typename Vec4<T>::t;
    __shared__ V4 tile[LDS ? BR::TILE : 1];
    __shared__ T ctile[(LDS && HAS_C && BR::PLANE) ? BR::TILE : 1];
    __shared__ SlotLds<T> tab;
    // the previous reaction's partial sums, then each wave's exception list
    __shared__ double scratch[128];
    static_assert(BR::N <= 256, "one 128-entry exception list per wave in 1 KB");
    uint16_t *list = (uint16_t *)scratch + 128 * (threadIdx.x / 64);
    // Each XCD takes a contiguous range of work items (sample major), so the
    // halos its bricks share stay in its L2.  When every XCD holds whole
    // samples (heavy_first), the bricks of a sample go in x slabs, the slabs
    // nearest the mid-span plane (notch and load pad, where the damaged bonds
    // and their costly exception pass are) first, so the cheapest bricks of
    // each XCD come last.  (Decided on the host: a read of device state here
    // would delay every block's start.)
    const int sample = (int)(item / a.tiles);
    int64_t t = item % a.tiles;
    if (LDS && a.heavy_first) {
        const int sr = (int)(t / a.chunk);    // slab rank, then the brick within the slab
        const int m = (a.nx / 2) / BR::BX;
        int bx = m;
        for (int q = 1, r = 0; r < sr; ++q) {   // ranks m, m - 1, m + 1, m - 2, ...
            const int cand = (q & 1) ? m - (q + 1) / 2 : m + q / 2;
            if (cand >= 0 && cand < a.nbx) {
                bx = cand;
                ++r;
            }
        }
        t = bx + (int64_t)a.nbx * (t % a.chunk);
    }
    const int64_t n = a.step_base[sample] + a.k_local;
    if (!a.force_only && t == 0 && n >= 1 && n <= a.n_steps) reduce_previous<T, BR::N>(a, sample, n, scratch);
    if (!a.force_only && n >= a.n_steps) return;   // whole block: finished sample
    const V4 *__restrict__ U = a.u_cur + (int64_t)sample * a.P;
    fill_slot_lds(tab);
    if constexpr (LDS) {
        const int bx = (int)(t % a.nbx), by = (int)((t / a.nbx) % a.nby), bz = (int)(t / ((int64_t)a.nbx * a.nby));
        // the tile's first padded cell is the brick origin (node + kHalo - kHalo);
        // a plane tile is the single row y = 0 (padded row kHalo)
        const int x0 = bx * BR::BX, y0 = by * BR::BY, z0 = bz * BR::BZ;
        constexpr int WX = BR::BX + 2 * kHalo;   // cells per row that hold data
        constexpr int YH = BR::PLANE ? 0 : kHalo; // y halo of the tile
        for (int q = threadIdx.x; q < WX * BR::LY * BR::LZ; q += BR::N) {
            const int lx = q % WX, ly = (q / WX) % BR::LY, lz = q / (WX * BR::LY);
            const int px = x0 + lx, py = y0 + ly + (kHalo - YH), pz = z0 + lz;
            const bool in = px < a.PX && py < a.PY && pz < a.PZ;
            const int64_t gi = px + (int64_t)py * a.PX + (int64_t)pz * a.PXY;
            V4 v{};
            if (in) v = U[gi];
            tile[lx + BR::LX * ly + BR::LXY * lz] = v;
            if constexpr (HAS_C && BR::PLANE)
                ctile[lx + BR::LX * ly + BR::LXY * lz] = in ? a.cpad[(int64_t)sample * a.P + gi] : T(0);
        }
        __syncthreads();
        const int tx = threadIdx.x % BR::BX, ty = (threadIdx.x / BR::BX) % BR::BY, tz = threadIdx.x / (BR::BX * BR::BY);
        const int ix = x0 + tx, iy = y0 + ty, iz = z0 + tz;
        const bool valid = ix < a.nx && iy < a.ny && iz < a.nz;
        const int64_t node = valid ? ix + (int64_t)a.nx * (iy + (int64_t)a.ny * iz) : 0;
        const int64_t p = valid ? (int64_t)(ix + kHalo) + (int64_t)(iy + kHalo) * a.PX + (int64_t)(iz + kHalo) * a.PXY : 0;
        const int c = (tx + kHalo) + BR::LX * (ty + YH) + BR::LXY * (tz + kHalo);
        const LdsSrc<T, BR> src{tile, ctile, c};
        node_step_mode<T, KAHAN, HAS_C, BR::PLANE>(a, src, tab, sample, n, node, p, tile[c], valid, list);
    } else {
        __syncthreads();
        const bool valid = t * BR::N + threadIdx.x < a.M;
        const int64_t node = valid ? t * BR::N + threadIdx.x : 0;
        const uint32_t nd = (uint32_t)node, nx = (uint32_t)a.nx, ny = (uint32_t)a.ny;
        const uint32_t r = nd / nx;
        const int ix = (int)(nd - r * nx);
        const int iz = (int)(r / ny);
        const int iy = (int)(r - (uint32_t)iz * ny);
        const int64_t p = (int64_t)(ix + kHalo) + (int64_t)(iy + kHalo) * a.PX + (int64_t)(iz + kHalo) * a.PXY;
        const GlobalSrc<T> src{U, (uint32_t)p * (uint32_t)sizeof(V4), a.PX, a.PXY,
                               HAS_C ? a.cpad + (int64_t)sample * a.P : nullptr, (uint32_t)p * (uint32_t)sizeof(T)};
        node_step_mode<T, KAHAN, HAS_C, BR::PLANE>(a, src, tab, sample, n, node, p, U[p], valid, list);
    }
}

template <typename T, bool KAHAN, bool HAS_C, bool LDS, typename BR>
__global__ __launch_bounds__(BR::N) void step_kernel(StepParams<T> a)
{
    const int64_t per_xcd = gridDim.x / kXcds;
    const int64_t item = (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
    if (item >= a.n_items) return;
    step_tile<T, KAHAN, HAS_C, LDS, BR>(a, item);
}

// One time tick of several solves (the levels of a batch) in one launch: the
// work items of solve i occupy [first[i], first[i] + p[i].n_items) of one
// work list, which the XCDs take in contiguous ranges as above.
constexpr int kMaxTickItems = 4;

template <typename T>
struct TickParams {
    StepParams<T> p[kMaxTickItems];
    int64_t first[kMaxTickItems + 1];
    int n;
};

template <typename T, bool KAHAN, bool HAS_C, bool LDS, typename BR>
__global__ __launch_bounds__(BR::N) void step_kernel_tick(TickParams<T> m)
{
    const int64_t per_xcd = gridDim.x / kXcds;
    const int64_t g = (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
    if (g >= m.first[m.n]) return;
    int i = 0;
    while (i + 1 < m.n && g >= m.first[i + 1]) ++i;
    step_tile<T, KAHAN, HAS_C, LDS, BR>(m.p[i], g - m.first[i]);
}

// Moves every sample's chunk base past the steps of one replayed chunk.
static __global__ void advance_kernel(int64_t *step_base, int64_t S, int64_t by)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < S) step_base[g] += by;
}

}  // namespace pdmi
