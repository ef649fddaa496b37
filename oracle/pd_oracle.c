/*
 * Reference oracle: a plain, slow FP64 implementation of the bond-based
 * peridynamic beam solve.  TEST INFRASTRUCTURE ONLY: it is used by the test
 * suite, the smoke check and the CPU baseline of the benchmark, and never by
 * the product library.  It shares no code with the GPU path.
 *
 * What it computes (one sample):
 *   - bond stretch s = (|xi + eta| - |xi|) / |xi|           (section 2.1, Eq. PD_Force_Function)
 *   - bond force f = c_b (1 - d_b) s along the deformed bond  (appendix A, Eq. exp_scalar_force)
 *   - irreversible damage d_b = D(kappa_b), kappa_b the largest stretch seen so
 *     far; D is the appendix-A softening law (Eq. exp_damage_parameter) or the
 *     piecewise-linear envelope with the same fracture energy
 *   - nodal force density L_i = sum_j f e_ij V_j              (section 2.1, Eq. PD_EOM_Dynamic)
 *   - damped velocity-Verlet under prescribed support / load displacements
 *   - support reaction R^n and its running maximum Q, the peak load (section 4, QoI)
 *
 * Every loop runs over the unique bond list in its given order; no fusion,
 * no reordering, no compensation.  The bond loop of a force evaluation is cut
 * into a fixed number of contiguous chunks, each summing into a buffer of its
 * own, and the buffers are added in chunk order: with OpenMP the chunks run
 * on the host's cores, and the result is the same for any thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* bond chunks of a force evaluation (fixed: results do not depend on threads) */
#define PDO_CHUNKS 16

#define PDO_PI 3.14159265358979323846
#define PDO_LAW_EXPLIN 0
#define PDO_LAW_TRILINEAR 1

typedef struct {
    int64_t n_nodes;
    int64_t n_bonds;
    const int32_t *bond_i;     /* [n_bonds], bond_i < bond_j */
    const int32_t *bond_j;     /* [n_bonds] */
    const double *xi;          /* [n_bonds][3] reference bond vector x_j - x_i */
    const double *s0_node;     /* [n_nodes] linear-elastic limit stretch */
    const double *c_node;      /* [n_nodes] micromodulus */
    int64_t n_support;
    const int32_t *support;    /* nodes with u_z = 0 */
    int64_t n_load;
    const int32_t *load;       /* nodes with u_z = -(n+1) du */
    double volume;             /* nodal volume dx^3 */
    double rho;                /* mass density */
    double damping;            /* viscous damping coefficient (force density per velocity) */
    double dt;
    double du;                 /* load displacement increment per step */
    int64_t n_steps;
    int32_t law;               /* PDO_LAW_* */
    double k, alpha;           /* softening shape parameters */
    double GF;                 /* fracture energy */
    double delta;              /* horizon */
    double load_offset;        /* load pad u_z = load_offset - (n+1) du (0 for a fresh run) */
    const double *gf_node;     /* [n_nodes] fracture energy per node, or NULL: GF everywhere */
    double thickness;          /* 0: 3D body; > 0: plane stress of this thickness */
} pdo_problem;

/* ---------------------------------------------------------------- material */

/* Critical stretch s_c.
 * EXPLIN: solve the 3D fracture-energy relation of appendix A
 *   G_F = pi c s0 delta^5 (s0 - sc) P / (10 k (e^k - 1)(1 + alpha)),
 *   P = 2k - 2e^k + alpha k - alpha k e^k + 2,
 * for sc.  (The printed rearrangement, Eq. exp_sc, drops the (1 + alpha)
 * factor inside the bracket; solving the energy relation itself is used.)
 * TRILINEAR: envelope through (s0, c s0), (s1, 0.2 c s0), (sc, 0) with
 * s1 = s0 + 0.2 (sc - s0); its softening area is 0.2 c s0 (sc - s0), and the
 * same fracture-energy integral G_F = (pi delta^5 / 5) * area gives sc. */
double pdo_critical_stretch(int32_t law, double s0, double c, double GF, double delta,
                            double k, double alpha)
{
    double d5 = pow(delta, 5.0);
    if (law == PDO_LAW_EXPLIN) {
        double ek = exp(k);
        double P = 2.0 * k - 2.0 * ek + alpha * k - alpha * k * ek + 2.0;
        double s0_minus_sc = GF * 10.0 * k * (ek - 1.0) * (1.0 + alpha) / (PDO_PI * c * s0 * d5 * P);
        return s0 - s0_minus_sc;
    }
    /* trilinear: GF = (pi d5 / 5) * 0.2 c s0 (sc - s0) */
    return s0 + GF * 5.0 / (PDO_PI * d5 * 0.2 * c * s0);
}

/* Critical stretch in plane stress (appendix A, two-dimensional case):
 * the same bond work integrated over the 2D horizon, Eq. exp_fracture_energy_2D,
 *   G_F = h c s0 delta^4 (s0 - sc) P / (4 k (e^k - 1)(1 + alpha))   (EXPLIN),
 *   G_F = (h delta^4 / 2) 0.2 c s0 (sc - s0)                        (TRILINEAR),
 * solved for sc (the printed Eq. exp_sc_2D is this rearrangement). */
double pdo_critical_stretch_2d(int32_t law, double s0, double c, double GF, double delta, double h,
                               double k, double alpha)
{
    double d4 = pow(delta, 4.0);
    if (law == PDO_LAW_EXPLIN) {
        double ek = exp(k);
        double P = 2.0 * k - 2.0 * ek + alpha * k - alpha * k * ek + 2.0;
        double s0_minus_sc = GF * 4.0 * k * (ek - 1.0) * (1.0 + alpha) / (h * c * s0 * d4 * P);
        return s0 - s0_minus_sc;
    }
    return s0 + GF / (0.5 * h * d4 * 0.2 * c * s0);
}

/* Damage d = D(kappa) for a bond with limit stretch s0 and critical stretch sc
 * (appendix A, Eq. exp_damage_parameter, clamped outside [s0, sc]). */
double pdo_damage(int32_t law, double kappa, double s0, double sc, double k, double alpha)
{
    if (!(kappa > s0)) return 0.0;
    if (kappa >= sc) return 1.0;
    if (law == PDO_LAW_EXPLIN) {
        double t = (kappa - s0) / (sc - s0);
        double bracket = 1.0 - (1.0 - exp(-k * t)) / (1.0 - exp(-k)) + alpha * (1.0 - t);
        return 1.0 - (s0 / kappa) * bracket / (1.0 + alpha);
    }
    /* trilinear envelope force / (c kappa) */
    double s1 = s0 + 0.2 * (sc - s0);
    double fenv;  /* envelope force divided by c */
    if (kappa <= s1)
        fenv = s0 * (1.0 - 0.8 * (kappa - s0) / (s1 - s0));
    else
        fenv = 0.2 * s0 * (sc - kappa) / (sc - s1);
    return 1.0 - fenv / kappa;
}

/* ---------------------------------------------------------------- force */

/* One bond: stretch, damage history (updated in place), force f e V added to
 * node i and subtracted from node j of the buffer L. */
static void bond_force(const pdo_problem *p, int64_t b, const double *u, double *kappa, const double *c_b,
                       const double *s0_b, const double *sc_b, double *L)
{
    int32_t i = p->bond_i[b], j = p->bond_j[b];
    const double *xi = p->xi + 3 * b;
    double y[3];
    for (int d = 0; d < 3; ++d) y[d] = xi[d] + (u[3 * j + d] - u[3 * i + d]);
    double ylen = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    double xlen = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
    double s = (ylen - xlen) / xlen;
    if (s > kappa[b]) kappa[b] = s;
    double dmg = pdo_damage(p->law, kappa[b], s0_b[b], sc_b[b], p->k, p->alpha);
    double f = c_b[b] * (1.0 - dmg) * s;
    for (int d = 0; d < 3; ++d) {
        double fd = f * (y[d] / ylen) * p->volume;
        L[3 * i + d] += fd;
        L[3 * j + d] -= fd;
    }
}

/* One force evaluation: L = sum over bonds of f e V, damage history updated in
 * place.  kappa[b] holds the largest stretch bond b has seen (-inf initially).
 * work: PDO_CHUNKS * 3 * n_nodes doubles (chunk buffers).  A chunk's bonds
 * touch a contiguous node range [lo, hi] (the bond list is sorted by node),
 * so only that range of its buffer is cleared and summed. */
static void force_eval(const pdo_problem *p, const double *u, double *kappa,
                       const double *c_b, const double *s0_b, const double *sc_b,
                       double *L, double *work)
{
    const int64_t M = p->n_nodes, M3 = 3 * M, nb = p->n_bonds;
    int64_t lo[PDO_CHUNKS], hi[PDO_CHUNKS];
#pragma omp parallel for schedule(static, 1)
    for (int ch = 0; ch < PDO_CHUNKS; ++ch) {
        double *Lc = work + (int64_t)ch * M3;
        const int64_t b0 = nb * ch / PDO_CHUNKS, b1 = nb * (ch + 1) / PDO_CHUNKS;
        int64_t a = M, z = -1;
        for (int64_t b = b0; b < b1; ++b) {
            const int64_t i = p->bond_i[b], j = p->bond_j[b];
            if (i < a) a = i;
            if (j < a) a = j;
            if (i > z) z = i;
            if (j > z) z = j;
        }
        lo[ch] = a;
        hi[ch] = z;
        if (z >= a) memset(Lc + 3 * a, 0, sizeof(double) * 3 * (z - a + 1));
        for (int64_t b = b0; b < b1; ++b) bond_force(p, b, u, kappa, c_b, s0_b, sc_b, Lc);
    }
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < M3; ++q) {
        const int64_t node = q / 3;
        double acc = 0.0;
        for (int ch = 0; ch < PDO_CHUNKS; ++ch)
            if (node >= lo[ch] && node <= hi[ch]) acc += work[(int64_t)ch * M3 + q];
        L[q] = acc;
    }
}

/* Threads of the force loop (OpenMP builds; 1 otherwise).  n <= 0 leaves the
 * setting unchanged.  Returns the number now in use. */
int pdo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

static double *chunk_work(const pdo_problem *p)
{
    return malloc(sizeof(double) * PDO_CHUNKS * 3 * (size_t)(p->n_nodes > 0 ? p->n_nodes : 1));
}

static void bond_params(const pdo_problem *p, double *c_b, double *s0_b, double *sc_b)
{
    for (int64_t b = 0; b < p->n_bonds; ++b) {
        int32_t i = p->bond_i[b], j = p->bond_j[b];
        c_b[b] = 0.5 * (p->c_node[i] + p->c_node[j]);
        s0_b[b] = 0.5 * (p->s0_node[i] + p->s0_node[j]);
        double gf_b = p->gf_node ? 0.5 * (p->gf_node[i] + p->gf_node[j]) : p->GF;
        sc_b[b] = p->thickness > 0
                      ? pdo_critical_stretch_2d(p->law, s0_b[b], c_b[b], gf_b, p->delta, p->thickness, p->k, p->alpha)
                      : pdo_critical_stretch(p->law, s0_b[b], c_b[b], gf_b, p->delta, p->k, p->alpha);
    }
}

/* Force on a frozen displacement field, with an optional damage history
 * (kappa may be NULL for an undamaged body; otherwise it is updated). */
int pdo_force(const pdo_problem *p, const double *u, double *kappa, double *L)
{
    int64_t nb = p->n_bonds;
    double *c_b = malloc(sizeof(double) * nb), *s0_b = malloc(sizeof(double) * nb),
           *sc_b = malloc(sizeof(double) * nb), *kap = NULL, *work = chunk_work(p);
    if (!c_b || !s0_b || !sc_b || !work) return -2;
    bond_params(p, c_b, s0_b, sc_b);
    if (!kappa) {
        kap = malloc(sizeof(double) * nb);
        for (int64_t b = 0; b < nb; ++b) kap[b] = -INFINITY;
    }
    force_eval(p, u, kappa ? kappa : kap, c_b, s0_b, sc_b, L, work);
    free(c_b); free(s0_b); free(sc_b); free(kap); free(work);
    return 0;
}

/* Bond stretches of a frozen displacement field (for inspection in tests). */
int pdo_stretch(const pdo_problem *p, const double *u, double *s_out)
{
    for (int64_t b = 0; b < p->n_bonds; ++b) {
        int32_t i = p->bond_i[b], j = p->bond_j[b];
        const double *xi = p->xi + 3 * b;
        double y[3];
        for (int d = 0; d < 3; ++d) y[d] = xi[d] + (u[3 * j + d] - u[3 * i + d]);
        double ylen = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
        double xlen = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
        s_out[b] = (ylen - xlen) / xlen;
    }
    return 0;
}

/* ---------------------------------------------------------------- time loop */

/* Damped velocity-Verlet with displacement control.  Per step n = 0..N-1:
 *   1. free DOFs: v += (dt / 2 rho) (L - damping v)
 *   2. all DOFs:  u += dt v
 *   3. supports: u_z = 0, v_z = 0; load pad: u_z = -(n+1) du, v_z = -du / dt
 *   4. L = force(u), damage history updated
 *   5. free DOFs: v = (v + (dt / 2 rho) L) / (1 + damping dt / 2 rho)
 *   6. R = -sum over supports of L_z V; Q = max R, nstar = first argmax (1-based)
 * u_init / v_init / kappa_init may be NULL (undamaged body at rest).
 * Outputs may be NULL except Q. */
int pdo_run(const pdo_problem *p, const double *u_init, const double *v_init,
            const double *kappa_init, double *Q_out, int64_t *nstar_out, double *R_hist,
            double *u_out, double *v_out, double *kappa_out)
{
    int64_t M = p->n_nodes, nb = p->n_bonds;
    double *u = calloc(3 * M, sizeof(double)), *v = calloc(3 * M, sizeof(double));
    double *L = calloc(3 * M, sizeof(double));
    double *kappa = malloc(sizeof(double) * nb);
    double *c_b = malloc(sizeof(double) * nb), *s0_b = malloc(sizeof(double) * nb),
           *sc_b = malloc(sizeof(double) * nb), *work = chunk_work(p);
    unsigned char *fixed_z = calloc(M, 1);
    if (!u || !v || !L || !kappa || !c_b || !s0_b || !sc_b || !fixed_z || !work) return -2;
    if (u_init) memcpy(u, u_init, sizeof(double) * 3 * M);
    if (v_init) memcpy(v, v_init, sizeof(double) * 3 * M);
    for (int64_t b = 0; b < nb; ++b) kappa[b] = kappa_init ? kappa_init[b] : -INFINITY;
    bond_params(p, c_b, s0_b, sc_b);
    for (int64_t a = 0; a < p->n_support; ++a) fixed_z[p->support[a]] = 1;
    for (int64_t a = 0; a < p->n_load; ++a) fixed_z[p->load[a]] = 1;

    /* the initial force of the (possibly pre-displaced) body */
    force_eval(p, u, kappa, c_b, s0_b, sc_b, L, work);

    double h = p->dt / (2.0 * p->rho);
    double Q = -INFINITY;
    int64_t nstar = 0;
    for (int64_t n = 0; n < p->n_steps; ++n) {
        for (int64_t i = 0; i < M; ++i)
            for (int d = 0; d < 3; ++d) {
                if (d == 2 && fixed_z[i]) continue;
                v[3 * i + d] += h * (L[3 * i + d] - p->damping * v[3 * i + d]);
            }
        for (int64_t i = 0; i < 3 * M; ++i) u[i] += p->dt * v[i];
        for (int64_t a = 0; a < p->n_support; ++a) {
            u[3 * p->support[a] + 2] = 0.0;
            v[3 * p->support[a] + 2] = 0.0;
        }
        for (int64_t a = 0; a < p->n_load; ++a) {
            u[3 * p->load[a] + 2] = p->load_offset - (double)(n + 1) * p->du;
            v[3 * p->load[a] + 2] = -p->du / p->dt;
        }
        force_eval(p, u, kappa, c_b, s0_b, sc_b, L, work);
        for (int64_t i = 0; i < M; ++i)
            for (int d = 0; d < 3; ++d) {
                if (d == 2 && fixed_z[i]) continue;
                v[3 * i + d] = (v[3 * i + d] + h * L[3 * i + d]) / (1.0 + p->damping * h);
            }
        double R = 0.0;
        for (int64_t a = 0; a < p->n_support; ++a) R -= L[3 * p->support[a] + 2] * p->volume;
        if (R_hist) R_hist[n] = R;
        if (R > Q) { Q = R; nstar = n + 1; }
    }
    *Q_out = Q;
    if (nstar_out) *nstar_out = nstar;
    if (u_out) memcpy(u_out, u, sizeof(double) * 3 * M);
    if (v_out) memcpy(v_out, v, sizeof(double) * 3 * M);
    if (kappa_out) memcpy(kappa_out, kappa, sizeof(double) * nb);
    free(u); free(v); free(L); free(kappa); free(c_b); free(s0_b); free(sc_b); free(fixed_z); free(work);
    return 0;
}

/* ---------------------------------------------------------------- adjoint */

/* keep = 1 - d as a function of (kappa, s0, sc), with its partial
 * derivatives.  Outside (s0, sc) keep is constant (1 or 0) and every
 * derivative is zero. */
static void keep_derivs(int32_t law, double kappa, double s0, double sc, double k, double alpha,
                        double *keep, double *dk, double *ds0, double *dsc)
{
    *dk = *ds0 = *dsc = 0.0;
    if (!(kappa > s0)) { *keep = 1.0; return; }
    if (kappa >= sc) { *keep = 0.0; return; }
    double w = sc - s0;
    double t = (kappa - s0) / w;
    double t_k = 1.0 / w, t_s0 = (kappa - sc) / (w * w), t_sc = -(kappa - s0) / (w * w);
    double g, g_t, g_s0;   /* keep = g / kappa with g = g(t, s0) */
    if (law == PDO_LAW_EXPLIN) {
        double ek = 1.0 - exp(-k);
        double br = 1.0 - (1.0 - exp(-k * t)) / ek + alpha * (1.0 - t);
        double br_t = -k * exp(-k * t) / ek - alpha;
        g = s0 * br / (1.0 + alpha);
        g_t = s0 * br_t / (1.0 + alpha);
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
    *keep = g / kappa;
    *dk = g_t * t_k / kappa - g / (kappa * kappa);
    *ds0 = (g_s0 + g_t * t_s0) / kappa;
    *dsc = g_t * t_sc / kappa;
}

/* exposed for tests */
void pdo_keep_derivs(int32_t law, double kappa, double s0, double sc, double k, double alpha, double *out4)
{
    keep_derivs(law, kappa, s0, sc, k, alpha, out4, out4 + 1, out4 + 2, out4 + 3);
}

/* Gradient of the peak reaction Q = R^{n*} (n* fixed by the forward run)
 * with respect to the per-node limit-stretch field s0 and micromodulus field
 * c, by the discrete adjoint of pdo_run's loop.  The forward pass keeps every
 * displacement u^n and, for the damage history, the list of bonds whose
 * largest stretch grew past their limit stretch at each step (with the old
 * value), so the reverse sweep can restore kappa^n exactly.  Written with the
 * half-step velocity w^n = v^n + (dt/2rho)(L^n - damping v^n) as the state:
 *   w^n = A D w^{n-1} + h (1 + A D) L^n,  u^{n+1} = u^n + dt w^n  (free DOFs),
 *   h = dt / 2rho, A = 1 - damping h, D = 1 / (1 + damping h),
 *   kappa^n = max(kappa^{n-1}, s(u^n)),  L^n = F(u^n, kappa^n; s0, c),
 *   R^n = -V sum_supports L^n_z.
 * Starts from rest.  dQ_ds0 / dQ_dc: [n_nodes], overwritten. */
int pdo_adjoint(const pdo_problem *p, double *Q_out, int64_t *nstar_out, double *dQ_ds0, double *dQ_dc)
{
    int64_t M = p->n_nodes, nb = p->n_bonds, N = p->n_steps;
    double V = p->volume, h = p->dt / (2.0 * p->rho);
    double A = 1.0 - p->damping * h, D = 1.0 / (1.0 + p->damping * h);
    double a1 = A * D, a2 = h * (1.0 + A * D);
    double *U = malloc(sizeof(double) * 3 * M * (N + 1));   /* u^0 .. u^N */
    double *v = calloc(3 * M, sizeof(double)), *L = calloc(3 * M, sizeof(double));
    double *kappa = malloc(sizeof(double) * nb);
    double *c_b = malloc(sizeof(double) * nb), *s0_b = malloc(sizeof(double) * nb),
           *sc_b = malloc(sizeof(double) * nb), *work = chunk_work(p);
    unsigned char *fixed_z = calloc(M, 1);
    int64_t *ev_start = calloc(N + 2, sizeof(int64_t));
    int64_t ev_cap = 1 << 16, ev_n = 0;
    int32_t *ev_bond = malloc(sizeof(int32_t) * ev_cap);
    double *ev_old = malloc(sizeof(double) * ev_cap);
    if (!U || !v || !L || !kappa || !c_b || !s0_b || !sc_b || !fixed_z || !ev_start || !ev_bond || !ev_old || !work)
        return -2;
    bond_params(p, c_b, s0_b, sc_b);
    for (int64_t b = 0; b < nb; ++b) kappa[b] = -INFINITY;
    for (int64_t a = 0; a < p->n_support; ++a) fixed_z[p->support[a]] = 1;
    for (int64_t a = 0; a < p->n_load; ++a) fixed_z[p->load[a]] = 1;
    memset(U, 0, sizeof(double) * 3 * M);

    /* forward (same arithmetic as pdo_run) */
    double Q = -INFINITY;
    int64_t nstar = 0;
    for (int64_t n = 0; n < N; ++n) {
        double *u0 = U + 3 * M * n, *u1 = U + 3 * M * (n + 1);
        for (int64_t i = 0; i < M; ++i)
            for (int d = 0; d < 3; ++d) {
                if (d == 2 && fixed_z[i]) continue;
                v[3 * i + d] += h * (L[3 * i + d] - p->damping * v[3 * i + d]);
            }
        for (int64_t i = 0; i < 3 * M; ++i) u1[i] = u0[i] + p->dt * v[i];
        for (int64_t a = 0; a < p->n_support; ++a) {
            u1[3 * p->support[a] + 2] = 0.0;
            v[3 * p->support[a] + 2] = 0.0;
        }
        for (int64_t a = 0; a < p->n_load; ++a) {
            u1[3 * p->load[a] + 2] = p->load_offset - (double)(n + 1) * p->du;
            v[3 * p->load[a] + 2] = -p->du / p->dt;
        }
        /* damage history events of step n+1 */
        ev_start[n + 1] = ev_n;
        for (int64_t b = 0; b < nb; ++b) {
            int32_t i = p->bond_i[b], j = p->bond_j[b];
            const double *xi = p->xi + 3 * b;
            double y[3];
            for (int d = 0; d < 3; ++d) y[d] = xi[d] + (u1[3 * j + d] - u1[3 * i + d]);
            double ylen = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
            double xlen = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
            double s = (ylen - xlen) / xlen;
            if (s > kappa[b] && s > s0_b[b]) {
                if (ev_n == ev_cap) {
                    ev_cap *= 2;
                    ev_bond = realloc(ev_bond, sizeof(int32_t) * ev_cap);
                    ev_old = realloc(ev_old, sizeof(double) * ev_cap);
                    if (!ev_bond || !ev_old) return -2;
                }
                ev_bond[ev_n] = (int32_t)b;
                ev_old[ev_n] = kappa[b];
                ++ev_n;
            }
        }
        force_eval(p, u1, kappa, c_b, s0_b, sc_b, L, work);
        for (int64_t i = 0; i < M; ++i)
            for (int d = 0; d < 3; ++d) {
                if (d == 2 && fixed_z[i]) continue;
                v[3 * i + d] = (v[3 * i + d] + h * L[3 * i + d]) / (1.0 + p->damping * h);
            }
        double R = 0.0;
        for (int64_t a = 0; a < p->n_support; ++a) R -= L[3 * p->support[a] + 2] * V;
        if (R > Q) { Q = R; nstar = n + 1; }
    }
    ev_start[N + 1] = ev_n;
    *Q_out = Q;
    if (nstar_out) *nstar_out = nstar;

    /* kappa^{n*}: undo the growth events of steps after n* */
    for (int64_t m = N; m > nstar; --m)
        for (int64_t e = ev_start[m + 1] - 1; e >= ev_start[m]; --e) kappa[ev_bond[e]] = ev_old[e];

    /* reverse sweep */
    double *ub_next = calloc(3 * M, sizeof(double)), *ub = calloc(3 * M, sizeof(double));
    double *wb = calloc(3 * M, sizeof(double)), *Lb = calloc(3 * M, sizeof(double));
    double *kb = calloc(nb, sizeof(double));
    unsigned char *active = calloc(nb, 1);
    if (!ub_next || !ub || !wb || !Lb || !kb || !active) return -2;
    memset(dQ_ds0, 0, sizeof(double) * M);
    memset(dQ_dc, 0, sizeof(double) * M);
    for (int64_t m = nstar; m >= 1; --m) {
        const double *um = U + 3 * M * m;
        /* u^{m+1} = u^m + dt w^m on free DOFs */
        for (int64_t i = 0; i < M; ++i)
            for (int d = 0; d < 3; ++d) {
                int64_t q = 3 * i + d;
                double g = (d == 2 && fixed_z[i]) ? 0.0 : ub_next[q];
                wb[q] = (d == 2 && fixed_z[i]) ? 0.0 : wb[q] + p->dt * g;
                ub[q] = g;
                Lb[q] = a2 * wb[q];
            }
        if (m == nstar)
            for (int64_t a = 0; a < p->n_support; ++a) Lb[3 * p->support[a] + 2] += -V;
        /* L^m = F(u^m, kappa^m) */
        for (int64_t e = ev_start[m]; e < ev_start[m + 1]; ++e) active[ev_bond[e]] = 1;
        for (int64_t b = 0; b < nb; ++b) {
            int32_t i = p->bond_i[b], j = p->bond_j[b];
            const double *xi = p->xi + 3 * b;
            double y[3], Fb[3];
            for (int d = 0; d < 3; ++d) y[d] = xi[d] + (um[3 * j + d] - um[3 * i + d]);
            double l = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
            double x0 = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
            double s = (l - x0) / x0;
            double yh[3] = {y[0] / l, y[1] / l, y[2] / l};
            for (int d = 0; d < 3; ++d) Fb[d] = Lb[3 * i + d] - Lb[3 * j + d];
            double proj = yh[0] * Fb[0] + yh[1] * Fb[1] + yh[2] * Fb[2];
            double keep, dk, ds0, dsc;
            keep_derivs(p->law, kappa[b], s0_b[b], sc_b[b], p->k, p->alpha, &keep, &dk, &ds0, &dsc);
            double cb = c_b[b];
            /* y-bar = V c keep [yh proj / |xi| + (s / l)(F - yh proj)] */
            double ybar[3];
            for (int d = 0; d < 3; ++d)
                ybar[d] = V * cb * keep * (yh[d] * proj / x0 + (s / l) * (Fb[d] - yh[d] * proj));
            /* damage history: F depends on kappa through keep */
            kb[b] += V * cb * s * dk * proj;
            /* fields: sc = s0 + G / (c s0), G from the fracture-energy relation */
            double Gm = (sc_b[b] - s0_b[b]) * cb * s0_b[b];
            double dsc_dc = -Gm / (cb * cb * s0_b[b]);
            double dsc_ds0 = 1.0 - Gm / (cb * s0_b[b] * s0_b[b]);
            double cbar = V * s * proj * (keep + cb * dsc * dsc_dc);
            double s0bar = V * cb * s * proj * (ds0 + dsc * dsc_ds0);
            dQ_dc[i] += 0.5 * cbar;
            dQ_dc[j] += 0.5 * cbar;
            dQ_ds0[i] += 0.5 * s0bar;
            dQ_ds0[j] += 0.5 * s0bar;
            /* kappa^m = max(kappa^{m-1}, s(u^m)) */
            if (active[b]) {
                for (int d = 0; d < 3; ++d) ybar[d] += kb[b] * yh[d] / x0;
                kb[b] = 0.0;
            }
            for (int d = 0; d < 3; ++d) {
                ub[3 * j + d] += ybar[d];
                ub[3 * i + d] -= ybar[d];
            }
        }
        /* restore kappa^{m-1} and clear the active marks */
        for (int64_t e = ev_start[m + 1] - 1; e >= ev_start[m]; --e) {
            kappa[ev_bond[e]] = ev_old[e];
            active[ev_bond[e]] = 0;
        }
        /* w^m = a1 w^{m-1} + a2 L^m */
        for (int64_t q = 0; q < 3 * M; ++q) {
            wb[q] *= a1;
            ub_next[q] = ub[q];
        }
    }
    free(U); free(v); free(L); free(kappa); free(c_b); free(s0_b); free(sc_b); free(fixed_z); free(work);
    free(ev_start); free(ev_bond); free(ev_old);
    free(ub_next); free(ub); free(wb); free(Lb); free(kb); free(active);
    return 0;
}
