/*
 * pd.h -- C ABI of the MI355X peridynamic MC/MLMC solver (libpdmi.so).
 *
 * The library runs the explicit bond-based peridynamic solve of a notched
 * three-point-bending beam once per Monte-Carlo / multilevel-Monte-Carlo
 * sample, on one AMD Instinct MI355X (gfx950), and reduces each run to its
 * peak support reaction.  Paper: Hobbs, Rappel, Dodwell, "A probabilistic
 * peridynamic framework with an application to the study of the statistical
 * size effect" (arXiv 2212.04415).
 *
 * Conventions for every entry point:
 *   - Return value: PD_OK (0) or a negative PD_E* code.  The message of the
 *     last error on the calling thread is available from pd_last_error().
 *     No C++ exception crosses this boundary.
 *   - Units: SI (m, kg, s, N, Pa) in FP64 host scalars.
 *   - Node order: cell-centred lattice, node (i, j, k) at ((i+1/2)dx,
 *     (j+1/2)dx, (k+1/2)dx) with index i + nx (j + ny k) (x fastest).
 *   - Handles (pd_mesh, pd_run_h, pd_kl) and every device array the library
 *     allocates for them are owned by the library and released by the
 *     matching pd_free_* call.  Buffers passed in by the caller stay owned by
 *     the caller and must stay valid until the stream work that uses them has
 *     completed.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *     Entry points marked "async" only enqueue work on that stream.
 */
#ifndef PD_H
#define PD_H

#include <stdint.h>

#if defined(__GNUC__)
#define PD_API __attribute__((visibility("default")))
#else
#define PD_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PD_OK = 0,
    PD_EINVAL = -1,      /* invalid argument or size */
    PD_ENOMEM = -2,      /* host or device allocation failed */
    PD_EDEVICE = -3,     /* HIP runtime error, or the HIP device is missing */
    PD_EUNSTABLE = -4,   /* dt above the explicit stability limit */
    PD_ENONFINITE = -5,  /* a run went non-finite (reaction or node state) */
    PD_ESTATE = -6       /* call out of order (e.g. bonds not built) */
};

enum { PD_LAW_EXPLIN = 0, PD_LAW_TRILINEAR = 1 };
enum { PD_FP32 = 0, PD_FP64 = 1 };
enum { PD_ACC_KAHAN = 0, PD_ACC_PLAIN = 1, PD_ACC_STATE_ONLY = 2, PD_ACC_FORCES_ONLY = 3 };
enum { PD_FIELD_S0 = 0, PD_FIELD_C = 1, PD_FIELD_GF = 2 };
enum { PD_DTYPE_F32 = 0, PD_DTYPE_F64 = 1 };
/* Launch shapes of the step kernel: nodes per block as an x-by-y-by-z brick
 * staged with its halo in LDS (the 12x4x4 brick, 192 threads, wastes fewer
 * lanes on meshes whose extents are not multiples of 16, such as the
 * 35-node-long coarsest beam), or 256 consecutive nodes read through the
 * caches.  On a mesh one node thick (a plane body) the three brick shapes
 * are 64x4, 32x8 and 32x4 patches of the x-z plane.  All shapes give
 * bit-identical results. */
enum {
    PD_SHAPE_AUTO = -1,
    PD_SHAPE_LDS_16x4x4 = 0,
    PD_SHAPE_LDS_8x8x4 = 1,
    PD_SHAPE_LDS_12x4x4 = 2,
    PD_SHAPE_GLOBAL_256 = 3,
    PD_N_SHAPES = 4
};

typedef struct pd_mesh_s *pd_mesh;
typedef struct pd_run_s *pd_run_h;
typedef struct pd_kl_s *pd_kl;

/* Beam geometry (paper section 6.2 set-up; section 2.1 horizon).
 * The body is the box [0, extent[0]] x [0, extent[1]] x [0, extent[2]]
 * (length, thickness, depth).  Each extent must be a whole number of dx.
 * The horizon is delta = m_ratio * dx (paper: m = 3.14).  Supports are two
 * pad_width x pad_width blocks on the bottom face centred on
 * x = extent[0]/2 -+ span/2; the load pad is one block on the top face centred
 * on x = extent[0]/2; every pad spans the whole thickness.  notch_depth > 0
 * cuts every bond crossing the plane x = extent[0]/2 below that height.
 * thickness = 0: a 3D body.  thickness > 0: a plane body of that thickness
 * (appendix A: nodal volume dx^2 t; critical stretch from
 * Eq. exp_fracture_energy_2D), in plane stress (plane_strain = 0,
 * Eq. bond_stiffness_constant: c = 9E / (pi t delta^3)) or plane strain
 * (plane_strain = 1: c = 48E / (5 pi t delta^3)), represented with one node
 * through the thickness (extent[1] = dx): every out-of-plane neighbour is
 * absent, so the 28 in-plane bonds remain.  plane_strain must be 0 for a 3D
 * body (PD_EINVAL otherwise). */
typedef struct {
    double extent[3];
    double dx;
    double m_ratio;
    double span;
    double notch_depth;
    double pad_width;
    double thickness;
    int32_t plane_strain;
} pd_mesh_desc;

/* Material, loading and numerics of a run.
 * E: Young's modulus (micromodulus c = 12 E / (pi delta^4), appendix A);
 * rho: density; GF: fracture energy; s0: homogeneous linear-elastic limit
 * stretch (used when no per-node field is set); k, alpha: softening shape
 * (appendix A); law: PD_LAW_*; damping: viscous damping coefficient
 * (force density per velocity); dt: time step; du: load-pad displacement
 * increment per step (the pad is at u_z = -n du after step n); n_steps;
 * precision: PD_FP32 (FP32 bond work and Verlet state with compensated
 * accumulation; FP64 reaction) or PD_FP64; accumulate (FP32 only):
 * PD_ACC_KAHAN (compensated force sums and compensated u / vh updates), or
 * one of the accuracy ablations PD_ACC_PLAIN (neither), PD_ACC_STATE_ONLY
 * (compensated updates, plain force sums) and PD_ACC_FORCES_ONLY
 * (compensated force sums, plain updates); the last two take no
 * micromodulus field (PD_EINVAL); record_history: keep R^n for every step;
 * checkpoint_every: adjoint checkpoint interval (0 = library default). */
typedef struct {
    double E, rho, GF, s0, k, alpha;
    int32_t law;
    double damping, dt, du;
    int64_t n_steps;
    int32_t precision;
    int32_t accumulate;
    int32_t record_history;
    int32_t checkpoint_every;
} pd_params;

/* Sizes of a built mesh. */
typedef struct {
    int32_t nx, ny, nz;
    int64_t n_nodes;
    int64_t n_bonds;        /* unique bonds after the notch cut (0 before pd_build_bonds) */
    int64_t n_cut;          /* bonds removed by the notch */
    int32_t n_support, n_load;
    int32_t n_stencil;      /* neighbours of an interior node */
    double delta;           /* horizon */
} pd_mesh_info_t;

/* Build the lattice and the support / load node sets (host only).
 * Fails with PD_EINVAL if an extent is not a multiple of dx, the notch
 * position or depth is not a multiple of dx/2, or a node centre lies on a pad
 * face, or if the grid with its three ghost layers per face has more than
 * 2^27 cells (the step kernels address one sample's arrays with 32-bit byte
 * offsets: an FP64 displacement cell is 32 bytes).  *out receives a new
 * handle. */
PD_API int pd_build_mesh(const pd_mesh_desc *desc, pd_mesh *out);

/* Neighbourhoods |x' - x| <= delta (paper section 2.1, Eq. PD_Horizon) as a
 * fixed integer-offset stencil, the notch cut, and the upload of the mesh's
 * device tables.  Idempotent.  *n_bonds_out (nullable) receives the number
 * of unique bonds. */
PD_API int pd_build_bonds(pd_mesh m, int64_t *n_bonds_out);

PD_API int pd_mesh_get_info(pd_mesh m, pd_mesh_info_t *info);

/* Node ids of the support and load pads (host arrays of n_support / n_load
 * int32 entries, caller-owned; either may be NULL). */
PD_API int pd_mesh_get_pads(pd_mesh m, int32_t *support, int32_t *load);

/* Per-node material field for the single-sample entry points (pd_run,
 * pd_force_eval).  field: PD_FIELD_S0 (limit stretch), PD_FIELD_C
 * (micromodulus) or PD_FIELD_GF (fracture energy, N/m; the bond's critical
 * stretch then follows from the endpoint mean of G_F, appendix A).  values: [n_samples][n_nodes] of dtype
 * PD_DTYPE_F32/F64, on the device if on_device else on the host; the library
 * copies them on stream, checks them on the device and synchronises the
 * stream before it returns.  PD_EINVAL, with the old field kept, if a value
 * is not finite and positive.  A C field also sets the largest micromodulus
 * that pd_run's stability check (PD_EUNSTABLE) compares with dt.  values =
 * NULL clears the field (back to the homogeneous pd_params value).  Bond
 * values are endpoint means (s0_b = (s0_i + s0_j)/2, c_b and G_F,b
 * likewise).  pd_qoi_grad takes its s0 / c fields as arguments and uses the
 * homogeneous G_F. */
PD_API int pd_set_material_field(pd_mesh m, int32_t field, int64_t n_samples, const void *values,
                          int32_t on_device, int32_t dtype, void *stream);

/* One force evaluation on frozen displacement fields (section 2.1,
 * Eq. PD_EOM_Dynamic): L_i = sum_j c_b (1 - d_b) s_ij e_ij V with undamaged
 * bonds (d_b = 0).  u_host: [n_samples][n_nodes][3] displacements (m);
 * L_host: [n_samples][n_nodes][3] force densities (N/m^3).  Host buffers;
 * synchronous.  Uses the sample's s0 / c fields when set.  n_samples: 1 to
 * 65535, within the one-launch bound of pd_run_batch. */
PD_API int pd_force_eval(pd_mesh m, const pd_params *p, int64_t n_samples, const double *u_host,
                  double *L_host, void *stream);

/* One sample of the explicit solve (async).  Per step n = 0..N-1, on the
 * free degrees of freedom: v += (dt/2rho)(L - damping v); u += dt v; then
 * supports u_z = 0 and the load pad u_z = -(n+1) du; L = force(u) with the
 * irreversible damage history; v = (v + (dt/2rho) L) / (1 + damping dt/2rho);
 * R^{n+1} = -sum_{supports} L_z V; Q = max_n R^n (section 4 QoI: peak load).
 * *out receives a run handle; read it with pd_qoi / pd_run_state.  Returns
 * PD_EUNSTABLE, before enqueuing anything, when dt exceeds the explicit
 * stability limit of the largest micromodulus (the mesh's c field if set,
 * else the homogeneous value). */
PD_API int pd_run(pd_mesh m, const pd_params *p, void *stream, pd_run_h *out);

/* Peak reaction Q = max_n R^n (N; the peak load of the beam, section 4),
 * its first step n* (1-based) and optionally the reaction history
 * R[n_steps] (needs record_history).  Synchronises the run's stream.
 * Returns PD_ENONFINITE if the run went non-finite and PD_EUNSTABLE if its
 * micromodulus field exceeds what dt allows. */
PD_API int pd_qoi(pd_run_h r, double *peak, int64_t *peak_step, double *history);

/* Final displacement u (m, [n_nodes][3]) and, optionally, the damage history
 * kappa of every bond direction as the library stores it (largest stretch
 * seen, [122][n_nodes] FP64, 0 where the bond never passed its limit
 * stretch).  Host buffers; synchronises. */
PD_API int pd_run_state(pd_run_h r, double *u_out, double *kappa_out);

PD_API int pd_free_run(pd_run_h r);

/* A batch of independent samples over one or more meshes (levels): each
 * item steps all its samples with one launch per time step, and the items
 * run as parallel branches of a captured HIP graph that is replayed.  Items
 * whose dt is an integer multiple of the finest dt step on the matching
 * ticks (ratios up to an lcm of 4096).  Per item: s0 (device,
 * [n_samples][n_nodes], dtype = field_dtype, NULL = homogeneous p->s0),
 * c (micromodulus, device or NULL), gf (fracture energy in N/m, device or
 * NULL = homogeneous p->GF); outputs qoi (device FP64 [n_samples]), nstar (device
 * int64 [n_samples], nullable), status (device int32 [n_samples], nullable;
 * PD_OK, PD_ENONFINITE, PD_EUNSTABLE for a sample whose micromodulus
 * field exceeds what dt allows, or PD_EINVAL for one whose micromodulus
 * field has a value that is not positive), u_out (device FP64 [n_samples][n_nodes][3],
 * nullable: each sample's displacement after its last step, in metres).
 * These are the independent level-l solves of one MLMC sweep (section 3,
 * Eq. MLMC_estimator and Algorithm 1): each sample runs the explicit solve
 * of pd_run with its own fields.
 *
 * Asynchronous: the call validates the items, runs set-up (and, for a mesh
 * with no pinned or cached launch shape, the autotuner, which synchronises),
 * enqueues the whole solve on stream and returns.  The outputs are valid,
 * and the inputs may be released or overwritten, once the stream's work
 * enqueued so far has completed.  Work buffers come from the stream-ordered
 * allocator and are released in stream order; the captured graph is
 * destroyed by a later pd_run_batch or by pd_batch_sync.  On an error the
 * call synchronises the stream before it returns.  All items share
 * precision and accumulate.  The environment variable
 * PD_BATCH_SCHEDULE=tick replaces the per-item graph branches by one step
 * launch per tick over every item that steps at that tick (FP32
 * compensated 3D items with a common micromodulus mode, at most 4 of
 * them; other batches keep the branches); the results are the same bit for
 * bit.  n_samples per item: 1 to 65535, and at most as
 * many as one step launch over the mesh's tiles can hold (2^32 - 1
 * work-items for every launch shape); PD_EINVAL otherwise. */
typedef struct {
    pd_mesh mesh;
    const pd_params *params;
    int64_t n_samples;
    const void *s0;
    const void *c;
    const void *gf;
    int32_t field_dtype;
    double *qoi;
    int64_t *nstar;
    int32_t *status;
    double *u_out;
} pd_batch_item;

PD_API int pd_run_batch(const pd_batch_item *items, int32_t n_items, void *stream);

/* Waits for every pd_run_batch enqueued on stream and destroys their
 * graphs.  Calling it is optional: graphs of completed batches are also
 * destroyed by the next pd_run_batch call. */
PD_API int pd_batch_sync(void *stream);

/* pd_run_batch for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid allocation):
 * the same items, results bit-identical to pd_run_batch's, but every work
 * buffer of the solve (displacement, velocity and compensation state, damage
 * history and bits, padded fields, reaction partial sums; nstar and status
 * when the item leaves them NULL) is carved from one 256 MiB device array
 * that the library holds on each device it runs on until the process ends.
 * It calls no hipMalloc, hipFree or other allocating routine and captures
 * no graph: one step launch per item and time step on stream, items
 * interleaved on their common clock (dt integer multiples of the finest, no
 * lcm bound).  The launch shape is the mesh's pinned one, else the
 * autotuner's cached choice for the configuration, else the 16x4x4 brick;
 * it is never measured here.  Async: only enqueues on stream.  Every call
 * on a device shares that device's array, which keeps the last call's
 * contents (each call re-initialises what it uses): calls that overlap on
 * one device (other streams, other host threads) race and must be
 * serialised by the caller.  Fails with PD_EINVAL, before enqueuing
 * anything, when the items' work buffers exceed 256 MiB (about 110
 * level-0 samples or 15 level-1 samples of the beam), for more than 8
 * items, or for the same argument errors as pd_run_batch; with PD_ESTATE
 * when a mesh's tables are not on the device yet (pd_build_bonds uploads
 * them when a device is present). */
PD_API int pd_run_batch_static(const pd_batch_item *items, int32_t n_items, void *stream);

/* Launch-shape autotuner (no paper counterpart: it only changes how the
 * work of one time step is mapped onto the GPU).  Measures every shape that
 * the configuration (mesh dims, n_samples, p->precision, p->accumulate,
 * micromodulus field set or not) can use over a few time steps of a
 * throw-away solve with homogeneous fields, caches the fastest for the rest
 * of the process, and returns it in *shape_out; us_per_step_out (nullable,
 * host FP64 [PD_N_SHAPES]) receives each shape's time per step (-1 for shapes
 * the configuration cannot use).  FP64 has one shape (PD_SHAPE_GLOBAL_256).
 * pd_run and pd_run_batch tune a configuration the same way the first time
 * they meet it, unless the mesh has a pinned shape.  Synchronous on
 * stream; allocates a solve's buffers for the duration of the call. */
PD_API int pd_autotune(pd_mesh m, const pd_params *p, int64_t n_samples, void *stream, int32_t *shape_out,
                       double *us_per_step_out);

/* Pins the launch shape of every later run on this mesh (PD_SHAPE_AUTO
 * restores tuning).  Shapes a configuration cannot use fall back to one it
 * can (FP64: PD_SHAPE_GLOBAL_256; the ablations other than PD_ACC_KAHAN:
 * the 16x4x4 brick or the global shape).  Fails with PD_EINVAL for an unknown
 * shape. */
PD_API int pd_set_launch_shape(pd_mesh m, int32_t shape);

/* Gradient of the peak reaction Q = R^{n*} with respect to the per-node
 * limit-stretch field s0 and micromodulus field c, by a hand-written
 * discrete adjoint of the time loop with forward checkpoints every
 * p->checkpoint_every steps.  No counterpart in the paper, which samples Q
 * only (section 4); the forward pass is pd_run's solve, so Q and n* equal
 * pd_run's for the same fields.  PD_EUNSTABLE if c_dev exceeds what dt
 * allows.  s0_dev / c_dev: device FP64 [n_nodes]
 * (nullable: homogeneous values).  dq_ds0_dev, dq_dc_dev: device FP64
 * [n_nodes] outputs (either nullable).  *peak_out and *peak_step_out
 * (nullable) receive Q and n*.  Synchronous on stream. */
PD_API int pd_qoi_grad(pd_mesh m, const pd_params *p, const double *s0_dev, const double *c_dev,
                double *dq_ds0_dev, double *dq_dc_dev, double *peak_out, int64_t *peak_step_out,
                void *stream);

/* Karhunen-Loeve basis of a unit-variance Gaussian field with correlation
 * exp(-r^2 / (2 corr_len^2)) on the mesh's box (paper section 5, KL
 * expansion): the n_modes largest separable eigenpairs, from an n_quad-point
 * Gauss-Legendre Nystrom solve per axis, evaluated at the node centres and
 * uploaded (FP64).  Each 1D eigenfunction is signed positive at x = 0; equal
 * eigenvalue products (relative 1e-9) are ordered by their 1D indices. */
PD_API int pd_kl_build(pd_mesh m, double corr_len, int32_t n_modes, int32_t n_quad, pd_kl *out);

/* Eigenvalues of the selected modes (host FP64 [n_modes]). */
PD_API int pd_kl_eigenvalues(pd_kl kl, double *lam_out);

/* Lognormal field s0 = exp(mu + sigma g), g = sum_m sqrt(lambda_m) phi_m xi_m,
 * sigma^2 = ln(1 + cov^2), mu = ln(mean) - sigma^2 / 2.  xi_dev: device FP64
 * [n_samples][n_modes]; out_dev: device [n_samples][n_nodes] of out_dtype.
 * Async. */
PD_API int pd_kl_field(pd_kl kl, const double *xi_dev, int64_t n_samples, double mean, double cov,
                void *out_dev, int32_t out_dtype, void *stream);

PD_API int pd_kl_free(pd_kl kl);

/* Covariance families of a KL basis. */
enum { PD_COV_SQEXP = 0, PD_COV_EXP = 1 };

/* KL basis of the paper's exponential covariance exp(-|x - x'| / corr_len),
 * unit variance, Euclidean distance (section 5,
 * Eq. exponential_correlation_function), by Nystrom's method on the mesh's
 * own node centres with midpoint weights w = dx^3 (on a plane-stress mesh
 * the field is 2D: w = dx^2 and the centres are taken on the plane y = 0):
 * the largest eigenpairs of
 * w K from a dense symmetric eigensolver on the device, phi_k(x_j) =
 * psi_kj / sqrt(w).  Eigenvalues equal to 1e-8 (relative) form a cluster
 * whose basis is made canonical: the Gram-Schmidt orthonormalisation of the
 * projections of the probe vectors r_j(i) = cos((i + 1)(j + 1) 0.6180339887498949)
 * for j = 0, 1, ... (node order i); a single mode thus has <phi, r_0> > 0.
 * n_modes is extended to the end of a cluster it would split (read the
 * count with pd_kl_n_modes).  The mesh is the quadrature of every later
 * pd_kl_extend: build it on the coarsest level.  Limit: n_nodes <= 20000
 * (dense n^2 matrix).  Synchronous. */
PD_API int pd_kl_build_exp(pd_mesh m, double corr_len, int32_t n_modes, pd_kl *out);

/* The exponential basis kl evaluated at another mesh's node centres by the
 * Nystrom extension phi_k(x) = (1 / lambda_k) sum_j w rho(x, x_j) phi_k(x_j),
 * which reproduces the basis at the quadrature nodes, so every level sees
 * the same continuous field.  *out is a new handle for `target`.  Fails with
 * PD_EINVAL for a squared-exponential basis, and when one of the two meshes
 * is plane-stress and the other 3D.  Synchronous. */
PD_API int pd_kl_extend(pd_kl kl, pd_mesh target, pd_kl *out);

PD_API int pd_kl_n_modes(pd_kl kl, int32_t *n_modes_out);

/* Unit-variance Gaussian field g = sum_k sqrt(lambda_k) phi_k xi_k at the
 * basis' mesh nodes.  xi_dev: device FP64 [n_samples][n_modes]; g_dev: device
 * FP64 [n_samples][n_nodes].  Async. */
PD_API int pd_kl_gaussian(pd_kl kl, const double *xi_dev, int64_t n_samples, double *g_dev, void *stream);

/* The paper's material model (section 5 and section 6.2): the compressive
 * strength has a Weibull marginal of modulus weibull_m and mean fcm through
 * the Gaussian copula, f_c = lambda (-ln(1 - Phi(g)))^(1/m), lambda = fcm /
 * Gamma(1 + 1/m); E, f_t and G_F follow from the fib Model Code 2010
 * relations the paper cites: E = alpha_E 21.5 GPa (f_c / 10 MPa)^(1/3),
 * f_t = 0.3 MPa (f_ck / MPa)^(2/3) with f_ck = max(f_c - delta_f, fck_min),
 * G_F = 73 N/m (f_c / MPa)^0.18.  Per node: s0 = f_t / E, c = 12 E / (pi
 * delta^4) with the mesh's horizon (a plane mesh of thickness t:
 * c = 9 E / (pi t delta^3) in plane stress, 48 E / (5 pi t delta^3) in plane
 * strain, appendix A), G_F.  All in SI. */
typedef struct {
    double fcm;        /* mean compressive strength, Pa (paper: 42.3e6) */
    double weibull_m;  /* Weibull modulus (paper: 3) */
    double alpha_E;    /* aggregate factor of E (1 for quartzite) */
    double delta_f;    /* f_ck = f_c - delta_f (8e6 Pa) ... */
    double fck_min;    /* ... but at least fck_min (the relations need f_ck > 0) */
} pd_fib_params;

/* Per-node limit stretch, micromodulus and fracture energy from a Gaussian
 * field g_dev (device FP64 [n_samples][n_nodes]) into s0_out, c_out, gf_out
 * (device [n_samples][n_nodes] of out_dtype; any may be NULL).  Async. */
PD_API int pd_fib_fields(pd_mesh m, const double *g_dev, int64_t n_samples, const pd_fib_params *fp, void *s0_out,
                         void *c_out, void *gf_out, int32_t out_dtype, void *stream);

/* FP64 level sums of an MLMC level: Y = q_fine - q_coarse (q_coarse NULL:
 * Y = q_fine), sums_dev[0] = N, [1] = sum Y, [2] = sum Y^2 (device FP64,
 * overwritten).  Deterministic (fixed reduction order).  Async. */
PD_API int pd_level_stats(const double *q_fine_dev, const double *q_coarse_dev, int64_t n,
                   double *sums_dev, void *stream);

/* MLMC estimate from the level sums of pd_level_stats (paper section 4:
 * Eq. MC_estimator, Eq. sample_variance, Eq. MLMC_estimator, Eq. MLMC_error).
 * sums_dev: device FP64 [n_levels][3] = (N_l, sum Y_l, sum Y_l^2), level 0
 * first.  out_host: host FP64 [2 + 3 n_levels] = (estimate sum_l mean_l,
 * sampling variance sum_l V_l / N_l, then per level: mean_l, V_l with 1/N,
 * V_l with 1/(N-1)).  Synchronises stream. */
PD_API int pd_mlmc_estimate(const double *sums_dev, int32_t n_levels, double *out_host, void *stream);

/* Multilevel inverse CDF and CDF of the peak load (paper section 7, after
 * Gregory et al.): with R_l the ascending order statistics of the n_samples[l]
 * level-l fine samples q_fine_dev[l] and Rc_l those of their coarse partners
 * q_coarse_dev[l] (the level l-1 solves on the same random inputs; unused for
 * l = 0),
 *   F^-1(u) = R_0[ceil(N_0 u)] + sum_{l>=1} (R_l[ceil(N_l u)] - Rc_l[ceil(N_l u)])
 * (1-based, index clamped to 1..N_l), for each u_host[k] in (0, 1]
 * -> quantiles_host[k]; and the empirical CDF of those n_u values at the
 * n_x points x_host -> cdf_host (n_x = 0: skipped).  q_*_dev: host arrays of
 * n_levels device FP64 pointers (1 <= n_levels <= PD_MAX_CDF_LEVELS).  Ties
 * are ordered by input position.  Synchronises stream; allocates scratch. */
enum { PD_MAX_CDF_LEVELS = 8 };
PD_API int pd_mlmc_cdf(const double *const *q_fine_dev, const double *const *q_coarse_dev, const int64_t *n_samples,
                       int32_t n_levels, const double *u_host, int64_t n_u, double *quantiles_host,
                       const double *x_host, int64_t n_x, double *cdf_host, void *stream);

/* Optimal MLMC sample allocation (paper section 4.3, Eq. sample_allocation):
 * N_l = eps_s^-2 (sum_k sqrt(V_k C_k)) sqrt(V_l / C_l) for levels 0..n_levels-1,
 * the minimum-cost allocation whose sampling error sum_l V_l / N_l equals
 * eps_s^2.  V: level variances (>= 0), C: cost per sample (> 0), host FP64
 * [n_levels].  n_real_out (nullable): the real-valued N_l; n_out: N_l rounded
 * down, as in the paper's tables.  Host only. */
PD_API int pd_mlmc_allocation(const double *V, const double *C, int32_t n_levels, double eps_s, double *n_real_out,
                              int64_t *n_out);

/* Bias estimate of the finest level (paper section 4.3, Eq. bias_error):
 * |y_last_mean| / (r refinement^alpha - 1), where refinement is the growth of
 * the degrees of freedom per level (8 for a 3D lattice when dx halves) and
 * alpha the weak convergence rate.  Fails with PD_EINVAL unless
 * r refinement^alpha > 1.  Host only. */
PD_API int pd_mlmc_bias(double y_last_mean, double alpha, double refinement, double r, double *bias_out);

/* Least-squares fit of log|y| = intercept + slope log x over n >= 2 points
 * (host FP64 arrays; x > 0, y != 0): the convergence rates of section 4.2
 * (|E[Y_l]| ~ M_l^-alpha, V[Y_l] ~ M_l^-beta, C_l ~ M_l^gamma) are -slope,
 * -slope and slope of such fits.  intercept_out is nullable.  Host only. */
PD_API int pd_mlmc_fit_rate(const double *x, const double *y, int32_t n, double *slope_out, double *intercept_out);

PD_API int pd_free_mesh(pd_mesh m);

/* Message of the last failed call on this thread ("" if none). */
PD_API const char *pd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PD_H */
