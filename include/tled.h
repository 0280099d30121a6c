/*
 * tled.h -- C-ABI of the MI355X coupled thermo-visco-hyperelastic TLED +
 * explicit Pennes bioheat solver (Zhang, Lay, Roberts, Chauhan,
 * arXiv 2009.10400).
 *
 * One time step of the method (Section 4, Eqs. 12-28):
 *   per element: F from nodal displacements and precomputed dh/dX (Eq. 17);
 *     thermal split F = F_el F_th with F_th = lambda I (Eqs. 7-8, 11);
 *     fibre-reinforced neo-Hookean stress on the elastic part (Eq. 9,
 *     Table 5 model) pulled back to the reference configuration (Eq. 10);
 *     Prony relaxation (recursion after Eq. 27); nodal forces V0 F S dh/dX
 *     (Eqs. 24-26, 28); pulled-back conduction loads (Eqs. 16, 18-19);
 *   per node: forward Euler on temperature (Eq. 20) and central difference
 *     with mass-proportional damping on displacement (Eqs. 22, 27).
 *
 * Conventions
 *   - Units are SI; temperatures in kelvin.
 *   - Host inputs are double arrays, row-major ("n x 3" = x,y,z per row).
 *     The library copies every input at call time; the caller keeps
 *     ownership of its buffers.  Device state is single precision and owned
 *     by the library (allocated at tled_finalize through the allocator set
 *     with tled_set_allocator, else hipMalloc, and freed by tled_destroy).
 *   - Node and element numbers are those of the caller; the library may
 *     reorder internally and undoes it on every read.
 *   - Every call returns a tled_status; nothing aborts and no C++ exception
 *     crosses the boundary.  tled_last_error() gives the message of the last
 *     failure on a handle.
 *   - tled_step is asynchronous on the library's stream; errors raised on the
 *     device (non-finite values, inverted elements) surface as
 *     TLED_E_UNSTABLE at the next tled_sync, read or monitor call.
 *   - A handle is not thread-safe; calls on one handle must be serialised.
 */
#ifndef TLED_H
#define TLED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TLED_OK = 0,
    TLED_E_ARG = -1,          /* bad argument (null pointer, size, range)          */
    TLED_E_MESH = -2,         /* degenerate or inverted element, bad connectivity  */
    TLED_E_STATE = -3,        /* call out of order (e.g. step before finalize)     */
    TLED_E_HIP = -4,          /* HIP runtime error                                 */
    TLED_E_OOM = -5,          /* host or device allocation failed                  */
    TLED_E_UNSTABLE = -6,     /* device raised non-finite values or J <= 0         */
    TLED_E_UNSUPPORTED = -7   /* option not available on this build                */
} tled_status;

typedef struct tled_sim tled_sim;

/* Element types: the value is the number of nodes per element. */
enum { TLED_T4 = 4, TLED_H8 = 8 };

/* Bits of tled_monitors.flags. */
enum { TLED_FLAG_NONFINITE = 1u, TLED_FLAG_INVERTED = 2u };

/*
 * Material and load parameters (Tables 1 and 5).
 * Strain energy Psi = mu/2 (I1bar - 3) + eta/2 (I4bar - 1)^2 + kappa/2 (J - 1)^2
 * (Table 5) evaluated on the elastic deformation.  Thermal stretch
 * lambda = 1 + alpha (T - T0) (Section 3.2, after Eq. 11).
 */
typedef struct {
    double rho;          /* reference density, kg/m^3                                  */
    double mu;           /* shear modulus at T0, Pa                                    */
    double kappa;        /* bulk modulus, Pa                                           */
    double eta;          /* fibre coefficient eta_a, Pa (0: isotropic neo-Hookean)    */
    double alpha;        /* thermal expansion coefficient, 1/K                         */
    double alpha_m;      /* expansion along the fibre m = a0 when expan_mode = 1 or 2  */
    double alpha_n;      /* expansion along the second axis n when expan_mode = 2      */
    double T0;           /* stress-free reference and initial temperature, K          */
    double k;            /* thermal conductivity, W/(m K)                              */
    double k_m;          /* conductivity along the fibre when cond_mode = 1            */
    double c;            /* specific heat capacity, J/(kg K)                           */
    double wbcb;         /* blood perfusion w_b c_b, W/(m^3 K)                         */
    double T_art;        /* arterial blood temperature, K                              */
    double Q_met;        /* metabolic heat generation, W/m^3                           */
    double g[4];         /* Prony relative moduli phi_i (sum < 1)                      */
    double tau[4];       /* Prony relaxation times, s                                  */
    double muT_lo, muT_hi, muT_drop;           /* mu, eta scaled by 1 - drop * clamp((T - lo)/(hi - lo)) */
    double shrink_T, shrink_width, shrink_eps; /* lambda scaled by 1 + eps * clamp((T - shrink_T)/width)  */
    double ckT_lo, ckT_hi, c_hi, k_hi;         /* c(T), k(T) linear from (lo: c, k) to (hi: c_hi, k_hi) */
    double hg_coef;      /* H8 hourglass coefficient (stiffness hg_coef (kappa + 4 mu/3) V0 sum|dh/dX|^2 / 8) */
    int32_t n_prony;     /* 0..4                                                       */
    int32_t expan_mode;  /* Eq. 11.  0: F_th = lambda I; 1: lambda I + (lambda_m - lambda) m m
                            (transversely isotropic, m = a0); 2: orthotropic,
                            lambda I + (lambda_m - lambda) m m + (lambda_n - lambda) n n, with n
                            from tled_set_expansion_axes                                  */
    int32_t cond_mode;   /* Eqs. 15-16.  0: D = k I; 1: D = k I + (k_m - k) a0 a0; 2: per-element
                            tensor from tled_set_conductivity (times k(T)/k with ckT_on)  */
    int32_t muT_on;      /* 1: temperature-dependent mu and eta                        */
    int32_t shrink_on;   /* 1: shrinkage factor on lambda                             */
    int32_t ckT_on;      /* 1: temperature-dependent c (per node) and k (per element)  */
} tled_material;

/* Execution options (all optional; zero fields keep the defaults). */
typedef struct {
    int32_t graph_steps;      /* steps per chunk: a chunk is one hipGraph replay (default 50;
                                 < 0: eager launches in chunks of 100).  Monitors are reduced
                                 at the last step of every chunk and of every tled_step call.
                                 Batches default to eager steps, each of which launches only
                                 the scenarios still running; a batch's graph launches those
                                 running at its first step and is captured again when that
                                 set has changed.                                             */
    int32_t kernel_variant;   /* 0: default (2 for T4, 3 for H8); 1: two-pass element/node
                                 kernels with precomputed geometry; 2: fused patch kernels
                                 rebuilding the geometry from patch-local coordinates; 3: fused
                                 patch kernels reading the precomputed geometry               */
    int32_t reorder;          /* 0: auto (= 1); 1: elements along a Morton curve of their
                                 centroids, and for the fused variants patches cut by recursive
                                 coordinate bisection; 2: Morton order, patches are runs of it;
                                 -1: keep the caller's order (patches are runs of it)          */
    int32_t block_size;       /* threads per workgroup of the fused patch kernel: 0 (256),
                                 256, or 512 (single T4 problems only)                        */
    int32_t patch_elems;      /* elements per patch for the fused variant.  0: H8 256; T4 at
                                 most 504 (704 with block_size 512), sized so the patch count
                                 just fills whole rounds of the 1024 (512) workgroups that are
                                 resident at once on 256 CUs, at least 128                     */
    double  ablation_T;       /* threshold of the ablated-volume monitor, K (0: 333.15 K)     */
    int32_t batch_schedule;   /* batches only, set before finalize.  0: each step launches the
                                 patches of the scenarios still running, counted on the host
                                 (eager steps, or hipGraph chunks captured again whenever that
                                 set changes); 1: persistent: the patch kernel runs with the
                                 workgroups that are resident at once, which walk the step's
                                 patches (each XCD's workgroups an eighth of them), and the
                                 running scenarios are counted on the device from the step
                                 counter, so one captured chunk of graph_steps steps (default
                                 100) serves the whole batch                                             */
    int32_t shared_update;    /* set before finalize.  How the nodes shared between patches are
                                 advanced (Eqs. 20 and 27 on their summed patch partials):
                                 0: default (= 2); 1: inside the next step's patch kernel:
                                 every patch holding a shared node sums its partials and
                                 advances it while staging, the patch that wrote its first
                                 partial stores it, and one shared-node kernel ends each chunk
                                 (single problems with kernel_variant 2, 256-thread workgroups
                                 and neither the orthotropic expansion nor the tensor
                                 conduction; elsewhere as 2); 2: a shared-node kernel after
                                 every step's patch kernel.  The fields are the same bits
                                 either way                                                   */
} tled_options;

typedef struct {
    int64_t step;            /* steps completed since tled_finalize                          */
    double  t;               /* simulated time = step * dt, s                                 */
    double  kinetic;         /* 1/2 sum_a M_a |v_a|^2 with v at the half step, J              */
    double  strain;          /* sum_e V0 det(F_th) Psi (+ H8 hourglass energy), J             */
    double  T_max;           /* max nodal temperature, K                                      */
    double  T_min;           /* min nodal temperature, K                                      */
    double  ablated_volume;  /* lumped volume of nodes with T >= ablation_T, m^3              */
    uint32_t flags;          /* TLED_FLAG_* raised since finalize                            */
    uint32_t reserved;
} tled_monitors;

typedef struct {
    int64_t n_nodes, n_elems;
    int32_t elem_type;
    int32_t n_prony;
    int64_t n_swapped;       /* T4 elements repaired by swapping their last two nodes         */
    int32_t kernel_variant;  /* variant in use after finalize                                 */
    int32_t n_patches;       /* fused variant: number of element patches                     */
    int64_t n_shared_nodes;  /* fused variant: nodes assembled across patches                */
    int32_t patch_max_nodes; /* fused variant: largest number of nodes of one patch           */
    int32_t patch_lds_bytes; /* fused variant: dynamic LDS per workgroup                      */
    int64_t device_bytes;    /* device memory held by the handle                              */
    double  dt, dt_critical;
    int32_t patch_wgs_per_cu; /* fused variant on a device: resident patch workgroups per CU  */
    int32_t shared_update;   /* fused variant with shared nodes: 1 advanced inside the next
                                step's patch kernel, 2 by a kernel of their own each step (see
                                tled_options.shared_update); else 0                           */
    double  dt_thermal;      /* explicit thermal stability bound (Gershgorin, reference
                                geometry, largest k and smallest c the material reaches);
                                finalize refuses a dt above it                             */
} tled_info;

/* --- lifetime ----------------------------------------------------------
 * tled_create: device >= 0 selects a GPU ordinal; device = -1 creates a
 * host-only handle that supports set-up, tled_critical_dt, tled_get_lumped and
 * tled_finalize (precompute only) but no stepping (TLED_E_STATE).           */
tled_status tled_create(tled_sim **out, int device);
void        tled_destroy(tled_sim *sim);

/* Optional device allocator: alloc(bytes, ctx) returns device memory or NULL;
 * release(ptr, ctx) frees it.  Must be set before tled_finalize. */
tled_status tled_set_allocator(tled_sim *sim, void *(*alloc)(size_t, void *),
                               void (*release)(void *, void *), void *ctx);
/* Stream (hipStream_t) used for every launch and copy; NULL = the null stream.
 * Must be set before tled_finalize. */
tled_status tled_set_stream(tled_sim *sim, void *hip_stream);
tled_status tled_set_options(tled_sim *sim, const tled_options *opt);

/* --- problem definition (before tled_finalize) --------------------------
 * Mesh (Section 4.1, low-order elements): elem_type TLED_T4 or TLED_H8;
 * X n_nodes x 3 reference coordinates; conn n_elems x elem_type node indices
 * (0-based).  H8 local order (xi,eta,zeta) = (---),(+--),(++-),(-+-),(--+),
 * (+-+),(+++),(-++).  T4 elements of negative volume are repaired by swapping
 * their last two nodes (counted in tled_info.n_swapped); a zero-volume T4 or
 * an H8 with det J0 <= 0 makes tled_finalize fail with TLED_E_MESH. */
tled_status tled_set_mesh(tled_sim *sim, int elem_type, int64_t n_nodes, const double *X,
                          int64_t n_elems, const int32_t *conn);
tled_status tled_set_material(tled_sim *sim, const tled_material *m);
/* Fibre directions a0, n_elems x 3, normalised inside (Table 5: unit vector a0).
 * Default: (1, 0, 0) for every element. */
tled_status tled_set_fibres(tled_sim *sim, const double *a0);
/* Second axis n of the orthotropic thermal expansion (Eq. 11, expan_mode 2),
 * n_elems x 3.  Made orthonormal to the element's fibre m = a0 inside (its
 * component along m is removed, then it is normalised); tled_finalize fails
 * with TLED_E_ARG when expan_mode is 2 and no axes were given, or when an n is
 * parallel to its m.  NULL clears.  Single problems only (a batch refuses
 * expan_mode 2 with TLED_E_UNSUPPORTED). */
tled_status tled_set_expansion_axes(tled_sim *sim, const double *n0);
/* Element conductivity tensors D of Eq. 15 (cond_mode 2), n_elems x 6 in the
 * order xx yy zz xy yz xz, W/(m K).  Used as given (fixed in space), pulled
 * back with the total deformation as J F^-1 D F^-T (Eq. 16), and scaled by
 * k(T)/k when ckT_on is set.  tled_finalize fails with TLED_E_ARG when
 * cond_mode is 2 and no tensors were given.  NULL clears.  Single problems
 * only (a batch refuses cond_mode 2 with TLED_E_UNSUPPORTED). */
tled_status tled_set_conductivity(tled_sim *sim, const double *D);
/* Fixed displacement components (the essential boundary condition of
 * Section 6.1's verification model, whose right face is held in position): node[i] with
 * mask[i] bits 0..2 = x, y, z.  Fixed components stay at zero displacement.
 * Repeated calls accumulate. */
tled_status tled_set_fixed_dofs(tled_sim *sim, int64_t n, const int32_t *node, const uint8_t *mask);
/* Fixed temperatures: node[i] held at T[i] (K), the essential boundary
 * condition of the Pennes equation (Eq. 1).  The paper's own cases use none:
 * their exterior is adiabatic (Section 6.1, Table 5), which is what every
 * boundary without a fixed temperature gets here. */
tled_status tled_set_fixed_temperature(tled_sim *sim, int64_t n, const int32_t *node, const double *T);
/* Regional heat source Q_r (Eq. 1) per element, W/m^3, lumped to nodes with the
 * reference volume V0/npe; active while t_on <= step*dt < t_off. */
tled_status tled_set_heat_source(tled_sim *sim, const double *q_elem, double t_on, double t_off);
/* Time step dt (s) and mass-proportional damping coefficient gamma (1/s),
 * D = gamma M (Eq. 21).  tled_finalize fails with TLED_E_ARG if dt exceeds
 * the critical step. */
tled_status tled_set_time(tled_sim *sim, double dt, double damping_gamma);
/* Critical time step of the explicit central difference (the stability limit
 * that Section 7 discusses for the time step): min_e L_e / c_d, with
 * c_d = sqrt((kappa + 4 mu/3 + 4 eta)/rho) and L_e = 3 V0 / A_max (T4) or
 * V0 / A_max (H8).  Needs mesh and material. */
tled_status tled_critical_dt(tled_sim *sim, double *dt_cr);

/* Precompute (FP64 on the host: dh/dX, V0, lumped M, C, K_b, Q), reorder,
 * build the assembly lists, round to FP32 and upload.  Initial state:
 * u = v = 0, T = T0 (fixed-T nodes at their value), Prony state 0. */
tled_status tled_finalize(tled_sim *sim);

/* --- stepping -----------------------------------------------------------
 * tled_step advances n_steps time steps of Section 4's loop (element physics,
 * assembly, Eq. 20 and Eq. 27 node updates), asynchronously on the library's
 * stream, in hipGraph chunks (tled_options.graph_steps).  Monitors are
 * reduced at the last step of every chunk. */
tled_status tled_step(tled_sim *sim, int64_t n_steps);
/* Captures and instantiates, without running anything, the hipGraphs that a
 * following tled_step(sim, n_steps) replays: the chunk of graph_steps steps and
 * a shorter last chunk.  A last chunk shorter than graph_steps is otherwise
 * enqueued as eager launches unless a graph of its length is already cached
 * (up to 8 graphs are kept per handle, least recently used first out).  For a
 * batch only the graphs at the current step are captured (its graphs depend
 * on the scenarios still running).  Set-up work for callers that time or
 * repeat tled_step calls of one length. */
tled_status tled_prepare_steps(tled_sim *sim, int64_t n_steps);
/* Wait for the stream and report device-raised errors (non-finite values or
 * det F <= 0, which the explicit scheme of Section 4 produces when dt is too
 * large or an element inverts). */
tled_status tled_sync(tled_sim *sim);

/* --- outputs (synchronous; caller numbering) ----------------------------- */
tled_status tled_read_u(tled_sim *sim, double *u /* n_nodes x 3 */);
tled_status tled_read_T(tled_sim *sim, double *T /* n_nodes, K */);
/* Device-to-device copy of the fields in caller numbering, FP32:
 * u_dst n_nodes x 3, T_dst n_nodes (K).  Either pointer may be NULL.
 * Asynchronous on the library's stream. */
tled_status tled_copy_fields_device(tled_sim *sim, float *u_dst, float *T_dst);
tled_status tled_get_monitors(tled_sim *sim, tled_monitors *out);
tled_status tled_get_info(tled_sim *sim, tled_info *out);
/* Lumped host-precomputed quantities in caller numbering (any may be NULL):
 * reference volume, mass, heat capacity (at T0), perfusion, metabolic and source loads. */
tled_status tled_get_lumped(tled_sim *sim, double *Vl, double *M, double *C, double *Kb,
                            double *Qm, double *Qr);

/* --- thermal dose ---------------------------------------------------------
 * Section 7 names thermal-damage models as the clinical measures of an
 * ablation besides an isotherm (the 60 C ablated-volume monitor above).  With
 * tled_set_thermal_dose (single problems, before tled_finalize) every step adds,
 * per node and at the temperature T the step ends at (K; T_C = T - 273.15):
 *   CEM43 (Sapareto and Dewey), equivalent minutes at 43 C:
 *     (dt / 60) R^(43 - T_C), R = 0.5 for T_C >= 43 and 0.25 below;
 *   the Arrhenius damage integral (Henriques and Moritz):
 *     dt A exp(-Ea / (R_gas T)), R_gas = 8.314462618 J/(mol K),
 * with the caller's frequency factor A (1/s; 0 leaves the integral at zero)
 * and activation energy Ea (J/mol).  Both sums are held in FP64 on the device
 * and updated by a kernel of their own after each step (the shared nodes are
 * then advanced by their own kernel every step, whatever shared_update asks);
 * they are part of the opaque state.  TLED_E_UNSUPPORTED on batch handles,
 * TLED_E_ARG for negative or non-finite parameters.
 * tled_read_thermal_dose: both sums in caller numbering, n_nodes each (either
 * pointer may be NULL); TLED_E_STATE when the dose was not enabled. */
tled_status tled_set_thermal_dose(tled_sim *sim, double arrhenius_A, double arrhenius_Ea);
tled_status tled_read_thermal_dose(tled_sim *sim, double *cem43_min, double *omega);

/* --- state --------------------------------------------------------------
 * Typed state in caller numbering: u n_nodes x 3 (m), v n_nodes x 3 velocity
 * at the last half step (m/s), T n_nodes (K), theta n_elems x n_prony x 6
 * Prony state (xx, yy, zz, xy, yz, xz; Pa), step.  Any array may be NULL on
 * read; on write NULL leaves that part unchanged. */
tled_status tled_read_state(tled_sim *sim, double *u, double *v, double *T, double *theta,
                            int64_t *step);
tled_status tled_write_state(tled_sim *sim, const double *u, const double *v, const double *T,
                             const double *theta, int64_t step);
/* Opaque bitwise checkpoint of the device state (restoring it and stepping
 * reproduces the uninterrupted run bit for bit). */
tled_status tled_state_size(tled_sim *sim, size_t *bytes);
tled_status tled_get_state(tled_sim *sim, void *buf);
tled_status tled_set_state(tled_sim *sim, const void *buf);

/* --- measurement ---------------------------------------------------------
 * Runs n_steps eagerly on the library's stream with a HIP event pair taken by
 * the dispatch of every element and node launch (hipExtLaunchKernelGGL; the
 * monitor reduction by a pair of recorded events) and returns the mean
 * duration (ms) per launch of each kernel kind: ms[0] element (or fused patch)
 * kernel, ms[1] node (or shared-node) kernel, ms[2] monitor reduction.
 * Advances the state like tled_step. */
tled_status tled_kernel_times(tled_sim *sim, int64_t n_steps, double ms[3]);

/* --- batched scenarios (planning sweeps) ----------------------------------
 * Many independent problems of one element type and one Prony term count run
 * together: every step of the fused kernels advances all of them, each with its
 * own mesh, material, fibres, source, fixed dofs, dt and damping; a scenario
 * stops after its own n_steps and holds its state while the others go on.
 * A batch handle is created by tled_batch_create and destroyed by
 * tled_batch_destroy; tled_set_stream, tled_set_options, tled_step, tled_sync,
 * tled_get_monitors (sums and extrema over all scenarios), tled_get_state,
 * tled_set_state, tled_kernel_times, tled_get_info and tled_last_error accept
 * it; the single-problem set-up and read calls refuse it (TLED_E_STATE). */
typedef struct tled_sim tled_batch;

typedef struct {
    int32_t n_scenarios;
    int32_t n_patches;
    int64_t n_elems, n_nodes;
    int64_t n_shared_nodes;
    int64_t max_steps;       /* largest n_steps of the scenarios */
    int64_t step;            /* batch steps taken                */
    int64_t device_bytes;
    int32_t kernel_variant;
    int32_t reserved;
} tled_batch_info;

tled_status tled_batch_create(tled_batch **out, int device);
void        tled_batch_destroy(tled_batch *b);
/* Add one scenario (arguments as in the single-problem set-up calls; arrays are
 * copied).  n_fixed nodes fixed_nodes[i] with component mask fixed_mask[i];
 * patch_elems 0 = default (T4 448, H8 256; the single-problem rule for whole
 * rounds of resident workgroups does not apply to a batch's union of patches).
 * A scenario's results are bitwise those of the same problem run alone with the
 * same patch_elems.  *index receives the scenario number. */
tled_status tled_batch_add(tled_batch *b, int elem_type, int64_t n_nodes, const double *X, int64_t n_elems,
                           const int32_t *conn, const tled_material *m, const double *a0, const double *q_elem,
                           double t_on, double t_off, int64_t n_fixed, const int32_t *fixed_nodes,
                           const uint8_t *fixed_mask, double dt, double damping_gamma, int64_t n_steps,
                           int32_t patch_elems, int32_t *index);
/* Let finalize choose scenario's time step and step count: dt = cfl times the
 * scenario's critical step (0 < cfl <= 1), n_steps = max(1, round(t_end / dt)).
 * The dt (may then be 0) and n_steps given to tled_batch_add are replaced. */
tled_status tled_batch_set_duration(tled_batch *b, int32_t scenario, double cfl, double t_end);
tled_status tled_batch_finalize(tled_batch *b);
/* After finalize: the time step and step count of one scenario. */
tled_status tled_batch_scenario_steps(tled_batch *b, int32_t scenario, double *dt, int64_t *n_steps);
/* Enqueue steps until every scenario has reached its n_steps (asynchronous). */
tled_status tled_batch_run(tled_batch *b);
/* Displacement (n_nodes x 3) and temperature (n_nodes, K) of one scenario in its
 * caller numbering; either pointer may be NULL. */
tled_status tled_batch_read(tled_batch *b, int32_t scenario, double *u, double *T);
/* Every scenario's displacement and temperature at once (one device-to-host
 * copy), concatenated in the order the scenarios were added, each in its
 * caller numbering: u (sum of n_nodes) x 3, T sum of n_nodes.  Either may be NULL. */
tled_status tled_batch_read_all(tled_batch *b, double *u, double *T);
/* Per scenario: maximum nodal temperature and lumped volume of the nodes at or
 * above ablation_T (e.g. 333.15 K, the 60 C isotherm). */
tled_status tled_batch_monitors(tled_batch *b, double ablation_T, double *T_max, double *ablated_volume);
tled_status tled_batch_get_info(tled_batch *b, tled_batch_info *out);

/* --- measurement ---------------------------------------------------------
 * Plain streaming copy of `bytes` (a multiple of 16; both pointers 16-byte
 * aligned device memory of GPU `device`) on `hip_stream` (NULL: the default
 * stream): the reference bandwidth that the solver's HBM throughput is quoted
 * against, and a kernel of known traffic for calibrating hardware counters.
 * Asynchronous; TLED_E_ARG for a bad size or alignment. */
tled_status tled_stream_copy(int device, void *dst, const void *src, size_t bytes, void *hip_stream);

const char *tled_status_string(tled_status s);
const char *tled_last_error(const tled_sim *sim);

#ifdef __cplusplus
}
#endif
#endif /* TLED_H */
