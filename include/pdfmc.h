/*
 * pdfmc.h -- C ABI of the MI355X particle-advance library for the non-hybrid
 * joint velocity-frequency-scalar PDF method of Bakosi, Franzese & Boybeyi
 * (arXiv:1006.0549).
 *
 * What a time step computes (Sec. II, last paragraph: forward Euler; Eulerian
 * statistics estimated on the grid and evaluated at the particles; the mean
 * pressure from a projection on the grid):
 *   - particle tracking on the unstructured grid (Sec. I, grid role (iii)) with
 *     no-slip imposed on particles at walls and periodic edges,
 *   - the position SDE, Eq.(2), and the generalized Langevin velocity SDE,
 *     Eq.(4), driven by the same Wiener increment dW_i,
 *   - the turbulent-frequency SDE, Eq.(5), with the source S_omega of Eq.(6),
 *   - IECM micromixing of the scalars, Eq.(9), plus concentrated sources,
 *   - the shape-weighted statistics at gridpoints (Sec. I, grid role (i)),
 *   - the Eulerian fields: recovered gradients, the elliptic-relaxation G_ij
 *     (Sec. II, after Eq.(4)) and the pressure projection (grid role (ii)).
 * The points the paper leaves open are fixed by numbered readings (R-nn)
 * that this library and its test oracle implement alike.
 *
 * Conventions for every call:
 *  - Returns PDFMC_OK or an error code; pdfmc_last_error() gives the message.
 *    Nothing aborts or throws across this boundary.
 *  - Host pointers are borrowed for the duration of the call only.
 *  - Device memory: the library never allocates. pdfmc_workspace_query()
 *    returns the size of one device buffer that the caller allocates and
 *    binds with pdfmc_workspace_bind(); it stays owned by the caller and must
 *    outlive the context (or the next bind).
 *  - All device work is enqueued on the caller's HIP stream given at
 *    pdfmc_create(); calls that return host data synchronise that stream.
 *  - A context is used by one host thread at a time.
 */
#ifndef PDFMC_H
#define PDFMC_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdfmc_ctx pdfmc_ctx;

typedef enum {
    PDFMC_OK = 0,
    PDFMC_E_INVALID = 1,      /* bad argument */
    PDFMC_E_MESH = 2,         /* mesh rejected (orientation, manifoldness, periodic matching) */
    PDFMC_E_NOMEM = 3,        /* bound workspace too small */
    PDFMC_E_HIP = 4,          /* a HIP call failed */
    PDFMC_E_STATE = 5,        /* call out of order (e.g. step before bind/init) */
    PDFMC_E_UNSUPPORTED = 6
} pdfmc_status;

typedef enum { PDFMC_FP64 = 0, PDFMC_FP32 = 1 } pdfmc_precision;
typedef enum { PDFMC_BC_WALL = 0, PDFMC_BC_PERIODIC = 1 } pdfmc_bc_type;
/* 0: Eulerian fields frozen at the uploaded values;
 * 1: simplified Langevin model, G_ij = -(1/2 + 3/4 C0)<omega> delta_ij, frozen
 *    mean pressure gradient (R-20);
 * 2: elliptic relaxation for G_ij and pressure projection (R-19, R-27). */
typedef enum { PDFMC_MODE_FROZEN = 0, PDFMC_MODE_SLM = 1, PDFMC_MODE_ER = 2 } pdfmc_mode;

#define PDFMC_NF 22        /* Eulerian field slots per node (R-06)          */
#define PDFMC_MAX_SCALARS 4
#define PDFMC_N_COUNTERS 13

typedef struct {
    int32_t type;          /* pdfmc_bc_type                                  */
    double u_wall[3];      /* wall velocity (walls)                          */
    double shift[2];       /* translation onto the partner edge (periodic)   */
} pdfmc_bc;

typedef struct {
    int32_t n_nodes;  const double* xy;        /* [2*n_nodes] interleaved x,y      */
    int32_t n_elems;  const int32_t* tri;      /* [3*n_elems] counter-clockwise;
                                                  n_elems < 2^23 per case        */
    const int32_t* edge_tag;  /* [3*n_elems]; edge k is opposite vertex k;
                                 -1 interior, else an index into bc[]           */
    int32_t n_bc;     const pdfmc_bc* bc;
} pdfmc_mesh_desc;

typedef struct {
    int32_t mode;                                  /* pdfmc_mode                 */
    double dt, nu;                                 /* time step, viscosity (rho=1) */
    double C0, C3, C4, Cw1, Cw2, Cphi;             /* Eq.(4),(5),(6); R-24        */
    double C1, C2, gamma5, Cv, CL, Ceta;           /* elliptic relaxation, R-19   */
    double dpdx[2];        /* mode 1: frozen d<P>/dx_j; mode 2: driving gradient */
    int32_t n_scalars;     /* 0..PDFMC_MAX_SCALARS                              */
    int32_t n_bins;        /* 1 (IEM limit) or 8 velocity octants, R-23          */
    int32_t n_min;         /* smaller cells pool into a residual cell, R-23      */
    double src[PDFMC_MAX_SCALARS][4];  /* cx, cy, r, value; r <= 0: none, R-26   */
    double k_floor, eps_floor;                     /* R-18                        */
    double cg_rtol; int32_t cg_maxit;              /* R-28                        */
    uint64_t seed; uint32_t stream;                /* RNG key and stream, R-09    */
    double n_eff_min;    /* least effective sample size W^2/sum (w N)^2 of a
                            node estimate; below it the node keeps its previous
                            moments (R-34) */
    int32_t reaction;    /* closed scalar source S(psi) of Eq.(8)-(9), R-35:
                            0 none; 1 first-order decay S_a = -k_a psi_a;
                            2 A + B -> P on scalars 0, 1, 2 at the rate
                              k_0 psi_0 psi_1 (needs n_scalars >= 3)        */
    double k_react[PDFMC_MAX_SCALARS];  /* rate constants, finite and >= 0    */
    int32_t rebin;       /* velocity bins of IECM, Eq.(9) (variant R-36 of R-23):
                            0 formed against the fields of the step that moved
                            the particle; 1 formed again, with the cell means,
                            against the new fields at the end of the step (one
                            more particle pass per step)                    */
} pdfmc_case_params;

/* Particle ensemble on the host, structure of arrays, always FP64 here (the
 * FP32 context converts on upload/download). psi is [n_scalars*n],
 * scalar-major. elem is the case-local element holding (x, y); id is the
 * RNG identity (R-32); bin may be NULL on upload. */
typedef struct {
    int64_t n;
    double *x, *y, *u, *v, *w, *omega, *weight, *psi;
    int32_t* elem;
    uint32_t* id;
    uint8_t* bin;
} pdfmc_particles_host;

/* Context on the caller's stream (a hipStream_t, NULL = default stream). */
pdfmc_status pdfmc_create(pdfmc_ctx** out, int32_t precision, void* hip_stream);
void         pdfmc_destroy(pdfmc_ctx* ctx);
const char*  pdfmc_last_error(const pdfmc_ctx* ctx);   /* valid until the next call */

/* Mesh upload (Sec. I: the unstructured grid) and case settings. The mesh is
 * validated and its tables derived on the host (neighbours, periodic
 * partners, merged periodic nodes, element records of R-05). capacity is the
 * largest particle count the case will hold. Must precede workspace_query. */
pdfmc_status pdfmc_add_case(pdfmc_ctx* ctx, const pdfmc_mesh_desc* mesh, const pdfmc_case_params* params,
                            int64_t capacity, int32_t* case_id);
/* Statistics nodes of a case (periodic images merged, R-33): count and the
 * map raw node -> statistics node (may be NULL). */
pdfmc_status pdfmc_case_info(pdfmc_ctx* ctx, int32_t case_id, int32_t* n_stat_nodes, int32_t* stat_node);

/* Device workspace: size in bytes (alignment 256) for all cases added so far;
 * bind uploads the mesh tables into it (asynchronously on the stream). */
pdfmc_status pdfmc_workspace_query(pdfmc_ctx* ctx, uint64_t* bytes);
pdfmc_status pdfmc_workspace_bind(pdfmc_ctx* ctx, void* dev_ptr, uint64_t bytes);

/* Particle ensemble (Sec. II, closing paragraph: the flow is represented by
 * a large number of particles carrying position, velocity, frequency and
 * compositions). Upload copies an ensemble from the host (n <= capacity);
 * the whole ensemble is checked before any device work, and an element id
 * outside the case, a non-finite x, y, U, omega, weight or scalar, or a
 * weight that is not positive gives PDFMC_E_INVALID (these checks need no
 * bound workspace; the copy itself then needs one, PDFMC_E_STATE before).
 * The particle counters restart at 0. Particles keep their id (the RNG
 * identity of R-32) across sorts. */
pdfmc_status pdfmc_particles_upload(pdfmc_ctx* ctx, int32_t case_id, const pdfmc_particles_host* p);

/* Initial ensemble drawn on the device (readings R-29..R-32 of the paper's
 * unstated initial conditions): ppe particles per element, particle i in
 * element i / ppe with id i, its draws from the case's Philox generator with
 * purpose 1 (counter (id, 0, stream, 256 + block), blocks 0..4, uniforms
 * u_0..u_9 formed as for the Wiener increments):
 *   position uniform in the element: s = sqrt(u_0), lambda = (1 - s,
 *     s (1 - u_1), s u_1), X = (lambda_0 x_0 + lambda_1 x_1) + lambda_2 x_2;
 *   velocity U_i = u_std g_i, Box-Muller Gaussians g_0, g_1 from (u_2, u_3)
 *     and g_2 from (u_4, u_5);
 *   frequency Gamma(4, omega_scale): -omega_scale (sum of ln u_6..u_9);
 *   scalar a = disk[a][3] inside its disk (centre disk[a][0..1], radius
 *     disk[a][2] > 0), else 0; mass weight A_e / ppe (R-31); bin 0.
 * Computed in FP64 in either precision (an FP32 context stores the rounded
 * values). Errors: PDFMC_E_INVALID for ppe < 1, ne * ppe above the case's
 * capacity, u_std < 0, omega_scale <= 0 or non-finite values; PDFMC_E_STATE
 * before a workspace is bound. Synchronises the stream; counters restart. */
typedef struct {
    double u_std;                       /* velocity standard deviation per component */
    double omega_scale;                 /* scale of the Gamma(4, scale) frequency     */
    double disk[PDFMC_MAX_SCALARS][4];  /* cx, cy, r, value; r <= 0: no disk          */
} pdfmc_init_params;
pdfmc_status pdfmc_particles_init(pdfmc_ctx* ctx, int32_t case_id, int32_t ppe, const pdfmc_init_params* p);
pdfmc_status pdfmc_particles_download(pdfmc_ctx* ctx, int32_t case_id, pdfmc_particles_host* p);

/* The Eulerian fields evaluated at the particles (Sec. II, after Eq.(3):
 * the mean fields on the right-hand sides of Eqs.(4), (5) and (9) are
 * evaluated at the particle positions; reading R-06 lists them), per raw
 * node, [n_nodes*PDFMC_NF] node-major, slots:
 * 0-2 <U_i>; 3-4 d<P>/dx_j; 5-10 d<U_i>/dx_j (i-major); 11-13 lap <U_i>;
 * 14-18 G11,G12,G21,G22,G33; 19 <omega>; 20 C0 eps; 21 S_omega.
 * Upload copies them in (periodic images take the value of the image with
 * the lowest raw index); every value must be finite (PDFMC_E_INVALID). Bit q
 * of freeze_mask keeps slot q of this case at the uploaded value in the
 * fields the particles see, also in modes 1 and 2 where the step derives
 * the fields from the statistics (the other fields of the same step are
 * derived from the computed values); mode 0 freezes every slot anyway.
 * Bits above slot 21: PDFMC_E_INVALID. Synchronises the stream. */
pdfmc_status pdfmc_fields_upload(pdfmc_ctx* ctx, int32_t case_id, const double* F, uint32_t freeze_mask);
/* The fields in force, same layout as the upload; synchronises the stream. */
pdfmc_status pdfmc_fields_download(pdfmc_ctx* ctx, int32_t case_id, double* F);
/* The mean pressure <P> per raw node (Sec. II, closing paragraph: the mean
 * pressure of Eq.(4) from the projection on the grid, reading R-27: the
 * potential phi of the last projection, whose recovered gradient corrects
 * the particle velocities at the start of the next step; in mode 2 the
 * field slots d<P>/dx_j then hold the driving gradient alone). 0 in modes 0
 * and 1, and before the first step. Synchronises the stream. */
pdfmc_status pdfmc_pressure_download(pdfmc_ctx* ctx, int32_t case_id, double* P);

/* Initialisation pass over every case (the state the first forward-Euler
 * step of Sec. II starts from): grid statistics of the uploaded or drawn
 * ensemble (Sec. I, grid role (i)), the Eulerian fields derived from them
 * (not in mode 0), velocity bins and cell means of IECM (Eq.(9), R-23).
 * PDFMC_E_STATE before a workspace is bound. Synchronises the stream. */
pdfmc_status pdfmc_init(pdfmc_ctx* ctx);
/* Only recompute the velocity bins and cell means of Eq.(9) (R-23) against
 * the fields in force (after a fields upload). Synchronises the stream. */
pdfmc_status pdfmc_rebin(pdfmc_ctx* ctx);
/* Advance every case by n_steps time steps (asynchronous on the stream).
 * One step is the forward-Euler step of Sec. II, closing paragraph: the
 * particle SDEs Eqs.(2), (4), (5), (9) with tracking and boundary
 * conditions, then the grid statistics of the new state (Sec. I, role (i)),
 * then the Eulerian fields, relaxation and projection (role (ii)); the
 * order is reading R-08. stage_mask selects stages (tests isolate kernels
 * with it; PDFMC_STAGE_ALL is the method's step):
 *   PDFMC_STAGE_ADVANCE  the particle increments, walk and sources; without
 *                        it the particles stay where they are
 *   PDFMC_STAGE_STATS    node statistics and cell means of the new state;
 *                        without it they keep their values
 *   PDFMC_STAGE_FIELDS   the Eulerian fields from the statistics; without it
 *                        they keep their values
 * The step index (R-09) advances in every case. Reports launch failures
 * only; anomalies inside a step are counted (pdfmc_counters). Errors:
 * PDFMC_E_INVALID for n_steps < 0 or unknown stage bits, PDFMC_E_STATE
 * before init. */
#define PDFMC_STAGE_ADVANCE 1u
#define PDFMC_STAGE_STATS 2u
#define PDFMC_STAGE_FIELDS 4u
#define PDFMC_STAGE_ALL 7u
pdfmc_status pdfmc_step(pdfmc_ctx* ctx, int32_t n_steps, uint32_t stage_mask);
/* Time-step index that enters the RNG counter (R-09): a restart that sets
 * the index and uploads particles and fields continues the same sample
 * path. Synchronises the stream. */
pdfmc_status pdfmc_set_step_index(pdfmc_ctx* ctx, uint32_t n);

/* Statistics readback (Sec. I, grid role (i): Eulerian statistics extracted
 * at the gridpoints; estimator of reading R-11, thin-node rule R-34), per
 * raw node: [n_nodes*(12+2*n_scalars)]:
 * W, rho, <U_1..3>, <u1u1>,<u2u2>,<u3u3>,<u1u2>,<u1u3>,<u2u3>, <omega>,
 * <psi_a> (n_scalars), <psi_a'^2> (n_scalars). Synchronises the stream. */
pdfmc_status pdfmc_stats_readback(pdfmc_ctx* ctx, int32_t case_id, double* out);
/* Raw weighted node sums of the last statistics pass, [n_nodes*(12+2*n_s)]:
 * sum_p w N_n(X_p) Q_p for Q = 1, U_1..3, U1U1,U2U2,U3U3,U1U2,U1U3,U2U3,
 * omega, psi_a, psi_a^2, then sum_p (w N_n(X_p))^2 (for the effective
 * sample size of R-34). */
pdfmc_status pdfmc_node_sums(pdfmc_ctx* ctx, int32_t case_id, double* out);
/* Cell means of the IECM conditional mean, [n_elems*8*n_s], and cell
 * particle counts [n_elems*8] (either pointer may be NULL). */
pdfmc_status pdfmc_cell_means(pdfmc_ctx* ctx, int32_t case_id, double* mean, int32_t* count);
/* Counters since upload or initial draw (the failure detection around the
 * readings the paper leaves open: R-13 walk fallback, R-14 reflections,
 * R-15 periodic crossings, R-21 frequency sign flips, R-34 thin nodes,
 * R-18 floors, R-28 solver iterations), [PDFMC_N_COUNTERS]: walk fallbacks, reflections,
 * periodic crossings, omega sign flips, empty nodes, non-finite particles,
 * walk steps, ER CG iterations, projection CG iterations, CG failures,
 * k floor hits, eps floor hits, scatter overflows (a workgroup's element sums
 * that found no record slot, belong to an element with more than 256
 * records in the pass or found the pass's overflow list full, and were added
 * with FP64 atomics instead: while this
 * counter is 0, every statistic is summed in a fixed order and a step repeats
 * bit for bit). The five relaxation components of a case
 * are solved as one system with five right-hand sides: its iterations count
 * once per component (the iterations until every component converged). */
pdfmc_status pdfmc_counters(pdfmc_ctx* ctx, int32_t case_id, int64_t* out);

/* Execution options: re-sort the particles by element every sort_interval
 * steps (0 = never), particle-kernel block size (64, 128 or 256: a divisor of
 * the 256-particle tile, so that a workgroup never spans two cases),
 * capture the step sequence into a HIP graph (0/1; needs a non-NULL stream,
 * else PDFMC_E_INVALID). */
pdfmc_status pdfmc_set_options(pdfmc_ctx* ctx, int32_t sort_interval, int32_t block_size, int32_t use_graph);
/* Eulerian solver options (the FP64 multigrid-preconditioned CG of the
 * elliptic relaxation and the projection, reading R-28 of the step contract;
 * the relaxation's five components share their matrix and run as one system
 * with five right-hand sides, each with its own Krylov sequence).
 * Every step runs `iterations` CG iterations as row-parallel phase kernels
 * over all systems of all cases (a system that has converged skips the rest
 * at once), then completes any system that needs more in one workgroup per
 * system. iterations = 0 (the default) adapts the count to what the previous
 * steps needed (read back asynchronously every 8 steps and applied two steps
 * later, so the count changes at the same steps in every run): each system
 * hands over to the one-workgroup completion at an iteration set from its
 * own solves, and the phases are unrolled for the system that needs the
 * most. Multigrid levels with more than tail_rows unknowns (default
 * 64) are processed by the row-parallel phases, smaller ones by one
 * workgroup per system. Results do not depend on either option beyond FP64
 * summation order. Every scalar of the CG is summed in a fixed order (the
 * row-parallel workgroups' shares, then the system's shares in block order),
 * so the solves repeat bit for bit, and a case's solution does not depend on
 * the other cases of the context (its hand-over iteration and the lanes per
 * entry of its coarse operators come from its own systems). Errors: PDFMC_E_INVALID for iterations
 * outside 0..100000 or tail_rows < 0. */
pdfmc_status pdfmc_set_solver(pdfmc_ctx* ctx, int32_t iterations, int32_t tail_rows);
/* Current unrolled iteration count and number of row-parallel levels
 * (either pointer may be NULL). */
pdfmc_status pdfmc_solver_info(pdfmc_ctx* ctx, int32_t* iterations, int32_t* large_levels);

/* Projection solver (the mean-pressure projection, reading R-27). The
 * projection matrix of a case is constant for the whole run, so by default
 * pdfmc_add_case factors it once on the host (nested dissection by
 * coordinate bisection, supernodal Cholesky with statistics node 0
 * decoupled, FP64) and every projection is two sweeps over the factor on the
 * GPU, followed by removing the mean: the same solution as the iterative
 * solve, to rounding. PDFMC_PROJ_PCG solves it with the multigrid PCG of the
 * relaxation instead. The factor is used only when every mode-2 case has one
 * (a case whose factor has a supernode or reach above 2048 unknowns has
 * none). Results do not depend on the choice beyond the solver tolerance.
 * The sweeps apply the updates of an unknown from the supernodes below it in
 * a fixed (supernode) order and split each supernode's sums by its own size,
 * so a projection repeats bit for bit and a case's projection does not
 * depend on the other cases of the context.
 * Errors: PDFMC_E_INVALID for another method. */
typedef enum { PDFMC_PROJ_DIRECT = 0, PDFMC_PROJ_PCG = 1 } pdfmc_projection_method;
pdfmc_status pdfmc_set_projection_solver(pdfmc_ctx* ctx, int32_t method);
/* Method in effect (or that would be, before binding), height of the tallest
 * supernode tree (-1: no factor) and FP64 values stored in all factors
 * (any pointer may be NULL). */
pdfmc_status pdfmc_projection_info(pdfmc_ctx* ctx, int32_t* method, int32_t* height, int64_t* factor_values);
/* Autotuner of the batched step (what the step's cost depends on besides the
 * workload): times real steps of the bound workload for each trial setting
 * and keeps the fastest, by coordinate descent over
 *   particle-kernel block size   64, 128, 256
 *   sort interval                1, 2, 5, 10, 20 steps
 *   multigrid tail threshold     0, 64, 256, 512, 1024, 2048 rows (pdfmc_set_solver)
 * Each trial runs one untimed step, then max(steps_per_trial, a multiple of
 * the sort interval) timed steps. The trial steps advance the simulation
 * exactly like pdfmc_step (the results do not depend on the settings beyond
 * FP64 summation order). Fills *out (may be NULL) with the chosen settings
 * and their time per step. Errors: PDFMC_E_STATE before init or while live
 * timing is enabled, PDFMC_E_INVALID for steps_per_trial outside 1..1000. */
typedef struct {
    int32_t block_size, sort_interval, tail_rows;
    int32_t trials, steps;       /* trial settings timed, time steps advanced */
    double ms_per_step;
} pdfmc_tune_result;
pdfmc_status pdfmc_autotune(pdfmc_ctx* ctx, int32_t steps_per_trial, pdfmc_tune_result* out);
/* Sort the particles of every case by element, and inside an element by id,
 * now. The order is a layout choice only: the particles keep their ids, which
 * fix their random draws (R-32), so a sorted run takes the same path as an
 * unsorted one. The temporaries live in the workspace. Synchronises the
 * stream. PDFMC_E_STATE before a workspace is bound. */
pdfmc_status pdfmc_sort(pdfmc_ctx* ctx);
/* pdfmc_sort without allocating and without synchronising: for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, hosts that forbid hipMalloc). The same kernels with the same result
 * as pdfmc_sort, asynchronous on the context's stream; the temporaries live
 * in a static device array of PDFMC_SORT_NOALLOC_BYTES, one per device, held
 * until the process ends. Its address is looked up when a workspace is bound,
 * for the device current at pdfmc_workspace_bind. The sort needs
 * 32 NE + 20 NP + 8 (NE / 1024 + 1) bytes plus at most 2.5 KiB of alignment
 * (NE elements, NP particle slots: every case's capacity rounded up to 256);
 * beyond PDFMC_SORT_NOALLOC_BYTES: PDFMC_E_INVALID (use pdfmc_sort).
 * Every call on one device shares the array and finds the last call's
 * contents (the counts are cleared by the call itself): calls that overlap
 * on one device (two streams, contexts or threads) race and give wrong
 * orders, so serialise them. PDFMC_E_STATE before a workspace is bound;
 * PDFMC_E_HIP if the array's address could not be looked up. */
#define PDFMC_SORT_NOALLOC_BYTES (32u << 20)
pdfmc_status pdfmc_sort_noalloc(pdfmc_ctx* ctx);
pdfmc_status pdfmc_synchronize(pdfmc_ctx* ctx);

/* Live timing of the particle kernel: while enabled, every time-step launch
 * of the particle kernel is bracketed by two HIP events on the context's
 * stream (graph replay is suspended meanwhile). timing_read synchronises,
 * returns the summed kernel time in ms and the number of launches since the
 * last read or enable, and restarts the count. */
pdfmc_status pdfmc_timing(pdfmc_ctx* ctx, int32_t enable);
pdfmc_status pdfmc_timing_read(pdfmc_ctx* ctx, double* total_ms, int64_t* launches);

/* Device-side draws of the Wiener increments for n particles (test hook of
 * R-09/R-10): ids, out are DEVICE pointers; out is [6*n] (FP64 context:
 * doubles; FP32 context: floats), increment j of particle i at out[6*i+j]. */
pdfmc_status pdfmc_draw_gaussians(pdfmc_ctx* ctx, uint64_t seed, uint32_t step, uint32_t stream,
                                  const uint32_t* ids, int64_t n, void* out);

#ifdef __cplusplus
}
#endif
#endif
