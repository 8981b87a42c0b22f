/*
 * oracle.h -- plain, slow, single-threaded FP64 CPU implementation of the
 * particle advance of the non-hybrid joint velocity-frequency-scalar PDF
 * method (Bakosi, Franzese & Boybeyi, arXiv:1006.0549).
 *
 * THIS IS TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it. It shares no source with the
 * GPU library; both implement the same written contract from the paper:
 *
 *   position SDE            Eq.(2)
 *   GLM velocity SDE        Eq.(4)   (same Wiener increment as Eq.(2), Sec. II)
 *   frequency SDE           Eq.(5) with the source Eq.(6)
 *   IECM micromixing        Eq.(9)
 *   forward Euler, grid statistics, pressure projection   Sec. II, last paragraph
 *   grid roles (i) statistics, (ii) Eulerian solves, (iii) tracking   Sec. I
 *
 * Every point the paper leaves open is fixed by a numbered reading (R-nn),
 * listed in the design notes of the repository and restated where used.
 *
 * Pins (CPU tests, each tied to something other than this code): the
 * generator (rocRAND's Philox, libm, distributions), the initial ensemble
 * against the distributions it draws from, location against brute
 * force, the boundary conditions against their closed forms, the SDEs against
 * Ornstein-Uhlenbeck, Gamma and SLM-decay recurrences, interpolation through
 * a frozen linear mean velocity, mixing invariants and its clamp, the
 * estimator against partition of unity and brute force, recovery and the
 * FEM solves against exact and manufactured solutions, production and
 * S_omega under homogeneous shear, and the elliptic-relaxation source (its
 * production part under simple shear, A_v and length-scale limits,
 * isotropic part, wall values, G_ij and C0 eps) against hand-derived closed
 * forms, and the freeze mask against the frozen-field mode.
 *
 * Parity unpinned: the fully coupled model over many steps (relaxation and
 * projection feeding back into the particles). The paper prints no numbers
 * for it (its figures are not part of the text), so beyond the pins of each
 * part its output is tied to the GPU path only.
 *
 * Ownership: every pointer argument is borrowed for the duration of the call.
 * Errors: functions return 0 on success and a positive code otherwise; the
 * message is available from orc_last_error(). Nothing aborts.
 */
#ifndef PDFMC_ORACLE_H
#define PDFMC_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_E_INVALID = 1, ORC_E_MESH = 2, ORC_E_STATE = 5 };
enum { ORC_BC_WALL = 0, ORC_BC_PERIODIC = 1 };
/* modes: 0 = every Eulerian field frozen at the uploaded values,
 *        1 = simplified Langevin model (G from <omega>), frozen pressure gradient,
 *        2 = elliptic relaxation for G_ij + pressure projection (R-19, R-27) */
enum { ORC_MODE_FROZEN = 0, ORC_MODE_SLM = 1, ORC_MODE_ER = 2 };

#define ORC_NF 22      /* Eulerian fields per node (R-06 field list) */
#define ORC_MAXS 4     /* scalars per case */
#define ORC_NCOUNT 12

typedef struct {
    int32_t type;        /* ORC_BC_WALL or ORC_BC_PERIODIC */
    double u_wall[3];    /* wall velocity (wall only) */
    double shift[2];     /* translation to the partner edge (periodic only) */
} orc_bc;

typedef struct {
    int32_t n_nodes; const double* xy;     /* [2*n_nodes] interleaved */
    int32_t n_elems; const int32_t* tri;   /* [3*n_elems], counter-clockwise */
    const int32_t* edge_tag;               /* [3*n_elems]; edge k is opposite vertex k;
                                              -1 interior, else index into bc[] */
    int32_t n_bc; const orc_bc* bc;
} orc_mesh_desc;

typedef struct {
    int32_t mode;
    double dt, nu;
    double C0, C3, C4, Cw1, Cw2, Cphi;            /* R-20, R-22, R-24 */
    double C1, C2, gamma5, Cv, CL, Ceta;          /* R-19 */
    double dpdx[2];      /* frozen (mode 1) or driving (mode 2) mean pressure gradient */
    int32_t n_scalars, n_bins, n_min;             /* R-23 */
    double src[ORC_MAXS][4];   /* per scalar: cx, cy, r, value; r <= 0 = no source (R-26) */
    double k_floor, eps_floor;                    /* R-18 */
    double cg_rtol; int32_t cg_maxit;             /* R-28 */
    uint64_t seed; uint32_t stream;               /* R-09 key and counter word 2 */
    double n_eff_min;    /* R-34: least effective sample size of a node estimate */
    int32_t reaction;    /* R-35: closed chemistry S_alpha(psi) of Eq.(8)-(9):
                            0 none; 1 first-order decay S_a = -k_a psi_a;
                            2 A + B -> P on scalars 0, 1, 2 at the rate
                              k_0 psi_0 psi_1 (further scalars inert) */
    double k_react[ORC_MAXS];   /* rate constants, >= 0 */
    int32_t rebin;       /* R-36: 1 = the velocity bins and cell means are formed
                            again against the new fields at the end of a step */
} orc_params;

typedef struct {
    int64_t n;
    double *x, *y, *u, *v, *w, *omega, *weight;
    double* psi;          /* [n_scalars*n], scalar-major */
    int32_t* elem;        /* case-local element index */
    uint32_t* id;         /* RNG identity (R-32) */
    uint8_t* bin;         /* IECM velocity bin (R-23) */
} orc_particles;

typedef struct orc_ctx orc_ctx;

orc_ctx*    orc_create(void);
void        orc_destroy(orc_ctx* c);
const char* orc_last_error(const orc_ctx* c);

int orc_add_case(orc_ctx* c, const orc_mesh_desc* m, const orc_params* p, int32_t* case_id);
int orc_mesh_info(orc_ctx* c, int32_t cs, int32_t* n_stat_nodes, int32_t* stat_node /*[n_nodes]*/,
                  int32_t* nbr /*[3*ne] or NULL*/, double* rec /*[8*ne] or NULL*/,
                  double* vol /*[n_nodes] or NULL*/);
int orc_particles_upload(orc_ctx* c, int32_t cs, const orc_particles* p);
/* Initial ensemble of a case (R-29, R-30, R-31, R-32): ppe particles per
 * element, particle i in element i / ppe with id i, drawn from the case's
 * generator with purpose 1 (counter (id, 0, stream, 256 + block), blocks
 * 0..4, uniforms u_0..u_9):
 *   position uniform in the element: s = sqrt(u_0), lambda = (1 - s,
 *     s (1 - u_1), s u_1), X = (lambda_0 x_0 + lambda_1 x_1) + lambda_2 x_2;
 *   velocity U_i = u_std g_i with Box-Muller Gaussians g_0, g_1 from
 *     (u_2, u_3) and g_2 from (u_4, u_5);
 *   frequency Gamma(4, omega_scale): omega = -omega_scale (((ln u_6 +
 *     ln u_7) + ln u_8) + ln u_9);
 *   scalar a = disk[a][3] inside its disk (centre disk[a][0..1], radius
 *     disk[a][2] > 0), else 0; mass weight A_e / ppe; bin 0. */
typedef struct {
    double u_std, omega_scale;
    double disk[ORC_MAXS][4];
} orc_init_params;
int orc_particles_init(orc_ctx* c, int32_t cs, int32_t ppe, const orc_init_params* ip);
int orc_particles_download(orc_ctx* c, int32_t cs, orc_particles* p);
/* F: [n_nodes*ORC_NF], node-major, per raw node (periodic images must agree).
 * Bit q of freeze_mask keeps slot q at the uploaded value whenever the
 * fields are derived from the statistics (applied after the whole
 * derivation, so the other slots see the derived values). */
int orc_fields_upload(orc_ctx* c, int32_t cs, const double* F, uint32_t freeze_mask);
int orc_fields_download(orc_ctx* c, int32_t cs, double* F);
/* P: [n_nodes] mean pressure per raw node; sets <P> and the velocity
 * correction -dt grad <P> that the next step applies (R-27) */
int orc_pressure_upload(orc_ctx* c, int32_t cs, const double* P);
int orc_pressure_download(orc_ctx* c, int32_t cs, double* P /*[n_nodes]*/);
/* initialisation pass: statistics of the uploaded state, Eulerian fields
 * (except in mode 0), velocity bins and cell means */
int orc_init(orc_ctx* c);
/* only the bins + cell means of the current state against the current fields */
int orc_rebin(orc_ctx* c);
int orc_step(orc_ctx* c, int32_t n_steps);
int orc_set_step_index(orc_ctx* c, uint32_t n);
/* statistics per raw node: [n_nodes*(12+2*n_s)]:
 * W, rho, <U1..3>, <u1u1>,<u2u2>,<u3u3>,<u1u2>,<u1u3>,<u2u3>, <omega>, <psi_a>.., <psi_a'^2>.. */
int orc_stats(orc_ctx* c, int32_t cs, double* out);
/* raw node sums sum_p w N_n(X_p) Q_p per raw node: [n_nodes*(11+2n_s)]:
 * 1, U1..3, U1U1,U2U2,U3U3,U1U2,U1U3,U2U3, omega, psi_a.., psi_a^2.. */
int orc_node_sums(orc_ctx* c, int32_t cs, double* out);
/* cell means [n_elems*8*n_s] and cell counts [n_elems*8] */
int orc_cell_means(orc_ctx* c, int32_t cs, double* mean, int32_t* count);
int orc_counters(orc_ctx* c, int32_t cs, int64_t* out /*[ORC_NCOUNT]*/);

/* ---- individual steps, exported so that tests can pin them ---- */
void   orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_ln(double u);
void   orc_sincos2pi(double u, double* s, double* c);
void   orc_gauss6(uint64_t seed, uint32_t id, uint32_t step, uint32_t stream, double xi[6]);
void   orc_uniform6(uint64_t seed, uint32_t id, uint32_t step, uint32_t stream, double u[6]);
/* barycentric coordinates of (x,y) in element e of a case (R-05) */
int orc_bary(orc_ctx* c, int32_t cs, int32_t e, double x, double y, double lam[3]);
/* brute-force location (R-13): lowest-index element with min(lam) >= 0, else -1 */
int32_t orc_locate_brute(orc_ctx* c, int32_t cs, double x, double y);
/* the walk of R-12..R-15 from element e0; updates x,y,u (3 comps); returns element */
int32_t orc_walk(orc_ctx* c, int32_t cs, int32_t e0, double* x, double* y, double* u3);
/* recovered nodal gradient and Laplacian of a nodal field f (per raw node), R-16 */
int orc_recover(orc_ctx* c, int32_t cs, const double* f, double* gx, double* gy, double* lap);
/* Galerkin P1 solve of (M + K_L) s = M r with nodal L^2 and nodal r (per raw
 * node); Dirichlet values dval where dmask != 0. tol: relative residual. */
int orc_fem_helmholtz(orc_ctx* c, int32_t cs, const double* L2, const double* r,
                      const int32_t* dmask, const double* dval, double tol, double* s);
/* P1 projection solve: int grad N . grad phi = (1/dt) int grad N . U, zero mean */
int orc_fem_projection(orc_ctx* c, int32_t cs, const double* U1, const double* U2,
                       double dt, double tol, double* phi);

/* ---- test hooks of the Eulerian side ---- */
/* overwrite the node statistics (per raw node, the layout of orc_stats) */
int orc_set_stats(orc_ctx* c, int32_t cs, const double* stats);
/* derive the Eulerian fields from the current node statistics (R-16..R-20,
 * R-19 relaxation, and with project != 0 the projection of R-27) */
int orc_derive(orc_ctx* c, int32_t cs, int32_t project);
/* the elliptic-relaxation source of R-19 at one node:
 * stress = <u1u1>,<u2u2>,<u3u3>,<u1u2>,<u1u3>,<u2u3>; grad = d<U_i>/dx_j,
 * i-major, j = x, y; k and eps as used (floored); n = wall normal.
 * Out: r and dval for the components 11, 12, 21, 22, 33, L^2 and A_v. */
int orc_relax_source(const orc_params* p, const double stress[6], const double grad[6], double k, double eps,
                     const double n[2], double r[5], double dval[5], double* L2, double* Av);

#ifdef __cplusplus
}
#endif
#endif
