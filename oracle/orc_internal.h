/* Internal structures of the FP64 oracle (test infrastructure). */
#ifndef PDFMC_ORC_INTERNAL_H
#define PDFMC_ORC_INTERNAL_H
#include "oracle.h"
#include <stddef.h>

/* counters, in this order on both the oracle and the GPU library */
enum {
    CNT_WALK_FALLBACK = 0, CNT_REFLECT = 1, CNT_PERIODIC = 2, CNT_OMEGA_FLIP = 3,
    CNT_EMPTY_NODE = 4, CNT_NAN = 5, CNT_WALK_STEPS = 6, CNT_CG_ER = 7,
    CNT_CG_P = 8, CNT_CG_FAIL = 9, CNT_K_FLOOR = 10, CNT_EPS_FLOOR = 11
};

/* field slots of the node-major Eulerian field array (R-06) */
enum {
    F_U1 = 0, F_U2, F_U3, F_DPX, F_DPY,
    F_DU1X, F_DU1Y, F_DU2X, F_DU2Y, F_DU3X, F_DU3Y,
    F_LAP1, F_LAP2, F_LAP3,
    F_G11, F_G12, F_G21, F_G22, F_G33,
    F_OMEGA, F_C0EPS, F_SOMEGA
};

typedef struct {
    int nn, ne, nbc;
    double *x, *y;         /* raw node coordinates */
    int *tri;              /* raw vertex ids */
    int *tag;              /* edge tags */
    orc_bc* bc;
    int *nbr;              /* neighbour element across edge k, or -1 */
    int *partner;          /* element across a periodic edge, or -1 */
    int nsn;               /* number of statistics nodes (periodic images merged) */
    int *snode;            /* raw node -> statistics node */
    int *rep;              /* statistics node -> its lowest raw node */
    int *tri_s;            /* statistics node ids per element vertex */
    double *rec;           /* per element: x1, y1, b0, b1, b2, c0, c1, c2 (R-05) */
    double *area;
    double *vol;           /* lumped node area, per statistics node */
    int *inc_ptr, *inc;    /* statistics node -> list of (3*e + k) */
    int *is_wall;          /* per statistics node */
    double *wnx, *wny;     /* unit wall normal per statistics node */
} omesh;

typedef struct {
    orc_params p;
    omesh m;
    int64_t np;
    double *x, *y, *u, *v, *w, *om, *wt, *psi;
    int32_t* elem; uint32_t* id; uint8_t* bin;
    double *F;       /* [nsn*ORC_NF] */
    double *Ffrz;    /* [nsn*ORC_NF] uploaded fields, for the frozen slots */
    uint32_t freeze; /* bit q: slot q keeps its uploaded value */
    double *stats;   /* [nsn*(12+2ns)] */
    double *sums;    /* [nsn*(11+2ns)] raw sums of the last statistics pass */
    double *cmean;   /* [ne*8*ns] */
    int32_t *ccount; /* [ne*8] */
    double *P;       /* mean pressure, per statistics node */
    double *gphi;    /* [nsn*2] its recovered gradient: the velocity correction of the next step (R-27) */
    int have_stats;
    int64_t cnt[ORC_NCOUNT];
} ocase;

struct orc_ctx {
    int ncase;
    ocase** cases;
    uint32_t step;
    int initialised;
    char err[512];
};

int  orc_err(orc_ctx* c, int code, const char* fmt, ...);
void* orc_alloc(size_t n);

/* mesh */
int  omesh_build(orc_ctx* c, omesh* m, const orc_mesh_desc* d);
void omesh_free(omesh* m);
void omesh_bary(const omesh* m, int e, double x, double y, double lam[3]);

/* rng */
void orc_uniforms(uint64_t seed, uint32_t id, uint32_t step, uint32_t stream, double u[6]);
void orc_init_uniforms(uint64_t seed, uint32_t id, uint32_t stream, double u[10]);

/* locate */
int  orc_walk_case(ocase* cs, int e0, double* x, double* y, double u3[3]);
int  orc_brute(const omesh* m, double x, double y);

/* model */
int  orc_case_init(orc_ctx* c, ocase* cs);
int  orc_case_step(orc_ctx* c, ocase* cs, uint32_t n);
int  orc_case_rebin(ocase* cs);
int  orc_node_moments(ocase* cs);
int  orc_derive_fields(orc_ctx* c, ocase* cs, int project);
void orc_relax_node(const orc_params* P, const double R[3][3], const double dU[3][3], double K, double E,
                    double nx, double ny, double r[5], double dval[5], double* L2, double* Av_out);
void orc_recover_grad(const omesh* m, const double* f, double* gx, double* gy);
void orc_recover_lap(const omesh* m, const double* gx, const double* gy, double* lap);

/* fem */
int  orc_helmholtz(const omesh* m, const double* L2, const double* r, const int* dmask,
                   const double* dval, double tol, int maxit, double* s, int* iters);
int  orc_projection(const omesh* m, const double* U1, const double* U2, double dt,
                    double tol, int maxit, double* phi, int* iters);
#endif
