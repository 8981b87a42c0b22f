// C ABI of the particle-advance library: contexts, cases, the caller-owned
// device workspace, uploads/readbacks and the step sequence.
//
// One step (reading R-08), every case in each launch:
//   clear accumulators -> particle kernel (advance + statistics + cell sums)
//   -> node statistics -> cell means -> recovered gradients -> derived fields
//   -> [elliptic relaxation: assemble, 5 CG solves, G_ij/C0 eps]
//   -> [projection: right-hand side, CG, <P> update, recovered grad <P>]
//   -> FP32 mirror of the fields -> step index + 1.
// The sequence can be captured once into a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pdfmc.h"
#include "pdfmc_amg.h"
#include "pdfmc_chol.h"
#include "pdfmc_kernels.h"
#include "pdfmc_mesh.h"

using namespace pdfmc;

// The sort's temporaries for pdfmc_sort_noalloc, which allocates nothing.
// Each device holds its own copy for the life of the process. In host code
// this name is only a stand-in for the symbol: kernels and fills get the
// device address looked up by static_scratch_address.
static __device__ __align__(256) unsigned char scratch[PDFMC_SORT_NOALLOC_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;      // by device ordinal; nullptr until looked up

// The device address of `scratch` on device `dev`, looked up once per
// device with that device current (the caller's current device is restored).
hipError_t static_scratch_address(int dev, void** out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0) return hipErrorInvalidDevice;
    if ((int)g_scratch_addr.size() <= dev) g_scratch_addr.resize(dev + 1, nullptr);
    if (!g_scratch_addr[dev]) {
        int prev = -1;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void* ptr = nullptr;
        e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (prev != dev) {
            const hipError_t e2 = hipSetDevice(prev);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_addr[dev] = ptr;
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

// ELL forms of one hierarchy: A on levels >= 1, P and R on every level but
// the coarsest, and the Galerkin lists with ELL source/destination positions.
struct HierEll {
    std::vector<EllH> A, P, R;
    std::vector<std::vector<int>> gptr, gidx, gdst;
    std::vector<std::vector<double>> gcoef;
};

// Offsets of one hierarchy's arrays inside the flat int/double regions.
struct HierOff {
    int64_t Acol[AMG_MAXL], Aval[AMG_MAXL], Pcol[AMG_MAXL], Pval[AMG_MAXL], Rcol[AMG_MAXL], Rval[AMG_MAXL];
    int64_t Alen[AMG_MAXL], Plen[AMG_MAXL], Rlen[AMG_MAXL];   // entries per row (padding after them)
    int64_t Gptr[AMG_MAXL], Gidx[AMG_MAXL], Gdst[AMG_MAXL], Gcoef[AMG_MAXL];
};

struct Case {
    pdfmc_case_params p{};
    MeshHost m;
    int64_t cap = 0, np = 0;
    int64_t poff = 0, psioff = 0, cmoff = 0, csoff = 0, inc_off = 0;
    int eoff = 0, noff = 0, bcoff = 0;
    int64_t rec_off = 0;          // scatter records (doubles)
    int rec_stride = 0;
    uint32_t freeze = 0;          // field slots kept at their uploaded values
    // Galerkin matrix pattern of the case in ELL form (mode 2)
    EllH ell0;
    int64_t ell_off = 0;
    // multigrid hierarchies of the two Eulerian solves (mode 2): 0 elliptic
    // relaxation (wall rows isolated), 1 projection
    bool has_amg = false;
    AmgH amg[2];
    HierEll he[2];
    double rho[2][AMG_MAXL] = {};  // spectral radius estimate of D^-1 A per level
    HierOff hoff[2];
    int amg_index = -1;           // position among the cases with hierarchies
    int64_t vec_off = 0;          // per-system solver vectors
    int64_t dinv_off = 0;         // inverse diagonals of both hierarchies
    // nested-dissection Cholesky factor of the projection matrix (mode 2)
    bool has_chol = false;
    CholFactor chol;
    int ds_case_index = -1;
};

void build_hier_ell(const AmgH& H, const EllH& ell0, HierEll& E)
{
    const int L = (int)H.lv.size();
    E.A.assign(L, EllH());
    E.P.assign(L, EllH());
    E.R.assign(L, EllH());
    E.gptr.assign(L, {}); E.gidx.assign(L, {}); E.gdst.assign(L, {}); E.gcoef.assign(L, {});
    for (int l = 1; l < L; ++l) to_ell(H.lv[l].A, true, E.A[l]);
    for (int l = 0; l + 1 < L; ++l) {
        to_ell(H.lv[l].P, false, E.P[l]);
        to_ell(H.lv[l].R, false, E.R[l]);
        const std::vector<int>& src_map = l == 0 ? ell0.map : E.A[l].map;
        E.gptr[l] = H.lv[l].gptr;
        E.gcoef[l] = H.lv[l].gcoef;
        E.gidx[l].resize(H.lv[l].gidx.size());
        for (size_t j = 0; j < H.lv[l].gidx.size(); ++j) E.gidx[l][j] = src_map[H.lv[l].gidx[j]];
        E.gdst[l] = E.A[l + 1].map;
    }
}

// serialise (or only size) one hierarchy into the flat regions
void pack_hier(const HierEll& E, HierOff& o, std::vector<int32_t>* ai, std::vector<double>* ad, int64_t& ni, int64_t& nd)
{
    auto puti = [&](const std::vector<int>& v) {
        int64_t at = ni;
        if (ai) ai->insert(ai->end(), v.begin(), v.end());
        ni += (int64_t)v.size();
        return at;
    };
    auto putd = [&](const std::vector<double>& v) {
        int64_t at = nd;
        if (ad) ad->insert(ad->end(), v.begin(), v.end());
        nd += (int64_t)v.size();
        return at;
    };
    const int L = (int)E.A.size();
    for (int l = 0; l < L; ++l) {
        if (l >= 1) { o.Acol[l] = puti(E.A[l].col); o.Aval[l] = putd(E.A[l].val); o.Alen[l] = puti(E.A[l].len); }
        if (l + 1 < L) {
            o.Pcol[l] = puti(E.P[l].col); o.Pval[l] = putd(E.P[l].val); o.Plen[l] = puti(E.P[l].len);
            o.Rcol[l] = puti(E.R[l].col); o.Rval[l] = putd(E.R[l].val); o.Rlen[l] = puti(E.R[l].len);
            o.Gptr[l] = puti(E.gptr[l]); o.Gidx[l] = puti(E.gidx[l]); o.Gdst[l] = puti(E.gdst[l]);
            o.Gcoef[l] = putd(E.gcoef[l]);
        }
    }
}

// spectral radius of D^-1 A by power iteration, bounded below by 4/3
double spectral_radius(const CsrH& A)
{
    std::vector<double> d(A.n, 1.0), v(A.n), w(A.n);
    for (int i = 0; i < A.n; ++i)
        for (int j = A.ptr[i]; j < A.ptr[i + 1]; ++j)
            if (A.col[j] == i && A.val[j] != 0.0) d[i] = A.val[j];
    for (int i = 0; i < A.n; ++i) v[i] = 1.0 + 0.5 * std::sin(0.7 * i + 0.3);
    double rho = 1.0;
    for (int it = 0; it < 30; ++it) {
        double nw = 0.0, nv = 0.0;
        for (int i = 0; i < A.n; ++i) {
            double s = 0.0;
            for (int j = A.ptr[i]; j < A.ptr[i + 1]; ++j) s += A.val[j] * v[A.col[j]];
            w[i] = s / d[i];
            nw += w[i] * w[i]; nv += v[i] * v[i];
        }
        rho = std::sqrt(nw / std::max(nv, 1e-300));
        const double sc = 1.0 / std::sqrt(std::max(nw, 1e-300));
        for (int i = 0; i < A.n; ++i) v[i] = w[i] * sc;
    }
    return std::min(20.0 / 3.0, std::max(4.0 / 3.0, rho));
}

// Chebyshev smoother of degree 2 for D^-1 A on [rho/10, 1.1 rho]:
// y1 = y0 + sa D^-1 (b - A y0); y2 = y1 + (se - 1)(y1 - y0) + sc D^-1 (b - A y1)
void chebyshev2(double rho, double& sa, double& se, double& sc)
{
    const double hi = 1.1 * rho, lo = rho / 10.0;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    const double r0 = 1.0 / sigma, r1 = 1.0 / (2.0 * sigma - r0);
    sa = 1.0 / theta;
    se = 1.0 + r1 * r0;
    sc = 2.0 * r1 / delta;
}

// Solver-system layout: vectors of one system at [off, off + mg_vec_len)
int64_t mg_vec_len(const AmgH& H)
{
    int64_t n = 5 * (int64_t)H.lv[0].A.n;                  // r[2], p[2], q
    for (auto& lv : H.lv) n += 4 * (int64_t)lv.A.n;         // lb, ly, la, lt
    return n;
}

int64_t mg_blocks(int64_t n) { return (n + 255) / 256; }
// row blocks of a row-parallel solver phase: one lane per (row, column) pair
int mg_rows_per_block(int nv) { return 256 / nv; }
int64_t mg_blocks_nv(int64_t n, int nv) { return (n + mg_rows_per_block(nv) - 1) / mg_rows_per_block(nv); }

// Stiffness matrix of the case on its own Galerkin pattern (host copy used
// only to build the hierarchies).
CsrH host_stiffness(const MeshHost& m)
{
    CsrH K;
    K.n = K.m = m.nsn;
    K.ptr = m.csr_ptr;
    K.col = m.csr_col;
    K.val.assign(m.csr_col.size(), 0.0);
    for (int s = 0; s < m.nsn; ++s)
        for (int j = m.inc_ptr[s]; j < m.inc_ptr[s + 1]; ++j) {
            const int e = m.inc[j] / 3, a = m.inc[j] % 3;
            const double* rc = &m.rec[8 * (size_t)e];
            for (int cc = 0; cc < 3; ++cc)
                K.val[m.incpos[3 * (size_t)j + cc]] += m.area[e] * (rc[2 + a] * rc[2 + cc] + rc[5 + a] * rc[5 + cc]);
        }
    return K;
}

struct PartBufs {
    char *x, *y, *u, *v, *w, *om, *wt, *psi;   // Real arrays (FP64 or FP32)
    int32_t* elem;
    uint32_t* id;
    uint8_t* bin;
};

}  // namespace

struct pdfmc_ctx {
    int prec = PDFMC_FP64;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<Case> cases;
    // totals
    int64_t NP = 0, PSI = 0, CM = 0, CS = 0;
    int NE = 0, NN = 0, NBC = 0, ntiles = 0;
    int64_t NELL = 0;
    // workspace
    bool bound = false, initialised = false;
    bool have_stats = false;        // node statistics have been formed once
    char* ws = nullptr;
    uint64_t ws_bytes = 0;
    int device = -1;                // device current at workspace bind
    void* d_static_scratch = nullptr;   // that device's address of the static sort scratch
    std::string static_scratch_err;     // why the address lookup failed, if it did
    // device arrays
    CaseDev* d_cases = nullptr;
    int32_t *d_tile_case = nullptr, *d_node_case = nullptr, *d_elem_case = nullptr;
    char* d_rec = nullptr;          // Real records for the particle kernel
    double* d_rec64 = nullptr;      // FP64 records for the node kernels
    char* d_exy = nullptr;
    double* d_exy64 = nullptr;      // FP64 vertex coordinates (initial ensemble)
    int4 *d_tri_s = nullptr, *d_nbr = nullptr, *d_partner = nullptr;
    BcDev* d_bc = nullptr;
    double *d_area = nullptr, *d_vol = nullptr, *d_wnx = nullptr, *d_wny = nullptr;
    int32_t *d_inc_ptr = nullptr, *d_inc = nullptr, *d_incpos = nullptr, *d_ell_col = nullptr, *d_ell_len = nullptr,
            *d_is_wall = nullptr;
    PartBufs part[2]{};
    int cur = 0;
    double *d_F = nullptr, *d_nsum = nullptr, *d_stats = nullptr;
    // scatter records: regular slots of every case, then the pool; per-element
    // record lists, overflow sums, element vertex sums (see pdfmc_dev.h)
    double* d_srec = nullptr;
    int64_t SREC = 0, pool_off = 0;
    int pool_cap = 0;
    int32_t *d_pool_cnt = nullptr, *d_ecnt = nullptr, *d_eof = nullptr, *d_wgcnt = nullptr;
    int64_t* d_eslot = nullptr;
    int64_t* d_ovl = nullptr;       // the element lists' overflow list
    int32_t* d_ovl_el = nullptr;
    int32_t ovl_cap = 0;
    double *d_eo = nullptr, *d_etot = nullptr;
    char* d_Fel = nullptr;          // element-major fields in the particle precision
    double* d_Ffrz = nullptr;       // uploaded fields, for the slots a case keeps frozen
    char* d_cmean = nullptr;
    int32_t* d_ccnt = nullptr;
    double *d_kf = nullptr, *d_ef = nullptr, *d_L2 = nullptr, *d_er_r = nullptr, *d_er_dval = nullptr, *d_er_b = nullptr,
           *d_er_x = nullptr, *d_er_val = nullptr, *d_pk_val = nullptr, *d_pb = nullptr, *d_phi = nullptr, *d_P = nullptr, *d_gphi = nullptr;
    // Eulerian solves: systems (relaxation first, then projection), their
    // vectors, accumulators and state; row-block tables of the phase kernels
    MgJob* d_mg_jobs = nullptr;
    int n_jobs_er = 0, n_jobs_p = 0;
    double* d_mg_vec = nullptr;
    double* d_mg_acc = nullptr;
    int32_t* d_mg_state = nullptr;
    unsigned int* d_mg_need = nullptr;
    double* d_mg_dinv = nullptr;
    double* d_mg_ainv = nullptr;
    int4* d_mg_tab = nullptr;      // (system, first row, hierarchy, 0)
    double* d_mg_part = nullptr;   // the row blocks' partial sums of a phase, per system
    int4* d_mg_tab_dinv = nullptr;
    int64_t MGV = 0, MGD = 0, MGT = 0, MGTD = 0, MGP = 0;
    struct TabRange { int64_t off = 0; int n_er = 0, n_all = 0; };
    TabRange tab0;                  // level-0 rows of every system
    TabRange tabl[AMG_MAXL];        // level-l rows of the systems with more than l large levels
    int n_tab_dinv = 0, n_tab_dinv_er = 0;     // entries; those of the relaxation hierarchies first
    int maxbig_er = 0, maxbig_all = 0;
    // solver options: unrolled iterations (adaptive when mg_auto), small-level threshold
    int mg_iters = 32, mg_auto = 1, tail_rows = 64;
    unsigned int* h_need = nullptr;   // pinned, per system: iterations its solves needed in the last window
    size_t h_need_n = 0;
    std::vector<int32_t> ksw;         // per system: the iteration at which the phases hand it over
    std::vector<int32_t> ksw_low;     // per system: consecutive windows that needed far fewer
    hipEvent_t need_ev = nullptr;
    int need_tick = 0;                 // steps since the last readback of the needed iterations
    int need_wait = 0;                 // steps since that readback was enqueued
    bool need_pending = false;
    std::vector<AmgDev> h_amgdev;   // host copies of what the solver tables point at
    std::vector<MgJob> h_jobs;
    std::vector<int4> h_tab;
    std::vector<int4> h_tab_dinv;
    unsigned long long* d_counters = nullptr;
    uint32_t* d_step = nullptr;
    int32_t* d_sort_count = nullptr;
    int64_t *d_sort_scan = nullptr, *d_sort_bsum = nullptr, *d_sort_cursor = nullptr, *d_sort_start = nullptr;
    int32_t *d_sort_big = nullptr, *d_sort_nbig = nullptr;
    // options
    int sort_interval = 0, block = 256, use_graph = 0;
    int steps_since_sort = 0;
    hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [buffer set][sort at the end]
    hipStream_t side = nullptr;                  // the sort's stream, beside the fields phase
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    uint32_t graph_stages = PDFMC_STAGE_ALL;   // stages of the captured graphs
    bool any_er = false, any_eul = false, any_scalars = false, any_rebin = false;
    bool any_freeze = false;        // some case keeps field slots frozen
    // multigrid data: flat int/double regions, hierarchy descriptors,
    // Galerkin jobs of the relaxation hierarchies per level, per-job vectors
    int64_t AMG_I = 0, AMG_D = 0;
    int n_amg = 0, amg_levels = 0;
    int32_t* d_amg_i = nullptr;
    double* d_amg_d = nullptr;
    AmgDev* d_amg = nullptr;
    GalJob* d_gal = nullptr;           // [AMG_MAXL][n_amg]: relaxation, then projection at [AMG_MAXL*n_amg + ...]
    // Galerkin jobs of each level; each job's lanes per coarse entry come
    // from its own hierarchy, so a case's coarse values do not depend on the
    // other cases of the batch
    int n_gal[AMG_MAXL] = {};
    int n_gal_p[AMG_MAXL] = {};
    int64_t gal_max[AMG_MAXL] = {}, gal_max_p[AMG_MAXL] = {};   // largest nnz * lanes per entry
    // projection by the Cholesky factors: supernodes, their unknown indices
    // and values, the factored cases, supernodes ordered by height
    DsNode* d_ds_nodes = nullptr;
    int32_t* d_ds_idx = nullptr;
    double* d_ds_val = nullptr;
    DsCase* d_ds_cases = nullptr;
    int32_t* d_ds_list = nullptr;
    int32_t* d_ds_cptr = nullptr;      // [NN + 1] per unknown, its contributors in d_ds_clist
    int32_t* d_ds_clist = nullptr;     // contributor slots, per unknown in supernode order
    double* d_ds_contrib = nullptr;    // the forward sweep's updates of later unknowns
    int64_t DSN = 0, DSI = 0, DSV = 0, DSR = 0;
    int DSC = 0, ds_height = -1;
    std::vector<int64_t> ds_hoff;      // list offsets per height
    std::vector<int> ds_hwide;         // per height: sweep variant (small, 256 threads, 1024 threads)
    int proj_method = PDFMC_PROJ_DIRECT;   // requested
    bool proj_direct = false;              // in effect (every mode-2 case factored)
    // live timing of the particle kernel: one event pair per launch
    bool timing = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
};

namespace {

pdfmc_status fail(pdfmc_ctx* c, pdfmc_status s, const std::string& msg)
{
    if (c) c->err = msg;
    return s;
}

#define HIPCHK(ctx, call)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(ctx, PDFMC_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

#define LAUNCHCHK(ctx)                                                                         \
    do {                                                                                       \
        hipError_t e_ = hipGetLastError();                                                     \
        if (e_ != hipSuccess)                                                                  \
            return fail(ctx, PDFMC_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

size_t rsz(const pdfmc_ctx* c) { return c->prec == PDFMC_FP32 ? 4 : 8; }

struct Carver {
    char* base;
    uint64_t off = 0;
    bool assign;
    template <typename T>
    void take(T*& ptr, size_t count, size_t elsize = sizeof(T))
    {
        off = (off + 255) & ~uint64_t(255);
        if (assign) ptr = reinterpret_cast<T*>(base + off);
        off += std::max<size_t>(count, 1) * elsize;
    }
};

void carve(pdfmc_ctx* c, Carver& k)
{
    const size_t R = rsz(c);
    const int64_t NP = c->NP;
    k.take(c->d_cases, c->cases.size());
    k.take(c->d_tile_case, c->ntiles);
    k.take(c->d_node_case, c->NN);
    k.take(c->d_elem_case, c->NE);
    k.take(c->d_rec, 8 * (size_t)c->NE, R);
    k.take(c->d_rec64, 8 * (size_t)c->NE);
    k.take(c->d_exy, 6 * (size_t)c->NE, R);
    k.take(c->d_exy64, 6 * (size_t)c->NE);
    k.take(c->d_tri_s, c->NE);
    k.take(c->d_nbr, c->NE);
    k.take(c->d_partner, c->NE);
    k.take(c->d_bc, c->NBC);
    k.take(c->d_area, c->NE);
    k.take(c->d_vol, c->NN);
    k.take(c->d_wnx, c->NN);
    k.take(c->d_wny, c->NN);
    k.take(c->d_inc_ptr, c->NN + 1);
    k.take(c->d_inc, 3 * (size_t)c->NE);
    k.take(c->d_incpos, 9 * (size_t)c->NE);
    k.take(c->d_ell_col, c->NELL);
    k.take(c->d_ell_len, c->NN);
    k.take(c->d_is_wall, c->NN);
    for (int b = 0; b < 2; ++b) {
        PartBufs& P = c->part[b];
        k.take(P.x, NP, R); k.take(P.y, NP, R); k.take(P.u, NP, R); k.take(P.v, NP, R);
        k.take(P.w, NP, R); k.take(P.om, NP, R); k.take(P.wt, NP, R);
        k.take(P.psi, c->PSI, R);
        k.take(P.elem, NP); k.take(P.id, NP); k.take(P.bin, NP);
    }
    k.take(c->d_F, (size_t)c->NN * NF);
    k.take(c->d_Fel, (size_t)c->NE * 3 * NFE, R);
    k.take(c->d_Ffrz, (size_t)c->NN * NF);
    k.take(c->d_nsum, (size_t)c->NN * NQ);
    k.take(c->d_stats, (size_t)c->NN * NST);
    k.take(c->d_srec, c->SREC);
    k.take(c->d_pool_cnt, 2);       // record pool count, overflow-list count
    k.take(c->d_ecnt, c->NE);
    k.take(c->d_eslot, (size_t)c->NE * SC_K);
    c->ovl_cap = (int32_t)std::max<int64_t>(65536, c->NE);
    k.take(c->d_ovl, (size_t)c->ovl_cap);
    k.take(c->d_ovl_el, (size_t)c->ovl_cap);
    k.take(c->d_eof, c->NE);
    k.take(c->d_eo, (size_t)c->NE * SC_VMAX);
    k.take(c->d_wgcnt, 4 * (size_t)c->ntiles);
    k.take(c->d_etot, (size_t)c->NE * 3 * NQ);
    k.take(c->d_cmean, c->CM, R);
    k.take(c->d_ccnt, 8 * (size_t)c->NE);
    k.take(c->d_kf, c->NN); k.take(c->d_ef, c->NN); k.take(c->d_L2, c->NN);
    k.take(c->d_er_r, (size_t)NER * c->NN); k.take(c->d_er_dval, (size_t)NER * c->NN);
    k.take(c->d_er_b, (size_t)NER * c->NN); k.take(c->d_er_x, (size_t)NER * c->NN);
    k.take(c->d_er_val, c->NELL); k.take(c->d_pk_val, c->NELL);
    k.take(c->d_pb, c->NN); k.take(c->d_phi, c->NN); k.take(c->d_P, c->NN); k.take(c->d_gphi, 2 * (size_t)c->NN);
    k.take(c->d_mg_jobs, (NER + 1) * c->cases.size());
    k.take(c->d_mg_vec, c->MGV);
    k.take(c->d_mg_acc, (size_t)(NER + 1) * c->cases.size() * MG_NSLOT * MG_SLOT);
    k.take(c->d_mg_state, (size_t)(NER + 1) * c->cases.size() * 2);
    k.take(c->d_mg_need, (NER + 1) * c->cases.size());   // per system
    k.take(c->d_mg_dinv, c->MGD);
    k.take(c->d_mg_ainv, 2 * (size_t)std::max(c->n_amg, 1) * AMG_MAXC * AMG_MAXC);
    k.take(c->d_mg_tab, c->MGT);
    k.take(c->d_mg_part, (size_t)std::max<int64_t>(c->MGP, 1) * MG_PART);
    k.take(c->d_mg_tab_dinv, c->MGTD);
    k.take(c->d_counters, NCNT * c->cases.size());
    k.take(c->d_step, 1);
    k.take(c->d_sort_count, c->NE);
    k.take(c->d_sort_scan, c->NE);
    k.take(c->d_sort_bsum, c->NE / SCAN_B + 1);
    k.take(c->d_sort_cursor, c->NE);
    k.take(c->d_sort_start, c->NE);
    k.take(c->d_sort_big, c->NE);
    k.take(c->d_sort_nbig, 1);
    k.take(c->d_amg_i, c->AMG_I);
    k.take(c->d_amg_d, c->AMG_D);
    k.take(c->d_amg, 2 * (size_t)std::max(c->n_amg, 1));
    k.take(c->d_gal, 2 * (size_t)AMG_MAXL * std::max(c->n_amg, 1));
    k.take(c->d_ds_nodes, c->DSN);
    k.take(c->d_ds_idx, c->DSI);
    k.take(c->d_ds_val, c->DSV);
    k.take(c->d_ds_cases, c->DSC);
    k.take(c->d_ds_list, c->DSN);
    k.take(c->d_ds_cptr, c->DSC > 0 ? (size_t)c->NN + 1 : 1);
    k.take(c->d_ds_clist, (size_t)std::max<int64_t>(c->DSR, 1));
    k.take(c->d_ds_contrib, (size_t)std::max<int64_t>(c->DSR, 1));
}

void compute_offsets(pdfmc_ctx* c)
{
    int64_t NP = 0, PSI = 0, CM = 0, CS = 0, NELL = 0;
    int NE = 0, NN = 0, NBC = 0;
    for (auto& cs : c->cases) {
        cs.poff = NP;
        NP += (cs.cap + TILE - 1) / TILE * TILE;
        cs.psioff = PSI; PSI += (int64_t)cs.p.n_scalars * cs.cap;
        cs.cmoff = CM; CM += (int64_t)cs.m.ne * 8 * cs.p.n_scalars;
        cs.csoff = CS; CS += (int64_t)cs.m.ne * 8 * (1 + cs.p.n_scalars);
        cs.eoff = NE; NE += cs.m.ne;
        cs.noff = NN; NN += cs.m.nsn;
        cs.bcoff = NBC; NBC += (int)cs.m.bc.size();
        cs.ell_off = NELL; NELL += cs.p.mode == 2 ? (int64_t)cs.ell0.w * cs.m.nsn : 0;
        cs.inc_off = 3 * (int64_t)cs.eoff;
    }
    // scatter records: SC_RT regular slots per particle tile of each case,
    // each of the case's stride (header + vertex sums + cell sums), then a
    // pool of eight records per tile at the largest stride; the sort's
    // temporaries (20 bytes per particle) reuse the region between steps
    int64_t srec = 0;
    for (auto& cs : c->cases) {
        cs.rec_stride = SC_HDR + sc_nvals(cs.p.n_scalars, true);
        cs.rec_off = srec;
        srec += (cs.cap + TILE - 1) / TILE * SC_RT * (int64_t)cs.rec_stride;
    }
    c->pool_off = srec;
    c->pool_cap = (int)std::min<int64_t>(INT32_MAX / 2, 8 * (NP / TILE) + 64);
    srec += (int64_t)c->pool_cap * (SC_HDR + SC_VMAX);
    srec = std::max<int64_t>(srec, (20 * NP + 7) / 8 + 3 * 32);
    c->SREC = srec;
    int64_t ni = 0, nd = 0, nv = 0, ndv = 0, nt = 0, ntd = 0, np0 = 0;
    int na = 0, maxlev = 0;
    for (auto& cs : c->cases) {
        if (!cs.has_amg) { cs.amg_index = -1; continue; }
        cs.amg_index = na++;
        cs.vec_off = nv;
        cs.dinv_off = ndv;
        for (int h = 0; h < 2; ++h) {
            pack_hier(cs.he[h], cs.hoff[h], nullptr, nullptr, ni, nd);
            maxlev = std::max(maxlev, (int)cs.amg[h].lv.size());
            const int ncol = h == 0 ? NER : 1;      // right-hand sides of the system
            nv += ncol * mg_vec_len(cs.amg[h]);
            for (auto& lv : cs.amg[h].lv) {
                ndv += lv.A.n;
                ntd += mg_blocks(lv.A.n);
                nt += mg_blocks_nv(lv.A.n, ncol);
            }
            nt += mg_blocks_nv(cs.amg[h].lv[0].A.n, ncol);
            np0 += mg_blocks_nv(cs.amg[h].lv[0].A.n, ncol);
        }
    }
    c->AMG_I = ni; c->AMG_D = nd; c->n_amg = na; c->amg_levels = maxlev;
    int64_t dsn = 0, dsi = 0, dsv = 0, dsr = 0;
    int dsc = 0, dsh = -1;
    for (auto& cs : c->cases) {
        if (!cs.has_chol) { cs.ds_case_index = -1; continue; }
        cs.ds_case_index = dsc++;
        dsn += (int64_t)cs.chol.nodes.size();
        dsi += cs.chol.n_idx;
        dsv += cs.chol.n_val;
        for (const CholNode& S : cs.chol.nodes) dsr += (int64_t)S.str.size();
        dsh = std::max(dsh, cs.chol.height);
    }
    c->DSN = dsn; c->DSI = dsi; c->DSV = dsv; c->DSC = dsc; c->ds_height = dsh; c->DSR = dsr;
    c->MGV = nv; c->MGD = ndv; c->MGT = nt; c->MGTD = ntd; c->MGP = np0;
    c->NP = NP; c->PSI = PSI; c->CM = CM; c->CS = CS; c->NE = NE; c->NN = NN; c->NBC = NBC; c->NELL = NELL;
    c->ntiles = (int)(NP / TILE);
}

CaseDev make_case_dev(const pdfmc_ctx* c, const Case& cs)
{
    CaseDev d{};
    const pdfmc_case_params& p = cs.p;
    d.poff = cs.poff; d.np = cs.np; d.psioff = cs.psioff; d.cap = cs.cap; d.cmoff = cs.cmoff; d.csoff = cs.csoff;
    d.eoff = cs.eoff; d.ne = cs.m.ne; d.noff = cs.noff; d.nsn = cs.m.nsn; d.bcoff = cs.bcoff; d.nbc = (int)cs.m.bc.size();
    d.ns = p.n_scalars; d.nbins = p.n_bins; d.nmin = p.n_min; d.mode = p.mode;
    d.seed_lo = (uint32_t)p.seed; d.seed_hi = (uint32_t)(p.seed >> 32); d.stream = p.stream;
    d.ell_w = cs.p.mode == 2 ? cs.ell0.w : 0; d.ell_off = cs.ell_off; d.inc_off = cs.inc_off;
    // the same expressions as the step contract: 2 nu, sqrt(2 nu dt), 2 C3 C4, Cphi/2
    d.dt = p.dt; d.tnu = 2.0 * p.nu; d.sq_nu = std::sqrt(d.tnu * p.dt); d.C3 = p.C3;
    d.c34 = 2.0 * p.C3 * p.C4; d.hphi = 0.5 * p.Cphi;
    d.fdt = (float)d.dt; d.ftnu = (float)d.tnu; d.fsq_nu = (float)d.sq_nu; d.fC3 = (float)d.C3;
    d.fc34 = (float)d.c34; d.fhphi = (float)d.hphi;
    for (int a = 0; a < MAXS; ++a)
        for (int j = 0; j < 4; ++j) { d.src[a][j] = p.src[a][j]; d.srcf[a][j] = (float)p.src[a][j]; }
    d.nu = p.nu; d.C0 = p.C0; d.Cw1 = p.Cw1; d.Cw2 = p.Cw2; d.C1 = p.C1; d.C2 = p.C2; d.gamma5 = p.gamma5;
    d.Cv = p.Cv; d.CL = p.CL; d.Ceta = p.Ceta; d.nu34 = std::sqrt(p.nu * std::sqrt(p.nu));
    d.k_floor = p.k_floor; d.eps_floor = p.eps_floor; d.dpdx[0] = p.dpdx[0]; d.dpdx[1] = p.dpdx[1];
    d.cg_rtol = p.cg_rtol; d.cg_maxit = p.cg_maxit; d.neff_min = p.n_eff_min;
    d.reaction = p.reaction;
    d.rebin = p.rebin;
    d.rec_off = cs.rec_off; d.rec_stride = cs.rec_stride; d.freeze = cs.freeze;
    for (int a = 0; a < MAXS; ++a) { d.kr[a] = p.k_react[a]; d.fkr[a] = (float)p.k_react[a]; }
    (void)c;
    return d;
}

template <typename T>
pdfmc_status h2d(pdfmc_ctx* c, T* dst, const std::vector<T>& src)
{
    if (src.empty()) return PDFMC_OK;
    HIPCHK(c, hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    return PDFMC_OK;
}

#define TRY(x) do { pdfmc_status s_ = (x); if (s_ != PDFMC_OK) return s_; } while (0)

NodeArgs node_args(pdfmc_ctx* c)
{
    NodeArgs A{};
    A.first_stats = c->have_stats ? 0 : 1;
    A.nn = c->NN; A.ne = c->NE; A.cases = c->d_cases; A.node_case = c->d_node_case; A.elem_case = c->d_elem_case;
    A.rec = c->d_rec64; A.area = c->d_area; A.vol = c->d_vol; A.tri_s = c->d_tri_s;
    A.inc_ptr = c->d_inc_ptr; A.inc = c->d_inc; A.incpos = c->d_incpos; A.ell_col = c->d_ell_col; A.ell_len = c->d_ell_len;
    A.is_wall = c->d_is_wall; A.wnx = c->d_wnx; A.wny = c->d_wny;
    A.nsum = c->d_nsum; A.stats = c->d_stats; A.F = c->d_F; A.csum = nullptr; A.ccnt = c->d_ccnt;
    A.srec = c->d_srec; A.pool_off = c->pool_off; A.pool_stride = SC_HDR + SC_VMAX;
    A.ecnt = c->d_ecnt; A.eslot = c->d_eslot; A.eof = c->d_eof; A.eo = c->d_eo; A.wgcnt = c->d_wgcnt; A.etot = c->d_etot;
    A.ovl = c->d_ovl; A.ovl_el = c->d_ovl_el; A.ovl_n = c->d_pool_cnt + 1; A.ovl_cap = c->ovl_cap;
    A.kf = c->d_kf; A.ef = c->d_ef; A.L2 = c->d_L2; A.er_r = c->d_er_r; A.er_dval = c->d_er_dval; A.er_b = c->d_er_b;
    A.er_x = c->d_er_x; A.er_val = c->d_er_val; A.pk_val = c->d_pk_val; A.pb = c->d_pb; A.phi = c->d_phi; A.P = c->d_P; A.gphi = c->d_gphi;
    A.counters = c->d_counters;
    return A;
}

template <typename R>
StepArgs<R> step_args(pdfmc_ctx* c, int advance, int do_bins, int scatter, int rebin_only)
{
    StepArgs<R> A{};
    PartBufs& B = c->part[c->cur];
    A.P = Particles<R>{(R*)B.x, (R*)B.y, (R*)B.u, (R*)B.v, (R*)B.w, (R*)B.om, (R*)B.wt, (R*)B.psi, B.elem, B.id, B.bin};
    A.M = MeshDev<R>{(const R*)c->d_rec, c->d_tri_s, c->d_nbr, c->d_partner, (const R*)c->d_exy, c->d_bc};
    A.cases = c->d_cases;
    A.tile_case = c->d_tile_case;
    A.Fel = (const R*)c->d_Fel;
    A.cmean = (const R*)c->d_cmean;
    A.srec = c->d_srec; A.pool_off = c->pool_off; A.pool_stride = SC_HDR + SC_VMAX; A.pool_cap = c->pool_cap;
    A.pool_cnt = c->d_pool_cnt; A.wgcnt = c->d_wgcnt; A.eof = c->d_eof; A.eo = c->d_eo;
    A.counters = c->d_counters; A.step = c->d_step;
    A.ntiles = c->ntiles; A.advance = advance; A.do_bins = do_bins; A.scatter = scatter; A.rebin_only = rebin_only;
    return A;
}

unsigned nblk(int64_t n, int b) { return (unsigned)std::max<int64_t>(1, (n + b - 1) / b); }

pdfmc_status enqueue_fill(pdfmc_ctx* c, double* p, int64_t n)
{
    if (n <= 0) return PDFMC_OK;
    hipLaunchKernelGGL(k_fill_f64, dim3(std::min<int64_t>(nblk(n, 256), 4096)), dim3(256), 0, c->stream, p, n, 0.0);
    LAUNCHCHK(c);
    return PDFMC_OK;
}

pdfmc_status enqueue_fill_i(pdfmc_ctx* c, int32_t* p, int64_t n)
{
    if (n <= 0) return PDFMC_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3(std::min<int64_t>(nblk(n, 256), 4096)), dim3(256), 0, c->stream, p, n, 0);
    LAUNCHCHK(c);
    return PDFMC_OK;
}

// advance: move the particles; do_bins: velocity bins and cell means;
// scatter: the records and their sums; node_stats: the node statistics from
// those sums (a re-binning pass leaves them as they are).
pdfmc_status enqueue_particles(pdfmc_ctx* c, int advance, int do_bins, int scatter, bool node_stats,
                               int rebin_only = 0)
{
    if (c->ntiles == 0) return PDFMC_OK;
    const int64_t threads = (int64_t)c->ntiles * TILE;
    const int b = c->block;
    const bool timed = c->timing && advance;
    if (timed) {
        while (c->ev.size() < c->ev_used + 2) {
            hipEvent_t e;
            HIPCHK(c, hipEventCreate(&e));
            c->ev.push_back(e);
        }
        HIPCHK(c, hipEventRecord(c->ev[c->ev_used], c->stream));
    }
    if (c->prec == PDFMC_FP64)
        hipLaunchKernelGGL(k_particle_step<double>, dim3(nblk(threads, b)), dim3(b), 0, c->stream,
                           step_args<double>(c, advance, do_bins, scatter, rebin_only));
    else
        hipLaunchKernelGGL(k_particle_step<float>, dim3(nblk(threads, b)), dim3(b), 0, c->stream,
                           step_args<float>(c, advance, do_bins, scatter, rebin_only));
    LAUNCHCHK(c);
    if (timed) {
        HIPCHK(c, hipEventRecord(c->ev[c->ev_used + 1], c->stream));
        c->ev_used += 2;
    }
    if (!scatter) return PDFMC_OK;
    // the records -> element lists -> element vertex sums and cell means ->
    // node statistics
    NodeArgs N = node_args(c);
    hipLaunchKernelGGL(k_scatter_register, dim3(nblk((int64_t)c->ntiles * SC_RT + c->pool_cap, 256)), dim3(256), 0,
                       c->stream, N, c->ntiles, b, (const int32_t*)c->d_tile_case, (const int32_t*)c->d_pool_cnt,
                       c->pool_cap, c->d_counters, do_bins);
    if (c->prec == PDFMC_FP64)
        hipLaunchKernelGGL(k_elem_reduce<double>, dim3(nblk(c->NE, 4)), dim3(256), 0, c->stream, N,
                           (double*)c->d_cmean, do_bins, rebin_only);
    else
        hipLaunchKernelGGL(k_elem_reduce<float>, dim3(nblk(c->NE, 4)), dim3(256), 0, c->stream, N,
                           (float*)c->d_cmean, do_bins, rebin_only);
    if (node_stats) hipLaunchKernelGGL(k_node_reduce, dim3(nblk(c->NN, 256)), dim3(256), 0, c->stream, N);
    LAUNCHCHK(c);
    return PDFMC_OK;
}

// Before a particle-kernel launch: the record pool and the element lists'
// overflow list start empty (the element pass leaves the per-element lists
// and overflow sums cleared).
pdfmc_status enqueue_accum_clear(pdfmc_ctx* c)
{
    return enqueue_fill_i(c, c->d_pool_cnt, 2);
}

void drop_graphs(pdfmc_ctx* c);

int mg_nbig(const pdfmc_ctx* c, const AmgDev& D)
{
    int nb = 0;
    while (nb < D.nlev - 1 && D.n[nb] > c->tail_rows) ++nb;
    return nb;
}

// Systems, accumulator slots and row-block tables of the phase solver.
pdfmc_status build_mg_jobs(pdfmc_ctx* c)
{
    for (auto& D : c->h_amgdev) D.nbig = mg_nbig(c, D);
    if (c->n_amg > 0) TRY(h2d(c, c->d_amg, c->h_amgdev));
    std::vector<MgJob> jer, jp;
    for (size_t ci = 0; ci < c->cases.size(); ++ci) {
        const Case& cs = c->cases[ci];
        if (cs.p.mode != 2) continue;
        int64_t voff = cs.vec_off;
        // one system of NER columns for the relaxed tensor, one of a single
        // column for the pressure increment
        for (int h = 0; h < 2; ++h) {
            const bool proj = h == 1;
            const int nv = proj ? 1 : NER;
            const int hi = 2 * cs.amg_index + h;
            const AmgDev& D = c->h_amgdev[hi];
            MgJob J{};
            J.hier = hi;
            J.mean_free = proj ? 1 : 0;
            // the relaxed tensor changes slowly between steps; the pressure
            // increment is new every step, so its solve starts from zero
            J.warm = proj ? 0 : 1;
            J.maxit = cs.p.cg_maxit;
            J.n = cs.m.nsn;
            J.tol = cs.p.cg_rtol;
            J.nv = nv;
            J.b = proj ? c->d_pb + cs.noff : c->d_er_b + (int64_t)NER * cs.noff;
            J.x = proj ? c->d_phi + cs.noff : c->d_er_x + (int64_t)NER * cs.noff;
            double* v = c->d_mg_vec + voff;
            const int64_t n0 = (int64_t)nv * D.n[0];
            J.r[0] = v; J.r[1] = v + n0; J.p[0] = v + 2 * n0; J.p[1] = v + 3 * n0; J.q = v + 4 * n0;
            v += 5 * n0;
            for (int l = 0; l < D.nlev; ++l) {
                const int64_t nl = (int64_t)nv * D.n[l];
                J.lb[l] = v; J.ly[l] = v + nl; J.la[l] = v + 2 * nl; J.lt[l] = v + 3 * nl;
                v += 4 * nl;
            }
            voff += nv * mg_vec_len(cs.amg[h]);
            J.iters = c->d_counters + (int64_t)ci * NCNT + (proj ? C_CG_P : C_CG_ER);
            J.fails = c->d_counters + (int64_t)ci * NCNT + C_CG_FAIL;
            (proj ? jp : jer).push_back(J);
        }
    }
    c->n_jobs_er = (int)jer.size();
    c->n_jobs_p = (int)jp.size();
    jer.insert(jer.end(), jp.begin(), jp.end());
    int64_t aoff = 0, poff = 0;
    for (size_t j = 0; j < jer.size(); ++j) {
        jer[j].acc = c->d_mg_acc + aoff;
        aoff += (int64_t)jer[j].nv * MG_NSLOT * MG_SLOT;
        jer[j].state = c->d_mg_state + 2 * j;
        jer[j].need = c->d_mg_need + j;
        jer[j].nblk0 = (int32_t)mg_blocks_nv(jer[j].n, jer[j].nv);
        jer[j].part = c->d_mg_part + poff * MG_PART;
        poff += jer[j].nblk0;
    }
    if (poff > c->MGP) return fail(c, PDFMC_E_STATE, "solver partial sums exceed their reservation");
    // the hand-over iteration of each system: kept across rebuilds of the
    // tables (same systems in the same order), else the unrolled count
    if (c->ksw.size() != jer.size()) {
        c->ksw.assign(jer.size(), c->mg_iters);
        c->ksw_low.assign(jer.size(), 0);
    }
    for (size_t j = 0; j < jer.size(); ++j) jer[j].ksw = std::min(c->ksw[j], jer[j].maxit);
    c->h_jobs = jer;
    TRY(h2d(c, c->d_mg_jobs, c->h_jobs));
    const int nj = (int)jer.size();
    std::vector<int4>& tab = c->h_tab;
    tab.clear();
    auto add_rows = [&](int j, int rows) {
        const int rpb = mg_rows_per_block(jer[j].nv);
        for (int r0 = 0; r0 < rows; r0 += rpb) tab.push_back(make_int4(j, r0, jer[j].hier, 0));
    };
    c->tab0.off = 0;
    for (int j = 0; j < c->n_jobs_er; ++j) add_rows(j, jer[j].n);
    c->tab0.n_er = (int)tab.size();
    for (int j = c->n_jobs_er; j < nj; ++j) add_rows(j, jer[j].n);
    c->tab0.n_all = (int)tab.size();
    c->maxbig_er = c->maxbig_all = 0;
    for (int l = 0; l < AMG_MAXL; ++l) {
        auto& T = c->tabl[l];
        T.off = (int64_t)tab.size();
        for (int j = 0; j < nj; ++j) {
            if (j == c->n_jobs_er) T.n_er = (int)(tab.size() - T.off);
            const AmgDev& D = c->h_amgdev[jer[j].hier];
            if (D.nbig > l) {
                add_rows(j, D.n[l]);
                if (j < c->n_jobs_er) c->maxbig_er = std::max(c->maxbig_er, l + 1);
                c->maxbig_all = std::max(c->maxbig_all, l + 1);
            }
        }
        if (c->n_jobs_er == nj) T.n_er = (int)(tab.size() - T.off);
        T.n_all = (int)(tab.size() - T.off);
    }
    if ((int64_t)tab.size() > c->MGT) return fail(c, PDFMC_E_STATE, "solver tables exceed their reservation");
    TRY(h2d(c, c->d_mg_tab, tab));
    std::vector<int4>& td = c->h_tab_dinv;
    td.clear();
    // the relaxation hierarchies (even index: refreshed every solve), then
    // the projection hierarchies (odd: their matrices are constant, refreshed
    // once when the workspace is bound)
    for (int h = 0; h < 2; ++h) {
        for (int hi = h; hi < 2 * c->n_amg; hi += 2) {
            const AmgDev& D = c->h_amgdev[hi];
            for (int l = 0; l < D.nlev; ++l)
                for (int r0 = 0; r0 < D.n[l]; r0 += 256) td.push_back(make_int4(hi, l, r0, 0));
        }
        if (h == 0) c->n_tab_dinv_er = (int)td.size();
    }
    if ((int64_t)td.size() > c->MGTD) return fail(c, PDFMC_E_STATE, "solver tables exceed their reservation");
    c->n_tab_dinv = (int)td.size();
    TRY(h2d(c, c->d_mg_tab_dinv, td));
    return PDFMC_OK;
}

// The projection of every case by its Cholesky factor: mean-free right-hand
// side, forward sweep by increasing supernode height, backward sweep by
// decreasing height, mean-free solution.
pdfmc_status enqueue_direct_projection(pdfmc_ctx* c)
{
    hipStream_t st = c->stream;
    hipLaunchKernelGGL(k_ds_prep, dim3(c->DSC), dim3(1024), 0, st, (const DsCase*)c->d_ds_cases,
                       (const double*)c->d_pb, c->d_phi);
    // per height, the variant its largest supernode needs
    for (int h = 0; h <= c->ds_height; ++h) {
        const int64_t n = c->ds_hoff[h + 1] - c->ds_hoff[h];
        if (n == 0) continue;
        const int32_t* lst = c->d_ds_list + c->ds_hoff[h];
        const DsNode* nd = c->d_ds_nodes;
        const int32_t* ix = c->d_ds_idx;
        const double* vl = c->d_ds_val;
        const DsUpd U{c->d_ds_cptr, c->d_ds_clist, c->d_ds_contrib};
        if (c->ds_hwide[h] == 2)
            hipLaunchKernelGGL((k_ds_forward<1024, DS_MAXS>), dim3((unsigned)n), dim3(1024), 0, st, nd, lst, ix, vl, c->d_phi, U);
        else if (c->ds_hwide[h] == 1)
            hipLaunchKernelGGL((k_ds_forward<1024, DS_SMALL>), dim3((unsigned)n), dim3(1024), 0, st, nd, lst, ix, vl, c->d_phi, U);
        else
            hipLaunchKernelGGL((k_ds_forward<256, DS_SMALL>), dim3((unsigned)n), dim3(256), 0, st, nd, lst, ix, vl, c->d_phi, U);
    }
    for (int h = c->ds_height; h >= 0; --h) {
        const int64_t n = c->ds_hoff[h + 1] - c->ds_hoff[h];
        if (n == 0) continue;
        const int32_t* lst = c->d_ds_list + c->ds_hoff[h];
        const DsNode* nd = c->d_ds_nodes;
        const int32_t* ix = c->d_ds_idx;
        const double* vl = c->d_ds_val;
        if (c->ds_hwide[h] == 2)
            hipLaunchKernelGGL((k_ds_backward<1024, DS_MAXS>), dim3((unsigned)n), dim3(1024), 0, st, nd, lst, ix, vl, c->d_phi);
        else if (c->ds_hwide[h] == 1)
            hipLaunchKernelGGL((k_ds_backward<1024, DS_SMALL>), dim3((unsigned)n), dim3(1024), 0, st, nd, lst, ix, vl, c->d_phi);
        else
            hipLaunchKernelGGL((k_ds_backward<256, DS_SMALL>), dim3((unsigned)n), dim3(256), 0, st, nd, lst, ix, vl, c->d_phi);
    }
    hipLaunchKernelGGL(k_ds_post, dim3(c->DSC), dim3(1024), 0, st, (const DsCase*)c->d_ds_cases, c->d_phi);
    LAUNCHCHK(c);
    return PDFMC_OK;
}

// The multigrid-PCG solves: the relaxation systems of every case, and the
// projection systems when `project` (c->mg_iters PCG iterations as phase
// kernels over all systems, then k_mg_finish for any system that needs more).
pdfmc_status enqueue_mg(pdfmc_ctx* c, bool project)
{
    const int nj = c->n_jobs_er + (project ? c->n_jobs_p : 0);
    if (nj == 0) return PDFMC_OK;
    auto cnt = [&](const pdfmc_ctx::TabRange& t) { return (unsigned)(project ? t.n_all : t.n_er); };
    const int maxbig = project ? c->maxbig_all : c->maxbig_er;
    const MgJob* J = c->d_mg_jobs;
    const AmgDev* H = c->d_amg;
    const int4* T0 = c->d_mg_tab + c->tab0.off;
    const int32_t* S = c->d_mg_state;
    const unsigned g0 = cnt(c->tab0);
    hipStream_t st = c->stream;
    // the relaxation matrices change every step; the projection hierarchies
    // were prepared when the workspace was bound
    hipLaunchKernelGGL(k_mg_dinv, dim3(c->n_tab_dinv_er), dim3(256), 0, st, H, (const int4*)c->d_mg_tab_dinv);
    hipLaunchKernelGGL(k_mg_coarse, dim3(c->n_amg), dim3(1024), 0, st, H, 0, 2);
    // every phase whose workgroups each hold a share of a system's sums is
    // followed by k_mg_reduce, which adds the shares in block order
    auto reduce = [&](int k, int word0, int M, int setup, int big_only) {
        hipLaunchKernelGGL(k_mg_reduce, dim3(nj), dim3(256), 0, st, J, H, S, k, word0, M, setup, big_only);
    };
    hipLaunchKernelGGL(k_mg_setup1, dim3(g0), dim3(256), 0, st, J, T0, S);
    reduce(0, 0, 2, 1, 0);
    hipLaunchKernelGGL(k_mg_setup2, dim3(g0), dim3(256), 0, st, J, H, T0, S);
    reduce(0, 2, 1, 1, 0);
    LAUNCHCHK(c);
    auto vcycle = [&](int k) -> pdfmc_status {
        if (maxbig >= 1)
            hipLaunchKernelGGL(k_mg_res, dim3(cnt(c->tabl[0])), dim3(256), 0, st, J, H,
                               (const int4*)(c->d_mg_tab + c->tabl[0].off), S, 0, k);
        for (int l = 1; l < maxbig; ++l) {
            const int4* Tl = c->d_mg_tab + c->tabl[l].off;
            const dim3 gl(cnt(c->tabl[l]));
            hipLaunchKernelGGL(k_mg_restrict, gl, dim3(256), 0, st, J, H, Tl, S, l, k);
            hipLaunchKernelGGL(k_mg_pre, gl, dim3(256), 0, st, J, H, Tl, S, l, k);
            hipLaunchKernelGGL(k_mg_res, gl, dim3(256), 0, st, J, H, Tl, S, l, k);
        }
        hipLaunchKernelGGL(k_mg_tail, dim3(nj), dim3(1024), 0, st, J, H, S, k);
        for (int l = maxbig - 1; l >= 0; --l) {
            const int4* Tl = c->d_mg_tab + c->tabl[l].off;
            const dim3 gl(cnt(c->tabl[l]));
            hipLaunchKernelGGL(k_mg_prolong, gl, dim3(256), 0, st, J, H, Tl, S, l, k);
            hipLaunchKernelGGL(k_mg_post1, gl, dim3(256), 0, st, J, H, Tl, S, l, k);
            hipLaunchKernelGGL(k_mg_post2, gl, dim3(256), 0, st, J, H, Tl, S, l, k);
            if (l == 0) reduce(k, 3, 2, 0, 1);
        }
        LAUNCHCHK(c);
        return PDFMC_OK;
    };
    hipLaunchKernelGGL(k_mg_pb, dim3(g0), dim3(256), 0, st, J, H, T0, S, -1, 1);
    reduce(-1, 1, 2, 0, 0);
    TRY(vcycle(-1));
    for (int k = 0; k < c->mg_iters; ++k) {
        hipLaunchKernelGGL(k_mg_pa, dim3(g0), dim3(256), 0, st, J, H, T0, S, k);
        reduce(k, 0, 1, 0, 0);
        hipLaunchKernelGGL(k_mg_pb, dim3(g0), dim3(256), 0, st, J, H, T0, S, k, 0);
        reduce(k, 1, 2, 0, 0);
        TRY(vcycle(k));
    }
    hipLaunchKernelGGL(k_mg_finish, dim3(nj), dim3(512), 0, st, J, H, c->mg_iters);
    LAUNCHCHK(c);
    return PDFMC_OK;
}

// The Eulerian solves of every case: the relaxation (multigrid PCG) and, when
// `project`, the projection (Cholesky sweeps, or multigrid PCG together with
// the relaxation).
pdfmc_status enqueue_solve(pdfmc_ctx* c, bool project)
{
    TRY(enqueue_mg(c, project && !c->proj_direct));
    if (project && c->proj_direct && c->DSC > 0) TRY(enqueue_direct_projection(c));
    LAUNCHCHK(c);
    return PDFMC_OK;
}

// After a step: fetch the iteration count the solves needed (asynchronously);
// before a step: adapt the number of unrolled iterations to what was needed,
// NEED_LAG steps after the readback was enqueued, so that the count changes
// at the same steps in every run.
constexpr int NEED_EVERY = 8;
constexpr int NEED_LAG = 2;

pdfmc_status mg_after_step(pdfmc_ctx* c)
{
    if (!c->mg_auto || !c->any_er || c->need_pending || !c->h_need) return PDFMC_OK;
    // one readback every NEED_EVERY steps: a copy between two graph launches
    // costs more than the adaptation gains from reacting a few steps sooner
    // (a system that needs more iterations meanwhile is completed by
    // k_mg_finish)
    if (++c->need_tick < NEED_EVERY) return PDFMC_OK;
    c->need_tick = 0;
    // the counter holds the largest count of the steps since the last
    // readback (the solves only raise it); it restarts after the copy
    const size_t nj = c->h_jobs.size();
    HIPCHK(c, hipMemcpyAsync(c->h_need, c->d_mg_need, nj * sizeof(unsigned int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipEventRecord(c->need_ev, c->stream));
    TRY(enqueue_fill_i(c, (int32_t*)c->d_mg_need, (int64_t)nj));
    c->need_pending = true;
    c->need_wait = 0;
    return PDFMC_OK;
}

pdfmc_status mg_adapt(pdfmc_ctx* c)
{
    if (!c->mg_auto || !c->need_pending) return PDFMC_OK;
    // a fixed number of steps after the readback (by then the copy has long
    // completed: the wait only bounds how far the host runs ahead)
    if (++c->need_wait < NEED_LAG) return PDFMC_OK;
    if (hipEventSynchronize(c->need_ev) != hipSuccess) return PDFMC_OK;
    c->need_pending = false;
    // per system, from its own solves only: the one-workgroup completion is
    // many times slower per iteration than the phases, so keep a margin above
    // what the window needed; lower the hand-over only after two low windows
    bool changed = false;
    int most = 1;
    for (size_t j = 0; j < c->h_jobs.size(); ++j) {
        const int need = (int)c->h_need[j];
        const int margin = std::max(2, need / 8);
        int want = c->ksw[j];
        if (need + 1 > c->ksw[j]) {
            want = need + margin;
            c->ksw_low[j] = 0;
        } else if (need + 2 * margin < c->ksw[j]) {
            if (++c->ksw_low[j] >= 2) { want = need + margin; c->ksw_low[j] = 0; }
        } else {
            c->ksw_low[j] = 0;
        }
        want = std::max(1, std::min(want, 400));
        if (want != c->ksw[j]) { c->ksw[j] = want; changed = true; }
        c->h_jobs[j].ksw = std::min(want, c->h_jobs[j].maxit);
        most = std::max(most, c->h_jobs[j].ksw);
    }
    if (changed) TRY(h2d(c, c->d_mg_jobs, c->h_jobs));
    // the phases are unrolled for the system that needs the most
    if (most != c->mg_iters) {
        c->mg_iters = most;
        drop_graphs(c);
    }
    return PDFMC_OK;
}

// Coarse operators of one level for n hierarchies (max_lanes: the largest
// nnz * lanes per entry of the jobs)
pdfmc_status enqueue_galerkin(pdfmc_ctx* c, const GalJob* jobs, int n, int64_t max_lanes)
{
    if (n == 0) return PDFMC_OK;
    const dim3 g(std::min<int64_t>(nblk(max_lanes, 256), 1024), n);
    hipLaunchKernelGGL(k_galerkin, g, dim3(256), 0, c->stream, jobs);
    LAUNCHCHK(c);
    return PDFMC_OK;
}

// The element-major copy of the fields that the particle kernel reads.
pdfmc_status enqueue_fields_elem(pdfmc_ctx* c)
{
    const dim3 g(nblk((int64_t)c->NE * 3 * NFE, 256)), b(256);
    if (c->prec == PDFMC_FP64)
        hipLaunchKernelGGL(k_fields_elem<double>, g, b, 0, c->stream, (const double*)c->d_F, (const double*)c->d_gphi,
                           (const int4*)c->d_tri_s,
                           (double*)c->d_Fel, c->NE);
    else
        hipLaunchKernelGGL(k_fields_elem<float>, g, b, 0, c->stream, (const double*)c->d_F, (const double*)c->d_gphi,
                           (const int4*)c->d_tri_s,
                           (float*)c->d_Fel, c->NE);
    LAUNCHCHK(c);
    return PDFMC_OK;
}

pdfmc_status enqueue_fields(pdfmc_ctx* c, bool project)
{
    NodeArgs A = node_args(c);
    const dim3 g(nblk(c->NN, 256)), b(256);
    if (c->any_eul) {
        hipLaunchKernelGGL(k_fields_grad, g, b, 0, c->stream, A);
        hipLaunchKernelGGL(k_fields_derived, g, b, 0, c->stream, A);
        LAUNCHCHK(c);
    }
    if (c->any_er) {
        hipLaunchKernelGGL(k_er_assemble, g, b, 0, c->stream, A);
        if (project) hipLaunchKernelGGL(k_proj_rhs, g, b, 0, c->stream, A);
        for (int l = 0; l < AMG_MAXL; ++l)
            TRY(enqueue_galerkin(c, c->d_gal + (size_t)l * c->n_amg, c->n_gal[l], c->gal_max[l]));
        // relaxation and projection systems of every case together
        TRY(enqueue_solve(c, project));
        hipLaunchKernelGGL(k_er_finish, g, b, 0, c->stream, A);
        LAUNCHCHK(c);
        if (project) {
            hipLaunchKernelGGL(k_proj_update, g, b, 0, c->stream, A);
            LAUNCHCHK(c);
        }
        hipLaunchKernelGGL(k_proj_grad, g, b, 0, c->stream, A);
        LAUNCHCHK(c);
    }
    if (c->any_freeze) {
        hipLaunchKernelGGL(k_fields_freeze, dim3(nblk((int64_t)c->NN * NF, 256)), dim3(256), 0, c->stream,
                           (const CaseDev*)c->d_cases, (const int32_t*)c->d_node_case, (const double*)c->d_Ffrz,
                           c->d_F, c->NN);
        LAUNCHCHK(c);
    }
    TRY(enqueue_fields_elem(c));
    return PDFMC_OK;
}

// The temporaries of one sort: per-element counts, scans, cursors, segment
// starts and the list of long segments, and per-particle placed ids, their
// sources and the final permutation.
struct SortScratch {
    int32_t* count; int64_t *scan, *bsum, *cursor, *start; int32_t *big, *nbig;
    int64_t *perm, *tmp_src; uint32_t* tmp_id;
};

// The temporaries carved from one contiguous region (256-byte aligned
// pieces); with base == nullptr only the size is computed.
uint64_t sort_scratch_carve(char* base, int64_t ne, int64_t np, SortScratch* sc)
{
    Carver k{base, 0, base != nullptr};
    SortScratch t{};
    k.take(t.count, ne); k.take(t.scan, ne); k.take(t.bsum, ne / SCAN_B + 1); k.take(t.cursor, ne);
    k.take(t.start, ne); k.take(t.big, ne); k.take(t.nbig, 1);
    k.take(t.perm, np); k.take(t.tmp_src, np); k.take(t.tmp_id, np);
    if (sc) *sc = t;
    return k.off;
}

// The sort's temporaries in the bound workspace: per-element arrays of their
// own, per-particle ones in the scatter-record region, which holds nothing
// between steps.
SortScratch sort_scratch_ws(pdfmc_ctx* c)
{
    SortScratch t{};
    t.count = c->d_sort_count; t.scan = c->d_sort_scan; t.bsum = c->d_sort_bsum; t.cursor = c->d_sort_cursor;
    t.start = c->d_sort_start; t.big = c->d_sort_big; t.nbig = c->d_sort_nbig;
    t.perm = (int64_t*)c->d_srec;
    t.tmp_src = t.perm + c->NP;
    t.tmp_id = (uint32_t*)(t.tmp_src + c->NP);
    return t;
}

pdfmc_status enqueue_sort(pdfmc_ctx* c, const SortScratch& T);

// One step restricted to the stages in `stages` (PDFMC_STAGE_*): without
// ADVANCE the particles stay where they are (the statistics of the current
// state are formed), without STATS the node statistics and cell means keep
// their values, without FIELDS the Eulerian fields keep theirs.
pdfmc_status enqueue_step_body(pdfmc_ctx* c, uint32_t stages, bool sort_after)
{
    const bool adv = stages & PDFMC_STAGE_ADVANCE, st = stages & PDFMC_STAGE_STATS;
    if (adv || st) {
        TRY(enqueue_accum_clear(c));
        TRY(enqueue_particles(c, adv ? 1 : 0, 1, st ? 1 : 0, st));
    }
    // a sort due before the next step runs on the side stream while the
    // fields are formed: it reads and writes only the particle arrays and its
    // temporaries in the record region, which the fields phase does not touch
    if (sort_after) {
        HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
        HIPCHK(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
        hipStream_t main_stream = c->stream;
        c->stream = c->side;
        const pdfmc_status ss = enqueue_sort(c, sort_scratch_ws(c));
        c->stream = main_stream;
        TRY(ss);
        HIPCHK(c, hipEventRecord(c->ev_join, c->side));
    }
    if (stages & PDFMC_STAGE_FIELDS) TRY(enqueue_fields(c, true));
    if (sort_after) HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
    // R-36: the cases that form their bins and cell means again against the
    // new fields (a statistics-free particle pass over their tiles); after the
    // sort has joined, since both use the particle arrays and the record region
    if ((stages & PDFMC_STAGE_FIELDS) && c->any_rebin) {
        TRY(enqueue_accum_clear(c));
        TRY(enqueue_particles(c, 0, 1, 1, false, 1));
    }
    hipLaunchKernelGGL(k_step_increment, dim3(1), dim3(64), 0, c->stream, c->d_step);
    LAUNCHCHK(c);
    return PDFMC_OK;
}

pdfmc_status enqueue_sort(pdfmc_ctx* c, const SortScratch& T)
{
    if (c->ntiles == 0) return PDFMC_OK;
    SortArgs S{};
    S.cases = c->d_cases; S.tile_case = c->d_tile_case; S.elem_case = c->d_elem_case;
    S.ntiles = c->ntiles; S.ne = c->NE; S.elem = c->part[c->cur].elem;
    S.count = T.count; S.scan = T.scan; S.bsum = T.bsum; S.cursor = T.cursor;
    S.start = T.start; S.big = T.big; S.nbig = T.nbig;
    S.perm = T.perm; S.tmp_src = T.tmp_src; S.tmp_id = T.tmp_id;
    // counts and the long-segment count start at zero (fill kernels, so the
    // sequence can be captured)
    TRY(enqueue_fill_i(c, T.count, c->NE));
    TRY(enqueue_fill_i(c, T.nbig, 1));
    const int64_t threads = (int64_t)c->ntiles * TILE;
    hipLaunchKernelGGL(k_sort_hist, dim3(nblk(threads, 256)), dim3(256), 0, c->stream, S);
    const int nb = (int)nblk(c->NE, SCAN_B);
    hipLaunchKernelGGL(k_sort_scan_blocks, dim3(nb), dim3(SCAN_B), 0, c->stream, S);
    hipLaunchKernelGGL(k_sort_scan_totals, dim3(1), dim3(SCAN_B), 0, c->stream, S, nb);
    hipLaunchKernelGGL(k_sort_cursor, dim3(nb), dim3(SCAN_B), 0, c->stream, S);
    hipLaunchKernelGGL(k_sort_place, dim3(nblk(threads, 256)), dim3(256), 0, c->stream, S,
                       (const uint32_t*)c->part[c->cur].id);
    hipLaunchKernelGGL(k_sort_order, dim3(nblk(c->NE, 4)), dim3(256), 0, c->stream, S);
    hipLaunchKernelGGL(k_sort_order_big, dim3(64), dim3(1024), 0, c->stream, S);
    LAUNCHCHK(c);
    PartBufs& A = c->part[c->cur];
    PartBufs& B = c->part[1 - c->cur];
    if (c->prec == PDFMC_FP64) {
        Particles<double> src{(double*)A.x, (double*)A.y, (double*)A.u, (double*)A.v, (double*)A.w, (double*)A.om,
                              (double*)A.wt, (double*)A.psi, A.elem, A.id, A.bin};
        Particles<double> dst{(double*)B.x, (double*)B.y, (double*)B.u, (double*)B.v, (double*)B.w, (double*)B.om,
                              (double*)B.wt, (double*)B.psi, B.elem, B.id, B.bin};
        hipLaunchKernelGGL(k_sort_gather<double>, dim3(nblk(threads, 256)), dim3(256), 0, c->stream, S, src, dst);
    } else {
        Particles<float> src{(float*)A.x, (float*)A.y, (float*)A.u, (float*)A.v, (float*)A.w, (float*)A.om,
                             (float*)A.wt, (float*)A.psi, A.elem, A.id, A.bin};
        Particles<float> dst{(float*)B.x, (float*)B.y, (float*)B.u, (float*)B.v, (float*)B.w, (float*)B.om,
                             (float*)B.wt, (float*)B.psi, B.elem, B.id, B.bin};
        hipLaunchKernelGGL(k_sort_gather<float>, dim3(nblk(threads, 256)), dim3(256), 0, c->stream, S, src, dst);
    }
    LAUNCHCHK(c);
    c->cur = 1 - c->cur;
    c->steps_since_sort = 0;
    return PDFMC_OK;
}

pdfmc_status check_case(pdfmc_ctx* c, int32_t cs)
{
    if (!c) return PDFMC_E_INVALID;
    if (cs < 0 || cs >= (int32_t)c->cases.size()) return fail(c, PDFMC_E_INVALID, "bad case id");
    return PDFMC_OK;
}

pdfmc_status check_bound(pdfmc_ctx* c)
{
    if (!c->bound) return fail(c, PDFMC_E_STATE, "bind a workspace first");
    return PDFMC_OK;
}

void drop_graphs(pdfmc_ctx* c)
{
    for (auto& gs : c->graph)
        for (auto& g : gs)
            if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
}

}  // namespace

// ============================================================== ABI

extern "C" {

pdfmc_status pdfmc_create(pdfmc_ctx** out, int32_t precision, void* hip_stream)
{
    if (!out) return PDFMC_E_INVALID;
    *out = nullptr;
    if (precision != PDFMC_FP64 && precision != PDFMC_FP32) return PDFMC_E_INVALID;
    pdfmc_ctx* c = new (std::nothrow) pdfmc_ctx();
    if (!c) return PDFMC_E_NOMEM;
    c->prec = precision;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return PDFMC_OK;
}

void pdfmc_destroy(pdfmc_ctx* c)
{
    if (!c) return;
    if (c->bound) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->side) (void)hipStreamSynchronize(c->side);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->side) (void)hipStreamDestroy(c->side);
    for (auto e : c->ev) (void)hipEventDestroy(e);
    if (c->need_ev) (void)hipEventDestroy(c->need_ev);
    if (c->h_need) (void)hipHostFree(c->h_need);
    delete c;
}

const char* pdfmc_last_error(const pdfmc_ctx* c) { return c ? c->err.c_str() : "null context"; }

pdfmc_status pdfmc_add_case(pdfmc_ctx* c, const pdfmc_mesh_desc* mesh, const pdfmc_case_params* p, int64_t capacity,
                            int32_t* case_id)
{
    if (!c) return PDFMC_E_INVALID;
    if (!mesh || !p || !case_id) return fail(c, PDFMC_E_INVALID, "add_case: null argument");
    if (c->bound) return fail(c, PDFMC_E_STATE, "add_case: cases must be added before the workspace is bound");
    if (p->n_scalars < 0 || p->n_scalars > PDFMC_MAX_SCALARS) return fail(c, PDFMC_E_INVALID, "add_case: n_scalars must be 0..4");
    if (p->n_bins != 1 && p->n_bins != 8) return fail(c, PDFMC_E_INVALID, "add_case: n_bins must be 1 or 8");
    if (p->mode < 0 || p->mode > 2) return fail(c, PDFMC_E_INVALID, "add_case: mode must be 0, 1 or 2");
    if (!(p->dt > 0.0) || !(p->nu >= 0.0)) return fail(c, PDFMC_E_INVALID, "add_case: need dt > 0 and nu >= 0");
    if (!(p->n_eff_min >= 0.0)) return fail(c, PDFMC_E_INVALID, "add_case: n_eff_min must be >= 0");
    if (p->reaction < 0 || p->reaction > 2) return fail(c, PDFMC_E_INVALID, "add_case: reaction must be 0, 1 or 2");
    if (p->rebin < 0 || p->rebin > 1) return fail(c, PDFMC_E_INVALID, "add_case: rebin must be 0 or 1");
    if (p->reaction == 2 && p->n_scalars < 3)
        return fail(c, PDFMC_E_INVALID, "add_case: reaction 2 (A + B -> P) needs at least 3 scalars");
    for (int a = 0; a < PDFMC_MAX_SCALARS; ++a)
        if (!(p->k_react[a] >= 0.0 && p->k_react[a] < 1e300))
            return fail(c, PDFMC_E_INVALID, "add_case: k_react must be finite and >= 0");
    if (capacity < 0 || capacity > ((int64_t)1 << 31)) return fail(c, PDFMC_E_INVALID, "add_case: bad capacity");
    Case cs;
    cs.p = *p;
    cs.cap = capacity;
    std::string err;
    int rc = derive_mesh(*mesh, cs.m, err);
    if (rc != PDFMC_OK) return fail(c, (pdfmc_status)rc, err);
    if (p->mode == 2) {
        const CsrH K = host_stiffness(cs.m);
        to_ell(K, true, cs.ell0);
        amg_setup(K, cs.m.is_wall, cs.amg[0], AMG_MAXC, AMG_MAXL);
        amg_setup(K, std::vector<int>(), cs.amg[1], AMG_MAXC, AMG_MAXL);
        cs.has_amg = cs.amg[0].lv.back().A.n <= AMG_MAXC && cs.amg[1].lv.back().A.n <= AMG_MAXC;
        if (!cs.has_amg)
            return fail(c, PDFMC_E_UNSUPPORTED, "add_case: the multigrid hierarchy of the Eulerian solves does not reach a "
                                                "coarsest level of at most 64 unknowns within 8 levels");
        for (int h = 0; h < 2 && cs.has_amg; ++h) {
            for (size_t l = 0; l < cs.amg[h].lv.size(); ++l) cs.rho[h][l] = spectral_radius(cs.amg[h].lv[l].A);
            build_hier_ell(cs.amg[h], cs.ell0, cs.he[h]);
        }
        // the projection matrix is constant: factor it once (statistics
        // node 0 decoupled); without a factor the projection runs on the
        // multigrid PCG like the relaxation
        std::vector<double> sx(cs.m.nsn), sy(cs.m.nsn);
        for (int sn = 0; sn < cs.m.nsn; ++sn) { sx[sn] = cs.m.x[cs.m.rep[sn]]; sy[sn] = cs.m.y[cs.m.rep[sn]]; }
        std::string ferr;
        cs.has_chol = chol_factor(K, sx, sy, 0, 64, cs.chol, ferr) && cs.chol.max_s <= DS_MAXS &&
                      cs.chol.max_m <= DS_MAXS;
        if (!cs.has_chol) cs.chol = CholFactor();
    }
    c->cases.push_back(std::move(cs));
    *case_id = (int32_t)c->cases.size() - 1;
    compute_offsets(c);
    return PDFMC_OK;
}

pdfmc_status pdfmc_case_info(pdfmc_ctx* c, int32_t cs, int32_t* n_stat_nodes, int32_t* stat_node)
{
    TRY(check_case(c, cs));
    const Case& k = c->cases[cs];
    if (n_stat_nodes) *n_stat_nodes = k.m.nsn;
    if (stat_node) std::copy(k.m.snode.begin(), k.m.snode.end(), stat_node);
    return PDFMC_OK;
}

pdfmc_status pdfmc_workspace_query(pdfmc_ctx* c, uint64_t* bytes)
{
    if (!c || !bytes) return PDFMC_E_INVALID;
    Carver k{nullptr, 0, false};
    carve(c, k);
    *bytes = k.off + 256;
    return PDFMC_OK;
}

pdfmc_status pdfmc_workspace_bind(pdfmc_ctx* c, void* dev, uint64_t bytes)
{
    if (!c) return PDFMC_E_INVALID;
    if (!dev) return fail(c, PDFMC_E_INVALID, "workspace_bind: null pointer");
    if (c->cases.empty()) return fail(c, PDFMC_E_STATE, "workspace_bind: add a case first");
    uint64_t need = 0;
    TRY(pdfmc_workspace_query(c, &need));
    if (bytes < need) return fail(c, PDFMC_E_NOMEM, "workspace_bind: need " + std::to_string(need) + " bytes");
    // record keys (workgroup index * 512 + position) stay below 2^32 at the smallest block size
    if (c->NP > ((int64_t)1 << 29))
        return fail(c, PDFMC_E_INVALID, "workspace_bind: at most 2^29 particle slots in one context");
    char* base = (char*)(((uintptr_t)dev + 255) & ~(uintptr_t)255);
    Carver k{base, 0, true};
    carve(c, k);
    drop_graphs(c);
    c->ws = (char*)dev; c->ws_bytes = bytes; c->cur = 0;
    c->any_er = c->any_eul = c->any_scalars = c->any_rebin = false;
    for (auto& cs : c->cases) {
        c->any_rebin |= cs.p.rebin != 0;
        c->any_er |= cs.p.mode == 2;
        c->any_eul |= cs.p.mode >= 1;
        c->any_scalars |= cs.p.n_scalars > 0;
    }
    // ---- host staging of the global tables
    const int NE = c->NE, NN = c->NN;
    std::vector<CaseDev> cd;
    std::vector<int32_t> tile_case(c->ntiles), node_case(NN), elem_case(NE);
    std::vector<double> rec64(8 * (size_t)NE), exy64(6 * (size_t)NE), area(NE), vol(NN), wnx(NN), wny(NN);
    std::vector<int4> tri_s(NE), nbr(NE), partner(NE);
    std::vector<BcDev> bc(std::max(c->NBC, 1));
    std::vector<int32_t> inc_ptr(NN + 1), inc(3 * (size_t)NE), incpos(9 * (size_t)NE), ell_len(NN, 0),
        ell_col(std::max<int64_t>(c->NELL, 1), 0), is_wall(NN);
    int ci = 0;
    for (auto& cs : c->cases) {
        const MeshHost& m = cs.m;
        cd.push_back(make_case_dev(c, cs));
        for (int64_t t = cs.poff / TILE; t < (cs.poff + (cs.cap + TILE - 1) / TILE * TILE) / TILE; ++t) tile_case[t] = ci;
        for (int s = 0; s < m.nsn; ++s) {
            const int g = cs.noff + s;
            node_case[g] = ci;
            vol[g] = m.vol[s];
            wnx[g] = m.wnx[s]; wny[g] = m.wny[s];
            is_wall[g] = m.is_wall[s];
            inc_ptr[g] = 3 * cs.eoff + m.inc_ptr[s];
            if (cs.p.mode == 2) ell_len[g] = cs.ell0.len[s];
        }
        for (int e = 0; e < m.ne; ++e) {
            const int g = cs.eoff + e;
            elem_case[g] = ci;
            std::copy(&m.rec[8 * (size_t)e], &m.rec[8 * (size_t)e + 8], &rec64[8 * (size_t)g]);
            for (int k = 0; k < 3; ++k) {
                exy64[6 * (size_t)g + 2 * k] = m.x[m.tri[3 * e + k]];
                exy64[6 * (size_t)g + 2 * k + 1] = m.y[m.tri[3 * e + k]];
            }
            area[g] = m.area[e];
            tri_s[g] = make_int4(cs.noff + m.tri_s[3 * e], cs.noff + m.tri_s[3 * e + 1], cs.noff + m.tri_s[3 * e + 2], ci);
            int nb[3], pt[3];
            for (int k = 0; k < 3; ++k) {
                const int n = m.nbr[3 * e + k];
                nb[k] = n >= 0 ? cs.eoff + n : -1 - (cs.bcoff + m.tag[3 * e + k]);
                pt[k] = m.partner[3 * e + k] >= 0 ? cs.eoff + m.partner[3 * e + k] : -1;
            }
            nbr[g] = make_int4(nb[0], nb[1], nb[2], 0);
            partner[g] = make_int4(pt[0], pt[1], pt[2], 0);
        }
        for (size_t j = 0; j < m.inc.size(); ++j) {
            const int ent = m.inc[j];
            inc[3 * (size_t)cs.eoff + j] = 3 * (cs.eoff + ent / 3) + ent % 3;
            for (int k = 0; k < 3; ++k)
                incpos[3 * (3 * (size_t)cs.eoff + j) + k] = cs.p.mode == 2 ? (int32_t)(cs.ell_off + cs.ell0.map[m.incpos[3 * j + k]]) : 0;
        }
        if (cs.p.mode == 2) std::copy(cs.ell0.col.begin(), cs.ell0.col.end(), ell_col.begin() + cs.ell_off);
        for (size_t b = 0; b < m.bc.size(); ++b) {
            BcDev& d = bc[cs.bcoff + b];
            d.type = m.bc[b].type;
            for (int i = 0; i < 3; ++i) { d.uw[i] = m.bc[b].u_wall[i]; d.uwf[i] = (float)m.bc[b].u_wall[i]; }
            for (int i = 0; i < 2; ++i) { d.shift[i] = m.bc[b].shift[i]; d.shiftf[i] = (float)m.bc[b].shift[i]; }
        }
        ++ci;
    }
    inc_ptr[NN] = 3 * NE;
    TRY(h2d(c, c->d_cases, cd));
    TRY(h2d(c, c->d_tile_case, tile_case));
    TRY(h2d(c, c->d_node_case, node_case));
    TRY(h2d(c, c->d_elem_case, elem_case));
    TRY(h2d(c, c->d_rec64, rec64));
    TRY(h2d(c, c->d_exy64, exy64));
    TRY(h2d(c, c->d_tri_s, tri_s));
    TRY(h2d(c, c->d_nbr, nbr));
    TRY(h2d(c, c->d_partner, partner));
    TRY(h2d(c, c->d_bc, bc));
    TRY(h2d(c, c->d_area, area));
    TRY(h2d(c, c->d_vol, vol));
    TRY(h2d(c, c->d_wnx, wnx));
    TRY(h2d(c, c->d_wny, wny));
    TRY(h2d(c, c->d_inc_ptr, inc_ptr));
    TRY(h2d(c, c->d_inc, inc));
    TRY(h2d(c, c->d_incpos, incpos));
    TRY(h2d(c, c->d_ell_col, ell_col));
    TRY(h2d(c, c->d_ell_len, ell_len));
    TRY(h2d(c, c->d_is_wall, is_wall));
    std::vector<float> rec32, exy32;
    if (c->prec == PDFMC_FP64) {
        TRY(h2d(c, (double*)c->d_rec, rec64));
        TRY(h2d(c, (double*)c->d_exy, exy64));
    } else {
        rec32.assign(rec64.begin(), rec64.end());
        exy32.assign(exy64.begin(), exy64.end());
        TRY(h2d(c, (float*)c->d_rec, rec32));
        TRY(h2d(c, (float*)c->d_exy, exy32));
    }
    // multigrid hierarchies: flat arrays, descriptors, Galerkin jobs
    std::vector<AmgDev> amgdev(2 * (size_t)std::max(c->n_amg, 1));
    std::vector<GalJob> gal(2 * (size_t)AMG_MAXL * std::max(c->n_amg, 1));
    for (int l = 0; l < AMG_MAXL; ++l) {
        c->n_gal[l] = 0; c->n_gal_p[l] = 0; c->gal_max[l] = 0; c->gal_max_p[l] = 0;
    }
    if (c->n_amg > 0) {
        std::vector<int32_t> ai;
        std::vector<double> ad;
        ai.reserve(c->AMG_I);
        ad.reserve(c->AMG_D);
        int64_t ni = 0, nd = 0;
        for (auto& cs : c->cases) {
            if (!cs.has_amg) continue;
            for (int h = 0; h < 2; ++h) pack_hier(cs.he[h], cs.hoff[h], &ai, &ad, ni, nd);
        }
        TRY(h2d(c, c->d_amg_i, ai));
        TRY(h2d(c, c->d_amg_d, ad));
        for (auto& cs : c->cases) {
            if (!cs.has_amg) continue;
            const int a = cs.amg_index;
            for (int h = 0; h < 2; ++h) {
                const AmgH& H = cs.amg[h];
                const HierOff& o = cs.hoff[h];
                AmgDev& D = amgdev[2 * a + h];
                D = AmgDev{};
                D.nlev = (int)H.lv.size();
                D.nbig = 0;                     // set by build_mg_jobs
                D.coarse_shift = h == 0 ? 1e-12 : 1e-6;
                D.ainv = c->d_mg_ainv + (size_t)(2 * a + h) * AMG_MAXC * AMG_MAXC;
                const HierEll& E = cs.he[h];
                int64_t doff = cs.dinv_off;
                if (h == 1) for (auto& lv : cs.amg[0].lv) doff += lv.A.n;
                for (int l = 0; l < D.nlev; ++l) {
                    D.n[l] = H.lv[l].A.n;
                    D.dinv[l] = c->d_mg_dinv + doff;
                    doff += D.n[l];
                    chebyshev2(cs.rho[h][l], D.sa[l], D.se[l], D.sc[l]);
                    if (l == 0)
                        D.A[0] = EllDev{cs.m.nsn, cs.ell0.w, c->d_ell_col + cs.ell_off,
                                        (h == 0 ? c->d_er_val : c->d_pk_val) + cs.ell_off, c->d_ell_len + cs.noff};
                    else
                        D.A[l] = EllDev{E.A[l].n, E.A[l].w, c->d_amg_i + o.Acol[l], c->d_amg_d + o.Aval[l],
                                        c->d_amg_i + o.Alen[l]};
                    if (l + 1 < D.nlev) {
                        D.P[l] = EllDev{E.P[l].n, E.P[l].w, c->d_amg_i + o.Pcol[l], c->d_amg_d + o.Pval[l],
                                        c->d_amg_i + o.Plen[l]};
                        D.R[l] = EllDev{E.R[l].n, E.R[l].w, c->d_amg_i + o.Rcol[l], c->d_amg_d + o.Rval[l],
                                        c->d_amg_i + o.Rlen[l]};
                    }
                }
                // Galerkin jobs: level l -> l+1
                for (int l = 0; l + 1 < D.nlev; ++l) {
                    GalJob G{};
                    G.nnz = (int32_t)E.gdst[l].size();
                    G.gptr = c->d_amg_i + o.Gptr[l];
                    G.gidx = c->d_amg_i + o.Gidx[l];
                    G.gdst = c->d_amg_i + o.Gdst[l];
                    G.gcoef = c->d_amg_d + o.Gcoef[l];
                    G.src = l == 0 ? (h == 0 ? c->d_er_val : c->d_pk_val) + cs.ell_off : c->d_amg_d + o.Aval[l];
                    G.dst = c->d_amg_d + o.Aval[l + 1];
                    // lanes per coarse entry from the mean contribution-list length
                    const double terms = G.nnz > 0 ? (double)E.gidx[l].size() / G.nnz : 0.0;
                    G.lpe = terms >= 5.0 ? 16 : (terms >= 2.0 ? 4 : 1);
                    if (h == 0) {
                        gal[(size_t)l * c->n_amg + c->n_gal[l]++] = G;
                        c->gal_max[l] = std::max<int64_t>(c->gal_max[l], (int64_t)G.nnz * G.lpe);
                    } else {
                        gal[(size_t)(AMG_MAXL + l) * c->n_amg + c->n_gal_p[l]++] = G;
                        c->gal_max_p[l] = std::max<int64_t>(c->gal_max_p[l], (int64_t)G.nnz * G.lpe);
                    }
                }
            }
        }
        TRY(h2d(c, c->d_amg, amgdev));
        TRY(h2d(c, c->d_gal, gal));
    }
    {
        const size_t nn = (NER + 1) * c->cases.size();
        if (c->h_need && c->h_need_n < nn) {
            (void)hipHostFree(c->h_need);
            c->h_need = nullptr;
        }
        if (!c->h_need) {
            HIPCHK(c, hipHostMalloc((void**)&c->h_need, nn * sizeof(unsigned int), hipHostMallocDefault));
            c->h_need_n = nn;
        }
        for (size_t j = 0; j < nn; ++j) c->h_need[j] = 0;
    }
    c->ksw.clear();
    if (!c->need_ev) HIPCHK(c, hipEventCreateWithFlags(&c->need_ev, hipEventDisableTiming));
    c->need_pending = false;
    // projection factors: supernodes with global unknown indices, listed by height
    c->ds_hoff.assign(1, 0);
    if (c->DSC > 0) {
        std::vector<DsNode> nodes;
        std::vector<int32_t> idx;
        std::vector<double> val;
        std::vector<DsCase> dcs;
        idx.reserve(c->DSI);
        val.reserve(c->DSV);
        std::vector<std::vector<int32_t>> byh(c->ds_height + 1);
        // contributors of each unknown, in supernode order (children before parents)
        std::vector<int32_t> ccnt((size_t)c->NN + 1, 0);
        std::vector<std::pair<int32_t, int32_t>> cpairs;     // (unknown, slot)
        int64_t cof = 0;
        for (auto& cs : c->cases) {
            if (!cs.has_chol) continue;
            dcs.push_back(DsCase{cs.noff, cs.m.nsn, cs.chol.pin, 0});
            for (const CholNode& S : cs.chol.nodes) {
                DsNode d;
                d.s = (int32_t)S.vars.size();
                d.m = (int32_t)S.str.size();
                d.idx = (int64_t)idx.size();
                d.val = (int64_t)val.size();
                d.cof = cof;
                for (int r = 0; r < d.m; ++r) {
                    const int32_t u = cs.noff + S.str[r];
                    cpairs.emplace_back(u, (int32_t)(cof + r));
                    ++ccnt[(size_t)u + 1];
                }
                cof += d.m;
                for (int v : S.vars) idx.push_back(cs.noff + v);
                for (int u : S.str) idx.push_back(cs.noff + u);
                val.insert(val.end(), S.linv.begin(), S.linv.end());
                val.insert(val.end(), S.l21.begin(), S.l21.end());
                byh[S.height].push_back((int32_t)nodes.size());
                nodes.push_back(d);
            }
        }
        std::vector<int32_t> list;
        c->ds_hwide.clear();
        for (auto& v : byh) {
            // variant by the largest supernode of the height: 0: 256 threads,
            // LDS for DS_SMALL unknowns; 1: 1024 threads (16 waves share the
            // rows of L11 and L21, each a latency-bound reduction) with the
            // same LDS; 2: 1024 threads, LDS for DS_MAXS unknowns
            int wide = 0;
            for (int32_t q : v) {
                const int sq = nodes[q].s, mq = nodes[q].m;
                const int kind = (sq > DS_SMALL || mq > DS_SMALL) ? 2 : (sq + mq > 128 ? 1 : 0);
                wide = std::max(wide, kind);
            }
            c->ds_hwide.push_back(wide);
            list.insert(list.end(), v.begin(), v.end());
            c->ds_hoff.push_back((int64_t)list.size());
        }
        TRY(h2d(c, c->d_ds_nodes, nodes));
        TRY(h2d(c, c->d_ds_idx, idx));
        TRY(h2d(c, c->d_ds_val, val));
        TRY(h2d(c, c->d_ds_cases, dcs));
        TRY(h2d(c, c->d_ds_list, list));
        if (cof != c->DSR) return fail(c, PDFMC_E_STATE, "projection factor updates differ from their reservation");
        for (size_t u = 1; u < ccnt.size(); ++u) ccnt[u] += ccnt[u - 1];
        std::vector<int32_t> clist((size_t)std::max<int64_t>(cof, 1), 0), pos(ccnt.begin(), ccnt.end() - 1);
        for (const auto& pr : cpairs) clist[(size_t)pos[pr.first]++] = pr.second;   // stable: supernode order
        TRY(h2d(c, c->d_ds_cptr, ccnt));
        TRY(h2d(c, c->d_ds_clist, clist));
    }
    c->proj_direct = c->proj_method == PDFMC_PROJ_DIRECT && c->n_amg > 0 && c->DSC == c->n_amg;
    // solver systems: one five-column relaxation system per mode-2 case,
    // then one projection system per mode-2 case
    c->h_amgdev = amgdev;
    TRY(build_mg_jobs(c));
    // state that starts at zero
    TRY(enqueue_fill(c, c->d_F, (int64_t)NN * NF));
    TRY(enqueue_fill(c, c->d_stats, (int64_t)NN * NST));
    TRY(enqueue_fill(c, c->d_er_x, (int64_t)NER * NN));
    TRY(enqueue_fill(c, c->d_phi, NN));
    TRY(enqueue_fill(c, c->d_P, NN));
    TRY(enqueue_fill(c, c->d_gphi, 2 * (int64_t)NN));
    TRY(enqueue_fill(c, c->d_pb, NN));
    TRY(enqueue_fill(c, c->d_mg_vec, c->MGV));
    TRY(enqueue_fill(c, c->d_mg_acc, (int64_t)(NER + 1) * c->cases.size() * MG_NSLOT * MG_SLOT));
    TRY(enqueue_fill_i(c, c->d_mg_state, (int64_t)(NER + 1) * c->cases.size() * 2));
    TRY(enqueue_fill_i(c, (int32_t*)c->d_mg_need, 1));
    TRY(enqueue_fill(c, (double*)c->d_counters, (int64_t)NCNT * c->cases.size()));
    TRY(enqueue_fill_i(c, (int32_t*)c->d_step, 1));
    if (c->any_er) {
        hipLaunchKernelGGL(k_stiffness_assemble, dim3(nblk(NN, 256)), dim3(256), 0, c->stream, node_args(c));
        LAUNCHCHK(c);
        for (int l = 0; l < AMG_MAXL; ++l) {
            TRY(enqueue_galerkin(c, c->d_gal + (size_t)(AMG_MAXL + l) * c->n_amg, c->n_gal_p[l], c->gal_max_p[l]));
            LAUNCHCHK(c);
        }
        // the projection hierarchies' inverse diagonals and coarsest inverses,
        // once: their matrices are constant
        if (c->n_tab_dinv > c->n_tab_dinv_er)
            hipLaunchKernelGGL(k_mg_dinv, dim3(c->n_tab_dinv - c->n_tab_dinv_er), dim3(256), 0, c->stream,
                               (const AmgDev*)c->d_amg, (const int4*)c->d_mg_tab_dinv + c->n_tab_dinv_er);
        if (c->n_amg > 0)
            hipLaunchKernelGGL(k_mg_coarse, dim3(c->n_amg), dim3(1024), 0, c->stream, (const AmgDev*)c->d_amg, 1, 2);
        LAUNCHCHK(c);
    }
    // the scatter's per-element lists and overflow sums start empty (the
    // element pass clears what it consumes)
    TRY(enqueue_fill_i(c, c->d_ecnt, c->NE));
    TRY(enqueue_fill_i(c, c->d_eof, c->NE));
    TRY(enqueue_fill(c, c->d_eo, (int64_t)c->NE * SC_VMAX));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->have_stats = false;
    // the static scratch of pdfmc_sort_noalloc on this device (set-up only;
    // a failed lookup fails that entry point, not the bind)
    c->d_static_scratch = nullptr;
    c->static_scratch_err.clear();
    hipError_t se = hipGetDevice(&c->device);
    if (se == hipSuccess) se = static_scratch_address(c->device, &c->d_static_scratch);
    if (se != hipSuccess) {
        c->d_static_scratch = nullptr;
        c->static_scratch_err = hipGetErrorString(se);
        (void)hipGetLastError();
    }
    c->bound = true;
    c->initialised = false;
    return PDFMC_OK;
}

pdfmc_status pdfmc_particles_upload(pdfmc_ctx* c, int32_t ci, const pdfmc_particles_host* p)
{
    TRY(check_case(c, ci));
    Case& cs = c->cases[ci];
    // the whole ensemble is checked on the host before any device work
    if (!p || p->n < 0 || p->n > cs.cap) return fail(c, PDFMC_E_INVALID, "particles_upload: n must be 0..capacity");
    if (!p->x || !p->y || !p->u || !p->v || !p->w || !p->omega || !p->weight || !p->elem || !p->id ||
        (cs.p.n_scalars > 0 && !p->psi))
        return fail(c, PDFMC_E_INVALID, "particles_upload: null array");
    const int64_t n = p->n;
    for (int64_t i = 0; i < n; ++i)
        if (p->elem[i] < 0 || p->elem[i] >= cs.m.ne)
            return fail(c, PDFMC_E_INVALID, "particles_upload: particle " + std::to_string(i) + " has element " +
                                                std::to_string(p->elem[i]) + " outside the case");
    if (p->bin)
        for (int64_t i = 0; i < n; ++i)
            if (p->bin[i] >= (cs.p.n_bins == 8 ? 8 : 1))
                return fail(c, PDFMC_E_INVALID, "particles_upload: particle " + std::to_string(i) + " has bin " +
                                                    std::to_string(p->bin[i]));
    for (int64_t i = 0; i < n; ++i) {
        const double vals[7] = {p->x[i], p->y[i], p->u[i], p->v[i], p->w[i], p->omega[i], p->weight[i]};
        static const char* names[7] = {"x", "y", "u", "v", "w", "omega", "weight"};
        for (int k = 0; k < 7; ++k)
            if (!std::isfinite(vals[k]))
                return fail(c, PDFMC_E_INVALID, std::string("particles_upload: particle ") + std::to_string(i) +
                                                    " has a non-finite " + names[k]);
        if (!(p->weight[i] > 0.0))
            return fail(c, PDFMC_E_INVALID, "particles_upload: particle " + std::to_string(i) +
                                                " has a mass weight that is not positive");
        for (int a = 0; a < cs.p.n_scalars; ++a)
            if (!std::isfinite(p->psi[(size_t)a * n + i]))
                return fail(c, PDFMC_E_INVALID, "particles_upload: particle " + std::to_string(i) +
                                                    " has a non-finite scalar " + std::to_string(a));
    }
    TRY(check_bound(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    PartBufs& B = c->part[c->cur];
    const size_t R = rsz(c);
    auto put = [&](char* dbase, int64_t off, const double* src, int64_t cnt) -> pdfmc_status {
        if (cnt == 0) return PDFMC_OK;
        char* dst = (char*)dbase + off * R;
        if (R == 8) {
            HIPCHK(c, hipMemcpy(dst, src, cnt * 8, hipMemcpyHostToDevice));
        } else {
            std::vector<float> tmp(src, src + cnt);
            HIPCHK(c, hipMemcpy(dst, tmp.data(), cnt * 4, hipMemcpyHostToDevice));
        }
        return PDFMC_OK;
    };
    TRY(put(B.x, cs.poff, p->x, n)); TRY(put(B.y, cs.poff, p->y, n));
    TRY(put(B.u, cs.poff, p->u, n)); TRY(put(B.v, cs.poff, p->v, n)); TRY(put(B.w, cs.poff, p->w, n));
    TRY(put(B.om, cs.poff, p->omega, n)); TRY(put(B.wt, cs.poff, p->weight, n));
    for (int a = 0; a < cs.p.n_scalars; ++a) TRY(put(B.psi, cs.psioff + a * cs.cap, p->psi + a * n, n));
    std::vector<int32_t> el(n);
    for (int64_t i = 0; i < n; ++i) el[i] = p->elem[i] + cs.eoff;
    std::vector<uint8_t> bins(n, 0);
    if (p->bin) std::copy(p->bin, p->bin + n, bins.begin());
    if (n) {
        HIPCHK(c, hipMemcpy(B.elem + cs.poff, el.data(), n * 4, hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(B.id + cs.poff, p->id, n * 4, hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(B.bin + cs.poff, bins.data(), n, hipMemcpyHostToDevice));
    }
    cs.np = n;
    CaseDev d = make_case_dev(c, cs);
    HIPCHK(c, hipMemcpy(c->d_cases + ci, &d, sizeof d, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemset(c->d_counters + (int64_t)ci * NCNT, 0, NCNT * sizeof(unsigned long long)));
    return PDFMC_OK;
}

pdfmc_status pdfmc_particles_init(pdfmc_ctx* c, int32_t ci, int32_t ppe, const pdfmc_init_params* ip)
{
    TRY(check_case(c, ci));
    Case& cs = c->cases[ci];
    if (!ip) return fail(c, PDFMC_E_INVALID, "particles_init: null parameters");
    if (ppe < 1) return fail(c, PDFMC_E_INVALID, "particles_init: ppe must be >= 1");
    const int64_t n = (int64_t)cs.m.ne * ppe;
    if (n > cs.cap)
        return fail(c, PDFMC_E_INVALID, "particles_init: " + std::to_string(n) + " particles exceed the capacity " +
                                            std::to_string(cs.cap));
    if (!(std::isfinite(ip->u_std) && ip->u_std >= 0.0))
        return fail(c, PDFMC_E_INVALID, "particles_init: u_std must be finite and >= 0");
    if (!(std::isfinite(ip->omega_scale) && ip->omega_scale > 0.0))
        return fail(c, PDFMC_E_INVALID, "particles_init: omega_scale must be finite and > 0");
    for (int a = 0; a < PDFMC_MAX_SCALARS; ++a)
        for (int j = 0; j < 4; ++j)
            if (!std::isfinite(ip->disk[a][j])) return fail(c, PDFMC_E_INVALID, "particles_init: non-finite disk");
    TRY(check_bound(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    cs.np = n;
    CaseDev d = make_case_dev(c, cs);
    HIPCHK(c, hipMemcpy(c->d_cases + ci, &d, sizeof d, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemset(c->d_counters + (int64_t)ci * NCNT, 0, NCNT * sizeof(unsigned long long)));
    if (n > 0) {
        PartBufs& B = c->part[c->cur];
        auto launch = [&](auto tag) -> pdfmc_status {
            using R = decltype(tag);
            InitArgs<R> A{};
            A.P = Particles<R>{(R*)B.x, (R*)B.y, (R*)B.u, (R*)B.v, (R*)B.w, (R*)B.om, (R*)B.wt, (R*)B.psi, B.elem, B.id, B.bin};
            A.cases = c->d_cases; A.exy = c->d_exy64; A.area = c->d_area;
            A.n = n; A.cs = ci; A.ppe = ppe; A.u_std = ip->u_std; A.omega_scale = ip->omega_scale;
            for (int a = 0; a < MAXS; ++a)
                for (int j = 0; j < 4; ++j) A.disk[a][j] = a < cs.p.n_scalars ? ip->disk[a][j] : 0.0;
            hipLaunchKernelGGL(k_particles_init<R>, dim3(nblk(n, 256)), dim3(256), 0, c->stream, A);
            LAUNCHCHK(c);
            return PDFMC_OK;
        };
        if (c->prec == PDFMC_FP64) TRY(launch(double{}));
        else TRY(launch(float{}));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PDFMC_OK;
}

pdfmc_status pdfmc_particles_download(pdfmc_ctx* c, int32_t ci, pdfmc_particles_host* p)
{
    TRY(check_case(c, ci));
    TRY(check_bound(c));
    Case& cs = c->cases[ci];
    if (!p || p->n != cs.np) return fail(c, PDFMC_E_INVALID, "particles_download: n must equal the uploaded count");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    PartBufs& B = c->part[c->cur];
    const size_t R = rsz(c);
    const int64_t n = cs.np;
    auto get = [&](const char* dbase, int64_t off, double* dst, int64_t cnt) -> pdfmc_status {
        if (!dst || cnt == 0) return PDFMC_OK;
        const char* src = (const char*)dbase + off * R;
        if (R == 8) {
            HIPCHK(c, hipMemcpy(dst, src, cnt * 8, hipMemcpyDeviceToHost));
        } else {
            std::vector<float> tmp(cnt);
            HIPCHK(c, hipMemcpy(tmp.data(), src, cnt * 4, hipMemcpyDeviceToHost));
            std::copy(tmp.begin(), tmp.end(), dst);
        }
        return PDFMC_OK;
    };
    TRY(get(B.x, cs.poff, p->x, n)); TRY(get(B.y, cs.poff, p->y, n));
    TRY(get(B.u, cs.poff, p->u, n)); TRY(get(B.v, cs.poff, p->v, n)); TRY(get(B.w, cs.poff, p->w, n));
    TRY(get(B.om, cs.poff, p->omega, n)); TRY(get(B.wt, cs.poff, p->weight, n));
    if (p->psi)
        for (int a = 0; a < cs.p.n_scalars; ++a) TRY(get(B.psi, cs.psioff + a * cs.cap, p->psi + a * n, n));
    if (n) {
        if (p->elem) {
            HIPCHK(c, hipMemcpy(p->elem, B.elem + cs.poff, n * 4, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < n; ++i) p->elem[i] -= cs.eoff;
        }
        if (p->id) HIPCHK(c, hipMemcpy(p->id, B.id + cs.poff, n * 4, hipMemcpyDeviceToHost));
        if (p->bin) HIPCHK(c, hipMemcpy(p->bin, B.bin + cs.poff, n, hipMemcpyDeviceToHost));
    }
    return PDFMC_OK;
}

pdfmc_status pdfmc_fields_upload(pdfmc_ctx* c, int32_t ci, const double* F, uint32_t freeze_mask)
{
    TRY(check_case(c, ci));
    if (!F) return fail(c, PDFMC_E_INVALID, "fields_upload: null");
    if (freeze_mask >> NF) return fail(c, PDFMC_E_INVALID, "fields_upload: freeze_mask has bits above slot 21");
    Case& cs = c->cases[ci];
    for (int64_t i = 0; i < (int64_t)cs.m.nn * NF; ++i)
        if (!std::isfinite(F[i])) return fail(c, PDFMC_E_INVALID, "fields_upload: non-finite field value");
    TRY(check_bound(c));
    std::vector<double> tmp((size_t)cs.m.nsn * NF);
    for (int s = 0; s < cs.m.nsn; ++s) std::copy(F + (size_t)cs.m.rep[s] * NF, F + (size_t)cs.m.rep[s] * NF + NF, &tmp[(size_t)s * NF]);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->d_F + (size_t)cs.noff * NF, tmp.data(), tmp.size() * 8, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_Ffrz + (size_t)cs.noff * NF, tmp.data(), tmp.size() * 8, hipMemcpyHostToDevice));
    if (cs.freeze != freeze_mask) {
        cs.freeze = freeze_mask;
        CaseDev d = make_case_dev(c, cs);
        HIPCHK(c, hipMemcpy(c->d_cases + ci, &d, sizeof d, hipMemcpyHostToDevice));
        c->any_freeze = false;
        for (auto& k : c->cases) c->any_freeze |= k.freeze != 0;
        drop_graphs(c);
    }
    TRY(enqueue_fields_elem(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PDFMC_OK;
}

pdfmc_status pdfmc_fields_download(pdfmc_ctx* c, int32_t ci, double* F)
{
    TRY(check_case(c, ci));
    TRY(check_bound(c));
    if (!F) return fail(c, PDFMC_E_INVALID, "fields_download: null");
    const Case& cs = c->cases[ci];
    std::vector<double> tmp((size_t)cs.m.nsn * NF);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(tmp.data(), c->d_F + (size_t)cs.noff * NF, tmp.size() * 8, hipMemcpyDeviceToHost));
    for (int i = 0; i < cs.m.nn; ++i)
        std::copy(&tmp[(size_t)cs.m.snode[i] * NF], &tmp[(size_t)cs.m.snode[i] * NF] + NF, F + (size_t)i * NF);
    return PDFMC_OK;
}

pdfmc_status pdfmc_pressure_download(pdfmc_ctx* c, int32_t ci, double* P)
{
    TRY(check_case(c, ci));
    TRY(check_bound(c));
    if (!P) return fail(c, PDFMC_E_INVALID, "pressure_download: null");
    const Case& cs = c->cases[ci];
    std::vector<double> tmp(std::max(cs.m.nsn, 1));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(tmp.data(), c->d_P + cs.noff, cs.m.nsn * 8, hipMemcpyDeviceToHost));
    for (int i = 0; i < cs.m.nn; ++i) P[i] = tmp[cs.m.snode[i]];
    return PDFMC_OK;
}

pdfmc_status pdfmc_init(pdfmc_ctx* c)
{
    if (!c) return PDFMC_E_INVALID;
    TRY(check_bound(c));
    // statistics of the uploaded state
    TRY(enqueue_accum_clear(c));
    TRY(enqueue_particles(c, 0, 0, 1, true));
    c->have_stats = true;
    // Eulerian fields (no projection at initialisation: <P> starts at 0)
    TRY(enqueue_fields(c, false));
    // bins and cell means against those fields (the statistics pass is
    // repeated with the same sums, so the node statistics do not change)
    TRY(enqueue_accum_clear(c));
    TRY(enqueue_particles(c, 0, 1, 1, false));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->initialised = true;
    return PDFMC_OK;
}

pdfmc_status pdfmc_rebin(pdfmc_ctx* c)
{
    if (!c) return PDFMC_E_INVALID;
    TRY(check_bound(c));
    TRY(enqueue_fields_elem(c));
    TRY(enqueue_accum_clear(c));
    TRY(enqueue_particles(c, 0, 1, 1, false));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->initialised = true;
    return PDFMC_OK;
}

// The side stream and the events that fork the sort off the main stream and
// join it back (default priority, like the main stream).
static pdfmc_status ensure_side_stream(pdfmc_ctx* c)
{
    if (c->side) return PDFMC_OK;
    HIPCHK(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    return PDFMC_OK;
}

pdfmc_status pdfmc_step(pdfmc_ctx* c, int32_t n_steps, uint32_t stage_mask)
{
    if (!c) return PDFMC_E_INVALID;
    if (n_steps < 0) return fail(c, PDFMC_E_INVALID, "step: n_steps < 0");
    if (stage_mask & ~(uint32_t)PDFMC_STAGE_ALL) return fail(c, PDFMC_E_INVALID, "step: unknown stage bits");
    TRY(check_bound(c));
    if (!c->initialised) return fail(c, PDFMC_E_STATE, "step: call pdfmc_init (or pdfmc_rebin) first");
    if (stage_mask != c->graph_stages) {
        drop_graphs(c);
        c->graph_stages = stage_mask;
    }
    TRY(ensure_side_stream(c));
    for (int s = 0; s < n_steps; ++s) {
        TRY(mg_adapt(c));
        // the periodic sort comes at the end of the step after which it is
        // due, so that it overlaps the fields phase
        const bool sort_after = c->sort_interval > 0 && c->ntiles > 0 && c->steps_since_sort + 1 >= c->sort_interval;
        const int cur0 = c->cur;
        if (c->use_graph && !c->timing) {
            hipGraphExec_t& g = c->graph[cur0][sort_after ? 1 : 0];
            if (!g) {
                hipGraph_t graph = nullptr;
                HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
                pdfmc_status st = enqueue_step_body(c, stage_mask, sort_after);
                hipError_t e2 = hipStreamEndCapture(c->stream, &graph);
                c->cur = cur0;           // the replay below performs the step
                if (st != PDFMC_OK) { if (graph) (void)hipGraphDestroy(graph); return st; }
                if (e2 != hipSuccess) return fail(c, PDFMC_E_HIP, std::string("graph capture: ") + hipGetErrorString(e2));
                hipError_t e3 = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e3 != hipSuccess) { g = nullptr; return fail(c, PDFMC_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e3)); }
            }
            HIPCHK(c, hipGraphLaunch(g, c->stream));
            if (sort_after) c->cur = 1 - cur0;    // the graph's sort wrote the other buffer set
        } else {
            TRY(enqueue_step_body(c, stage_mask, sort_after));
        }
        TRY(mg_after_step(c));
        c->steps_since_sort = sort_after ? 0 : c->steps_since_sort + 1;
    }
    return PDFMC_OK;
}

pdfmc_status pdfmc_set_step_index(pdfmc_ctx* c, uint32_t n)
{
    if (!c) return PDFMC_E_INVALID;
    TRY(check_bound(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->d_step, &n, 4, hipMemcpyHostToDevice));
    return PDFMC_OK;
}

pdfmc_status pdfmc_stats_readback(pdfmc_ctx* c, int32_t ci, double* out)
{
    TRY(check_case(c, ci));
    TRY(check_bound(c));
    if (!out) return fail(c, PDFMC_E_INVALID, "stats_readback: null");
    const Case& cs = c->cases[ci];
    const int ns = cs.p.n_scalars, nst = 12 + 2 * ns;
    std::vector<double> tmp((size_t)std::max(cs.m.nsn, 1) * NST);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(tmp.data(), c->d_stats + (size_t)cs.noff * NST, (size_t)cs.m.nsn * NST * 8, hipMemcpyDeviceToHost));
    for (int i = 0; i < cs.m.nn; ++i) {
        const double* s = &tmp[(size_t)cs.m.snode[i] * NST];
        std::copy(s, s + nst, out + (size_t)i * nst);
    }
    return PDFMC_OK;
}

pdfmc_status pdfmc_node_sums(pdfmc_ctx* c, int32_t ci, double* out)
{
    TRY(check_case(c, ci));
    TRY(check_bound(c));
    if (!out) return fail(c, PDFMC_E_INVALID, "node_sums: null");
    const Case& cs = c->cases[ci];
    const int ns = cs.p.n_scalars, nq = 12 + 2 * ns;
    std::vector<double> tmp((size_t)std::max(cs.m.nsn, 1) * NQ);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(tmp.data(), c->d_nsum + (size_t)cs.noff * NQ, (size_t)cs.m.nsn * NQ * 8, hipMemcpyDeviceToHost));
    for (int i = 0; i < cs.m.nn; ++i) {
        const double* s = &tmp[(size_t)cs.m.snode[i] * NQ];
        std::copy(s, s + nq, out + (size_t)i * nq);
    }
    return PDFMC_OK;
}

pdfmc_status pdfmc_cell_means(pdfmc_ctx* c, int32_t ci, double* mean, int32_t* count)
{
    TRY(check_case(c, ci));
    TRY(check_bound(c));
    const Case& cs = c->cases[ci];
    const int ns = cs.p.n_scalars;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (mean && ns > 0) {
        const size_t cnt = (size_t)cs.m.ne * 8 * ns;
        if (c->prec == PDFMC_FP64) {
            HIPCHK(c, hipMemcpy(mean, (double*)c->d_cmean + cs.cmoff, cnt * 8, hipMemcpyDeviceToHost));
        } else {
            std::vector<float> tmp(cnt);
            HIPCHK(c, hipMemcpy(tmp.data(), (float*)c->d_cmean + cs.cmoff, cnt * 4, hipMemcpyDeviceToHost));
            std::copy(tmp.begin(), tmp.end(), mean);
        }
    }
    if (count) HIPCHK(c, hipMemcpy(count, c->d_ccnt + 8 * (size_t)cs.eoff, 8 * (size_t)cs.m.ne * 4, hipMemcpyDeviceToHost));
    return PDFMC_OK;
}

pdfmc_status pdfmc_counters(pdfmc_ctx* c, int32_t ci, int64_t* out)
{
    TRY(check_case(c, ci));
    TRY(check_bound(c));
    if (!out) return fail(c, PDFMC_E_INVALID, "counters: null");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(out, c->d_counters + (int64_t)ci * NCNT, NCNT * 8, hipMemcpyDeviceToHost));
    return PDFMC_OK;
}

pdfmc_status pdfmc_set_options(pdfmc_ctx* c, int32_t sort_interval, int32_t block_size, int32_t use_graph)
{
    if (!c) return PDFMC_E_INVALID;
    if (sort_interval < 0) return fail(c, PDFMC_E_INVALID, "set_options: sort_interval < 0");
    // a workgroup must not straddle two particle tiles (two cases)
    if (block_size != 64 && block_size != 128 && block_size != 256)
        return fail(c, PDFMC_E_INVALID, "set_options: block size must be 64, 128 or 256");
    if (use_graph && c->stream == nullptr)
        return fail(c, PDFMC_E_INVALID, "set_options: graph capture needs a stream other than the default (NULL) stream");
    if (block_size != c->block) drop_graphs(c);
    c->sort_interval = sort_interval;
    c->block = block_size;
    c->use_graph = use_graph ? 1 : 0;
    return PDFMC_OK;
}

pdfmc_status pdfmc_set_solver(pdfmc_ctx* c, int32_t iterations, int32_t tail_rows)
{
    if (!c) return PDFMC_E_INVALID;
    if (iterations < 0 || iterations > 100000) return fail(c, PDFMC_E_INVALID, "set_solver: iterations must be 0..100000");
    if (tail_rows < 0) return fail(c, PDFMC_E_INVALID, "set_solver: tail_rows must be >= 0");
    const bool retable = tail_rows != c->tail_rows;
    c->mg_auto = iterations == 0 ? 1 : 0;
    if (iterations > 0 && iterations != c->mg_iters) { c->mg_iters = iterations; drop_graphs(c); }
    if (iterations > 0) {
        // a fixed count: every system runs it in the phases
        c->ksw.assign(c->ksw.size(), iterations);
        c->ksw_low.assign(c->ksw_low.size(), 0);
        if (c->bound && !c->h_jobs.empty()) {
            for (auto& J : c->h_jobs) J.ksw = std::min(iterations, J.maxit);
            TRY(h2d(c, c->d_mg_jobs, c->h_jobs));
        }
    }
    c->tail_rows = tail_rows;
    if (retable && c->bound) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        drop_graphs(c);
        TRY(build_mg_jobs(c));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return PDFMC_OK;
}

pdfmc_status pdfmc_solver_info(pdfmc_ctx* c, int32_t* iterations, int32_t* large_levels)
{
    if (!c) return PDFMC_E_INVALID;
    if (iterations) *iterations = c->mg_iters;
    if (large_levels) *large_levels = c->proj_direct ? c->maxbig_er : c->maxbig_all;
    return PDFMC_OK;
}

pdfmc_status pdfmc_set_projection_solver(pdfmc_ctx* c, int32_t method)
{
    if (!c) return PDFMC_E_INVALID;
    if (method != PDFMC_PROJ_DIRECT && method != PDFMC_PROJ_PCG)
        return fail(c, PDFMC_E_INVALID, "set_projection_solver: method must be PDFMC_PROJ_DIRECT or PDFMC_PROJ_PCG");
    c->proj_method = method;
    if (c->bound) {
        const bool direct = method == PDFMC_PROJ_DIRECT && c->n_amg > 0 && c->DSC == c->n_amg;
        if (direct != c->proj_direct) {
            HIPCHK(c, hipStreamSynchronize(c->stream));
            drop_graphs(c);
            c->proj_direct = direct;
        }
    }
    return PDFMC_OK;
}

pdfmc_status pdfmc_projection_info(pdfmc_ctx* c, int32_t* method, int32_t* height, int64_t* factor_values)
{
    if (!c) return PDFMC_E_INVALID;
    const bool direct = c->bound ? c->proj_direct
                                 : (c->proj_method == PDFMC_PROJ_DIRECT && c->n_amg > 0 && c->DSC == c->n_amg);
    if (method) *method = direct ? PDFMC_PROJ_DIRECT : PDFMC_PROJ_PCG;
    if (height) *height = c->ds_height;
    if (factor_values) *factor_values = c->DSV;
    return PDFMC_OK;
}

pdfmc_status pdfmc_sort(pdfmc_ctx* c)
{
    if (!c) return PDFMC_E_INVALID;
    TRY(check_bound(c));
    TRY(enqueue_sort(c, sort_scratch_ws(c)));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PDFMC_OK;
}

pdfmc_status pdfmc_sort_noalloc(pdfmc_ctx* c)
{
    if (!c) return PDFMC_E_INVALID;
    TRY(check_bound(c));
    const uint64_t need = sort_scratch_carve(nullptr, c->NE, c->NP, nullptr);
    if (need > (uint64_t)PDFMC_SORT_NOALLOC_BYTES)
        return fail(c, PDFMC_E_INVALID, "sort_noalloc: the sort needs " + std::to_string(need) +
                                            " bytes of scratch, the static scratch holds " +
                                            std::to_string((uint64_t)PDFMC_SORT_NOALLOC_BYTES) + " (use pdfmc_sort)");
    if (!c->d_static_scratch)
        return fail(c, PDFMC_E_HIP, "sort_noalloc: no device address for the static scratch: " + c->static_scratch_err);
    SortScratch T{};
    sort_scratch_carve((char*)c->d_static_scratch, c->NE, c->NP, &T);
    return enqueue_sort(c, T);
}

pdfmc_status pdfmc_synchronize(pdfmc_ctx* c)
{
    if (!c) return PDFMC_E_INVALID;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PDFMC_OK;
}

pdfmc_status pdfmc_timing(pdfmc_ctx* c, int32_t enable)
{
    if (!c) return PDFMC_E_INVALID;
    c->timing = enable != 0;
    c->ev_used = 0;
    return PDFMC_OK;
}

pdfmc_status pdfmc_timing_read(pdfmc_ctx* c, double* total_ms, int64_t* launches)
{
    if (!c || !total_ms || !launches) return PDFMC_E_INVALID;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double sum = 0.0;
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
        sum += ms;
    }
    *total_ms = sum;
    *launches = (int64_t)(c->ev_used / 2);
    c->ev_used = 0;
    return PDFMC_OK;
}

// Milliseconds of n steps with the options in force (one untimed step first,
// which also captures a new graph when graphs are enabled).
static pdfmc_status tune_time(pdfmc_ctx* c, int n, double* ms)
{
    TRY(pdfmc_step(c, 1, PDFMC_STAGE_ALL));
    hipEvent_t a = nullptr, b = nullptr;
    HIPCHK(c, hipEventCreate(&a));
    HIPCHK(c, hipEventCreate(&b));
    pdfmc_status st = PDFMC_OK;
    float f = 0.0f;
    if (hipEventRecord(a, c->stream) != hipSuccess) st = fail(c, PDFMC_E_HIP, "autotune: event record");
    if (st == PDFMC_OK) st = pdfmc_step(c, n, PDFMC_STAGE_ALL);
    if (st == PDFMC_OK && hipEventRecord(b, c->stream) != hipSuccess) st = fail(c, PDFMC_E_HIP, "autotune: event record");
    if (st == PDFMC_OK && hipEventSynchronize(b) != hipSuccess) st = fail(c, PDFMC_E_HIP, "autotune: event sync");
    if (st == PDFMC_OK && hipEventElapsedTime(&f, a, b) != hipSuccess) st = fail(c, PDFMC_E_HIP, "autotune: elapsed");
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = f;
    return st;
}

pdfmc_status pdfmc_autotune(pdfmc_ctx* c, int32_t steps_per_trial, pdfmc_tune_result* out)
{
    if (!c) return PDFMC_E_INVALID;
    TRY(check_bound(c));
    if (!c->initialised) return fail(c, PDFMC_E_STATE, "autotune: call pdfmc_init first");
    if (steps_per_trial < 1 || steps_per_trial > 1000) return fail(c, PDFMC_E_INVALID, "autotune: steps_per_trial must be 1..1000");
    if (c->timing) return fail(c, PDFMC_E_STATE, "autotune: disable timing first");
    int best_b = c->block, best_s = c->sort_interval > 0 ? c->sort_interval : 10, best_t = c->tail_rows;
    double best = 1e300;
    int trials = 0, steps = 0;
    auto trial = [&](int b, int s, int t, int n, double& per) -> pdfmc_status {
        TRY(pdfmc_set_options(c, s, b, c->use_graph));
        TRY(pdfmc_set_solver(c, c->mg_auto ? 0 : c->mg_iters, t));
        double ms = 0.0;
        TRY(tune_time(c, n, &ms));
        per = ms / n;
        ++trials;
        steps += n + 1;
        return PDFMC_OK;
    };
    // coordinate descent: block size, then sort interval, then the small-level threshold
    const int blocks[] = {64, 128, 256};
    const int sorts[] = {1, 2, 5, 10, 20};
    const int tails[] = {0, 64, 256, 512, 1024, 2048};
    for (int b : blocks) {
        double per;
        TRY(trial(b, best_s, best_t, std::max(steps_per_trial, best_s), per));
        if (per < best) { best = per; best_b = b; }
    }
    best = 1e300;
    for (int s : sorts) {
        double per;
        TRY(trial(best_b, s, best_t, std::max(steps_per_trial, 2 * s), per));
        if (per < best) { best = per; best_s = s; }
    }
    best = 1e300;
    for (int t : tails) {
        double per;
        TRY(trial(best_b, best_s, t, std::max(steps_per_trial, best_s), per));
        if (per < best) { best = per; best_t = t; }
    }
    TRY(pdfmc_set_options(c, best_s, best_b, c->use_graph));
    TRY(pdfmc_set_solver(c, c->mg_auto ? 0 : c->mg_iters, best_t));
    if (out) {
        out->block_size = best_b;
        out->sort_interval = best_s;
        out->tail_rows = best_t;
        out->trials = trials;
        out->steps = steps;
        out->ms_per_step = best;
    }
    return PDFMC_OK;
}

pdfmc_status pdfmc_draw_gaussians(pdfmc_ctx* c, uint64_t seed, uint32_t step, uint32_t stream, const uint32_t* ids,
                                  int64_t n, void* out)
{
    if (!c) return PDFMC_E_INVALID;
    if (n < 0 || (n > 0 && (!ids || !out))) return fail(c, PDFMC_E_INVALID, "draw_gaussians: bad arguments");
    if (n == 0) return PDFMC_OK;
    if (c->prec == PDFMC_FP64)
        hipLaunchKernelGGL(k_draw_gaussians<double>, dim3(nblk(n, 256)), dim3(256), 0, c->stream, (uint32_t)seed,
                           (uint32_t)(seed >> 32), step, stream, ids, n, (double*)out);
    else
        hipLaunchKernelGGL(k_draw_gaussians<float>, dim3(nblk(n, 256)), dim3(256), 0, c->stream, (uint32_t)seed,
                           (uint32_t)(seed >> 32), step, stream, ids, n, (float*)out);
    LAUNCHCHK(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PDFMC_OK;
}

}  // extern "C"
