// Declarations of the kernels launched by the host library.
#pragma once
#include "pdfmc_dev.h"
#include "pdfmc_nodes.h"
#include "pdfmc_sort.h"

namespace pdfmc {

template <typename R> __global__ void k_particle_step(StepArgs<R> A);
template <typename R> __global__ void k_particles_init(InitArgs<R> A);
template <typename R> __global__ void k_draw_gaussians(uint32_t slo, uint32_t shi, uint32_t step, uint32_t stream,
                                                       const uint32_t* ids, int64_t n, R* out);
__global__ void k_fill_f64(double* a, int64_t n, double v);
__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v);
__global__ void k_step_increment(uint32_t* step);
__global__ void k_scatter_register(NodeArgs A, int ntiles, int block, const int32_t* tile_case, const int32_t* pool_cnt,
                                   int pool_cap, unsigned long long* counters, int cells_on);
template <typename R> __global__ void k_elem_reduce(NodeArgs A, R* cmean, int cells_on, int rebin_only);
__global__ void k_node_reduce(NodeArgs A);
__global__ void k_fields_grad(NodeArgs A);
__global__ void k_fields_derived(NodeArgs A);
__global__ void k_er_assemble(NodeArgs A);
__global__ void k_stiffness_assemble(NodeArgs A);
__global__ void k_er_finish(NodeArgs A);
__global__ void k_proj_rhs(NodeArgs A);
__global__ void k_proj_update(NodeArgs A);
__global__ void k_proj_grad(NodeArgs A);
__global__ void k_fields_freeze(const CaseDev* cases, const int32_t* node_case, const double* Ffrz, double* F, int nn);
template <typename R> __global__ void k_fields_elem(const double* F, const double* gphi, const int4* tri_s, R* Fel, int ne);
__global__ void k_mg_dinv(const AmgDev* hs, const int4* tab);
__global__ void k_mg_coarse(const AmgDev* hs, int first, int stride);
__global__ void k_mg_setup1(const MgJob* jobs, const int4* tab, const int32_t* st);
__global__ void k_mg_setup2(const MgJob* jobs, const AmgDev* hs, const int4* tab, const int32_t* st);
__global__ void k_mg_pa(const MgJob* jobs, const AmgDev* hs, const int4* tab, const int32_t* st, int k);
__global__ void k_mg_pb(const MgJob* jobs, const AmgDev* hs, const int4* tab, const int32_t* st, int k, int first);
__global__ void k_mg_res(const MgJob* jobs, const AmgDev* hs, const int4* tab, const int32_t* st, int l, int k);
__global__ void k_mg_restrict(const MgJob* jobs, const AmgDev* hs, const int4* tab, const int32_t* st, int l, int k);
__global__ void k_mg_pre(const MgJob* jobs, const AmgDev* hs, const int4* tab, const int32_t* st, int l, int k);
__global__ void k_mg_tail(const MgJob* jobs, const AmgDev* hs, const int32_t* st, int k);
__global__ void k_mg_prolong(const MgJob* jobs, const AmgDev* hs, const int4* tab, const int32_t* st, int l, int k);
__global__ void k_mg_post1(const MgJob* jobs, const AmgDev* hs, const int4* tab, const int32_t* st, int l, int k);
__global__ void k_mg_post2(const MgJob* jobs, const AmgDev* hs, const int4* tab, const int32_t* st, int l, int k);
__global__ void k_mg_finish(const MgJob* jobs, const AmgDev* hs, int k0);
__global__ void k_mg_reduce(const MgJob* jobs, const AmgDev* hs, const int32_t* st, int k, int word0, int M, int setup,
                            int big_only);
__global__ void k_galerkin(const GalJob* jobs);
__global__ void k_ds_prep(const DsCase* cs, const double* b, double* x);
template <int DSB, int CAP>
__global__ void k_ds_forward(const DsNode* nodes, const int32_t* list, const int32_t* idx, const double* val, double* x,
                             DsUpd U);
template <int DSB, int CAP>
__global__ void k_ds_backward(const DsNode* nodes, const int32_t* list, const int32_t* idx, const double* val, double* x);
__global__ void k_ds_post(const DsCase* cs, double* x);
__global__ void k_sort_hist(SortArgs A);
__global__ void k_sort_scan_blocks(SortArgs A);
__global__ void k_sort_scan_totals(SortArgs A, int nb);
__global__ void k_sort_cursor(SortArgs A);
__global__ void k_sort_place(SortArgs A, const uint32_t* ids);
__global__ void k_sort_order(SortArgs A);
__global__ void k_sort_order_big(SortArgs A);
template <typename R> __global__ void k_sort_gather(SortArgs A, Particles<R> src, Particles<R> dst);

}  // namespace pdfmc
