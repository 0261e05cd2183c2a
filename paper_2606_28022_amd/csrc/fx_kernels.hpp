// Kernel declarations shared by the kernel sources and the host driver.
#pragma once

#include <hip/hip_runtime.h>

#include "fx_device.hpp"

namespace fx {

// integrals / lists / fields (fx_integrals.hip)
__global__ void k_cn(DevSystem sys, int nchunk, double* part);
__global__ void k_pair_contacts(DevSystem sys, const int* frag_atoms, const int* frag_off, int rule, double cut2,
                                double lam2, double lam3, int8_t* flag);
__global__ void k_build_system(DevSystem sys, DevBatch bt, const int* list, DevBatch mono, int from_mono);
__global__ void k_field_partial(DevSystem sys, const double* q, int nchunk, double* part);
__global__ void k_field_partial_f32(DevSystem sys, const double* q, int nchunk, double* part);
__global__ void k_field_reduce(int nshells, int nchunk, const double* part, double* phi);
__global__ void k_field_sym(DevSystem sys, const double* q, int group, int ngmax, double* rowpart, double* colpart);
__global__ void k_field_sym_reduce(DevSystem sys, int group, int ngmax, const double* rowpart,
                                   const double* colpart, double* phi);
__global__ void k_cluster_phi(DevSystem sys, DevBatch bt, const double* Phi, const double* qmono);
__global__ void k_esd_pairs(DevSystem sys, const int* pairs, long long npairs, const int* frag_atoms,
                            const int* frag_off, const double* q, double* out);

// SCC (fx_scc.hip)
__global__ void k_cluster_healed(DevSystem sys, DevBatch bt, const double* Phi, const double* qmono, double* dEV,
                                 double* dE);
__global__ void k_vhop(DevBatch bt, double vhop);
__global__ void k_ghost_cn(DevSystem sys, const int* bonds, int nbonds, double* cn);
__global__ void k_reset_state(DevBatch bt, const int* list, int nl, int keep_err);
__global__ void k_hist_reset(DevBatch bt, const int* list, int nl);
// work-groups of a launch over nl systems of tps tiles each, numbered by
// xcd_slot_tile: 8 ceil(nl / 8) tps
inline long long xcd_grid(int nl, int tps) { return 8LL * ((nl + 7) / 8) * tps; }
__global__ void k_compact_active(const int* status, const int* list, int nl, int* act, int* count);
__global__ void k_precond_step(DevBatch bt, double* out);
__global__ void k_cholinv(DevBatch bt, const int* list, const double* Apool, double* Lpool, double* Xpool);
__global__ void k_cluster_init_ct(DevBatch bt, const int* list, DevBatch mono, const long long* warm_off);
__global__ void k_warm_start(DevBatch bt, const long long* mat_off_old, const long long* sh_off_old,
                             const double* Cold, const double* qold);
__global__ void k_fock(DevSystem sys, DevBatch bt, const int* list);
__global__ void k_fock_f32(DevSystem sys, DevBatch bt, const int* list, const float* H0f, const float* Sf, float* Ff);
__global__ void k_to_f32(const double* src, float* dst, long long n);
template <int MODE, typename TA, typename TB, typename TC>
__global__ void k_gemm_f32(DevBatch bt, const int* list, int nl, int tiles_per_sys, const TA* Abase, const TB* Bbase,
                           TC* Cbase, const double* wbase, int skip_done, int sym, int occ_list);
// k_precond_build runs 1024 threads (16 waves); each thread holds PRE_ROWS x
// PRE_COLS elements of K, so systems of up to 192 shells
// (ROWS = PRE_ROWS_SMALL for up to 16 PRE_ROWS_SMALL shells: fewer
// accumulators, no register spills)
constexpr int PRE_ROWS = 12, PRE_ROWS_SMALL = 9, PRE_COLS = 3, PRE_THREADS = 1024;
constexpr int PRE_MAXSH = 16 * PRE_ROWS < 64 * PRE_COLS ? 16 * PRE_ROWS : 64 * PRE_COLS;
template <int ROWS>
__global__ void k_precond_build(DevSystem sys, DevBatch bt, const int* list, DevBatch mono, const double* Mmono,
                                float* pre, int* ok);
__global__ void k_mirror_tiles(DevBatch bt, const int* list, double* Abase);
template <int MODE, int WIN>
__global__ void k_gemm_mfma(DevBatch bt, const int* list, int nl, int tiles_per_sys, const double* Abase,
                            const double* Bbase, double* Cbase, const double* wbase, int skip_done, int sym,
                            int occ_list);
__global__ void k_gemm(DevBatch bt, const int* list, int mode, const double* A, const double* B, double* C,
                       const double* w, int skip_done);
__global__ void k_jacobi(DevBatch bt, const int* list, int max_sweeps, double rel_tol, double thr_scale,
                         double cap_err, int* sweeps_out);
// LDS layout of k_jacobi_lds for an n x n system: packed strict upper
// triangle (elt bytes per element), FP64 diagonal, `chunk` steps of rotation
// log, an nw-column tile of V and the reduction slots (16-byte aligned parts).
struct JacobiLdsLayout {
  unsigned ap, dg, cs, pq, vt, red, total;
};
__host__ __device__ inline unsigned jl_align(unsigned x) { return (x + 15u) & ~15u; }
__host__ __device__ inline JacobiLdsLayout jacobi_lds_layout(int n, int elt, int chunk, int nw) {
  const unsigned nb = (unsigned)(n + (n & 1)) / 2;
  JacobiLdsLayout L;
  unsigned o = 0;
  L.ap = o;
  o = jl_align(o + (unsigned)n * (unsigned)(n - 1) / 2u * (unsigned)elt);
  L.dg = o;
  o = jl_align(o + 8u * (unsigned)n);
  L.cs = o;
  o = jl_align(o + 16u * (unsigned)chunk * nb);
  L.pq = o;
  o = jl_align(o + 4u * (unsigned)chunk * nb);
  L.vt = o;
  o = jl_align(o + 8u * (unsigned)nw * (unsigned)(n + 1));
  L.red = o;
  o = jl_align(o + 8u * 64u);
  L.total = o;
  return L;
}
// LDS of k_jacobi_rot: 2 x 2 tiles of the upper block triangle (m/2 (m/2 + 1)
// / 2 tiles of four elt-byte elements, m = n rounded up to a multiple of
// four), FP64 diagonal (m), (c, s) of the block step and of two consecutive
// rounds (double2; the FP32 form keeps the rounds' as two float4 per
// quartet), the quartets' blocks of two rounds, the table of quartet pairs,
// a reduction slot
struct JacobiRotLayout {
  unsigned ap, dg, cs, csf, qr, pt, red, total;
};
__host__ __device__ inline JacobiRotLayout jacobi_rot_layout(int n, int elt) {
  const unsigned m = (unsigned)(n + 3) & ~3u, nb2 = m / 2u;
  JacobiRotLayout L;
  unsigned o = 0;
  L.ap = o;
  o = jl_align(o + nb2 * (nb2 + 1u) / 2u * 4u * (unsigned)elt);
  L.dg = o;
  o = jl_align(o + 8u * m);
  L.cs = o;  // block step, and (FP64 form) the quartets of two rounds
  o = jl_align(o + (elt == 4 ? 16u * m : 32u * m));
  L.csf = o;  // FP32 form: the quartets of two rounds
  o = jl_align(o + (elt == 4 ? 16u * m : 0u));
  L.qr = o;  // per quartet of two rounds: its blocks X | Y << 16, sign bit: rotates
  o = jl_align(o + 8u * (m / 4u));
  L.pt = o;  // quartet pairs a | b << 8 (| 1 << 16: wave 0's) of the off-diagonal pass
  o = jl_align(o + 4u * (m / 4u) * (m / 4u - 1u) / 2u);
  L.red = o;
  o = jl_align(o + 8u * 64u);
  L.total = o;
  return L;
}
size_t apply_rot_lds_bytes(int n);
int apply_rot_tile(int n);  // columns per work-group of k_apply_rot (64 or 128)
int apply_rot_waves(int n);
long long jacobi_rot_log_entries(int n);  // rotation log entries per sweep
template <typename T>
__global__ void k_cholinv_lds(DevBatch bt, const int* list, const double* Apool, double* Xpool);
__global__ void k_ns_poly(DevBatch bt, const int* list, double* Hpool, const double* H2pool);
size_t cholinv_lds_bytes(int n, int elt);
__global__ void k_cholinv_block2(DevBatch bt, const int* list, DevBatch mono, const double* Apool, double* Xpool);
size_t cholinv_block2_lds_bytes(int n1, int n2);
constexpr int CHOL_THREADS_HOST = 1024;
template <typename T>
__global__ void k_jacobi_rot(DevBatch bt, const int* list, int max_sweeps, double rel_tol, double thr_scale,
                             double cap_err, double early_err, int early_sweeps, int* sweeps_out, double2* logbuf,
                             long long log_stride, int max_log, int* nlog, int* queue, int nl);
__global__ void k_queue_reset(int* queue);
__global__ void k_apply_rot(DevBatch bt, const int* list, int nl, int tiles_per_sys, int tile_w,
                            const double2* logbuf, long long log_stride, const int* nlog);
// two quartets per lane, for systems of 129 to 256 AOs: 512 threads, 64-column tiles
__global__ void k_apply_rot_dual(DevBatch bt, const int* list, int nl, int tiles_per_sys, const double2* logbuf,
                                 long long log_stride, const int* nlog);
size_t apply_rot_dual_lds_bytes(int n);
template <typename T>
__global__ void k_jacobi_lds(DevBatch bt, const int* list, int max_sweeps, double rel_tol, double thr_scale,
                             double cap_err, int* sweeps_out, int chunk);
__global__ void k_eigh_batched(const int* nvec, const long long* off, double* Abuf, double* Vbuf, double* wbuf,
                               const long long* woff, int max_sweeps, double rel_tol);
__global__ void k_fermi(DevSystem sys, DevBatch bt, const int* list);
__global__ void k_charges_mix(DevSystem sys, DevBatch bt, const int* list, double tol, double etol, int max_iter,
                              double beta);

// FMO assembly (fx_fmo.hip)
__global__ void k_gather_shell(DevBatch bt, const double* src_global, double* dst_local);
__global__ void k_scatter_shell(DevBatch bt, const double* src_local, double* dst_global);
__global__ void k_absdiff_part(const double* a, const double* b, int n, double* part);
__global__ void k_max_reduce(const double* part, int np, double* out);
__global__ void k_cluster_terms(DevBatch bt, const double* qmono, const double* e_mono, double* ddq, double* dEV,
                                double* dE);
__global__ void k_sum_neumaier(const double* const* arrays, const long long* lens, int narrays, double* out);
__global__ void k_hist_gram_part(const double* R, long long n, Slots sl, double* part);
__global__ void k_hist_solve(const double* part, int np, Slots sl, double* coef);
__global__ void k_hist_mix(const double* X, const double* R, long long n, Slots sl, const double* coef, double beta,
                           double* q);
__global__ void k_hist_store(const double* x, const double* y, long long n, int slot, double* X, double* R);

// response and gradient kernels
__global__ void k_mo_order(DevBatch bt, const int* nocc, int* order);
__global__ void k_resp_Q(DevSystem sys, DevBatch bt, const double* SCt, const int* order, const int* nocc,
                         const long long* qoff, double* Q);
__global__ void k_resp_M(DevBatch bt, const int* order, const int* nocc, const long long* qoff, const double* Q,
                         double* M);
size_t resp_M_lds_bytes(int nsh);
// k_resp_M_mfma: systems of at most 16 RMM_MAXB shells
constexpr int RMM_MAXB = 8;
__global__ void k_resp_M_mfma(DevBatch bt, const int* order, const int* nocc, const long long* qoff, const double* Q,
                              double* M);
size_t resp_M_mfma_lds_bytes(int nsh);
constexpr int RQ_CH = 16;        // AOs per staged run of k_resp_Q
size_t resp_Q_lds_bytes(int n);  // dynamic LDS of k_resp_Q for systems of up to n AOs
__global__ void k_resp_R(DevSystem sys, DevBatch bt, const double* M, double* Wk, double* R);
// k_resp_R_lds: systems of at most MAXN_RESP_LDS shells (the matrix in LDS)
constexpr int MAXN_RESP_LDS = 96, RR_THREADS = 512;
__global__ void k_resp_R_lds(DevSystem sys, DevBatch bt, const double* M, double* R);
__global__ void k_resp_apply(DevBatch bt, const double* R, const double* M, const double* y, double* w, double* u);
__global__ void k_resp_Z(DevBatch bt, const int* order, const int* nocc, const long long* qoff, const double* Q,
                         const double* w, double* Zm, double* Ze);
__global__ void k_rowscale(DevBatch bt, const double* wsh, const double* P, double* out);
__global__ void k_sym_inplace(DevBatch bt, double* A);
__global__ void k_resp_DS(DevBatch bt, const double* Zb, const double* WZ, const double* X2, const double* wsh,
                          double* DS, double* gx);
__global__ void k_trimer_corr(long long ntri, const double* dEIJK, const double* dE_scc, long long nscc,
                              const double* dE_esd, const long long* sub, double* out);
__global__ void k_cluster_cross(DevSystem sys, DevBatch bt, const double* x, const double* qmono, const double* w,
                                double* out, double* out_gh);
__global__ void k_sub_healed(DevBatch bt, const double* vgh, double* v);
__global__ void k_gather_csr(int n, const int* rowptr, const int* ent, const double* src, const double* base,
                             double sign, double* dst);
__global__ void k_axpy(long long n, const double* x, double a, const double* y, double* out);
__global__ void k_grad_contract(DevSystem sys, DevBatch bt, const int* list, const double* DHp, const double* DSp,
                                const double* gx, const double* gy, const double* wsys, int with_rep, int accumulate,
                                double* g_out, double* F_out, double* scratch);
__global__ void k_grad_pair_corr(DevSystem sys, DevBatch bt, const double* qmono, const double* ddq,
                                 const double* wct, const int* qqmask, double* g_out, double* ghost_out);
__global__ void k_hop_grad(DevSystem sys, DevBatch bt, const double* Dmp, double* DSp, const double* wsys,
                           const int* bonds, double V, long long slot_base, double* hop_f);
__global__ void k_healed_ct(DevBatch bt, const double* w, const double* qmono, double* qbar);
__global__ void k_add_ext_forces(int N, int NB, const int* bonds, const double* f_ext, double* grad);
__global__ void k_scale_cluster(DevBatch bt, const double* w, const double* src, double* dst);
__global__ void k_force_inter(DevSystem sys, const double* q, const double* av, int nchunk, double* part);
__global__ void k_force_reduce(int N, int nchunk, const double* part, double* out);
__global__ void k_cn_grad(DevSystem sys, const double* Ftot, int nchunk, double* part);
__global__ void k_gather_atoms(int N, const int* rowptr, const int* ent_batch, const long long* ent_off,
                               const double* const* g_batches, const double* const* F_batches, double* g_tot,
                               double* F_tot, int mode);
__global__ void k_final_shift(DevSystem sys, DevBatch bt, double* wvec);
__global__ void k_make_DS(DevBatch bt, const double* P, const double* W, double* out);

// learned initial guess
__global__ void k_mlp_features(DevSystem sys, float* out);
__global__ void k_mlp_forward(const float* wr, const float* X, float* Y, long long n);
__global__ void k_mlp_grad_partial(const float* wr, const float* X, const float* Yl, long long n, float* part,
                                   double* loss_part);
__global__ void k_mlp_grad_reduce(const float* part, int nparts, float* grad);
__global__ void k_mlp_loss_reduce(const double* loss_part, int nparts, double inv_count, double* out);
__global__ void k_mlp_adam(float* master, float* m, float* v, const float* g, int t, float lr, float* wr);
__global__ void k_mlp_round(const float* master, float* wr);
__global__ void k_guess_assemble(DevSystem sys, const float* Y, double* q);
__global__ void k_guess_project(DevSystem sys, const int* frag_atoms, const int* frag_off, const int* frag_charge,
                                double* q);
__global__ void k_guess_fallback(DevBatch bt, const int* list, int nl, int phase, double tau, int* flag);
}  // namespace fx
