// Kernel declarations shared by the kernel sources and the host driver.
#pragma once

#include <hip/hip_runtime.h>

#include "fx_device.hpp"

namespace fx {

// integrals / lists / fields (fx_integrals.hip)
__global__ void k_cn(DevSystem sys, double* cn_out);
__global__ void k_pair_contacts(DevSystem sys, const int* frag_atoms, const int* frag_off, double cut2,
                                int8_t* flag);
__global__ void k_build_system(DevSystem sys, DevBatch bt, const int* list);
__global__ void k_field_partial(DevSystem sys, const double* q, int nchunk, double* part);
__global__ void k_field_reduce(int nshells, int nchunk, const double* part, double* phi);
__global__ void k_cluster_phi(DevSystem sys, DevBatch bt, const double* Phi, const double* qmono);
__global__ void k_esd_pairs(DevSystem sys, const int* pairs, long long npairs, const int* frag_atoms,
                            const int* frag_off, const double* q, double* out);

// SCC (fx_scc.hip)
__global__ void k_reset_state(DevBatch bt, const int* list, int nl);
__global__ void k_cholinv(DevBatch bt, const int* list, const double* Apool, double* Lpool, double* Xpool);
__global__ void k_cluster_init_ct(DevBatch bt, const int* list, DevBatch mono);
__global__ void k_fock(DevSystem sys, DevBatch bt, const int* list);
__global__ void k_gemm_mfma(DevBatch bt, const int* list, int nl, int tiles_per_sys, int mode, const double* A,
                            const double* B, double* C, const double* w);
__global__ void k_gemm(DevBatch bt, const int* list, int mode, const double* A, const double* B, double* C,
                       const double* w);
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
__global__ void k_max_absdiff(const double* a, const double* b, int n, double* out);
__global__ void k_cluster_terms(DevBatch bt, const double* qmono, const double* e_mono, double* ddq, double* dEV,
                                double* dE);
__global__ void k_sum_neumaier(const double* const* arrays, const long long* lens, int narrays, double* out);
__global__ void k_hist_gram(const double* R, long long n, Slots sl, double* B);
__global__ void k_hist_coef(const double* B, Slots sl, double* coef);
__global__ void k_hist_mix(const double* X, const double* R, long long n, Slots sl, const double* coef, double beta,
                           double* q);
__global__ void k_hist_store(const double* x, const double* y, long long n, int slot, double* X, double* R);

}  // namespace fx
