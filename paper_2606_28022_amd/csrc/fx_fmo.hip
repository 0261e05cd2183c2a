// FMO bookkeeping kernels: moving shell charges between the supersystem and
// the fragment batches, the dimer/trimer terms of the many-body energy, and
// the fixed-order energy sum.
//
// Cluster terms (section "Fragment molecular orbital method"): the charge
// transfer ddq = dq^X - (dq^I + dq^J (+ dq^K)) of eq. ddq_calc / ctijk, the
// embedding correction Delta E^V = ddq . phi^X of eqs.
// dimer_embedding_correction and trimer_embedding, and the interaction
// energy Delta E_X = E_X - sum E_I + Delta E^V of eqs.
// fmo2-energy-components and trimer_interaction_energy.
#include <hip/hip_runtime.h>

#include "fx_device.hpp"
#include "fx_kernels.hpp"

namespace fx {

__global__ void k_gather_shell(DevBatch bt, const double* src_global, double* dst_local) {
  int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  for (int s = threadIdx.x; s < d.nsh; s += blockDim.x)
    dst_local[d.sh_off + s] = src_global[bt.sys_sh_global[d.sh_off + s]];
}

__global__ void k_scatter_shell(DevBatch bt, const double* src_local, double* dst_global) {
  int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  for (int s = threadIdx.x; s < d.nsh; s += blockDim.x)
    dst_global[bt.sys_sh_global[d.sh_off + s]] = src_local[d.sh_off + s];
}

// max |a - b| in two stages: one partial per work-group (grid-stride), then
// one work-group over the partials (the maximum does not depend on the order)
__global__ void k_absdiff_part(const double* a, const double* b, int n, double* part) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) m = fmax(m, fabs(a[i] - b[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_max_reduce(const double* part, int np, double* out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) m = fmax(m, part[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// per cluster system: ddq (written per local shell), Delta E^V and Delta E_X
__global__ void k_cluster_terms(DevBatch bt, const double* qmono, const double* e_mono, double* ddq, double* dEV,
                                double* dE) {
  int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  __shared__ double red[256];
  double loc = 0.0;
  for (int s = threadIdx.x; s < d.nsh; s += blockDim.x) {
    double v = bt.q_out[d.sh_off + s] - qmono[bt.sys_sh_global[d.sh_off + s]];
    ddq[d.sh_off + s] = v;
    loc += v * bt.phi[d.sh_off + s];
  }
  red[threadIdx.x] = loc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double ev = red[0];
    double e = bt.e_int[si];
    for (int k = 0; k < d.nfrag; ++k) e -= e_mono[d.frag[k]];
    dEV[si] = ev;
    dE[si] = e + ev;
  }
}

// Neumaier-compensated sum of several arrays in a fixed order: 256 threads
// each sum a contiguous slice of the concatenated sequence, thread 0 then
// adds the 256 partial sums in order.  Deterministic for a given input.
__device__ inline void neu_add(double& s, double& c, double v) {
  double t = s + v;
  if (fabs(s) >= fabs(v)) c += (s - t) + v;
  else c += (v - t) + s;
  s = t;
}

__global__ void k_sum_neumaier(const double* const* arrays, const long long* lens, int narrays, double* out) {
  __shared__ double ps[256], pc[256];
  long long total = 0;
  for (int k = 0; k < narrays; ++k) total += lens[k];
  long long per = (total + blockDim.x - 1) / blockDim.x;
  long long b = per * threadIdx.x, e = b + per < total ? b + per : total;
  double s = 0.0, c = 0.0;
  long long base = 0;
  for (int k = 0; k < narrays; ++k) {
    long long lo = b > base ? b : base;
    long long hi = e < base + lens[k] ? e : base + lens[k];
    for (long long i = lo; i < hi; ++i) neu_add(s, c, arrays[k][i - base]);
    base += lens[k];
  }
  ps[threadIdx.x] = s;
  pc[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    double S = 0.0, C = 0.0;
    for (int t = 0; t < (int)blockDim.x; ++t) {
      neu_add(S, C, ps[t]);
      neu_add(S, C, pc[t]);
    }
    *out = S + C;
  }
}

// ---------------------------------------------------------------------------
// Anderson (Pulay) mixing of a long vector (the monomer charges of the
// self-consistent embedding).  History slots are passed oldest first.
// B_ij = r_i . r_j, one work-group per (i, j), fixed-order tree reduction
// Gram matrix of the history residuals in one pass over them: each
// work-group accumulates all m (m + 1) / 2 products of its slice (grid-stride)
// and writes them to part[block][HIST_TRI]; k_hist_solve adds the partials in
// block order (deterministic).
constexpr int HIST_TRI = HIST * (HIST + 1) / 2;
__global__ void __launch_bounds__(256) k_hist_gram_part(const double* R, long long n, Slots sl, double* part) {
  const int m = sl.m;
  double acc[HIST_TRI];
#pragma unroll
  for (int t = 0; t < HIST_TRI; ++t) acc[t] = 0.0;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
    double r[HIST];
#pragma unroll
    for (int i = 0; i < HIST; ++i) r[i] = i < m ? R[(long long)sl.id[i] * n + k] : 0.0;
    int t = 0;
#pragma unroll
    for (int i = 0; i < HIST; ++i)
#pragma unroll
      for (int j = i; j < HIST; ++j) acc[t++] += r[i] * r[j];
  }
  __shared__ double red[4][HIST_TRI];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < HIST_TRI; ++t) {
    double v = acc[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[wave][t] = v;
  }
  __syncthreads();
  if (threadIdx.x < HIST_TRI)
    part[(long long)blockIdx.x * HIST_TRI + threadIdx.x] =
        red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

// B_ij from the partials (block order), then the mixing coefficients:
// minimise |sum c_k r_k| subject to sum c_k = 1 (bordered normal equations,
// Gaussian elimination with partial pivoting, in LDS by one thread)
__global__ void k_hist_solve(const double* part, int np, Slots sl, double* coef) {
  const int m = sl.m, M = m + 1;
  __shared__ double tri[HIST_TRI];
  __shared__ double A[(HIST + 1) * (HIST + 1)], rhs[HIST + 1];
  for (int t = threadIdx.x; t < HIST_TRI; t += blockDim.x) {
    double v = 0.0;
    for (int p = 0; p < np; ++p) v += part[(long long)p * HIST_TRI + t];
    tri[t] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  auto Bij = [&](int i, int j) {
    const int a = i < j ? i : j, b = i < j ? j : i;
    return tri[a * HIST - a * (a - 1) / 2 + (b - a)];  // row a of the packed upper triangle
  };
  double tr = 0.0;
  for (int i = 0; i < m; ++i) tr += Bij(i, i);
  for (int i = 0; i < M; ++i) {
    rhs[i] = (i == m) ? 1.0 : 0.0;
    for (int j = 0; j < M; ++j) {
      double v;
      if (i < m && j < m) v = Bij(i, j) + (i == j ? 1e-14 * tr : 0.0);
      else if (i == m && j == m) v = 0.0;
      else v = 1.0;
      A[i * M + j] = v;
    }
  }
  for (int c = 0; c < M; ++c) {
    int piv = c;
    for (int r = c + 1; r < M; ++r)
      if (fabs(A[r * M + c]) > fabs(A[piv * M + c])) piv = r;
    if (piv != c) {
      for (int k = 0; k < M; ++k) {
        double t = A[c * M + k];
        A[c * M + k] = A[piv * M + k];
        A[piv * M + k] = t;
      }
      double t = rhs[c];
      rhs[c] = rhs[piv];
      rhs[piv] = t;
    }
    double dv = A[c * M + c];
    if (fabs(dv) < 1e-300) dv = 1e-300;
    for (int r = c + 1; r < M; ++r) {
      double f = A[r * M + c] / dv;
      for (int k = c; k < M; ++k) A[r * M + k] -= f * A[c * M + k];
      rhs[r] -= f * rhs[c];
    }
  }
  for (int c = M - 1; c >= 0; --c) {
    double v = rhs[c];
    for (int k = c + 1; k < M; ++k) v -= A[c * M + k] * rhs[k];
    double dv = A[c * M + c];
    rhs[c] = v / (fabs(dv) < 1e-300 ? 1e-300 : dv);
  }
  for (int i = 0; i < m; ++i) coef[i] = rhs[i];
}

// q = sum_k c_k (x_k + beta r_k)
__global__ void k_hist_mix(const double* X, const double* R, long long n, Slots sl, const double* coef, double beta,
                           double* q) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double v = 0.0;
  for (int i = 0; i < sl.m; ++i) {
    long long o = (long long)sl.id[i] * n + k;
    v += coef[i] * (X[o] + beta * R[o]);
  }
  q[k] = v;
}

// store x and r = y - x into history slot `slot`, and max |r| into *dmax
__global__ void k_hist_store(const double* x, const double* y, long long n, int slot, double* X, double* R) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  X[(long long)slot * n + k] = x[k];
  R[(long long)slot * n + k] = y[k] - x[k];
}

// Trimer corrections Delta E_IJK - Delta E_IJ - Delta E_IK - Delta E_JK
// (eq. fmo3_energy; an ES-DIM sub-pair enters with its ES-DIM value): sub
// holds, per trimer, the three sub-pairs as an index into dE_scc or nscc +
// an index into dE_esd.
__global__ void k_trimer_corr(long long ntri, const double* dEIJK, const double* dE_scc, long long nscc,
                              const double* dE_esd, const long long* sub, double* out) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= ntri) return;
  double v = dEIJK[k];
  for (int p = 0; p < 3; ++p) {
    const long long e = sub[3 * k + p];
    v -= e < nscc ? dE_scc[e] : dE_esd[e - nscc];
  }
  out[k] = v;
}

}  // namespace fx
