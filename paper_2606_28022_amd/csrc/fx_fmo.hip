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

__global__ void k_max_absdiff(const double* a, const double* b, int n, double* out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, fabs(a[i] - b[i]));
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

}  // namespace fx
