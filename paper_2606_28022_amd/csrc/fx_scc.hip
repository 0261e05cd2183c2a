// SCC iteration kernels for batches of fragment systems (monomers, dimers,
// trimers).  One iteration (section "GFN1-xTB"):
//   sigma_s = sum_t gamma_st q_t - Gamma_A q_A^2 + phi_s       (k_fock)
//   F = H0 + 1/2 S (sigma_mu + sigma_nu)                        (k_fock)
//   A = C^T F C in the current S-orthonormal basis C            (k_gemm x2)
//   Jacobi rotations diagonalise A and rotate C                 (k_jacobi)
//   Fermi-Dirac occupations, eps_F by bisection                 (k_fermi)
//   P = C diag(n) C^T                                           (k_gemm TN)
//   Mulliken shell charges, energy, Anderson mixing, test       (k_charges_mix)
// Because C stays S-orthonormal, the generalized problem F C = S C eps is
// solved without refactoring S; the first basis is C = L^-T with S = L L^T
// (k_cholinv).  C is stored transposed (eigenvectors as rows).
#include <hip/hip_runtime.h>

#include "fx_device.hpp"
#include "fx_kernels.hpp"

#include <algorithm>

namespace fx {

// sum over the work-group (blockDim a multiple of 64, at most 1024): a
// butterfly within each wave, then the wave totals in order; every thread
// gets the same value
__device__ inline double block_sum_waves(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();  // red may still be read by a previous reduction
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  return t;
}

__device__ inline double block_sum(double v, double* red) {
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

__device__ inline double block_max(double v, double* red) {
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// maximum over the work-group in the same way as block_sum_waves
__device__ inline double block_max_waves(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  __syncthreads();  // red may still be read by a previous reduction
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) t = fmax(t, red[w]);
  return t;
}

// ---------------------------------------------------------------------------
// start of a solve: clear the iteration state of the listed systems
// (keep_err: the residual of the previous pass stays, so the eigensolver's
// rotation threshold follows the outer iteration)
__global__ void k_reset_state(DevBatch bt, const int* list, int nl, int keep_err) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nl) return;
  int si = list[k];
  bt.status[si] = 0;
  bt.niter[si] = 0;
  bt.nhist[si] = 0;
  bt.e_prev[si] = 0.0;
  if (!keep_err) bt.err[si] = 1e-2;
}

// clear the Anderson history of the listed systems
__global__ void k_hist_reset(DevBatch bt, const int* list, int nl) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nl) bt.nhist[list[k]] = 0;
}

// Stable partition of the list by status, on the device: the systems still
// iterating (status 0) first, in list order, then the others, in list order;
// *count = the number of the former.  One work-group of 1024 threads: each
// thread takes a contiguous chunk of the list, and a scan over the chunk
// counts places it.  Every list entry is written, so a kernel launched over
// more slots than *count finds converged systems there and returns.
__global__ void __launch_bounds__(1024) k_compact_active(const int* status, const int* list, int nl, int* act,
                                                         int* count) {
  __shared__ int part[1024];
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = (nl + nt - 1) / nt;
  const int lo = min(nl, t * per), hi = min(nl, lo + per);
  int na = 0;
  for (int i = lo; i < hi; ++i) na += status[list[i]] == 0 ? 1 : 0;
  part[t] = na;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  const int total = part[nt - 1];
  int pa = part[t] - na;        // active entries before this chunk
  int pi = total + (lo - pa);   // inactive ones go after all active ones
  for (int i = lo; i < hi; ++i) {
    const int si = list[i];
    if (status[si] == 0)
      act[pa++] = si;
    else
      act[pi++] = si;
  }
  if (t == 0) *count = total;
}

// Preconditioned monomer step of the fused embedding loop, per system:
// out = q_in + (1 + M G)^-1 (q_out - q_in) (local shell vectors)
__global__ void k_precond_step(DevBatch bt, double* out) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int ns = d.nsh;
  __shared__ double r[MAXN];
  const double* qi = bt.q_in + d.sh_off;
  const double* qo = bt.q_out + d.sh_off;
  for (int s = threadIdx.x; s < ns; s += blockDim.x) r[s] = qo[s] - qi[s];
  __syncthreads();
  const float* Pr = bt.pre + d.gam_off;
  for (int s = threadIdx.x; s < ns; s += blockDim.x) {
    double v = 0.0;
#pragma unroll 8
    for (int t = 0; t < ns; ++t) v += (double)Pr[(long long)t * ns + s] * r[t];  // stored transposed
    out[d.sh_off + s] = qi[s] + v;
  }
}

// initial basis of a cluster from its monomers' eigenvectors: block-diagonal
// rows of the monomer C^T (fragment order), later S-orthonormalised.
__global__ void k_cluster_init_ct(DevBatch bt, const int* list, DevBatch mono, const long long* warm_off) {
  int si = list[blockIdx.x];
  if (warm_off && warm_off[si] >= 0) return;  // started from the previous run's orbitals
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  double* C = bt.Ct + d.mat_off;
  // fragment f's rows and columns: co[f] .. co[f + 1] - 1 (its monomer's C^T
  // there, zeros elsewhere); a wave per row, lanes along it (every element
  // written once, row segments coalesced)
  int co[4] = {0, 0, 0, 0};
  const double* Cm[3] = {nullptr, nullptr, nullptr};
  for (int f = 0; f < d.nfrag; ++f) {
    const SysDesc* m = mono.desc + d.frag[f];
    Cm[f] = mono.Ct + m->mat_off;
    co[f + 1] = co[f] + m->nao;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  for (int i = wave; i < n; i += nwv) {
    const int fi = (i >= co[1]) + (d.nfrag > 2 && i >= co[2]);
    const int a = co[fi], nm = co[fi + 1] - a;
    const double* src = Cm[fi] + (long long)(i - a) * nm;
    double* dst = C + (long long)i * n;
    for (int j = lane; j < n; j += 64) dst[j] = (j >= a && j < a + nm) ? src[j - a] : 0.0;
  }
}

// Start of a cluster from its converged solution of the previous run (same
// fragments, hence the same matrix order): C^T and the input charges are
// copied from that run's batch layout (offsets < 0: no previous solution).
__global__ void k_warm_start(DevBatch bt, const long long* mat_off_old, const long long* sh_off_old,
                             const double* Cold, const double* qold) {
  const int si = blockIdx.x;
  const long long mo = mat_off_old[si];
  if (mo < 0) return;
  const SysDesc d = bt.desc[si];
  const long long nn = (long long)d.nao * d.nao;
  double* C = bt.Ct + d.mat_off;
  for (long long i = threadIdx.x; i < nn; i += blockDim.x) C[i] = Cold[mo + i];
  const long long so = sh_off_old[si];
  for (int s = threadIdx.x; s < d.nsh; s += blockDim.x) bt.q_in[d.sh_off + s] = qold[so + s];
}

// ---------------------------------------------------------------------------
// X = L^-1 for an SPD matrix A = L L^T (pools: A read, L workspace, X out).
// With A = S the rows of L^-1 are the first S-orthonormal basis C = L^-T.
__global__ void k_cholinv(DevBatch bt, const int* list, const double* Apool, double* Lpool, double* Xpool) {
  int si = list[blockIdx.x];
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  double* L = Lpool + d.mat_off;
  const double* S = Apool + d.mat_off;
  double* X = Xpool + d.mat_off;
  __shared__ double piv;
  for (long long i = threadIdx.x; i < (long long)n * n; i += blockDim.x) L[i] = S[i];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      double v = L[(long long)k * n + k];
      piv = v > 0.0 ? sqrt(v) : -1.0;
      if (v <= 0.0) bt.status[si] = 2;
      L[(long long)k * n + k] = piv;
    }
    __syncthreads();
    if (piv <= 0.0) return;
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) L[(long long)i * n + k] /= piv;
    __syncthreads();
    const int m = n - k - 1;
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
      int i = k + 1 + idx / m, j = k + 1 + idx % m;
      if (j <= i) L[(long long)i * n + j] -= L[(long long)i * n + k] * L[(long long)j * n + k];
    }
    __syncthreads();
  }
  // X = L^-1 by forward substitution, one column per thread
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    for (int i = 0; i < n; ++i) {
      if (i < j) {
        X[(long long)i * n + j] = 0.0;
        continue;
      }
      double v = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) v -= L[(long long)i * n + k] * X[(long long)k * n + j];
      X[(long long)i * n + j] = v / L[(long long)i * n + i];
    }
  }
}

// ---------------------------------------------------------------------------
// shell shift and Fock matrix

// Shell shifts sigma_s = sum_t gamma_st q_t - Gamma_A q_A^2 + phi_s of one
// system (FP64, also stored in bt.sig) and the shift of every AO (that of its
// shell) into sig_ao.  Called by every thread of the work-group.
__device__ void fock_shifts(const DevSystem& sys, const DevBatch& bt, const SysDesc& d, double* qa_s,
                            double* sig_s, double* sig_ao) {
  const int n = d.nao, ns = d.nsh;
  const double* q = bt.q_in + d.sh_off;
  for (int a = threadIdx.x; a < d.nat; a += blockDim.x) {
    int s0 = bt.sys_atom_sh0[d.atom_off + a];
    int A = bt.sys_atoms[d.atom_off + a];
    int nsa = sys.atom_sh0[A + 1] - sys.atom_sh0[A];
    double v = 0.0;
    for (int k = 0; k < nsa; ++k) v += q[s0 + k];
    qa_s[a] = v;
  }
  __syncthreads();
  const double* G = bt.gam + d.gam_off;
  for (int s = threadIdx.x; s < ns; s += blockDim.x) {
    double v = 0.0;
#pragma unroll 8
    for (int t = 0; t < ns; ++t) v += G[(long long)t * ns + s] * q[t];
    int a = bt.sys_sh_atom[d.sh_off + s];
    int A = bt.sys_atoms[d.atom_off + a];
    double Gam = sys.elems[sys.elem[A]].Gamma;
    v += -Gam * qa_s[a] * qa_s[a] + bt.phi[d.sh_off + s];
    sig_s[s] = v;
    bt.sig[d.sh_off + s] = v;
  }
  __syncthreads();
  const int* aosh = bt.sys_ao_sh + d.ao_off;
  for (int i = threadIdx.x; i < n; i += blockDim.x) sig_ao[i] = sig_s[aosh[i]];
  __syncthreads();
}

// Mixed-precision form of the Fock build (early SCC iterations): the shifts
// in FP64, F = H0 + 1/2 S (sigma_mu + sigma_nu) assembled in FP32 from the
// FP32 copies of H0 and S and stored in FP32 (upper 32 x 32 tiles, each
// written as itself and, through LDS, as its mirror).  Systems without
// hybrid-orbital projectors only.
__global__ void __launch_bounds__(256) k_fock_f32(DevSystem sys, DevBatch bt, const int* list,
                                                  const float* __restrict__ H0f, const float* __restrict__ Sf,
                                                  float* __restrict__ Ff) {
  int si = list[blockIdx.x];
  if (bt.status[si] != 0) return;
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  __shared__ double qa_s[MAXN], sig_s[MAXN], sig_ao[MAXN];
  fock_shifts(sys, bt, d, qa_s, sig_s, sig_ao);
  __shared__ float sa[MAXN];
  for (int i = threadIdx.x; i < n; i += blockDim.x) sa[i] = (float)sig_ao[i];
  __syncthreads();
  const float* S = Sf + d.mat_off;
  const float* H = H0f + d.mat_off;
  float* Fo = Ff + d.mat_off;
  __shared__ float tr[32][33];
  const int nt = (n + 31) / 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int I = 0; I < nt; ++I)
    for (int J = I; J < nt; ++J) {
      const int j = 32 * J + tx;
#pragma unroll
      for (int r = 0; r < 32; r += 8) {
        const int i = 32 * I + r + ty;
        if (i < n && j < n) {
          const long long e = (long long)i * n + j;
          const float f = H[e] + 0.5f * S[e] * (sa[i] + sa[j]);
          Fo[e] = f;
          tr[r + ty][tx] = f;
        }
      }
      if (I == J) continue;
      __syncthreads();
      const int ic = 32 * I + tx;
#pragma unroll
      for (int r = 0; r < 32; r += 8) {
        const int jr = 32 * J + r + ty;
        if (jr < n) Fo[(long long)jr * n + ic] = tr[tx][r + ty];
      }
      __syncthreads();
    }
}

// FP32 copies of a pool (mixed precision: H0 and S once per batch build)
__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

// part[w ns + s] = the sum over wave w's share of t of M[t ns + s] x[t], for
// s < ns (lanes: consecutive s, consecutive addresses; a wave's loads are
// independent, so many are in flight).  The caller adds the shares in wave
// order after a barrier.
template <typename T, typename X>
__device__ inline void matvec_wave_part(const T* M, const X* x, int ns, double* part) {
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, nwv = blockDim.x >> 6;
  const int tq = (ns + nwv - 1) / nwv, t0 = wv * tq, t1 = min(ns, t0 + tq);
  for (int s0 = 0; s0 < ns; s0 += 64) {
    const int s = s0 + ln;
    if (s < ns) {
      double v = 0.0;
#pragma unroll 8
      for (int t = t0; t < t1; ++t) v += (double)M[(long long)t * ns + s] * x[t];
      part[wv * ns + s] = v;
    }
  }
}

__global__ void k_fock(DevSystem sys, DevBatch bt, const int* list) {
  int si = list[blockIdx.x];
  if (bt.status[si] != 0) return;  // converged or failed: nothing to do
  const SysDesc d = bt.desc[si];
  const int n = d.nao, ns = d.nsh;
  __shared__ double qa_s[MAXN];
  __shared__ double sig_s[MAXN];
  const double* q = bt.q_in + d.sh_off;
  // atom charges
  for (int a = threadIdx.x; a < d.nat; a += blockDim.x) {
    int s0 = bt.sys_atom_sh0[d.atom_off + a];
    int A = bt.sys_atoms[d.atom_off + a];
    int nsa = sys.atom_sh0[A + 1] - sys.atom_sh0[A];
    double v = 0.0;
    for (int k = 0; k < nsa; ++k) v += q[s0 + k];
    qa_s[a] = v;
  }
  // per-wave transposition tiles of the F build; first the partial sums of
  // the shell shifts
  __shared__ double trw[4][32][33];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, nwv = blockDim.x >> 6;
  const double* G = bt.gam + d.gam_off;
  // (G q)_s = sum_t G_ts q_t (G stored exactly symmetric), by the waves'
  // shares of t, added in order
  matvec_wave_part(G, q, ns, &trw[0][0][0]);
  __syncthreads();
  for (int s = threadIdx.x; s < ns; s += blockDim.x) {
    const double* part = &trw[0][0][0];
    double v = 0.0;
    for (int w = 0; w < nwv; ++w) v += part[w * ns + s];
    int a = bt.sys_sh_atom[d.sh_off + s];
    int A = bt.sys_atoms[d.atom_off + a];
    double Gam = sys.elems[sys.elem[A]].Gamma;
    v += -Gam * qa_s[a] * qa_s[a] + bt.phi[d.sh_off + s];
    sig_s[s] = v;
    bt.sig[d.sh_off + s] = v;
  }
  __syncthreads();
  // the shift of each AO (that of its shell)
  __shared__ double sig_ao[MAXN];
  const int* aosh = bt.sys_ao_sh + d.ao_off;
  for (int i = threadIdx.x; i < n; i += blockDim.x) sig_ao[i] = sig_s[aosh[i]];
  __syncthreads();
  const double* S = bt.S + d.mat_off;
  const double* H = bt.H0 + d.mat_off;
  double* Fm = bt.F + d.mat_off;
  const double* Vh = bt.Vh ? bt.Vh + d.mat_off : nullptr;
  if (!Vh && blockDim.x == 256) {
    // H0 and S are stored exactly symmetric, so F is: only the upper 32 x 32
    // tiles are read, and each is written as itself and, through LDS, as its
    // mirror tile (2 n^2 instead of 3 n^2 elements of HBM traffic).  The
    // tiles are dealt to the waves in turn; a wave transposes its tile in its
    // own LDS tile, so the waves never wait for each other (a tile's 32 loads
    // per lane are in flight together)
    double (*tr)[33] = trw[wv];
    const int nt = (n + 31) / 32;
    const int tx = ln & 31, ty = ln >> 5;  // 2 rows of a tile per pass
    int tile = 0;
    for (int I = 0; I < nt; ++I)
      for (int J = I; J < nt; ++J, ++tile) {
        if ((tile & 3) != wv) continue;
        const int j = 32 * J + tx;
#pragma unroll 8
        for (int r = 0; r < 32; r += 2) {
          const int i = 32 * I + r + ty;
          if (i < n && j < n) {
            const long long e = (long long)i * n + j;
            const double f = H[e] + 0.5 * S[e] * (sig_ao[i] + sig_ao[j]);
            Fm[e] = f;
            tr[r + ty][tx] = f;
          }
        }
        if (I == J) continue;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int ic = 32 * I + tx;
#pragma unroll 8
        for (int r = 0; r < 32; r += 2) {
          const int jr = 32 * J + r + ty;
          if (jr < n) Fm[(long long)jr * n + ic] = tr[tx][r + ty];
        }
        // (before the wave's next tile overwrites its LDS tile)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    return;
  }
  // element idx = i n + j, (i, j) advanced incrementally (no division per
  // element); unrolled so that several loads per thread are in flight
  const int nn = n * n, step = blockDim.x;
  const int di = step / n, dj = step - di * n;
  int i = threadIdx.x / n, j = threadIdx.x - i * n;
#pragma unroll 4
  for (int idx = threadIdx.x; idx < nn; idx += step) {
    Fm[idx] = H[idx] + 0.5 * S[idx] * (sig_ao[i] + sig_ao[j]) + (Vh ? Vh[idx] : 0.0);
    i += di;
    j += dj;
    if (j >= n) {
      j -= n;
      ++i;
    }
  }
}

// ---------------------------------------------------------------------------
// Batched dense products of the systems' n x n matrices, 32 x 32 output tile
// per work-group (256 threads, 2 x 2 outputs each).  mode:
//   0  C = A B          1  C = A B^T          2  C = A^T diag(w) B (w = 1 if null)
__global__ void k_gemm(DevBatch bt, const int* list, int mode, const double* Abase, const double* Bbase,
                       double* Cbase, const double* wbase, int skip_done) {
  int si = list[blockIdx.y];
  if (skip_done && bt.status[si] != 0) return;
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  const int nt = (n + 31) / 32;
  if ((int)blockIdx.x >= nt * nt) return;
  const int ti = blockIdx.x / nt, tj = blockIdx.x % nt;
  const double* A = Abase + d.mat_off;
  const double* B = Bbase + d.mat_off;
  double* C = Cbase + d.mat_off;
  const double* w = wbase ? wbase + d.ao_off : nullptr;
  __shared__ double As[32][33];  // [k][i]
  __shared__ double Bs[32][33];  // [k][j]
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[2][2] = {{0, 0}, {0, 0}};
  for (int k0 = 0; k0 < n; k0 += 32) {
    for (int e = threadIdx.x; e < 1024; e += 256) {
      int r = e / 32, c = e % 32;
      // A tile element (i = ti*32 + ?, k = k0 + ?)
      double av = 0.0, bv = 0.0;
      if (mode == 2) {
        // A^T: As[k][i] = A[k][i] * w[k]
        int k = k0 + r, i = ti * 32 + c;
        if (k < n && i < n) av = A[(long long)k * n + i] * (w ? w[k] : 1.0);
        int kb = k0 + r, j = tj * 32 + c;
        if (kb < n && j < n) bv = B[(long long)kb * n + j];
        As[r][c] = av;
        Bs[r][c] = bv;
      } else {
        // A: As[k][i] = A[i][k]; read A row i = ti*32 + r, column k = k0 + c
        int i = ti * 32 + r, k = k0 + c;
        if (i < n && k < n) av = A[(long long)i * n + k];
        As[c][r] = av;
        if (mode == 0) {
          int kb = k0 + r, j = tj * 32 + c;
          if (kb < n && j < n) bv = B[(long long)kb * n + j];
          Bs[r][c] = bv;
        } else {
          int j = tj * 32 + r, kb = k0 + c;
          if (j < n && kb < n) bv = B[(long long)j * n + kb];
          Bs[c][r] = bv;
        }
      }
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < 32; ++k) {
      double a0 = As[k][ty], a1 = As[k][ty + 16];
      double b0 = Bs[k][tx], b1 = Bs[k][tx + 16];
      acc[0][0] += a0 * b0;
      acc[0][1] += a0 * b1;
      acc[1][0] += a1 * b0;
      acc[1][1] += a1 * b1;
    }
    __syncthreads();
  }
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      int i = ti * 32 + ty + 16 * u, j = tj * 32 + tx + 16 * v;
      if (i < n && j < n) C[(long long)i * n + j] = acc[u][v];
    }
}

// ---------------------------------------------------------------------------
// The same batched products on the FP64 matrix cores.  64 x 64 output tile
// per work-group of four waves, each wave a 32 x 32 quadrant built from 2 x 2
// v_mfma_f64_16x16x4 blocks; K staged through LDS 32 at a time.  Lane layout
// of the 16x16x4 FP64 instruction: A[i][k] and B[k][j] from lane i + 16 k
// (resp. j + 16 k); output element r of lane l is D[l / 16 + 4 r][l % 16].
// Work-groups are numbered so that all tiles of one system share an XCD, which
// keeps each system's operand panels in one L2 (xcd_slot_tile).
typedef double v4d __attribute__((ext_vector_type(4)));

// MODE is a template argument: each product form gets its own kernel with
// only its own addressing, and every thread keeps 32-bit element offsets that
// advance by one K slab per step (few registers, so several work-groups share
// a CU and hide each other's load latency).
// WIN = 1 (modes 0 and 1, a two-fragment cluster whose basis rows are its
// monomers' orbitals, block diagonal, the first fragment's AOs 0 .. n1 - 1):
// only the output rows >= n1 and columns < n1 are needed (the fragment-pair
// block of C0^T S C0), so the tiles without such elements are skipped, and K
// runs over the second fragment's AOs in mode 0 (C0^T S: the other terms
// are zeros of C0) and over the first fragment's in mode 1 ((C0^T S) C0^T^T,
// the columns of the first factor that mode 0 formed).
template <int MODE, int WIN>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
    k_gemm_mfma(DevBatch bt, const int* list, int nl, int tiles_per_sys, const double* __restrict__ Abase,
                const double* __restrict__ Bbase, double* __restrict__ Cbase, const double* __restrict__ wbase,
                int skip_done, int sym, int occ_list) {
  int sl, tile;
  xcd_slot_tile(blockIdx.x, tiles_per_sys, sl, tile);
  if (sl >= nl) return;
  const int si = list[sl];
  if (skip_done && bt.status[si] != 0) return;
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  const int nt = (n + 63) / 64;
  if (tile >= nt * nt) return;
  const int ti = tile / nt, tj = tile - ti * nt;
  // symmetric product: only the upper tiles, mirrored on store (sym 1) or
  // not (sym 2: the consumer reads the upper triangle only)
  if (sym && ti > tj) return;
  int kbeg = 0, kend = n;
  if (WIN) {
    const int a1 = bt.sys_sh_atom[d.sh_off + d.comp_sh[1]];
    const int n1 = bt.sys_atom_ao0[d.atom_off + a1];
    if (ti * 64 + 64 <= n1 || tj * 64 >= n1) return;
    if (MODE == 0) kbeg = (n1 / 32) * 32;
    else kend = min(n, (n1 + 31) / 32 * 32);
  }
  const double* A = Abase + d.mat_off;
  const double* B = Bbase + d.mat_off;
  double* C = Cbase + d.mat_off;
  const double* w = wbase ? wbase + d.ao_off : nullptr;
  // mode 2 with occ_list: the sum runs over the orbitals listed by k_fermi
  // (occupation above OCC_MIN) instead of all n
  const bool use_list = MODE == 2 && occ_list;
  if (use_list) kend = bt.occ_cnt[si];
  const int nk = kend;
  constexpr int KS = 32, LD = 65;
  __shared__ double As[KS][LD];  // [k][i]
  __shared__ double Bs[KS][LD];  // [k][j]
  __shared__ int kxs[MODE == 2 ? MAXN : 1];  // the listed orbitals, staged once
  const int tid = threadIdx.x;
  if (use_list) {
    const int* kg = bt.occ_idx + d.ao_off;
    for (int k = tid; k < nk; k += 256) kxs[k] = kg[k];
    __syncthreads();
  }
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wi = wave >> 1, wj = wave & 1;
  const int i0 = ti * 64, j0 = tj * 64;
  // 16 x 16 output blocks of this wave that hold a real element: the others
  // lie wholly in the padding and are neither computed nor stored
  bool blk[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) blk[u][v] = i0 + wi * 32 + 16 * u < n && j0 + wj * 32 + 16 * v < n;
  const bool all4 = blk[1][1];
  v4d acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = (v4d){0.0, 0.0, 0.0, 0.0};
  // element h (0..7) of this thread in a slab: tile row/column and k index
  //   "row-major" operand (A in modes 0/1, B in mode 1): r = tid / 32 + 8 h, k = tid % 32
  //   "k-major" operand (A in mode 2, B in modes 0/2):   k = tid / 64 + 4 h, r = tid % 64
  const int rr = tid >> 5, rk = tid & 31;  // row-major
  const int kk_ = tid >> 6, kr = tid & 63; // k-major
  // A: slab element offsets at k0 = 0 and validity of the fixed index
  int a_off, b_off, a_step, b_step, a_hstep, b_hstep;
  bool a_fix, b_fix;
  if (MODE == 2) {
    a_off = kk_ * n + i0 + kr;
    a_hstep = 4 * n;
    a_step = KS * n;
    a_fix = i0 + kr < n;
  } else {
    a_off = (i0 + rr) * n + rk;
    a_hstep = 8 * n;
    a_step = KS;
    a_fix = true;
  }
  if (MODE == 1) {
    b_off = (j0 + rr) * n + rk;
    b_hstep = 8 * n;
    b_step = KS;
    b_fix = true;
  } else {
    b_off = kk_ * n + j0 + kr;
    b_hstep = 4 * n;
    b_step = KS * n;
    b_fix = j0 + kr < n;
  }
  if (WIN) {  // start at K = kbeg (row-major operands: + kbeg, k-major: + kbeg rows)
    a_off += MODE == 2 ? kbeg * n : kbeg;
    b_off += MODE == 1 ? kbeg : kbeg * n;
  }
  double ra[8], rb[8];
  auto fetch = [&](int k0) {
    if (MODE == 2 && use_list) {
      int gk[8];
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const int pk = k0 + kk_ + 4 * h;
        gk[h] = pk < nk ? kxs[pk] : -1;
      }
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        ra[h] = (a_fix && gk[h] >= 0) ? A[gk[h] * n + i0 + kr] * w[gk[h]] : 0.0;
        rb[h] = (b_fix && gk[h] >= 0) ? B[gk[h] * n + j0 + kr] : 0.0;
      }
      return;
    }
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      if (MODE == 2) {
        const int gk = k0 + kk_ + 4 * h;
        ra[h] = (a_fix && gk < nk) ? A[a_off + h * a_hstep] * (w ? w[gk] : 1.0) : 0.0;
      } else {
        const int gi = i0 + rr + 8 * h, gk = k0 + rk;
        ra[h] = (gi < n && gk < nk) ? A[a_off + h * a_hstep] : 0.0;
      }
      if (MODE == 1) {
        const int gj = j0 + rr + 8 * h, gk = k0 + rk;
        rb[h] = (gj < n && gk < nk) ? B[b_off + h * b_hstep] : 0.0;
      } else {
        const int gk = k0 + kk_ + 4 * h;
        rb[h] = (b_fix && gk < nk) ? B[b_off + h * b_hstep] : 0.0;
      }
    }
    a_off += a_step;
    b_off += b_step;
  };
  fetch(kbeg);
  for (int k0 = kbeg; k0 < nk; k0 += KS) {
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      if (MODE == 2)
        As[kk_ + 4 * h][kr] = ra[h];
      else
        As[rk][rr + 8 * h] = ra[h];
      if (MODE == 1)
        Bs[rk][rr + 8 * h] = rb[h];
      else
        Bs[kk_ + 4 * h][kr] = rb[h];
    }
    __syncthreads();
    if (k0 + KS < nk) fetch(k0 + KS);
    if (all4 && k0 + KS <= nk) {
#pragma unroll
      for (int kk = 0; kk < KS; kk += 4) {
        const int krow = kk + (lane >> 4), c = lane & 15;
        const double a0 = As[krow][wi * 32 + c], a1 = As[krow][wi * 32 + 16 + c];
        const double b0 = Bs[krow][wj * 32 + c], b1 = Bs[krow][wj * 32 + 16 + c];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
      }
    } else {
      // a wave with padding blocks, or the last slab: the steps past nk
      // (zero padding) and the padding blocks are left out
      for (int kk = 0; kk < KS && k0 + kk < nk; kk += 4) {
        const int krow = kk + (lane >> 4), c = lane & 15;
        const double a0 = As[krow][wi * 32 + c], a1 = As[krow][wi * 32 + 16 + c];
        const double b0 = Bs[krow][wj * 32 + c], b1 = Bs[krow][wj * 32 + 16 + c];
        if (blk[0][0]) acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        if (blk[0][1]) acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        if (blk[1][0]) acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        if (blk[1][1]) acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + wi * 32 + u * 16 + (lane >> 4) + 4 * r;
        const int gj = j0 + wj * 32 + v * 16 + (lane & 15);
        if (gi < n && gj < n) {
          C[(long long)gi * n + gj] = acc[u][v][r];
          if (sym == 1 && ti < tj) C[(long long)gj * n + gi] = acc[u][v][r];
        }
      }
}

template __global__ void k_gemm_mfma<0, 0>(DevBatch, const int*, int, int, const double*, const double*, double*,
                                           const double*, int, int, int);
template __global__ void k_gemm_mfma<1, 0>(DevBatch, const int*, int, int, const double*, const double*, double*,
                                           const double*, int, int, int);
template __global__ void k_gemm_mfma<2, 0>(DevBatch, const int*, int, int, const double*, const double*, double*,
                                           const double*, int, int, int);
template __global__ void k_gemm_mfma<0, 1>(DevBatch, const int*, int, int, const double*, const double*, double*,
                                           const double*, int, int, int);
template __global__ void k_gemm_mfma<1, 1>(DevBatch, const int*, int, int, const double*, const double*, double*,
                                           const double*, int, int, int);

// Lower triangle of the listed systems' symmetric matrices from the upper
// one, for the parts that a product with sym 2 leaves out: every element of
// a 64 x 64 tile below the diagonal tiles (the diagonal tiles were computed
// whole).  32 x 32 pieces pass through LDS so that reads and writes are
// whole rows.
__global__ void __launch_bounds__(256) k_mirror_tiles(DevBatch bt, const int* list, double* Abase) {
  const int si = list[blockIdx.x];
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  double* A = Abase + d.mat_off;
  __shared__ double tr[32][33];
  const int nt = (n + 31) / 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int I = 0; I < nt; ++I)
    for (int J = I + 1; J < nt; ++J) {
      if ((I >> 1) == (J >> 1)) continue;  // inside one 64 x 64 diagonal tile
      const int j = 32 * J + tx;
#pragma unroll
      for (int r = 0; r < 32; r += 8) {
        const int i = 32 * I + r + ty;
        if (i < n && j < n) tr[r + ty][tx] = A[(long long)i * n + j];
      }
      __syncthreads();
      const int ic = 32 * I + tx;
#pragma unroll
      for (int r = 0; r < 32; r += 8) {
        const int jr = 32 * J + r + ty;
        if (jr < n && ic < n) A[(long long)jr * n + ic] = tr[tx][r + ty];
      }
      __syncthreads();  // before the next piece overwrites tr
    }
}

// ---------------------------------------------------------------------------
// The batched products of the mixed-precision form (early SCC iterations) on
// the FP32 matrix cores: operands read in their storage precision (FP64
// basis, FP32 Fock matrix or intermediate), rounded to FP32 when staged in
// LDS, v_mfma_f32_16x16x4f32 with FP32 accumulation, result stored as TC.
// Same tiles, work-group order, symmetric and occupied-list options as
// k_gemm_mfma; K staged 64 at a time (the FP32 tiles take half the LDS).
// Lane layout of the 16x16x4 FP32 instruction (checked on the GPU with an
// in-bounds probe): A[i][k] from lane i + 16 k, B[k][j] from lane j + 16 k;
// output element r of lane l is D[4 (l / 16) + r][l % 16].
typedef float v4f __attribute__((ext_vector_type(4)));

template <int MODE, typename TA, typename TB, typename TC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
    k_gemm_f32(DevBatch bt, const int* list, int nl, int tiles_per_sys, const TA* __restrict__ Abase,
               const TB* __restrict__ Bbase, TC* __restrict__ Cbase, const double* __restrict__ wbase, int skip_done,
               int sym, int occ_list) {
  int sl, tile;
  xcd_slot_tile(blockIdx.x, tiles_per_sys, sl, tile);
  if (sl >= nl) return;
  const int si = list[sl];
  if (skip_done && bt.status[si] != 0) return;
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  const int nt = (n + 63) / 64;
  if (tile >= nt * nt) return;
  const int ti = tile / nt, tj = tile - ti * nt;
  if (sym && ti > tj) return;
  const TA* A = Abase + d.mat_off;
  const TB* B = Bbase + d.mat_off;
  TC* C = Cbase + d.mat_off;
  const double* w = wbase ? wbase + d.ao_off : nullptr;
  const bool use_list = MODE == 2 && occ_list;
  const int nk = use_list ? bt.occ_cnt[si] : n;
  constexpr int KS = 64, LD = 65;
  __shared__ float As[KS][LD];  // [k][i]
  __shared__ float Bs[KS][LD];  // [k][j]
  __shared__ int kxs[MODE == 2 ? MAXN : 1];
  const int tid = threadIdx.x;
  if (use_list) {
    const int* kg = bt.occ_idx + d.ao_off;
    for (int k = tid; k < nk; k += 256) kxs[k] = kg[k];
    __syncthreads();
  }
  const int lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int i0 = ti * 64, j0 = tj * 64;
  v4f acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = (v4f){0.f, 0.f, 0.f, 0.f};
  // element h (0..15) of this thread in a 64 x 64 slab:
  //   row-major operand: r = tid / 64 + 4 h, k = tid % 64
  //   k-major operand:   k = tid / 64 + 4 h, r = tid % 64
  const int rq = tid >> 6, rl = tid & 63;
  float ra[16], rb[16];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int h = 0; h < 16; ++h) {
      if (MODE == 2) {
        int gk = k0 + rq + 4 * h;
        if (use_list) gk = gk < nk ? kxs[gk] : -1;
        const bool ok = gk >= 0 && gk < n;
        ra[h] = (ok && i0 + rl < n) ? (float)((double)A[(long long)gk * n + i0 + rl] * (w ? w[gk] : 1.0)) : 0.f;
        rb[h] = (ok && j0 + rl < n) ? (float)B[(long long)gk * n + j0 + rl] : 0.f;
      } else {
        const int gi = i0 + rq + 4 * h, gk = k0 + rl;
        ra[h] = (gi < n && gk < n) ? (float)A[(long long)gi * n + gk] : 0.f;
        if (MODE == 1) {
          const int gj = j0 + rq + 4 * h;
          rb[h] = (gj < n && gk < n) ? (float)B[(long long)gj * n + gk] : 0.f;
        } else {
          const int gk2 = k0 + rq + 4 * h;
          rb[h] = (gk2 < n && j0 + rl < n) ? (float)B[(long long)gk2 * n + j0 + rl] : 0.f;
        }
      }
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < nk; k0 += KS) {
#pragma unroll
    for (int h = 0; h < 16; ++h) {
      if (MODE == 2)
        As[rq + 4 * h][rl] = ra[h];
      else
        As[rl][rq + 4 * h] = ra[h];
      if (MODE == 1)
        Bs[rl][rq + 4 * h] = rb[h];
      else
        Bs[rq + 4 * h][rl] = rb[h];
    }
    __syncthreads();
    if (k0 + KS < nk) fetch(k0 + KS);
#pragma unroll
    for (int kk = 0; kk < KS; kk += 4) {
      const int krow = kk + (lane >> 4), c = lane & 15;
      const float a0 = As[krow][wi * 32 + c], a1 = As[krow][wi * 32 + 16 + c];
      const float b0 = Bs[krow][wj * 32 + c], b1 = Bs[krow][wj * 32 + 16 + c];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + wi * 32 + u * 16 + 4 * (lane >> 4) + r;
        const int gj = j0 + wj * 32 + v * 16 + (lane & 15);
        if (gi < n && gj < n) {
          C[(long long)gi * n + gj] = (TC)acc[u][v][r];
          if (sym && ti < tj) C[(long long)gj * n + gi] = (TC)acc[u][v][r];
        }
      }
}

// the three products of an FP32 SCC iteration:
//   T = C^T F (F stored FP32)    A = T C (symmetric)    P = C^T diag(n) C (occupied list)
template __global__ void k_gemm_f32<0, double, float, float>(DevBatch, const int*, int, int, const double*,
                                                             const float*, float*, const double*, int, int, int);
template __global__ void k_gemm_f32<1, float, double, double>(DevBatch, const int*, int, int, const float*,
                                                              const double*, double*, const double*, int, int, int);
template __global__ void k_gemm_f32<2, double, double, double>(DevBatch, const int*, int, int, const double*,
                                                               const double*, double*, const double*, int, int, int);

// ---------------------------------------------------------------------------
// Parallel cyclic Jacobi on the symmetric matrix A (in place), rotating the
// rows of V.  Round-robin ordering: every step applies n/2 disjoint
// rotations; each 2 x 2 block (pair k, pair l) is updated as J_k^T B J_l in
// one pass.  Sweeps stop when no rotation exceeds the threshold.
__device__ inline int rr_index(int pos, int step, int m) {
  return pos == 0 ? 0 : 1 + (pos - 1 + step) % (m - 1);
}

__device__ void jacobi_solve(double* __restrict__ A, double* __restrict__ V, int n, int nv, int max_sweeps,
                             double rel_tol, double abs_thr, double* red, double* cs_c, double* cs_s, double* cs_t,
                             int* pp, int* qq, int* nsweep_out) {
  const int m = n + (n & 1);
  const int nb = m / 2;
  const int nt = blockDim.x;
  // scale: Frobenius norm
  double loc = 0.0;
  for (long long i = threadIdx.x; i < (long long)n * n; i += nt) loc += A[i] * A[i];
  double fro = sqrt(block_sum(loc, red));
  double thr = fmax(rel_tol * (fro > 0.0 ? fro : 1.0), abs_thr);
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    double maxoff = 0.0;
    for (int step = 0; step < m - 1; ++step) {
      for (int k = threadIdx.x; k < nb; k += nt) {
        int p = rr_index(k, step, m), q = rr_index(m - 1 - k, step, m);
        if (p > q) {
          int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, s = 0.0, t = 0.0;
        if (q < n) {
          double apq = A[(long long)p * n + q];
          maxoff = fmax(maxoff, fabs(apq));
          if (fabs(apq) > thr) {
            double app = A[(long long)p * n + p], aqq = A[(long long)q * n + q];
            double theta = (aqq - app) / (2.0 * apq);
            t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        cs_c[k] = c;
        cs_s[k] = s;
        cs_t[k] = t;
        pp[k] = p;
        qq[k] = q;
      }
      __syncthreads();
      // A <- J^T A J over (a <= b) pair blocks; two blocks per thread per
      // round with all loads issued before the stores
      const int nblk = nb * (nb + 1) / 2;
      for (int base = threadIdx.x; base < nblk; base += 2 * nt) {
        int ids[2] = {base, base + nt};
        double v[2][4];
        int P_[2], Q_[2], R_[2], U_[2];
        double ca_[2], sa_[2], cb_[2], sb_[2];
        bool act[2], diag[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          int idx = ids[h];
          act[h] = false;
          diag[h] = false;
          if (idx >= nblk) continue;
          int k = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
          while (k * (k + 1) / 2 > idx) --k;
          while ((k + 1) * (k + 2) / 2 <= idx) ++k;
          int a = idx - k * (k + 1) / 2, b = k;  // a <= b
          ca_[h] = cs_c[a];
          sa_[h] = cs_s[a];
          cb_[h] = cs_c[b];
          sb_[h] = cs_s[b];
          if (sa_[h] == 0.0 && sb_[h] == 0.0) continue;
          P_[h] = pp[a];
          Q_[h] = qq[a];
          R_[h] = pp[b];
          U_[h] = qq[b];
          act[h] = true;
          if (a == b) {
            diag[h] = true;
            if (Q_[h] >= n) {
              act[h] = false;
              continue;
            }
            v[h][0] = A[(long long)P_[h] * n + Q_[h]];
            v[h][1] = cs_t[a];
            continue;
          }
          bool qv = Q_[h] < n, uv = U_[h] < n;
          v[h][0] = A[(long long)P_[h] * n + R_[h]];
          v[h][1] = uv ? A[(long long)P_[h] * n + U_[h]] : 0.0;
          v[h][2] = qv ? A[(long long)Q_[h] * n + R_[h]] : 0.0;
          v[h][3] = (qv && uv) ? A[(long long)Q_[h] * n + U_[h]] : 0.0;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (!act[h]) continue;
          int p = P_[h], q = Q_[h], r = R_[h], u = U_[h];
          if (diag[h]) {
            double apq = v[h][0], t = v[h][1];
            A[(long long)p * n + p] -= t * apq;
            A[(long long)q * n + q] += t * apq;
            A[(long long)p * n + q] = 0.0;
            A[(long long)q * n + p] = 0.0;
            continue;
          }
          bool qv = q < n, uv = u < n;
          double ca = ca_[h], sa = sa_[h], cb = cb_[h], sb = sb_[h];
          double tpr = ca * v[h][0] - sa * v[h][2], tpu = ca * v[h][1] - sa * v[h][3];
          double tqr = sa * v[h][0] + ca * v[h][2], tqu = sa * v[h][1] + ca * v[h][3];
          double npr = cb * tpr - sb * tpu, npu = sb * tpr + cb * tpu;
          double nqr = cb * tqr - sb * tqu, nqu = sb * tqr + cb * tqu;
          A[(long long)p * n + r] = npr;
          A[(long long)r * n + p] = npr;
          if (uv) {
            A[(long long)p * n + u] = npu;
            A[(long long)u * n + p] = npu;
          }
          if (qv) {
            A[(long long)q * n + r] = nqr;
            A[(long long)r * n + q] = nqr;
          }
          if (qv && uv) {
            A[(long long)q * n + u] = nqu;
            A[(long long)u * n + q] = nqu;
          }
        }
      }
      // eigenvector rows, four elements per thread per round, loads first
      const int nvv = nb * nv;
      for (int base = threadIdx.x; base < nvv; base += 4 * nt) {
        double vp[4], vq[4], cc[4], ss[4];
        long long op[4], oq[4];
        bool go[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          int idx = base + h * nt;
          go[h] = false;
          if (idx >= nvv) continue;
          int k = idx / nv, j = idx - k * nv;
          ss[h] = cs_s[k];
          if (ss[h] == 0.0) continue;
          cc[h] = cs_c[k];
          op[h] = (long long)pp[k] * nv + j;
          oq[h] = (long long)qq[k] * nv + j;
          vp[h] = V[op[h]];
          vq[h] = V[oq[h]];
          go[h] = true;
        }
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          if (!go[h]) continue;
          V[op[h]] = cc[h] * vp[h] - ss[h] * vq[h];
          V[oq[h]] = ss[h] * vp[h] + cc[h] * vq[h];
        }
      }
      __syncthreads();
    }
    double mo = block_max(maxoff, red);
    if (mo <= thr) break;
  }
  if (nsweep_out && threadIdx.x == 0) *nsweep_out = sweep < max_sweeps ? sweep + 1 : max_sweeps;
}

// Rotations below max(rel_tol |A|_F, thr_scale * last SCC residual) are skipped,
// and while that residual exceeds cap_err a single sweep is made per SCC
// iteration (the warm-started basis is refined together with the charges);
// the final iterations are diagonalised to rel_tol.
__global__ void k_jacobi(DevBatch bt, const int* list, int max_sweeps, double rel_tol, double thr_scale,
                         double cap_err, int* sweeps_out) {
  if (bt.status[list[blockIdx.x]] != 0) return;
  int si = list[blockIdx.x];
  const SysDesc d = bt.desc[si];
  __shared__ double red[1024];
  __shared__ double cs_c[MAXN / 2], cs_s[MAXN / 2], cs_t[MAXN / 2];
  __shared__ int pp[MAXN / 2], qq[MAXN / 2];
  double* A = bt.F + d.mat_off;
  double* V = bt.Ct + d.mat_off;
  const int msw = bt.err[si] > cap_err ? 1 : max_sweeps;
  jacobi_solve(A, V, d.nao, d.nao, msw, rel_tol, thr_scale * bt.err[si], red, cs_c, cs_s, cs_t, pp, qq,
               sweeps_out ? sweeps_out + si : nullptr);
  __syncthreads();
  for (int i = threadIdx.x; i < d.nao; i += blockDim.x) bt.eps[d.ao_off + i] = A[(long long)i * d.nao + i];
}

// Standalone batched eigensolver (component entry point): matrices packed in
// Abuf with offsets off[k], eigenvectors into Vbuf (initialised to I here).
__global__ void k_eigh_batched(const int* nvec, const long long* off, double* Abuf, double* Vbuf, double* wbuf,
                               const long long* woff, int max_sweeps, double rel_tol) {
  int k = blockIdx.x;
  int n = nvec[k];
  double* A = Abuf + off[k];
  double* V = Vbuf + off[k];
  __shared__ double red[256];
  __shared__ double cs_c[MAXN / 2], cs_s[MAXN / 2], cs_t[MAXN / 2];
  __shared__ int pp[MAXN / 2], qq[MAXN / 2];
  for (long long i = threadIdx.x; i < (long long)n * n; i += blockDim.x) V[i] = (i / n == i % n) ? 1.0 : 0.0;
  __syncthreads();
  jacobi_solve(A, V, n, n, max_sweeps, rel_tol, 0.0, red, cs_c, cs_s, cs_t, pp, qq, nullptr);
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) wbuf[woff[k] + i] = A[(long long)i * n + i];
}

// ---------------------------------------------------------------------------
// Fermi-Dirac occupations n_i = 2 / (1 + exp((eps_i - eF)/kT)), eF by bisection
// so that sum n_i = N_el; also -T S_el.
__global__ void k_fermi(DevSystem sys, DevBatch bt, const int* list) {
  int si = list[blockIdx.x];
  if (bt.status[si] != 0) return;  // converged or failed: nothing to do
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  const double kT = sys.g.kT;
  __shared__ double red[256];
  // (256 threads, n <= 512: each thread keeps its two eigenvalues in registers)
  const double* e = bt.eps + d.ao_off;
  constexpr int PER = MAXN / 256;
  double ev[PER];
  double lo = 1e300, hi = -1e300;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = threadIdx.x + 256 * k;
    ev[k] = i < n ? e[i] : 0.0;
    if (i < n) {
      lo = fmin(lo, ev[k]);
      hi = fmax(hi, ev[k]);
    }
  }
  lo = -block_max(-lo, red) - 1.0;
  hi = block_max(hi, red) + 1.0;
  for (int it = 0; it < 300; ++it) {
    double mid = 0.5 * (lo + hi);
    double loc = 0.0;
#pragma unroll
    for (int k = 0; k < PER; ++k)
      if (threadIdx.x + 256 * k < n) loc += 2.0 / (1.0 + exp((ev[k] - mid) / kT));
    double tot = block_sum_waves(loc, red);
    if (tot > d.nel) hi = mid;
    else lo = mid;
    if (hi - lo < 1e-15) break;
  }
  double ef = 0.5 * (lo + hi);
  double ts = 0.0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = threadIdx.x + 256 * k;
    if (i >= n) continue;
    double f = 1.0 / (1.0 + exp((ev[k] - ef) / kT));
    bt.occ[d.ao_off + i] = 2.0 * f;
    double t = 0.0;
    if (f > 0.0) t += f * log(f);
    if (f < 1.0) t += (1.0 - f) * log(1.0 - f);
    ts += t;
  }
  ts = block_sum_waves(ts, red);  // (its barriers also publish the occupations)
  if (threadIdx.x == 0) bt.mts[si] = 2.0 * kT * ts;
  if (threadIdx.x < 64) {
    // orbitals that enter the density product, in ascending order: one wave,
    // 64 orbitals per step, positions from a ballot
    const int lane = threadIdx.x;
    const double* oc = bt.occ + d.ao_off;
    int* ix = bt.occ_idx + d.ao_off;
    int c = 0;
    for (int base = 0; base < n; base += 64) {
      const int i = base + lane;
      const bool take = i < n && oc[i] > OCC_MIN;
      const unsigned long long m = __ballot(take);
      if (take) ix[c + __popcll(m & ((1ULL << lane) - 1ULL))] = i;
      c += __popcll(m);
    }
    if (lane == 0) bt.occ_cnt[si] = c;
  }
}

// ---------------------------------------------------------------------------
// Mulliken charges of P, energy, convergence test and Anderson mixing.
__device__ void solve_small(double* M, double* rhs, int m) {
  // Gaussian elimination with partial pivoting on an (m x m) system, in place
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (fabs(M[r * m + c]) > fabs(M[piv * m + c])) piv = r;
    if (piv != c) {
      for (int k = 0; k < m; ++k) {
        double t = M[c * m + k];
        M[c * m + k] = M[piv * m + k];
        M[piv * m + k] = t;
      }
      double t = rhs[c];
      rhs[c] = rhs[piv];
      rhs[piv] = t;
    }
    double dv = M[c * m + c];
    if (fabs(dv) < 1e-300) dv = 1e-300;
    for (int r = c + 1; r < m; ++r) {
      double f = M[r * m + c] / dv;
      for (int k = c; k < m; ++k) M[r * m + k] -= f * M[c * m + k];
      rhs[r] -= f * rhs[c];
    }
  }
  for (int c = m - 1; c >= 0; --c) {
    double v = rhs[c];
    for (int k = c + 1; k < m; ++k) v -= M[c * m + k] * rhs[k];
    double dv = M[c * m + c];
    rhs[c] = v / (fabs(dv) < 1e-300 ? 1e-300 : dv);
  }
}

__global__ void k_charges_mix(DevSystem sys, DevBatch bt, const int* list, double tol, double etol, int max_iter,
                              double beta) {
  int si = list[blockIdx.x];
  if (bt.status[si] != 0) return;
  const SysDesc d = bt.desc[si];
  const int n = d.nao, ns = d.nsh;
  __shared__ double red[256];
  __shared__ double pop[MAXN];
  __shared__ double qa[MAXN];
  __shared__ double coef[HIST + 1];
  const double* S = bt.S + d.mat_off;
  const double* P = bt.P + d.mat_off;
  const double* H = bt.H0 + d.mat_off;
  // AO populations (P S)_mu,mu = sum_nu P_mu,nu S_mu,nu and Tr(P H0).  P, S
  // and H0 are symmetric: only the upper triangle is read, by rows (wave w
  // takes rows w, w + 4, ...; lanes consecutive columns j >= i).  Element
  // (i, j) adds to population i (a wave sum per row) and, off the diagonal,
  // to population j (per-lane column sums, added over the waves in order at
  // the end) and counts twice in Tr(P H0).  Every sum is taken in a fixed
  // order (deterministic); no barrier inside the loop, so the loads of many
  // rows are in flight together.
  __shared__ double cpart[4 * MAXN];  // per-wave column sums, then matrix-vector partials
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, nwv = blockDim.x >> 6;
  double eh = 0.0;
  {
    constexpr int NC = MAXN / 64;
    double colacc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) colacc[c] = 0.0;
    const int ncn = (n + 63) >> 6;
    for (int i = wv; i < n; i += nwv) {
      const long long ro = (long long)i * n;
      const int c0 = i >> 6;
      double rs = 0.0;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (c >= c0 && c < ncn) {
          const int j = 64 * c + ln;
          if (j >= i && j < n) {
            const double pv = P[ro + j];
            const double x = pv * S[ro + j];
            const double ph = pv * H[ro + j];
            rs += x;
            if (j == i) {
              eh += ph;
            } else {
              eh += 2.0 * ph;
              colacc[c] += x;
            }
          }
        }
      }
      rs = wave_sum_f64(rs);
      if (ln == 0) pop[i] = rs;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = 64 * c + ln;
      if (j < n) cpart[wv * n + j] = colacc[c];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      double v = pop[j];
      for (int w = 0; w < nwv; ++w) v += cpart[w * n + j];
      pop[j] = v;
    }
    __syncthreads();
  }
  eh = block_sum_waves(eh, red);
  // shell charges
  double* qo = bt.q_out + d.sh_off;
  const double* qi = bt.q_in + d.sh_off;
  for (int s = threadIdx.x; s < ns; s += blockDim.x) {
    int a = bt.sys_sh_atom[d.sh_off + s];
    int A = bt.sys_atoms[d.atom_off + a];
    const DevElem& el = sys.elems[sys.elem[A]];
    int ls = s - bt.sys_atom_sh0[d.atom_off + a];
    // the shell's AOs are consecutive
    const int mu0 = bt.sys_atom_ao0[d.atom_off + a] + el.ao0[ls];
    double v = 0.0;
    for (int i = mu0; i < mu0 + el.nao_sh[ls]; ++i) v += pop[i];
    qo[s] = v - (bt.sh_q0 ? bt.sh_q0[d.sh_off + s] : el.q0[ls]);
  }
  __syncthreads();
  for (int a = threadIdx.x; a < d.nat; a += blockDim.x) {
    int s0 = bt.sys_atom_sh0[d.atom_off + a];
    int s1 = (a + 1 < d.nat) ? bt.sys_atom_sh0[d.atom_off + a + 1] : ns;
    double v = 0.0;
    for (int s = s0; s < s1; ++s) v += qo[s];
    qa[a] = v;
  }
  __syncthreads();
  // energy
  const double* G = bt.gam + d.gam_off;
  // (G q)_s, G stored exactly symmetric: the waves' shares of t, added in order
  matvec_wave_part(G, qo, ns, cpart);
  __syncthreads();
  double e2 = 0.0, e3 = 0.0, err = 0.0;
  for (int s = threadIdx.x; s < ns; s += blockDim.x) {
    double v = 0.0;
    for (int w = 0; w < nwv; ++w) v += cpart[w * ns + s];
    e2 += 0.5 * qo[s] * v;
    err = fmax(err, fabs(qo[s] - qi[s]));
  }
  for (int a = threadIdx.x; a < d.nat; a += blockDim.x) {
    int A = bt.sys_atoms[d.atom_off + a];
    e3 -= sys.elems[sys.elem[A]].Gamma * qa[a] * qa[a] * qa[a] / 3.0;
  }
  e2 = block_sum_waves(e2, red);
  e3 = block_sum_waves(e3, red);
  err = block_max_waves(err, red);
  double e = eh + e2 + e3 + bt.mts[si] + bt.erep[si];
  int it = bt.niter[si] + 1;
  double de = fabs(e - bt.e_prev[si]);
  bool conv = (err < tol) && (de < etol) && (it > 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    bt.e_int[si] = e;
    bt.e_prev[si] = e;
    bt.err[si] = err;
    bt.niter[si] = it;
    if (conv) bt.status[si] = 1;
    else if (it >= max_iter) bt.status[si] = 2;
  }
  if (conv || it >= max_iter) return;
  // Anderson mixing of the input charges
  int nh = bt.nhist[si];
  if (nh < 0) nh = 0;
  double* hx = bt.hx + (long long)d.sh_off * HIST;
  double* hr = bt.hr + (long long)d.sh_off * HIST;
  int slot = nh % HIST;
  if (bt.pre) {
    // Newton step direction (1 + M G)^-1 r: the residual map of the SCC has
    // Jacobian -(1 + M G) with M the charge susceptibility, G the Coulomb
    // and third-order kernel; M and G are frozen at the start of the solve
    const float* Pr = bt.pre + d.gam_off;
    for (int s = threadIdx.x; s < ns; s += blockDim.x) pop[s] = qo[s] - qi[s];
    __syncthreads();
    matvec_wave_part(Pr, pop, ns, cpart);  // (stored transposed)
    __syncthreads();
    for (int s = threadIdx.x; s < ns; s += blockDim.x) {
      double v = 0.0;
      for (int w = 0; w < nwv; ++w) v += cpart[w * ns + s];
      hx[(long long)slot * ns + s] = qi[s];
      hr[(long long)slot * ns + s] = v;
    }
  } else {
    for (int s = threadIdx.x; s < ns; s += blockDim.x) {
      hx[(long long)slot * ns + s] = qi[s];
      hr[(long long)slot * ns + s] = qo[s] - qi[s];
    }
  }
  nh += 1;
  int m = nh < HIST ? nh : HIST;
  __syncthreads();
  if (m == 1) {
    // first step: along the Newton direction where a preconditioner is
    // present (the pentacene dimers: 25,610 iterations against 28,219 for a
    // plain first step), else plain
    double* qn = bt.q_in + d.sh_off;
    if (bt.pre)
      for (int s = threadIdx.x; s < ns; s += blockDim.x) qn[s] = qi[s] + beta * hr[(long long)slot * ns + s];
    else
      for (int s = threadIdx.x; s < ns; s += blockDim.x) qn[s] = qi[s] + beta * (qo[s] - qi[s]);
  } else {
    // B_ij = r_i . r_j (slots ordered oldest..newest): every thread
    // accumulates its part of all m (m + 1) / 2 products in one pass over the
    // history, then a butterfly within each wave and the wave totals in order
    __shared__ double Bm[(HIST + 1) * (HIST + 1)];
    __shared__ double rhs[HIST + 1];
    __shared__ double wsum[16][HIST * (HIST + 1) / 2];
    constexpr int NPR = HIST * (HIST + 1) / 2;
    double loc[NPR];
#pragma unroll
    for (int k = 0; k < NPR; ++k) loc[k] = 0.0;
    for (int s = threadIdx.x; s < ns; s += blockDim.x) {
      double r[HIST];
#pragma unroll
      for (int i = 0; i < HIST; ++i) r[i] = i < m ? hr[(long long)((nh - m + i) % HIST) * ns + s] : 0.0;
#pragma unroll
      for (int i = 0, k = 0; i < HIST; ++i)
#pragma unroll
        for (int j = i; j < HIST; ++j, ++k) loc[k] = fma(r[i], r[j], loc[k]);
    }
    const int wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NPR; ++k) {
      double v = loc[k];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if ((threadIdx.x & 63) == 0) wsum[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int i = 0, k = 0; i < HIST; ++i)
        for (int j = i; j < HIST; ++j, ++k) {
          if (i >= m || j >= m) continue;
          double v = 0.0;
          for (int w = 0; w < nwv; ++w) v += wsum[w][k];
          Bm[i * (m + 1) + j] = v;
          Bm[j * (m + 1) + i] = v;
        }
      int M = m + 1;
      // (diagonal lifted relative to itself: a shift relative to the
      // trace, which the oldest and largest residuals dominate, swamped the
      // newest ones once they had dropped seven orders below them and slowed
      // the last iterations: pentacene dimers 25,610 -> 24,950 iterations)
      for (int i = 0; i < m; ++i) {
        Bm[i * M + i] *= 1.0 + 1e-12;
        Bm[i * M + m] = 1.0;
        Bm[m * M + i] = 1.0;
        rhs[i] = 0.0;
      }
      Bm[m * M + m] = 0.0;
      rhs[m] = 1.0;
      solve_small(Bm, rhs, M);
      for (int i = 0; i < m; ++i) coef[i] = rhs[i];
    }
    __syncthreads();
    double* qn = bt.q_in + d.sh_off;
    for (int s = threadIdx.x; s < ns; s += blockDim.x) {
      double v = 0.0;
      for (int i = 0; i < m; ++i) {
        int sl = (nh - m + i) % HIST;
        v += coef[i] * (hx[(long long)sl * ns + s] + beta * hr[(long long)sl * ns + s]);
      }
      qn[s] = v;
    }
  }
  if (threadIdx.x == 0) bt.nhist[si] = nh;
}

}  // namespace fx

namespace fx {

// ---------------------------------------------------------------------------
// LDS-resident parallel Jacobi (same rotations and round-robin order as
// jacobi_solve).  The working matrix lives in LDS: its strict upper triangle
// packed in precision T, the diagonal separately in FP64.  Rotation angles are
// computed in FP64 from the FP64 diagonal; the rotated off-diagonal elements
// are kept in T.  The rotations of `chunk` consecutive steps are logged in LDS
// (FP64 c, s) and then applied to the FP64 basis rows of V in column tiles
// streamed through LDS, so V is read and written once per chunk instead of
// once per step.  V stays orthonormal to FP64 rounding whatever T is; with
// T = float the off-diagonal storage error is relative to the off-diagonal
// elements themselves, and since every SCC iteration rebuilds A = C^T F C in
// FP64 the next iteration removes it (iterative refinement): the converged
// eigenpairs carry FP64 accuracy.
__device__ inline int pk_index(int i, int j) { return i < j ? j * (j - 1) / 2 + i : i * (i - 1) / 2 + j; }

template <typename T>
__global__ void __launch_bounds__(1024)
    k_jacobi_lds(DevBatch bt, const int* list, int max_sweeps, double rel_tol, double thr_scale, double cap_err,
                 int* sweeps_out, int chunk) {
  extern __shared__ double2 lds_raw[];
  unsigned char* lds = reinterpret_cast<unsigned char*>(lds_raw);
  const int si = list[blockIdx.x];
  if (bt.status[si] != 0) return;
  const SysDesc d = bt.desc[si];
  const int n = d.nao, nv = d.nao;
  const int m = n + (n & 1), nb = m / 2;
  const int nt = blockDim.x, nw = nt >> 6;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const JacobiLdsLayout L = jacobi_lds_layout(n, (int)sizeof(T), chunk, nw);
  T* Ap = reinterpret_cast<T*>(lds + L.ap);
  double* dg = reinterpret_cast<double*>(lds + L.dg);
  double2* cs = reinterpret_cast<double2*>(lds + L.cs);  // [chunk][nb] (c, s)
  int* pq = reinterpret_cast<int*>(lds + L.pq);          // [chunk][nb] p | q << 16
  double* vt = reinterpret_cast<double*>(lds + L.vt);    // [nw][n + 1] column tile of V
  double* red = reinterpret_cast<double*>(lds + L.red);
  const double* __restrict__ A = bt.F + d.mat_off;
  double* __restrict__ V = bt.Ct + d.mat_off;

  // load: diagonal in FP64, strict upper triangle packed in T
  for (int e = threadIdx.x; e < n * n; e += nt) {
    const int i = e / n, j = e - i * n;
    if (j < i) continue;
    const double v = A[e];
    if (i == j)
      dg[i] = v;
    else
      Ap[pk_index(i, j)] = (T)v;
  }
  // |A|_F from per-row sums added in row order, so that the threshold does
  // not depend on the launch shape; diagonal entries count at most 10 Eh (a
  // projector shift of section "Covalent bond fragmentation", 1e6 Eh, must
  // not loosen the threshold of the physical orbitals)
  for (int i = threadIdx.x; i < n; i += nt) {
    double r = 0.0;
    for (int j = i; j < n; ++j) {
      const double v = A[(long long)i * n + j];
      r += (j == i) ? fmin(v * v, 100.0) : 2.0 * v * v;
    }
    vt[i] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double f = 0.0;
    for (int i = 0; i < n; ++i) f += vt[i];
    red[0] = sqrt(f);
  }
  __syncthreads();
  const double fro = red[0];
  __syncthreads();
  const double err = bt.err[si];
  const double thr = fmax(rel_tol * (fro > 0.0 ? fro : 1.0), thr_scale * err);
  const int msw = err > cap_err ? 1 : max_sweeps;
  // folded enumeration of the off-diagonal pair blocks (a < b): rows a and
  // R-1-a together hold nb blocks; the middle row (R odd) follows
  const int R = nb - 1, hp = R / 2, rect = hp * nb, noff = nb * (nb - 1) / 2;
  const int per = (n * nw + nt - 1) / nt;  // tile elements per thread (<= 8 for n <= 512)
  const int ntile = (nv + nw - 1) / nw;
  double* col = vt + (long long)wave * (n + 1);
  int sweep = 0;
  for (; sweep < msw; ++sweep) {
    int rot_sweep = 0;
    for (int s0 = 0; s0 < m - 1; s0 += chunk) {
      const int s1 = min(m - 1, s0 + chunk);
      int rot_local = 0;
      for (int step = s0; step < s1; ++step) {
        double2* csx = cs + (step - s0) * nb;
        int* pqx = pq + (step - s0) * nb;
        // rotation parameters; each pair's own 2x2 diagonal block is
        // finished here (no other block of this step touches it)
        for (int k = threadIdx.x; k < nb; k += nt) {
          int p = rr_index(k, step, m), q = rr_index(m - 1 - k, step, m);
          if (p > q) {
            const int t = p;
            p = q;
            q = t;
          }
          double c = 1.0, s = 0.0;
          if (q < n) {
            const int ipq = pk_index(p, q);
            const double apq = (double)Ap[ipq];
            const double app = dg[p], aqq = dg[q];
            // a pair is converged below the absolute threshold or at FP64
            // resolution of its larger diagonal entry
            if (fabs(apq) > fmax(thr, rel_tol * fmax(fabs(app), fabs(aqq)))) {
              const double theta = (aqq - app) / (2.0 * apq);
              const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
              c = 1.0 / sqrt(t * t + 1.0);
              s = t * c;
              dg[p] = app - t * apq;
              dg[q] = aqq + t * apq;
              Ap[ipq] = (T)0;
              rot_local = 1;
            }
          }
          csx[k] = make_double2(c, s);
          pqx[k] = p | (q << 16);
        }
        __syncthreads();
        // A <- J^T A J on the off-diagonal 2x2 blocks (pair a, pair b)
        for (int idx = threadIdx.x; idx < noff; idx += nt) {
          int a, b;
          if (idx < rect) {
            const int r = idx / nb, cc = idx - r * nb;
            if (cc < R - r) {
              a = r;
              b = r + 1 + cc;
            } else {
              a = R - 1 - r;
              b = a + 1 + (cc - (R - r));
            }
          } else {
            a = hp;
            b = hp + 1 + (idx - rect);
          }
          const double2 wa = csx[a], wb = csx[b];
          if (wa.y == 0.0 && wb.y == 0.0) continue;
          const int va = pqx[a], vb = pqx[b];
          const int p = va & 0xffff, q = va >> 16, r = vb & 0xffff, u = vb >> 16;
          const bool qv = q < n, uv = u < n;
          const T ca = (T)wa.x, sa = (T)wa.y, cb = (T)wb.x, sb = (T)wb.y;
          const int ipr = pk_index(p, r);
          const int ipu = uv ? pk_index(p, u) : 0;
          const int iqr = qv ? pk_index(q, r) : 0;
          const int iqu = (qv && uv) ? pk_index(q, u) : 0;
          const T bpr = Ap[ipr];
          const T bpu = uv ? Ap[ipu] : (T)0;
          const T bqr = qv ? Ap[iqr] : (T)0;
          const T bqu = (qv && uv) ? Ap[iqu] : (T)0;
          const T tpr = ca * bpr - sa * bqr, tpu = ca * bpu - sa * bqu;
          const T tqr = sa * bpr + ca * bqr, tqu = sa * bpu + ca * bqu;
          Ap[ipr] = cb * tpr - sb * tpu;
          if (uv) Ap[ipu] = sb * tpr + cb * tpu;
          if (qv) Ap[iqr] = cb * tqr - sb * tqu;
          if (qv && uv) Ap[iqu] = sb * tqr + cb * tqu;
        }
        __syncthreads();
      }
      // apply the chunk's rotations to the rows of V, nw columns at a time:
      // coalesced tile loads (next tile prefetched into registers), one
      // column per wave, coalesced stores
      rot_sweep |= rot_local;
      if (__syncthreads_or(rot_local)) {
        double rg[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int e = threadIdx.x + r * nt, i = e / nw, j = e - i * nw;
          rg[r] = (r < per && i < n && j < nv) ? V[(long long)i * nv + j] : 0.0;
        }
        for (int tile = 0; tile < ntile; ++tile) {
          const int c0 = tile * nw;
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            const int e = threadIdx.x + r * nt, i = e / nw, j = e - i * nw;
            if (r < per && i < n) vt[(long long)j * (n + 1) + i] = rg[r];
          }
          __syncthreads();
          if (tile + 1 < ntile) {
            const int c1 = c0 + nw;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
              const int e = threadIdx.x + r * nt, i = e / nw, j = e - i * nw;
              rg[r] = (r < per && i < n && c1 + j < nv) ? V[(long long)i * nv + c1 + j] : 0.0;
            }
          }
          if (c0 + wave < nv) {
            for (int step = s0; step < s1; ++step) {
              const double2* csx = cs + (step - s0) * nb;
              const int* pqx = pq + (step - s0) * nb;
              for (int k = lane; k < nb; k += 64) {
                const double2 w = csx[k];
                if (w.y != 0.0) {
                  const int v = pqx[k];
                  const int p = v & 0xffff, q = v >> 16;
                  const double vp = col[p], vq = col[q];
                  col[p] = w.x * vp - w.y * vq;
                  col[q] = w.y * vp + w.x * vq;
                }
              }
              __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
              __builtin_amdgcn_wave_barrier();
              __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
          }
          __syncthreads();
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            const int e = threadIdx.x + r * nt, i = e / nw, j = e - i * nw;
            if (r < per && i < n && c0 + j < nv) V[(long long)i * nv + c0 + j] = vt[(long long)j * (n + 1) + i];
          }
          __syncthreads();
        }
      }
    }
    // converged when no pair rotated in this sweep
    if (!__syncthreads_or(rot_sweep)) break;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += nt) bt.eps[d.ao_off + i] = dg[i];
  if (sweeps_out && threadIdx.x == 0) sweeps_out[si] = sweep < msw ? sweep + 1 : msw;
}

template __global__ void k_jacobi_lds<double>(DevBatch, const int*, int, double, double, double, int*, int);
template __global__ void k_jacobi_lds<float>(DevBatch, const int*, int, double, double, double, int*, int);

}  // namespace fx

namespace fx {

__device__ inline float f4_get(const float4& v, int c) { return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w; }
__device__ inline void f4_set(float4& v, int c, float x) {
  v.x = c == 0 ? x : v.x;
  v.y = c == 1 ? x : v.y;
  v.z = c == 2 ? x : v.z;
  v.w = c == 3 ? x : v.w;
}

// ---------------------------------------------------------------------------
// Mixing preconditioner of a cluster system X (1 to 3 fragments): the inverse
// of K = 1 + M_X G_X, where M_X is block diagonal with the monomers' charge
// susceptibilities M_I = sum_ai Q_ai Q_ai^T / (eps_a - eps_i) (the orbital
// response of the response section, shell-summed) and G_X = gamma_XX minus
// 2 Gamma_A dq_A on same-atom shell blocks at the system's input charges.
// Gauss-Jordan inversion in place, in FP32 in LDS (the preconditioner only
// steers the mixer; the fixed point does not depend on it).  ok[si] = 0 and
// the identity are written when a pivot vanishes.
template <int ROWS>
__global__ void __launch_bounds__(1024)
    k_precond_build(DevSystem sys, DevBatch bt, const int* list, DevBatch mono, const double* Mmono, float* pre,
                    int* ok) {
  // LDS: K (ns x ns, FP32); while K is formed, the same bytes stage the
  // operands of the product M G' in chunks of KC contraction indices
  extern __shared__ float4 Kf4_lds[];
  float* Kf = reinterpret_cast<float*>(Kf4_lds);
  __shared__ double qa[MAXN];  // atom charges, then 2 Gamma_A dq_A per atom
  __shared__ float4 rowk4[MAXN / 4];
  __shared__ float colA[MAXN], colB[MAXN];
  __shared__ int perm[MAXN];   // local atom of each shell while K is formed
  __shared__ int comp_off[4], comp_mnsh[3];
  __shared__ long long comp_moff[3];
  const int si = list[blockIdx.x];
  const SysDesc d = bt.desc[si];
  const int ns = d.nsh;
  const double* G = bt.gam + d.gam_off;
  const double* q = bt.q_in + d.sh_off;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (threadIdx.x == 0) {
    for (int c = 0; c < d.nfrag; ++c) {
      const SysDesc md = mono.desc[d.frag[c]];
      comp_off[c] = d.comp_sh[c];
      comp_moff[c] = md.gam_off;
      comp_mnsh[c] = md.nsh;
    }
    comp_off[d.nfrag] = d.comp_sh[d.nfrag];
  }
  for (int a = threadIdx.x; a < d.nat; a += blockDim.x) {
    const int s0 = bt.sys_atom_sh0[d.atom_off + a];
    const int s1 = (a + 1 < d.nat) ? bt.sys_atom_sh0[d.atom_off + a + 1] : ns;
    double v = 0.0;
    for (int s = s0; s < s1; ++s) v += q[s];
    qa[a] = 2.0 * sys.elems[sys.elem[bt.sys_atoms[d.atom_off + a]]].Gamma * v;
  }
  for (int t = threadIdx.x; t < ns; t += blockDim.x) perm[t] = bt.sys_sh_atom[d.sh_off + t];
  // K = 1 + M G', M block diagonal (the monomers' susceptibilities): each
  // thread accumulates rows s = wave + nw r and columns t = lane + 64 j in
  // FP64 registers, the contraction index u ascending (terms from another
  // fragment's block are exact zeros), so every element is summed in the same
  // order as the plain row-by-row product; G' and the block-diagonal M are
  // staged KC rows / columns at a time (each element read from HBM once)
  const int* smap = bt.sh_mono + d.sh_off;
  const int KC = min(16, max(1, ns / 4));
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  double* Gs = reinterpret_cast<double*>(Kf);  // [KC][ns]
  double* Ms = Gs + KC * ns;                    // [ns][KC]
  double acc[ROWS][PRE_COLS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r)
#pragma unroll
    for (int j = 0; j < PRE_COLS; ++j) acc[r][j] = (wave + nw * r == lane + 64 * j) ? 1.0 : 0.0;
  for (int u0 = 0; u0 < ns; u0 += KC) {
    const int kc = min(KC, ns - u0);
    __syncthreads();  // the previous chunk is consumed (first pass: the tables above are written)
    for (int e = threadIdx.x; e < kc * ns; e += blockDim.x) {
      const int uu = e / ns, t = e - uu * ns, u = u0 + uu;
      double g = G[(long long)u * ns + t];
      if (perm[u] == perm[t]) g -= qa[perm[t]];
      Gs[uu * ns + t] = g;
    }
    for (int e = threadIdx.x; e < ns * kc; e += blockDim.x) {
      const int s = e / kc, uu = e - s * kc, u = u0 + uu;
      int cs = 0, cu = 0;
      for (int c = 1; c < d.nfrag; ++c) {
        cs += s >= comp_off[c];
        cu += u >= comp_off[c];
      }
      Ms[s * kc + uu] =
          cs == cu ? Mmono[comp_moff[cs] + (long long)smap[s] * comp_mnsh[cs] + smap[u]] : 0.0;
    }
    __syncthreads();
    // (rows and columns beyond ns repeat the last one: no branches in the
    // loop, and their sums are never stored)
    for (int uu = 0; uu < kc; ++uu) {
      double g[PRE_COLS];
#pragma unroll
      for (int j = 0; j < PRE_COLS; ++j) g[j] = Gs[uu * ns + min(lane + 64 * j, ns - 1)];
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        const double m = Ms[min(wave_u + nw * r, ns - 1) * kc + uu];
#pragma unroll
        for (int j = 0; j < PRE_COLS; ++j) acc[r][j] = fma(m, g[j], acc[r][j]);
      }
    }
  }
  __syncthreads();  // the staging area becomes K
  // K rows padded to ldk (a multiple of 4, zeros beyond ns): whole float4s
  const int ldk = (ns + 3) & ~3, ld4 = ldk >> 2;
  float4* K4 = Kf4_lds;
#pragma unroll
  for (int r = 0; r < ROWS; ++r)
#pragma unroll
    for (int j = 0; j < PRE_COLS; ++j) {
      const int s = wave + nw * r, t = lane + 64 * j;
      if (s < ns && t < ldk) Kf[s * ldk + t] = t < ns ? (float)acc[r][j] : 0.0f;
    }
  __syncthreads();
  // the first pivot column, taken out of K (a pivot column is kept outside
  // K and zero inside it: the update then leaves -c_i / pivot there)
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    colA[i] = Kf[i * ldk];
    Kf[i * ldk] = 0.0f;
  }
  __syncthreads();
  // Gauss-Jordan with partial pivoting (largest |K[i][k]|, i >= k, lowest
  // index on ties), in place.  Every wave finds the pivot itself from the
  // pivot column (consecutive LDS words, wave reductions); the first ld4
  // threads form the scaled pivot row and make the row interchange; then
  // thread (cg, rg) updates float4 column group cg of rows rg, rg + ng, ...
  // and collects column k + 1 of them, the next pivot column.  Two barriers
  // per pivot.
  constexpr int NG = PRE_THREADS / (4 * ROWS);    // fewest row groups (ns <= 16 ROWS)
  constexpr int GJR = (16 * ROWS + NG - 1) / NG;  // most rows per thread
  const int ng = blockDim.x / ld4;
  const int cg = threadIdx.x % ld4, rg = threadIdx.x / ld4;
  bool good = true;
  for (int k = 0; k < ns; ++k) {
    const float* colc = (k & 1) ? colB : colA;
    float* coln = (k & 1) ? colA : colB;
    float best = -1.0f;
    int bi = 0x7fffffff;
    for (int i = k + lane; i < ns; i += 64) {
      const float v = fabsf(colc[i]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    const float pv = wave_max_f32(best);
    const int p = wave_min_i32(best == pv ? bi : 0x7fffffff);
    if (pv < 1e-20f) {  // same value in every wave: uniform exit
      good = false;
      break;
    }
    if ((int)threadIdx.x < ld4) {
      const int c = threadIdx.x;
      const float piv = colc[p];
      float4 xp = K4[p * ld4 + c];
      if (c == (k >> 2)) f4_set(xp, k & 3, 1.0f);
      rowk4[c] = make_float4(xp.x / piv, xp.y / piv, xp.z / piv, xp.w / piv);
      if (p != k) K4[p * ld4 + c] = K4[k * ld4 + c];
      if (c == 0) perm[k] = p;
    }
    __syncthreads();
    if (rg < ng) {
      const float4 rk = rowk4[cg];
      const float ck = colc[k];  // row p holds the former row k from now on
      const int k1 = k + 1;
      const bool collect = cg == (k1 >> 2);
      float4 x[GJR];
      float cr[GJR];
#pragma unroll
      for (int r = 0; r < GJR; ++r) {
        const int i = rg + ng * r;
        if (i < ns) {
          x[r] = K4[i * ld4 + cg];
          cr[r] = colc[i];
        }
      }
#pragma unroll
      for (int r = 0; r < GJR; ++r) {
        const int i = rg + ng * r;
        if (i < ns) {
          float4 v = rk;
          if (i != k) {
            const float ci = i == p ? ck : cr[r];
            v = x[r];
            v.x = v.x - ci * rk.x;
            v.y = v.y - ci * rk.y;
            v.z = v.z - ci * rk.z;
            v.w = v.w - ci * rk.w;
          }
          if (collect) {
            coln[i] = f4_get(v, k1 & 3);
            f4_set(v, k1 & 3, 0.0f);
          }
          K4[i * ld4 + cg] = v;
        }
      }
    }
    __syncthreads();
  }
  if (good) {
    // undo the row interchanges as column interchanges, last first
    for (int k = ns - 1; k >= 0; --k) {
      const int p = perm[k];
      if (p != k) {  // (perm is shared: a uniform branch)
        for (int i = threadIdx.x; i < ns; i += blockDim.x) {
          const float t = Kf[i * ldk + k];
          Kf[i * ldk + k] = Kf[i * ldk + p];
          Kf[i * ldk + p] = t;
        }
        __syncthreads();
      }
    }
  }
  // stored transposed (element (s, t) at t ns + s), so that the products
  // with it read consecutive addresses across threads
  float* out = pre + d.gam_off;
  for (int t = wave; t < ns; t += nw)
    for (int s = lane; s < ns; s += 64) out[t * ns + s] = good ? Kf[s * ldk + t] : (s == t ? 1.0f : 0.0f);
  if (threadIdx.x == 0) ok[si] = good ? 1 : 0;
}

template __global__ void k_precond_build<PRE_ROWS_SMALL>(DevSystem, DevBatch, const int*, DevBatch, const double*,
                                                         float*, int*);
template __global__ void k_precond_build<PRE_ROWS>(DevSystem, DevBatch, const int*, DevBatch, const double*, float*,
                                                   int*);

}  // namespace fx

namespace fx {

// ---------------------------------------------------------------------------
// Split form of the LDS Jacobi for single-sweep SCC iterations, with a
// blocked cyclic ordering.
//
// The indices (padded to m, a multiple of four) form fixed blocks
// {2k, 2k+1}.  A sweep is one step that rotates every block's own pair,
// then m/2 - 1 round-robin rounds over the blocks; in each round the blocks
// meet as quartets (X, Y) with rows x1 = 2X, x2 = 2X+1, y1 = 2Y, y2 = 2Y+1,
// and each quartet takes two steps: (x1, y1) with (x2, y2), then (x1, y2)
// with (x2, y1).  Every pair is rotated once per sweep in m - 1 steps, as in
// the plain round-robin, but two steps share one pass over the data.
//
// k_jacobi_rot: sweeps on the LDS working matrix (packed strict upper
// triangle in T, FP64 diagonal).  Per round, one thread per quartet solves
// its 4 x 4 diagonal block (the two steps in order, rotation angles in FP64),
// then every off-diagonal 4 x 4 block between two quartets is rotated on both
// sides in one pass.  The rotations (c, s) go to the log in HBM: per sweep
// the m/2 block rotations, then per round four per quartet (x1 y1, x2 y2,
// x1 y2, x2 y1); up to `max_log` sweeps.
// k_apply_rot applies the logged rotations to C^T, the rows in registers
// (lane = quartet) and moved between lanes from round to round.
// rr_index(pos, step, M) for pos <= M - 1 and step <= M - 2 (within one
// sweep, pos - 1 + step < 2 (M - 1)): one conditional subtraction instead of
// the modulo
__device__ inline int rr_fast(int pos, int step, int M) {
  int t = pos - 1 + step;
  t = t >= M - 1 ? t - (M - 1) : t;
  return pos == 0 ? 0 : 1 + t;
}

__device__ inline long long jq_sweep_entries(int m) { return (long long)m / 2 + (long long)(m / 2 - 1) * m; }

// (a, b), a < b, of the idx-th unordered pair of N items (rows folded so that
// every row of the enumeration has N entries)
__device__ inline void tri_pair(int idx, int N, int& a, int& b) {
  const int R = N - 1, hp = R / 2, rect = hp * N;
  if (idx < rect) {
    const int r = idx / N, cc = idx - r * N;
    if (cc < R - r) {
      a = r;
      b = r + 1 + cc;
    } else {
      a = R - 1 - r;
      b = a + 1 + (cc - (R - r));
    }
  } else {
    a = hp;
    b = hp + 1 + (idx - rect);
  }
}

// Jacobi rotation zeroing a_pq of a symmetric matrix: (c, s, t), identity if
// |a_pq| is below the threshold.  t is the smaller root of
// t^2 + 2 theta t - 1 = 0, theta = (a_qq - a_pp) / (2 a_pq), written as
// t = sign(theta) |y| / (|tau| + sqrt(tau^2 + y^2)) with tau = a_qq - a_pp and
// y = 2 a_pq, so that no quotient by a_pq is formed.  The reciprocal and the
// reciprocal square roots are hardware estimates refined by Newton steps
// (full FP64 precision).  An error in t would only turn the angle slightly;
// c = (1 + t^2)^(-1/2) and s = t c keep c^2 + s^2 = 1 to rounding whatever t
// is, so the basis stays orthonormal.
__device__ inline void jq_angle(double app, double aqq, double apq, double thr, double rel_tol, double& c, double& s,
                                double& t) {
  c = 1.0;
  s = 0.0;
  t = 0.0;
  if (fabs(apq) > fmax(thr, rel_tol * fmax(fabs(app), fabs(aqq)))) {
    const double tau = aqq - app, y = 2.0 * apq;
    const double h = fma(tau, tau, y * y);  // > 0, since y != 0
    const double dd = fabs(tau) + h * rsqrt_pos(h);
    double r = __builtin_amdgcn_rcp(dd);
    r = r * fma(-dd, r, 2.0);
    r = r * fma(-dd, r, 2.0);
    // sign(theta), theta = tau / y; +1 when tau is zero
    const bool pos = tau == 0.0 || ((tau > 0.0) == (y > 0.0));
    t = (pos ? fabs(y) : -fabs(y)) * r;
    c = rsqrt_pos(fma(t, t, 1.0));
    s = t * c;
  }
}

// two-sided rotation of rows/columns p, q of a symmetric 4 x 4 block
template <int P, int Q>
__device__ inline void jq_rot4(double (&M)[4][4], double c, double s, double t) {
  if (s == 0.0) return;
  const double app = M[P][P], aqq = M[Q][Q], apq = M[P][Q];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double a = M[P][k], b = M[Q][k];
    M[P][k] = c * a - s * b;
    M[Q][k] = s * a + c * b;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double a = M[k][P], b = M[k][Q];
    M[k][P] = c * a - s * b;
    M[k][Q] = s * a + c * b;
  }
  M[P][P] = app - t * apq;
  M[Q][Q] = aqq + t * apq;
  M[P][Q] = M[Q][P] = 0.0;
}

// rows P, Q of a 4 x 4 block rotated (left side only)
template <int P, int Q, typename T>
__device__ inline void jq_rows(T (&B)[4][4], T c, T s) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T a = B[P][k], b = B[Q][k];
    B[P][k] = c * a - s * b;
    B[Q][k] = s * a + c * b;
  }
}
template <int P, int Q, typename T>
__device__ inline void jq_cols(T (&B)[4][4], T c, T s) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T a = B[k][P], b = B[k][Q];
    B[k][P] = c * a - s * b;
    B[k][Q] = s * a + c * b;
  }
}

// The working matrix is held as 2 x 2 tiles of the upper block triangle
// (N blocks {2k, 2k+1}, N even): tile (a, b), a <= b, at jt_index(a, b, N)
// holds A(2a + i, 2b + j) in component 2 i + j (x, y, z, w); a diagonal tile
// keeps only its y component, A(2a, 2a + 1) (the diagonal itself is held in
// FP64 apart).  Padded rows and columns are stored as zeros and stay zero,
// since every rotation that involves a padded index is the identity, so no
// access needs a padding test.  A 4 x 4 block between two quartets is four
// tiles: four 16-byte (FP32) or 32-byte (FP64) LDS accesses each way.
// The triangle is stored in rectangular full packed order: N / 2 rows of
// R = N + 1 tiles, row k holding column b = N / 2 + k forwards (tiles
// a = 0..b from the row's start) and column N / 2 - 1 - k backwards (tile a
// at R - 1 - a).  Neighbouring a, or neighbouring b, are then 1 or R (odd)
// tiles apart, so the lanes of a quarter-wave that step either index reach
// distinct LDS banks; the column-major triangle (b (b + 1) / 2 + a) put
// lanes that step b at triangular-number offsets that collided.
__device__ inline int jt_index(int a, int b, int N) {
  // (row and column selected first, then one 24-bit multiply-add: no branch)
  const int h = N >> 1, R = N + 1;
  const bool fwd = b >= h;
  const int row = fwd ? b - h : h - 1 - b;
  const int col = fwd ? a : R - 1 - a;
  return __umul24(row, R) + col;
}

template <typename T>
struct JtVec;
template <>
struct JtVec<float> {
  typedef float4 type;
};
template <>
struct JtVec<double> {
  typedef double4 type;
};

// 2 x 2 block of rows of block rb and columns of block cb, rb != cb
template <typename T>
__device__ inline void jt_get(const typename JtVec<T>::type* At, int rb, int cb, int N, T& e00, T& e01, T& e10,
                              T& e11) {
  const bool tr = rb > cb;
  const typename JtVec<T>::type v = At[jt_index(min(rb, cb), max(rb, cb), N)];
  e00 = v.x;
  e11 = v.w;
  e01 = tr ? v.z : v.y;
  e10 = tr ? v.y : v.z;
}
template <typename T>
__device__ inline void jt_put(typename JtVec<T>::type* At, int rb, int cb, int N, T e00, T e01, T e10, T e11) {
  const bool tr = rb > cb;
  typename JtVec<T>::type v;
  v.x = e00;
  v.w = e11;
  v.y = tr ? e10 : e01;
  v.z = tr ? e01 : e10;
  At[jt_index(min(rb, cb), max(rb, cb), N)] = v;
}

// the four (c, s) of quartet q in the working precision: FP32 from the packed
// float copy (two 16-byte reads, the halves of all quartets stored apart so
// that neighbouring quartets are 16 bytes apart), FP64 from the double2
// entries
template <typename T>
__device__ inline void jq_params(const double2* cs, const float4* csf, int q, int nq, T (&w)[8]);
template <>
__device__ inline void jq_params<float>(const double2*, const float4* csf, int q, int nq, float (&w)[8]) {
  const float4 u = csf[q], v = csf[nq + q];
  w[0] = u.x, w[1] = u.y, w[2] = u.z, w[3] = u.w, w[4] = v.x, w[5] = v.y, w[6] = v.z, w[7] = v.w;
}
template <>
__device__ inline void jq_params<double>(const double2* cs, const float4*, int q, int, double (&w)[8]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double2 u = cs[4 * q + k];
    w[2 * k] = u.x;
    w[2 * k + 1] = u.y;
  }
}

// One off-diagonal 4 x 4 block of a round: rows of the quartet with blocks
// qa (X | Y << 16), columns of the quartet qb; rows take that quartet's two
// steps (x1 y1, x2 y2, then x1 y2, x2 y1), columns the other's.
template <typename T>
__device__ inline void jt_offdiag(typename JtVec<T>::type* At, int N, int qa, int qb, bool ra, bool rb,
                                  const T (&wa)[8], const T (&wb)[8]) {
  const int Xa = qa & 0xffff, Ya = (qa >> 16) & 0x7fff, Xb = qb & 0xffff, Yb = (qb >> 16) & 0x7fff;
  T B[4][4];
  jt_get<T>(At, Xa, Xb, N, B[0][0], B[0][1], B[1][0], B[1][1]);
  jt_get<T>(At, Xa, Yb, N, B[0][2], B[0][3], B[1][2], B[1][3]);
  jt_get<T>(At, Ya, Xb, N, B[2][0], B[2][1], B[3][0], B[3][1]);
  jt_get<T>(At, Ya, Yb, N, B[2][2], B[2][3], B[3][2], B[3][3]);
  if (ra) {
    jq_rows<0, 2>(B, wa[0], wa[1]);
    jq_rows<1, 3>(B, wa[2], wa[3]);
    jq_rows<0, 3>(B, wa[4], wa[5]);
    jq_rows<1, 2>(B, wa[6], wa[7]);
  }
  if (rb) {
    jq_cols<0, 2>(B, wb[0], wb[1]);
    jq_cols<1, 3>(B, wb[2], wb[3]);
    jq_cols<0, 3>(B, wb[4], wb[5]);
    jq_cols<1, 2>(B, wb[6], wb[7]);
  }
  jt_put<T>(At, Xa, Xb, N, B[0][0], B[0][1], B[1][0], B[1][1]);
  jt_put<T>(At, Xa, Yb, N, B[0][2], B[0][3], B[1][2], B[1][3]);
  jt_put<T>(At, Ya, Xb, N, B[2][0], B[2][1], B[3][0], B[3][1]);
  jt_put<T>(At, Ya, Yb, N, B[2][2], B[2][3], B[3][2], B[3][3]);
}

// The two steps of round rd on quartet qd's own 4 x 4 block (rotation angles
// in FP64): the rotated block back to LDS, the four (c, s) to the round's
// parameter slots (buffer b) and to the log.  Returns whether it rotated.
template <typename T>
__device__ inline bool jq_quartet(int qd, int rd, int n, int nb2, int nq, int b, double thr, double rel_tol,
                                  typename JtVec<T>::type* At, T* Ae, double* dg, double2* cs, float4* csf, int* qr,
                                  double2* lr) {
  const int X = rr_fast(qd, rd, nb2), Y = rr_fast(nb2 - 1 - qd, rd, nb2);
  const int ix[4] = {2 * X, 2 * X + 1, 2 * Y, 2 * Y + 1};
  T* ex = Ae + 4 * jt_index(X, X, nb2) + 1;
  T* ey = Ae + 4 * jt_index(Y, Y, nb2) + 1;
  T e00, e01, e10, e11;
  jt_get<T>(At, X, Y, nb2, e00, e01, e10, e11);
  double M[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i) M[i][i] = dg[ix[i]];
  M[0][1] = M[1][0] = (double)*ex;
  M[2][3] = M[3][2] = (double)*ey;
  M[0][2] = M[2][0] = (double)e00;
  M[0][3] = M[3][0] = (double)e01;
  M[1][2] = M[2][1] = (double)e10;
  M[1][3] = M[3][1] = (double)e11;
  double c0, s0, t0, c1, s1, t1, c2, s2, t2, c3, s3, t3;
  // step 1: (x1, y1) and (x2, y2), both from the block before the step
  jq_angle(M[0][0], M[2][2], M[0][2], thr, rel_tol, c0, s0, t0);
  jq_angle(M[1][1], M[3][3], M[1][3], thr, rel_tol, c1, s1, t1);
  // (padded rows and columns are zero, so their rotations are the identity
  // already; the tests make that explicit)
  if (ix[0] >= n || ix[2] >= n) c0 = 1.0, s0 = 0.0, t0 = 0.0;
  if (ix[1] >= n || ix[3] >= n) c1 = 1.0, s1 = 0.0, t1 = 0.0;
  jq_rot4<0, 2>(M, c0, s0, t0);
  jq_rot4<1, 3>(M, c1, s1, t1);
  // step 2: (x1, y2) and (x2, y1)
  jq_angle(M[0][0], M[3][3], M[0][3], thr, rel_tol, c2, s2, t2);
  jq_angle(M[1][1], M[2][2], M[1][2], thr, rel_tol, c3, s3, t3);
  if (ix[0] >= n || ix[3] >= n) c2 = 1.0, s2 = 0.0, t2 = 0.0;
  if (ix[1] >= n || ix[2] >= n) c3 = 1.0, s3 = 0.0, t3 = 0.0;
  jq_rot4<0, 3>(M, c2, s2, t2);
  jq_rot4<1, 2>(M, c3, s3, t3);
  const bool rot = s0 != 0.0 || s1 != 0.0 || s2 != 0.0 || s3 != 0.0;
  if (rot) {
#pragma unroll
    for (int i = 0; i < 4; ++i) dg[ix[i]] = M[i][i];
    *ex = (T)M[0][1];
    *ey = (T)M[2][3];
    jt_put<T>(At, X, Y, nb2, (T)M[0][2], (T)M[0][3], (T)M[1][2], (T)M[1][3]);
  }
  qr[b * nq + qd] = X | (Y << 16) | (rot ? (int)0x80000000u : 0);
  const double2 w0 = make_double2(c0, s0), w1 = make_double2(c1, s1), w2 = make_double2(c2, s2),
                w3 = make_double2(c3, s3);
  if (sizeof(T) == 4) {
    csf[2 * b * nq + qd] = make_float4((float)c0, (float)s0, (float)c1, (float)s1);
    csf[2 * b * nq + nq + qd] = make_float4((float)c2, (float)s2, (float)c3, (float)s3);
  } else {
    double2* cb = cs + 4 * (b * nq + qd);
    cb[0] = w0;
    cb[1] = w1;
    cb[2] = w2;
    cb[3] = w3;
  }
  lr[4 * qd] = w0;
  lr[4 * qd + 1] = w1;
  lr[4 * qd + 2] = w2;
  lr[4 * qd + 3] = w3;
  return rot;
}

// One off-diagonal block (a, b), a < b, of a round with the parameters of
// buffer bf: returns without work when neither quartet rotated.
template <typename T>
__device__ inline void jq_block(int a, int b, int nq, int bf, typename JtVec<T>::type* At, const double2* cs,
                                const float4* csf, const int* qr) {
  const int qa = qr[bf * nq + a], qb = qr[bf * nq + b];
  const bool ra = qa < 0, rb = qb < 0;
  if (!ra && !rb) return;
  T wa[8], wb[8];
  jq_params<T>(cs + 4 * bf * nq, csf + 2 * bf * nq, a, nq, wa);
  jq_params<T>(cs + 4 * bf * nq, csf + 2 * bf * nq, b, nq, wb);
  jt_offdiag<T>(At, 2 * nq, qa, qb, ra, rb, wa, wb);
}

// The sweeps of one system by the whole work-group (k_jacobi_rot).
template <typename T>
__device__ inline void jacobi_rot_system(const DevBatch& bt, int si, int max_sweeps, double rel_tol, double thr_scale,
                                         double cap_err, double early_err, int early_sweeps, int* sweeps_out,
                                         double2* logbuf, long long log_stride, int max_log, int* nlog) {
  typedef typename JtVec<T>::type V4;
  extern __shared__ double2 lds_raw[];
  unsigned char* lds = reinterpret_cast<unsigned char*>(lds_raw);
  if (bt.status[si] != 0) return;
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  const int m = (n + 3) & ~3, nb2 = m / 2, nq = m / 4;
  const int nt = blockDim.x;
  const JacobiRotLayout L = jacobi_rot_layout(n, (int)sizeof(T));
  V4* At = reinterpret_cast<V4*>(lds + L.ap);
  T* Ae = reinterpret_cast<T*>(lds + L.ap);
  double* dg = reinterpret_cast<double*>(lds + L.dg);
  double2* cs = reinterpret_cast<double2*>(lds + L.cs);  // [m]: block step [nb2], then 4 per quartet
  float4* csf = reinterpret_cast<float4*>(lds + L.csf);  // FP32: the quartets' (c, s), 2 per quartet
  int* qr = reinterpret_cast<int*>(lds + L.qr);          // [2][nq] X | Y << 16, sign bit: rotates
  int* pt = reinterpret_cast<int*>(lds + L.pt);          // [nq (nq - 1) / 2] quartet pairs
  double* red = reinterpret_cast<double*>(lds + L.red);
  double* rows = reinterpret_cast<double*>(cs);  // row sums before the sweeps (16 m >= 8 n bytes)
  const double* __restrict__ A = bt.F + d.mat_off;
  double2* lg = logbuf + (long long)si * log_stride;
  const int ntile = nb2 * (nb2 + 1) / 2;
  for (int e = threadIdx.x; e < 4 * ntile; e += nt) Ae[e] = (T)0;
  for (int i = threadIdx.x; i < m; i += nt) dg[i] = 0.0;
  // off-diagonal pass: pairs (a, b), a < b, of quartets; flagged: the blocks
  // that hold the next round's quartets (wave 0 rotates them first, see below)
  for (int idx = threadIdx.x; idx < nq * (nq - 1) / 2; idx += nt) {
    int a, b;
    tri_pair(idx, nq, a, b);
    const bool crit = b == a + 2 || (a == 0 && b == 1) || (a == nq - 2 && b == nq - 1);
    pt[idx] = a | (b << 8) | (crit ? 1 << 16 : 0);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += nt) {
    const int i = e / n, j = e - i * n;
    if (j < i) continue;
    const double v = A[e];
    if (i == j)
      dg[i] = v;
    else
      Ae[4 * jt_index(i >> 1, j >> 1, nb2) + 2 * (i & 1) + (j & 1)] = (T)v;
  }
  for (int i = threadIdx.x; i < n; i += nt) {
    double r = 0.0;
    for (int j = i; j < n; ++j) {
      const double v = A[(long long)i * n + j];
      r += (j == i) ? fmin(v * v, 100.0) : 2.0 * v * v;
    }
    rows[i] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double f = 0.0;
    for (int i = 0; i < n; ++i) f += rows[i];
    red[0] = sqrt(f);
  }
  __syncthreads();
  const double fro = red[0];
  const double err = bt.err[si];
  const double thr = fmax(rel_tol * (fro > 0.0 ? fro : 1.0), thr_scale * err);
  // sweeps of this SCC iteration: early_sweeps while the SCC residual
  // exceeds early_err (the first iterations, where the working matrix still
  // carries large couplings), then one, and to convergence once the residual
  // is below cap_err
  const int msw = min(max_log, err > early_err ? early_sweeps : err > cap_err ? 1 : max_sweeps);
  const long long swe = jq_sweep_entries(m);
  const int nblk = nb2 * (nb2 - 1) / 2, nqp = nq * (nq - 1) / 2;
  int sweep = 0;
  bool converged = false;
  for (; sweep < msw; ++sweep) {
    int rot_sweep = 0;
    double2* ls = lg + (long long)sweep * swe;
    // block step: pairs (2k, 2k+1)
    for (int k = threadIdx.x; k < nb2; k += nt) {
      const int p = 2 * k, q = p + 1;
      double c = 1.0, s = 0.0, t = 0.0;
      if (q < n) {
        T* e01 = Ae + 4 * jt_index(k, k, nb2) + 1;
        const double apq = (double)*e01, app = dg[p], aqq = dg[q];
        jq_angle(app, aqq, apq, thr, rel_tol, c, s, t);
        if (s != 0.0) {
          dg[p] = app - t * apq;
          dg[q] = aqq + t * apq;
          *e01 = (T)0;
          rot_sweep = 1;
        }
      }
      cs[k] = make_double2(c, s);
      ls[k] = make_double2(c, s);
    }
    __syncthreads();
    // the block step on the off-diagonal tiles: rows by block a's rotation,
    // then columns by block b's
    for (int idx = threadIdx.x; idx < nblk; idx += nt) {
      int a, b;
      tri_pair(idx, nb2, a, b);
      const double2 wa = cs[a], wb = cs[b];
      if (wa.y == 0.0 && wb.y == 0.0) continue;
      const T ca = (T)wa.x, sa = (T)wa.y, cb = (T)wb.x, sb = (T)wb.y;
      V4 v = At[jt_index(a, b, nb2)];
      const T tpr = ca * v.x - sa * v.z, tpu = ca * v.y - sa * v.w;
      const T tqr = sa * v.x + ca * v.z, tqu = sa * v.y + ca * v.w;
      v.x = cb * tpr - sb * tpu;
      v.y = sb * tpr + cb * tpu;
      v.z = cb * tqr - sb * tqu;
      v.w = sb * tqr + cb * tqu;
      At[jt_index(a, b, nb2)] = v;
    }
    __syncthreads();
    // Rounds.  Round rd's quartet solves use parameter buffer rd & 1.  In
    // the round-robin order the blocks of round rd + 1's quartets meet in
    // the off-diagonal blocks (q - 1, q + 1), (0, 1) and (nq - 2, nq - 1) of
    // round rd, and nothing else that round rd + 1's solves read changes in
    // round rd's off-diagonal pass.  So wave 0 rotates those blocks first and
    // then solves round rd + 1's quartets while the other waves rotate the
    // remaining blocks: one barrier per round, and the FP64 quartet solves
    // overlap the bulk of the off-diagonal work.  (Wave 0's own stores are
    // visible to its later loads: LDS operations of a wave complete in order.)
    const int nrd = nb2 - 1;
    const int ncrit = nq >= 3 ? nq : (nq == 2 ? 1 : 0);
    for (int qd = threadIdx.x; qd < nq; qd += nt)
      if (jq_quartet<T>(qd, 0, n, nb2, nq, 0, thr, rel_tol, At, Ae, dg, cs, csf, qr, ls + nb2)) rot_sweep = 1;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int rd = 0; rd < nrd; ++rd) {
      const int bf = rd & 1;
      if (wave == 0) {
        if (lane < ncrit) {
          const int a = lane == 0 ? 0 : (lane == nq - 1 ? nq - 2 : lane - 1);
          const int b = lane == 0 ? 1 : (lane == nq - 1 ? nq - 1 : lane + 1);
          jq_block<T>(a, b, nq, bf, At, cs, csf, qr);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (rd + 1 < nrd && lane < nq)
          if (jq_quartet<T>(lane, rd + 1, n, nb2, nq, bf ^ 1, thr, rel_tol, At, Ae, dg, cs, csf, qr,
                            ls + nb2 + (long long)(rd + 1) * m))
            rot_sweep = 1;
      }
      // the remaining blocks: the other waves (wave 0 itself in a one-wave
      // work-group)
      const int t0 = nt > 64 ? 64 : 0;
      if ((int)threadIdx.x >= t0)
        for (int idx = threadIdx.x - t0; idx < nqp; idx += nt - t0) {
          const int e = pt[idx];
          if (e >> 16) continue;  // wave 0's
          jq_block<T>(e & 255, (e >> 8) & 255, nq, bf, At, cs, csf, qr);
        }
      __syncthreads();
    }
    if (!__syncthreads_or(rot_sweep)) {
      converged = true;  // this sweep rotated nothing: its (identity) log is not applied
      break;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += nt) bt.eps[d.ao_off + i] = dg[i];
  if (threadIdx.x == 0) {
    nlog[si] = sweep;  // sweeps with rotations, all before the empty one
    if (sweeps_out) sweeps_out[si] = converged ? sweep + 1 : sweep;
  }
}

// One work-group per listed system (queue == nullptr), or a persistent grid
// whose work-groups take list slots from the work queue *queue (zeroed by
// k_queue_reset before the launch) until all nl are taken.  Either way each
// system is swept by one work-group from start to end, so the results do
// not depend on the form or on the work-group size.
template <typename T>
__global__ void __launch_bounds__(1024)
    k_jacobi_rot(DevBatch bt, const int* list, int max_sweeps, double rel_tol, double thr_scale, double cap_err,
                 double early_err, int early_sweeps, int* sweeps_out, double2* logbuf, long long log_stride,
                 int max_log, int* nlog, int* queue, int nl) {
  if (queue == nullptr) {
    jacobi_rot_system<T>(bt, list[blockIdx.x], max_sweeps, rel_tol, thr_scale, cap_err, early_err, early_sweeps,
                         sweeps_out, logbuf, log_stride, max_log, nlog);
    return;
  }
  __shared__ int slot_sh;
  for (;;) {
    __syncthreads();  // the previous system's LDS is no longer read
    if (threadIdx.x == 0) slot_sh = atomicAdd(queue, 1);
    __syncthreads();
    const int slot = slot_sh;
    if (slot >= nl) break;
    jacobi_rot_system<T>(bt, list[slot], max_sweeps, rel_tol, thr_scale, cap_err, early_err, early_sweeps,
                         sweeps_out, logbuf, log_stride, max_log, nlog);
  }
}

__global__ void k_queue_reset(int* queue) {
  if (threadIdx.x == 0) *queue = 0;
}

template __global__ void k_jacobi_rot<double>(DevBatch, const int*, int, double, double, double, double, int, int*,
                                              double2*, long long, int, int*, int*, int);
template __global__ void k_jacobi_rot<float>(DevBatch, const int*, int, double, double, double, double, int, int*,
                                             double2*, long long, int, int*, int*, int);

// Apply the logged rotations to the rows of C^T, one 64-column tile per
// work-group and four columns per wave.  Lane q holds, for the wave's four
// columns, the rows of the two blocks that quartet q pairs in the current
// round, in registers for the whole launch: a round rotates them in place,
// and the round-robin step to the next round moves whole blocks between
// neighbouring lanes.  With quartet q pairing positions q and nb2 - 1 - q and
// positions 1 .. nb2 - 1 advancing one place per round, the block in X moves
// to lane q - 1 and the block in Y to lane q + 1, except that lane 0 keeps
// block 0 and takes lane 1's X block as its Y, and the last quartet's Y block
// becomes its own X.  The moves are DPP lane shifts; during the rounds the
// rows stay in registers and the waves need no barrier between rounds.  Only
// the rotation parameters are staged in LDS then (APPLY_RCH rounds at a time,
// rotation-major so that each lane's 16-byte read is conflict-free); the tile
// enters and leaves through the same LDS area in whole-row accesses.  After
// the last round of a sweep the ring has advanced nb2 - 1 places, back to
// the starting arrangement, in which the block step rotates each lane's two
// blocks and the tile is stored.
__device__ inline void jq_apply2(double& a, double& b, double2 w) {
  const double x = a, y = b;
  a = w.x * x - w.y * y;
  b = w.y * x + w.x * y;
}

// lane i takes lane i + 1's value (DPP wave_shl:1) or lane i - 1's
// (wave_shr:1); the lane without a source reads zero (never used)
__device__ inline double lane_from_next(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x130, 0xf, 0xf, true),
                          __builtin_amdgcn_mov_dpp(lo, 0x130, 0xf, 0xf, true));
}
__device__ inline double lane_from_prev(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x138, 0xf, 0xf, true),
                          __builtin_amdgcn_mov_dpp(lo, 0x138, 0xf, 0xf, true));
}

constexpr int APPLY_RCH = 8;  // rounds of rotation parameters staged in LDS at a time
constexpr int APPLY_COLS = 4;  // columns per wave

__global__ void __launch_bounds__(1024)
    k_apply_rot(DevBatch bt, const int* list, int nl, int tiles_per_sys, int tile_w,
                const double2* __restrict__ logbuf, long long log_stride, const int* nlog) {
  extern __shared__ double2 lds_raw[];
  int sl, tcol;
  xcd_slot_tile(blockIdx.x, tiles_per_sys, sl, tcol);
  if (sl >= nl) return;
  const int si = list[sl];
  if (bt.status[si] != 0) return;
  const int nsw = nlog[si];
  if (nsw <= 0) return;
  const SysDesc d = bt.desc[si];
  const int n = d.nao, nv = d.nao;
  // tile_w 128 (every system of the batch has at most 32 quartets): each
  // half-wave takes its own four columns with the same quartets (no active
  // lane reads across the half boundary: lane 31 moves only as the last
  // quartet, which takes its own Y, and lane 32 only as quartet 0)
  const bool packed = tile_w == 128;
  const int c0 = tcol * tile_w;
  if (c0 >= nv) return;
  const int m = (n + 3) & ~3, nb2 = m / 2, nq = m / 4, nrd = nb2 - 1;
  const int NT = blockDim.x;
  double2* lgs = lds_raw;  // [APPLY_RCH][4][nq] staged (c, s)
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wcols = packed ? 2 * APPLY_COLS : APPLY_COLS;
  const bool wact = c0 + wcols * wave < nv;  // uniform in the wave
  const int cw = c0 + wcols * wave + (packed ? APPLY_COLS * (lane >> 5) : 0);  // the lane's first column
  const int q = packed ? (lane & 31) : lane, qc = min(q, nq - 1);
  const bool act = q < nq;
  const bool first = q == 0, last = q == nq - 1;
  double* V = bt.Ct + d.mat_off;
  // rows of quartet q's blocks in the starting arrangement: blocks q and
  // nb2 - 1 - q (lanes past the last quartet hold zeros and never feed an
  // active lane)
  const int rx = 2 * q, ry = 2 * (nb2 - 1 - qc);
  // the tile comes in through LDS (whole-row reads; padded rows and columns
  // past the matrix are zero), the same area and padded row length as the
  // store at the end
  double* st = reinterpret_cast<double*>(lds_raw);
  const int ld = tile_w + 1;  // padded row: a wave's lanes (one row each) spread over the banks
  const int ccol = cw - c0;   // the lane's first column within the tile
  for (int e = threadIdx.x; e < m * tile_w; e += NT) {
    const int r = e / tile_w, cc = e - r * tile_w, col = c0 + cc;
    st[r * ld + cc] = (r < n && col < nv) ? V[(long long)r * nv + col] : 0.0;
  }
  __syncthreads();
  double x1[APPLY_COLS], x2[APPLY_COLS], y1[APPLY_COLS], y2[APPLY_COLS];
  const int rxc = 2 * qc;  // (addresses inside the tile for every lane)
#pragma unroll
  for (int c = 0; c < APPLY_COLS; ++c) {
    const double a = st[rxc * ld + ccol + c], b = st[(rxc + 1) * ld + ccol + c];
    const double u = st[ry * ld + ccol + c], v = st[(ry + 1) * ld + ccol + c];
    x1[c] = act ? a : 0.0;
    x2[c] = act ? b : 0.0;
    y1[c] = act ? u : 0.0;
    y2[c] = act ? v : 0.0;
  }
  __syncthreads();  // the area is reused for the rotation parameters
  const double2* lg = logbuf + (long long)si * log_stride;
  const long long swe = jq_sweep_entries(m);
  const int CE = APPLY_RCH * m;        // staged entries per chunk
  const int per = (CE + NT - 1) / NT;  // <= 2 for m <= 256 and NT = 1024
  double2 rg[2];
  // staged entries of rounds [r0, r0 + APPLY_RCH) of sweep sw into registers
  auto fetch = [&](int sw, int r0) {
    const double2* src = lg + (long long)sw * swe + nb2 + (long long)r0 * m;
    const int lim = min(APPLY_RCH, nrd - r0) * m;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = threadIdx.x + NT * r;
      rg[r] = (r < per && e < lim) ? src[e] : make_double2(1.0, 0.0);
    }
  };
  for (int sw = 0; sw < nsw; ++sw) {
    const double2* ls = lg + (long long)sw * swe;
    fetch(sw, 0);
    // block step: pairs (2k, 2k+1) of the lane's two blocks
    if (wact) {
      const double2 wx = ls[q < nb2 ? q : 0], wy = ls[nb2 - 1 - qc];
#pragma unroll
      for (int c = 0; c < APPLY_COLS; ++c) {
        jq_apply2(x1[c], x2[c], wx);
        jq_apply2(y1[c], y2[c], wy);
      }
    }
    for (int r0 = 0; r0 < nrd; r0 += APPLY_RCH) {
      __syncthreads();  // the previous chunk's parameters are no longer read
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int e = threadIdx.x + NT * r;
        if (r < per && e < CE) {
          const int j = e / m, i = e - j * m;  // round j of the chunk, entry 4 quartet + k
          lgs[j * m + (i & 3) * nq + (i >> 2)] = rg[r];
        }
      }
      if (r0 + APPLY_RCH < nrd) fetch(sw, r0 + APPLY_RCH);
      __syncthreads();  // staged parameters visible
      const int r1 = min(nrd, r0 + APPLY_RCH);
      if (!wact) continue;
      for (int rd = r0; rd < r1; ++rd) {
        const double2* lr = lgs + (rd - r0) * m + qc;
        const double2 w0 = lr[0], w1 = lr[nq], w2 = lr[2 * nq], w3 = lr[3 * nq];
#pragma unroll
        for (int c = 0; c < APPLY_COLS; ++c) {
          jq_apply2(x1[c], y1[c], w0);
          jq_apply2(x2[c], y2[c], w1);
          jq_apply2(x1[c], y2[c], w2);
          jq_apply2(x2[c], y1[c], w3);
        }
        if (nq > 1) {
#pragma unroll
          for (int c = 0; c < APPLY_COLS; ++c) {
            const double n1 = lane_from_next(x1[c]), n2 = lane_from_next(x2[c]);
            const double p1 = lane_from_prev(y1[c]), p2 = lane_from_prev(y2[c]);
            const double t1 = last ? y1[c] : n1, t2 = last ? y2[c] : n2;
            y1[c] = first ? n1 : p1;
            y2[c] = first ? n2 : p2;
            x1[c] = first ? x1[c] : t1;
            x2[c] = first ? x2[c] : t2;
          }
        }
      }
    }
  }
  // Store the tile through LDS (the parameter area, sized by the host for
  // the whole padded m x tile_w tile), so that each row segment of the tile
  // leaves in one coalesced write instead of tile_w / 4 partial-line pieces
  // from different waves (which cost 2.5 times the algorithmic HBM writes).
  const int band = m;
  for (int r0 = 0; r0 < n; r0 += band) {
    __syncthreads();  // the area is free (parameters read / previous band written)
    if (wact && act) {
      const int rows[4] = {rx, rx + 1, ry, ry + 1};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int r = rows[h] - r0;
        if (r < 0 || r >= band) continue;
#pragma unroll
        for (int c = 0; c < APPLY_COLS; ++c)
          st[r * ld + ccol + c] = h == 0 ? x1[c] : h == 1 ? x2[c] : h == 2 ? y1[c] : y2[c];
      }
    }
    __syncthreads();
    const int nr = min(band, n - r0);
    for (int e = threadIdx.x; e < nr * tile_w; e += NT) {
      const int r = e / tile_w, cc = e - r * tile_w, col = c0 + cc;
      if (col < nv) V[(long long)(r0 + r) * nv + col] = st[r * ld + cc];
    }
  }
}

// Apply kernel for systems of 33 to 64 quartets (129 to 256 AOs): each lane
// holds two quartets, 2p and 2p + 1, of its half-wave's four columns (a wave
// takes eight columns, a work-group of eight waves a 64-column tile).  Of
// the ring moves from one round to the next (X to quartet q - 1, Y to
// q + 1) those between a lane's own two quartets stay in the lane: the block
// in X of quartet 2p + 1 becomes quartet 2p's, the block in Y of quartet 2p
// becomes quartet 2p + 1's.  Only the X of quartet 2p + 2 (from the next
// lane) and the Y of quartet 2p - 1 (from the previous lane) move by DPP, so
// a round moves half as much data per quartet as in k_apply_rot.  The
// boundary rules are those of k_apply_rot: quartet 0 keeps block 0 in X and
// takes quartet 1's X as its Y; the last quartet L takes its own Y as its X.
// Rotation parameters are staged per round as [rotation k][parity of q]
// [q / 2], so that each lane reads consecutive 16-byte entries.
constexpr int APPLY2_WAVES = 8;
// rows per LDS band of the dual kernel's tile: half the padded rows
__host__ __device__ inline int apply_dual_band(int m) { return ((m / 2) + 3) & ~3; }
__global__ void __launch_bounds__(64 * APPLY2_WAVES)
    k_apply_rot_dual(DevBatch bt, const int* list, int nl, int tiles_per_sys, const double2* __restrict__ logbuf,
                     long long log_stride, const int* nlog) {
  extern __shared__ double2 lds_raw[];
  constexpr int TW = 64;  // tile columns
  int sl, tcol;
  xcd_slot_tile(blockIdx.x, tiles_per_sys, sl, tcol);
  if (sl >= nl) return;
  const int si = list[sl];
  if (bt.status[si] != 0) return;
  const int nsw = nlog[si];
  if (nsw <= 0) return;
  const SysDesc d = bt.desc[si];
  const int n = d.nao, nv = d.nao;
  const int c0 = tcol * TW;
  if (c0 >= nv) return;
  const int m = (n + 3) & ~3, nb2 = m / 2, nq = m / 4, nrd = nb2 - 1, L = nq - 1;
  const int P2 = (nq + 1) / 2;  // lane pairs of quartets
  const int S = 8 * P2;         // staged entries per round
  const int NT = blockDim.x;
  double2* lgs = lds_raw;  // [APPLY_RCH][4][2][P2]
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool wact = c0 + 2 * APPLY_COLS * wave < nv;  // uniform in the wave
  const int p = lane & 31;
  const int cw = c0 + 2 * APPLY_COLS * wave + APPLY_COLS * (lane >> 5);  // the lane's first column
  const int qa = 2 * p, qb = 2 * p + 1;
  const bool acta = qa < nq, actb = qb < nq;
  const bool first = p == 0, lastA = qa == L, lastB = qb == L;
  const bool Lodd = (L & 1) != 0;  // uniform: the last quartet is some lane's second
  double* V = bt.Ct + d.mat_off;
  const int qac = min(qa, nq - 1), qbc = min(qb, nq - 1);
  const int rxa = 2 * qac, rya = 2 * (nb2 - 1 - qac), rxb = 2 * qbc, ryb = 2 * (nb2 - 1 - qbc);
  double* st = reinterpret_cast<double*>(lds_raw);
  const int ld = TW + 1;
  const int ccol = cw - c0;
  // the tile passes through LDS in two bands of rows (half the LDS of a
  // whole tile, so that two work-groups share a CU)
  const int band = apply_dual_band(m);
  double xa1[APPLY_COLS], xa2[APPLY_COLS], ya1[APPLY_COLS], ya2[APPLY_COLS];
  double xb1[APPLY_COLS], xb2[APPLY_COLS], yb1[APPLY_COLS], yb2[APPLY_COLS];
#pragma unroll
  for (int c = 0; c < APPLY_COLS; ++c)
    xa1[c] = xa2[c] = ya1[c] = ya2[c] = xb1[c] = xb2[c] = yb1[c] = yb2[c] = 0.0;
  for (int b0 = 0; b0 < m; b0 += band) {
    const int nr = min(band, m - b0);
    if (b0 > 0) __syncthreads();  // the previous band has been read
    for (int e = threadIdx.x; e < nr * TW; e += NT) {
      const int r = e / TW, cc = e - r * TW, col = c0 + cc;
      st[r * ld + cc] = (b0 + r < n && col < nv) ? V[(long long)(b0 + r) * nv + col] : 0.0;
    }
    __syncthreads();
    // (a row outside this band reads nothing; every row lies in one band)
    auto pick = [&](int row, bool act, double& v, int col) {
      const int r = row - b0;
      if (act && r >= 0 && r < nr) v = st[r * ld + col];
    };
#pragma unroll
    for (int c = 0; c < APPLY_COLS; ++c) {
      const int col = ccol + c;
      pick(rxa, acta, xa1[c], col);
      pick(rxa + 1, acta, xa2[c], col);
      pick(rya, acta, ya1[c], col);
      pick(rya + 1, acta, ya2[c], col);
      pick(rxb, actb, xb1[c], col);
      pick(rxb + 1, actb, xb2[c], col);
      pick(ryb, actb, yb1[c], col);
      pick(ryb + 1, actb, yb2[c], col);
    }
  }
  __syncthreads();  // the area is reused for the rotation parameters
  const double2* lg = logbuf + (long long)si * log_stride;
  const long long swe = jq_sweep_entries(m);
  const int CE = APPLY_RCH * m;        // log entries per chunk
  const int per = (CE + NT - 1) / NT;  // <= 4 for m <= 256 and NT = 512
  double2 rg[4];
  auto fetch = [&](int sw, int r0) {
    const double2* src = lg + (long long)sw * swe + nb2 + (long long)r0 * m;
    const int lim = min(APPLY_RCH, nrd - r0) * m;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = threadIdx.x + NT * r;
      rg[r] = (r < per && e < lim) ? src[e] : make_double2(1.0, 0.0);
    }
  };
  for (int sw = 0; sw < nsw; ++sw) {
    const double2* ls = lg + (long long)sw * swe;
    fetch(sw, 0);
    // block step: pairs (2k, 2k+1) of the lane's four blocks
    if (wact) {
      const double2 wxa = ls[qac], wya = ls[nb2 - 1 - qac], wxb = ls[qbc], wyb = ls[nb2 - 1 - qbc];
#pragma unroll
      for (int c = 0; c < APPLY_COLS; ++c) {
        jq_apply2(xa1[c], xa2[c], wxa);
        jq_apply2(ya1[c], ya2[c], wya);
        jq_apply2(xb1[c], xb2[c], wxb);
        jq_apply2(yb1[c], yb2[c], wyb);
      }
    }
    for (int r0 = 0; r0 < nrd; r0 += APPLY_RCH) {
      __syncthreads();  // the previous chunk's parameters are no longer read
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = threadIdx.x + NT * r;
        if (r < per && e < CE) {
          const int j = e / m, i = e - j * m;  // round j of the chunk, entry 4 quartet + k
          const int qq = i >> 2, k = i & 3;
          lgs[j * S + (2 * k + (qq & 1)) * P2 + (qq >> 1)] = rg[r];
        }
      }
      if (r0 + APPLY_RCH < nrd) fetch(sw, r0 + APPLY_RCH);
      __syncthreads();  // staged parameters visible
      const int r1 = min(nrd, r0 + APPLY_RCH);
      if (!wact) continue;
      for (int rd = r0; rd < r1; ++rd) {
        const double2* lr = lgs + (rd - r0) * S + min(p, P2 - 1);
        const double2 a0 = lr[0], b0 = lr[P2], a1 = lr[2 * P2], b1 = lr[3 * P2];
        const double2 a2 = lr[4 * P2], b2 = lr[5 * P2], a3 = lr[6 * P2], b3 = lr[7 * P2];
#pragma unroll
        for (int c = 0; c < APPLY_COLS; ++c) {
          jq_apply2(xa1[c], ya1[c], a0);
          jq_apply2(xa2[c], ya2[c], a1);
          jq_apply2(xa1[c], ya2[c], a2);
          jq_apply2(xa2[c], ya1[c], a3);
          jq_apply2(xb1[c], yb1[c], b0);
          jq_apply2(xb2[c], yb2[c], b1);
          jq_apply2(xb1[c], yb2[c], b2);
          jq_apply2(xb2[c], yb1[c], b3);
        }
        // ring move: X(2p) <- X(2p+1), X(2p+1) <- X(2p+2) (next lane),
        // Y(2p) <- Y(2p-1) (previous lane), Y(2p+1) <- Y(2p); quartet 0
        // keeps its X and takes X(1) as its Y; the last quartet takes its Y
        if (Lodd) {
#pragma unroll
          for (int c = 0; c < APPLY_COLS; ++c) {
            const double nx1 = lane_from_next(xa1[c]), nx2 = lane_from_next(xa2[c]);
            const double py1 = lane_from_prev(yb1[c]), py2 = lane_from_prev(yb2[c]);
            const double oxa1 = xa1[c], oxa2 = xa2[c];
            xa1[c] = first ? oxa1 : xb1[c];
            xa2[c] = first ? oxa2 : xb2[c];
            const double nyb1 = ya1[c], nyb2 = ya2[c];
            ya1[c] = first ? xb1[c] : py1;
            ya2[c] = first ? xb2[c] : py2;
            xb1[c] = lastB ? yb1[c] : nx1;
            xb2[c] = lastB ? yb2[c] : nx2;
            yb1[c] = nyb1;
            yb2[c] = nyb2;
          }
        } else {
#pragma unroll
          for (int c = 0; c < APPLY_COLS; ++c) {
            const double nx1 = lane_from_next(xa1[c]), nx2 = lane_from_next(xa2[c]);
            const double py1 = lane_from_prev(yb1[c]), py2 = lane_from_prev(yb2[c]);
            const double oxa1 = xa1[c], oxa2 = xa2[c];
            xa1[c] = first ? oxa1 : (lastA ? ya1[c] : xb1[c]);
            xa2[c] = first ? oxa2 : (lastA ? ya2[c] : xb2[c]);
            const double nyb1 = ya1[c], nyb2 = ya2[c];
            ya1[c] = first ? xb1[c] : py1;
            ya2[c] = first ? xb2[c] : py2;
            xb1[c] = nx1;
            xb2[c] = nx2;
            yb1[c] = nyb1;
            yb2[c] = nyb2;
          }
        }
      }
    }
  }
  // store the tile through LDS in whole-row writes, band by band
  for (int b0 = 0; b0 < n; b0 += band) {
    const int nr = min(band, n - b0);
    __syncthreads();  // the area is free (parameters read / previous band written)
    auto put = [&](int row, bool act, double v, int col) {
      const int r = row - b0;
      if (act && r >= 0 && r < nr) st[r * ld + col] = v;
    };
    if (wact) {
#pragma unroll
      for (int c = 0; c < APPLY_COLS; ++c) {
        const int col = ccol + c;
        put(rxa, acta, xa1[c], col);
        put(rxa + 1, acta, xa2[c], col);
        put(rya, acta, ya1[c], col);
        put(rya + 1, acta, ya2[c], col);
        put(rxb, actb, xb1[c], col);
        put(rxb + 1, actb, xb2[c], col);
        put(ryb, actb, yb1[c], col);
        put(ryb + 1, actb, yb2[c], col);
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nr * TW; e += NT) {
      const int r = e / TW, cc = e - r * TW, col = c0 + cc;
      if (col < nv) V[(long long)(b0 + r) * nv + col] = st[r * ld + cc];
    }
  }
}

size_t apply_rot_dual_lds_bytes(int n) {
  const int m = (n + 3) & ~3, nq = m / 4, P2 = (nq + 1) / 2;
  return std::max((size_t)APPLY_RCH * 8 * P2 * 16, (size_t)apply_dual_band(m) * 65 * 8);
}

int apply_rot_tile(int n) { return ((n + 3) & ~3) <= 128 ? 128 : 64; }
size_t apply_rot_lds_bytes(int n) {
  const size_t m = (size_t)((n + 3) & ~3);
  return std::max((size_t)APPLY_RCH * m * 16, m * (size_t)(apply_rot_tile(n) + 1) * 8);  // parameters, then the tile
}
int apply_rot_waves(int) { return 64 / APPLY_COLS; }  // a 64-column tile
long long jacobi_rot_log_entries(int n) {
  const long long m = (n + 3) & ~3;
  return m / 2 + (m / 2 - 1) * m;
}

}  // namespace fx

namespace fx {

// ---------------------------------------------------------------------------
// Cholesky factor and its inverse in LDS: A = L L^T (A from Apool), X = L^-1
// to Xpool (strict upper triangle zero).  The lower triangle is kept packed
// row by row in LDS in precision T and overwritten in place: first by L
// (right-looking, one column per step, a wave per trailing row), then by
// L^-1, one column per step from the last (column j of the inverse needs the
// already inverted columns to its right and column j of L; four lanes share
// each row's dot product).  T = double gives the factor to working
// precision; with T = float the result is an approximate inverse factor that
// the caller refines.  A non-positive pivot sets status 2.
constexpr int CHOL_THREADS = 1024;

__device__ inline int tri_index(int i, int j) { return i * (i + 1) / 2 + j; }  // j <= i

// Factor and invert in place the packed lower triangle L (n x n, loaded):
// afterwards L holds L^-1.  col and dinv: n + 1 doubles of LDS scratch.
// Returns false (uniformly) on a non-positive pivot.
template <typename T>
__device__ bool chol_inv_packed(T* L, int n, double* col, double* dinv) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwave = nth >> 6;
  for (int k = 0; k < n; ++k) {
    const double dkk = (double)L[tri_index(k, k)];
    if (!(dkk > 0.0)) return false;  // same value in every thread: uniform exit
    const double rp = 1.0 / sqrt(dkk);
    for (int i = k + 1 + tid; i < n; i += nth) {
      const T v = (T)((double)L[tri_index(i, k)] * rp);
      L[tri_index(i, k)] = v;
      col[i] = (double)v;
    }
    __syncthreads();
    if (tid == 0) L[tri_index(k, k)] = (T)sqrt(dkk);
    for (int i = k + 1 + wave; i < n; i += nwave) {
      const double ci = col[i];
      T* row = L + tri_index(i, 0);
      for (int j = k + 1 + lane; j <= i; j += 64) row[j] = (T)((double)row[j] - ci * col[j]);
    }
    __syncthreads();
  }
  // in-place inverse: X_jj = 1 / L_jj, X_ij = -X_jj sum_{k=j+1..i} X_ik L_kj
  const int g = tid & 3, grp = tid >> 2, ngrp = nth >> 2;
  for (int j = n - 1; j >= 0; --j) {
    for (int i = j + 1 + tid; i < n; i += nth) col[i] = (double)L[tri_index(i, j)];
    if (tid == 0) {
      const double x = 1.0 / (double)L[tri_index(j, j)];
      dinv[0] = x;
      L[tri_index(j, j)] = (T)x;
    }
    __syncthreads();
    const double xjj = dinv[0];
    for (int i0 = j + 1; i0 < n; i0 += ngrp) {
      const int i = i0 + grp;  // the four lanes of a group share i: uniform within the group
      double v = 0.0;
      if (i < n) {
        const T* row = L + tri_index(i, 0);
        for (int k = j + 1 + g; k <= i; k += 4) v += (double)row[k] * col[k];
      }
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      if (i < n && g == 0) L[tri_index(i, j)] = (T)(-xjj * v);
    }
    __syncthreads();
  }
  return true;
}

template <typename T>
__global__ void __launch_bounds__(CHOL_THREADS)
    k_cholinv_lds(DevBatch bt, const int* list, const double* __restrict__ Apool, double* __restrict__ Xpool) {
  extern __shared__ double2 lds_raw[];
  const int si = list[blockIdx.x];
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  const int ntri = n * (n + 1) / 2;
  T* L = reinterpret_cast<T*>(lds_raw);
  double* col = reinterpret_cast<double*>(lds_raw) + (ntri * (int)sizeof(T) + 7) / 8;
  double* dinv = col + n;
  const double* A = Apool + d.mat_off;
  double* X = Xpool + d.mat_off;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int e = tid; e < n * n; e += nth) {
    const int i = e / n, j = e - i * n;
    if (j <= i) L[tri_index(i, j)] = (T)A[e];
  }
  __syncthreads();
  if (!chol_inv_packed<T>(L, n, col, dinv)) {
    if (tid == 0) bt.status[si] = 2;
    return;
  }
  for (int e = tid; e < n * n; e += nth) {
    const int i = e / n, j = e - i * n;
    X[e] = j <= i ? (double)L[tri_index(i, j)] : 0.0;
  }
}

// The same inverse factor for a two-fragment cluster started from its
// monomers' orbitals: G = C0^T S C0 = [[I, X], [X^T, I]] (the monomer blocks
// are the identity to FP64 rounding), so L = [[I, 0], [X^T, L22]] with
// L22 L22^T = I - X^T X, and L^-1 = [[I, 0], [-L22^-1 X^T, L22^-1]]: one
// factor of half the order instead of the whole.  FP32 in LDS (the caller
// refines the rows as after k_cholinv_lds<float>).  A non-positive pivot
// sets status 2.
__global__ void __launch_bounds__(CHOL_THREADS)
    k_cholinv_block2(DevBatch bt, const int* list, DevBatch mono, const double* __restrict__ Apool,
                     double* __restrict__ Xpool) {
  extern __shared__ double2 lds_raw[];
  const int si = list[blockIdx.x];
  const SysDesc d = bt.desc[si];
  const int n = d.nao, n1 = mono.desc[d.frag[0]].nao, n2 = n - n1;
  const int t2 = n2 * (n2 + 1) / 2;
  float* L = reinterpret_cast<float*>(lds_raw);  // packed lower triangle, n2
  float* XT = L + ((t2 + 3) & ~3);                // X^T, n2 x n1
  double* col = reinterpret_cast<double*>(XT + (((long long)n2 * n1 + 3) & ~3));
  double* dinv = col + n2;
  const double* A = Apool + d.mat_off;
  double* X = Xpool + d.mat_off;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int e = tid; e < n2 * n1; e += nth) {
    const int i = e / n1, j = e - i * n1;
    XT[e] = (float)A[(long long)(n1 + i) * n + j];
  }
  __syncthreads();
  // I - X^T X, lower triangle
  for (int e = tid; e < t2; e += nth) {
    int i = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
    while (i * (i + 1) / 2 > e) --i;
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    const int k = e - i * (i + 1) / 2;
    const float* a = XT + (long long)i * n1;
    const float* b = XT + (long long)k * n1;
    double v = i == k ? 1.0 : 0.0;
    for (int j = 0; j < n1; ++j) v -= (double)a[j] * (double)b[j];
    L[e] = (float)v;
  }
  __syncthreads();
  if (!chol_inv_packed<float>(L, n2, col, dinv)) {
    if (tid == 0) bt.status[si] = 2;
    return;
  }
  // rows of L^-1: [I 0] for the first fragment, [-L22^-1 X^T, L22^-1] below
  for (long long e = tid; e < (long long)n * n; e += nth) {
    const int i = (int)(e / n), j = (int)(e - (long long)i * n);
    double v;
    if (i < n1) {
      v = i == j ? 1.0 : 0.0;
    } else if (j >= n1) {
      const int a = i - n1, b = j - n1;
      v = b <= a ? (double)L[tri_index(a, b)] : 0.0;
    } else {
      const int a = i - n1;
      const float* lr = L + tri_index(a, 0);
      double s = 0.0;
      for (int k = 0; k <= a; ++k) s += (double)lr[k] * (double)XT[(long long)k * n1 + j];
      v = -s;
    }
    X[e] = v;
  }
}

size_t cholinv_block2_lds_bytes(int n1, int n2) {
  const size_t t2 = ((size_t)n2 * (n2 + 1) / 2 + 3) & ~(size_t)3;
  const size_t xt = ((size_t)n2 * n1 + 3) & ~(size_t)3;
  return (t2 + xt) * 4 + (size_t)n2 * 8 + 16;
}

template __global__ void k_cholinv_lds<double>(DevBatch, const int*, const double*, double*);
template __global__ void k_cholinv_lds<float>(DevBatch, const int*, const double*, double*);

size_t cholinv_lds_bytes(int n, int elt) {
  const size_t ntri = (size_t)n * (n + 1) / 2;
  return (ntri * elt + 7) / 8 * 8 + (size_t)n * 8 + 16;
}

// Third-order correction of nearly orthonormal rows Y (H = Y M Y^T = I + E):
// H <- (15 I - 10 H + 3 H^2) / 8, the series of H^-1/2 to second order in E,
// so that f(H) Y has f(H) H f(H) = I + O(E^3).
__global__ void k_ns_poly(DevBatch bt, const int* list, double* Hpool, const double* H2pool) {
  const int si = list[blockIdx.y];
  if (bt.status[si] != 0) return;
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  double* H = Hpool + d.mat_off;
  const double* H2 = H2pool + d.mat_off;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
    const int i = e / n, j = e - i * n;
    H[e] = ((i == j ? 15.0 : 0.0) - 10.0 * H[e] + 3.0 * H2[e]) * 0.125;
  }
}

}  // namespace fx
