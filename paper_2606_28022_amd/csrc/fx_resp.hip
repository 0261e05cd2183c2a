// Response of the self-consistent embedding for the FMO2 gradient.
//
// The energy depends on the monomer charges q^K through the Lagrangian
// potential v_K of eq. esp_lagrangian.  The charges respond to a geometry
// change through each monomer's SCC response: with the shell-summed
// occupied-virtual transition charges Q_ai,s of eq. lagrangian,
//   M = sum_ai Q_ai Q_ai^T / (eps_a - eps_i),  G = gamma_KK - 2 Gamma_A dq_A,
// the adjoint of the monomer self-consistency is y = v + Gamma_off chi y with
// chi = -(1 + M G)^-1 M, solved by Anderson-accelerated sweeps (each sweep is
// one embedding-field pass).  With w = (1 + G M)^-1 y the Z-vector is
// Z_ai = -2 (w . Q_ai) / (eps_a - eps_i) (the solution of eq. sczv for this
// Hamiltonian); its AO forms (eqs. Z_AO, WZ_def) and the Mulliken term of the
// fixed-orbital charge change (eq. resp_addlag) enter the same derivative
// contraction as the explicit gradient.
#include <hip/hip_runtime.h>

#include "fx_device.hpp"
#include "fx_kernels.hpp"

namespace fx {

// order the MOs of every system: the nocc lowest eigenvalues first (ties by
// index), then the virtuals, both ascending.
__global__ void k_mo_order(DevBatch bt, const int* nocc, int* order) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const double* e = bt.eps + d.ao_off;
  for (int i = threadIdx.x; i < d.nao; i += blockDim.x) {
    int r = 0;
    double ei = e[i];
    for (int j = 0; j < d.nao; ++j) r += (e[j] < ei || (e[j] == ei && j < i)) ? 1 : 0;
    order[d.ao_off + r] = i;
  }
  (void)nocc;
}

// AO range of local shell s of a system: first AO and count
__device__ inline void shell_aos(const DevSystem& sys, const DevBatch& bt, const SysDesc& d, int s, int& mu0,
                                 int& nao) {
  const int la = bt.sys_sh_atom[d.sh_off + s];
  const DevElem& el = sys.elems[sys.elem[bt.sys_atoms[d.atom_off + la]]];
  const int ls = s - bt.sys_atom_sh0[d.atom_off + la];
  mu0 = bt.sys_atom_ao0[d.atom_off + la] + el.ao0[ls];
  nao = el.nao_sh[ls];
}

// Q[s][a'][i'] = sum_{mu in s} (C_mu,a (SC)_mu,i + C_mu,i (SC)_mu,a)
// (Ct rows are MOs; SCt = Ct S holds (SC)^T).  The shells are taken in runs
// of at most RQ_CH consecutive AOs; the run's columns of Ct and SCt (every
// MO) are staged in LDS with coalesced row-segment reads, then each shell's
// nv x no block of Q is written with consecutive addresses.
size_t resp_Q_lds_bytes(int n) { return (size_t)2 * RQ_CH * n * sizeof(double) + (size_t)n * sizeof(int); }

__global__ void __launch_bounds__(256) k_resp_Q(DevSystem sys, DevBatch bt, const double* SCt, const int* order,
                                                const int* nocc, const long long* qoff, double* Q) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int n = d.nao, no = nocc[si], nv = n - no, ns = d.nsh;
  const double* Ct = bt.Ct + d.mat_off;
  const double* T = SCt + d.mat_off;
  extern __shared__ double rq_lds[];
  double* cs = rq_lds;                                  // [RQ_CH][n]: C of the run's AOs, every MO
  double* ts = cs + RQ_CH * n;                          // [RQ_CH][n]: SC likewise
  int* ord = reinterpret_cast<int*>(ts + RQ_CH * n);    // [n]
  for (int k = threadIdx.x; k < n; k += blockDim.x) ord[k] = order[d.ao_off + k];
  const int K = nv * no;
  double* Qs = Q + qoff[si];
  for (int s = 0; s < ns;) {
    int mua, na;
    shell_aos(sys, bt, d, s, mua, na);
    int s1 = s + 1, mub = mua + na;
    while (s1 < ns) {
      int m1, n1;
      shell_aos(sys, bt, d, s1, m1, n1);
      if (m1 + n1 - mua > RQ_CH) break;
      mub = m1 + n1;
      ++s1;
    }
    const int w = mub - mua;
    __syncthreads();  // the previous run is consumed (and ord written)
    for (int e = threadIdx.x; e < n * w; e += blockDim.x) {
      const int r = e / w, u = e - r * w;
      cs[u * n + r] = Ct[(long long)r * n + mua + u];
      ts[u * n + r] = T[(long long)r * n + mua + u];
    }
    __syncthreads();
    for (int t = s; t < s1; ++t) {
      int m0, nu;
      shell_aos(sys, bt, d, t, m0, nu);
      const int u0 = m0 - mua;
      double* Qt = Qs + (long long)t * K;
      for (int idx = threadIdx.x; idx < K; idx += blockDim.x) {
        const int ap = idx / no, ip = idx - ap * no;
        const int a = ord[no + ap], i = ord[ip];
        double v = 0.0;
        for (int u = u0; u < u0 + nu; ++u) v += cs[u * n + a] * ts[u * n + i] + cs[u * n + i] * ts[u * n + a];
        Qt[idx] = v;
      }
    }
    s = s1;
  }
}

// M = sum_ai Q_ai Q_ai^T / (eps_a - eps_i), per system (into the nsh^2
// pool): the (a, i) index is staged through LDS 64 columns at a time
// together with the inverse gaps; each thread accumulates a 4 x 4 block of
// the upper block triangle in registers over all chunks in order (eight LDS
// reads per sixteen products), then writes it and its mirror (on the
// diagonal blocks the upper entries, mirrored, so that M is exactly
// symmetric).
constexpr int RM_KC = 64, RM_LD = RM_KC + 1;
__global__ void __launch_bounds__(256) k_resp_M(DevBatch bt, const int* order, const int* nocc, const long long* qoff,
                                                const double* Q, double* M) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int n = d.nao, no = nocc[si], nv = n - no, ns = d.nsh;
  const int* ord = order + d.ao_off;
  const double* e = bt.eps + d.ao_off;
  const long long K = (long long)nv * no;
  const double* Qs = Q + qoff[si];
  extern __shared__ double rm_lds[];
  const int nb = (ns + 3) / 4, nrow = 4 * nb;
  double* qt = rm_lds;                   // [4 nb][RM_LD] (rows past ns zero)
  double* idn = rm_lds + nrow * RM_LD;   // [RM_KC]
  const int nblk = nb * (nb + 1) / 2;
  double* Mo = M + d.gam_off;
  for (int g0 = 0; g0 < nblk; g0 += (int)blockDim.x) {
    const int blk = g0 + (int)threadIdx.x;
    int bs = 0, bb = 0;
    if (blk < nblk) {
      // upper-triangle block number -> (bs, bb), bs <= bb
      int rem = blk;
      while (rem >= nb - bs) {
        rem -= nb - bs;
        ++bs;
      }
      bb = bs + rem;
    }
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    for (long long k0 = 0; k0 < K; k0 += RM_KC) {
      const int kn = (int)((K - k0) < RM_KC ? (K - k0) : RM_KC);
      __syncthreads();
      for (int x = threadIdx.x; x < nrow * RM_KC; x += blockDim.x) {
        const int sh = x / RM_KC, k = x - sh * RM_KC;
        qt[sh * RM_LD + k] = (k < kn && sh < ns) ? Qs[(long long)sh * K + k0 + k] : 0.0;
      }
      for (int k = threadIdx.x; k < RM_KC; k += blockDim.x) {
        double v = 0.0;
        if (k < kn) {
          const long long kk = k0 + k;
          const int ap = (int)(kk / no), ip = (int)(kk - (long long)ap * no);
          v = 1.0 / (e[ord[no + ap]] - e[ord[ip]]);
        }
        idn[k] = v;
      }
      __syncthreads();
      if (blk < nblk) {
        const double* qa = qt + 4 * bs * RM_LD;
        const double* qb = qt + 4 * bb * RM_LD;
        for (int k = 0; k < kn; ++k) {
          const double w = idn[k];
          double a[4], b[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            a[u] = qa[u * RM_LD + k] * w;
            b[u] = qb[u * RM_LD + k];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
        }
      }
    }
    if (blk < nblk) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int s = 4 * bs + u, t = 4 * bb + v;
          if (s >= ns || t >= ns || (bs == bb && v < u)) continue;
          Mo[(long long)s * ns + t] = acc[u][v];
          Mo[(long long)t * ns + s] = acc[u][v];
        }
    }
  }
}

// The same M on the FP64 matrix cores for systems of up to 16 RMM_MAXB
// shells: the upper 16 x 16 blocks of M = (Q diag(w)) Q^T, dealt to the four
// waves in turn, each accumulated with v_mfma_f64_16x16x4 over the staged
// (a, i) chunks (rows padded to whole blocks with zeros, the chunk's tail
// steps with zero weights), then written with their mirrors (on the
// diagonal blocks the upper entries, so that M is exactly symmetric).
typedef double rm_v4d __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_resp_M_mfma(DevBatch bt, const int* order, const int* nocc,
                                                     const long long* qoff, const double* Q, double* M) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int n = d.nao, no = nocc[si], nv = n - no, ns = d.nsh;
  const int* ord = order + d.ao_off;
  const double* e = bt.eps + d.ao_off;
  const long long K = (long long)nv * no;
  const double* Qs = Q + qoff[si];
  extern __shared__ double rm_lds[];
  const int nb = (ns + 15) / 16, nrow = 16 * nb;
  double* qt = rm_lds;                  // [nrow][RM_LD] (rows past ns zero)
  double* idn = rm_lds + nrow * RM_LD;  // [RM_KC]
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nblk = nb * (nb + 1) / 2;
  constexpr int QB = (RMM_MAXB * (RMM_MAXB + 1) / 2 + 3) / 4;  // blocks per wave, at most
  int bsr[QB], bbr[QB];
  rm_v4d acc[QB];
  int nmine = 0;
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    acc[q] = (rm_v4d){0.0, 0.0, 0.0, 0.0};
    const int blk = wave + 4 * q;
    int bs = 0, rem = blk < nblk ? blk : 0;
    while (rem >= nb - bs) {
      rem -= nb - bs;
      ++bs;
    }
    bsr[q] = bs;
    bbr[q] = bs + rem;
    nmine += blk < nblk;
  }
  const int i16 = lane & 15, kq = lane >> 4;
  for (long long k0 = 0; k0 < K; k0 += RM_KC) {
    const int kn = (int)((K - k0) < RM_KC ? (K - k0) : RM_KC);
    __syncthreads();
    for (int x = threadIdx.x; x < nrow * RM_KC; x += blockDim.x) {
      const int sh = x / RM_KC, k = x - sh * RM_KC;
      qt[sh * RM_LD + k] = (k < kn && sh < ns) ? Qs[(long long)sh * K + k0 + k] : 0.0;
    }
    for (int k = threadIdx.x; k < RM_KC; k += blockDim.x) {
      double v = 0.0;
      if (k < kn) {
        const long long kk = k0 + k;
        const int ap = (int)(kk / no), ip = (int)(kk - (long long)ap * no);
        v = 1.0 / (e[ord[no + ap]] - e[ord[ip]]);
      }
      idn[k] = v;
    }
    __syncthreads();
    for (int kk = 0; kk < kn; kk += 4) {
      const int k = kk + kq;
      const double w = idn[k];
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        if (q < nmine) {
          const double a = qt[(16 * bsr[q] + i16) * RM_LD + k] * w;
          const double b = qt[(16 * bbr[q] + i16) * RM_LD + k];
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
        }
      }
    }
  }
  double* Mo = M + d.gam_off;
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    if (q >= nmine) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int s = 16 * bsr[q] + kq + 4 * r, t = 16 * bbr[q] + i16;
      if (s >= ns || t >= ns || (bsr[q] == bbr[q] && t < s)) continue;
      Mo[(long long)s * ns + t] = acc[q][r];
      Mo[(long long)t * ns + s] = acc[q][r];
    }
  }
}

size_t resp_M_mfma_lds_bytes(int nsh) {
  return ((size_t)(16 * ((nsh + 15) / 16)) * RM_LD + RM_KC) * sizeof(double);
}

// dynamic LDS of k_resp_M for systems of up to nsh shells
size_t resp_M_lds_bytes(int nsh) { return ((size_t)(4 * ((nsh + 3) / 4)) * RM_LD + RM_KC) * sizeof(double); }

// R = (1 + G M)^-1 with G = gamma - 2 Gamma_A dq_A on same-atom shell blocks
// (Gauss-Jordan with partial pivoting on a work copy in Wk; one work-group).
__global__ void k_resp_R(DevSystem sys, DevBatch bt, const double* M, double* Wk, double* R) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int ns = d.nsh;
  const double* G = bt.gam + d.gam_off;
  double* A = Wk + d.gam_off;
  double* X = R + d.gam_off;
  __shared__ double qa[MAXN];
  __shared__ int piv;
  __shared__ double pv;
  const double* q = bt.q_out + d.sh_off;
  for (int a = threadIdx.x; a < d.nat; a += blockDim.x) {
    int s0 = bt.sys_atom_sh0[d.atom_off + a];
    int s1 = (a + 1 < d.nat) ? bt.sys_atom_sh0[d.atom_off + a + 1] : ns;
    double v = 0.0;
    for (int s = s0; s < s1; ++s) v += q[s];
    qa[a] = v;
  }
  __syncthreads();
  // A = I + G' M
  for (int idx = threadIdx.x; idx < ns * ns; idx += blockDim.x) {
    int s = idx / ns, t = idx % ns;
    double v = (s == t) ? 1.0 : 0.0;
    int as = bt.sys_sh_atom[d.sh_off + s];
    for (int k = 0; k < ns; ++k) {
      double g = G[(long long)s * ns + k];
      if (bt.sys_sh_atom[d.sh_off + k] == as) {
        int Aat = bt.sys_atoms[d.atom_off + as];
        g -= 2.0 * sys.elems[sys.elem[Aat]].Gamma * qa[as];
      }
      v += g * M[d.gam_off + (long long)k * ns + t];
    }
    A[idx] = v;
    X[idx] = (s == t) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int c = 0; c < ns; ++c) {
    if (threadIdx.x == 0) {
      int p = c;
      double best = fabs(A[(long long)c * ns + c]);
      for (int r = c + 1; r < ns; ++r) {
        double v = fabs(A[(long long)r * ns + c]);
        if (v > best) {
          best = v;
          p = r;
        }
      }
      piv = p;
    }
    __syncthreads();
    if (piv != c) {
      for (int k = threadIdx.x; k < ns; k += blockDim.x) {
        double t = A[(long long)c * ns + k];
        A[(long long)c * ns + k] = A[(long long)piv * ns + k];
        A[(long long)piv * ns + k] = t;
        t = X[(long long)c * ns + k];
        X[(long long)c * ns + k] = X[(long long)piv * ns + k];
        X[(long long)piv * ns + k] = t;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) pv = A[(long long)c * ns + c];
    __syncthreads();
    for (int k = threadIdx.x; k < ns; k += blockDim.x) {
      A[(long long)c * ns + k] /= pv;
      X[(long long)c * ns + k] /= pv;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < ns * ns; idx += blockDim.x) {
      int r = idx / ns, k = idx % ns;
      if (r == c) continue;
      double f = A[(long long)r * ns + c];
      if (k == c) continue;
      A[(long long)r * ns + k] -= f * A[(long long)c * ns + k];
      X[(long long)r * ns + k] -= f * X[(long long)c * ns + k];
    }
    __syncthreads();
    for (int r = threadIdx.x; r < ns; r += blockDim.x) {
      if (r == c) continue;
      double f = A[(long long)r * ns + c];
      X[(long long)r * ns + c] -= f * X[(long long)c * ns + c];
      A[(long long)r * ns + c] = 0.0;
    }
    __syncthreads();
  }
}

// The same R for systems whose ns x ns matrix fits in LDS (ns even-padded
// rows of double2): A = I + G' M with M read by column from HBM (consecutive
// threads, consecutive t) and G' rows from LDS, then Gauss-Jordan in place
// with partial pivoting (largest |A_ik|, i >= k, lowest index on ties), as
// the mixing preconditioner's: every wave finds the pivot itself from the
// pivot column, which is kept outside A (zero inside it, so the update leaves
// -c_i / pivot there), the first ld2 threads form the scaled pivot row and
// make the row interchange, thread (cg, rg) updates column pair cg of rows
// rg, rg + ng, ... and collects the next pivot column; two barriers per pivot.
// A singular A (pivot below 1e-300) leaves the identity.
__global__ void __launch_bounds__(RR_THREADS) k_resp_R_lds(DevSystem sys, DevBatch bt, const double* M, double* R) {
  extern __shared__ double2 A2[];  // [ns][ld2]
  double* A = reinterpret_cast<double*>(A2);
  __shared__ double gcor[MAXN];    // 2 Gamma_A dq_A of each shell's atom
  __shared__ int shat[MAXN];       // local atom of each shell
  __shared__ double colA[MAXN], colB[MAXN];
  __shared__ double2 rowk2[MAXN / 2];
  __shared__ int perm[MAXN];
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int ns = d.nsh, ldk = (ns + 1) & ~1, ld2 = ldk >> 1;
  const int lane = threadIdx.x & 63;
  const double* G = bt.gam + d.gam_off;
  const double* Mm = M + d.gam_off;
  const double* q = bt.q_out + d.sh_off;
  for (int a = threadIdx.x; a < d.nat; a += blockDim.x) {
    const int s0 = bt.sys_atom_sh0[d.atom_off + a];
    const int s1 = (a + 1 < d.nat) ? bt.sys_atom_sh0[d.atom_off + a + 1] : ns;
    double v = 0.0;
    for (int s = s0; s < s1; ++s) v += q[s];
    const double c = 2.0 * sys.elems[sys.elem[bt.sys_atoms[d.atom_off + a]]].Gamma * v;
    for (int s = s0; s < s1; ++s) {
      gcor[s] = c;
      shat[s] = a;
    }
  }
  __syncthreads();
  // G' into LDS (row-major, ldk)
  for (int e = threadIdx.x; e < ns * ns; e += blockDim.x) {
    const int s = e / ns, k = e - s * ns;
    double g = G[e];
    if (shat[s] == shat[k]) g -= gcor[s];
    A[s * ldk + k] = g;
  }
  __syncthreads();
  // A = I + G' M, each thread's elements in registers, then over G'
  constexpr int EPT = (MAXN_RESP_LDS * MAXN_RESP_LDS + RR_THREADS - 1) / RR_THREADS;
  double av[EPT];
  const int ne = ns * ns;
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    const int e = threadIdx.x + RR_THREADS * r;
    double v = 0.0;
    if (e < ne) {
      const int s = e / ns, t = e - s * ns;
      v = s == t ? 1.0 : 0.0;
      const double* gr = A + s * ldk;
#pragma unroll 8
      for (int k = 0; k < ns; ++k) v += gr[k] * Mm[(long long)k * ns + t];
    }
    av[r] = v;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < EPT; ++r) {
    const int e = threadIdx.x + RR_THREADS * r;
    if (e < ne) {
      const int s = e / ns, t = e - s * ns;
      A[s * ldk + t] = av[r];
    }
  }
  for (int s = threadIdx.x; s < ns; s += blockDim.x)
    if (ldk > ns) A[s * ldk + ns] = 0.0;  // the padding column
  __syncthreads();
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    colA[i] = A[i * ldk];
    A[i * ldk] = 0.0;
  }
  __syncthreads();
  // (fewest row groups: RR_THREADS / (MAXN_RESP_LDS / 2); most rows per thread)
  constexpr int NGMIN = RR_THREADS / (MAXN_RESP_LDS / 2);
  constexpr int RPT = (MAXN_RESP_LDS + NGMIN - 1) / NGMIN;
  const int ng = blockDim.x / ld2;
  const int cg = threadIdx.x % ld2, rg = threadIdx.x / ld2;
  bool good = true;
  for (int k = 0; k < ns; ++k) {
    const double* colc = (k & 1) ? colB : colA;
    double* coln = (k & 1) ? colA : colB;
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int i = k + lane; i < ns; i += 64) {
      const double v = fabs(colc[i]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    const double pvv = wave_max_f64(best);
    const int p = wave_min_i32(best == pvv ? bi : 0x7fffffff);
    if (!(pvv >= 1e-300)) {  // same value in every wave: uniform exit
      good = false;
      break;
    }
    if ((int)threadIdx.x < ld2) {
      const int c = threadIdx.x;
      const double piv = colc[p];
      double2 xp = A2[p * ld2 + c];
      if (c == (k >> 1)) {
        if (k & 1) xp.y = 1.0;
        else xp.x = 1.0;
      }
      rowk2[c] = make_double2(xp.x / piv, xp.y / piv);
      if (p != k) A2[p * ld2 + c] = A2[k * ld2 + c];
      if (c == 0) perm[k] = p;
    }
    __syncthreads();
    if (rg < ng) {
      const double2 rk = rowk2[cg];
      const double ck = colc[k];  // row p holds the former row k from now on
      const int k1 = k + 1;
      const bool collect = cg == (k1 >> 1);
      double2 x[RPT];
      double cr[RPT];
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int i = rg + ng * r;
        if (i < ns) {
          x[r] = A2[i * ld2 + cg];
          cr[r] = colc[i];
        }
      }
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int i = rg + ng * r;
        if (i < ns) {
          double2 v = rk;
          if (i != k) {
            const double ci = i == p ? ck : cr[r];
            v = x[r];
            v.x = v.x - ci * rk.x;
            v.y = v.y - ci * rk.y;
          }
          if (collect) {
            if (k1 & 1) {
              coln[i] = v.y;
              v.y = 0.0;
            } else {
              coln[i] = v.x;
              v.x = 0.0;
            }
          }
          A2[i * ld2 + cg] = v;
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
          const double t = A[i * ldk + k];
          A[i * ldk + k] = A[i * ldk + p];
          A[i * ldk + p] = t;
        }
        __syncthreads();
      }
    }
  }
  double* X = R + d.gam_off;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    const int s = e / ns, t = e - s * ns;
    X[e] = good ? A[s * ldk + t] : (s == t ? 1.0 : 0.0);
  }
}

// w = R y,  u = -M w   (local shell vectors)
__global__ void k_resp_apply(DevBatch bt, const double* R, const double* M, const double* y, double* w, double* u) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int ns = d.nsh;
  __shared__ double ws[MAXN];
  for (int s = threadIdx.x; s < ns; s += blockDim.x) {
    double v = 0.0;
    for (int t = 0; t < ns; ++t) v += R[d.gam_off + (long long)s * ns + t] * y[d.sh_off + t];
    ws[s] = v;
    w[d.sh_off + s] = v;
  }
  __syncthreads();
  for (int s = threadIdx.x; s < ns; s += blockDim.x) {
    double v = 0.0;
    for (int t = 0; t < ns; ++t) v += M[d.gam_off + (long long)s * ns + t] * ws[t];
    u[d.sh_off + s] = -v;
  }
}

// Z in the MO basis: Zm[a][i] = -2 (w . Q_ai) / (eps_a - eps_i) and
// Ze[a][i] = Zm[a][i] eps_i (zero elsewhere)
__global__ void k_resp_Z(DevBatch bt, const int* order, const int* nocc, const long long* qoff, const double* Q,
                         const double* w, double* Zm, double* Ze) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int n = d.nao, no = nocc[si], nv = n - no, ns = d.nsh;
  const int* ord = order + d.ao_off;
  const double* e = bt.eps + d.ao_off;
  const long long K = (long long)nv * no;
  for (long long idx = threadIdx.x; idx < (long long)n * n; idx += blockDim.x) {
    Zm[d.mat_off + idx] = 0.0;
    Ze[d.mat_off + idx] = 0.0;
  }
  __syncthreads();
  for (long long k = threadIdx.x; k < K; k += blockDim.x) {
    int ap = (int)(k / no), ip = (int)(k % no);
    int a = ord[no + ap], i = ord[ip];
    double v = 0.0;
    for (int s = 0; s < ns; ++s) v += w[d.sh_off + s] * Q[qoff[si] + (long long)s * K + k];
    double z = -2.0 * v / (e[a] - e[i]);
    Zm[d.mat_off + (long long)a * n + i] = z;
    Ze[d.mat_off + (long long)a * n + i] = z * e[i];
  }
}

// out = diag(w_shell) P  (row scaling by the shell value of each AO)
__global__ void k_rowscale(DevBatch bt, const double* wsh, const double* P, double* out) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  const int* aosh = bt.sys_ao_sh + d.ao_off;
  for (long long idx = threadIdx.x; idx < (long long)n * n; idx += blockDim.x) {
    int i = (int)(idx / n);
    out[d.mat_off + idx] = wsh[d.sh_off + aosh[i]] * P[d.mat_off + idx];
  }
}

// symmetrise a matrix pool in place: A <- (A + A^T) / 2
__global__ void k_sym_inplace(DevBatch bt, double* A) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  for (long long idx = threadIdx.x; idx < (long long)n * n; idx += blockDim.x) {
    int i = (int)(idx / n), j = (int)(idx % n);
    if (j <= i) continue;
    double a = A[d.mat_off + (long long)i * n + j], b = A[d.mat_off + (long long)j * n + i];
    double m = 0.5 * (a + b);
    A[d.mat_off + (long long)i * n + j] = m;
    A[d.mat_off + (long long)j * n + i] = m;
  }
}

// D_S of the response: 1/2 (sig_i + sig_j) Zb - sym(WZ) + 1/2 (w_i + w_j) P - 1/4 (X2 + X2^T)
// and gx = 2 Q^Z with Q^Z_s = sum_{mu in s} sum_nu Zb_mu,nu S_mu,nu
__global__ void k_resp_DS(DevBatch bt, const double* Zb, const double* WZ, const double* X2, const double* wsh,
                          double* DS, double* gx) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  const int* aosh = bt.sys_ao_sh + d.ao_off;
  const double* sg = bt.sig + d.sh_off;
  const double* w = wsh + d.sh_off;
  const double* P = bt.P + d.mat_off;
  const double* S = bt.S + d.mat_off;
  const long long o = d.mat_off;
  for (long long idx = threadIdx.x; idx < (long long)n * n; idx += blockDim.x) {
    int i = (int)(idx / n), j = (int)(idx % n);
    long long ij = o + idx, ji = o + (long long)j * n + i;
    int si_ = aosh[i], sj_ = aosh[j];
    DS[ij] = 0.5 * (sg[si_] + sg[sj_]) * Zb[ij] - 0.5 * (WZ[ij] + WZ[ji]) + 0.5 * (w[si_] + w[sj_]) * P[idx] -
             0.25 * (X2[ij] + X2[ji]);
  }
  __shared__ double pop[MAXN];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double v = 0.0;
    for (int j = 0; j < n; ++j) v += Zb[o + (long long)i * n + j] * S[(long long)i * n + j];
    pop[i] = v;
  }
  __syncthreads();
  for (int s = threadIdx.x; s < d.nsh; s += blockDim.x) {
    double v = 0.0;
    for (int i = 0; i < n; ++i)
      if (aosh[i] == s) v += pop[i];
    gx[d.sh_off + s] = 2.0 * v;
  }
}

// per cluster system: cross-fragment potential of a local shell vector x,
// out_s = sum_{t in X, frag(t) != frag(s)} gamma_st x_t
__global__ void k_cluster_cross(DevSystem sys, DevBatch bt, const double* x, const double* qmono, const double* w,
                                double* out, double* out_gh) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int* shg = bt.sys_sh_global + d.sh_off;
  const int h0 = bt.healed_off ? bt.healed_off[si] : 0, h1 = bt.healed_off ? bt.healed_off[si + 1] : 0;
  const double wx = w ? w[si] : 1.0;
  for (int s = threadIdx.x; s < d.nsh; s += blockDim.x) {
    int fs = sys.sh_frag[shg[s]];
    double v = 0.0;
    for (int t = 0; t < d.nsh; ++t) {
      if (sys.sh_frag[shg[t]] == fs) continue;
      v += bt.gam[d.gam_off + (long long)s * d.nsh + t] * x[d.sh_off + t];
    }
    // the charge transfer -w q of the ghosts healed inside the cluster (eq.
    // ctij_ghost) on the shells of the other fragment
    const int gs = shg[s], As = sys.sh_atom[gs];
    for (int e = h0; e < h1; ++e) {
      const int t = bt.healed_sh[e], G = sys.sh_atom[t];
      if (sys.sh_frag[t] == fs) continue;
      double R2 = 0.0;
      for (int k = 0; k < 3; ++k) {
        const double dx = sys.xyz[3 * As + k] - sys.xyz[3 * G + k];
        R2 += dx * dx;
      }
      v += gamma_pair(sys.g, sqrt(R2), sys.sh_eta[gs], sys.sh_eta[t]) * (-wx * qmono[t]);
    }
    out[d.sh_off + s] = v;
  }
  // the same cross-fragment potential at the healed ghosts' own shells (they
  // are monomer shells of one of the cluster's fragments, outside its basis)
  if (!out_gh) return;
  for (int e = h0 + threadIdx.x; e < h1; e += blockDim.x) {
    const int gs = bt.healed_sh[e], fs = sys.sh_frag[gs], As = sys.sh_atom[gs];
    auto gam = [&](int t) {
      const int At = sys.sh_atom[t];
      double R2 = 0.0;
      for (int k = 0; k < 3; ++k) {
        const double dx = sys.xyz[3 * As + k] - sys.xyz[3 * At + k];
        R2 += dx * dx;
      }
      return gamma_pair(sys.g, sqrt(R2), sys.sh_eta[gs], sys.sh_eta[t]);
    };
    double v = 0.0;
    for (int t = 0; t < d.nsh; ++t)
      if (sys.sh_frag[shg[t]] != fs) v += gam(shg[t]) * x[d.sh_off + t];
    for (int e2 = h0; e2 < h1; ++e2) {
      const int t = bt.healed_sh[e2];
      if (sys.sh_frag[t] != fs) v += gam(t) * (-wx * qmono[t]);
    }
    out_gh[e] = v;
  }
}

// v[s] -= cross-fragment potential of the cluster that heals ghost shell s
__global__ void k_sub_healed(DevBatch bt, const double* vgh, double* v) {
  const int si = blockIdx.x;
  for (int e = bt.healed_off[si] + threadIdx.x; e < bt.healed_off[si + 1]; e += blockDim.x)
    v[bt.healed_sh[e]] -= vgh[e];
}

// dst[s] = base[s] + sign * sum over CSR entries of src[entry] (fixed order)
__global__ void k_gather_csr(int n, const int* rowptr, const int* ent, const double* src, const double* base,
                             double sign, double* dst) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  double v = 0.0;
  for (int e = rowptr[s]; e < rowptr[s + 1]; ++e) v += src[ent[e]];
  dst[s] = (base ? base[s] : 0.0) + sign * v;
}

__global__ void k_axpy(long long n, const double* x, double a, const double* y, double* out) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = x[k] + a * y[k];
}

}  // namespace fx
