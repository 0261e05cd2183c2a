// Kernels of the FMO2 and FMO3 analytic gradients (section "Analytic energy
// gradients" and its FMO3 extension).
//
// The gradient is assembled from the energy identity
//   E = sum_I c_I E^emb_I + sum_SCC s_IJ E^emb_IJ + sum_T E^emb_IJK
//       - sum_ESD (1 - n_T(IJ)) dq^I gamma dq^J,
//   n_T(IJ) = trimers containing I and J, s_IJ = 1 - n_T(IJ),
//   c_I = 1 - (SCC pairs containing I) + sum over trimers T containing I of
//         (SCC sub-pairs of T containing I - 1)
// (FMO2: no trimers, s = 1), whose fragment terms are stationary in their
// own densities:
//  * per fragment system: the single-system gradient of eq. xtb_grad with the
//    W matrix of eq. W_matrix (sigma containing the embedding potential), the
//    H0 derivative split of eq. H0_deriv and the CN sensitivity of
//    eq. cn_factor (k_grad_contract);
//  * inter-fragment kernel derivatives: ES-DIM (eq. esd_grad), charge-transfer
//    embedding (eq. ctij) and the response charges (eq. ZxG_inter) in one
//    N-body force pass over all cross-fragment shell pairs (k_force_inter)
//    with a per-cluster correction (k_grad_pair_corr);
//  * the CN chain of eq. cn_grad over all atoms (k_cn_grad);
//  * the response: the Lagrangian potential of eq. esp_lagrangian, the
//    fragment charge response built from the transition charges of
//    eq. lagrangian, the Z-vector and its AO forms of eqs. Z_AO, WZ_def,
//    contracted with the derivative integrals as in eqs. ZxHB .. ZxG and
//    resp_addlag (k_resp_*).
// Every per-atom sum is formed by one thread in a fixed order (no atomics),
// so the gradient is bitwise reproducible.
#include <hip/hip_runtime.h>

#include "fx_device.hpp"
#include "fx_kernels.hpp"

namespace fx {

__device__ inline double gamma_and_deriv(const DevGlobals& g, double R, double eta_s, double eta_t, double* dg) {
  double inv_eta = 0.5 * (1.0 / eta_s + 1.0 / eta_t);
  if (g.kg == 2.0) {
    double x = 1.0 / sqrt(R * R + inv_eta * inv_eta);
    *dg = -R * x * x * x;
    return x;
  }
  double base = pow(R, g.kg) + pow(inv_eta, g.kg);
  double gam = pow(base, -1.0 / g.kg);
  *dg = -pow(R, g.kg - 1.0) * pow(base, -1.0 / g.kg - 1.0);
  return gam;
}

// The overlap block of an atom pair, R = A - B (STO-6G s and p shells; a
// second s shell orthogonalised against the first, |s2'> = N (|s2> - S12 |s1>))
// and the contraction sum_ij W_ij dS_ij / dR of its
// derivative with a weight block W, added to g, without forming dS.  The
// orthogonalisation of a second s shell is a fixed linear map T on the AO
// index (S' = T_a S T_b^T), so the weights are moved through it once
// (W' = T_a^T W T_b) and contracted with the raw derivatives.  Per shell pair
// every primitive term has the form s00 times a polynomial in R with
// primitive-dependent coefficients fa = -b / (a + b), fb = a / (a + b),
// h = 1 / (2 (a + b)) and d s00 / dR_k = -2 mu R_k s00, so the primitive sums
// reduce to at most four scalars, and the block and the contraction follow
// from them and from R:
//   s s:  S = sum s00;                 g_k += W R_k sum(-2 mu s00)
//   p s:  S_u = R_u sum(fa s00);       g_k += W_k sum(fa s00) + (W.R) R_k sum(-2 mu fa s00)
//   s p:  likewise with fb and the columns of W
//   p p:  S_uv = R_u R_v sum(fa fb s00) + delta_uv sum(h s00);
//         g_k += ((W R)_k + (W^T R)_k) sum(fa fb s00)
//                + R_k (R.W.R sum(-2 mu fa fb s00) + tr W sum(-2 mu h s00))
__device__ void atom_pair_overlap_contract(const DevElem& ea, const DevElem& eb, const double Rv[3],
                                           double (&W)[MAXAO_EL][MAXAO_EL], double S[MAXAO_EL][MAXAO_EL],
                                           double g[3]) {
  const double PI = 3.14159265358979323846;
  const double R2 = Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2];
  if (ea.orth) {
#pragma unroll
    for (int j = 0; j < MAXAO_EL; ++j) {
      W[0][j] -= ea.orthN * ea.orthS12 * W[1][j];
      W[1][j] *= ea.orthN;
    }
  }
  if (eb.orth) {
#pragma unroll
    for (int i = 0; i < MAXAO_EL; ++i) {
      W[i][0] -= eb.orthN * eb.orthS12 * W[i][1];
      W[i][1] *= eb.orthN;
    }
  }
#pragma unroll
  for (int i = 0; i < MAXAO_EL; ++i)
#pragma unroll
    for (int j = 0; j < MAXAO_EL; ++j) S[i][j] = 0.0;
#pragma unroll
  for (int sa = 0; sa < MAXSH_EL; ++sa)
#pragma unroll
    for (int sb = 0; sb < MAXSH_EL; ++sb) {
      if (sa >= ea.nsh || sb >= eb.nsh) continue;
      const int la = ea.l[sa], lb = eb.l[sb];
      const int kind = 2 * la + lb;  // 0 s s, 1 s p, 2 p s, 3 p p
      // shell-pair sums over the primitives
      double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
#pragma unroll 1
      for (int i = 0; i < NPRIM; ++i) {
        const double a = ea.alpha[sa][i];
        for (int j = 0; j < NPRIM; ++j) {
          const double b = eb.alpha[sb][j];
          const double ip = 1.0 / (a + b);
          const double mu = a * b * ip;
          const double s00 = ea.coef[sa][i] * eb.coef[sb][j] * PI * ip * sqrt(PI * ip) * exp(-mu * R2);
          const double d00 = -2.0 * mu * s00;
          const double fa = -b * ip, fb = a * ip;
          if (kind == 0) {
            t0 += s00;
            t1 += d00;
          } else if (kind == 2) {
            t0 += fa * s00;
            t1 += fa * d00;
          } else if (kind == 1) {
            t0 += fb * s00;
            t1 += fb * d00;
          } else {
            const double ff = fa * fb, h = 0.5 * ip;
            t0 += ff * s00;
            t1 += ff * d00;
            t2 += h * s00;
            t3 += h * d00;
          }
        }
      }
      const int oa = sa, ob = sb;
      if (kind == 0) {
        S[oa][ob] = t0;
        for (int k = 0; k < 3; ++k) g[k] += W[oa][ob] * Rv[k] * t1;
      } else if (kind == 2) {
        double wr = 0.0;
        for (int u = 0; u < 3; ++u) {
          S[oa + u][ob] = Rv[u] * t0;
          wr += W[oa + u][ob] * Rv[u];
        }
        for (int k = 0; k < 3; ++k) g[k] += W[oa + k][ob] * t0 + wr * Rv[k] * t1;
      } else if (kind == 1) {
        double wc = 0.0;
        for (int v = 0; v < 3; ++v) {
          S[oa][ob + v] = Rv[v] * t0;
          wc += W[oa][ob + v] * Rv[v];
        }
        for (int k = 0; k < 3; ++k) g[k] += W[oa][ob + k] * t0 + wc * Rv[k] * t1;
      } else {
        double rw = 0.0, tr = 0.0, wr[3], wc[3];
        for (int u = 0; u < 3; ++u) {
          wr[u] = 0.0;
          wc[u] = 0.0;
          for (int v = 0; v < 3; ++v) {
            S[oa + u][ob + v] = Rv[u] * Rv[v] * t0 + (u == v ? t2 : 0.0);
            wr[u] += W[oa + u][ob + v] * Rv[v];
            wc[u] += W[oa + v][ob + u] * Rv[v];
          }
          rw += wr[u] * Rv[u];
          tr += W[oa + u][ob + u];
        }
        for (int k = 0; k < 3; ++k) g[k] += (wr[k] + wc[k]) * t0 + Rv[k] * (rw * t1 + tr * t3);
      }
    }
  if (ea.orth) {
#pragma unroll
    for (int j = 0; j < MAXAO_EL; ++j) S[1][j] = ea.orthN * (S[1][j] - ea.orthS12 * S[0][j]);
  }
  if (eb.orth) {
#pragma unroll
    for (int i = 0; i < MAXAO_EL; ++i) S[i][1] = eb.orthN * (S[i][1] - eb.orthS12 * S[i][0]);
  }
}

// ---------------------------------------------------------------------------
// Per-system derivative contraction:
//   d/dR_a [ sum D_H H0 + sum D_S S + 1/2 sum_{s,t} gx_s gamma_st gy_t + E_rep ]
// at fixed CN, for every atom a of the system, and the CN sensitivity
// F_a = d/dCN_a of the D_H term.  Results are multiplied by the system weight
// and written (or added) to the per-system atom arrays.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
    k_grad_contract(DevSystem sys, DevBatch bt, const int* list, const double* DHp, const double* DSp,
                                const double* gx, const double* gy, const double* wsys, int with_rep, int accumulate,
                                double* g_out, double* F_out, double* scratch) {
  const int si = list[blockIdx.x];
  const SysDesc d = bt.desc[si];
  const int n = d.nao, nat = d.nat;
  const double* DH = DHp + d.mat_off;
  const double* DS = DSp + d.mat_off;
  const int* atoms = bt.sys_atoms + d.atom_off;
  const int* aao = bt.sys_atom_ao0 + d.atom_off;
  const int* ash = bt.sys_atom_sh0 + d.atom_off;
  const double cw = wsys ? wsys[si] : 1.0;
  // every pair term is a function of R_a - R_b: each unordered pair (a < b)
  // is evaluated once, its gradient enters a with + and b with -, plus the
  // CN sensitivities of both atoms; 5 values per pair in the scratch block
  // (5 nat (nat - 1) / 2 <= n^2 doubles), then gathered per atom in order
  double* pb = scratch + d.mat_off;
  const int np = nat * (nat - 1) / 2;
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    int a = 0, rem = p;
    while (rem >= nat - 1 - a) {
      rem -= nat - 1 - a;
      ++a;
    }
    const int b = a + 1 + rem;
    const int A = atoms[a], B = atoms[b];
    const DevElem& ea = sys.elems[sys.elem[A]];
    const DevElem& eb = sys.elems[sys.elem[B]];
    const double cnA = sys.cn[A], cnB = sys.cn[B];
    const int oa = aao[a], ob = aao[b];
    double g[3] = {0.0, 0.0, 0.0};
    double Fa = 0.0, Fb = 0.0;
    double Rv[3] = {sys.xyz[3 * A] - sys.xyz[3 * B], sys.xyz[3 * A + 1] - sys.xyz[3 * B + 1],
                    sys.xyz[3 * A + 2] - sys.xyz[3 * B + 2]};
    double R = sqrt(Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2]);
    double uR[3] = {Rv[0] / R, Rv[1] / R, Rv[2] / R};
    double den = ea.EN - eb.EN;
    double enf = 1.0 + sys.g.kEN * den * den;
    double rcov = ea.rcov + eb.rcov;
    double x = sqrt(R / rcov);
    double dx = 0.5 / sqrt(R * rcov);
    // shell-pair factors (shell 0: AO 0; shell 1: AOs 1..)
    double fac[MAXSH_EL][MAXSH_EL], sumDHS[MAXSH_EL][MAXSH_EL];
#pragma unroll
    for (int sa = 0; sa < MAXSH_EL; ++sa)
#pragma unroll
      for (int sb = 0; sb < MAXSH_EL; ++sb) {
        sumDHS[sa][sb] = 0.0;
        fac[sa][sb] = 0.0;
        if (sa >= ea.nsh || sb >= eb.nsh) continue;
        const double kll = 0.5 * (sys.g.kl[ea.l[sa]] + sys.g.kl[eb.l[sb]]);
        const double ha = ea.level[sa] * (1.0 + ea.kcn[sa] * cnA);
        const double hb = eb.level[sb] * (1.0 + eb.kcn[sb] * cnB);
        const double pa = 1.0 + ea.kpoly[sa] * x, pbb = 1.0 + eb.kpoly[sb] * x;
        fac[sa][sb] = sys.g.KAB * kll * enf * 0.5 * (ha + hb) * pa * pbb;
      }
    // d/dR of sum (D_H H0 + D_S S) over the pair's overlap block: weights
    // 2 (fac D_H + D_S) (both triangles) contracted with dS / dR
    double W[MAXAO_EL][MAXAO_EL], S[MAXAO_EL][MAXAO_EL];
#pragma unroll
    for (int i = 0; i < MAXAO_EL; ++i)
#pragma unroll
      for (int j = 0; j < MAXAO_EL; ++j) {
        W[i][j] = 0.0;
        if (i >= ea.nao || j >= eb.nao) continue;
        const int sa = i == 0 ? 0 : 1, sb = j == 0 ? 0 : 1;
        const long long mn = (long long)(oa + i) * n + ob + j;
        W[i][j] = 2.0 * (fac[sa][sb] * DH[mn] + DS[mn]);
      }
    atom_pair_overlap_contract(ea, eb, Rv, W, S, g);
#pragma unroll
    for (int i = 0; i < MAXAO_EL; ++i)
#pragma unroll
      for (int j = 0; j < MAXAO_EL; ++j) {
        if (i >= ea.nao || j >= eb.nao) continue;
        const int sa = i == 0 ? 0 : 1, sb = j == 0 ? 0 : 1;
        sumDHS[sa][sb] += DH[(long long)(oa + i) * n + ob + j] * S[i][j];
      }
#pragma unroll
    for (int sa = 0; sa < MAXSH_EL; ++sa)
#pragma unroll
      for (int sb = 0; sb < MAXSH_EL; ++sb) {
        if (sa >= ea.nsh || sb >= eb.nsh) continue;
        const double kll = 0.5 * (sys.g.kl[ea.l[sa]] + sys.g.kl[eb.l[sb]]);
        const double ha = ea.level[sa] * (1.0 + ea.kcn[sa] * cnA);
        const double hb = eb.level[sb] * (1.0 + eb.kcn[sb] * cnB);
        const double hav = 0.5 * (ha + hb);
        const double pa = 1.0 + ea.kpoly[sa] * x, pbb = 1.0 + eb.kpoly[sb] * x;
        const double Pi = pa * pbb;
        const double dPi = (ea.kpoly[sa] * pbb + pa * eb.kpoly[sb]) * dx;
        const double base = sys.g.KAB * kll * enf;
        const double t = 2.0 * sumDHS[sa][sb] * base * hav * dPi;
        for (int k = 0; k < 3; ++k) g[k] += t * uR[k];
        Fa += 2.0 * sumDHS[sa][sb] * base * Pi * 0.5 * ea.level[sa] * ea.kcn[sa];
        Fb += 2.0 * sumDHS[sa][sb] * base * Pi * 0.5 * eb.level[sb] * eb.kcn[sb];
      }
    if (gx) {
      int s0 = ash[a], t0 = ash[b];
      for (int sa = 0; sa < ea.nsh; ++sa)
        for (int sb = 0; sb < eb.nsh; ++sb) {
          double dg;
          gamma_and_deriv(sys.g, R, ea.eta[sa], eb.eta[sb], &dg);
          double c = 0.5 * (gx[d.sh_off + s0 + sa] * gy[d.sh_off + t0 + sb] +
                            gy[d.sh_off + s0 + sa] * gx[d.sh_off + t0 + sb]);
          for (int k = 0; k < 3; ++k) g[k] += c * dg * uR[k];
        }
    }
    if (with_rep) {
      double al = sqrt(ea.arep * eb.arep);
      // repulsion charges of boundary atoms are scaled (detached atom, ghost)
      const double zs = bt.atom_zs ? bt.atom_zs[d.atom_off + a] * bt.atom_zs[d.atom_off + b] : 1.0;
      double e = zs * ea.zeff * eb.zeff / R * exp(-al * pow(R, sys.g.kf));
      double de = e * (-1.0 / R - al * sys.g.kf * pow(R, sys.g.kf - 1.0));
      for (int k = 0; k < 3; ++k) g[k] += de * uR[k];
    }
    double* o = pb + 5LL * p;
    o[0] = g[0];
    o[1] = g[1];
    o[2] = g[2];
    o[3] = Fa;
    o[4] = Fb;
  }
  __syncthreads();
  for (int a = threadIdx.x; a < nat; a += blockDim.x) {
    const int A = atoms[a];
    const DevElem& ea = sys.elems[sys.elem[A]];
    const int oa = aao[a];
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < ea.nsh; ++s)
      for (int u = 0; u < ea.nao_sh[s]; ++u) {
        int mu = oa + ea.ao0[s] + u;
        t[3] += DH[(long long)mu * n + mu] * ea.level[s] * ea.kcn[s];
      }
    for (int b = 0; b < nat; ++b) {
      if (b == a) continue;
      if (b > a) {
        const double* q = pb + 5LL * (a * (2 * nat - a - 1) / 2 + (b - a - 1));
        t[0] += q[0];
        t[1] += q[1];
        t[2] += q[2];
        t[3] += q[3];
      } else {
        const double* q = pb + 5LL * (b * (2 * nat - b - 1) / 2 + (a - b - 1));
        t[0] -= q[0];
        t[1] -= q[1];
        t[2] -= q[2];
        t[3] += q[4];
      }
    }
    long long o = (long long)d.atom_off + a;
    for (int k = 0; k < 3; ++k) {
      double v = cw * t[k];
      g_out[3 * o + k] = accumulate ? g_out[3 * o + k] + v : v;
    }
    F_out[o] = accumulate ? F_out[o] + cw * t[3] : cw * t[3];
  }
}

// For an SCC dimer (I, K): remove the cross-fragment pairs of the all-pairs
// inter-fragment force, c_st = q_s q_t + ddq_s q_t + q_s ddq_t (added to the
// dimer's atom arrays).
// Correction of the all-pairs force pass inside each cluster X (an SCC dimer
// or a trimer): for every atom pair of different fragments of X it removes
//   w_X (ddq^X_s q_t + q_s ddq^X_t)   (the charge transfer acts only on
//                                      fragments outside X)
// and, for the sub-pairs selected by qqmask (bit 0: fragments 0,1; bit 1:
// 0,2; bit 2: 1,2; null = every sub-pair), q_s q_t (an SCC pair has no
// ES-DIM term; an ES-DIM sub-pair inside a trimer carries 1 - n_T of it).
// w null: w_X = 1.
__global__ void k_grad_pair_corr(DevSystem sys, DevBatch bt, const double* qmono, const double* ddq,
                                 const double* wct, const int* qqmask, double* g_out, double* ghost_out) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int nat = d.nat;
  const int* atoms = bt.sys_atoms + d.atom_off;
  const int* ash = bt.sys_atom_sh0 + d.atom_off;
  const double wx = wct ? wct[si] : 1.0;
  const int mask = qqmask ? qqmask[si] : 7;
  // ghosts of bonds healed inside the cluster: not atoms of the cluster, but
  // their monomer charges are cross-fragment charges of the all-pairs pass
  // and their charge transfer is -q (eq. ctij_ghost)
  const int h0 = bt.healed_off ? bt.healed_off[si] : 0, h1 = bt.healed_off ? bt.healed_off[si + 1] : 0;
  for (int a = threadIdx.x; a < nat; a += blockDim.x) {
    const int A = atoms[a];
    const DevElem& ea = sys.elems[sys.elem[A]];
    const int fa = sys.frag[A];
    const int pa = fa == d.frag[0] ? 0 : (fa == d.frag[1] ? 1 : 2);
    double g[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < nat; ++b) {
      const int B = atoms[b];
      const int fb = sys.frag[B];
      if (fb == fa) continue;
      const int pb = fb == d.frag[0] ? 0 : (fb == d.frag[1] ? 1 : 2);
      const int sub = pa + pb - 1;  // (0,1) -> 0, (0,2) -> 1, (1,2) -> 2
      const double wqq = (mask >> sub) & 1 ? 1.0 : 0.0;
      const DevElem& eb = sys.elems[sys.elem[B]];
      double Rv[3] = {sys.xyz[3 * A] - sys.xyz[3 * B], sys.xyz[3 * A + 1] - sys.xyz[3 * B + 1],
                      sys.xyz[3 * A + 2] - sys.xyz[3 * B + 2]};
      double R = sqrt(Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2]);
      for (int sa = 0; sa < ea.nsh; ++sa)
        for (int sb = 0; sb < eb.nsh; ++sb) {
          int ls = ash[a] + sa, lt = ash[b] + sb;
          double qs = qmono[sys.atom_sh0[A] + sa], qt = qmono[sys.atom_sh0[B] + sb];
          double c = wqq * qs * qt + wx * (ddq[d.sh_off + ls] * qt + qs * ddq[d.sh_off + lt]);
          double dg;
          gamma_and_deriv(sys.g, R, ea.eta[sa], eb.eta[sb], &dg);
          for (int k = 0; k < 3; ++k) g[k] -= c * dg * Rv[k] / R;
        }
    }
    for (int e = h0; e < h1; ++e) {
      const int t = bt.healed_sh[e], G = sys.sh_atom[t];
      if (sys.frag[G] == fa) continue;
      double Rv[3] = {sys.xyz[3 * A] - sys.xyz[3 * G], sys.xyz[3 * A + 1] - sys.xyz[3 * G + 1],
                      sys.xyz[3 * A + 2] - sys.xyz[3 * G + 2]};
      double R = sqrt(Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2]);
      if (R == 0.0) continue;  // a ghost on its own detached atom: gamma is flat there
      const double qt = qmono[t];
      for (int sa = 0; sa < ea.nsh; ++sa) {
        const double qs = qmono[sys.atom_sh0[A] + sa];
        const double c = qs * qt + wx * (ddq[d.sh_off + ash[a] + sa] * qt - qs * qt);
        double dg;
        gamma_and_deriv(sys.g, R, ea.eta[sa], sys.sh_eta[t], &dg);
        for (int k = 0; k < 3; ++k) g[k] -= c * dg * Rv[k] / R;
      }
    }
    long long o = (long long)d.atom_off + a;
    for (int k = 0; k < 3; ++k) g_out[3 * o + k] += g[k];
  }
  // the opposite forces on the healed ghosts (one entry per healed shell)
  for (int e = h0 + threadIdx.x; e < h1; e += blockDim.x) {
    const int t = bt.healed_sh[e], G = sys.sh_atom[t];
    const double qt = qmono[t];
    double g[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < nat; ++a) {
      const int A = atoms[a];
      if (sys.frag[A] == sys.frag[G]) continue;
      const DevElem& ea = sys.elems[sys.elem[A]];
      double Rv[3] = {sys.xyz[3 * A] - sys.xyz[3 * G], sys.xyz[3 * A + 1] - sys.xyz[3 * G + 1],
                      sys.xyz[3 * A + 2] - sys.xyz[3 * G + 2]};
      double R = sqrt(Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2]);
      if (R == 0.0) continue;
      for (int sa = 0; sa < ea.nsh; ++sa) {
        const double qs = qmono[sys.atom_sh0[A] + sa];
        const double c = qs * qt + wx * (ddq[d.sh_off + ash[a] + sa] * qt - qs * qt);
        double dg;
        gamma_and_deriv(sys.g, R, ea.eta[sa], sys.sh_eta[t], &dg);
        for (int k = 0; k < 3; ++k) g[k] += c * dg * Rv[k] / R;
      }
    }
    for (int k = 0; k < 3; ++k) ghost_out[3LL * e + k] = g[k];
  }
}

// Explicit derivative of Tr(Dm V^HOP) at fixed Dm for the boundary entries of
// every system of a batch, V^HOP = S D S (eq. vhop), D = V h h^T on a
// detached atom and V (1_sp - h h^T) on a ghost, h = 1/2 s + sqrt(3)/2 b.p:
//  * overlap part (eq. hopsder): Dm S D + D S Dm is added to the system's
//    D_S matrix, which k_grad_contract contracts with the overlap derivative;
//  * hybrid-coefficient part (eq. hopcoder): with db/dR_attached =
//    (1 - b b^T) / |R_attached - R_detached|, the force on the attached atom
//    is +-2 V sqrt(3)/2 (1 - b b^T) w_p / |R| with w = (S Dm S) h on the
//    boundary atom (+ detached atom, - ghost) and the detached atom takes
//    the opposite; both, times the system weight, go to hop_f at slot
//    2 (slot_base + entry) (attached) and the next (detached).
// Dm: the density (explicit terms) or the symmetric Z-vector density (the
// response, eq. hop_resp).  One work-group per system, entries in order.
__global__ void __launch_bounds__(256) k_hop_grad(DevSystem sys, DevBatch bt, const double* Dmp, double* DSp,
                                                  const double* wsys, const int* bonds, double V, long long slot_base,
                                                  double* hop_f) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  const double* Dm = Dmp + d.mat_off;
  const double* S = bt.S + d.mat_off;
  double* DS = DSp + d.mat_off;
  const double cw = wsys ? wsys[si] : 1.0;
  __shared__ double X[MAXN][4];
  __shared__ double Y[MAXN][4];
  __shared__ double red[256][4];
  const double cp = 0.5 * sqrt(3.0);
  for (int e = bt.hop_off[si]; e < bt.hop_off[si + 1]; ++e) {
    const int la = bt.hop_atom[e];
    const int o = bt.sys_atom_ao0[d.atom_off + la];
    const double* bv = bt.hop_b + 3 * e;
    const double h[4] = {0.5, cp * bv[0], cp * bv[1], cp * bv[2]};
    const bool bda = bt.hop_kind[e] == 1;
    double D[4][4];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) D[i][j] = bda ? V * h[i] * h[j] : V * ((i == j ? 1.0 : 0.0) - h[i] * h[j]);
    // X = Dm S[:, boundary AOs], Y = X D
    for (int mu = threadIdx.x; mu < n; mu += blockDim.x) {
      double x[4] = {0.0, 0.0, 0.0, 0.0};
      for (int nu = 0; nu < n; ++nu) {
        const double p = Dm[(long long)mu * n + nu];
        for (int j = 0; j < 4; ++j) x[j] += p * S[(long long)nu * n + o + j];
      }
      for (int j = 0; j < 4; ++j) {
        X[mu][j] = x[j];
        double y = 0.0;
        for (int k = 0; k < 4; ++k) y += x[k] * D[k][j];
        Y[mu][j] = y;
      }
    }
    __syncthreads();
    for (int mu = threadIdx.x; mu < n; mu += blockDim.x)
      for (int j = 0; j < 4; ++j) DS[(long long)mu * n + o + j] += Y[mu][j];
    __syncthreads();
    for (int mu = threadIdx.x; mu < n; mu += blockDim.x)
      for (int j = 0; j < 4; ++j) DS[(long long)(o + j) * n + mu] += Y[mu][j];
    // w_i = sum_mu S[o + i][mu] (X h)[mu]: partial sums per thread, fixed order
    double wpart[4] = {0.0, 0.0, 0.0, 0.0};
    for (int mu = threadIdx.x; mu < n; mu += blockDim.x) {
      const double xh = X[mu][0] * h[0] + X[mu][1] * h[1] + X[mu][2] * h[2] + X[mu][3] * h[3];
      for (int i = 0; i < 4; ++i) wpart[i] += S[(long long)(o + i) * n + mu] * xh;
    }
    for (int i = 0; i < 4; ++i) red[threadIdx.x][i] = wpart[i];
    __syncthreads();
    if (threadIdx.x == 0) {
      double w[4] = {0.0, 0.0, 0.0, 0.0};
      for (int t = 0; t < (int)blockDim.x; ++t)
        for (int i = 0; i < 4; ++i) w[i] += red[t][i];
      const int kb = bt.hop_bond[e];
      const int det = bonds[2 * kb], att = bonds[2 * kb + 1];
      double u[3], L2 = 0.0;
      for (int k = 0; k < 3; ++k) {
        u[k] = sys.xyz[3 * att + k] - sys.xyz[3 * det + k];
        L2 += u[k] * u[k];
      }
      const double L = sqrt(L2);
      const double bw = bv[0] * w[1] + bv[1] * w[2] + bv[2] * w[3];
      const double pre = cw * (bda ? 1.0 : -1.0) * 2.0 * V * cp / L;
      double* f = hop_f + 6 * (slot_base + e);
      for (int k = 0; k < 3; ++k) {
        const double fk = pre * (w[1 + k] - bv[k] * bw);
        f[k] = fk;
        f[3 + k] = -fk;
      }
    }
    __syncthreads();
  }
}

// accumulated charge transfer of the ghosts of bonds healed inside each
// cluster: qbar += -w_X q (eq. ctij_ghost); every ghost shell is healed in
// at most one cluster of a batch
__global__ void k_healed_ct(DevBatch bt, const double* w, const double* qmono, double* qbar) {
  const int si = blockIdx.x;
  const double wx = w ? w[si] : 1.0;
  for (int e = bt.healed_off[si] + threadIdx.x; e < bt.healed_off[si + 1]; e += blockDim.x) {
    const int t = bt.healed_sh[e];
    qbar[t] += -wx * qmono[t];
  }
}

// forces of the extended atoms (real atoms, then one ghost per cut bond) added
// to the real atoms: a ghost sits on its detached atom (fixed order)
__global__ void k_add_ext_forces(int N, int NB, const int* bonds, const double* f_ext, double* grad) {
  const int A = blockIdx.x * blockDim.x + threadIdx.x;
  if (A >= N) return;
  double g[3] = {f_ext[3 * A], f_ext[3 * A + 1], f_ext[3 * A + 2]};
  for (int k = 0; k < NB; ++k)
    if (bonds[2 * k] == A)
      for (int c = 0; c < 3; ++c) g[c] += f_ext[3LL * (N + k) + c];
  for (int c = 0; c < 3; ++c) grad[3 * A + c] += g[c];
}

// dst = w_X src on the shells of every system X of a batch
__global__ void k_scale_cluster(DevBatch bt, const double* w, const double* src, double* dst) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const double wx = w[si];
  for (int s = threadIdx.x; s < d.nsh; s += blockDim.x) dst[d.sh_off + s] = wx * src[d.sh_off + s];
}

// All cross-fragment shell pairs: force on atom A from
//   c_st = q_s (q_t + a_t) + a_s q_t,   s on A, t on B, frag(A) != frag(B)
// split over source chunks (deterministic reduction afterwards).
__global__ void k_force_inter(DevSystem sys, const double* q, const double* av, int nchunk, double* part) {
  int A = blockIdx.x * blockDim.x + threadIdx.x;
  int chunk = blockIdx.y;
  int N = sys.natoms;
  int per = (N + nchunk - 1) / nchunk;
  int b_begin = chunk * per, b_end = min(N, b_begin + per);
  __shared__ double sx[256], sy[256], sz[256], seta[256][MAXSH_EL], sq[256][MAXSH_EL], sa_[256][MAXSH_EL];
  __shared__ double sio[256][MAXSH_EL];  // 1/(2 eta) per source shell (kg = 2)
  __shared__ int sf[256], sn[256];
  double xa = 0, ya = 0, za = 0, ea[MAXSH_EL] = {1.0, 1.0}, qa[MAXSH_EL] = {0, 0}, aa[MAXSH_EL] = {0, 0};
  int fa = -1, na = 0;
  if (A < N) {
    xa = sys.xyz[3 * A];
    ya = sys.xyz[3 * A + 1];
    za = sys.xyz[3 * A + 2];
    fa = sys.frag[A];
    int sh0 = sys.atom_sh0[A];
    na = sys.atom_sh0[A + 1] - sh0;
    for (int k = 0; k < na; ++k) {
      ea[k] = sys.sh_eta[sh0 + k];
      qa[k] = q[sh0 + k];
      aa[k] = av[sh0 + k];
    }
  }
  double f[3] = {0.0, 0.0, 0.0};
  // kg = 2: gamma = (R^2 + c^2)^(-1/2), c = iota_s + iota_t, and
  // dgamma/dR / R = -gamma^3 (no square root or division; an absent second
  // shell has q = a = 0 and adds exactly zero)
  const bool kg2 = sys.g.kg == 2.0;
  double ia[MAXSH_EL] = {0.5, 0.5};
  if (A < N)
    for (int k = 0; k < na; ++k) ia[k] = sys.sh_ieta[sys.atom_sh0[A] + k];
  for (int b0 = b_begin; b0 < b_end; b0 += 256) {
    int b = b0 + threadIdx.x;
    __syncthreads();
    if (b < b_end) {
      sx[threadIdx.x] = sys.xyz[3 * b];
      sy[threadIdx.x] = sys.xyz[3 * b + 1];
      sz[threadIdx.x] = sys.xyz[3 * b + 2];
      sf[threadIdx.x] = sys.frag[b];
      int s0 = sys.atom_sh0[b];
      int nsb = sys.atom_sh0[b + 1] - s0;
      sn[threadIdx.x] = nsb;
      for (int k = 0; k < MAXSH_EL; ++k) {
        seta[threadIdx.x][k] = k < nsb ? sys.sh_eta[s0 + k] : 1.0;
        sio[threadIdx.x][k] = k < nsb ? sys.sh_ieta[s0 + k] : 0.5;
        sq[threadIdx.x][k] = k < nsb ? q[s0 + k] : 0.0;
        sa_[threadIdx.x][k] = k < nsb ? av[s0 + k] : 0.0;
      }
    }
    __syncthreads();
    int nb = min(256, b_end - b0);
    if (A < N && kg2) {
      for (int k = 0; k < nb; ++k) {
        const double dx = xa - sx[k], dy = ya - sy[k], dz = za - sz[k];
        const double R2 = dx * dx + dy * dy + dz * dz;
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < MAXSH_EL; ++u)
#pragma unroll
          for (int v = 0; v < MAXSH_EL; ++v) {
            const double c = ia[u] + sio[k][v];
            const double x = rsqrt_pos(R2 + c * c);
            acc -= (qa[u] * (sq[k][v] + sa_[k][v]) + aa[u] * sq[k][v]) * (x * x * x);
          }
        acc = sf[k] == fa ? 0.0 : acc;  // own fragment: adds exactly +0 (a select, no branch)
        f[0] += acc * dx;
        f[1] += acc * dy;
        f[2] += acc * dz;
      }
    } else if (A < N) {
      for (int k = 0; k < nb; ++k) {
        if (sf[k] == fa) continue;
        double dx = xa - sx[k], dy = ya - sy[k], dz = za - sz[k];
        double R = sqrt(dx * dx + dy * dy + dz * dz);
        if (R == 0.0) continue;  // a ghost on its own detached atom: gamma is flat there
        double acc = 0.0;
        for (int u = 0; u < na; ++u)
          for (int v = 0; v < sn[k]; ++v) {
            double dg;
            gamma_and_deriv(sys.g, R, ea[u], seta[k][v], &dg);
            acc += (qa[u] * (sq[k][v] + sa_[k][v]) + aa[u] * sq[k][v]) * dg;
          }
        acc /= R;
        f[0] += acc * dx;
        f[1] += acc * dy;
        f[2] += acc * dz;
      }
    }
  }
  if (A < N)
    for (int k = 0; k < 3; ++k) part[((long long)chunk * N + A) * 3 + k] = f[k];
}

__global__ void k_force_reduce(int N, int nchunk, const double* part, double* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * N) return;
  double acc = 0.0;
  for (int c = 0; c < nchunk; ++c) acc += part[(long long)c * 3 * N + i];
  out[i] = acc;
}

// CN chain: g_C = sum_{A != C} (F_A + F_C) f'(R_AC) (R_C - R_A) / R_AC
// (partners split into nchunk slices as in k_cn; part[(chunk N + C) 3 + k]
// over the N real atoms, summed by k_force_reduce)
__global__ void k_cn_grad(DevSystem sys, const double* Ftot, int nchunk, double* part) {
  const int C = blockIdx.x * blockDim.x + threadIdx.x;
  const int NR = sys.nreal, N = sys.nreal, chunk = blockIdx.y;
  const int per = (NR + nchunk - 1) / nchunk;
  const int b_begin = chunk * per, b_end = min(NR, b_begin + per);
  __shared__ double sx[256], sy[256], sz[256], sr[256], sF[256];
  double xc = 0, yc = 0, zc = 0, rc = 0, Fc = 0;
  if (C < NR) {
    xc = sys.xyz[3 * C];
    yc = sys.xyz[3 * C + 1];
    zc = sys.xyz[3 * C + 2];
    rc = sys.elems[sys.elem[C]].rcov;
    Fc = Ftot[C];
  }
  double f[3] = {0.0, 0.0, 0.0};
  for (int b0 = b_begin; b0 < b_end; b0 += 256) {
    int b = b0 + threadIdx.x;
    __syncthreads();
    if (b < b_end) {
      sx[threadIdx.x] = sys.xyz[3 * b];
      sy[threadIdx.x] = sys.xyz[3 * b + 1];
      sz[threadIdx.x] = sys.xyz[3 * b + 2];
      sr[threadIdx.x] = sys.elems[sys.elem[b]].rcov;
      sF[threadIdx.x] = Ftot[b];
    }
    __syncthreads();
    int nb = min(256, b_end - b0);
    if (C < NR) {
      for (int k = 0; k < nb; ++k) {
        if (b0 + k == C) continue;
        double dx = xc - sx[k], dy = yc - sy[k], dz = zc - sz[k];
        const double ri = rsqrt(dx * dx + dy * dy + dz * dz);  // 1 / R
        double rcs = rc + sr[k];
        double x = -sys.g.k1 * (sys.g.k2 * rcs * ri - 1.0);
        double fv = 1.0 / (1.0 + exp(x));
        // df/dR / R = -f (1 - f) k1 k2 rcs / R^3
        double w = (sF[k] + Fc) * (-fv * (1.0 - fv) * sys.g.k1 * sys.g.k2 * rcs * (ri * ri * ri));
        f[0] += w * dx;
        f[1] += w * dy;
        f[2] += w * dz;
      }
    }
  }
  if (C < N)
    for (int k = 0; k < 3; ++k) part[((long long)chunk * N + C) * 3 + k] = f[k];
}

// Per-atom gather of the per-system contributions in a fixed order.
// entries: CSR over atoms of (batch id, local atom offset into that batch's arrays)
__global__ void k_gather_atoms(int N, const int* rowptr, const int* ent_batch, const long long* ent_off,
                               const double* const* g_batches, const double* const* F_batches, double* g_tot,
                               double* F_tot, int mode) {
  int A = blockIdx.x * blockDim.x + threadIdx.x;
  if (A >= N) return;
  if (mode == 0) {
    double F = 0.0;
    for (int e = rowptr[A]; e < rowptr[A + 1]; ++e) F += F_batches[ent_batch[e]][ent_off[e]];
    F_tot[A] = F;
  } else {
    double g[3] = {g_tot[3 * A], g_tot[3 * A + 1], g_tot[3 * A + 2]};
    for (int e = rowptr[A]; e < rowptr[A + 1]; ++e) {
      const double* gb = g_batches[ent_batch[e]];
      for (int k = 0; k < 3; ++k) g[k] += gb[3 * ent_off[e] + k];
    }
    for (int k = 0; k < 3; ++k) g_tot[3 * A + k] = g[k];
  }
}

// ---------------------------------------------------------------------------
// small per-system helpers

// final shell shift sigma = gamma q_out - Gamma q_A^2 + phi (into sig) and the
// weights n_i eps_i for the energy-weighted density (into wvec)
__global__ void k_final_shift(DevSystem sys, DevBatch bt, double* wvec) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  __shared__ double qa[MAXN];
  const double* q = bt.q_out + d.sh_off;
  for (int a = threadIdx.x; a < d.nat; a += blockDim.x) {
    int s0 = bt.sys_atom_sh0[d.atom_off + a];
    int A = bt.sys_atoms[d.atom_off + a];
    int nsa = sys.atom_sh0[A + 1] - sys.atom_sh0[A];
    double v = 0.0;
    for (int k = 0; k < nsa; ++k) v += q[s0 + k];
    qa[a] = v;
  }
  __syncthreads();
  const double* G = bt.gam + d.gam_off;
  for (int s = threadIdx.x; s < d.nsh; s += blockDim.x) {
    double v = 0.0;
    for (int t = 0; t < d.nsh; ++t) v += G[(long long)s * d.nsh + t] * q[t];
    int a = bt.sys_sh_atom[d.sh_off + s];
    int A = bt.sys_atoms[d.atom_off + a];
    v += -sys.elems[sys.elem[A]].Gamma * qa[a] * qa[a] + bt.phi[d.sh_off + s];
    bt.sig[d.sh_off + s] = v;
  }
  for (int i = threadIdx.x; i < d.nao; i += blockDim.x) wvec[d.ao_off + i] = bt.occ[d.ao_off + i] * bt.eps[d.ao_off + i];
}

// D_S = 1/2 (sigma_mu + sigma_nu) P - W  (eq. W_matrix with the embedding in sigma)
__global__ void k_make_DS(DevBatch bt, const double* P, const double* W, double* out) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  const int* aosh = bt.sys_ao_sh + d.ao_off;
  const double* sg = bt.sig + d.sh_off;
  for (long long idx = threadIdx.x; idx < (long long)n * n; idx += blockDim.x) {
    int i = (int)(idx / n), j = (int)(idx % n);
    out[d.mat_off + idx] = 0.5 * (sg[aosh[i]] + sg[aosh[j]]) * P[d.mat_off + idx] - W[d.mat_off + idx];
  }
}

}  // namespace fx
