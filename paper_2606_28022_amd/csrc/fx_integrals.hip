// Supersystem coordination numbers, pair classification, and the per-system
// S / H0 / gamma / repulsion build.
//
// Formulas (section "GFN1-xTB"): CN of eq. cn_def without cutoff; H0 of
// eq. h0_hamiltonian with the polynomial Pi of eq.
// xtb1_polynomial_correction and the CN-dependent levels of eq.
// xtb1_diagonal_h0; gamma = (R^kg + eta^-kg)^(-1/kg) with eta the harmonic
// mean of the shell hardnesses; repulsion of eq. gfn1_rep_energy over the
// unordered atom pairs of the system.  Overlaps of the STO-6G contracted
// Cartesian s/p shells use the Gaussian product theorem; a second s shell on
// an atom is orthogonalised against the first.
#include <hip/hip_runtime.h>

#include "fx_device.hpp"
#include "fx_kernels.hpp"

namespace fx {

__device__ inline double gamma_fn(const DevGlobals& g, double R2, double eta_s, double eta_t) {
  double inv_eta = 0.5 * (1.0 / eta_s + 1.0 / eta_t);   // 1 / harmonic-mean hardness
  if (g.kg == 2.0) return 1.0 / sqrt(R2 + inv_eta * inv_eta);
  double R = sqrt(R2);
  return pow(pow(R, g.kg) + pow(inv_eta, g.kg), -1.0 / g.kg);
}

// ---------------------------------------------------------------------------
// coordination numbers: one thread per atom, all partners (no cutoff); the
// partners are split into nchunk slices over the second grid dimension
// (enough work-groups to fill the chip), whose partial sums k_field_reduce
// adds in fixed order
__global__ void k_cn(DevSystem sys, int nchunk, double* part) {
  const int A = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = sys.nreal, chunk = blockIdx.y;
  const int per = (N + nchunk - 1) / nchunk;
  const int b_begin = chunk * per, b_end = min(N, b_begin + per);
  __shared__ double sx[256], sy[256], sz[256], sr[256];
  double xa = 0, ya = 0, za = 0, ra = 0;
  if (A < N) {
    xa = sys.xyz[3 * A];
    ya = sys.xyz[3 * A + 1];
    za = sys.xyz[3 * A + 2];
    ra = sys.elems[sys.elem[A]].rcov;
  }
  double acc = 0.0;
  for (int b0 = b_begin; b0 < b_end; b0 += 256) {
    int b = b0 + threadIdx.x;
    __syncthreads();
    if (b < b_end) {
      sx[threadIdx.x] = sys.xyz[3 * b];
      sy[threadIdx.x] = sys.xyz[3 * b + 1];
      sz[threadIdx.x] = sys.xyz[3 * b + 2];
      sr[threadIdx.x] = sys.elems[sys.elem[b]].rcov;
    }
    __syncthreads();
    int nb = min(256, b_end - b0);
    if (A < N) {
      for (int k = 0; k < nb; ++k) {
        if (b0 + k == A) continue;
        double dx = xa - sx[k], dy = ya - sy[k], dz = za - sz[k];
        double x = -sys.g.k1 * (sys.g.k2 * (ra + sr[k]) * rsqrt(dx * dx + dy * dy + dz * dz) - 1.0);
        acc += 1.0 / (1.0 + exp(x));
      }
    }
  }
  if (A < N) part[(long long)chunk * N + A] = acc;
}

// ---------------------------------------------------------------------------
// Fragment-pair selection (section "Computational Details"), one flag per
// pair I < J: bit 0 = SCC dimer, bit 1 = the pair counts towards the trimer
// rule (at least two of a trimer's three pairs).
//   rule 0: closest contact d2 < cut2 (both bits);
//   rule 1: some atom pair a, b with d2 < (lam (r_a + r_b))^2, van der Waals
//           radii r; bit 0 with lam = lam2, bit 1 with lam = lam3.
// d2 = (dx*dx + dy*dy) + dz*dz and the threshold lam * (r_a + r_b), squared,
// with every operation rounded separately (no contraction).
__global__ void k_pair_contacts(DevSystem sys, const int* frag_atoms, const int* frag_off, int rule, double cut2,
                                double lam2, double lam3, int8_t* flag) {
#pragma clang fp contract(off)
  int I = blockIdx.x;
  int F = sys.nfrag;
  int a0 = frag_off[I], a1 = frag_off[I + 1];
  long long base = (long long)I * F - (long long)I * (I + 1) / 2;  // index of (I, I+1)
  for (int J = I + 1 + threadIdx.x; J < F; J += blockDim.x) {
    int b0 = frag_off[J], b1 = frag_off[J + 1];
    double best = 1e300;
    int bits = 0;
    for (int ia = a0; ia < a1; ++ia) {
      int a = frag_atoms[ia];
      double xa = sys.xyz[3 * a], ya = sys.xyz[3 * a + 1], za = sys.xyz[3 * a + 2];
      const double ra = sys.elems[sys.elem[a]].rvdw;
      for (int ib = b0; ib < b1; ++ib) {
        int b = frag_atoms[ib];
        double dx = xa - sys.xyz[3 * b];
        double dy = ya - sys.xyz[3 * b + 1];
        double dz = za - sys.xyz[3 * b + 2];
        double xx = __dmul_rn(dx, dx);
        double yy = __dmul_rn(dy, dy);
        double zz = __dmul_rn(dz, dz);
        double d2 = __dadd_rn(__dadd_rn(xx, yy), zz);
        if (rule == 0) {
          best = d2 < best ? d2 : best;
        } else {
          const double rs = __dadd_rn(ra, sys.elems[sys.elem[b]].rvdw);
          const double t2 = __dmul_rn(lam2, rs), t3 = __dmul_rn(lam3, rs);
          if (d2 < __dmul_rn(t2, t2)) bits |= 1;
          if (d2 < __dmul_rn(t3, t3)) bits |= 2;
        }
      }
    }
    if (rule == 0) bits = best < cut2 ? 3 : 0;
    flag[base + (J - I - 1)] = (int8_t)bits;
  }
}

// ---------------------------------------------------------------------------
// overlap block between two atoms (raw contracted shells, then the on-site
// orthogonalisation), R = A - B.  out is nao_a x nao_b, row-major, ld = 4.
// Every primitive term of a shell pair is s00 times a polynomial in R whose
// coefficients depend on the primitive pair only through fa = -b / (a + b),
// fb = a / (a + b) and h = 1 / (2 (a + b)): s s sum s00; p s R_u sum(fa s00);
// s p R_v sum(fb s00); p p R_u R_v sum(fa fb s00) + delta_uv sum(h s00).  So
// the primitive loop accumulates at most two scalars per shell pair.
__device__ void atom_pair_overlap(const DevElem& ea, const DevElem& eb, double Rx, double Ry,
                                  double Rz, double out[MAXAO_EL][MAXAO_EL]) {
  const double PI = 3.14159265358979323846;
  double R2 = Rx * Rx + Ry * Ry + Rz * Rz;
  double Rv[3] = {Rx, Ry, Rz};
  for (int i = 0; i < MAXAO_EL; ++i)
    for (int j = 0; j < MAXAO_EL; ++j) out[i][j] = 0.0;
  // shell 0 is an s shell at AO 0, shell 1 (if any) starts at AO 1 (checked
  // when the parameters are loaded): compile-time block indices, so the
  // block stays in registers
#pragma unroll
  for (int sa = 0; sa < MAXSH_EL; ++sa) {
#pragma unroll
    for (int sb = 0; sb < MAXSH_EL; ++sb) {
      if (sa >= ea.nsh || sb >= eb.nsh) continue;
      const int kind = 2 * ea.l[sa] + eb.l[sb];  // 0 s s, 1 s p, 2 p s, 3 p p
      double t0 = 0.0, t2 = 0.0;
#pragma unroll 1
      for (int i = 0; i < NPRIM; ++i) {
        const double a = ea.alpha[sa][i];
        for (int j = 0; j < NPRIM; ++j) {
          const double b = eb.alpha[sb][j];
          const double ip = 1.0 / (a + b);
          const double mu = a * b * ip;
          const double s00 = ea.coef[sa][i] * eb.coef[sb][j] * PI * ip * sqrt(PI * ip) * exp(-mu * R2);
          if (kind == 0) {
            t0 += s00;
          } else if (kind == 2) {
            t0 += -b * ip * s00;
          } else if (kind == 1) {
            t0 += a * ip * s00;
          } else {
            t0 += (-b * ip) * (a * ip) * s00;
            t2 += 0.5 * ip * s00;
          }
        }
      }
      const int oa = sa, ob = sb;
      if (kind == 0) {
        out[oa][ob] = t0;
      } else if (kind == 2) {
        for (int k = 0; k < 3; ++k) out[oa + k][ob] = Rv[k] * t0;
      } else if (kind == 1) {
        for (int k = 0; k < 3; ++k) out[oa][ob + k] = Rv[k] * t0;
      } else {
        for (int u = 0; u < 3; ++u)
          for (int v = 0; v < 3; ++v) out[oa + u][ob + v] = Rv[u] * Rv[v] * t0 + (u == v ? t2 : 0.0);
      }
    }
  }
  if (ea.orth) {  // rows: second s shell of A (AO 1) against the first (AO 0)
#pragma unroll
    for (int j = 0; j < MAXAO_EL; ++j) out[1][j] = ea.orthN * (out[1][j] - ea.orthS12 * out[0][j]);
  }
  if (eb.orth) {
#pragma unroll
    for (int i = 0; i < MAXAO_EL; ++i) out[i][1] = eb.orthN * (out[i][1] - eb.orthS12 * out[i][0]);
  }
}

// H0 prefactor of a shell pair on different atoms (everything but S).
__device__ inline double h0_prefactor(const DevGlobals& g, const DevElem& ea, int sa, double cna,
                                      const DevElem& eb, int sb, double cnb, double R) {
  double kll = 0.5 * (g.kl[ea.l[sa]] + g.kl[eb.l[sb]]);
  double den = ea.EN - eb.EN;
  double ha = ea.level[sa] * (1.0 + ea.kcn[sa] * cna);
  double hb = eb.level[sb] * (1.0 + eb.kcn[sb] * cnb);
  double x = sqrt(R / (ea.rcov + eb.rcov));
  double Pi = (1.0 + ea.kpoly[sa] * x) * (1.0 + eb.kpoly[sb] * x);
  return g.KAB * kll * 0.5 * (ha + hb) * (1.0 + g.kEN * den * den) * Pi;
}

// S and H0 blocks of the atom pair (a, b), a != b, written in both
// triangles; returns the pair's repulsion energy
__device__ inline double pair_block(const DevSystem& sys, const DevBatch& bt, const SysDesc& d, int n,
                                    const int* atoms, const int* aao, int a, int b, double* S, double* H) {
  const int A = atoms[a], B = atoms[b];
  const DevElem& ea = sys.elems[sys.elem[A]];
  const DevElem& eb = sys.elems[sys.elem[B]];
  const double Rx = sys.xyz[3 * A] - sys.xyz[3 * B];
  const double Ry = sys.xyz[3 * A + 1] - sys.xyz[3 * B + 1];
  const double Rz = sys.xyz[3 * A + 2] - sys.xyz[3 * B + 2];
  const double R = sqrt(Rx * Rx + Ry * Ry + Rz * Rz);
  double blk[MAXAO_EL][MAXAO_EL];
  atom_pair_overlap(ea, eb, Rx, Ry, Rz, blk);
  const int oa = aao[a], ob = aao[b];
  double f[MAXSH_EL][MAXSH_EL];
#pragma unroll
  for (int sa = 0; sa < MAXSH_EL; ++sa)
#pragma unroll
    for (int sb = 0; sb < MAXSH_EL; ++sb)
      f[sa][sb] =
          (sa < ea.nsh && sb < eb.nsh) ? h0_prefactor(sys.g, ea, sa, sys.cn[A], eb, sb, sys.cn[B], R) : 0.0;
#pragma unroll
  for (int i = 0; i < MAXAO_EL; ++i)
#pragma unroll
    for (int j = 0; j < MAXAO_EL; ++j) {
      if (i >= ea.nao || j >= eb.nao) continue;
      const double sv = blk[i][j];
      const double hv = f[i == 0 ? 0 : 1][j == 0 ? 0 : 1] * sv;
      S[(long long)(oa + i) * n + ob + j] = sv;
      S[(long long)(ob + j) * n + oa + i] = sv;
      H[(long long)(oa + i) * n + ob + j] = hv;
      H[(long long)(ob + j) * n + oa + i] = hv;
    }
  const double al = sqrt(ea.arep * eb.arep);
  const double zs = bt.atom_zs ? bt.atom_zs[d.atom_off + a] * bt.atom_zs[d.atom_off + b] : 1.0;
  return zs * ea.zeff * eb.zeff / R * exp(-al * pow(R, sys.g.kf));
}

// ---------------------------------------------------------------------------
// per-system S, H0, gamma and repulsion; one work-group per system.
// from_mono (clusters of fragments without cut bonds, whose components are
// their monomers' atoms in the monomers' order): every block within one
// component equals the monomer's (the same atom pairs, CN and shells), so it
// is copied from the monomer batch, and only the pairs between components
// are evaluated; the repulsion adds the monomers' own.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
    k_build_system(DevSystem sys, DevBatch bt, const int* list, DevBatch mono, int from_mono) {
  int si = list ? list[blockIdx.x] : blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  double* S = bt.S + d.mat_off;
  double* H = bt.H0 + d.mat_off;
  const int* atoms = bt.sys_atoms + d.atom_off;
  const int* aao = bt.sys_atom_ao0 + d.atom_off;
  __shared__ double red[256];
  double erep = 0.0;
  const int nc = d.nfrag;
  const bool copy = from_mono && nc > 1;
  // component c: atoms ca[c] .., AOs co[c] .., shells csh[c] ..; the atom
  // pairs between components as rectangles (rc1, rc2), c1 < c2, at pair
  // offsets roff
  __shared__ int ca[4], co[4], roff[4], rc1[3], rc2[3], nrect, cfrag[3], csh[4];
  if (copy) {
    if (threadIdx.x == 0) {
      ca[0] = co[0] = 0;
      const SysDesc* dp = bt.desc + si;  // (indexed in memory, not copied)
      for (int c = 0; c < nc; ++c) {
        cfrag[c] = dp->frag[c];
        csh[c] = dp->comp_sh[c];
        ca[c + 1] = ca[c] + mono.desc[cfrag[c]].nat;
        co[c + 1] = co[c] + mono.desc[cfrag[c]].nao;
      }
      csh[nc] = dp->comp_sh[nc];
      int nr = 0;
      roff[0] = 0;
      for (int c1 = 0; c1 < nc; ++c1)
        for (int c2 = c1 + 1; c2 < nc; ++c2) {
          rc1[nr] = c1;
          rc2[nr] = c2;
          roff[nr + 1] = roff[nr] + (ca[c1 + 1] - ca[c1]) * (ca[c2 + 1] - ca[c2]);
          ++nr;
        }
      nrect = nr;
    }
    __syncthreads();
    for (int c = 0; c < nc; ++c) {
      const SysDesc* md = mono.desc + cfrag[c];
      const int m = md->nao, msh = md->nsh;
      const double* mS = mono.S + md->mat_off;
      const double* mH = mono.H0 + md->mat_off;
      for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        const int i = e / m, j = e - i * m;
        const long long o = (long long)(co[c] + i) * n + co[c] + j;
        S[o] = mS[e];
        H[o] = mH[e];
      }
      const double* mG = mono.gam + md->gam_off;
      double* G = bt.gam + d.gam_off;
      const int s0 = csh[c];
      for (int e = threadIdx.x; e < msh * msh; e += blockDim.x) {
        const int i = e / msh, j = e - i * msh;
        G[(long long)(s0 + i) * d.nsh + s0 + j] = mG[e];
      }
    }
  } else {
    // diagonal atom blocks
    for (int a = threadIdx.x; a < d.nat; a += blockDim.x) {
      int A = atoms[a];
      const DevElem& e = sys.elems[sys.elem[A]];
      int o = aao[a];
      for (int i = 0; i < e.nao; ++i)
        for (int j = 0; j < e.nao; ++j) {
          S[(long long)(o + i) * n + o + j] = (i == j) ? 1.0 : 0.0;
          H[(long long)(o + i) * n + o + j] = 0.0;
        }
      for (int s = 0; s < e.nsh; ++s) {
        double h = e.level[s] * (1.0 + e.kcn[s] * sys.cn[A]);
        for (int k = 0; k < e.nao_sh[s]; ++k) H[(long long)(o + e.ao0[s] + k) * n + o + e.ao0[s] + k] = h;
      }
    }
  }
  // off-diagonal atom blocks: the unordered pairs a < b, row a holding
  // pairs off(a) = a nat - a (a + 1) / 2 .. off(a + 1) - 1; with copied
  // components, the pairs between components only
  const int nat = d.nat, np = copy ? roff[nrect] : nat * (nat - 1) / 2;
  for (int idx = threadIdx.x; idx < np; idx += blockDim.x) {
    int a, b;
    if (copy) {
      int k = 0;
      while (idx >= roff[k + 1]) ++k;
      const int w = ca[rc2[k] + 1] - ca[rc2[k]], loc = idx - roff[k];
      a = ca[rc1[k]] + loc / w;
      b = ca[rc2[k]] + loc % w;
    } else {
      const double c = 2.0 * nat - 1.0;
      a = (int)floor(0.5 * (c - sqrt(c * c - 8.0 * idx)));
      a = max(0, min(a, nat - 2));
      while (a > 0 && a * nat - a * (a + 1) / 2 > idx) --a;
      while ((a + 1) * nat - (a + 1) * (a + 2) / 2 <= idx) ++a;
      b = idx - (a * nat - a * (a + 1) / 2) + a + 1;
    }
    erep += pair_block(sys, bt, d, n, atoms, aao, a, b, S, H);
  }
  // gamma of the system's shells (with copied components: between them)
  double* G = bt.gam + d.gam_off;
  const int* shg = bt.sys_sh_global + d.sh_off;
  for (int idx = threadIdx.x; idx < d.nsh * d.nsh; idx += blockDim.x) {
    int s = idx / d.nsh, t = idx - s * d.nsh;
    if (copy) {
      int cs = 0, ct = 0;
      for (int c = 1; c < nc; ++c) {
        cs += s >= csh[c];
        ct += t >= csh[c];
      }
      if (cs == ct) continue;
    }
    int gs = shg[s], gt = shg[t];
    int As = sys.sh_atom[gs], At = sys.sh_atom[gt];
    double dx = sys.xyz[3 * As] - sys.xyz[3 * At];
    double dy = sys.xyz[3 * As + 1] - sys.xyz[3 * At + 1];
    double dz = sys.xyz[3 * As + 2] - sys.xyz[3 * At + 2];
    G[idx] = gamma_fn(sys.g, dx * dx + dy * dy + dz * dz, sys.sh_eta[gs], sys.sh_eta[gt]);
  }
  // deterministic reduction of the repulsion energy (plus the copied
  // components' own)
  red[threadIdx.x] = erep;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double e = red[0];
    if (copy)
      for (int c = 0; c < nc; ++c) e += mono.erep[cfrag[c]];
    bt.erep[si] = e;
  }
}

// ---------------------------------------------------------------------------
// Embedding field: phi_s = sum_{t in other fragments} gamma_st q_t.
// One thread per target atom (all its shells); the source atoms are split
// into `nchunk` slices handled by separate work-groups, whose partial sums
// are combined in fixed order by k_field_reduce (deterministic).
// CN of each ghost atom: that of the detached atom it copies
__global__ void k_ghost_cn(DevSystem sys, const int* bonds, int nbonds, double* cn) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nbonds) cn[sys.nreal + k] = cn[bonds[2 * k]];
}

__global__ void __launch_bounds__(256) k_field_partial(DevSystem sys, const double* q, int nchunk, double* part) {
  const int A = blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y;
  const int N = sys.natoms;
  const int per = (N + nchunk - 1) / nchunk;
  const int b_begin = chunk * per, b_end = min(N, b_begin + per);
  // source tile: position, fragment and up to two shells per atom (an absent
  // second shell carries q = 0, so it adds exactly zero)
  __shared__ double sx[256], sy[256], sz[256], si0[256], si1[256], sq0[256], sq1[256];
  __shared__ int sf[256];
  const bool kg2 = sys.g.kg == 2.0;
  double xa = 0, ya = 0, za = 0, ia0 = 0.5, ia1 = 0.5, ea[MAXSH_EL] = {1.0, 1.0};
  int fa = -1, na = 0, sh0 = 0;
  if (A < N) {
    xa = sys.xyz[3 * A];
    ya = sys.xyz[3 * A + 1];
    za = sys.xyz[3 * A + 2];
    fa = sys.frag[A];
    sh0 = sys.atom_sh0[A];
    na = sys.atom_sh0[A + 1] - sh0;
    for (int k = 0; k < na; ++k) ea[k] = sys.sh_eta[sh0 + k];
    ia0 = sys.sh_ieta[sh0];
    ia1 = na > 1 ? sys.sh_ieta[sh0 + 1] : 0.5;
  }
  double acc0 = 0.0, acc1 = 0.0;
  for (int b0 = b_begin; b0 < b_end; b0 += 256) {
    const int b = b0 + threadIdx.x;
    __syncthreads();
    if (b < b_end) {
      sx[threadIdx.x] = sys.xyz[3 * b];
      sy[threadIdx.x] = sys.xyz[3 * b + 1];
      sz[threadIdx.x] = sys.xyz[3 * b + 2];
      sf[threadIdx.x] = sys.frag[b];
      const int s0 = sys.atom_sh0[b];
      const int nsb = sys.atom_sh0[b + 1] - s0;
      si0[threadIdx.x] = sys.sh_ieta[s0];
      sq0[threadIdx.x] = q[s0];
      si1[threadIdx.x] = nsb > 1 ? sys.sh_ieta[s0 + 1] : 0.5;
      sq1[threadIdx.x] = nsb > 1 ? q[s0 + 1] : 0.0;
    }
    __syncthreads();
    const int nb = min(256, b_end - b0);
    if (A < N && kg2) {
      // gamma = (R^2 + (1/eta_st)^2)^(-1/2); a source in the target's own
      // fragment adds exactly +0 (a select, no branch per source)
#pragma unroll 2
      for (int k = 0; k < nb; ++k) {
        const double dx = xa - sx[k], dy = ya - sy[k], dz = za - sz[k];
        const double R2 = dx * dx + dy * dy + dz * dz;
        const double t00 = ia0 + si0[k], t01 = ia0 + si1[k], t10 = ia1 + si0[k], t11 = ia1 + si1[k];
        const double q0 = sq0[k], q1 = sq1[k];
        const double g0 = rsqrt_pos(R2 + t00 * t00) * q0 + rsqrt_pos(R2 + t01 * t01) * q1;
        const double g1 = rsqrt_pos(R2 + t10 * t10) * q0 + rsqrt_pos(R2 + t11 * t11) * q1;
        const bool own = sf[k] == fa;
        acc0 += own ? 0.0 : g0;
        acc1 += own ? 0.0 : g1;
      }
    } else if (A < N) {
      for (int k = 0; k < nb; ++k) {
        if (sf[k] == fa) continue;
        const double dx = xa - sx[k], dy = ya - sy[k], dz = za - sz[k];
        const double R2 = dx * dx + dy * dy + dz * dz;
        const double e0 = 0.5 / si0[k], e1 = 0.5 / si1[k];
        acc0 += gamma_fn(sys.g, R2, ea[0], e0) * sq0[k] + gamma_fn(sys.g, R2, ea[0], e1) * sq1[k];
        acc1 += gamma_fn(sys.g, R2, ea[1], e0) * sq0[k] + gamma_fn(sys.g, R2, ea[1], e1) * sq1[k];
      }
    }
  }
  if (A < N) {
    part[(long long)chunk * sys.nshells + sh0] = acc0;
    if (na > 1) part[(long long)chunk * sys.nshells + sh0 + 1] = acc1;
  }
}

// Mixed-precision form of the field pass (early monomer steps only): FP32
// positions relative to the target, FP32 rsqrt and FP32 sums within a source
// chunk; the chunk partials are added in FP64 by k_field_reduce.
__global__ void __launch_bounds__(256) k_field_partial_f32(DevSystem sys, const double* q, int nchunk, double* part) {
  const int A = blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y;
  const int N = sys.natoms;
  const int per = (N + nchunk - 1) / nchunk;
  const int b_begin = chunk * per, b_end = min(N, b_begin + per);
  __shared__ double sx[256], sy[256], sz[256];
  __shared__ float si0[256], si1[256], sq0[256], sq1[256];
  __shared__ int sf[256];
  double xa = 0, ya = 0, za = 0;
  float ia0 = 0.5f, ia1 = 0.5f;
  int fa = -1, na = 0, sh0 = 0;
  if (A < N) {
    xa = sys.xyz[3 * A];
    ya = sys.xyz[3 * A + 1];
    za = sys.xyz[3 * A + 2];
    fa = sys.frag[A];
    sh0 = sys.atom_sh0[A];
    na = sys.atom_sh0[A + 1] - sh0;
    ia0 = (float)sys.sh_ieta[sh0];
    ia1 = na > 1 ? (float)sys.sh_ieta[sh0 + 1] : 0.5f;
  }
  float acc0 = 0.0f, acc1 = 0.0f;
  for (int b0 = b_begin; b0 < b_end; b0 += 256) {
    const int b = b0 + threadIdx.x;
    __syncthreads();
    if (b < b_end) {
      sx[threadIdx.x] = sys.xyz[3 * b];
      sy[threadIdx.x] = sys.xyz[3 * b + 1];
      sz[threadIdx.x] = sys.xyz[3 * b + 2];
      sf[threadIdx.x] = sys.frag[b];
      const int s0 = sys.atom_sh0[b];
      const int nsb = sys.atom_sh0[b + 1] - s0;
      si0[threadIdx.x] = (float)sys.sh_ieta[s0];
      sq0[threadIdx.x] = (float)q[s0];
      si1[threadIdx.x] = nsb > 1 ? (float)sys.sh_ieta[s0 + 1] : 0.5f;
      sq1[threadIdx.x] = nsb > 1 ? (float)q[s0 + 1] : 0.0f;
    }
    __syncthreads();
    const int nb = min(256, b_end - b0);
    if (A < N)
#pragma unroll 2
      for (int k = 0; k < nb; ++k) {
        const float dx = (float)(xa - sx[k]), dy = (float)(ya - sy[k]), dz = (float)(za - sz[k]);
        const float R2 = dx * dx + dy * dy + dz * dz;
        const float t00 = ia0 + si0[k], t01 = ia0 + si1[k], t10 = ia1 + si0[k], t11 = ia1 + si1[k];
        const float g0 = rsqrtf(R2 + t00 * t00) * sq0[k] + rsqrtf(R2 + t01 * t01) * sq1[k];
        const float g1 = rsqrtf(R2 + t10 * t10) * sq0[k] + rsqrtf(R2 + t11 * t11) * sq1[k];
        const bool own = sf[k] == fa;  // own fragment: adds exactly +0
        acc0 += own ? 0.0f : g0;
        acc1 += own ? 0.0f : g1;
      }
  }
  if (A < N) {
    part[(long long)chunk * sys.nshells + sh0] = acc0;
    if (na > 1) part[(long long)chunk * sys.nshells + sh0 + 1] = acc1;
  }
}

// Symmetric form of the FP64 field pass for kg = 2 (gamma_st = gamma_ts):
// every inter-fragment atom pair is evaluated once and used in both
// directions.  Atoms form blocks of 64; one wave (the whole work-group) takes
// a target block I and source blocks J = I + g G .. I + g G + G - 1 (J >= I).
// Lane i holds target atom 64 I + i; in step r it meets source atom
// k = (i + r) mod 64 of block J, adds gamma q_k to its own row sums and
// gamma q_i to the column sums of atom k, which move one lane down after each
// step (DPP rotation), so that after 64 steps lane k holds the column sums of
// its own source atom.  The diagonal block (J = I) is taken in one direction
// only (r = 1 .. 63, row sums).  Row sums go to rowpart[(I, g)], column sums
// to colpart[(I, J)] (I < J); k_field_sym_reduce adds them in fixed order.
__device__ inline double wave_rol1(double v) {
  // lane i reads lane i + 1 (lane 63 reads lane 0)
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x134, 0xf, 0xf, true),
                          __builtin_amdgcn_mov_dpp(lo, 0x134, 0xf, 0xf, true));
}

// One off-diagonal block pair (64 steps); OWN: some target and source atom
// may share a fragment (such pairs add exactly +0)
template <bool OWN>
__device__ inline void field_block_pair(const double4* sa, const double4* sb, int lane, double xa, double ya, double za,
                                        double ia0, double ia1, double qa0, double qa1, double fa, double& r0,
                                        double& r1, double& c0, double& c1) {
  for (int r = 0; r < 64; ++r) {
    const int k = (lane + r) & 63;
    const double4 a = sa[k], b = sb[k];
    const double dx = xa - a.x, dy = ya - a.y, dz = za - a.z;
    const double R2 = dx * dx + dy * dy + dz * dz;
    const double t00 = ia0 + a.w, t01 = ia0 + b.x, t10 = ia1 + a.w, t11 = ia1 + b.x;
    const double x00 = rsqrt_pos(R2 + t00 * t00), x01 = rsqrt_pos(R2 + t01 * t01);
    const double x10 = rsqrt_pos(R2 + t10 * t10), x11 = rsqrt_pos(R2 + t11 * t11);
    const double g0 = x00 * b.y + x01 * b.z, g1 = x10 * b.y + x11 * b.z;
    const double h0 = x00 * qa0 + x10 * qa1, h1 = x01 * qa0 + x11 * qa1;
    if (OWN) {
      const bool own = b.w == fa;
      r0 += own ? 0.0 : g0;
      r1 += own ? 0.0 : g1;
      c0 = wave_rol1(c0 + (own ? 0.0 : h0));
      c1 = wave_rol1(c1 + (own ? 0.0 : h1));
    } else {
      r0 += g0;
      r1 += g1;
      c0 = wave_rol1(c0 + h0);
      c1 = wave_rol1(c1 + h1);
    }
  }
}

__global__ void __launch_bounds__(64) k_field_sym(DevSystem sys, const double* q, int group, int ngmax,
                                                  double* rowpart, double* colpart) {
  const int N = sys.natoms;
  const int nb = (N + 63) / 64;
  const int I = blockIdx.x, g = blockIdx.y;
  const int J0 = I + g * group;
  if (J0 >= nb) return;
  const int J1 = min(nb, J0 + group);
  const int lane = threadIdx.x;
  // source block: position and ieta0 | ieta1, q0, q1, fragment
  __shared__ double4 sa[64], sb[64];
  // target atom of this lane (an absent atom or second shell carries q = 0)
  double xa = 0.0, ya = 0.0, za = 0.0, ia0 = 0.5, ia1 = 0.5, qa0 = 0.0, qa1 = 0.0, fa = -1.0;
  {
    const int A = 64 * I + lane;
    if (A < N) {
      xa = sys.xyz[3 * A];
      ya = sys.xyz[3 * A + 1];
      za = sys.xyz[3 * A + 2];
      fa = (double)sys.frag[A];
      const int s0 = sys.atom_sh0[A], ns = sys.atom_sh0[A + 1] - s0;
      ia0 = sys.sh_ieta[s0];
      qa0 = q[s0];
      if (ns > 1) {
        ia1 = sys.sh_ieta[s0 + 1];
        qa1 = q[s0 + 1];
      }
    }
  }
  // fragments of the target block (absent atoms excluded)
  const int fmin_t = wave_min_i32(fa >= 0.0 ? (int)fa : 0x7fffffff);
  const int fmax_t = wave_max_i32(fa >= 0.0 ? (int)fa : -1);
  double r0 = 0.0, r1 = 0.0;
  for (int J = J0; J < J1; ++J) {
    __syncthreads();
    int fmin_s, fmax_s;
    {
      const int B = 64 * J + lane;
      double4 a = make_double4(0.0, 0.0, 0.0, 0.5), b = make_double4(0.5, 0.0, 0.0, -2.0);
      if (B < N) {
        a.x = sys.xyz[3 * B];
        a.y = sys.xyz[3 * B + 1];
        a.z = sys.xyz[3 * B + 2];
        const int s0 = sys.atom_sh0[B], ns = sys.atom_sh0[B + 1] - s0;
        a.w = sys.sh_ieta[s0];
        b.y = q[s0];
        if (ns > 1) {
          b.x = sys.sh_ieta[s0 + 1];
          b.z = q[s0 + 1];
        }
        b.w = (double)sys.frag[B];
      }
      sa[lane] = a;
      sb[lane] = b;
      fmin_s = wave_min_i32(b.w >= 0.0 ? (int)b.w : 0x7fffffff);
      fmax_s = wave_max_i32(b.w >= 0.0 ? (int)b.w : -1);
    }
    __syncthreads();
    if (J == I) {
      for (int r = 1; r < 64; ++r) {
        const int k = (lane + r) & 63;
        const double4 a = sa[k], b = sb[k];
        const double dx = xa - a.x, dy = ya - a.y, dz = za - a.z;
        const double R2 = dx * dx + dy * dy + dz * dz;
        const double t00 = ia0 + a.w, t01 = ia0 + b.x, t10 = ia1 + a.w, t11 = ia1 + b.x;
        const double g0 = rsqrt_pos(R2 + t00 * t00) * b.y + rsqrt_pos(R2 + t01 * t01) * b.z;
        const double g1 = rsqrt_pos(R2 + t10 * t10) * b.y + rsqrt_pos(R2 + t11 * t11) * b.z;
        const bool own = b.w == fa;  // own fragment: adds exactly +0
        r0 += own ? 0.0 : g0;
        r1 += own ? 0.0 : g1;
      }
    } else {
      double c0 = 0.0, c1 = 0.0;  // column sums of source atom (lane + r) mod 64
      // blocks whose fragment ranges are disjoint share no fragment: no test
      if (fmax_t < fmin_s || fmax_s < fmin_t)
        field_block_pair<false>(sa, sb, lane, xa, ya, za, ia0, ia1, qa0, qa1, fa, r0, r1, c0, c1);
      else
        field_block_pair<true>(sa, sb, lane, xa, ya, za, ia0, ia1, qa0, qa1, fa, r0, r1, c0, c1);
      // lane holds the column sums of its own source atom 64 J + lane
      double* cp = colpart + ((long long)J * (J - 1) / 2 + I) * 128;
      cp[2 * lane] = c0;
      cp[2 * lane + 1] = c1;
    }
  }
  double* rp = rowpart + ((long long)I * ngmax + g) * 128;
  rp[2 * lane] = r0;
  rp[2 * lane + 1] = r1;
}

// phi of each atom's shells: its row sums (groups g in order), then its
// column sums (target blocks I < its block, in order)
__global__ void k_field_sym_reduce(DevSystem sys, int group, int ngmax, const double* rowpart,
                                   const double* colpart, double* phi) {
  const int A = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = sys.natoms;
  if (A >= N) return;
  const int nb = (N + 63) / 64;
  const int B = A >> 6, l = A & 63;
  const int ng = (nb - B + group - 1) / group;
  double v0 = 0.0, v1 = 0.0;
  const double* rp = rowpart + (long long)B * ngmax * 128 + 2 * l;
  for (int g = 0; g < ng; ++g) {
    v0 += rp[(long long)g * 128];
    v1 += rp[(long long)g * 128 + 1];
  }
  const double* cp = colpart + (long long)B * (B - 1) / 2 * 128 + 2 * l;
#pragma unroll 4
  for (int I = 0; I < B; ++I) {
    v0 += cp[(long long)I * 128];
    v1 += cp[(long long)I * 128 + 1];
  }
  const int s0 = sys.atom_sh0[A], ns = sys.atom_sh0[A + 1] - s0;
  phi[s0] = v0;
  if (ns > 1) phi[s0 + 1] = v1;
}

__global__ void k_field_reduce(int nshells, int nchunk, const double* part, double* phi) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nshells) return;
  double acc = 0.0;
  for (int c = 0; c < nchunk; ++c) acc += part[(long long)c * nshells + s];
  phi[s] = acc;
}

// ---------------------------------------------------------------------------
// cluster (dimer / trimer) embedding from the monomer field:
// phi^X_s = Phi_s - sum_{t in X, frag(t) != frag(s)} gamma_st q_t
__global__ void k_cluster_phi(DevSystem sys, DevBatch bt, const double* Phi, const double* qmono) {
  int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int* shg = bt.sys_sh_global + d.sh_off;
  for (int s = threadIdx.x; s < d.nsh; s += blockDim.x) {
    int gs = shg[s];
    int fs = sys.sh_frag[gs];
    double v = Phi[gs];
    for (int t = 0; t < d.nsh; ++t) {
      int gt = shg[t];
      if (sys.sh_frag[gt] == fs) continue;
      v -= bt.gam[d.gam_off + (long long)s * d.nsh + t] * qmono[gt];
    }
    if (bt.healed_off) {
      // ghosts healed inside the cluster belong to its fragments but are not
      // part of its basis: their monomer charges are not environment either
      const double xs = sys.xyz[3 * sys.sh_atom[gs]], ys = sys.xyz[3 * sys.sh_atom[gs] + 1],
                   zs = sys.xyz[3 * sys.sh_atom[gs] + 2];
      for (int e = bt.healed_off[si]; e < bt.healed_off[si + 1]; ++e) {
        const int gt = bt.healed_sh[e];
        if (sys.sh_frag[gt] == fs) continue;
        const int At = sys.sh_atom[gt];
        const double dx = xs - sys.xyz[3 * At], dy = ys - sys.xyz[3 * At + 1], dz = zs - sys.xyz[3 * At + 2];
        v -= gamma_fn(sys.g, dx * dx + dy * dy + dz * dz, sys.sh_eta[gs], sys.sh_eta[gt]) * qmono[gt];
      }
    }
    bt.phi[d.sh_off + s] = v;
  }
}

// Embedding correction of the ghosts healed inside a cluster: their charge
// transfer is minus the monomer ghost charge (eq. ctij_ghost), acting on the
// environment potential at the ghost shells:
//   dEV += sum_g (-q_g) (Phi_g - sum_{t in cluster, other fragment} gamma_gt q_t)
// with the cluster's own shells and its other healed ghosts as t.
__global__ void k_cluster_healed(DevSystem sys, DevBatch bt, const double* Phi, const double* qmono, double* dEV,
                                 double* dE) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int e0 = bt.healed_off[si], e1 = bt.healed_off[si + 1];
  __shared__ double red[128];
  double loc = 0.0;
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int g = bt.healed_sh[e];
    const int fg = sys.sh_frag[g];
    const int Ag = sys.sh_atom[g];
    const double xg = sys.xyz[3 * Ag], yg = sys.xyz[3 * Ag + 1], zg = sys.xyz[3 * Ag + 2];
    double v = Phi[g];
    for (int t = 0; t < d.nsh; ++t) {
      const int gt = bt.sys_sh_global[d.sh_off + t];
      if (sys.sh_frag[gt] == fg) continue;
      const int At = sys.sh_atom[gt];
      const double dx = xg - sys.xyz[3 * At], dy = yg - sys.xyz[3 * At + 1], dz = zg - sys.xyz[3 * At + 2];
      v -= gamma_fn(sys.g, dx * dx + dy * dy + dz * dz, sys.sh_eta[g], sys.sh_eta[gt]) * qmono[gt];
    }
    for (int e2 = e0; e2 < e1; ++e2) {
      const int gt = bt.healed_sh[e2];
      if (sys.sh_frag[gt] == fg) continue;
      const int At = sys.sh_atom[gt];
      const double dx = xg - sys.xyz[3 * At], dy = yg - sys.xyz[3 * At + 1], dz = zg - sys.xyz[3 * At + 2];
      v -= gamma_fn(sys.g, dx * dx + dy * dy + dz * dz, sys.sh_eta[g], sys.sh_eta[gt]) * qmono[gt];
    }
    loc += -qmono[g] * v;
  }
  red[threadIdx.x] = loc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && e1 > e0) {
    dEV[si] += red[0];
    dE[si] += red[0];
  }
}

// HOP projector of each system, V = S D S (eq. vhop): D = V_HOP h h^T on a
// detached atom (eq. dd_bda), V_HOP (1_sp - h h^T) on a ghost (eq. dd_ghost),
// h = 1/2 s + sqrt(3)/2 (b . p) the bond-pointing sp3 hybrid (eq. hybrid).
__global__ void k_vhop(DevBatch bt, double vhop) {
  const int si = blockIdx.x;
  const SysDesc d = bt.desc[si];
  const int n = d.nao;
  double* Vh = bt.Vh + d.mat_off;
  const double* S = bt.S + d.mat_off;
  const int e0 = bt.hop_off[si], e1 = bt.hop_off[si + 1];
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int mu = idx / n, nu = idx - mu * n;
    double v = 0.0;
    for (int e = e0; e < e1; ++e) {
      const int o = bt.sys_atom_ao0[d.atom_off + bt.hop_atom[e]];
      const double* b = bt.hop_b + 3 * e;
      const double h[4] = {0.5, 0.8660254037844386 * b[0], 0.8660254037844386 * b[1], 0.8660254037844386 * b[2]};
      double xm[4], xn[4];
      for (int l = 0; l < 4; ++l) {
        xm[l] = S[(long long)mu * n + o + l];
        xn[l] = S[(long long)(o + l) * n + nu];
      }
      const double hm = h[0] * xm[0] + h[1] * xm[1] + h[2] * xm[2] + h[3] * xm[3];
      const double hn = h[0] * xn[0] + h[1] * xn[1] + h[2] * xn[2] + h[3] * xn[3];
      if (bt.hop_kind[e] == 1) {
        v += vhop * hm * hn;
      } else {
        const double xx = xm[0] * xn[0] + xm[1] * xn[1] + xm[2] * xn[2] + xm[3] * xn[3];
        v += vhop * (xx - hm * hn);
      }
    }
    Vh[idx] = v;
  }
}

// ES-DIM pair energies dq^I gamma_IJ dq^J for a list of pairs.
// One wave per ES-DIM pair (I, J): lane = atom of I, J's atoms taken in
// turn by the whole wave (uniform loads); with kg = 2 the kernel
// (R^2 + (iota_s + iota_t)^2)^(-1/2) with iota = 1/(2 eta), as in the field
// pass; lane sums combined by a fixed butterfly (deterministic).
__global__ void __launch_bounds__(64) k_esd_pairs(DevSystem sys, const int* pairs, long long npairs,
                                                  const int* frag_atoms, const int* frag_off, const double* q,
                                                  double* out) {
  const long long k = blockIdx.x;
  if (k >= npairs) return;
  const int lane = threadIdx.x;
  const int I = pairs[2 * k], J = pairs[2 * k + 1];
  const int j0 = frag_off[J], j1 = frag_off[J + 1];
  const bool kg2 = sys.g.kg == 2.0;
  double acc = 0.0;
  for (int ia = frag_off[I] + lane; ia < frag_off[I + 1]; ia += 64) {
    const int a = frag_atoms[ia];
    const double xa = sys.xyz[3 * a], ya = sys.xyz[3 * a + 1], za = sys.xyz[3 * a + 2];
    const int sa0 = sys.atom_sh0[a], nsa = sys.atom_sh0[a + 1] - sa0;
    const double qa0 = q[sa0], qa1 = nsa > 1 ? q[sa0 + 1] : 0.0;
    const double ia0 = sys.sh_ieta[sa0], ia1 = nsa > 1 ? sys.sh_ieta[sa0 + 1] : 0.5;
    for (int ib = j0; ib < j1; ++ib) {
      const int b = frag_atoms[ib];
      const double dx = xa - sys.xyz[3 * b], dy = ya - sys.xyz[3 * b + 1], dz = za - sys.xyz[3 * b + 2];
      const double R2 = dx * dx + dy * dy + dz * dz;
      const int sb0 = sys.atom_sh0[b], nsb = sys.atom_sh0[b + 1] - sb0;
      if (kg2) {
        // an absent second shell carries q = 0 and adds exactly zero
        const double qb0 = q[sb0], qb1 = nsb > 1 ? q[sb0 + 1] : 0.0;
        const double ib0 = sys.sh_ieta[sb0], ib1 = nsb > 1 ? sys.sh_ieta[sb0 + 1] : 0.5;
        const double t00 = ia0 + ib0, t01 = ia0 + ib1, t10 = ia1 + ib0, t11 = ia1 + ib1;
        acc += qa0 * (rsqrt_pos(R2 + t00 * t00) * qb0 + rsqrt_pos(R2 + t01 * t01) * qb1) +
               qa1 * (rsqrt_pos(R2 + t10 * t10) * qb0 + rsqrt_pos(R2 + t11 * t11) * qb1);
      } else {
        for (int s = sa0; s < sa0 + nsa; ++s)
          for (int t = sb0; t < sb0 + nsb; ++t) acc += q[s] * gamma_fn(sys.g, R2, sys.sh_eta[s], sys.sh_eta[t]) * q[t];
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) out[k] = acc;
}

}  // namespace fx
