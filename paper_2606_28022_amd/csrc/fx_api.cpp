// Host driver and C ABI of the FMO-xTB library.
//
// The driver owns the supersystem tables in device memory, builds fragment
// batches (monomers, SCC dimers, trimers), runs the batched SCC kernels
// until every system of a batch has converged, and assembles the FMO
// energy.  All arithmetic of the method runs in the HIP kernels; the host
// only builds index tables, launches kernels and reads convergence flags.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/fmoxtb.h"
#include "fx_device.hpp"
#include "fx_kernels.hpp"
#include "fx_host.hpp"
#include "json_mini.hpp"

using namespace fx;

// ---------------------------------------------------------------------------
// parameters

namespace fx {

static double prim_norm(int l, double a) {
  double n = std::pow(2.0 * a / M_PI, 0.75);
  if (l == 1) n *= 2.0 * std::sqrt(a);
  return n;
}

HostParams load_params(const std::string& path) {
  std::ifstream f(path);
  if (!f) throw FxError(FX_E_INVALID, "cannot open parameter file " + path);
  std::stringstream ss;
  ss << f.rdbuf();
  JVal root = JParser(ss.str()).parse();
  HostParams P;
  const JVal& g = root["globals"];
  P.g.kg = g["kg"].d();
  P.g.kf = g["kf"].d();
  P.g.kEN = g["kEN"].d();
  P.g.k1 = g["k1"].d();
  P.g.k2 = g["k2"].d();
  for (int l = 0; l < 3; ++l) P.g.kl[l] = l < (int)g["kl"].size() ? g["kl"][l].d() : 0.0;
  P.g.KAB = g["KAB"].d();
  P.g.kT = g["Tel_K"].d() * g["kB_Eh_per_K"].d();
  P.g.VHOP = g.has("VHOP") ? g["VHOP"].d() : 1e6;
  double a2b = g["angstrom_to_bohr"].d();
  std::map<std::string, std::pair<std::vector<double>, std::vector<double>>> basis;
  for (auto& kv : root["basis"].obj) {
    const JVal& b = kv.second;
    std::vector<double> al, co;
    for (auto& x : b["alpha"].arr) al.push_back(x.d());
    for (auto& x : b["coef"].arr) co.push_back(x.d());
    if ((int)al.size() != NPRIM || (int)co.size() != NPRIM)
      throw FxError(FX_E_UNSUPPORTED, "basis expansions must have 6 primitives");
    basis[std::to_string(b["n"].i()) + ":" + std::to_string(b["l"].i())] = {al, co};
  }
  for (auto& kv : root["elements"].obj) {
    const JVal& e = kv.second;
    int Z = e["Z"].i();
    if (Z < 1 || Z > 118) throw FxError(FX_E_INVALID, "bad element number");
    DevElem el;
    std::memset(&el, 0, sizeof(el));
    const JVal& shells = e["shells"];
    if ((int)shells.size() > MAXSH_EL) throw FxError(FX_E_UNSUPPORTED, "too many shells for element " + kv.first);
    el.nsh = (int)shells.size();
    int ao = 0;
    for (int s = 0; s < el.nsh; ++s) {
      const JVal& sh = shells[s];
      int n = sh["n"].i(), l = sh["l"].i();
      if (l > 1) throw FxError(FX_E_UNSUPPORTED, "only s and p shells are supported");
      auto it = basis.find(std::to_string(n) + ":" + std::to_string(l));
      if (it == basis.end()) throw FxError(FX_E_UNSUPPORTED, "no basis expansion for a shell of " + kv.first);
      double zeta = sh["zeta"].d();
      el.l[s] = l;
      el.nao_sh[s] = l == 0 ? 1 : 3;
      el.ao0[s] = ao;
      ao += el.nao_sh[s];
      el.level[s] = sh["level"].d();
      el.kcn[s] = sh["kcn"].d();
      el.kpoly[s] = sh["kpoly"].d();
      el.eta[s] = (1.0 + sh["kappa"].d()) * e["eta"].d();
      el.q0[s] = sh["q0"].d();
      double norm2 = 0.0;
      for (int i = 0; i < NPRIM; ++i) {
        el.alpha[s][i] = it->second.first[i] * zeta * zeta;
        el.coef[s][i] = it->second.second[i] * prim_norm(l, el.alpha[s][i]);
      }
      for (int i = 0; i < NPRIM; ++i)
        for (int j = 0; j < NPRIM; ++j) {
          double p = el.alpha[s][i] + el.alpha[s][j];
          double v = std::pow(M_PI / p, 1.5);
          if (l == 1) v /= 2.0 * p;
          norm2 += el.coef[s][i] * el.coef[s][j] * v;
        }
      for (int i = 0; i < NPRIM; ++i) el.coef[s][i] /= std::sqrt(norm2);
    }
    el.nao = ao;
    // the derivative kernels address AO blocks by shell position: shell 0 an
    // s shell (AO 0), shell 1 (if any) from AO 1
    if (el.nsh < 1 || el.nsh > MAXSH_EL || el.l[0] != 0)
      throw FxError(FX_E_UNSUPPORTED, "element " + kv.first + ": the first shell must be an s shell (at most " +
                                          std::to_string(MAXSH_EL) + " shells)");
    el.orth = 0;
    if (el.nsh == 2 && el.l[0] == 0 && el.l[1] == 0) {
      double s12 = 0.0;
      for (int i = 0; i < NPRIM; ++i)
        for (int j = 0; j < NPRIM; ++j)
          s12 += el.coef[0][i] * el.coef[1][j] * std::pow(M_PI / (el.alpha[0][i] + el.alpha[1][j]), 1.5);
      el.orth = 1;
      el.orthS12 = s12;
      el.orthN = 1.0 / std::sqrt(1.0 - s12 * s12);
    }
    el.EN = e["EN"].d();
    el.rcov = e["rcov_angstrom"].d() * a2b;
    el.Gamma = e["Gamma"].d();
    el.zeff = e["zeff"].d();
    el.arep = e["alpha_rep"].d();
    el.rvdw = e.has("rvdw_angstrom") ? e["rvdw_angstrom"].d() * a2b : 0.0;
    el.Z = Z;
    P.elem_of_Z[Z] = (int)P.elems.size();
    P.elems.push_back(el);
  }
  return P;
}

}  // namespace fx

struct fx_params {
  fx::HostParams P;
};

// ---------------------------------------------------------------------------
// context helpers

namespace fx {

thread_local DevMem* g_devmem = nullptr;

void Ctx::check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw FxError(FX_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void Ctx::sync() { check(hipStreamSynchronize(stream), "hipStreamSynchronize"); }

double Ctx::now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

DevSystem Ctx::dev_system() const {
  DevSystem s;
  s.natoms = Ne;
  s.nreal = N;
  s.nshells = Nsh;
  s.nfrag = F;
  s.xyz = d_xyz.p;
  s.elem = d_elem.p;
  s.frag = d_frag.p;
  s.atom_sh0 = d_atom_sh0.p;
  s.cn = d_cn.p;
  s.sh_atom = d_sh_atom.p;
  s.sh_frag = d_sh_frag.p;
  s.sh_eta = d_sh_eta.p;
  s.sh_ieta = d_sh_ieta.p;
  s.elems = d_elems.p;
  s.g = P.g;
  return s;
}

// Build a batch of fragment systems (each a tuple of 1..3 fragments).
void Ctx::build_batch(Batch& b, const std::vector<std::array<int, 3>>& clusters, int nfrag_each) {
  b.init_from_mono = false;
  if (b.h_system_gen == system_gen && b.h_nfrag == nfrag_each && b.h_clusters == clusters) {
    // the same clusters of the same system as the last build: the tables
    // (atoms, shells, offsets, boundary charges) stand and the pools keep
    // their layout; only the projector bond directions follow the
    // coordinates
    if (b.has_hop) {
      std::vector<double> hb(3 * (size_t)b.n_hop);
      for (int e = 0; e < b.n_hop; ++e) {
        const int kb = b.h_hop_bond[e], a = bonds[2 * kb], bb = bonds[2 * kb + 1];
        double v[3], r2 = 0.0;
        for (int c = 0; c < 3; ++c) {
          v[c] = xyz_h[3 * bb + c] - xyz_h[3 * a + c];
          r2 += v[c] * v[c];
        }
        const double r = std::sqrt(r2);
        for (int c = 0; c < 3; ++c) hb[3 * e + c] = v[c] / r;
      }
      b.hop_b.upload(hb);
    }
    b.has_pre = false;
    check(hipMemsetAsync(b.phi.p, 0, sizeof(double) * std::max(1, b.tot_sh), stream), "memset");
    return;
  }
  b.max_nao = 0;
  b.h_clusters = clusters;
  b.h_nfrag = nfrag_each;
  b.h_system_gen = -1;  // set once the build has completed
  const int ns = (int)clusters.size();
  b.nsys = ns;
  std::vector<SysDesc> desc(ns);
  std::vector<int> atoms, atom_ao0, atom_sh0, sh_global, sh_atom, ao_sh;
  // covalent-boundary tables (section "Covalent bond fragmentation")
  std::vector<double> sh_q0, atom_zs, hop_b;
  std::vector<int> hop_off(1, 0), hop_atom, hop_kind, hop_bond, healed_off(1, 0), healed_sh;
  std::vector<int> loc(Ne, -1);  // local index of an extended atom in the current system
  std::vector<int> sh_mono;      // index of each local shell within its fragment's monomer
  long long mat = 0, gam = 0;
  int sh_off = 0, ao_off = 0, atom_off = 0;
  for (int k = 0; k < ns; ++k) {
    SysDesc& d = desc[k];
    d.nfrag = nfrag_each;
    d.atom_off = atom_off;
    d.sh_off = sh_off;
    d.ao_off = ao_off;
    d.mat_off = mat;
    d.gam_off = gam;
    int nat = 0, nsh = 0, nao = 0;
    double charge = 0.0;
    for (int f = 0; f < 3; ++f) d.frag[f] = -1;
    for (int f = 0; f < 4; ++f) d.comp_sh[f] = 0;
    auto inside = [&](int fr) {
      for (int c = 0; c < nfrag_each; ++c)
        if (clusters[k][c] == fr) return true;
      return false;
    };
    std::vector<int> sys_atoms;
    for (int f = 0; f < nfrag_each; ++f) {
      const int I = clusters[k][f];
      d.frag[f] = I;
      d.comp_sh[f] = nsh;
      charge += frag_charge[I];
      int msh = 0;
      for (int ia = frag_off[I]; ia < frag_off[I + 1]; ++ia) {
        const int A = frag_atoms[ia];
        const DevElem& el = P.elems[elem[A]];
        // a ghost whose detached atom is inside too: the bond is healed
        if (A >= N && inside(frag[bonds[2 * (A - N)]])) {
          msh += el.nsh;
          continue;
        }
        for (int s = 0; s < el.nsh; ++s) sh_mono.push_back(msh + s);
        msh += el.nsh;
        loc[A] = nat;
        sys_atoms.push_back(A);
        atoms.push_back(A);
        atom_ao0.push_back(nao);
        atom_sh0.push_back(nsh);
        for (int s = 0; s < el.nsh; ++s) {
          sh_global.push_back(atom_sh0_g[A] + s);
          sh_atom.push_back(nat);
          sh_q0.push_back(el.q0[s]);
          for (int u = 0; u < el.nao_sh[s]; ++u) ao_sh.push_back(nsh);
          ++nsh;
        }
        atom_zs.push_back(1.0);
        nao += el.nao;
        ++nat;
      }
    }
    d.comp_sh[nfrag_each] = nsh;
    // boundary atoms of this system: detached atoms whose partner is outside
    // give up one electron (1/4 s, 3/4 p) and get the projector of their
    // bond hybrid; ghosts of bonds whose detached atom is outside carry one
    // electron (1/4 s, 3/4 p); repulsion charges scale by (v-1)/v and 1/v
    for (int f = 0; f < nfrag_each; ++f) {
      const int I = clusters[k][f];
      for (int kb : bda_bonds[I]) {
        const int a = bonds[2 * kb], bb = bonds[2 * kb + 1];
        if (inside(frag[bb])) continue;
        hop_atom.push_back(loc[a]);
        hop_kind.push_back(1);
        hop_bond.push_back(kb);
        for (int c = 0; c < 3; ++c) hop_b.push_back(xyz_h[3 * bb + c] - xyz_h[3 * a + c]);
      }
      for (int kb : ghost_bonds[I]) {
        const int a = bonds[2 * kb];
        if (inside(frag[a])) {
          const int g = N + kb;
          for (int s = atom_sh0_g[g]; s < atom_sh0_g[g + 1]; ++s) healed_sh.push_back(s);
          continue;
        }
        const int bb = bonds[2 * kb + 1];
        hop_atom.push_back(loc[N + kb]);
        hop_kind.push_back(2);
        hop_bond.push_back(kb);
        for (int c = 0; c < 3; ++c) hop_b.push_back(xyz_h[3 * bb + c] - xyz_h[3 * a + c]);
      }
    }
    for (int e = hop_off.back(); e < (int)hop_atom.size(); ++e) {
      double* bv = &hop_b[3 * e];
      const double r = std::sqrt(bv[0] * bv[0] + bv[1] * bv[1] + bv[2] * bv[2]);
      for (int c = 0; c < 3; ++c) bv[c] /= r;
      const int la = hop_atom[e];
      const int s0 = atom_sh0[atom_off + la];
      const double v = sh_q0[sh_off + s0] + sh_q0[sh_off + s0 + 1];
      if (hop_kind[e] == 1) {
        sh_q0[sh_off + s0] -= 0.25;
        sh_q0[sh_off + s0 + 1] -= 0.75;
        atom_zs[atom_off + la] *= (v - 1.0) / v;
      } else {
        sh_q0[sh_off + s0] = 0.25;
        sh_q0[sh_off + s0 + 1] = 0.75;
        atom_zs[atom_off + la] *= 1.0 / v;
      }
    }
    hop_off.push_back((int)hop_atom.size());
    healed_off.push_back((int)healed_sh.size());
    for (int A : sys_atoms) loc[A] = -1;
    double nel = -charge;
    for (int s = 0; s < nsh; ++s) nel += sh_q0[sh_off + s];
    if (nao > MAXN) throw FxError(FX_E_UNSUPPORTED, "fragment system larger than 512 AOs");
    d.nat = nat;
    d.nsh = nsh;
    d.nao = nao;
    d.nel = nel;
    atom_off += nat;
    sh_off += nsh;
    ao_off += nao;
    mat += (long long)nao * nao;
    gam += (long long)nsh * nsh;
    b.max_nao = std::max(b.max_nao, nao);
  }
  b.sh_mono.upload(sh_mono);
  b.h_hop_off = hop_off;
  b.h_hop_bond = hop_bond;
  b.h_healed_off = healed_off;
  b.h_healed_sh = healed_sh;
  b.has_hop = !hop_atom.empty();
  b.n_hop = (int)hop_atom.size();
  b.has_healed = !healed_sh.empty();
  if (b.has_hop || b.has_healed) {
    b.sh_q0.upload(sh_q0);
    b.atom_zs.upload(atom_zs);
    b.hop_off.upload(hop_off);
    b.hop_atom.upload(hop_atom.empty() ? std::vector<int>{0} : hop_atom);
    b.hop_kind.upload(hop_kind.empty() ? std::vector<int>{0} : hop_kind);
    b.hop_bond.upload(hop_bond.empty() ? std::vector<int>{0} : hop_bond);
    b.hop_b.upload(hop_b.empty() ? std::vector<double>{0.0} : hop_b);
    b.healed_off.upload(healed_off);
    b.healed_sh.upload(healed_sh.empty() ? std::vector<int>{0} : healed_sh);
  }
  b.h_desc = desc;
  b.tot_sh = sh_off;
  b.tot_ao = ao_off;
  b.tot_mat = mat;
  b.tot_gam = gam;
  b.has_pre = false;
  b.d_desc.upload(desc);
  b.d_atoms.upload(atoms);
  b.h_atoms = atoms;
  b.d_atom_ao0.upload(atom_ao0);
  b.d_atom_sh0.upload(atom_sh0);
  b.d_sh_global.upload(sh_global);
  b.h_sh_global = sh_global;
  b.d_sh_atom.upload(sh_atom);
  b.d_ao_sh.upload(ao_sh);
  b.S.alloc(mat);
  b.H0.alloc(mat);
  b.Fm.alloc(mat);
  b.Ct.alloc(mat);
  b.Pm.alloc(mat);
  b.Tm.alloc(mat);
  b.gam.alloc(gam);
  b.q_in.alloc(sh_off);
  b.q_out.alloc(sh_off);
  b.phi.alloc(sh_off);
  b.sig.alloc(sh_off);
  b.hx.alloc((long long)sh_off * HIST);
  b.hr.alloc((long long)sh_off * HIST);
  b.eps.alloc(ao_off);
  b.occ.alloc(ao_off);
  b.occ_idx.alloc(ao_off);
  b.occ_cnt.alloc(ns);
  b.erep.alloc(ns);
  b.e_int.alloc(ns);
  b.e_prev.alloc(ns);
  b.mts.alloc(ns);
  b.err.alloc(ns);
  b.status.alloc(ns);
  b.niter.alloc(ns);
  b.nhist.alloc(ns);
  b.sweeps.alloc(ns);
  std::vector<int> all(ns);
  for (int k = 0; k < ns; ++k) all[k] = k;
  b.d_all.upload(all);
  check(hipMemsetAsync(b.phi.p, 0, sizeof(double) * std::max(1, sh_off), stream), "memset");
  b.h_system_gen = system_gen;
}

DevBatch Batch::dev() {
  DevBatch d;
  d.nsys = nsys;
  d.desc = d_desc.p;
  d.sys_atoms = d_atoms.p;
  d.sys_atom_ao0 = d_atom_ao0.p;
  d.sys_atom_sh0 = d_atom_sh0.p;
  d.sys_sh_global = d_sh_global.p;
  d.sys_sh_atom = d_sh_atom.p;
  d.sys_ao_sh = d_ao_sh.p;
  d.S = S.p;
  d.H0 = H0.p;
  d.F = Fm.p;
  d.Ct = Ct.p;
  d.P = Pm.p;
  d.T = Tm.p;
  d.gam = gam.p;
  d.q_in = q_in.p;
  d.q_out = q_out.p;
  d.phi = phi.p;
  d.sig = sig.p;
  d.pre = has_pre ? pre.p : nullptr;
  const bool hb = has_hop || has_healed;
  d.sh_q0 = hb ? sh_q0.p : nullptr;
  d.atom_zs = hb ? atom_zs.p : nullptr;
  d.Vh = has_hop ? Vh.p : nullptr;
  d.hop_off = hb ? hop_off.p : nullptr;
  d.hop_atom = hb ? hop_atom.p : nullptr;
  d.hop_kind = hb ? hop_kind.p : nullptr;
  d.hop_b = hb ? hop_b.p : nullptr;
  d.hop_bond = hb ? hop_bond.p : nullptr;
  d.healed_off = has_healed ? healed_off.p : nullptr;
  d.healed_sh = has_healed ? healed_sh.p : nullptr;
  d.sh_mono = sh_mono.p;
  d.hx = hx.p;
  d.hr = hr.p;
  d.eps = eps.p;
  d.occ = occ.p;
  d.occ_idx = occ_idx.p;
  d.occ_cnt = occ_cnt.p;
  d.erep = erep.p;
  d.e_int = e_int.p;
  d.e_prev = e_prev.p;
  d.mts = mts.p;
  d.err = err.p;
  d.status = status.p;
  d.niter = niter.p;
  d.nhist = nhist.p;
  return d;
}

void Ctx::init_device() {
  int v = 0;
  check(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device), "LDS size query");
  // dynamic LDS available to k_jacobi_lds: the per-workgroup limit minus the
  // kernels' static LDS; raising the dynamic limit is advisory (the runtime
  // rejects an oversized launch, which check() then reports)
  unsigned stat = 0;
  for (const void* k : {reinterpret_cast<const void*>(k_jacobi_lds<double>),
                        reinterpret_cast<const void*>(k_jacobi_lds<float>),
                        reinterpret_cast<const void*>(k_jacobi_rot<double>),
                        reinterpret_cast<const void*>(k_jacobi_rot<float>)}) {
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, k) == hipSuccess) stat = std::max(stat, (unsigned)fa.sharedSizeBytes);
  }
  lds_max = v - (int)stat;
  for (const void* k : {reinterpret_cast<const void*>(k_jacobi_lds<double>),
                        reinterpret_cast<const void*>(k_jacobi_lds<float>)})
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_resp_Q), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds_max);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_resp_M), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds_max);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_resp_M_mfma), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds_max);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_resp_R_lds), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds_max - 24576);
  for (const void* k : {reinterpret_cast<const void*>(k_precond_build<PRE_ROWS_SMALL>),
                        reinterpret_cast<const void*>(k_precond_build<PRE_ROWS>)})
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max - 16384);
  for (const void* k : {reinterpret_cast<const void*>(k_jacobi_rot<double>),
                        reinterpret_cast<const void*>(k_jacobi_rot<float>),
                        reinterpret_cast<const void*>(k_apply_rot),
                        reinterpret_cast<const void*>(k_apply_rot_dual),
                        reinterpret_cast<const void*>(k_cholinv_lds<double>),
                        reinterpret_cast<const void*>(k_cholinv_lds<float>),
                        reinterpret_cast<const void*>(k_cholinv_block2)})
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
  (void)hipGetLastError();
  check(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device), "CU count query");
  noalloc_init(device);
  if (verbose) std::fprintf(stderr, "[fx] LDS per workgroup %d B, static %u B\n", v, stat);
}

// Batched n x n products of the listed systems (first nl entries of dlist):
// the matrix-core kernel once a system spans more than one 32 x 32 tile.
void Ctx::gemm_batch(const Batch& b, const DevBatch& db, int nl, const int* dlist, int mode, const double* A,
                     const double* B, double* C, const double* w, double gflop, int skip_done, int sym,
                     bool occ_list, int win) {
  if (nl <= 0) return;
  const bool timed = !capturing;
  if (b.max_nao <= 32) {
    const int ev = timed ? timers.begin(stream) : -1;
    hipLaunchKernelGGL(k_gemm, dim3(1, nl), dim3(256), 0, stream, db, dlist, mode, A, B, C, w, skip_done);
    if (timed) timers.end(stream, ev, kt("fx::k_gemm"), gflop);
  } else {
    const int nt = (b.max_nao + 63) / 64;
    const long long grid = xcd_grid(nl, nt * nt);
    if (grid > 0x7fffffffLL) throw FxError(FX_E_INVALID, "batched product grid too large");
    const int ev = timed ? timers.begin(stream) : -1;
    if (win && mode == 0)
      hipLaunchKernelGGL((k_gemm_mfma<0, 1>), dim3((unsigned)grid), dim3(256), 0, stream, db, dlist, nl, nt * nt, A, B,
                         C, w, skip_done, 0, 0);
    else if (win && mode == 1)
      hipLaunchKernelGGL((k_gemm_mfma<1, 1>), dim3((unsigned)grid), dim3(256), 0, stream, db, dlist, nl, nt * nt, A, B,
                         C, w, skip_done, 0, 0);
    else if (mode == 0)
      hipLaunchKernelGGL((k_gemm_mfma<0, 0>), dim3((unsigned)grid), dim3(256), 0, stream, db, dlist, nl, nt * nt, A, B,
                         C, w, skip_done, sym, occ_list ? 1 : 0);
    else if (mode == 1)
      hipLaunchKernelGGL((k_gemm_mfma<1, 0>), dim3((unsigned)grid), dim3(256), 0, stream, db, dlist, nl, nt * nt, A, B,
                         C, w, skip_done, sym, occ_list ? 1 : 0);
    else
      hipLaunchKernelGGL((k_gemm_mfma<2, 0>), dim3((unsigned)grid), dim3(256), 0, stream, db, dlist, nl, nt * nt, A, B,
                         C, w, skip_done, sym, occ_list ? 1 : 0);
    if (timed) timers.end(stream, ev, kt("fx::k_gemm_mfma"), gflop);
  }
  check(hipGetLastError(), "batched product");
}

void Ctx::gemm_batch_f32(const Batch& b, const DevBatch& db, int nl, const int* dlist, int mode, const void* A,
                         const void* B, void* C, const double* w, double gflop, int skip_done, int sym,
                         bool occ_list) {
  if (nl <= 0) return;
  const int nt = (b.max_nao + 63) / 64;
  const long long grid = xcd_grid(nl, nt * nt);
  if (grid > 0x7fffffffLL) throw FxError(FX_E_INVALID, "batched product grid too large");
  const int ev = capturing ? -1 : timers.begin(stream);
  if (mode == 0)
    hipLaunchKernelGGL((k_gemm_f32<0, double, float, float>), dim3((unsigned)grid), dim3(256), 0, stream, db, dlist,
                       nl, nt * nt, (const double*)A, (const float*)B, (float*)C, w, skip_done, sym, occ_list ? 1 : 0);
  else if (mode == 1)
    hipLaunchKernelGGL((k_gemm_f32<1, float, double, double>), dim3((unsigned)grid), dim3(256), 0, stream, db,
                       dlist, nl, nt * nt, (const float*)A, (const double*)B, (double*)C, w, skip_done, sym,
                       occ_list ? 1 : 0);
  else
    hipLaunchKernelGGL((k_gemm_f32<2, double, double, double>), dim3((unsigned)grid), dim3(256), 0, stream, db,
                       dlist, nl, nt * nt, (const double*)A, (const double*)B, (double*)C, w, skip_done, sym,
                       occ_list ? 1 : 0);
  if (!capturing) timers.end(stream, ev, kt("fx::k_gemm_f32"), gflop);
  check(hipGetLastError(), "batched FP32 product");
}

unsigned Ctx::resp_M_lds(const Batch& b) const {
  int nsh = 0;
  for (const auto& d : b.h_desc) nsh = std::max(nsh, d.nsh);
  const size_t by = resp_M_lds_bytes(nsh);
  if ((long long)by > (long long)lds_max) throw FxError(FX_E_UNSUPPORTED, "monomer with too many shells");
  return (unsigned)by;
}

// M = sum_ai Q_ai Q_ai^T / (eps_a - eps_i) of every system of the batch: on
// the matrix cores where the shells fit, else the register-blocked kernel
void Ctx::launch_resp_M(const Batch& b, const DevBatch& db, const int* order, const int* nocc, const long long* qoff,
                        const double* Q, double* M) {
  int nsh = 0;
  for (const auto& d : b.h_desc) nsh = std::max(nsh, d.nsh);
  const size_t bm = resp_M_mfma_lds_bytes(nsh);
  if (nsh <= 16 * RMM_MAXB && (long long)bm <= (long long)lds_max)
    hipLaunchKernelGGL(k_resp_M_mfma, dim3(b.nsys), dim3(256), (unsigned)bm, stream, db, order, nocc, qoff, Q, M);
  else
    hipLaunchKernelGGL(k_resp_M, dim3(b.nsys), dim3(256), resp_M_lds(b), stream, db, order, nocc, qoff, Q, M);
}

// Charge susceptibilities of the monomers from their current orbitals
// (shell-summed transition charges Q and M = sum_ai Q Q^T / (eps_a - eps_i));
// closed-shell monomers only (returns false otherwise).
bool Ctx::monomer_response_setup() {
  resp_ok = false;
  Batch& b = mb;
  if (b.nsys == 0) return false;
  std::vector<int> nocc(b.nsys);
  std::vector<long long> qoff(b.nsys + 1, 0);
  for (int k = 0; k < b.nsys; ++k) {
    const SysDesc& d = b.h_desc[k];
    const int ne = (int)std::lround(d.nel);
    if (std::fabs(d.nel - ne) > 1e-9 || (ne & 1) || ne / 2 >= d.nao || ne <= 0) return false;
    nocc[k] = ne / 2;
    qoff[k + 1] = qoff[k] + (long long)d.nsh * nocc[k] * (d.nao - nocc[k]);
  }
  {
    int nsh = 0;
    for (const auto& d : b.h_desc) nsh = std::max(nsh, d.nsh);
    if ((long long)resp_M_lds_bytes(nsh) > (long long)lds_max) return false;
    if ((long long)resp_Q_lds_bytes(b.max_nao) > (long long)lds_max) return false;
  }
  DevBatch dmb = b.dev();
  resp_nocc.upload(nocc);
  resp_qoff.upload(qoff);
  resp_order.alloc(b.tot_ao);
  resp_Q.alloc(std::max(1LL, qoff[b.nsys]));
  resp_M.alloc(std::max(1LL, b.tot_gam));
  std::vector<int> all(b.nsys);
  for (int k = 0; k < b.nsys; ++k) all[k] = k;
  b.d_list.upload(all);
  hipLaunchKernelGGL(k_mo_order, dim3(b.nsys), dim3(256), 0, stream, dmb, resp_nocc.p, resp_order.p);
  // (S C)^T = Ct S into the GEMM scratch
  gemm_batch(b, dmb, b.nsys, b.d_list.p, 0, b.Ct.p, b.S.p, b.Tm.p, (const double*)nullptr, b.gemm_gflop_all());
  hipLaunchKernelGGL(k_resp_Q, dim3(b.nsys), dim3(256), (unsigned)resp_Q_lds_bytes(b.max_nao), stream, dev_system(),
                     dmb, b.Tm.p, resp_order.p,
                     resp_nocc.p, resp_qoff.p, resp_Q.p);
  launch_resp_M(b, dmb, resp_order.p, resp_nocc.p, resp_qoff.p, resp_Q.p, resp_M.p);
  check(hipGetLastError(), "monomer susceptibilities");
  resp_ok = true;
  return true;
}

// Newton preconditioners of the mixer for every system of the batch, from
// the monomer susceptibilities and the systems' current input charges.
void Ctx::build_precond(Batch& b) {
  b.has_pre = false;
  if (!precond || !resp_ok || b.nsys == 0) return;
  int nsmax = 0;
  for (const auto& d : b.h_desc) nsmax = std::max(nsmax, d.nsh);
  // K in FP32, and the operand chunks of its product (two KC x ns FP64
  // blocks, KC = min(16, max(1, ns / 4))) in the same bytes
  const unsigned ldk = ((unsigned)nsmax + 3u) & ~3u;  // K rows padded to whole float4s
  const unsigned bytes = std::max(4u * (unsigned)nsmax * ldk, 16u * (unsigned)nsmax);
  if ((int)bytes > lds_max - 16384 || nsmax > PRE_MAXSH) return;
  b.pre.alloc(std::max(1LL, b.tot_gam));
  DevBuf<int> ok;
  ok.alloc(b.nsys);
  DevBatch db = b.dev();
  if (nsmax <= 16 * PRE_ROWS_SMALL)
    hipLaunchKernelGGL(k_precond_build<PRE_ROWS_SMALL>, dim3(b.nsys), dim3(PRE_THREADS), bytes, stream, dev_system(),
                       db, b.d_all.p, mb.dev(), (const double*)resp_M.p, b.pre.p, ok.p);
  else
    hipLaunchKernelGGL(k_precond_build<PRE_ROWS>, dim3(b.nsys), dim3(PRE_THREADS), bytes, stream, dev_system(), db,
                       b.d_all.p, mb.dev(), (const double*)resp_M.p, b.pre.p, ok.p);
  check(hipGetLastError(), "k_precond_build");
  std::vector<int> h;
  ok.download(h, stream);
  sync();
  int bad = 0;
  for (int v : h) bad += v == 0;
  if (verbose) std::fprintf(stderr, "[fx] mixing preconditioner for %d systems (%d singular)\n", b.nsys, bad);
  b.has_pre = true;
}

// ---------------------------------------------------------------------------
// learned initial guess

void Ctx::mlp_set_master(const float* w) {
  std::vector<float> h(w, w + FX_MLP_NW);
  for (float v : h)
    if (!std::isfinite(v)) throw FxError(FX_E_INVALID, "non-finite weight");
  mlp_master.upload(h);
  std::vector<float> z(FX_MLP_NW, 0.0f);
  mlp_m.upload(z);
  mlp_v.upload(z);
  mlp_wr.alloc(FX_MLP_NW);
  mlp_grad.alloc(FX_MLP_NW);
  hipLaunchKernelGGL(k_mlp_round, dim3((FX_MLP_NW + 255) / 256), dim3(256), 0, stream, mlp_master.p, mlp_wr.p);
  check(hipGetLastError(), "k_mlp_round");
  sync();
  mlp_t = 0;
  mlp_loaded = true;
}

void Ctx::mlp_features(float* d_out) {
  if (!has_system) throw FxError(FX_E_STATE, "no system set");
  hipLaunchKernelGGL(k_mlp_features, dim3((N + 255) / 256), dim3(256), 0, stream, dev_system(), d_out);
  check(hipGetLastError(), "k_mlp_features");
}

void Ctx::mlp_infer(const float* d_x, float* d_y, long long n) {
  if (!mlp_loaded) throw FxError(FX_E_STATE, "no guess model loaded");
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, mlp_wr.p, d_x, d_y, n);
  check(hipGetLastError(), "k_mlp_forward");
}

// loss and gradient into mlp_grad (device); returns the loss
double Ctx::mlp_grad_impl(const float* d_x, const float* d_y, long long n) {
  if (!mlp_loaded) throw FxError(FX_E_STATE, "no guess model loaded");
  if (n <= 0) throw FxError(FX_E_INVALID, "no training rows");
  const long long nparts = (n + 31) / 32;
  if (nparts > 0x7fffffffLL) throw FxError(FX_E_INVALID, "too many training rows");
  mlp_part.alloc(nparts * FX_MLP_NW);
  mlp_lpart.alloc(nparts);
  mlp_loss.alloc(1);
  hipLaunchKernelGGL(k_mlp_grad_partial, dim3((unsigned)nparts), dim3(256), 0, stream, mlp_wr.p, d_x, d_y, n,
                     mlp_part.p, mlp_lpart.p);
  hipLaunchKernelGGL(k_mlp_grad_reduce, dim3((FX_MLP_NW + 255) / 256), dim3(256), 0, stream, mlp_part.p,
                     (int)nparts, mlp_grad.p);
  hipLaunchKernelGGL(k_mlp_loss_reduce, dim3(1), dim3(1), 0, stream, mlp_lpart.p, (int)nparts,
                     1.0 / (2.0 * (double)n), mlp_loss.p);
  check(hipGetLastError(), "mlp gradient");
  std::vector<double> h;
  mlp_loss.download(h, stream, 1);
  sync();
  return h[0];
}

// learned monomer charges into d_q (projected per fragment)
void Ctx::learned_guess() {
  if (!mlp_loaded) throw FxError(FX_E_STATE, "learned guess requested but no model loaded");
  mlp_feat.alloc((long long)N * FX_MLP_NFEAT);
  mlp_out.alloc(2LL * N);
  mlp_features(mlp_feat.p);
  mlp_infer(mlp_feat.p, mlp_out.p, N);
  DevBuf<int> fc;
  fc.upload(frag_charge);
  hipLaunchKernelGGL(k_guess_assemble, dim3((Ne + 255) / 256), dim3(256), 0, stream, dev_system(), mlp_out.p, d_q.p);
  hipLaunchKernelGGL(k_guess_project, dim3(F), dim3(256), 0, stream, dev_system(), d_frag_atoms.p, d_frag_off.p,
                     fc.p, d_q.p);
  check(hipGetLastError(), "learned guess");
  sync();
}

// Launch-shape autotuning of the LDS Jacobi for one size bucket: candidate
// (threads, chunk) pairs with the same working precision, each timed on fresh
// copies of the batch's A and C^T with HIP events; the fastest is returned.
JacobiPlan Ctx::autotune_jacobi(Batch& b, const int* dl, int na, const JacobiPlan& base, double cap) {
  const long long tm = b.tot_mat;
  DevBuf<double> A0, V0, A1, V1;
  A0.alloc(tm);
  V0.alloc(tm);
  A1.alloc(tm);
  V1.alloc(tm);
  DevBuf<int> sw;
  sw.alloc(b.nsys);
  check(hipMemcpyAsync(A0.p, b.Fm.p, sizeof(double) * tm, hipMemcpyDeviceToDevice, stream), "copy");
  check(hipMemcpyAsync(V0.p, b.Ct.p, sizeof(double) * tm, hipMemcpyDeviceToDevice, stream), "copy");
  DevBatch db = b.dev();
  db.F = A1.p;
  db.Ct = V1.p;
  std::vector<JacobiPlan> cand;
  for (int t : {256, 512, 1024})
    for (int k : {2, 4, 8, 12, 16}) {
      JacobiPlan p = base;
      p.threads = t;
      p.chunk = k;
      p.lds = jacobi_lds_layout(b.max_nao, base.elt, k, t / 64).total;
      if ((int)p.lds > lds_max) continue;
      if (t / 64 > 16) continue;
      cand.push_back(p);
    }
  JacobiPlan best = base;
  float best_ms = 1e30f;
  hipEvent_t e0, e1;
  check(hipEventCreate(&e0), "event");
  check(hipEventCreate(&e1), "event");
  for (const JacobiPlan& p : cand) {
    check(hipMemcpyAsync(A1.p, A0.p, sizeof(double) * tm, hipMemcpyDeviceToDevice, stream), "copy");
    check(hipMemcpyAsync(V1.p, V0.p, sizeof(double) * tm, hipMemcpyDeviceToDevice, stream), "copy");
    check(hipEventRecord(e0, stream), "event");
    if (p.elt == 8)
      hipLaunchKernelGGL(k_jacobi_lds<double>, dim3(na), dim3(p.threads), p.lds, stream, db, dl, jacobi_max_sweeps,
                         jacobi_tol, jacobi_thr_scale, cap, sw.p, p.chunk);
    else
      hipLaunchKernelGGL(k_jacobi_lds<float>, dim3(na), dim3(p.threads), p.lds, stream, db, dl, jacobi_max_sweeps,
                         jacobi_tol, jacobi_thr_scale, cap, sw.p, p.chunk);
    check(hipEventRecord(e1, stream), "event");
    check(hipGetLastError(), "autotune launch");
    check(hipEventSynchronize(e1), "event");
    float ms = 0.0f;
    check(hipEventElapsedTime(&ms, e0, e1), "event");
    if (verbose)
      std::fprintf(stderr, "[fx] autotune n<=%d %s: %d threads, chunk %d: %.3f ms\n", b.max_nao,
                   p.elt == 8 ? "fp64" : "fp32", p.threads, p.chunk, ms);
    if (ms < best_ms) {
      best_ms = ms;
      best = p;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

// Eigensolver for a batch whose largest system has n AOs: the LDS-resident
// kernel with an FP64 working matrix if it fits with a rotation log of at
// least 4 steps, else with an FP32 working matrix, else the global-memory
// kernel.  Workgroup size grows with n (one V column per wave).
JacobiPlan Ctx::jacobi_plan(int n, bool fp64_only, bool prefer_fp32) const {
  JacobiPlan jp;
  if (!jacobi_lds || n < 2 || n > MAXN) return jp;
  int t = n <= 32 ? 64 : n <= 96 ? 256 : n <= 160 ? 512 : 1024;
  if (const char* e = std::getenv("FX_JACOBI_LDS_THREADS")) t = std::atoi(e);
  const int chunks[] = {16, 8, 4, 2};
  for (int pass = 0; pass < 2; ++pass)
    for (int elt : {prefer_fp32 ? 4 : 8, prefer_fp32 ? 8 : 4})
      for (int k : chunks) {
        if (fp64_only && elt == 4) continue;
        if (pass == 0 && k < 4) continue;
        const unsigned bytes = jacobi_lds_layout(n, elt, k, t / 64).total;
        if ((int)bytes <= lds_max) {
          jp.elt = elt;
          jp.chunk = k;
          jp.threads = t;
          jp.lds = bytes;
          return jp;
        }
      }
  return jp;
}

// Eigenpairs of symmetric matrices with the eigensolver of the SCC: the
// LDS-resident Jacobi of a cold solve, run to convergence, then one
// iteration of the form every later SCC iteration runs (A' = V A V^T rebuilt
// in FP64 on the matrix cores, the rotation kernel on the LDS working matrix,
// the apply kernel on V); sizes without an LDS plan use the global-memory
// kernel.  Eigenvalues unsorted, eigenvectors as rows of V.
void Ctx::eigh_hot(const std::vector<int>& nv, const double* A, double* w, double* V, bool global_kernel) {
  const int nmat = (int)nv.size();
  Batch b;
  b.nsys = nmat;
  b.h_desc.resize(nmat);
  long long mat = 0, ao = 0;
  std::vector<long long> off(nmat), woff(nmat);
  for (int k = 0; k < nmat; ++k) {
    SysDesc& d = b.h_desc[k];
    d = SysDesc{};
    d.nao = nv[k];
    d.mat_off = mat;
    d.ao_off = (int)ao;
    for (int f = 0; f < 3; ++f) d.frag[f] = -1;
    off[k] = mat;
    woff[k] = ao;
    mat += (long long)nv[k] * nv[k];
    ao += nv[k];
    b.max_nao = std::max(b.max_nao, nv[k]);
  }
  b.tot_mat = mat;
  b.tot_ao = (int)ao;
  b.d_desc.upload(b.h_desc);
  std::vector<double> hA(A, A + mat), hI(mat, 0.0);
  for (int k = 0; k < nmat; ++k)
    for (int i = 0; i < nv[k]; ++i) hI[off[k] + (long long)i * nv[k] + i] = 1.0;
  b.Pm.upload(hA);  // the input, kept for the rebuild
  b.Fm.upload(hA);
  b.Ct.upload(hI);
  b.Tm.alloc(mat);
  b.eps.alloc(ao);
  b.status.upload(std::vector<int>(nmat, 0));
  b.err.upload(std::vector<double>(nmat, 0.0));
  b.sweeps.alloc(nmat);
  std::vector<int> all(nmat);
  for (int k = 0; k < nmat; ++k) all[k] = k;
  b.d_list.upload(all);
  DevBatch db = b.dev();
  const JacobiPlan jp = global_kernel ? JacobiPlan{} : jacobi_plan(b.max_nao, false, false);
  if (jp.elt == 0) {
    DevBuf<int> dn;
    dn.upload(nv);
    DevBuf<long long> doff, dwoff;
    doff.upload(off);
    dwoff.upload(woff);
    hipLaunchKernelGGL(k_eigh_batched, dim3(nmat), dim3(256), 0, stream, dn.p, doff.p, b.Fm.p, b.Ct.p, b.eps.p,
                       dwoff.p, 60, 1e-15);
    check(hipGetLastError(), "k_eigh_batched");
  } else {
    if (jp.elt == 8)
      hipLaunchKernelGGL(k_jacobi_lds<double>, dim3(nmat), dim3(jp.threads), jp.lds, stream, db, b.d_list.p,
                         jacobi_max_sweeps, jacobi_tol, jacobi_thr_scale, 1e300, b.sweeps.p, jp.chunk);
    else
      hipLaunchKernelGGL(k_jacobi_lds<float>, dim3(nmat), dim3(jp.threads), jp.lds, stream, db, b.d_list.p,
                         jacobi_max_sweeps, jacobi_tol, jacobi_thr_scale, 1e300, b.sweeps.p, jp.chunk);
    check(hipGetLastError(), "cold eigensolver");
    // the warm iteration: A' = V A V^T (FP64), then rotations and their
    // application to V
    gemm_batch(b, db, nmat, b.d_list.p, 0, b.Ct.p, b.Pm.p, b.Tm.p, nullptr, b.gemm_gflop(all), 0);
    gemm_batch(b, db, nmat, b.d_list.p, 1, b.Tm.p, b.Ct.p, b.Fm.p, nullptr, b.gemm_gflop_sym(all), 0, 1);
    const int m4 = (b.max_nao + 3) & ~3;
    const bool split_ok = (long long)apply_rot_lds_bytes(b.max_nao) <= lds_max &&
                          (int)jacobi_rot_layout(b.max_nao, jp.elt).total <= lds_max &&
                          8 * m4 <= 2 * 64 * apply_rot_waves(b.max_nao);
    if (split_ok) {
      const long long log_stride = (long long)jacobi_max_log * jacobi_rot_log_entries(b.max_nao);
      b.rotlog.alloc((long long)nmat * log_stride);
      b.nlog.alloc(nmat);
      const unsigned lds_rot = jacobi_rot_layout(b.max_nao, jp.elt).total;
      (void)lds_rot;
      launch_rot(b, db, b.d_list.p, nmat, jp.elt, jacobi_cap_err, RotShape{jp.threads, false}, log_stride);
      launch_apply(b, db, b.d_list.p, nmat, log_stride);
    } else if (jp.elt == 8) {
      hipLaunchKernelGGL(k_jacobi_lds<double>, dim3(nmat), dim3(jp.threads), jp.lds, stream, db, b.d_list.p,
                         jacobi_max_sweeps, jacobi_tol, jacobi_thr_scale, jacobi_cap_err, b.sweeps.p, jp.chunk);
    } else {
      hipLaunchKernelGGL(k_jacobi_lds<float>, dim3(nmat), dim3(jp.threads), jp.lds, stream, db, b.d_list.p,
                         jacobi_max_sweeps, jacobi_tol, jacobi_thr_scale, jacobi_cap_err, b.sweeps.p, jp.chunk);
    }
    check(hipGetLastError(), "warm eigensolver iteration");
  }
  b.eps.download_raw(w, ao, stream);
  b.Ct.download_raw(V, mat, stream);
  sync();
}

void Ctx::build_matrices(Batch& b, bool from_mono) {
  if (b.has_hop) b.Vh.alloc(std::max(1LL, b.tot_mat));
  DevBatch db = b.dev();
  // clusters of a system without cut bonds copy their monomers' blocks (the
  // monomer batch holds this geometry's matrices)
  const int copy = from_mono && bonds.empty() && b.h_nfrag > 1 ? 1 : 0;
  hipLaunchKernelGGL(k_build_system, dim3(b.nsys), dim3(256), 0, stream, dev_system(), db, nullptr, mb.dev(), copy);
  if (b.has_hop) hipLaunchKernelGGL(k_vhop, dim3(b.nsys), dim3(256), 0, stream, db, P.g.VHOP);
  check(hipGetLastError(), "k_build_system");
  // mixed precision: FP32 copies of H0 and S for the FP32 Fock builds
  b.has_f32 = opt.precision == FX_MIXED && !b.has_hop && b.max_nao > 32;
  if (b.has_f32) {
    const long long m = std::max(1LL, b.tot_mat);
    b.H0f.alloc(m);
    b.Sf.alloc(m);
    b.Ff.alloc(m);
    b.Tf.alloc(m);
    const unsigned g = (unsigned)std::min<long long>(65536, (m + 255) / 256);
    hipLaunchKernelGGL(k_to_f32, dim3(g), dim3(256), 0, stream, (const double*)b.H0.p, b.H0f.p, b.tot_mat);
    hipLaunchKernelGGL(k_to_f32, dim3(g), dim3(256), 0, stream, (const double*)b.S.p, b.Sf.p, b.tot_mat);
    check(hipGetLastError(), "k_to_f32");
  }
}

// SCC for the systems in `list` (indices into the batch).  q_in must hold the
// initial charges; `cold` builds the first basis from the Cholesky factor of S,
// otherwise the eigenvectors of the previous solve are reused.
// Returns the number of systems that failed to converge.
// single: exactly one iteration (no mixing, no convergence test), used by
// the fused monomer loop; the previous residual is kept for the eigensolver.
int Ctx::run_scc(Batch& b, const std::vector<int>& list, bool cold, long long* iters_out, bool single) {
  if (list.empty()) return 0;
  const double t_start = now_ms();
  DevBatch db = b.dev();
  DevSystem ds = dev_system();
  const int nl = (int)list.size();
  // reset per-system iteration state on the device
  b.d_list.upload(list);
  hipLaunchKernelGGL(k_reset_state, dim3((nl + 255) / 256), dim3(256), 0, stream, db, b.d_list.p, nl,
                     single ? 1 : 0);
  check(hipGetLastError(), "k_reset_state");
  if (cold) {
    const int nt = (b.max_nao + 31) / 32;
    // inverse Cholesky factor in LDS: FP64 where the packed triangle fits,
    // else FP32 followed by a third-order correction of the rows' S-norms
    // (H = Y S Y^T, C^T = (15 I - 10 H + 3 H^2) / 8 Y); the global-memory
    // kernel beyond that
    const double gf = b.gemm_gflop(list);
    const int chol_elt = (long long)cholinv_lds_bytes(b.max_nao, 8) <= lds_max   ? 8
                         : (long long)cholinv_lds_bytes(b.max_nao, 4) <= lds_max ? 4
                                                                                  : 0;
    const unsigned chol_lds = chol_elt ? (unsigned)cholinv_lds_bytes(b.max_nao, chol_elt) : 0;
    KernelTimer* kt_chol = kt(chol_elt == 8 ? "fx::k_cholinv_lds<double>"
                              : chol_elt == 4 ? "fx::k_cholinv_lds<float>" : "fx::k_cholinv");
    auto cholinv = [&](const double* A, double* X) {
      // factor and inverse: n^3 / 3 multiply-adds each
      const int ev = capturing ? -1 : timers.begin(stream);
      if (chol_elt == 8)
        hipLaunchKernelGGL(k_cholinv_lds<double>, dim3(nl), dim3(CHOL_THREADS_HOST), chol_lds, stream, db,
                           b.d_list.p, A, X);
      else if (chol_elt == 4)
        hipLaunchKernelGGL(k_cholinv_lds<float>, dim3(nl), dim3(CHOL_THREADS_HOST), chol_lds, stream, db,
                           b.d_list.p, A, X);
      else
        hipLaunchKernelGGL(k_cholinv, dim3(nl), dim3(256), 0, stream, db, b.d_list.p, A, b.Pm.p, X);
      if (!capturing) timers.end(stream, ev, kt_chol, gf / 3.0);
      check(hipGetLastError(), "k_cholinv");
    };
    // rows Y in Tm (approximately S-orthonormal) -> Ct
    auto refine_rows = [&]() {
      gemm_batch(b, db, nl, b.d_list.p, 0, b.Tm.p, b.S.p, b.Pm.p, (const double*)nullptr, gf);
      gemm_batch(b, db, nl, b.d_list.p, 1, b.Pm.p, b.Tm.p, b.Fm.p, (const double*)nullptr, gf, 0, 1);
      gemm_batch(b, db, nl, b.d_list.p, 1, b.Fm.p, b.Fm.p, b.Pm.p, (const double*)nullptr, gf, 0, 1);
      hipLaunchKernelGGL(k_ns_poly, dim3(8, nl), dim3(256), 0, stream, db, b.d_list.p, b.Fm.p, b.Pm.p);
      gemm_batch(b, db, nl, b.d_list.p, 0, b.Fm.p, b.Tm.p, b.Ct.p, (const double*)nullptr, gf);
    };
    if (b.init_from_mono && mb.nsys > 0) {
      // C0 = blockdiag(monomer C); G = C0^T S C0 = L L^T; C = C0 L^-T
      hipLaunchKernelGGL(k_cluster_init_ct, dim3(nl), dim3(256), 0, stream, db, b.d_list.p, mb.dev(),
                         b.has_warm ? (const long long*)b.warm_off.p : nullptr);
      // two-fragment clusters all started from their monomers: the factor
      // of I - X^T X (half the order) gives the same inverse factor, and
      // only the fragment-pair block X^T of G is formed
      bool block2 = chol_elt == 4 && !b.has_warm;
      int n1max = 0, n2max = 0;
      for (int k = 0; block2 && k < nl; ++k) {
        const SysDesc& sd = b.h_desc[list[k]];
        if (sd.nfrag != 2) {
          block2 = false;
          break;
        }
        const int n1 = mb.h_desc[sd.frag[0]].nao;
        n1max = std::max(n1max, n1);
        n2max = std::max(n2max, sd.nao - n1);
      }
      block2 = block2 && (long long)cholinv_block2_lds_bytes(n1max, n2max) <= lds_max;
      gemm_batch(b, db, nl, b.d_list.p, 0, b.Ct.p, b.S.p, b.Tm.p, (const double*)nullptr, gf, 0, 0, false,
                 block2 ? 1 : 0);
      gemm_batch(b, db, nl, b.d_list.p, 1, b.Tm.p, b.Ct.p, b.Fm.p, (const double*)nullptr, gf, 0, 1, false,
                 block2 ? 1 : 0);
      if (chol_elt == 0) {
        cholinv(b.Fm.p, b.Tm.p);  // (k_cholinv uses Pm as its workspace)
        gemm_batch(b, db, nl, b.d_list.p, 0, b.Tm.p, b.Ct.p, b.Fm.p, (const double*)nullptr, gf);
        check(hipMemcpyAsync(b.Ct.p, b.Fm.p, sizeof(double) * b.tot_mat, hipMemcpyDeviceToDevice, stream), "copy");
      } else {
        if (block2) {
          const int ev = capturing ? -1 : timers.begin(stream);
          hipLaunchKernelGGL(k_cholinv_block2, dim3(nl), dim3(CHOL_THREADS_HOST),
                             (unsigned)cholinv_block2_lds_bytes(n1max, n2max), stream, db, b.d_list.p, mb.dev(),
                             (const double*)b.Fm.p, b.Pm.p);
          // the factor and inverse of the n/2 block plus the two n/2 products: about n^3 / 6
          double g2 = 0.0;
          for (int k = 0; k < nl; ++k) g2 += 1e-9 * std::pow((double)b.h_desc[list[k]].nao, 3) / 6.0;
          if (!capturing) timers.end(stream, ev, kt("fx::k_cholinv_block2"), g2);
          check(hipGetLastError(), "k_cholinv_block2");
        } else {
          cholinv(b.Fm.p, b.Pm.p);
        }
        gemm_batch(b, db, nl, b.d_list.p, 0, b.Pm.p, b.Ct.p, b.Tm.p, (const double*)nullptr, gf);
        if (chol_elt == 4)
          refine_rows();
        else
          check(hipMemcpyAsync(b.Ct.p, b.Tm.p, sizeof(double) * b.tot_mat, hipMemcpyDeviceToDevice, stream),
                "copy");
      }
    } else if (chol_elt == 4) {
      cholinv(b.S.p, b.Tm.p);
      refine_rows();
    } else {
      cholinv(b.S.p, b.Ct.p);
    }
    check(hipGetLastError(), "initial basis");
  }
  JacobiPlan jp = jacobi_plan(b.max_nao, b.has_hop, false);
  {
    auto itp = tuned.find(jp_key(b.max_nao, jp.elt));
    if (itp != tuned.end()) jp = itp->second;
  }
  std::vector<int> active = list;
  std::vector<int> status(b.nsys), niter(b.nsys);
  DevBuf<int> d_act;
  KernelTimer* kt_jac = kt(jp.elt == 8 ? "fx::k_jacobi_lds<double>" : jp.elt == 4 ? "fx::k_jacobi_lds<float>"
                                                                                   : "fx::k_jacobi");
  const int max_it = single ? 1 : opt.max_iter + 1;
  // one SCC iteration over the systems in dl (na of them); converged systems
  // listed there return at once (device-side status)
  bool last_split = false;
  // split eigensolver: rotation log of up to jacobi_max_log sweeps per system
  const long long log_stride = (long long)jacobi_max_log * jacobi_rot_log_entries(b.max_nao);
  // (the apply kernel stages 8 rounds of (c, s), at most two entries per thread)
  const int m4 = (b.max_nao + 3) & ~3;
  const bool split_ok = jacobi_split && jp.elt != 0 && (long long)apply_rot_lds_bytes(b.max_nao) <= lds_max &&
                        (int)jacobi_rot_layout(b.max_nao, jp.elt).total <= lds_max &&
                        8 * m4 <= 2 * 64 * apply_rot_waves(b.max_nao);
  // cold solve by the split form (not in the mixed-precision form, whose
  // cold iteration builds only the FP32 Fock matrix)
  const bool cold_split = split_ok && jacobi_cold_log > 0 && cold && !b.init_from_mono && !(b.has_f32 && prod_mode != 0);
  const long long cold_stride = (long long)jacobi_cold_log * jacobi_rot_log_entries(b.max_nao);
  DevBuf<int> cold_list;
  if (split_ok) {
    b.rotlog.alloc((long long)b.nsys * (cold_split ? std::max(log_stride, cold_stride) : log_stride));
    b.nlog.alloc(b.nsys);
  }
  KernelTimer* kt_rot = kt(jp.elt == 8 ? "fx::k_jacobi_rot<double>" : "fx::k_jacobi_rot<float>");
  const int sym_A = jp.elt != 0 ? 2 : 1;
  KernelTimer* kt_app = kt(apply_dual(b.max_nao) ? "fx::k_apply_rot_dual" : "fx::k_apply_rot");
  // mixed precision: FP32 Fock build and FP32 matrix-core products for this
  // iteration (the basis, the rotation angles, the charges and the
  // convergence test stay FP64; a final solve's tolerance lies far below the
  // switch threshold, so its converged state comes from FP64 iterations).
  // Not with the captured graph, whose launches are fixed.
  const bool graph_mode = opt.schedule == FX_BATCHED_GRAPH && !single && !first_solve;
  const bool f32_ok = b.has_f32 && !graph_mode && prod_mode != 0;
  // per system: still in the FP32 phase (until its own SCC residual drops to
  // mixed_thr; its Anderson history is kept unless mixed_hist_reset is set)
  std::vector<char> is32(b.nsys, f32_ok ? 1 : 0);
  std::vector<int> switched;
  DevBuf<int> d_switched;
  // one SCC iteration over the na systems listed in dl, of which the first
  // n32 run the FP32 Fock build and products (mixed precision)
  auto launch_iteration = [&](const std::vector<int>& act, const int* dl, int na, int n32, double cap,
                              bool timed) {
    const int n64 = na - n32;
    const int* dl64 = dl + n32;
    const std::vector<int> a32(act.begin(), act.begin() + n32), a64(act.begin() + n32, act.end());
    if (n32 > 0) {
      hipLaunchKernelGGL(k_fock_f32, dim3(n32), dim3(256), 0, stream, ds, db, dl, (const float*)b.H0f.p,
                         (const float*)b.Sf.p, b.Ff.p);
      gemm_batch_f32(b, db, n32, dl, 0, b.Ct.p, b.Ff.p, b.Tf.p, nullptr, b.gemm_gflop(a32), 1, 0, false);
      gemm_batch_f32(b, db, n32, dl, 1, b.Tf.p, b.Ct.p, b.Fm.p, nullptr, b.gemm_gflop_sym(a32), 1, 1, false);
    }
    if (n64 > 0) {
      hipLaunchKernelGGL(k_fock, dim3(n64), dim3(256), 0, stream, ds, db, dl64);
      // A = C^T F C in the current basis, then Jacobi rotations
      gemm_batch(b, db, n64, dl64, 0, b.Ct.p, b.Fm.p, b.Tm.p, nullptr, b.gemm_gflop(a64), 1);
      // A = (C^T F) C is symmetric: upper tiles only, mirrored unless the
      // eigensolver is an LDS kernel (those read the upper triangle only)
      gemm_batch(b, db, n64, dl64, 1, b.Tm.p, b.Ct.p, b.Fm.p, nullptr, b.gemm_gflop_sym(a64), 1, sym_A);
    }
    if (split_ok && cap < 1e299) {
      const RotShape rs = rot_shape(b, db, dl, na, jp, cap, log_stride, timed);
      int ev = timed ? timers.begin(stream) : -1;
      launch_rot(b, db, dl, na, jp.elt, cap, rs, log_stride);
      if (timed) timers.end(stream, ev, kt_rot, 0.0);
      ev = timed ? timers.begin(stream) : -1;
      launch_apply(b, db, dl, na, log_stride);
      if (timed) timers.end(stream, ev, kt_app, 0.0);
      last_split = true;
    } else if (cold_split) {
      // passes of up to jacobi_cold_log sweeps; a system whose pass ended on
      // a sweep without rotations (fewer logged sweeps than the pass allows)
      // is done, the others start the next pass from C^T F C in the basis
      // this pass left (the Fock matrix is rebuilt: the products overwrite
      // it).  The launch shape is not tuned here but on a warm iteration.
      const RotShape rs = rot_shape(b, db, dl, na, jp, cap, cold_stride, false);
      std::vector<int> todo(na), nlog;
      check(hipMemcpyAsync(todo.data(), dl, sizeof(int) * na, hipMemcpyDeviceToHost, stream), "list copy");
      const int* dt = dl;
      const int max_pass = (jacobi_max_sweeps + jacobi_cold_log - 1) / jacobi_cold_log;
      for (int pass = 0; pass < max_pass && !todo.empty(); ++pass) {
        const int nt = (int)todo.size();
        if (pass > 0) {
          cold_list.upload(todo);
          dt = cold_list.p;
          hipLaunchKernelGGL(k_fock, dim3(nt), dim3(256), 0, stream, ds, db, dt);
          gemm_batch(b, db, nt, dt, 0, b.Ct.p, b.Fm.p, b.Tm.p, nullptr, 0.0, 1);
          gemm_batch(b, db, nt, dt, 1, b.Tm.p, b.Ct.p, b.Fm.p, nullptr, 0.0, 1, sym_A);
        }
        int ev = timed ? timers.begin(stream) : -1;
        launch_rot(b, db, dt, nt, jp.elt, cap, rs, cold_stride, jacobi_cold_log);
        if (timed) timers.end(stream, ev, kt_rot, 0.0);
        ev = timed ? timers.begin(stream) : -1;
        launch_apply(b, db, dt, nt, cold_stride);
        if (timed) timers.end(stream, ev, kt_app, 0.0);
        b.nlog.download(nlog, stream);
        sync();
        std::vector<int> next;
        for (int s : todo)
          if (nlog[s] >= jacobi_cold_log) next.push_back(s);
        todo.swap(next);
      }
      last_split = true;
    } else {
      last_split = false;
    const int ev = timed ? timers.begin(stream) : -1;
    if (jp.elt == 8)
      hipLaunchKernelGGL(k_jacobi_lds<double>, dim3(na), dim3(jp.threads), jp.lds, stream, db, dl, jacobi_max_sweeps,
                         jacobi_tol, jacobi_thr_scale, cap, b.sweeps.p, jp.chunk);
    else if (jp.elt == 4)
      hipLaunchKernelGGL(k_jacobi_lds<float>, dim3(na), dim3(jp.threads), jp.lds, stream, db, dl, jacobi_max_sweeps,
                         jacobi_tol, jacobi_thr_scale, cap, b.sweeps.p, jp.chunk);
    else
      hipLaunchKernelGGL(k_jacobi, dim3(na), dim3(jacobi_threads), 0, stream, db, dl, jacobi_max_sweeps, jacobi_tol,
                         jacobi_thr_scale, cap, b.sweeps.p);
    if (timed) timers.end(stream, ev, kt_jac, 0.0);
    }
    hipLaunchKernelGGL(k_fermi, dim3(na), dim3(256), 0, stream, ds, db, dl);
    if (n32 > 0)
      gemm_batch_f32(b, db, n32, dl, 2, b.Ct.p, b.Ct.p, b.Pm.p, b.occ.p, b.gemm_gflop_occ(a32), 1, 1, true);
    if (n64 > 0)
      // (the upper tiles only: the mixer reads those; the lower ones are
      // filled once the solve ends)
      gemm_batch(b, db, n64, dl64, 2, b.Ct.p, b.Ct.p, b.Pm.p, b.occ.p, b.gemm_gflop_occ(a64), 1, 2, true);
    // a system converges only in an FP64 iteration
    const double beta = b.has_pre ? precond_beta : mix_beta;
    if (n32 > 0)
      hipLaunchKernelGGL(k_charges_mix, dim3(n32), dim3(256), 0, stream, ds, db, dl, -1.0, -1.0,
                         single ? 1 : opt.max_iter, beta);
    if (n64 > 0)
      hipLaunchKernelGGL(k_charges_mix, dim3(n64), dim3(256), 0, stream, ds, db, dl64,
                         scc_tol_cur > 0 ? scc_tol_cur : opt.scc_tol, etol_cur > 0 ? etol_cur : opt.energy_tol,
                         single ? 1 : opt.max_iter, beta);
    check(hipGetLastError(), "scc iteration");
  };
  // FX_BATCHED_GRAPH: after the first (eager) iteration, the iteration over
  // the whole list is captured once into a hipGraph and replayed; converged
  // systems skip themselves on the device, the host only reads the status
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // device-driven form (the FP64 batched solves with the split eigensolver):
  // after each iteration k_compact_active rewrites d_act with the systems
  // still iterating first and copies their count to a pinned slot; the next
  // iteration is launched at once over ub slots, ub being the latest count
  // that has arrived (counts only fall, so ub bounds the true one, and the
  // converged systems in the slots beyond it return at once)
  const bool async = opt.schedule == FX_BATCHED && !single && !f32_ok && !verbose && split_ok;
  int ub = nl;
  std::deque<int> pending;
  const std::vector<int> no_list;
  if (async) {
    count_ring_init();
    d_act.alloc(nl);
    check(hipMemcpyAsync(d_act.p, b.d_list.p, sizeof(int) * nl, hipMemcpyDeviceToDevice, stream), "copy");
  }
  // launch shape of the fused LDS eigensolver, tuned once per size bucket on
  // the first iteration that runs it (the cold iteration of a solve from the
  // Cholesky basis when the split form is on, else the second iteration):
  // this iteration's A is formed once and every shape is timed on copies of
  // (A, C^T); all shapes give bitwise identical results
  auto want_tune = [&](int it) {
    if (!autotune || capturing || jp.elt == 0 || tuned.count(jp_key(b.max_nao, jp.elt))) return false;
    return split_ok ? (it == 0 && cold && !b.init_from_mono && !cold_split) : it == 1;
  };
  auto tune_fused = [&](const int* dl, int na, double cap) {
    hipLaunchKernelGGL(k_fock, dim3(na), dim3(256), 0, stream, ds, db, dl);
    gemm_batch(b, db, na, dl, 0, b.Ct.p, b.Fm.p, b.Tm.p, nullptr, 0.0, 1);
    gemm_batch(b, db, na, dl, 1, b.Tm.p, b.Ct.p, b.Fm.p, nullptr, 0.0, 1);
    jp = autotune_jacobi(b, dl, na, jp, cap);
    tuned[jp_key(b.max_nao, jp.elt)] = jp;
  };
  for (int it = 0; it < max_it && !active.empty(); ++it) {
    const double cap = (cold && it == 0 && !b.init_from_mono) ? 1e300 : jacobi_cap_err;
    if (graph_mode && it >= 1) {
      if (!gexec) {
        if (!gstream) check(hipStreamCreateWithFlags(&gstream, hipStreamNonBlocking), "hipStreamCreate");
        sync();
        hipStream_t saved = stream;
        stream = gstream;
        capturing = true;
        check(hipStreamBeginCapture(gstream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        launch_iteration(list, b.d_list.p, nl, 0, jacobi_cap_err, false);
        const hipError_t ec = hipStreamEndCapture(gstream, &graph);
        capturing = false;
        stream = saved;
        check(ec, "hipStreamEndCapture");
        check(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
      }
      const int ev = timers.begin(gstream);
      check(hipGraphLaunch(gexec, gstream), "hipGraphLaunch");
      timers.end(gstream, ev, kt("scc iteration (graph)"), 0.0);
      check(hipStreamSynchronize(gstream), "hipStreamSynchronize");
      b.status.download(status, stream);
      sync();
      timers.resolve();
      std::vector<int> next;
      for (int s : active)
        if (status[s] == 0) next.push_back(s);
      active.swap(next);
      continue;
    }
    if (async) {
      if (want_tune(it)) tune_fused(d_act.p, ub, cap);
      launch_iteration(no_list, d_act.p, ub, 0, cap, true);
      if (first_solve && it == 0) {
        // median first-iteration residual over the batch (all listed systems
        // took part in iteration 0)
        std::vector<double> e;
        b.err.download(e, stream);
        sync();
        std::vector<double> v;
        for (int s : list) v.push_back(e[s]);
        std::nth_element(v.begin(), v.begin() + v.size() / 2, v.end());
        res.first_residual_median = v[v.size() / 2];
      }
      if (first_solve && opt.guess == FX_GUESS_LEARNED &&
          ((it == 0 && opt.guess_tau > 0) || (opt.guess_max_iter > 0 && it + 1 == opt.guess_max_iter))) {
        hipLaunchKernelGGL(k_guess_fallback, dim3(ub), dim3(64), 0, stream, db, d_act.p, ub, it == 0 ? 0 : 1,
                           opt.guess_tau, fallback_flag.p);
        check(hipGetLastError(), "k_guess_fallback");
      }
      const int slot = it % CNT_RING;
      hipLaunchKernelGGL(k_compact_active, dim3(1), dim3(1024), 0, stream, (const int*)b.status.p,
                         (const int*)b.d_list.p, nl, d_act.p, cnt_dev.p + slot);
      check(hipGetLastError(), "k_compact_active");
      check(hipMemcpyAsync(cnt_host + slot, cnt_dev.p + slot, sizeof(int), hipMemcpyDeviceToHost, stream),
            "count copy");
      check(hipEventRecord(cnt_ev[slot], stream), "hipEventRecord");
      pending.push_back(slot);
      // take the counts that have arrived; block only when async_lag
      // iterations are already in flight behind the oldest one
      while (!pending.empty()) {
        const int k = pending.front();
        if ((int)pending.size() <= async_lag) {
          const hipError_t q = hipEventQuery(cnt_ev[k]);
          if (q == hipErrorNotReady) {
            (void)hipGetLastError();  // not an error: the copy is still queued
            break;
          }
          check(q, "hipEventQuery");
        } else {
          check(hipEventSynchronize(cnt_ev[k]), "hipEventSynchronize");
        }
        ub = std::min(ub, cnt_host[k]);
        pending.pop_front();
      }
      if (ub == 0) break;
      continue;
    }
    int n32 = 0;
    if (f32_ok) {
      std::vector<int> ordered;
      for (int s : active)
        if (is32[s]) ordered.push_back(s);
      n32 = (int)ordered.size();
      for (int s : active)
        if (!is32[s]) ordered.push_back(s);
      active.swap(ordered);
    }
    d_act.upload(active);
    const int na = (int)active.size();
    if (!switched.empty()) {
      d_switched.upload(switched);
      hipLaunchKernelGGL(k_hist_reset, dim3(((int)switched.size() + 255) / 256), dim3(256), 0, stream, db,
                         (const int*)d_switched.p, (int)switched.size());
      switched.clear();
    }
    if (want_tune(it)) tune_fused(d_act.p, na, cap);
    launch_iteration(active, d_act.p, na, n32, cap, true);
    res.iters_fp32 += n32;
    if (first_solve && it == 0) {
      // median first-iteration residual over the batch
      std::vector<double> e;
      b.err.download(e, stream);
      sync();
      std::vector<double> v;
      for (int s : active) v.push_back(e[s]);
      if (!v.empty()) {
        std::nth_element(v.begin(), v.begin() + v.size() / 2, v.end());
        res.first_residual_median = v[v.size() / 2];
      }
    }
    if (first_solve && opt.guess == FX_GUESS_LEARNED &&
        ((it == 0 && opt.guess_tau > 0) || (opt.guess_max_iter > 0 && it + 1 == opt.guess_max_iter))) {
      hipLaunchKernelGGL(k_guess_fallback, dim3(na), dim3(64), 0, stream, db, d_act.p, na, it == 0 ? 0 : 1,
                         opt.guess_tau, fallback_flag.p);
      check(hipGetLastError(), "k_guess_fallback");
    }
    b.status.download(status, stream);
    std::vector<double> errs;
    if ((n32 > 0 && prod_mode == 1) || verbose) b.err.download(errs, stream);
    sync();
    timers.resolve();
    // algorithmic work of the eigensolve of one SCC iteration, as budgeted
    // for a dense symmetric eigensolver: 3.3 n^3 (reduction about 1.3 n^3,
    // back-transformation of the eigenvectors 2 n^3), whatever the Jacobi
    // sweeps actually did; the split form credits the rotation kernel with
    // the first and the apply kernel with the second
    for (int s : active) {
      const double n = b.h_desc[s].nao, n3 = 1e-9 * n * n * n;
      if (last_split) {
        kt_rot->gflop += 1.3 * n3;
        kt_app->gflop += 2.0 * n3;
      } else {
        kt_jac->gflop += 3.3 * n3;
      }
    }
    if (verbose) {
      double emax = 0.0, emed = 0.0;
      std::vector<double> ev;
      for (int s : active) {
        emax = std::max(emax, errs[s]);
        ev.push_back(errs[s]);
      }
      if (!ev.empty()) {
        std::nth_element(ev.begin(), ev.begin() + ev.size() / 2, ev.end());
        emed = ev[ev.size() / 2];
      }
      std::fprintf(stderr, "[fx]   iteration %d: %d systems (%d fp32), residual max %.2e median %.2e\n", it,
                   (int)active.size(), n32, emax, emed);
    }
    std::vector<int> next;
    for (int s : active)
      if (status[s] == 0) next.push_back(s);
    const std::vector<int> active_prev = active;
    active.swap(next);
    if (n32 > 0 && prod_mode == 1) {
      for (int k = 0; k < n32; ++k) {
        const int s = active_prev[k];
        if (status[s] == 0 && errs[s] <= mixed_thr) {
          is32[s] = 0;
          if (mixed_hist_reset) switched.push_back(s);
        }
      }
    }
  }
  if (gexec) (void)hipGraphExecDestroy(gexec);
  if (graph) (void)hipGraphDestroy(graph);
  // the density's lower tiles (the iterations write the upper ones)
  if (b.max_nao > 64) {
    hipLaunchKernelGGL(k_mirror_tiles, dim3(nl), dim3(256), 0, stream, db, (const int*)b.d_list.p, b.Pm.p);
    check(hipGetLastError(), "k_mirror_tiles");
  }
  b.status.download(status, stream);
  b.niter.download(niter, stream);
  sync();
  if (async) {
    timers.resolve();
    // algorithmic work from the per-system iteration counts (the launches
    // were timed without it): the eigensolver as in the host-driven form,
    // the products by the forms each iteration runs
    KernelTimer* kt_g = kt(b.max_nao <= 32 ? "fx::k_gemm" : "fx::k_gemm_mfma");
    const bool cold_full = cold && !b.init_from_mono;
    for (int s : list) {
      const int its = niter[s];
      if (its <= 0) continue;
      const int n_full = cold_full ? 1 : 0, n_split = its - n_full;
      const double n = b.h_desc[s].nao, n3 = 1e-9 * n * n * n;
      kt_jac->gflop += 3.3 * n3 * n_full;
      kt_rot->gflop += 1.3 * n3 * n_split;
      kt_app->gflop += 2.0 * n3 * n_split;
      const std::vector<int> one{s};
      kt_g->gflop += its * (b.gemm_gflop(one) + b.gemm_gflop_sym(one) + b.gemm_gflop_occ(one));
    }
  }
  if (verbose) {
    long long tot = 0;
    int mx = 0;
    for (int s : list) {
      tot += niter[s];
      mx = std::max(mx, niter[s]);
    }
    std::fprintf(stderr,
                 "[fx] scc batch of %d systems (nao<=%d): %lld iterations, max %d, %.1f ms "
                 "(eigensolver: %s, chunk %d, %d threads, %u B LDS)\n",
                 nl, b.max_nao, tot, mx, now_ms() - t_start,
                 jp.elt == 8 ? "lds-fp64" : jp.elt == 4 ? "lds-fp32" : "global", jp.chunk, jp.threads, jp.lds);
  }
  int failed = 0;
  long long iters = 0;
  for (int s : list) {
    if (status[s] != 1) ++failed;
    iters += niter[s];
  }
  if (iters_out) *iters_out += iters;
  return single ? 0 : failed;
}

// The rotation kernel over the na systems listed in dl, one work-group per
// system or a persistent grid over a work queue (rs.persistent: as many
// work-groups as fit on the device at once, fed by an atomic counter)
void Ctx::launch_rot(const Batch& b, const DevBatch& db, const int* dl, int na, int elt, double cap,
                     const RotShape& rs, long long log_stride, int max_log) {
  const int ml = max_log > 0 ? max_log : jacobi_max_log;
  const unsigned lds_rot = jacobi_rot_layout(b.max_nao, elt).total;
  const void* fn = elt == 8 ? reinterpret_cast<const void*>(k_jacobi_rot<double>)
                            : reinterpret_cast<const void*>(k_jacobi_rot<float>);
  int grid = na, nl = 0;
  int* queue = nullptr;
  if (rs.persistent) {
    int per_cu = 0;
    check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, rs.threads, lds_rot), "occupancy query");
    grid = std::min(na, std::max(1, per_cu) * std::max(1, n_cu));
    if (rot_queue.n < 1) rot_queue.alloc(1);
    queue = rot_queue.p;
    nl = na;
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, stream, queue);
  }
  // (monomers start each solve from exact eigenvectors: one sweep)
  const int es = std::min(jacobi_early_sweeps, ml);
  const double ee = b.init_from_mono ? jacobi_early_err : 1e300;
  if (elt == 8)
    hipLaunchKernelGGL(k_jacobi_rot<double>, dim3(grid), dim3(rs.threads), lds_rot, stream, db, dl, jacobi_max_sweeps,
                       jacobi_tol, jacobi_thr_scale, cap, ee, es, b.sweeps.p, b.rotlog.p, log_stride, ml, b.nlog.p,
                       queue, nl);
  else
    hipLaunchKernelGGL(k_jacobi_rot<float>, dim3(grid), dim3(rs.threads), lds_rot, stream, db, dl, jacobi_max_sweeps,
                       jacobi_tol, jacobi_thr_scale, cap, ee, es, b.sweeps.p, b.rotlog.p, log_stride, ml, b.nlog.p,
                       queue, nl);
  check(hipGetLastError(), "k_jacobi_rot");
}

// The apply kernel over the na systems listed in dl: two quartets per lane
// for systems of 129 to 256 AOs, one otherwise
void Ctx::launch_apply(const Batch& b, const DevBatch& db, const int* dl, int na, long long log_stride) {
  if (apply_dual(b.max_nao)) {
    const int tps = (b.max_nao + 63) / 64;
    const long long grid = xcd_grid(na, tps);
    hipLaunchKernelGGL(k_apply_rot_dual, dim3((unsigned)grid), dim3(512), (unsigned)apply_rot_dual_lds_bytes(b.max_nao),
                       stream, db, dl, na, tps, (const double2*)b.rotlog.p, log_stride, (const int*)b.nlog.p);
  } else {
    const int tw = apply_rot_tile(b.max_nao);
    const int tps = (b.max_nao + tw - 1) / tw;
    const long long grid = xcd_grid(na, tps);
    hipLaunchKernelGGL(k_apply_rot, dim3((unsigned)grid), dim3(64 * apply_rot_waves(b.max_nao)),
                       (unsigned)apply_rot_lds_bytes(b.max_nao), stream, db, dl, na, tps, tw,
                       (const double2*)b.rotlog.p, log_stride, (const int*)b.nlog.p);
  }
  check(hipGetLastError(), "apply kernel");
}

// Launch shape of the rotation kernel for this size bucket: forced by the
// environment, tuned once per bucket by timing every candidate on the
// current iteration's input (the kernel only reads the working matrix, and
// every shape writes bitwise the same log and eigenvalues, so the timing
// launches change nothing), or the plan's default when tuning is off
Ctx::RotShape Ctx::rot_shape(Batch& b, const DevBatch& db, const int* dl, int na, const JacobiPlan& jp, double cap,
                             long long log_stride, bool may_tune) {
  RotShape def{jp.threads, false};
  if (force_rot_threads > 0 || force_rot_persistent >= 0) {
    RotShape f = def;
    if (force_rot_threads > 0) f.threads = force_rot_threads;
    if (force_rot_persistent >= 0) f.persistent = force_rot_persistent != 0;
    return f;
  }
  const long long key = jp_key(b.max_nao, jp.elt);
  auto it = tuned_rot.find(key);
  if (it != tuned_rot.end()) return it->second;
  if (!autotune || !may_tune || capturing) return def;
  hipEvent_t e0, e1;
  check(hipEventCreate(&e0), "event");
  check(hipEventCreate(&e1), "event");
  RotShape best = def;
  float best_ms = 1e30f;
  for (int t : {256, 512, 768, 1024})
    for (int p = 0; p < 2; ++p) {
      const RotShape c{t, p != 0};
      check(hipEventRecord(e0, stream), "event");
      launch_rot(b, db, dl, na, jp.elt, cap, c, log_stride);
      check(hipEventRecord(e1, stream), "event");
      check(hipEventSynchronize(e1), "event");
      float ms = 0.0f;
      check(hipEventElapsedTime(&ms, e0, e1), "event");
      if (verbose)
        std::fprintf(stderr, "[fx] autotune rotation kernel n<=%d: %d threads%s: %.3f ms\n", b.max_nao, t,
                     p ? " persistent" : "", ms);
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  tuned_rot[key] = best;
  return best;
}

void Ctx::count_ring_init() {
  if (cnt_host) return;
  if (cnt_dev.n < CNT_RING) cnt_dev.alloc(CNT_RING);
  cnt_ev.assign(CNT_RING, nullptr);
  for (auto& e : cnt_ev) check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
  check(hipHostMalloc((void**)&cnt_host, sizeof(int) * CNT_RING, hipHostMallocDefault), "hipHostMalloc");
}

// Automatic retry of the systems of a cluster batch whose SCC did not
// converge: from where each solve stopped, first with plain Anderson mixing
// of the raw residual (no Newton preconditioner) and a damping of 0.2, then,
// for those still unconverged, at a tenfold electronic temperature followed
// by a warm solve at the nominal one.  Products in FP64 throughout (the
// caller has left the mixed form).  Returns the number still unconverged.
int Ctx::retry_failed(Batch& b, long long* iters_out) {
  auto unconverged = [&]() {
    std::vector<int> st, l;
    b.status.download(st, stream);
    sync();
    for (int s = 0; s < b.nsys; ++s)
      if (st[s] != 1) l.push_back(s);
    return l;
  };
  std::vector<int> fail = unconverged();
  if (fail.empty()) return 0;
  res.scc_retries += (long long)fail.size();
  const int max_iter0 = opt.max_iter;
  const int cap = std::max(opt.max_iter, 200);
  opt.max_iter = retry_damped_iters > 0 ? retry_damped_iters : cap;
  const bool pre = b.has_pre;
  const double beta = mix_beta;
  b.has_pre = false;
  mix_beta = 0.2;
  int left = run_scc(b, fail, false, iters_out);
  b.has_pre = pre;
  mix_beta = beta;
  opt.max_iter = cap;
  if (left) {
    fail = unconverged();
    const double kT = P.g.kT;
    P.g.kT = 10.0 * kT;
    (void)run_scc(b, fail, false, iters_out);
    P.g.kT = kT;
    left = run_scc(b, fail, false, iters_out);
  }
  opt.max_iter = max_iter0;
  if (verbose) std::fprintf(stderr, "[fx] scc retry: %d systems still unconverged\n", left);
  return left;
}

// solve a batch either all at once or one system at a time
int Ctx::solve_batch(Batch& b, bool cold, long long* iters_out) {
  int failed = 0;
  if (opt.schedule == FX_PLAIN_LOOP) {
    for (int s = 0; s < b.nsys; ++s) failed += run_scc(b, std::vector<int>{s}, cold, iters_out);
  } else {
    std::vector<int> all(b.nsys);
    for (int s = 0; s < b.nsys; ++s) all[s] = s;
    failed += run_scc(b, all, cold, iters_out);
  }
  return failed;
}

void Ctx::max_absdiff(const double* a, const double* b, int n, double* out) {
  const int np = std::max(1, std::min(64, (n + 2047) / 2048));
  if (red_part.n < 64LL * 36) red_part.alloc(64LL * 36);
  hipLaunchKernelGGL(k_absdiff_part, dim3(np), dim3(256), 0, stream, a, b, n, red_part.p);
  hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, stream, red_part.p, np, out);
}

void Ctx::hist_coef(const double* R, long long n, const Slots& sl, double* coef) {
  const int np = (int)std::max(1LL, std::min(64LL, (n + 2047) / 2048));
  if (red_part.n < 64LL * 36) red_part.alloc(64LL * 36);  // 64 partials of HIST (HIST + 1) / 2 = 36
  hipLaunchKernelGGL(k_hist_gram_part, dim3(np), dim3(256), 0, stream, R, n, sl, red_part.p);
  hipLaunchKernelGGL(k_hist_solve, dim3(1), dim3(64), 0, stream, red_part.p, np, sl, coef);
}

void Ctx::field(const double* d_q, double* d_phi, bool fp32) {
  const DevSystem ds = dev_system();
  const int nbk = (Ne + 63) / 64;
  const long long ncol = (long long)nbk * (nbk - 1) / 2 * 128;
  if (!fp32 && ds.g.kg == 2.0 && ncol <= (1LL << 29)) {
    // symmetric pass: each inter-fragment atom pair once (4 source blocks per wave)
    const int group = 4, ngmax = (nbk + group - 1) / group;
    const long long nrow = (long long)nbk * ngmax * 128;
    if (nrow > field_part.n) field_part.alloc(nrow);
    if (ncol > field_col.n) field_col.alloc(std::max(1LL, ncol));
    const int ev = timers.begin(stream);
    hipLaunchKernelGGL(k_field_sym, dim3(nbk, ngmax), dim3(64), 0, stream, ds, d_q, group, ngmax, field_part.p,
                       field_col.p);
    timers.end(stream, ev, kt("fx::k_field_sym"), 8e-9 * field_pairs);
    hipLaunchKernelGGL(k_field_sym_reduce, dim3((Ne + 255) / 256), dim3(256), 0, stream, ds, group, ngmax,
                       (const double*)field_part.p, (const double*)field_col.p, d_phi);
    check(hipGetLastError(), "field");
    return;
  }
  const int nchunk = std::max(1, std::min(64, (Ne + 255) / 256 > 0 ? 2048 / ((Ne + 255) / 256) : 1));
  if ((long long)nchunk * Nsh > field_part.n) field_part.alloc((long long)nchunk * Nsh);
  dim3 grid((Ne + 255) / 256, nchunk);
  const int ev = timers.begin(stream);
  if (fp32) {
    hipLaunchKernelGGL(k_field_partial_f32, grid, dim3(256), 0, stream, dev_system(), d_q, nchunk, field_part.p);
    timers.end(stream, ev, kt("fx::k_field_partial_f32"), 8e-9 * field_pairs);
  } else {
    hipLaunchKernelGGL(k_field_partial, grid, dim3(256), 0, stream, dev_system(), d_q, nchunk, field_part.p);
    timers.end(stream, ev, kt("fx::k_field_partial"), 8e-9 * field_pairs);
  }
  hipLaunchKernelGGL(k_field_reduce, dim3((Nsh + 255) / 256), dim3(256), 0, stream, Nsh, nchunk, field_part.p,
                     d_phi);
  check(hipGetLastError(), "field");
}

void Ctx::compute_cn() {
  const int gA = (N + 255) / 256;
  const int nchunk = std::max(1, std::min(64, 2048 / std::max(1, gA)));
  if ((long long)nchunk * N > field_part.n) field_part.alloc((long long)nchunk * N);
  hipLaunchKernelGGL(k_cn, dim3(gA, nchunk), dim3(256), 0, stream, dev_system(), nchunk, field_part.p);
  hipLaunchKernelGGL(k_field_reduce, dim3(gA), dim3(256), 0, stream, N, nchunk, field_part.p, d_cn.p);
  if (NB > 0)
    hipLaunchKernelGGL(k_ghost_cn, dim3((NB + 255) / 256), dim3(256), 0, stream, dev_system(), d_bonds.p, NB, d_cn.p);
  check(hipGetLastError(), "k_cn");
}

void Ctx::build_lists_impl() {
  const long long npair = (long long)F * (F - 1) / 2;
  DevBuf<int8_t> flag;
  flag.alloc(std::max(1LL, npair));
  const bool vdw = opt.selection == FX_SELECT_VDW;
  if (vdw)
    for (int a = 0; a < N; ++a)
      if (!(P.elems[elem[a]].rvdw > 0.0))
        throw FxError(FX_E_UNSUPPORTED, "van der Waals radius missing from the parameters");
  if (F > 1) {
    hipLaunchKernelGGL(k_pair_contacts, dim3(F), dim3(256), 0, stream, dev_system(), d_frag_atoms_real.p,
                       d_frag_off_real.p, vdw ? 1 : 0, opt.cutoff_bohr * opt.cutoff_bohr, opt.vdw_dimer,
                       opt.vdw_trimer, flag.p);
    check(hipGetLastError(), "k_pair_contacts");
  }
  std::vector<int8_t> h(npair);
  if (npair) flag.download(h, stream);
  sync();
  scc_pairs.clear();
  esd_pairs.clear();
  trimers.clear();
  // flag bit 0: SCC dimer; bit 1: the pair counts for the trimer rule
  std::vector<std::vector<int>> nb(F);
  long long k = 0;
  for (int I = 0; I < F; ++I)
    for (int J = I + 1; J < F; ++J, ++k) {
      if (h[k] & 2) {
        nb[I].push_back(J);
        nb[J].push_back(I);
      }
      if (h[k] & 1) {
        scc_pairs.push_back(I);
        scc_pairs.push_back(J);
      } else {
        esd_pairs.push_back(I);
        esd_pairs.push_back(J);
      }
    }
  if (opt.order >= 3) {
    // trimers I<J<K with at least two sub-pairs meeting the trimer rule: every
    // such trimer has a fragment adjacent to both others; enumerate candidates
    // from neighbour lists
    std::vector<std::vector<char>> adj;
    auto near = [&](int a, int b) {
      const std::vector<int>& v = nb[a];
      return std::binary_search(v.begin(), v.end(), b);
    };
    for (auto& v : nb) std::sort(v.begin(), v.end());
    std::vector<std::array<int, 3>> tri;
    for (int c = 0; c < F; ++c) {
      const std::vector<int>& v = nb[c];
      for (size_t x = 0; x < v.size(); ++x)
        for (size_t y = x + 1; y < v.size(); ++y) {
          std::array<int, 3> t = {c, v[x], v[y]};
          std::sort(t.begin(), t.end());
          tri.push_back(t);
        }
    }
    std::sort(tri.begin(), tri.end());
    tri.erase(std::unique(tri.begin(), tri.end()), tri.end());
    for (auto& t : tri) {
      int cnt = (int)near(t[0], t[1]) + (int)near(t[0], t[2]) + (int)near(t[1], t[2]);
      if (cnt >= 2) {
        trimers.push_back(t[0]);
        trimers.push_back(t[1]);
        trimers.push_back(t[2]);
      }
    }
  }
  lists_built = true;
}

void Ctx::set_system(int32_t n_atoms, const int32_t* Z, const double* xyz, int32_t n_frag, const int32_t* atom_frag,
                     const int32_t* fchg, int32_t n_bonds, const int32_t* bonds_in) {
  if (n_atoms <= 0 || n_frag <= 0 || !Z || !xyz || !atom_frag || !fchg) throw FxError(FX_E_INVALID, "bad system");
  if (n_bonds < 0 || (n_bonds > 0 && !bonds_in)) throw FxError(FX_E_INVALID, "bad bond list");
  has_system = false;
  ++system_gen;
  N = n_atoms;
  F = n_frag;
  elem.assign(N, 0);
  frag.assign(atom_frag, atom_frag + N);
  frag_charge.assign(fchg, fchg + F);
  xyz_h.assign(xyz, xyz + 3 * N);
  for (int A = 0; A < N; ++A) {
    auto it = P.elem_of_Z.find(Z[A]);
    if (it == P.elem_of_Z.end()) throw FxError(FX_E_UNSUPPORTED, "no parameters for Z=" + std::to_string(Z[A]));
    elem[A] = it->second;
    if (frag[A] < 0 || frag[A] >= F) throw FxError(FX_E_INVALID, "atom fragment index out of range");
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(xyz[3 * A + k])) throw FxError(FX_E_INVALID, "non-finite coordinate");
  }
  // atoms closer than 0.3 bohr (cell grid)
  {
    const double cs = 2.0;
    std::map<std::array<long long, 3>, std::vector<int>> grid;
    for (int A = 0; A < N; ++A) {
      std::array<long long, 3> key = {(long long)std::floor(xyz[3 * A] / cs), (long long)std::floor(xyz[3 * A + 1] / cs),
                                      (long long)std::floor(xyz[3 * A + 2] / cs)};
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            auto it = grid.find({key[0] + dx, key[1] + dy, key[2] + dz});
            if (it == grid.end()) continue;
            for (int B : it->second) {
              double r2 = 0.0;
              for (int k = 0; k < 3; ++k) r2 += (xyz[3 * A + k] - xyz[3 * B + k]) * (xyz[3 * A + k] - xyz[3 * B + k]);
              if (r2 < 0.09) throw FxError(FX_E_INVALID, "atoms closer than 0.3 bohr");
            }
          }
      grid[key].push_back(A);
    }
  }
  // covalent boundaries: detached atom (stays in its fragment) and attached
  // atom; one ghost atom per bond joins the attached atom's fragment
  NB = n_bonds;
  bonds.clear();
  if (NB > 0) bonds.assign(bonds_in, bonds_in + 2 * NB);
  for (int k = 0; k < NB; ++k) {
    const int a = bonds[2 * k], b = bonds[2 * k + 1];
    if (a < 0 || a >= N || b < 0 || b >= N) throw FxError(FX_E_INVALID, "bond atom index out of range");
    if (frag[a] == frag[b]) throw FxError(FX_E_INVALID, "a cut bond must join two fragments");
    const DevElem& el = P.elems[elem[a]];
    if (el.nsh != 2 || el.l[0] != 0 || el.l[1] != 1)
      throw FxError(FX_E_UNSUPPORTED, "a detached atom needs one s and one p shell");
  }
  Ne = N + NB;
  // fragments, real atoms in ascending order (pair lists)
  frag_off_real.assign(F + 1, 0);
  for (int A = 0; A < N; ++A) frag_off_real[frag[A] + 1]++;
  for (int I = 0; I < F; ++I) {
    if (frag_off_real[I + 1] == 0) throw FxError(FX_E_INVALID, "empty fragment");
    frag_off_real[I + 1] += frag_off_real[I];
  }
  frag_atoms_real.assign(N, 0);
  {
    std::vector<int> fill(frag_off_real.begin(), frag_off_real.end() - 1);
    for (int A = 0; A < N; ++A) frag_atoms_real[fill[frag[A]]++] = A;
  }
  // extended atom tables: ghosts after the real atoms
  bda_bonds.assign(F, {});
  ghost_bonds.assign(F, {});
  for (int k = 0; k < NB; ++k) {
    const int a = bonds[2 * k], b = bonds[2 * k + 1];
    bda_bonds[frag[a]].push_back(k);
    ghost_bonds[frag[b]].push_back(k);
    elem.push_back(elem[a]);
    frag.push_back(frag[b]);
    for (int c = 0; c < 3; ++c) xyz_h.push_back(xyz[3 * a + c]);
  }
  // each fragment's monomer atoms: its real atoms, then its ghosts
  frag_off.assign(F + 1, 0);
  frag_atoms.clear();
  for (int I = 0; I < F; ++I) {
    for (int ia = frag_off_real[I]; ia < frag_off_real[I + 1]; ++ia) frag_atoms.push_back(frag_atoms_real[ia]);
    for (int k : ghost_bonds[I]) frag_atoms.push_back(N + k);
    frag_off[I + 1] = (int)frag_atoms.size();
  }
  // shells
  atom_sh0_g.assign(Ne + 1, 0);
  std::vector<int> sh_atom, sh_frag;
  std::vector<double> sh_eta;
  for (int A = 0; A < Ne; ++A) {
    const DevElem& el = P.elems[elem[A]];
    for (int s = 0; s < el.nsh; ++s) {
      sh_atom.push_back(A);
      sh_frag.push_back(frag[A]);
      sh_eta.push_back(el.eta[s]);
    }
    atom_sh0_g[A + 1] = (int)sh_atom.size();
  }
  Nsh = (int)sh_atom.size();
  {
    std::vector<double> nsh_f(F, 0.0);
    for (int A = 0; A < Ne; ++A) nsh_f[frag[A]] += atom_sh0_g[A + 1] - atom_sh0_g[A];
    field_pairs = (double)Nsh * Nsh;
    for (double v : nsh_f) field_pairs -= v * v;
  }
  d_xyz.upload(xyz_h);
  d_elem.upload(elem);
  d_frag.upload(frag);
  d_atom_sh0.upload(atom_sh0_g);
  d_sh_atom.upload(sh_atom);
  d_sh_frag.upload(sh_frag);
  d_sh_eta.upload(sh_eta);
  std::vector<double> sh_ieta(sh_eta.size());
  for (size_t k = 0; k < sh_eta.size(); ++k) sh_ieta[k] = 0.5 / sh_eta[k];
  d_sh_ieta.upload(sh_ieta);
  d_frag_atoms.upload(frag_atoms);
  d_frag_off.upload(frag_off);
  d_frag_atoms_real.upload(frag_atoms_real);
  d_frag_off_real.upload(frag_off_real);
  d_bonds.upload(bonds.empty() ? std::vector<int>{0, 0} : bonds);
  d_cn.alloc(Ne);
  d_q.alloc(Nsh);
  d_qnew.alloc(Nsh);
  d_phi.alloc(Nsh);
  d_scalar.alloc(8);
  guess.assign(Nsh, 0.0);
  warm_valid = false;
  has_system = true;
  lists_built = false;
  has_result = false;
  has_grad = false;
}

// New positions for the current system (same atoms, fragments and bonds):
// every geometry-derived table is rebuilt as by set_system; the starting
// charges of FX_GUESS_USER are kept.
void Ctx::set_coordinates(const double* xyz) {
  if (!has_system) throw FxError(FX_E_STATE, "no system set");
  if (!xyz) throw FxError(FX_E_INVALID, "null coordinates");
  std::vector<int32_t> Z(N), fr(frag.begin(), frag.begin() + N), ch(frag_charge.begin(), frag_charge.end());
  for (int A = 0; A < N; ++A) Z[A] = P.elems[elem[A]].Z;
  std::vector<int32_t> bd(bonds.begin(), bonds.end());
  const int nb = NB;
  std::vector<double> g = guess;
  const bool wv = warm_valid;
  set_system(N, Z.data(), xyz, F, fr.data(), ch.data(), nb, nb ? bd.data() : nullptr);
  guess = g;
  warm_valid = wv;  // same fragments: the last run's clusters remain valid starts
}

// Velocity Verlet (atomic units: bohr, electron masses, hbar/Eh):
//   x <- x + v dt + (1/2) a dt^2,  a = -grad E / m at the new x,
//   v <- v + (1/2) (a_old + a_new) dt.
// Every step after the first starts the monomer loop from the previous
// step's converged monomer charges (the fixed point does not depend on the
// start); pair and trimer lists are rebuilt at every geometry.
void Ctx::md_verlet(int n_steps, double dt, const double* mass, double* xyz, double* vel, double* e_pot,
                    double* e_kin) {
  if (!has_system) throw FxError(FX_E_STATE, "no system set");
  if (NB > 0) throw FxError(FX_E_UNSUPPORTED, "molecular dynamics needs the gradient (no cut bonds)");
  if (n_steps < 0 || !(dt > 0.0) || !std::isfinite(dt) || !mass || !xyz || !vel)
    throw FxError(FX_E_INVALID, "bad molecular dynamics arguments");
  for (int A = 0; A < N; ++A)
    if (!(mass[A] > 0.0) || !std::isfinite(mass[A])) throw FxError(FX_E_INVALID, "masses must be positive");
  for (long long k = 0; k < 3LL * N; ++k)
    if (!std::isfinite(vel[k]) || !std::isfinite(xyz[k])) throw FxError(FX_E_INVALID, "non-finite input");
  struct Restore {
    Ctx& c;
    fx_options o;
    ~Restore() { c.opt = o; }
  } restore{*this, opt};
  opt.want_gradient = 1;
  opt.warm_clusters = 1;
  const long long n3 = 3LL * N;
  std::vector<double> x(xyz, xyz + n3), v(vel, vel + n3), g(n3), gn(n3);
  auto kinetic = [&]() {
    double t = 0.0;
    for (int A = 0; A < N; ++A)
      for (int k = 0; k < 3; ++k) t += 0.5 * mass[A] * v[3 * A + k] * v[3 * A + k];
    return t;
  };
  auto energy_gradient = [&](int step) {
    set_coordinates(x.data());
    if (step > 0) opt.guess = FX_GUESS_USER;
    fx_result r;
    run(&r);
    if (!res.converged) throw FxError(FX_E_NOCONV, "molecular dynamics step " + std::to_string(step) +
                                                       ": a fragment SCC or the monomer loop did not converge");
    d_grad.download_raw(gn.data(), n3, stream);
    guess.resize(Nsh);
    d_q.download_raw(guess.data(), Nsh, stream);
    sync();
    return r.e_total;
  };
  double E = energy_gradient(0);
  g = gn;
  if (e_pot) e_pot[0] = E;
  if (e_kin) e_kin[0] = kinetic();
  for (int step = 1; step <= n_steps; ++step) {
    for (int A = 0; A < N; ++A)
      for (int k = 0; k < 3; ++k) {
        const long long i = 3LL * A + k;
        x[i] += v[i] * dt - 0.5 * g[i] / mass[A] * dt * dt;
      }
    E = energy_gradient(step);
    for (int A = 0; A < N; ++A)
      for (int k = 0; k < 3; ++k) {
        const long long i = 3LL * A + k;
        v[i] -= 0.5 * (g[i] + gn[i]) / mass[A] * dt;
      }
    g = gn;
    if (e_pot) e_pot[step] = E;
    if (e_kin) e_kin[step] = kinetic();
  }
  std::copy(x.begin(), x.end(), xyz);
  std::copy(v.begin(), v.end(), vel);
}

// ---------------------------------------------------------------------------

void Ctx::run(fx_result* out) {
  if (!has_system) throw FxError(FX_E_STATE, "no system set");
  const bool mixed = opt.precision == FX_MIXED;
  if (NB > 0 && opt.want_gradient && opt.order >= 3)
    throw FxError(FX_E_UNSUPPORTED, "the FMO3 gradient with cut covalent bonds is not available");
  std::memset(&res, 0, sizeof(res));
  ktimers.clear();
  resp_ok = false;
  bool all_conv = true;
  double t0 = now_ms();
  if (!lists_built) build_lists_impl();
  compute_cn();
  sync();
  double t1 = now_ms();
  res.ms_lists = t1 - t0;

  // ---- monomers: self-consistent embedding (Jacobi sweeps over monomers)
  std::vector<std::array<int, 3>> mono(F);
  for (int I = 0; I < F; ++I) mono[I] = {I, -1, -1};
  build_batch(mb, mono, 1);
  build_matrices(mb);
  DevBatch dmb = mb.dev();
  if (opt.guess == FX_GUESS_USER) d_q.upload_async(guess, stream);
  else if (opt.guess == FX_GUESS_LEARNED) learned_guess();
  else check(hipMemsetAsync(d_q.p, 0, sizeof(double) * Nsh, stream), "memset");
  hipLaunchKernelGGL(k_gather_shell, dim3(mb.nsys), dim3(64), 0, stream, dmb, d_q.p, mb.q_in.p);
  long long it_mono = 0;
  int macro = 0;
  double delta = 1e300;
  bool cold = true;
  // Anderson mixing of the monomer charge vector across sweeps
  DevBuf<double> hX, hR, hC;
  hX.alloc((long long)HIST * Nsh);
  hR.alloc((long long)HIST * Nsh);
  hC.alloc(HIST);
  std::vector<int> slots;
  int next_slot = 0;
  const unsigned gN = (unsigned)((Nsh + 255) / 256);
  mono_tmp.alloc(Nsh);
  DevBuf<double> d_tmp_local;
  d_tmp_local.alloc(mb.tot_sh);
  std::vector<int> all_mono(mb.nsys);
  for (int k = 0; k < mb.nsys; ++k) all_mono[k] = k;
  bool fused_mode = false;
  // mixed precision: FP32 field passes until the monomer charges move by
  // less than 1e-6, FP64 from then on (the fixed point is the FP64 one)
  bool field32 = mixed;
  for (macro = 1; macro <= opt.max_macro; ++macro) {
    if (field32 && delta < 1e-6) {
      field32 = false;
      slots.clear();
      next_slot = 0;
    }
    field(d_q.p, d_phi.p, field32);
    hipLaunchKernelGGL(k_gather_shell, dim3(mb.nsys), dim3(64), 0, stream, dmb, d_phi.p, mb.phi.p);
    int failed = 0;
    if (fused_mode) {
      // one SCC iteration of every monomer at the globally mixed charges
      hipLaunchKernelGGL(k_gather_shell, dim3(mb.nsys), dim3(64), 0, stream, dmb, d_q.p, mb.q_in.p);
      // (FP64 products in the fused steps: FP32 ones there cost more steps
      // than they save)
      run_scc(mb, all_mono, false, &it_mono, true);
    } else {
      if (cold)
        hipLaunchKernelGGL(k_gather_shell, dim3(mb.nsys), dim3(64), 0, stream, dmb, d_q.p, mb.q_in.p);
      else
        check(hipMemcpyAsync(mb.q_in.p, mb.q_out.p, sizeof(double) * mb.tot_sh, hipMemcpyDeviceToDevice, stream),
              "copy");
      // inner solves only as tight as the outer residual requires
      scc_tol_cur = std::max(opt.scc_tol, std::min(1e-4, 1e-3 * delta));
      etol_cur = std::max(opt.energy_tol, std::min(1e-4, 1e-4 * delta));
      first_solve = cold;
      if (cold) {
        fallback_flag.alloc(mb.nsys);
        check(hipMemsetAsync(fallback_flag.p, 0, sizeof(int) * mb.nsys, stream), "memset");
      }
      prod_mode = mixed ? 1 : 0;
      failed = solve_batch(mb, cold, &it_mono);
      prod_mode = 0;
      first_solve = false;
      if (cold) {
        std::vector<int> fl;
        fallback_flag.download(fl, stream);
        sync();
        for (int v : fl) res.guess_fallbacks += v;
      }
      scc_tol_cur = etol_cur = -1.0;
      if (cold && precond && monomer_response_setup()) build_precond(mb);
    }
    const bool was_cold = cold;
    cold = false;
    res.solves_mono += mb.nsys;
    hipLaunchKernelGGL(k_scatter_shell, dim3(mb.nsys), dim3(64), 0, stream, dmb, mb.q_out.p, d_qnew.p);
    max_absdiff(d_qnew.p, d_q.p, Nsh, d_scalar.p);
    std::vector<double> hs(1);
    d_scalar.download(hs, stream, 1);
    sync();
    delta = hs[0];
    if (verbose)
      std::fprintf(stderr, "[fx] monomer %s %d: max |dq_out - dq_in| = %.3e, %.1f ms\n",
                   fused_mode ? "step" : "sweep", macro, delta, now_ms() - t1);
    if (delta < opt.macro_tol) {
      if (failed) all_conv = false;
      check(hipMemcpyAsync(d_q.p, d_qnew.p, sizeof(double) * Nsh, hipMemcpyDeviceToDevice, stream), "copy");
      break;
    }
    if (was_cold && fused && mb.has_pre) {
      // switch to the fused loop from the charges of the first full solve
      check(hipMemcpyAsync(d_q.p, d_qnew.p, sizeof(double) * Nsh, hipMemcpyDeviceToDevice, stream), "copy");
      fused_mode = true;
      slots.clear();
      next_slot = 0;
      continue;
    }
    // history update and mixing; in the fused loop the residual is the
    // monomer-block Newton step (1 + M_I G_I)^-1 (q_out - q_in)
    const double* target = d_qnew.p;
    if (fused_mode) {
      hipLaunchKernelGGL(k_precond_step, dim3(mb.nsys), dim3(128), 0, stream, mb.dev(), d_tmp_local.p);
      hipLaunchKernelGGL(k_scatter_shell, dim3(mb.nsys), dim3(64), 0, stream, dmb, d_tmp_local.p, mono_tmp.p);
      target = mono_tmp.p;
    }
    int slot;
    if ((int)slots.size() < HIST) {
      slot = next_slot++;
    } else {
      slot = slots.front();
      slots.erase(slots.begin());
    }
    slots.push_back(slot);
    hipLaunchKernelGGL(k_hist_store, dim3(gN), dim3(256), 0, stream, d_q.p, target, (long long)Nsh, slot, hX.p,
                       hR.p);
    Slots sl;
    sl.m = (int)slots.size();
    for (int k = 0; k < sl.m; ++k) sl.id[k] = slots[k];
    hist_coef(hR.p, (long long)Nsh, sl, hC.p);
    hipLaunchKernelGGL(k_hist_mix, dim3(gN), dim3(256), 0, stream, hX.p, hR.p, (long long)Nsh, sl, hC.p,
                       fused_mode ? fused_beta : macro_beta, d_q.p);
    check(hipGetLastError(), "monomer mixing");
  }
  if (macro > opt.max_macro) {
    all_conv = false;
    macro = opt.max_macro;
  }
  res.macro_iter = macro;
  res.iters_mono = it_mono;
  // susceptibilities of the converged monomers: dimer preconditioners and the
  // response of the gradient
  resp_ok = false;
  if (precond || (opt.want_gradient && opt.want_response)) monomer_response_setup();
  // final embedding field of the converged charges
  field(d_q.p, d_phi.p);
  e_mono.alloc(F);
  check(hipMemcpyAsync(e_mono.p, mb.e_int.p, sizeof(double) * F, hipMemcpyDeviceToDevice, stream), "copy");
  sync();
  double t2 = now_ms();
  res.ms_monomer = t2 - t1;

  // ---- SCC dimers (and trimers) in the converged embedding
  const long long nscc = (long long)scc_pairs.size() / 2;
  dE_scc.alloc(std::max(1LL, nscc));
  dEV_scc.alloc(std::max(1LL, nscc));
  if (nscc > 0) {
    std::vector<std::array<int, 3>> cl(nscc);
    for (long long k = 0; k < nscc; ++k) cl[k] = {scc_pairs[2 * k], scc_pairs[2 * k + 1], -1};
    build_batch(db_, cl, 2);
    db_.init_from_mono = !db_.has_healed;
    build_matrices(db_, true);
    DevBatch ddb = db_.dev();
    hipLaunchKernelGGL(k_cluster_phi, dim3(db_.nsys), dim3(128), 0, stream, dev_system(), ddb, d_phi.p, d_q.p);
    hipLaunchKernelGGL(k_gather_shell, dim3(db_.nsys), dim3(64), 0, stream, ddb, d_q.p, db_.q_in.p);
    // dimers also solved in the last run start from that solution
    db_.has_warm = false;
    if (opt.warm_clusters && warm_valid && db_.init_from_mono) {
      std::unordered_map<long long, int> old;
      for (size_t k = 0; 2 * k < warm_pairs.size(); ++k) old[(long long)warm_pairs[2 * k] * F + warm_pairs[2 * k + 1]] = (int)k;
      std::vector<long long> mo(nscc, -1), so(nscc, -1);
      long long nwarm = 0;
      for (long long k = 0; k < nscc; ++k) {
        auto it = old.find((long long)scc_pairs[2 * k] * F + scc_pairs[2 * k + 1]);
        if (it == old.end()) continue;
        mo[k] = warm_matoff[it->second];
        so[k] = warm_shoff[it->second];
        ++nwarm;
      }
      if (nwarm > 0) {
        db_.warm_off.upload(mo);
        warm_so.upload(so);
        hipLaunchKernelGGL(k_warm_start, dim3(db_.nsys), dim3(256), 0, stream, ddb, db_.warm_off.p, warm_so.p,
                           warm_C.p, warm_q.p);
        check(hipGetLastError(), "k_warm_start");
        db_.has_warm = true;
      }
      res.warm_dimers = nwarm;
    }
    build_precond(db_);
    long long itd = 0;
    prod_mode = mixed ? 1 : 0;
    int failed = solve_batch(db_, true, &itd);
    prod_mode = 0;
    if (failed && opt.scc_retry) failed = retry_failed(db_, &itd);
    if (failed) all_conv = false;
    res.solves_dimer = nscc;
    res.iters_dimer = itd;
    ddq_scc.alloc(db_.tot_sh);
    hipLaunchKernelGGL(k_cluster_terms, dim3(db_.nsys), dim3(256), 0, stream, ddb, d_q.p, e_mono.p, ddq_scc.p,
                       dEV_scc.p, dE_scc.p);
    if (db_.has_healed)
      hipLaunchKernelGGL(k_cluster_healed, dim3(db_.nsys), dim3(128), 0, stream, dev_system(), ddb, d_phi.p, d_q.p,
                         dEV_scc.p, dE_scc.p);
    check(hipGetLastError(), "k_cluster_terms");
    db_.has_warm = false;
    if (opt.warm_clusters) {
      warm_pairs = scc_pairs;
      warm_matoff.resize(db_.nsys);
      warm_shoff.resize(db_.nsys);
      for (int k = 0; k < db_.nsys; ++k) {
        warm_matoff[k] = db_.h_desc[k].mat_off;
        warm_shoff[k] = db_.h_desc[k].sh_off;
      }
      warm_C.alloc(db_.tot_mat);
      warm_q.alloc(db_.tot_sh);
      check(hipMemcpyAsync(warm_C.p, db_.Ct.p, sizeof(double) * db_.tot_mat, hipMemcpyDeviceToDevice, stream),
            "copy");
      check(hipMemcpyAsync(warm_q.p, db_.q_out.p, sizeof(double) * db_.tot_sh, hipMemcpyDeviceToDevice, stream),
            "copy");
      warm_valid = true;
    }
  }
  if (nscc == 0) warm_valid = false;
  sync();
  double t3 = now_ms();
  res.ms_dimer = t3 - t2;

  const long long ntri = (long long)trimers.size() / 3;
  dE_tri.alloc(std::max(1LL, ntri));
  if (opt.order >= 3 && ntri > 0) {
    std::vector<std::array<int, 3>> cl(ntri);
    for (long long k = 0; k < ntri; ++k) cl[k] = {trimers[3 * k], trimers[3 * k + 1], trimers[3 * k + 2]};
    build_batch(tb_, cl, 3);
    tb_.init_from_mono = !tb_.has_healed;
    build_matrices(tb_, true);
    DevBatch dtb = tb_.dev();
    hipLaunchKernelGGL(k_cluster_phi, dim3(tb_.nsys), dim3(128), 0, stream, dev_system(), dtb, d_phi.p, d_q.p);
    hipLaunchKernelGGL(k_gather_shell, dim3(tb_.nsys), dim3(64), 0, stream, dtb, d_q.p, tb_.q_in.p);
    build_precond(tb_);
    long long itt = 0;
    prod_mode = mixed ? 1 : 0;
    int failed = solve_batch(tb_, true, &itt);
    prod_mode = 0;
    if (failed && opt.scc_retry) failed = retry_failed(tb_, &itt);
    if (failed) all_conv = false;
    res.solves_trimer = ntri;
    res.iters_trimer = itt;
    DevBuf<double> dEV, dEX;
    ddq_tri.alloc(tb_.tot_sh);
    dEV.alloc(ntri);
    dEX.alloc(ntri);
    hipLaunchKernelGGL(k_cluster_terms, dim3(tb_.nsys), dim3(256), 0, stream, dtb, d_q.p, e_mono.p, ddq_tri.p, dEV.p,
                       dEX.p);
    if (tb_.has_healed)
      hipLaunchKernelGGL(k_cluster_healed, dim3(tb_.nsys), dim3(128), 0, stream, dev_system(), dtb, d_phi.p, d_q.p,
                         dEV.p, dEX.p);
    d_dEIJK.alloc(ntri);
    check(hipMemcpyAsync(d_dEIJK.p, dEX.p, sizeof(double) * ntri, hipMemcpyDeviceToDevice, stream), "copy");
  }
  double t4 = now_ms();
  res.ms_trimer = t4 - t3;

  // ---- ES-DIM pairs and the energy
  const long long nesd = (long long)esd_pairs.size() / 2;
  dE_esd.alloc(std::max(1LL, nesd));
  if (nesd > 0) {
    DevBuf<int> dp;
    dp.upload(esd_pairs);
    if (nesd > 0x7fffffffLL) throw FxError(FX_E_INVALID, "too many ES-DIM pairs");
    hipLaunchKernelGGL(k_esd_pairs, dim3((unsigned)nesd), dim3(64), 0, stream, dev_system(), dp.p,
                       nesd, d_frag_atoms.p, d_frag_off.p, d_q.p, dE_esd.p);
    check(hipGetLastError(), "k_esd_pairs");
    sync();
  }
  {
    std::vector<const double*> arr = {e_mono.p, dE_scc.p, dE_esd.p};
    std::vector<long long> len = {F, nscc, nesd};
    DevBuf<const double*> da;
    da.upload(arr);
    DevBuf<long long> dl;
    dl.upload(len);
    hipLaunchKernelGGL(k_sum_neumaier, dim3(1), dim3(256), 0, stream, da.p, dl.p, 3, d_scalar.p);
    std::vector<double> hs(1);
    d_scalar.download(hs, stream, 1);
    sync();
    res.e_fmo2 = hs[0];
    res.e_total = hs[0];
  }
  if (opt.order >= 3 && ntri > 0) {
    // trimer corrections Delta E_IJK - Delta E_IJ - Delta E_IK - Delta E_JK on
    // the device; the host only locates each sub-pair in the pair lists
    // (index into dE_scc, or nscc + index into dE_esd)
    std::unordered_map<long long, long long> where;
    where.reserve((size_t)(nscc + nesd) * 2);
    for (long long k = 0; k < nscc; ++k) where[(long long)scc_pairs[2 * k] * F + scc_pairs[2 * k + 1]] = k;
    for (long long k = 0; k < nesd; ++k) where[(long long)esd_pairs[2 * k] * F + esd_pairs[2 * k + 1]] = nscc + k;
    std::vector<long long> sub_idx(3 * ntri);
    for (long long k = 0; k < ntri; ++k) {
      const int I = trimers[3 * k], J = trimers[3 * k + 1], K = trimers[3 * k + 2];
      sub_idx[3 * k] = where.at((long long)I * F + J);
      sub_idx[3 * k + 1] = where.at((long long)I * F + K);
      sub_idx[3 * k + 2] = where.at((long long)J * F + K);
    }
    DevBuf<long long> d_sub;
    d_sub.upload(sub_idx);
    hipLaunchKernelGGL(k_trimer_corr, dim3((unsigned)((ntri + 255) / 256)), dim3(256), 0, stream, ntri,
                       (const double*)d_dEIJK.p, (const double*)dE_scc.p, nscc, (const double*)dE_esd.p,
                       (const long long*)d_sub.p, dE_tri.p);
    check(hipGetLastError(), "k_trimer_corr");
    std::vector<const double*> arr = {d_scalar.p, dE_tri.p};
    std::vector<long long> len = {1, ntri};
    DevBuf<const double*> da;
    da.upload(arr);
    DevBuf<long long> dl;
    dl.upload(len);
    DevBuf<double> outv;
    outv.alloc(1);
    hipLaunchKernelGGL(k_sum_neumaier, dim3(1), dim3(256), 0, stream, da.p, dl.p, 2, outv.p);
    std::vector<double> hs(1);
    outv.download(hs, stream, 1);
    sync();
    res.e_total = hs[0];
  }
  double t5 = now_ms();
  res.ms_energy = t5 - t4;
  res.converged = all_conv ? 1 : 0;
  has_result = true;
  has_grad = false;
  if (opt.want_gradient) {
    gradient();
    has_grad = true;
  }
  res.ms_gradient = now_ms() - t5;
  {
    sync();
    timers.resolve();
    std::vector<const KernelTimer*> ks;
    for (const auto& t : ktimers) ks.push_back(&t);
    std::stable_sort(ks.begin(), ks.end(), [](const KernelTimer* a, const KernelTimer* b) { return a->ms > b->ms; });
    res.n_kstat = (int)std::min<size_t>(ks.size(), FX_MAX_KSTAT);
    for (int k = 0; k < res.n_kstat; ++k) {
      std::snprintf(res.kstat[k].name, sizeof(res.kstat[k].name), "%s", ks[k]->name.c_str());
      res.kstat[k].ms = ks[k]->ms;
      res.kstat[k].launches = ks[k]->launches;
      res.kstat[k].gflop = ks[k]->gflop;
    }
  }
  if (out) *out = res;
}

}  // namespace fx

// ---------------------------------------------------------------------------
// C ABI


static thread_local std::string g_param_error;

#define FX_GUARD(ctx, ...)                                   \
  fx::DevMemScope fx_mem_scope_(&(ctx)->mem);                \
  try {                                                      \
    __VA_ARGS__;                                             \
    (ctx)->c.last_error.clear();                             \
    return FX_OK;                                            \
  } catch (const fx::FxError& e) {                           \
    (ctx)->c.last_error = e.what();                          \
    return e.code;                                           \
  } catch (const std::exception& e) {                        \
    (ctx)->c.last_error = e.what();                          \
    return FX_E_INVALID;                                     \
  }

extern "C" {

int fx_params_load(const char* json_path, fx_params** out) {
  if (!json_path || !out) return FX_E_INVALID;
  try {
    auto* p = new fx_params();
    p->P = fx::load_params(json_path);
    *out = p;
    return FX_OK;
  } catch (const fx::FxError& e) {
    g_param_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_param_error = e.what();
    return FX_E_INVALID;
  }
}

void fx_params_free(fx_params* p) { delete p; }

int fx_ctx_create(const fx_params* p, int device, void* hip_stream, fx_ctx** out) {
  if (!p || !out) return FX_E_INVALID;
  auto* c = new fx_ctx();
  fx::DevMemScope scope(&c->mem);
  try {
    c->c.P = p->P;
    c->c.device = device;
    fx::Ctx::check(hipSetDevice(device), "hipSetDevice");
    c->c.stream = static_cast<hipStream_t>(hip_stream);
    c->c.init_device();
    c->c.d_elems.upload(c->c.P.elems);
    fx_default_options(&c->c.opt);
  } catch (const fx::FxError& e) {
    g_param_error = e.what();
    delete c;
    return e.code;
  }
  *out = c;
  return FX_OK;
}

void fx_ctx_destroy(fx_ctx* ctx) { delete ctx; }

int fx_workspace_size(fx_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return FX_E_INVALID;
  // the peak plus a margin: launch shapes chosen by timing (the eigensolver
  // autotuner) can change a few buffer sizes between otherwise identical runs
  const size_t p = ctx->mem.peak;
  *bytes = (p + p / 32 + (size_t(4) << 20) + fx::DevMem::kAlign - 1) / fx::DevMem::kAlign * fx::DevMem::kAlign;
  return FX_OK;
}

int fx_set_workspace(fx_ctx* ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return FX_E_INVALID;
  if (dev_ptr && (bytes == 0 || reinterpret_cast<uintptr_t>(dev_ptr) % fx::DevMem::kAlign != 0)) {
    ctx->c.last_error = "workspace must be non-empty and 256-byte aligned";
    return FX_E_INVALID;
  }
  if (!dev_ptr && bytes != 0) {
    ctx->c.last_error = "a NULL workspace must have size 0";
    return FX_E_INVALID;
  }
  fx::DevMemScope scope(&ctx->mem);
  try {
    // back to the state after fx_ctx_create: every buffer is released to the
    // memory it came from before the new memory takes over
    fx::HostParams P = ctx->c.P;
    const int device = ctx->c.device;
    hipStream_t stream = ctx->c.stream;
    const fx_options opt = ctx->c.opt;
    ctx->c.~Ctx();
    new (&ctx->c) fx::Ctx();
    if (!ctx->mem.live.empty()) throw fx::FxError(FX_E_STATE, "device buffers outlived the context reset");
    ctx->mem.release_cache();
    ctx->mem.base = static_cast<char*>(dev_ptr);
    ctx->mem.size = bytes;
    ctx->mem.top = 0;
    ctx->mem.peak = 0;
    ctx->mem.free_.clear();
    ctx->c.P = P;
    ctx->c.device = device;
    fx::Ctx::check(hipSetDevice(device), "hipSetDevice");
    ctx->c.stream = stream;
    ctx->c.init_device();
    ctx->c.d_elems.upload(ctx->c.P.elems);
    ctx->c.opt = opt;
    ctx->c.last_error.clear();
    return FX_OK;
  } catch (const fx::FxError& e) {
    ctx->c.last_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    ctx->c.last_error = e.what();
    return FX_E_INVALID;
  }
}

const char* fx_last_error(const fx_ctx* ctx) { return ctx ? ctx->c.last_error.c_str() : g_param_error.c_str(); }

int fx_default_options(fx_options* o) {
  if (!o) return FX_E_INVALID;
  o->order = 2;
  o->cutoff_bohr = 4.0 / 0.529177210903;
  o->precision = FX_FP64;
  o->schedule = FX_BATCHED;
  o->guess = FX_GUESS_SUPERPOSITION;
  o->guess_tau = 0.0;
  o->guess_max_iter = 50;
  o->scc_tol = 1e-10;
  o->energy_tol = 1e-11;
  o->macro_tol = 1e-10;
  o->max_iter = 200;
  o->max_macro = 200;
  o->want_gradient = 1;
  o->want_response = 1;
  o->selection = FX_SELECT_CUTOFF;
  o->vdw_dimer = 2.0;
  o->vdw_trimer = 1.5;
  o->warm_clusters = 0;
  o->max_response = 400;
  o->scc_retry = 1;
  return FX_OK;
}

int fx_set_options(fx_ctx* ctx, const fx_options* o) {
  if (!ctx || !o) return FX_E_INVALID;
  FX_GUARD(ctx, {
    if (o->order != 2 && o->order != 3) throw fx::FxError(FX_E_INVALID, "order must be 2 or 3");
    if (!(o->cutoff_bohr >= 0.0) || !(o->scc_tol > 0.0) || !(o->macro_tol > 0.0) || o->max_iter < 1 ||
        o->max_macro < 1)
      throw fx::FxError(FX_E_INVALID, "bad option value");
    if (o->precision != FX_FP64 && o->precision != FX_MIXED) throw fx::FxError(FX_E_INVALID, "bad precision");
    if (o->schedule != FX_BATCHED && o->schedule != FX_PLAIN_LOOP && o->schedule != FX_BATCHED_GRAPH &&
        o->schedule != FX_BATCHED_HOST_SYNC)
      throw fx::FxError(FX_E_INVALID, "bad schedule");
    if (o->guess != FX_GUESS_SUPERPOSITION && o->guess != FX_GUESS_LEARNED && o->guess != FX_GUESS_USER)
      throw fx::FxError(FX_E_INVALID, "bad guess");
    if (o->selection != FX_SELECT_CUTOFF && o->selection != FX_SELECT_VDW)
      throw fx::FxError(FX_E_INVALID, "bad selection rule");
    if (!(o->vdw_dimer > 0.0) || !(o->vdw_trimer > 0.0) || !std::isfinite(o->vdw_dimer) ||
        !std::isfinite(o->vdw_trimer))
      throw fx::FxError(FX_E_INVALID, "van der Waals scaling factors must be positive");
    if (o->warm_clusters != 0 && o->warm_clusters != 1) throw fx::FxError(FX_E_INVALID, "warm_clusters must be 0 or 1");
    if (o->max_response < 1) throw fx::FxError(FX_E_INVALID, "max_response must be positive");
    if (o->scc_retry != 0 && o->scc_retry != 1) throw fx::FxError(FX_E_INVALID, "scc_retry must be 0 or 1");
    const fx_options& c = ctx->c.opt;
    bool cutoff_changed = o->cutoff_bohr != c.cutoff_bohr || o->order != c.order || o->selection != c.selection ||
                          o->vdw_dimer != c.vdw_dimer || o->vdw_trimer != c.vdw_trimer;
    ctx->c.opt = *o;
    if (cutoff_changed) ctx->c.lists_built = false;
  });
}

int fx_set_system(fx_ctx* ctx, int32_t n_atoms, const int32_t* Z, const double* xyz_bohr, int32_t n_frag,
                  const int32_t* atom_frag, const int32_t* frag_charge, int32_t n_bonds, const int32_t* bonds) {
  if (!ctx) return FX_E_INVALID;
  FX_GUARD(ctx, ctx->c.set_system(n_atoms, Z, xyz_bohr, n_frag, atom_frag, frag_charge, n_bonds, bonds));
}

int fx_build_lists(fx_ctx* ctx, fx_counts* out) {
  if (!ctx) return FX_E_INVALID;
  FX_GUARD(ctx, {
    if (!ctx->c.has_system) throw fx::FxError(FX_E_STATE, "no system set");
    ctx->c.build_lists_impl();
    if (out) {
      out->n_scc_pairs = (int64_t)ctx->c.scc_pairs.size() / 2;
      out->n_esd_pairs = (int64_t)ctx->c.esd_pairs.size() / 2;
      out->n_trimers = (int64_t)ctx->c.trimers.size() / 3;
      out->n_shells = ctx->c.Nsh;
      out->n_fragments = ctx->c.F;
    }
  });
}

int fx_get_counts(fx_ctx* ctx, fx_counts* out) {
  if (!ctx || !out) return FX_E_INVALID;
  FX_GUARD(ctx, {
    if (!ctx->c.lists_built) throw fx::FxError(FX_E_STATE, "lists not built");
    out->n_scc_pairs = (int64_t)ctx->c.scc_pairs.size() / 2;
    out->n_esd_pairs = (int64_t)ctx->c.esd_pairs.size() / 2;
    out->n_trimers = (int64_t)ctx->c.trimers.size() / 3;
    out->n_shells = ctx->c.Nsh;
    out->n_fragments = ctx->c.F;
  });
}

int fx_get_lists(fx_ctx* ctx, int32_t* scc, int32_t* esd, int32_t* tri) {
  if (!ctx) return FX_E_INVALID;
  FX_GUARD(ctx, {
    if (!ctx->c.lists_built) throw fx::FxError(FX_E_STATE, "lists not built");
    if (scc) std::copy(ctx->c.scc_pairs.begin(), ctx->c.scc_pairs.end(), scc);
    if (esd) std::copy(ctx->c.esd_pairs.begin(), ctx->c.esd_pairs.end(), esd);
    if (tri) std::copy(ctx->c.trimers.begin(), ctx->c.trimers.end(), tri);
  });
}

int fx_set_guess(fx_ctx* ctx, const double* dq) {
  if (!ctx || !dq) return FX_E_INVALID;
  FX_GUARD(ctx, {
    if (!ctx->c.has_system) throw fx::FxError(FX_E_STATE, "no system set");
    for (int k = 0; k < ctx->c.Nsh; ++k)
      if (!std::isfinite(dq[k])) throw fx::FxError(FX_E_INVALID, "non-finite guess charge");
    ctx->c.guess.assign(dq, dq + ctx->c.Nsh);
  });
}

int fx_run(fx_ctx* ctx, fx_result* out) {
  if (!ctx) return FX_E_INVALID;
  fx::DevMemScope scope(&ctx->mem);
  try {
    const long long allocs0 = ctx->mem.hip_allocs;
    ctx->c.run(out);
    ctx->c.res.device_allocs = ctx->mem.hip_allocs - allocs0;
    if (out) out->device_allocs = ctx->c.res.device_allocs;
    ctx->c.last_error.clear();
    if (!ctx->c.res.converged) {
      ctx->c.last_error = "a fragment SCC or the monomer loop did not converge";
      return FX_E_NOCONV;
    }
    return FX_OK;
  } catch (const fx::FxError& e) {
    ctx->c.last_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    ctx->c.last_error = e.what();
    return FX_E_INVALID;
  }
}

int fx_get_energies(fx_ctx* ctx, double* E_mono, double* dE_scc, double* dE_esd, double* dE_tri) {
  if (!ctx) return FX_E_INVALID;
  FX_GUARD(ctx, {
    fx::Ctx& c = ctx->c;
    if (!c.has_result) throw fx::FxError(FX_E_STATE, "no result");
    const long long nscc = (long long)c.scc_pairs.size() / 2, nesd = (long long)c.esd_pairs.size() / 2,
                    ntri = (long long)c.trimers.size() / 3;
    if (E_mono) c.e_mono.download_raw(E_mono, c.F, c.stream);
    if (dE_scc && nscc) c.dE_scc.download_raw(dE_scc, nscc, c.stream);
    if (dE_esd && nesd) c.dE_esd.download_raw(dE_esd, nesd, c.stream);
    if (dE_tri && ntri && c.opt.order >= 3) c.dE_tri.download_raw(dE_tri, ntri, c.stream);
    c.sync();
  });
}

int fx_get_charges(fx_ctx* ctx, double* dq) {
  if (!ctx || !dq) return FX_E_INVALID;
  FX_GUARD(ctx, {
    if (!ctx->c.has_result) throw fx::FxError(FX_E_STATE, "no result");
    ctx->c.d_q.download_raw(dq, ctx->c.Nsh, ctx->c.stream);
    ctx->c.sync();
  });
}

int fx_get_gradient(fx_ctx* ctx, double* grad) {
  if (!ctx || !grad) return FX_E_INVALID;
  FX_GUARD(ctx, {
    if (!ctx->c.has_grad) throw fx::FxError(FX_E_STATE, "no gradient computed");
    ctx->c.d_grad.download_raw(grad, 3LL * ctx->c.N, ctx->c.stream);
    ctx->c.sync();
  });
}

int fx_set_coordinates(fx_ctx* ctx, const double* xyz_bohr) {
  if (!ctx || !xyz_bohr) return FX_E_INVALID;
  FX_GUARD(ctx, ctx->c.set_coordinates(xyz_bohr));
}

int fx_md_verlet(fx_ctx* ctx, int32_t n_steps, double dt, const double* mass, double* xyz_bohr, double* vel,
                 double* e_pot, double* e_kin) {
  if (!ctx) return FX_E_INVALID;
  FX_GUARD(ctx, ctx->c.md_verlet(n_steps, dt, mass, xyz_bohr, vel, e_pot, e_kin));
}

int fx_compute_cn(fx_ctx* ctx, double* cn) {
  if (!ctx || !cn) return FX_E_INVALID;
  FX_GUARD(ctx, {
    if (!ctx->c.has_system) throw fx::FxError(FX_E_STATE, "no system set");
    ctx->c.compute_cn();
    ctx->c.d_cn.download_raw(cn, ctx->c.N, ctx->c.stream);
    ctx->c.sync();
  });
}

int fx_cluster_matrices(fx_ctx* ctx, int32_t nfrag, const int32_t* frags, int32_t* nao_out, double* S, double* H0) {
  if (!ctx || !frags || nfrag < 1 || nfrag > 3) return FX_E_INVALID;
  FX_GUARD(ctx, {
    fx::Ctx& c = ctx->c;
    if (!c.has_system) throw fx::FxError(FX_E_STATE, "no system set");
    std::array<int, 3> cl = {-1, -1, -1};
    for (int k = 0; k < nfrag; ++k) {
      if (frags[k] < 0 || frags[k] >= c.F) throw fx::FxError(FX_E_INVALID, "fragment index out of range");
      cl[k] = frags[k];
    }
    fx::Batch b;
    c.build_batch(b, {cl}, nfrag);
    int nao = b.h_desc[0].nao;
    if (nao_out) *nao_out = nao;
    if (S || H0) {
      c.compute_cn();
      c.build_matrices(b);
      if (S) b.S.download_raw(S, (long long)nao * nao, c.stream);
      if (H0) b.H0.download_raw(H0, (long long)nao * nao, c.stream);
      c.sync();
    }
  });
}

int fx_embedding_field(fx_ctx* ctx, const double* dq, double* phi) {
  if (!ctx || !dq || !phi) return FX_E_INVALID;
  FX_GUARD(ctx, {
    fx::Ctx& c = ctx->c;
    if (!c.has_system) throw fx::FxError(FX_E_STATE, "no system set");
    fx::DevBuf<double> q, p;
    q.upload(std::vector<double>(dq, dq + c.Nsh));
    p.alloc(c.Nsh);
    c.field(q.p, p.p, c.opt.precision == FX_MIXED);
    p.download_raw(phi, c.Nsh, c.stream);
    c.sync();
  });
}

int fx_eigh_batched(fx_ctx* ctx, int32_t nmat, const int32_t* n, const double* A, double* w, double* V) {
  if (!ctx || nmat < 0 || !n || !A || !w || !V) return FX_E_INVALID;
  FX_GUARD(ctx, {
    std::vector<int> nv(n, n + nmat);
    for (int k = 0; k < nmat; ++k)
      if (nv[k] < 1 || nv[k] > fx::MAXN) throw fx::FxError(FX_E_INVALID, "matrix size out of range");
    if (nmat == 0) return FX_OK;
    // matrices smaller than any SCC system (8 AOs) go to the global-memory
    // kernel, the others through the SCC's eigensolver
    std::vector<long long> off(nmat + 1, 0), woff(nmat + 1, 0);
    for (int k = 0; k < nmat; ++k) {
      off[k + 1] = off[k] + (long long)nv[k] * nv[k];
      woff[k + 1] = woff[k] + nv[k];
    }
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<int> sel, ns;
      std::vector<double> a;
      for (int k = 0; k < nmat; ++k)
        if ((nv[k] >= 8) == (pass == 0)) {
          sel.push_back(k);
          ns.push_back(nv[k]);
          a.insert(a.end(), A + off[k], A + off[k + 1]);
        }
      if (sel.empty()) continue;
      long long tot = 0, wt = 0;
      for (int x : ns) {
        tot += (long long)x * x;
        wt += x;
      }
      std::vector<double> ws(wt), vs(tot);
      ctx->c.eigh_hot(ns, a.data(), ws.data(), vs.data(), pass == 1);
      long long o = 0, ow = 0;
      for (size_t i = 0; i < sel.size(); ++i) {
        const int k = sel[i];
        std::copy(vs.begin() + o, vs.begin() + o + (long long)nv[k] * nv[k], V + off[k]);
        std::copy(ws.begin() + ow, ws.begin() + ow + nv[k], w + woff[k]);
        o += (long long)nv[k] * nv[k];
        ow += nv[k];
      }
    }
  });
}


int fx_mlp_load(fx_ctx* ctx, const uint16_t* w, int64_t n) {
  if (!ctx || !w || n != FX_MLP_NW) return FX_E_INVALID;
  FX_GUARD(ctx, {
    std::vector<float> f(FX_MLP_NW);
    for (int i = 0; i < FX_MLP_NW; ++i) {
      const uint32_t u = (uint32_t)w[i] << 16;
      std::memcpy(&f[i], &u, 4);
    }
    ctx->c.mlp_set_master(f.data());
  });
}

int fx_mlp_save(fx_ctx* ctx, uint16_t* out, int64_t n) {
  if (!ctx || !out || n != FX_MLP_NW) return FX_E_INVALID;
  FX_GUARD(ctx, {
    if (!ctx->c.mlp_loaded) throw fx::FxError(FX_E_STATE, "no guess model loaded");
    std::vector<float> f;
    ctx->c.mlp_wr.download(f, ctx->c.stream, FX_MLP_NW);
    ctx->c.sync();
    for (int i = 0; i < FX_MLP_NW; ++i) {
      uint32_t u;
      std::memcpy(&u, &f[i], 4);
      out[i] = (uint16_t)(u >> 16);
    }
  });
}

int fx_mlp_set_master(fx_ctx* ctx, const float* w, int64_t n) {
  if (!ctx || !w || n != FX_MLP_NW) return FX_E_INVALID;
  FX_GUARD(ctx, ctx->c.mlp_set_master(w));
}

int fx_mlp_get_master(fx_ctx* ctx, float* w, int64_t n) {
  if (!ctx || !w || n != FX_MLP_NW) return FX_E_INVALID;
  FX_GUARD(ctx, {
    if (!ctx->c.mlp_loaded) throw fx::FxError(FX_E_STATE, "no guess model loaded");
    ctx->c.mlp_master.download_raw(w, FX_MLP_NW, ctx->c.stream);
    ctx->c.sync();
  });
}

int fx_mlp_features(fx_ctx* ctx, float* d_features) {
  if (!ctx || !d_features) return FX_E_INVALID;
  FX_GUARD(ctx, {
    ctx->c.mlp_features(d_features);
    ctx->c.sync();
  });
}

int fx_mlp_infer(fx_ctx* ctx, const float* d_features, float* d_out, int64_t n) {
  if (!ctx || !d_features || !d_out || n < 0) return FX_E_INVALID;
  FX_GUARD(ctx, {
    ctx->c.mlp_infer(d_features, d_out, n);
    ctx->c.sync();
  });
}

int fx_mlp_grad(fx_ctx* ctx, const float* d_features, const float* d_labels, int64_t n, double* loss, float* grad) {
  if (!ctx || !d_features || !d_labels || n <= 0) return FX_E_INVALID;
  FX_GUARD(ctx, {
    const double L = ctx->c.mlp_grad_impl(d_features, d_labels, n);
    if (loss) *loss = L;
    if (grad) {
      ctx->c.mlp_grad.download_raw(grad, FX_MLP_NW, ctx->c.stream);
      ctx->c.sync();
    }
  });
}

int fx_mlp_train_step(fx_ctx* ctx, const float* d_features, const float* d_labels, int64_t n, float lr,
                      double* loss) {
  if (!ctx || !d_features || !d_labels || n <= 0 || !(lr > 0.0f)) return FX_E_INVALID;
  FX_GUARD(ctx, {
    fx::Ctx& c = ctx->c;
    const double L = c.mlp_grad_impl(d_features, d_labels, n);
    c.mlp_t += 1;
    hipLaunchKernelGGL(fx::k_mlp_adam, dim3((FX_MLP_NW + 255) / 256), dim3(256), 0, c.stream, c.mlp_master.p,
                       c.mlp_m.p, c.mlp_v.p, c.mlp_grad.p, c.mlp_t, lr, c.mlp_wr.p);
    fx::Ctx::check(hipGetLastError(), "k_mlp_adam");
    c.sync();
    if (loss) *loss = L;
  });
}

}  // extern "C"
