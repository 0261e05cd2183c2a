// Host driver of the FMO2 and FMO3 analytic gradients: explicit fragment terms, the
// inter-fragment kernel derivatives, the response of the self-consistent
// embedding and the CN chain (section "Analytic energy gradients").  The
// host only builds index tables and launches kernels; per-atom sums are
// gathered on the device in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <unordered_map>
#include <vector>

#include "fx_host.hpp"
#include "fx_kernels.hpp"

namespace fx {

namespace {

// explicit per-system terms of one batch into (g_sys, F_sys); with boundary
// atoms also the projector derivative (its hybrid-coefficient forces into
// hop_f from slot slot_base on)
void explicit_terms(Ctx& c, Batch& b, const double* wsys, DevBuf<double>& g_sys, DevBuf<double>& F_sys,
                    double* hop_f, long long slot_base) {
  DevBatch db = b.dev();
  DevSystem ds = c.dev_system();
  DevBuf<double> wvec;
  wvec.alloc(b.tot_ao);
  hipLaunchKernelGGL(k_final_shift, dim3(b.nsys), dim3(256), 0, c.stream, ds, db, wvec.p);
  const int nt = (b.max_nao + 31) / 32;
  std::vector<int> all(b.nsys);
  for (int k = 0; k < b.nsys; ++k) all[k] = k;
  b.d_list.upload(all);
  // W = C diag(n eps) C^T into T (symmetric; over the orbitals of the last
  // occupation list, whose weights n eps vanish with n), D_S into F
  std::vector<int> all_sys(b.nsys);
  for (int k = 0; k < b.nsys; ++k) all_sys[k] = k;
  c.gemm_batch(b, db, (int)b.nsys, b.d_list.p, 2, b.Ct.p, b.Ct.p, b.Tm.p, (const double*)wvec.p,
               b.gemm_gflop_occ(all_sys), 0, 1, true);
  hipLaunchKernelGGL(k_make_DS, dim3(b.nsys), dim3(256), 0, c.stream, db, b.Pm.p, b.Tm.p, b.Fm.p);
  if (b.has_hop)
    hipLaunchKernelGGL(k_hop_grad, dim3(b.nsys), dim3(256), 0, c.stream, ds, db, (const double*)b.Pm.p, b.Fm.p, wsys,
                       (const int*)c.d_bonds.p, c.P.g.VHOP, slot_base, hop_f);
  int natot = 0;
  for (auto& d : b.h_desc) natot += d.nat;
  g_sys.alloc(3LL * natot);
  F_sys.alloc(natot);
  hipLaunchKernelGGL(k_grad_contract, dim3(b.nsys), dim3(256), 0, c.stream, ds, db, b.d_list.p, b.Pm.p, b.Fm.p,
                     b.q_out.p, b.q_out.p, wsys, 1, 0, g_sys.p, F_sys.p, b.Tm.p);
  Ctx::check(hipGetLastError(), "explicit gradient terms");
}

// CSR map global shell -> local shell slots of a cluster batch, in batch
// order (a counting sort of the batch's host shell map)
void cluster_csr(Ctx& c, Batch& b, DevBuf<int>& ptr, DevBuf<int>& ent) {
  const std::vector<int>& shg = b.h_sh_global;
  std::vector<int> cnt(c.Nsh + 1, 0), e(std::max<size_t>(1, shg.size()));
  for (int g : shg) ++cnt[g + 1];
  for (int s = 0; s < c.Nsh; ++s) cnt[s + 1] += cnt[s];
  std::vector<int> pos(cnt.begin(), cnt.end() - 1);
  for (int k = 0; k < (int)shg.size(); ++k) e[pos[shg[k]]++] = k;
  ptr.upload(cnt);
  ent.upload(e);
}

}  // namespace

void Ctx::gradient() {
  const double t0 = now_ms();
  DevSystem ds = dev_system();
  const long long nscc = (long long)scc_pairs.size() / 2;
  const long long ntri = opt.order >= 3 ? (long long)trimers.size() / 3 : 0;
  // ---- weights of the energy identity: monomers c_I, SCC dimers
  //      s_IJ = 1 - n_T(IJ), trimers 1; an ES-DIM sub-pair of a trimer
  //      (bit of tmask) takes one unit of its dq gamma dq term away
  std::vector<double> cw(F, 1.0), sw(std::max(1LL, nscc), 1.0);
  std::vector<int> tmask(std::max(1LL, ntri), 0);
  {
    std::unordered_map<long long, long long> sidx;
    for (long long k = 0; k < nscc; ++k) {
      const int I = scc_pairs[2 * k], J = scc_pairs[2 * k + 1];
      sidx[(long long)I * F + J] = k;
      cw[I] -= 1.0;
      cw[J] -= 1.0;
    }
    for (long long t = 0; t < ntri; ++t) {
      const int f[3] = {trimers[3 * t], trimers[3 * t + 1], trimers[3 * t + 2]};
      const int sub[3][2] = {{0, 1}, {0, 2}, {1, 2}};
      int nscc_of[3] = {0, 0, 0};
      for (int b = 0; b < 3; ++b) {
        const int a = sub[b][0], c = sub[b][1];
        auto it = sidx.find((long long)f[a] * F + f[c]);
        if (it != sidx.end()) {
          sw[it->second] -= 1.0;
          ++nscc_of[a];
          ++nscc_of[c];
        } else {
          tmask[t] |= 1 << b;
        }
      }
      for (int a = 0; a < 3; ++a) cw[f[a]] += nscc_of[a] - 1.0;
    }
  }
  DevBuf<double> d_cw, d_sw;
  DevBuf<int> d_tmask;
  d_cw.upload(cw);
  d_sw.upload(sw);
  d_tmask.upload(tmask);

  // ---- explicit fragment terms and the per-cluster corrections of the
  //      all-pairs force pass; projector forces of boundary entries in
  //      slots: monomers, SCC dimers, then the monomers' response terms
  const long long n_hop_m = mb.n_hop, n_hop_d = nscc > 0 ? db_.n_hop : 0;
  const long long n_slots = 2 * n_hop_m + n_hop_d;
  DevBuf<double> hop_f, ghost_f, zero_f;
  hop_f.alloc(std::max(1LL, 6 * n_slots));
  check(hipMemsetAsync(hop_f.p, 0, sizeof(double) * std::max(1LL, 6 * n_slots), stream), "memset");
  const long long n_healed = nscc > 0 && !db_.h_healed_sh.empty() ? (long long)db_.h_healed_sh.size() : 0;
  ghost_f.alloc(std::max(1LL, 3 * n_healed));
  DevBuf<double> gm, Fm_, gd, Fd, gt, Ft;
  explicit_terms(*this, mb, d_cw.p, gm, Fm_, hop_f.p, 0);
  if (nscc > 0) {
    explicit_terms(*this, db_, d_sw.p, gd, Fd, hop_f.p, n_hop_m);
    DevBatch ddb = db_.dev();
    hipLaunchKernelGGL(k_grad_pair_corr, dim3(db_.nsys), dim3(128), 0, stream, ds, ddb, d_q.p, ddq_scc.p, d_sw.p,
                       (const int*)nullptr, gd.p, ghost_f.p);
    check(hipGetLastError(), "k_grad_pair_corr");
  }
  if (ntri > 0) {
    explicit_terms(*this, tb_, nullptr, gt, Ft, nullptr, 0);
    DevBatch dtb = tb_.dev();
    hipLaunchKernelGGL(k_grad_pair_corr, dim3(tb_.nsys), dim3(128), 0, stream, ds, dtb, d_q.p, ddq_tri.p,
                       (const double*)nullptr, d_tmask.p, gt.p, ghost_f.p);
    check(hipGetLastError(), "k_grad_pair_corr (trimers)");
  }

  // ---- accumulated charge transfer qbar = sum_SCC s_IJ ddq^IJ + sum_T ddq^T
  //      and the Lagrangian potential v = field_excl(qbar) - sum over the
  //      clusters containing K of their weighted cross-fragment potential
  DevBuf<double> qbar, v, u, a;
  qbar.alloc(Nsh);
  v.alloc(Nsh);
  u.alloc(Nsh);
  a.alloc(Nsh);
  check(hipMemsetAsync(qbar.p, 0, sizeof(double) * Nsh, stream), "memset");
  check(hipMemsetAsync(u.p, 0, sizeof(double) * Nsh, stream), "memset");
  check(hipMemsetAsync(v.p, 0, sizeof(double) * Nsh, stream), "memset");
  const unsigned gS = (unsigned)((Nsh + 255) / 256);
  DevBuf<int> dptr, dent, tptr, tent;
  DevBuf<double> ddq_w, vc_d, vc_t, fq, vc_gh;
  if (nscc > 0) {
    cluster_csr(*this, db_, dptr, dent);
    DevBatch ddb = db_.dev();
    ddq_w.alloc(db_.tot_sh);
    vc_d.alloc(db_.tot_sh);
    hipLaunchKernelGGL(k_scale_cluster, dim3(db_.nsys), dim3(64), 0, stream, ddb, d_sw.p, ddq_scc.p, ddq_w.p);
    hipLaunchKernelGGL(k_gather_csr, dim3(gS), dim3(256), 0, stream, Nsh, dptr.p, dent.p, ddq_w.p,
                       (const double*)nullptr, 1.0, qbar.p);
    // the ghosts of bonds healed in a dimer carry -q (eq. ctij_ghost)
    if (db_.has_healed)
      hipLaunchKernelGGL(k_healed_ct, dim3(db_.nsys), dim3(64), 0, stream, ddb, (const double*)d_sw.p,
                         (const double*)d_q.p, qbar.p);
    vc_gh.alloc(std::max(1LL, n_healed));
    hipLaunchKernelGGL(k_cluster_cross, dim3(db_.nsys), dim3(128), 0, stream, ds, ddb, ddq_w.p, (const double*)d_q.p,
                       (const double*)d_sw.p, vc_d.p, db_.has_healed ? vc_gh.p : (double*)nullptr);
  }
  if (ntri > 0) {
    cluster_csr(*this, tb_, tptr, tent);
    DevBatch dtb = tb_.dev();
    vc_t.alloc(tb_.tot_sh);
    hipLaunchKernelGGL(k_gather_csr, dim3(gS), dim3(256), 0, stream, Nsh, tptr.p, tent.p, ddq_tri.p,
                       (const double*)qbar.p, 1.0, qbar.p);
    hipLaunchKernelGGL(k_cluster_cross, dim3(tb_.nsys), dim3(128), 0, stream, ds, dtb, ddq_tri.p, (const double*)d_q.p,
                       (const double*)nullptr, vc_t.p, (double*)nullptr);
  }
  if (nscc > 0 || ntri > 0) {
    fq.alloc(Nsh);
    field(qbar.p, fq.p);
    check(hipMemcpyAsync(v.p, fq.p, sizeof(double) * Nsh, hipMemcpyDeviceToDevice, stream), "copy");
    if (nscc > 0) {
      hipLaunchKernelGGL(k_gather_csr, dim3(gS), dim3(256), 0, stream, Nsh, dptr.p, dent.p, vc_d.p,
                         (const double*)v.p, -1.0, v.p);
      if (db_.has_healed)
        hipLaunchKernelGGL(k_sub_healed, dim3(db_.nsys), dim3(64), 0, stream, db_.dev(), (const double*)vc_gh.p, v.p);
    }
    if (ntri > 0)
      hipLaunchKernelGGL(k_gather_csr, dim3(gS), dim3(256), 0, stream, Nsh, tptr.p, tent.p, vc_t.p,
                         (const double*)v.p, -1.0, v.p);
    check(hipGetLastError(), "lagrangian potential");
  }

  // ---- per-atom gather map (host side; built while the response kernels
  // run when there is a response phase)
  std::vector<int> rowptr, ent_b;
  std::vector<long long> ent_o;
  bool force_map_built = false;
  auto build_force_map = [&]() {
    rowptr.assign(N + 1, 0);
    // a ghost (extended atom N + k) sits on the detached atom of bond k: its
    // forces and CN sensitivity go to that atom's row.  Entries are listed
    // in a fixed order and then sorted stably by row (a counting sort), so
    // each row keeps that order and its sums are deterministic.
    auto row_of = [&](int A) { return A < N ? A : bonds[2 * (A - N)]; };
    struct Ent {
      int row, b;
      long long o;
    };
    std::vector<Ent> ents;
    auto add = [&](int row, int id, long long o) { ents.push_back({row, id, o}); };
    auto add_batch = [&](Batch& b, int id) {
      const std::vector<int>& at = b.h_atoms;
      for (int k = 0; k < b.nsys; ++k) {
        const SysDesc& d = b.h_desc[k];
        for (int a = 0; a < d.nat; ++a) add(row_of(at[d.atom_off + a]), id, d.atom_off + a);
      }
    };
    add_batch(mb, 0);
    if (nscc > 0) add_batch(db_, 1);
    if (ntri > 0) add_batch(tb_, 2);
    // opposite forces on the ghosts healed in the SCC dimers (batch 3)
    for (long long e = 0; e < n_healed; ++e) {
      const int t = db_.h_healed_sh[e];
      const int G = (int)(std::upper_bound(atom_sh0_g.begin(), atom_sh0_g.end(), t) - atom_sh0_g.begin()) - 1;
      add(row_of(G), 3, e);
    }
    // projector hybrid-coefficient forces (batch 4): attached atom, detached atom
    auto add_hop = [&](const Batch& b, long long base) {
      for (int e = 0; e < b.n_hop; ++e) {
        const int kb = b.h_hop_bond[e];
        add(bonds[2 * kb + 1], 4, 2 * (base + e));
        add(bonds[2 * kb], 4, 2 * (base + e) + 1);
      }
    };
    add_hop(mb, 0);
    if (nscc > 0) add_hop(db_, n_hop_m);
    if (opt.want_response && (nscc > 0 || ntri > 0)) add_hop(mb, n_hop_m + n_hop_d);
    for (const Ent& e : ents) ++rowptr[e.row + 1];
    for (int A = 0; A < N; ++A) rowptr[A + 1] += rowptr[A];
    std::vector<int> pos(rowptr.begin(), rowptr.end() - 1);
    ent_b.resize(ents.size());
    ent_o.resize(ents.size());
    for (const Ent& e : ents) {
      const int k = pos[e.row]++;
      ent_b[k] = e.b;
      ent_o[k] = e.o;
    }
    force_map_built = true;
  };

  // ---- response of the monomer charges (adjoint of the self-consistency)
  if (opt.want_response && (nscc > 0 || ntri > 0)) {
    const double tr = now_ms();
    Batch& b = mb;
    DevBatch dmb = b.dev();
    std::vector<int> nocc(b.nsys);
    std::vector<long long> qoff(b.nsys + 1, 0);
    for (int k = 0; k < b.nsys; ++k) {
      const SysDesc& d = b.h_desc[k];
      int ne = (int)std::lround(d.nel);
      if (std::fabs(d.nel - ne) > 1e-9 || (ne & 1))
        throw FxError(FX_E_UNSUPPORTED, "the response term needs closed-shell monomers");
      nocc[k] = ne / 2;
      qoff[k + 1] = qoff[k] + (long long)d.nsh * nocc[k] * (d.nao - nocc[k]);
    }
    DevBuf<int> d_nocc, order;
    d_nocc.upload(nocc);
    DevBuf<long long> d_qoff;
    d_qoff.upload(qoff);
    DevBuf<double> Q, M, R, Wk, G1, G2, G3, w, y, yn, ul, gx;
    long long tot_gam = 0;
    for (auto& d : b.h_desc) tot_gam += (long long)d.nsh * d.nsh;
    if (!resp_ok) {
      order.alloc(b.tot_ao);
      Q.alloc(qoff[b.nsys]);
      M.alloc(tot_gam);
    }
    R.alloc(tot_gam);
    Wk.alloc(tot_gam);
    G1.alloc(b.tot_mat);
    G2.alloc(b.tot_mat);
    G3.alloc(b.tot_mat);
    w.alloc(b.tot_sh);
    y.alloc(b.tot_sh);
    ul.alloc(b.tot_sh);
    gx.alloc(b.tot_sh);
    std::vector<int> all(b.nsys);
    for (int k = 0; k < b.nsys; ++k) all[k] = k;
    b.d_list.upload(all);
    const int nt = (b.max_nao + 31) / 32;
    // the susceptibility blocks of the converged monomer orbitals are kept
    // from the monomer loop when available
    const int* p_order = order.p;
    const double* p_Q = Q.p;
    const double* p_M = M.p;
    if (resp_ok) {
      p_order = resp_order.p;
      p_Q = resp_Q.p;
      p_M = resp_M.p;
    } else {
      hipLaunchKernelGGL(k_mo_order, dim3(b.nsys), dim3(256), 0, stream, dmb, d_nocc.p, order.p);
      // (SC)^T = Ct S into G1
      gemm_batch(b, dmb, (int)b.nsys, b.d_list.p, 0, b.Ct.p, b.S.p, G1.p, (const double*)nullptr,
                 b.gemm_gflop_all());
      hipLaunchKernelGGL(k_resp_Q, dim3(b.nsys), dim3(256), (unsigned)resp_Q_lds_bytes(b.max_nao), stream, ds, dmb,
                         G1.p, order.p, d_nocc.p, d_qoff.p, Q.p);
      launch_resp_M(b, dmb, order.p, d_nocc.p, d_qoff.p, Q.p, M.p);
    }
    int nsmax = 0;
    for (const auto& dd : b.h_desc) nsmax = std::max(nsmax, dd.nsh);
    const size_t rr_bytes = (size_t)nsmax * (size_t)((nsmax + 1) & ~1) * sizeof(double);
    if (nsmax <= MAXN_RESP_LDS && (long long)rr_bytes <= lds_max - 24576)
      hipLaunchKernelGGL(k_resp_R_lds, dim3(b.nsys), dim3(RR_THREADS), rr_bytes, stream, ds, dmb, p_M, R.p);
    else
      hipLaunchKernelGGL(k_resp_R, dim3(b.nsys), dim3(256), 0, stream, ds, dmb, p_M, Wk.p, R.p);
    check(hipGetLastError(), "response setup");
    // adjoint sweeps y = v + field_excl(u(y)), Anderson-accelerated
    DevBuf<double> yg, yng, hX, hR, hC, fu;
    yg.alloc(Nsh);
    yng.alloc(Nsh);
    fu.alloc(Nsh);
    hX.alloc((long long)HIST * Nsh);
    hR.alloc((long long)HIST * Nsh);
    hC.alloc(HIST);
    check(hipMemcpyAsync(yg.p, v.p, sizeof(double) * Nsh, hipMemcpyDeviceToDevice, stream), "copy");
    std::vector<int> slots;
    int next_slot = 0;
    const unsigned gN = (unsigned)((Nsh + 255) / 256);
    double delta = 1e300;
    int it = 0;
    // mixed precision: FP32 field passes while the sweeps still change y by
    // more than 1e-6, FP64 from then on (the fixed point is the FP64 one; the
    // tolerance is only tested on FP64 sweeps)
    bool field32 = opt.precision == FX_MIXED;
    bool resp_converged = false;
    const int max_sweeps = opt.max_response;
    // the FP32 sweeps end after a quarter of the allowed sweeps at the latest
    const int max_fp32_sweeps = std::max(1, max_sweeps / 4);
    for (it = 1; it <= max_sweeps; ++it) {
      hipLaunchKernelGGL(k_gather_shell, dim3(b.nsys), dim3(64), 0, stream, dmb, yg.p, y.p);
      hipLaunchKernelGGL(k_resp_apply, dim3(b.nsys), dim3(256), 0, stream, dmb, R.p, p_M, y.p, w.p, ul.p);
      hipLaunchKernelGGL(k_scatter_shell, dim3(b.nsys), dim3(64), 0, stream, dmb, ul.p, u.p);
      field(u.p, fu.p, field32);
      hipLaunchKernelGGL(k_axpy, dim3(gN), dim3(256), 0, stream, (long long)Nsh, v.p, 1.0, fu.p, yng.p);
      max_absdiff(yng.p, yg.p, Nsh, d_scalar.p);
      std::vector<double> hs(1);
      d_scalar.download(hs, stream, 1);
      sync();
      delta = hs[0];
      if (verbose) std::fprintf(stderr, "[fx] response sweep %d: max |dy| = %.3e\n", it, delta);
      if (field32 && (delta < 1e-6 || it >= max_fp32_sweeps)) {
        field32 = false;
        slots.clear();
        next_slot = 0;
      } else if (!field32 && delta < response_tol) {
        resp_converged = true;
        break;
      }
      int slot;
      if ((int)slots.size() < HIST) {
        slot = next_slot++;
      } else {
        slot = slots.front();
        slots.erase(slots.begin());
      }
      slots.push_back(slot);
      hipLaunchKernelGGL(k_hist_store, dim3(gN), dim3(256), 0, stream, yg.p, yng.p, (long long)Nsh, slot, hX.p, hR.p);
      Slots sl;
      sl.m = (int)slots.size();
      for (int k = 0; k < sl.m; ++k) sl.id[k] = slots[k];
      hist_coef(hR.p, (long long)Nsh, sl, hC.p);
      hipLaunchKernelGGL(k_hist_mix, dim3(gN), dim3(256), 0, stream, hX.p, hR.p, (long long)Nsh, sl, hC.p, 1.0,
                         yg.p);
      check(hipGetLastError(), "response mixing");
    }
    response_sweeps = std::min(it, max_sweeps);
    if (!resp_converged) {
      res.converged = 0;
      if (verbose) std::fprintf(stderr, "[fx] response not converged after %d sweeps (max |dy| = %.3e)\n",
                                max_sweeps, delta);
    }
    // final w, u from the converged y
    hipLaunchKernelGGL(k_gather_shell, dim3(b.nsys), dim3(64), 0, stream, dmb, yng.p, y.p);
    hipLaunchKernelGGL(k_resp_apply, dim3(b.nsys), dim3(256), 0, stream, dmb, R.p, p_M, y.p, w.p, ul.p);
    hipLaunchKernelGGL(k_scatter_shell, dim3(b.nsys), dim3(64), 0, stream, dmb, ul.p, u.p);
    // Z and its AO forms
    hipLaunchKernelGGL(k_resp_Z, dim3(b.nsys), dim3(256), 0, stream, dmb, p_order, d_nocc.p, d_qoff.p, p_Q, w.p,
                       G2.p, G3.p);
    // Zt = Ct^T (Zm Ct) -> G1 ; WZ = Ct^T (Ze Ct) -> G2
    gemm_batch(b, dmb, (int)b.nsys, b.d_list.p, 0, G2.p, b.Ct.p, b.Tm.p, (const double*)nullptr, b.gemm_gflop_all());
    gemm_batch(b, dmb, (int)b.nsys, b.d_list.p, 2, b.Ct.p, b.Tm.p, G1.p, (const double*)nullptr, b.gemm_gflop_all());
    gemm_batch(b, dmb, (int)b.nsys, b.d_list.p, 0, G3.p, b.Ct.p, b.Tm.p, (const double*)nullptr, b.gemm_gflop_all());
    gemm_batch(b, dmb, (int)b.nsys, b.d_list.p, 2, b.Ct.p, b.Tm.p, G2.p, (const double*)nullptr, b.gemm_gflop_all());
    // X2 = P S (D_w P) -> G3
    hipLaunchKernelGGL(k_rowscale, dim3(b.nsys), dim3(256), 0, stream, dmb, w.p, b.Pm.p, b.Fm.p);
    gemm_batch(b, dmb, (int)b.nsys, b.d_list.p, 0, b.S.p, b.Fm.p, b.Tm.p, (const double*)nullptr, b.gemm_gflop_all());
    gemm_batch(b, dmb, (int)b.nsys, b.d_list.p, 0, b.Pm.p, b.Tm.p, G3.p, (const double*)nullptr, b.gemm_gflop_all());
    hipLaunchKernelGGL(k_sym_inplace, dim3(b.nsys), dim3(256), 0, stream, dmb, G1.p);
    hipLaunchKernelGGL(k_resp_DS, dim3(b.nsys), dim3(256), 0, stream, dmb, G1.p, G2.p, G3.p, w.p, b.Fm.p, gx.p);
    // the projector derivative with the Z-vector density (eq. hop_resp)
    if (b.has_hop)
      hipLaunchKernelGGL(k_hop_grad, dim3(b.nsys), dim3(256), 0, stream, ds, dmb, (const double*)G1.p, b.Fm.p,
                         (const double*)nullptr, (const int*)d_bonds.p, P.g.VHOP, n_hop_m + n_hop_d, hop_f.p);
    hipLaunchKernelGGL(k_grad_contract, dim3(b.nsys), dim3(256), 0, stream, ds, dmb, b.d_list.p, G1.p, b.Fm.p, gx.p,
                       b.q_out.p, (const double*)nullptr, 0, 1, gm.p, Fm_.p, b.Tm.p);
    check(hipGetLastError(), "response gradient terms");
    build_force_map();  // host work while the queued kernels run
    sync();
    res.ms_response = now_ms() - tr;
  }

  // ---- per-atom gather: F, CN chain, inter-fragment forces, fragment terms
  if (!force_map_built) build_force_map();
  DevBuf<int> d_rp, d_eb;
  DevBuf<long long> d_eo;
  d_rp.upload(rowptr);
  d_eb.upload(ent_b);
  d_eo.upload(ent_o);
  // batches 3 and 4 carry forces only: their CN sensitivities read zeros
  zero_f.alloc(std::max(1LL, std::max(n_healed, 2 * n_slots)));
  check(hipMemsetAsync(zero_f.p, 0, sizeof(double) * std::max(1LL, std::max(n_healed, 2 * n_slots)), stream),
        "memset");
  std::vector<const double*> gb = {gm.p, nscc > 0 ? gd.p : gm.p, ntri > 0 ? gt.p : gm.p, ghost_f.p, hop_f.p};
  std::vector<const double*> fb = {Fm_.p, nscc > 0 ? Fd.p : Fm_.p, ntri > 0 ? Ft.p : Fm_.p, zero_f.p, zero_f.p};
  DevBuf<const double*> d_gb, d_fb;
  d_gb.upload(gb);
  d_fb.upload(fb);
  DevBuf<double> Ftot;
  Ftot.alloc(N);
  d_grad.alloc(3LL * N);
  const unsigned gA = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL(k_gather_atoms, dim3(gA), dim3(256), 0, stream, N, d_rp.p, d_eb.p, d_eo.p, d_gb.p, d_fb.p,
                     d_grad.p, Ftot.p, 0);
  {
    const int nchunk = std::max(1, std::min(64, 2048 / (int)gA));
    DevBuf<double> part;
    part.alloc((long long)nchunk * 3 * N);
    hipLaunchKernelGGL(k_cn_grad, dim3(gA, nchunk), dim3(256), 0, stream, ds, Ftot.p, nchunk, part.p);
    hipLaunchKernelGGL(k_force_reduce, dim3((unsigned)((3 * N + 255) / 256)), dim3(256), 0, stream, N, nchunk, part.p,
                       d_grad.p);
  }
  // inter-fragment kernel derivatives with a = qbar + u
  hipLaunchKernelGGL(k_axpy, dim3((unsigned)((Nsh + 255) / 256)), dim3(256), 0, stream, (long long)Nsh, qbar.p, 1.0,
                     u.p, a.p);
  {
    // over the extended atoms (ghosts included), then every ghost's force
    // onto its detached atom
    const unsigned gE = (unsigned)((Ne + 255) / 256);
    const int nchunk = std::max(1, std::min(64, 2048 / (int)gE));
    DevBuf<double> part, fi;
    part.alloc((long long)nchunk * 3 * Ne);
    fi.alloc(3LL * Ne);
    hipLaunchKernelGGL(k_force_inter, dim3(gE, nchunk), dim3(256), 0, stream, ds, d_q.p, a.p, nchunk, part.p);
    hipLaunchKernelGGL(k_force_reduce, dim3((unsigned)((3 * Ne + 255) / 256)), dim3(256), 0, stream, Ne, nchunk,
                       part.p, fi.p);
    hipLaunchKernelGGL(k_add_ext_forces, dim3(gA), dim3(256), 0, stream, N, NB, (const int*)d_bonds.p,
                       (const double*)fi.p, d_grad.p);
  }
  hipLaunchKernelGGL(k_gather_atoms, dim3(gA), dim3(256), 0, stream, N, d_rp.p, d_eb.p, d_eo.p, d_gb.p, d_fb.p,
                     d_grad.p, Ftot.p, 1);
  check(hipGetLastError(), "gradient assembly");
  sync();
  if (verbose) std::fprintf(stderr, "[fx] gradient: %.1f ms (response %.1f ms, %d sweeps)\n", now_ms() - t0,
                            res.ms_response, response_sweeps);
}

}  // namespace fx
