// Host-side classes of the library: errors, device buffers, parameters,
// fragment batches and the context that drives a run.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <iterator>
#include <cmath>
#include <cstdlib>
#include <deque>
#include <map>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/fmoxtb.h"
#include "fx_device.hpp"

namespace fx {

struct FxError : std::runtime_error {
  int code;
  FxError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Device memory of one context.  Without a workspace every block comes from
// hipMalloc, and a freed block is kept in a cache keyed by its size and
// handed out again to a request it fits within 1/8 (repeated runs then call
// neither hipMalloc nor the synchronising hipFree); the cache is released
// when the context ends or takes a workspace.  With a caller-owned
// workspace every block is carved from it (first fit over 256-byte granules,
// freed neighbours merged) and hipMalloc is never called.  The first-fit
// layout is kept in both modes (in the first only as offsets), so the
// workspace size a sequence of calls needs is known from a run without one:
// replaying the same calls into a workspace of `peak` bytes reproduces the
// same layout.
struct DevMem {
  static constexpr size_t kAlign = 256;
  char* base = nullptr;  // workspace, or nullptr
  size_t size = 0;
  size_t top = 0;        // end of the highest block in use
  size_t peak = 0;       // largest `top` since the last reset
  long long hip_allocs = 0;
  std::map<size_t, size_t> free_;                                 // offset -> bytes below top
  std::unordered_map<void*, std::pair<size_t, size_t>> live;      // block -> (offset, bytes)
  std::multimap<size_t, void*> cache_;                             // freed hipMalloc blocks by size
  std::unordered_map<void*, size_t> hip_size_;                     // size of every hipMalloc block
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  ~DevMem() { release_cache(); }
  void release_cache() {
    for (auto& kv : cache_) {
      (void)hipFree(kv.second);
      hip_size_.erase(kv.second);
    }
    cache_.clear();
  }

  void* alloc(size_t bytes) {
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    size_t off = top;
    bool from_free = false;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        const size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        from_free = true;
        break;
      }
    }
    if (!from_free && base && top + bytes > size)
      throw FxError(FX_E_NOMEM, "workspace of " + std::to_string(size) + " bytes is too small (" +
                                    std::to_string(top + bytes) + " needed so far; fx_workspace_size reports the "
                                    "need after a run without a workspace)");
    void* p = nullptr;
    if (base) {
      p = base + off;
    } else {
      auto c = cache_.lower_bound(bytes);
      if (c != cache_.end() && c->first - bytes <= bytes / 8) {
        p = c->second;
        cache_.erase(c);
      } else {
        if (hipMalloc(&p, bytes) != hipSuccess) {
          if (from_free) give_back(off, bytes);
          throw FxError(FX_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
        ++hip_allocs;
        hip_size_[p] = bytes;
      }
    }
    if (!from_free) top += bytes;
    peak = std::max(peak, top);
    live[p] = {off, bytes};
    return p;
  }
  void free(void* p) {
    auto it = live.find(p);
    if (it == live.end()) return;
    const size_t off = it->second.first, bytes = it->second.second;
    live.erase(it);
    if (!base) {
      auto hs = hip_size_.find(p);
      if (hs != hip_size_.end())
        cache_.emplace(hs->second, p);
      else
        (void)hipFree(p);
    }
    give_back(off, bytes);
  }
  void give_back(size_t off, size_t bytes) {
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + bytes) {
      bytes += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        off = pv->first;
        bytes += pv->second;
        free_.erase(pv);
      }
    }
    if (off + bytes == top) {
      top = off;
    } else {
      free_[off] = bytes;
    }
  }
};

// the memory of the context whose call is running on this thread
extern thread_local DevMem* g_devmem;

// Sets g_devmem for the duration of a library call.
struct DevMemScope {
  DevMem* prev;
  explicit DevMemScope(DevMem* m) : prev(g_devmem) { g_devmem = m; }
  ~DevMemScope() { g_devmem = prev; }
};

// Owning device buffer; its memory comes from the context's DevMem (hipMalloc
// or the caller's workspace).
template <class T>
struct DevBuf {
  T* p = nullptr;
  long long n = 0;
  DevMem* mem = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), mem(o.mem), cap(o.cap) {
    o.p = nullptr;
    o.n = 0;
    o.cap = 0;
    o.mem = nullptr;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      cap = o.cap;
      mem = o.mem;
      o.p = nullptr;
      o.n = 0;
      o.cap = 0;
      o.mem = nullptr;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      if (mem)
        mem->free(p);
      else
        (void)hipFree(p);
    }
    p = nullptr;
    n = 0;
    cap = 0;
    mem = nullptr;
  }
  long long cap = 0;
  // keeps the allocation when it is already large enough (no new device
  // memory on repeated runs of the same system)
  void alloc(long long count) {
    if (p && count <= cap) {
      n = count;
      return;
    }
    release();
    size_t bytes = sizeof(T) * (size_t)(count > 0 ? count : 1);
    if (g_devmem) {
      p = static_cast<T*>(g_devmem->alloc(bytes));
      mem = g_devmem;
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      p = nullptr;
      throw FxError(FX_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    n = count;
    cap = count > 0 ? count : 1;
  }
  void upload(const std::vector<T>& v) {
    alloc((long long)v.size());
    if (!v.empty() && hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess)
      throw FxError(FX_E_DEVICE, "hipMemcpy H2D failed");
  }
  void upload_async(const std::vector<T>& v, hipStream_t s) {
    if ((long long)v.size() > n) alloc((long long)v.size());
    if (!v.empty() && hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s) != hipSuccess)
      throw FxError(FX_E_DEVICE, "hipMemcpyAsync H2D failed");
  }
  void download(std::vector<T>& v, hipStream_t s, long long count = -1) const {
    long long c = count < 0 ? n : count;
    v.resize((size_t)c);
    if (c > 0 && hipMemcpyAsync(v.data(), p, sizeof(T) * c, hipMemcpyDeviceToHost, s) != hipSuccess)
      throw FxError(FX_E_DEVICE, "hipMemcpyAsync D2H failed");
  }
  void download_raw(T* dst, long long count, hipStream_t s) const {
    if (count > 0 && hipMemcpyAsync(dst, p, sizeof(T) * count, hipMemcpyDeviceToHost, s) != hipSuccess)
      throw FxError(FX_E_DEVICE, "hipMemcpyAsync D2H failed");
  }
};

struct HostParams {
  DevGlobals g;
  std::vector<DevElem> elems;
  std::map<int, int> elem_of_Z;
};

HostParams load_params(const std::string& path);

struct Batch {
  int nsys = 0;
  int max_nao = 0;
  // what the tables were last built for (build_batch keeps them when the
  // same clusters of the same system come again)
  std::vector<std::array<int, 3>> h_clusters;
  int h_nfrag = 0;
  long long h_system_gen = -1;
  bool init_from_mono = false;  // first basis from the monomers' eigenvectors
  bool has_warm = false;        // some systems start from the previous run (warm_off >= 0)
  DevBuf<long long> warm_off;   // per system: C^T offset in the previous run's layout, or -1
  int tot_sh = 0, tot_ao = 0;
  long long tot_mat = 0;
  std::vector<SysDesc> h_desc;
  DevBuf<SysDesc> d_desc;
  DevBuf<int> d_atoms, d_atom_ao0, d_atom_sh0, d_sh_global, d_sh_atom, d_ao_sh, d_all, d_list;
  DevBuf<double> S, H0, Fm, Ct, Pm, Tm, gam, q_in, q_out, phi, sig, hx, hr, eps, occ;
  DevBuf<int> occ_idx, occ_cnt;  // significant orbitals of the last occupation (k_fermi)
  DevBuf<double> erep, e_int, e_prev, mts, err;
  DevBuf<int> status, niter, nhist, sweeps;
  // Newton preconditioner (1 + M G)^-1 of the Anderson residuals (FP32,
  // gam offsets, each block stored transposed); used by the mixer when has_pre is set
  DevBuf<float> pre;
  bool has_pre = false;
  // mixed precision: FP32 copies of H0 and S, the FP32 Fock matrix and the
  // FP32 intermediate of the congruence product (systems of more than 32 AOs
  // without hybrid-orbital projectors)
  DevBuf<float> H0f, Sf, Ff, Tf;
  bool has_f32 = false;
  // rotation log of the split eigensolver (k_jacobi_rot / k_apply_rot)
  DevBuf<double2> rotlog;
  DevBuf<int> nlog;
  // covalent boundaries: per local shell reference population, per local atom
  // repulsion-charge scale, boundary atoms (local atom, kind 1 detached /
  // 2 ghost, bond direction) and the ghosts healed inside each system
  bool has_hop = false, has_healed = false;
  DevBuf<double> sh_q0, atom_zs, hop_b, Vh;
  DevBuf<int> hop_off, hop_atom, hop_kind, hop_bond, healed_off, healed_sh, sh_mono;
  int n_hop = 0;  // boundary entries of the batch
  std::vector<int> h_hop_off, h_hop_bond, h_healed_off, h_healed_sh;  // host copies
  std::vector<int> h_sh_global;  // host copy of d_sh_global
  std::vector<int> h_atoms;      // host copy of d_atoms
  long long tot_gam = 0;
  DevBatch dev();
  // algorithmic work of one n x n product (2 n^3) summed over listed systems
  double gemm_gflop(const std::vector<int>& l) const {
    double g = 0.0;
    for (int s : l) g += 2e-9 * std::pow((double)h_desc[s].nao, 3);
    return g;
  }
  // the density product over the occupied orbitals only: 2 n^2 ceil(N_el / 2)
  double gemm_gflop_occ(const std::vector<int>& l) const {
    double g = 0.0;
    for (int s : l) {
      const double n = h_desc[s].nao, k = std::min(n, std::ceil(0.5 * h_desc[s].nel));
      g += 2e-9 * n * n * k;
    }
    return g;
  }
  // a symmetric product computes the upper 64 x 64 tiles only: 2 n^3 times
  // the fraction of tiles computed
  double gemm_gflop_sym(const std::vector<int>& l) const {
    double g = 0.0;
    for (int s : l) {
      const double n = h_desc[s].nao, nt = std::ceil(n / 64.0);
      g += 2e-9 * n * n * n * (nt * (nt + 1) / 2) / (nt * nt);
    }
    return g;
  }
  double gemm_gflop_all() const {
    double g = 0.0;
    for (const auto& d : h_desc) g += 2e-9 * std::pow((double)d.nao, 3);
    return g;
  }
};

// Event-timed accumulation of one kernel's launches on the context stream.
struct KernelTimer {
  std::string name;
  double ms = 0.0;
  long long launches = 0;
  double gflop = 0.0;
  void reset() {
    ms = 0.0;
    launches = 0;
    gflop = 0.0;
  }
};

// eigensolver choice for one batch (elt = 0: global-memory kernel)
struct JacobiPlan {
  int elt = 0, chunk = 0, threads = 0;
  unsigned lds = 0;
};

struct Ctx {
  ~Ctx() {
    if (gstream) (void)hipStreamDestroy(gstream);
    for (hipEvent_t e : cnt_ev)
      if (e) (void)hipEventDestroy(e);
    if (cnt_host) (void)hipHostFree(cnt_host);
  }
  HostParams P;
  int device = 0;
  hipStream_t stream = nullptr;
  fx_options opt{};
  std::string last_error;
  // numerical settings of the kernels
  int jacobi_max_sweeps = 40;
  double jacobi_tol = 1e-14;
  // rotations below thr_scale times the last SCC residual are skipped: at
  // 1e-3 the orbitals of an iteration were off by a few per cent of the
  // residual, which stalled the mixing of the slow dimers (C4: 43,497 dimer
  // iterations, at most 26 per dimer; at 1e-5: 38,555, at most 16)
  double jacobi_thr_scale = std::getenv("FX_JACOBI_THR_SCALE") ? std::atof(std::getenv("FX_JACOBI_THR_SCALE")) : 1e-5;
  double jacobi_cap_err = std::getenv("FX_JACOBI_CAP_ERR") ? std::atof(std::getenv("FX_JACOBI_CAP_ERR")) : 1e-9;
  // split eigensolver of clusters started from their monomers' orbitals:
  // jacobi_early_sweeps sweeps per SCC iteration while the residual exceeds
  // jacobi_early_err.  A single sweep left the first iterations' orbitals
  // inexact while the inter-fragment couplings were still large, which
  // slowed the mixing (C4 dimers, energy + gradient: 38,555 SCC iterations
  // with one sweep, 28,381 with two above 1e-3, 26,424 with converged
  // sweeps; step 0.451 -> 0.424 s)
  double jacobi_early_err = std::getenv("FX_JACOBI_EARLY_ERR") ? std::atof(std::getenv("FX_JACOBI_EARLY_ERR")) : 1e-3;
  int jacobi_early_sweeps = std::getenv("FX_JACOBI_EARLY_SWEEPS") ? std::atoi(std::getenv("FX_JACOBI_EARLY_SWEEPS")) : 2;
  int jacobi_threads = std::getenv("FX_JACOBI_THREADS") ? std::atoi(std::getenv("FX_JACOBI_THREADS")) : 1024;
  // LDS-resident eigensolver (k_jacobi_lds) where the system fits; FX_JACOBI_LDS=0
  // selects the global-memory kernel everywhere
  bool jacobi_lds = !(std::getenv("FX_JACOBI_LDS") && std::atoi(std::getenv("FX_JACOBI_LDS")) == 0);
  int lds_max = 65536;  // bytes of LDS one workgroup may allocate (queried)
  long long system_gen = 0;  // counts fx_set_system calls (batch tables depend on it)
  double mix_beta = 0.5;
  double macro_beta = 0.5;
  double scc_tol_cur = -1.0, etol_cur = -1.0;
  double response_tol = 1e-11;
  // mixed precision: FP32 products and Fock build while a system's SCC
  // residual is above mixed_thr.  prod_mode 0: FP64 products; 1: each system
  // of the solve runs FP32 iterations until its own residual drops to
  // mixed_thr, FP64 ones from then on
  double mixed_thr = std::getenv("FX_MIXED_THR") ? std::atof(std::getenv("FX_MIXED_THR")) : 1e-4;
  int prod_mode = 0;
  // clear a system's Anderson history when it leaves the FP32 phase (off: the
  // FP32 noise, about 1e-6 in the charges, is small against the 1e-4 residual
  // at the switch, and keeping the history saves iterations)
  bool mixed_hist_reset = std::getenv("FX_MIXED_HIST_RESET") && std::atoi(std::getenv("FX_MIXED_HIST_RESET")) != 0;
  int response_sweeps = 0;
  bool verbose = std::getenv("FX_VERBOSE") != nullptr;

  // supersystem
  bool has_system = false, lists_built = false, has_result = false, has_grad = false;
  // N real atoms; Ne = N + NB atoms with one ghost per cut covalent bond
  // (a copy of the detached atom in the attached atom's fragment)
  int N = 0, F = 0, Nsh = 0, NB = 0, Ne = 0;
  std::vector<int> bonds;                    // [NB][2] detached, attached
  std::vector<std::vector<int>> bda_bonds, ghost_bonds;  // per fragment
  std::vector<int> frag_off_real, frag_atoms_real;
  DevBuf<int> d_frag_atoms_real, d_frag_off_real, d_bonds;
  double field_pairs = 0.0;  // inter-fragment shell pairs of one field pass
  std::vector<int> elem, frag, frag_charge, frag_off, frag_atoms, atom_sh0_g;
  std::vector<double> xyz_h, guess;
  DevBuf<DevElem> d_elems;
  DevBuf<double> d_xyz, d_cn, d_sh_eta, d_sh_ieta, d_q, d_qnew, d_phi, d_scalar, field_part, d_grad;
  DevBuf<double> field_col;  // column partial sums of the symmetric field pass
  DevBuf<int> d_elem, d_frag, d_atom_sh0, d_sh_atom, d_sh_frag, d_frag_atoms, d_frag_off;

  // lists
  std::vector<int> scc_pairs, esd_pairs, trimers;

  // batches and results
  Batch mb, db_, tb_;
  DevBuf<double> e_mono, dE_scc, dEV_scc, dE_esd, dE_tri, ddq_scc, ddq_tri;
  // converged SCC dimers of the last run (warm_clusters): pair list, C^T and
  // charges in that run's batch layout
  bool warm_valid = false;
  std::vector<int> warm_pairs;
  std::vector<long long> warm_matoff, warm_shoff;
  DevBuf<double> warm_C, warm_q;  // last run's SCC dimer orbitals (C^T) and shell charges
  DevBuf<long long> warm_so;       // per dimer of this run: shell offset in warm_q, or -1
  DevBuf<double> d_dEIJK;  // Delta E_IJK of the trimers of the last run
  fx_result res{};
  // monomer susceptibility blocks (shell-summed transition charges Q and
  // M = sum_ai Q Q^T / (eps_a - eps_i)) of the current monomer orbitals
  DevBuf<int> resp_nocc, resp_order;
  DevBuf<long long> resp_qoff;
  DevBuf<double> resp_Q, resp_M;
  bool resp_ok = false;
  bool precond = !(std::getenv("FX_PRECOND") && std::atoi(std::getenv("FX_PRECOND")) == 0);
  double precond_beta = 1.0;
  // monomer loop: after the first full solve, one SCC iteration per monomer
  // per step with global (preconditioned) mixing of all monomer charges
  bool fused = !(std::getenv("FX_FUSED") && std::atoi(std::getenv("FX_FUSED")) == 0);
  double fused_beta = std::getenv("FX_FUSED_BETA") ? std::atof(std::getenv("FX_FUSED_BETA")) : 1.0;
  DevBuf<double> mono_tmp;
  bool monomer_response_setup();
  // dynamic LDS of k_resp_M for a batch (throws when a system is too large)
  unsigned resp_M_lds(const Batch& b) const;
  void launch_resp_M(const Batch& b, const DevBatch& db, const int* order, const int* nocc, const long long* qoff,
                     const double* Q, double* M);
  void build_precond(Batch& b);
  // learned initial guess: FP32 master weights, Adam moments, bfloat16-rounded copy
  DevBuf<float> mlp_master, mlp_m, mlp_v, mlp_wr, mlp_grad, mlp_part, mlp_feat, mlp_out;
  DevBuf<double> mlp_lpart, mlp_loss;
  int mlp_t = 0;
  bool mlp_loaded = false;
  void mlp_set_master(const float* w);
  void mlp_features(float* d_out);
  void mlp_infer(const float* d_x, float* d_y, long long n);
  double mlp_grad_impl(const float* d_x, const float* d_y, long long n);
  void learned_guess();
  // first monomer solve: record first-iteration residuals and apply the
  // learned-guess fallback
  bool first_solve = false;
  DevBuf<int> fallback_flag;
  std::deque<KernelTimer> ktimers;  // stable addresses
  KernelTimer* kt(const char* name) {
    for (auto& t : ktimers)
      if (t.name == name) return &t;
    ktimers.emplace_back();
    ktimers.back().name = name;
    return &ktimers.back();
  }
  // pool of HIP event pairs around kernel launches, resolved after a sync
  struct EventPool {
    std::vector<hipEvent_t> ev0, ev1;
    std::vector<KernelTimer*> who;
    std::vector<double> gf;
    int used = 0;
    int begin(hipStream_t s) {
      if (used == (int)ev0.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
          throw FxError(FX_E_DEVICE, "hipEventCreate failed");
        ev0.push_back(a);
        ev1.push_back(b);
        who.push_back(nullptr);
        gf.push_back(0.0);
      }
      if (hipEventRecord(ev0[used], s) != hipSuccess) throw FxError(FX_E_DEVICE, "hipEventRecord failed");
      return used++;
    }
    void end(hipStream_t s, int k, KernelTimer* t, double gflop) {
      if (hipEventRecord(ev1[k], s) != hipSuccess) throw FxError(FX_E_DEVICE, "hipEventRecord failed");
      who[k] = t;
      gf[k] = gflop;
    }
    void resolve() {
      for (int k = 0; k < used; ++k) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev0[k], ev1[k]) != hipSuccess) throw FxError(FX_E_DEVICE, "event time failed");
        who[k]->ms += ms;
        who[k]->launches += 1;
        who[k]->gflop += gf[k];
      }
      used = 0;
    }
  } timers;


  static void check(hipError_t e, const char* what);
  static double now_ms();
  void sync();
  DevSystem dev_system() const;
  void set_system(int32_t n_atoms, const int32_t* Z, const double* xyz, int32_t n_frag, const int32_t* atom_frag,
                  const int32_t* fchg, int32_t n_bonds, const int32_t* bonds);
  void build_lists_impl();
  void compute_cn();
  // max |a - b| over n entries into *out (device), and the Anderson mixing
  // coefficients of the history residuals R (slots sl, n entries each)
  DevBuf<double> red_part;
  void max_absdiff(const double* a, const double* b, int n, double* out);
  void hist_coef(const double* R, long long n, const Slots& sl, double* coef);
  void field(const double* d_q, double* d_phi, bool fp32 = false);
  void build_batch(Batch& b, const std::vector<std::array<int, 3>>& clusters, int nfrag_each);
  void build_matrices(Batch& b, bool from_mono = false);
  void eigh_hot(const std::vector<int>& nv, const double* A, double* w, double* V, bool global_kernel = false);
  void init_device();
  // embedding field through the chunked pass into caller-given device
  // buffers, partial sums in the library's static scratch (no allocation)
  void field_noalloc(const double* d_q, double* d_phi);
  JacobiPlan jacobi_plan(int n, bool fp64_only = false, bool prefer_fp32 = false) const;
  // autotuned eigensolver launch shapes per (size bucket, precision)
  bool autotune = !(std::getenv("FX_AUTOTUNE") && std::atoi(std::getenv("FX_AUTOTUNE")) == 0);
  // split eigensolver (rotation kernel + apply kernel) for single-sweep
  // iterations; FX_JACOBI_SPLIT=0 keeps the fused kernel everywhere
  bool jacobi_split = !(std::getenv("FX_JACOBI_SPLIT") && std::atoi(std::getenv("FX_JACOBI_SPLIT")) == 0);
  int jacobi_max_log = std::getenv("FX_JACOBI_MAX_LOG") ? std::atoi(std::getenv("FX_JACOBI_MAX_LOG")) : 2;
  // the cold eigensolve of a solve from the orthogonalised basis by the split
  // form too: passes of up to this many logged sweeps, each from a fresh
  // C^T F C, until every system has had a sweep without rotations
  // (FX_JACOBI_COLD_LOG=0: the fused kernel)
  int jacobi_cold_log = std::getenv("FX_JACOBI_COLD_LOG") ? std::atoi(std::getenv("FX_JACOBI_COLD_LOG")) : 8;
  std::map<long long, JacobiPlan> tuned;
  static long long jp_key(int n, int elt) { return (long long)n * 16 + elt; }
  // launch shape of the rotation kernel per size bucket: work-group size and
  // the persistent work-queue form (FX_JACOBI_ROT_THREADS and
  // FX_JACOBI_ROT_PERSISTENT force one; otherwise tuned by timing)
  struct RotShape {
    int threads = 0;
    bool persistent = false;
  };
  std::map<long long, RotShape> tuned_rot;
  int force_rot_threads = std::getenv("FX_JACOBI_ROT_THREADS") ? std::atoi(std::getenv("FX_JACOBI_ROT_THREADS")) : 0;
  int force_rot_persistent =
      std::getenv("FX_JACOBI_ROT_PERSISTENT") ? std::atoi(std::getenv("FX_JACOBI_ROT_PERSISTENT")) : -1;
  DevBuf<int> rot_queue;
  int n_cu = 1;
  // (max_log: sweeps the log holds per system; 0: jacobi_max_log)
  void launch_rot(const Batch& b, const DevBatch& db, const int* dl, int na, int elt, double cap, const RotShape& rs,
                  long long log_stride, int max_log = 0);
  // apply kernel with two quartets per lane for systems of 129 to 256 AOs
  // (FX_APPLY_DUAL=0: the one-quartet kernel everywhere)
  bool apply_dual_on = !(std::getenv("FX_APPLY_DUAL") && std::atoi(std::getenv("FX_APPLY_DUAL")) == 0);
  bool apply_dual(int max_nao) const { return apply_dual_on && max_nao > 128 && max_nao <= 256; }
  void launch_apply(const Batch& b, const DevBatch& db, const int* dl, int na, long long log_stride);
  RotShape rot_shape(Batch& b, const DevBatch& db, const int* dl, int na, const JacobiPlan& jp, double cap,
                     long long log_stride, bool may_tune);
  JacobiPlan autotune_jacobi(Batch& b, const int* dl, int na, const JacobiPlan& base, double cap);
  void gemm_batch(const Batch& b, const DevBatch& db, int nl, const int* dlist, int mode, const double* A,
                  const double* B, double* C, const double* w, double gflop, int skip_done = 0, int sym = 0,
                  bool occ_list = false, int win = 0);
  // the FP32 products of the mixed form (mode 0: double A, float B and C;
  // mode 1: float A, double B and C; mode 2: double A, B and C)
  void gemm_batch_f32(const Batch& b, const DevBatch& db, int nl, const int* dlist, int mode, const void* A,
                      const void* B, void* C, const double* w, double gflop, int skip_done, int sym, bool occ_list);
  // graph-captured SCC iterations (schedule FX_BATCHED_GRAPH)
  bool capturing = false;
  hipStream_t gstream = nullptr;
  // device-driven SCC iterations (schedule FX_BATCHED): the active list is
  // compacted on the device after every iteration; its count comes back
  // through a ring of pinned slots, each with an event, which the host polls
  // at most async_lag iterations behind the launches
  static constexpr int CNT_RING = 8;
  int async_lag = 2;
  int* cnt_host = nullptr;  // [CNT_RING], pinned
  std::vector<hipEvent_t> cnt_ev;
  DevBuf<int> cnt_dev;
  void count_ring_init();
  int run_scc(Batch& b, const std::vector<int>& list, bool cold, long long* iters_out, bool single = false);
  int solve_batch(Batch& b, bool cold, long long* iters_out);
  int retry_failed(Batch& b, long long* iters_out);
  // iteration cap of the damped retry stage (0: max(max_iter, 200));
  // FX_RETRY_DAMPED_ITERS lets a test force the second stage
  int retry_damped_iters = std::getenv("FX_RETRY_DAMPED_ITERS") ? std::atoi(std::getenv("FX_RETRY_DAMPED_ITERS")) : 0;
  void run(fx_result* out);
  void set_coordinates(const double* xyz);
  void md_verlet(int n_steps, double dt, const double* mass, double* xyz, double* vel, double* e_pot,
                 double* e_kin);
  void gradient();
};

// static device scratch of fx_embedding_field_noalloc: address lookup once per
// device (called from init_device with that device current) and the address
void noalloc_init(int device);
double* noalloc_scratch(int device);

}  // namespace fx

// the opaque context of the C ABI
struct fx_ctx {
  fx::DevMem mem;  // declared first: outlives every buffer of c
  fx::Ctx c;
};
