// Device-side data layout shared by the HIP kernels and the host driver.
//
// Atoms, shells and AOs of the supersystem are stored structure-of-arrays in
// HBM.  A "system" is one fragment calculation (monomer, dimer or trimer);
// every system owns dense row-major nao x nao matrices in per-batch pools and
// per-shell / per-AO vectors, located through SysDesc offsets.
#pragma once

#include <cstdint>

namespace fx {

constexpr int MAXSH_EL = 2;   // shells per element (minimal s/p basis)
constexpr int NPRIM = 6;      // STO-6G
constexpr int MAXAO_EL = 4;   // AOs per element
constexpr int HIST = 8;       // Anderson mixing memory
constexpr int MAXN = 512;     // largest system (AOs) handled by the SCC kernels

struct DevElem {
  int Z;
  int nsh, nao;
  int l[MAXSH_EL], nao_sh[MAXSH_EL], ao0[MAXSH_EL];
  double level[MAXSH_EL], kcn[MAXSH_EL], kpoly[MAXSH_EL], eta[MAXSH_EL], q0[MAXSH_EL];
  double alpha[MAXSH_EL][NPRIM], coef[MAXSH_EL][NPRIM];
  int orth;                 // second s shell orthogonalised against the first
  double orthN, orthS12;    // |s2'> = N (|s2> - S12 |s1>)
  double EN, rcov, Gamma, zeff, arep;
  double rvdw;              // van der Waals radius (bohr) of the pair selection rule; 0 if not given
};

struct DevGlobals {
  double kg, kf, kEN, k1, k2, kl[3], KAB, kT, VHOP;
};

struct SysDesc {
  int nat, nsh, nao, nfrag;
  int atom_off;   // into sys_atoms / sys_atom_ao0 / sys_atom_sh0
  int sh_off;     // into per-system shell vectors
  int ao_off;     // into per-system AO vectors
  int frag[3];
  int comp_sh[4];     // local shell offset of each fragment's block (comp_sh[nfrag] = nsh)
  long long mat_off;  // into n x n pools
  long long gam_off;  // into the nsh x nsh gamma pool
  double nel;
};

// History slots of a mixing scheme, oldest first.
struct Slots {
  int m;
  int id[HIST];
};

// Read-only supersystem tables.
struct DevSystem {
  int natoms, nshells, nfrag;
  int nreal;              // real atoms (the first nreal); the rest are ghosts
  const double* xyz;      // [3N]
  const int* elem;        // [N] element table index
  const int* frag;        // [N]
  const int* atom_sh0;    // [N+1] first global shell of each atom
  const double* cn;       // [N]
  const int* sh_atom;     // [Nsh]
  const int* sh_frag;     // [Nsh]
  const double* sh_eta;   // [Nsh] (1 + kappa) eta_A
  const double* sh_ieta;  // [Nsh] 1 / (2 (1 + kappa) eta_A): 1/eta_st = ieta_s + ieta_t
  const DevElem* elems;
  DevGlobals g;
};

// Per-batch tables and pools.
struct DevBatch {
  int nsys;
  const SysDesc* desc;
  const int* sys_atoms;     // global atom of each local atom
  const int* sys_atom_ao0;  // local AO offset of each local atom
  const int* sys_atom_sh0;  // local shell offset of each local atom
  const int* sys_sh_global; // global shell of each local shell
  const int* sys_sh_atom;   // local atom of each local shell
  const int* sys_ao_sh;     // local shell of each local AO
  double* S;
  double* H0;
  double* F;     // Fock matrix, then the projected matrix C^T F C
  double* Ct;    // eigenvectors as rows
  double* P;
  double* T;     // GEMM scratch
  double* gam;   // nsh x nsh gamma of the system
  double* q_in;
  double* q_out;
  double* phi;   // external shell potential
  double* sig;   // shell shift of the last Fock build
  const float* pre;  // nsh x nsh mixing preconditioner per system (gam offsets, stored transposed) or null
  const double* sh_q0;     // per local shell reference population (null: element values)
  const double* atom_zs;   // per local atom repulsion-charge scale (null: 1)
  double* Vh;              // HOP projector S D S per system (mat layout) or null
  const int* hop_bond;     // cut bond (index into the system's bond list) of each boundary entry
  const int* hop_off;      // [nsys+1] boundary atoms of each system
  const int* hop_atom;
  const int* hop_kind;     // 1 detached atom, 2 ghost
  const double* hop_b;     // [3] unit bond vector per entry
  const int* healed_off;   // [nsys+1] ghosts healed inside each system (or null)
  const int* healed_sh;    // their global shells
  const int* sh_mono;      // per local shell: its index within its fragment's monomer
  double* hx;    // Anderson history of inputs  [sh_off*HIST + k*nsh + s]
  double* hr;    // Anderson history of residuals
  double* eps;
  double* occ;
  double* erep;
  double* e_int;
  double* e_prev;
  double* mts;   // -T S of the last density
  double* err;   // max |q_out - q_in| of the last iteration
  int* status;   // 0 active, 1 converged, 2 failed
  int* niter;
  int* nhist;
  int* occ_idx;  // [ao_off + k]: the orbitals whose occupation exceeds OCC_MIN, ascending
  int* occ_cnt;  // per system: their number
};
// occupations below this bound are left out of the density product: each
// such term changes an element of P by less than 1e-30, far below the FP64
// rounding of any element that matters
constexpr double OCC_MIN = 1e-30;

// gamma_st at distance R (Klopman-Ohno form, eta_st the harmonic mean)
__device__ inline double gamma_pair(const DevGlobals& g, double R, double eta_s, double eta_t) {
  const double ie = 0.5 * (1.0 / eta_s + 1.0 / eta_t);
  if (g.kg == 2.0) return 1.0 / sqrt(R * R + ie * ie);
  return pow(pow(R, g.kg) + pow(ie, g.kg), -1.0 / g.kg);
}

// 1/sqrt(x) for positive finite x (the damped Coulomb kernels, where
// x = R^2 + c^2 with c > 0): the hardware estimate y followed by one step of
// the series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ..., e = 1 - x y^2, which
// triples the number of correct bits; no handling of zero, infinite or NaN
// arguments, which these callers never pass.
__device__ inline double rsqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}


// Maximum (minimum) over a whole wave (every lane active), returned in every
// lane: DPP row shifts leave each row's extreme in its lane 15, row
// broadcasts carry those to lane 63.
#define FX_WAVE_REDUCE(op, ctrl, rmask) v = op(v, dpp_as(v, __builtin_amdgcn_update_dpp(dpp_bits(v), dpp_bits(v), ctrl, rmask, 0xf, false)))
#define FX_WAVE_REDUCE_ALL(op) \
  FX_WAVE_REDUCE(op, 0x111, 0xf); \
  FX_WAVE_REDUCE(op, 0x112, 0xf); \
  FX_WAVE_REDUCE(op, 0x114, 0xf); \
  FX_WAVE_REDUCE(op, 0x118, 0xf); \
  FX_WAVE_REDUCE(op, 0x142, 0xa); \
  FX_WAVE_REDUCE(op, 0x143, 0xc)
__device__ inline int dpp_bits(int v) { return v; }
__device__ inline int dpp_bits(float v) { return __float_as_int(v); }
__device__ inline int dpp_as(int, int b) { return b; }
__device__ inline float dpp_as(float, int b) { return __int_as_float(b); }
__device__ inline float wave_max_f32(float v) {
  FX_WAVE_REDUCE_ALL(fmaxf);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ inline int wave_min_i32(int v) {
  FX_WAVE_REDUCE_ALL(min);
  return __builtin_amdgcn_readlane(v, 63);
}
__device__ inline int wave_max_i32(int v) {
  FX_WAVE_REDUCE_ALL(max);
  return __builtin_amdgcn_readlane(v, 63);
}
#undef FX_WAVE_REDUCE_ALL
#undef FX_WAVE_REDUCE

// Sum over a whole wave (every lane active), returned in every lane: the same
// tree, lanes without a source adding zero; a fixed order (deterministic)
template <int CTRL, int RMASK>
__device__ inline double dpp_or_zero(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, RMASK, 0xf, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, RMASK, 0xf, false));
}
template <int CTRL, int RMASK>
__device__ inline double dpp_or_self(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, CTRL, RMASK, 0xf, false),
                          __builtin_amdgcn_update_dpp(lo, lo, CTRL, RMASK, 0xf, false));
}
__device__ inline double wave_max_f64(double v) {
  v = fmax(v, dpp_or_self<0x111, 0xf>(v));
  v = fmax(v, dpp_or_self<0x112, 0xf>(v));
  v = fmax(v, dpp_or_self<0x114, 0xf>(v));
  v = fmax(v, dpp_or_self<0x118, 0xf>(v));
  v = fmax(v, dpp_or_self<0x142, 0xa>(v));
  v = fmax(v, dpp_or_self<0x143, 0xc>(v));
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}
__device__ inline double wave_sum_f64(double v) {
  v += dpp_or_zero<0x111, 0xf>(v);
  v += dpp_or_zero<0x112, 0xf>(v);
  v += dpp_or_zero<0x114, 0xf>(v);
  v += dpp_or_zero<0x118, 0xf>(v);
  v += dpp_or_zero<0x142, 0xa>(v);
  v += dpp_or_zero<0x143, 0xc>(v);
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}

// List slot and tile of work-group L in a launch of xcd_grid(nl, tps)
// work-groups over nl systems of tps tiles each.  The dispatcher deals
// consecutive work-group ids to the 8 XCDs in turn; slot s runs on XCD s % 8
// with all of its tiles, so that each system's operands stay in one L2, and
// the leading slots (the systems still iterating, in a list compacted on the
// device) spread evenly over the XCDs whatever the launch's slot bound.
__device__ inline void xcd_slot_tile(int L, int tps, int& sl, int& tile) {
  const int x = L & 7, j = L >> 3;
  const int q = j / tps;
  tile = j - q * tps;
  sl = 8 * q + x;
}
}  // namespace fx
