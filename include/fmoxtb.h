/*
 * fmoxtb.h -- C ABI of the MI355X (gfx950) FMO-xTB library.
 *
 * The library computes the fragment molecular orbital energy and analytic
 * gradient of a molecular system at the GFN1-xTB level, following the paper
 * "FMO-xTB: Fragment molecular orbital method with GFN1-xTB":
 *   - section "GFN1-xTB" (eqs. gfn1-energy .. gfn1_rep_energy, cn_def):
 *     the tight-binding Hamiltonian of every fragment calculation;
 *   - section "Fragment molecular orbital method" (eqs.
 *     fmo2-energy-components, dimer_embedding_correction, ddq_calc,
 *     esdimer-energy, fmo3_energy, trimer_interaction_energy,
 *     trimer_embedding): the many-body energy;
 *   - section "FMO-xTB" (eq. v_esp_matrix and the monomer self-consistency
 *     it describes): the electrostatic embedding;
 *   - section "Analytic energy gradients" (eqs. grad_decomp .. response_grad_full)
 *     and its subsection "Extension to FMO3": the FMO2 and FMO3 gradients
 *     including the response of the embedding.
 *
 * Conventions shared by every call
 *   - Units: bohr for lengths, Hartree for energies, Eh/bohr for gradients.
 *   - Charges: shell Mulliken charges dq = population - reference population
 *     (electron excess), one value per shell, shells ordered atom by atom
 *     (global atom order) and, within an atom, in parameter-file order.
 *   - Fragment lists: pairs (I, J) with I < J in lexicographic order, trimers
 *     (I, J, K) with I < J < K in lexicographic order, int32.
 *   - All pointers in this header are HOST pointers; the library copies inputs
 *     and results between host and its own device memory.  The caller keeps
 *     ownership of every buffer it passes.
 *   - Return codes: FX_OK on success, a negative FX_E_* code otherwise; the
 *     message of the last error of a context is available from
 *     fx_last_error().  No C++ exception crosses this boundary.
 *   - A context is not thread-safe; independent contexts are.  Work runs on
 *     the HIP stream given at creation; every call returns after that stream
 *     has finished the call's work.
 */
#ifndef FMOXTB_H
#define FMOXTB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FX_OK = 0,
  FX_E_INVALID = -1,      /* bad argument, NaN coordinate, atoms closer than 0.3 bohr */
  FX_E_NOMEM = -2,        /* device allocation failed */
  FX_E_DEVICE = -3,       /* HIP runtime error */
  FX_E_NOCONV = -4,       /* an SCC or the monomer loop did not converge; results readable */
  FX_E_STATE = -5,        /* call out of order (e.g. fx_run before fx_set_system) */
  FX_E_UNSUPPORTED = -6   /* element or shell type missing from the parameters */
};

enum { FX_FP64 = 0, FX_MIXED = 1 };           /* precision */
/* schedule of the fragment solves:
 * FX_BATCHED launches each SCC iteration over all still-active systems of a
 *   kind.  The active list is compacted on the device after every iteration
 *   (systems still iterating first); the next iteration is launched at once,
 *   over as many slots as the latest count that has come back to the host,
 *   and the host waits for a count only when two iterations are already in
 *   flight behind it (FP64 solves with the split eigensolver; the others
 *   run as FX_BATCHED_HOST_SYNC).
 * FX_BATCHED_HOST_SYNC compacts the active list on the host and
 *   synchronises once per iteration.
 * FX_PLAIN_LOOP solves one system at a time.
 * FX_BATCHED_GRAPH captures the iteration over all systems of a solve once
 *   into a hipGraph and replays it (converged systems skip themselves on the
 *   device), after an eager first iteration.
 * All four give bitwise identical results. */
enum { FX_BATCHED = 0, FX_PLAIN_LOOP = 1, FX_BATCHED_GRAPH = 2, FX_BATCHED_HOST_SYNC = 3 };
enum { FX_GUESS_SUPERPOSITION = 0, FX_GUESS_LEARNED = 1, FX_GUESS_USER = 2 };
/* fragment-pair selection (section "Computational Details"): a fixed
 * closest-contact cutoff, or van der Waals-scaled contacts */
enum { FX_SELECT_CUTOFF = 0, FX_SELECT_VDW = 1 };

typedef struct fx_params fx_params;
typedef struct fx_ctx fx_ctx;

typedef struct fx_options {
  int32_t order;          /* 2 (FMO2) or 3 (FMO3) */
  double cutoff_bohr;     /* FX_SELECT_CUTOFF: a pair is an SCC dimer when its
                             closest interatomic distance is below this value,
                             otherwise ES-DIM; a trimer is computed when at
                             least two of its three pairs are SCC dimers */
  int32_t precision;      /* FX_FP64, or FX_MIXED: while an SCC residual is
                             above 1e-4, the Fock matrix is assembled in FP32
                             from FP32 copies of H0 and S and the congruence
                             product C^T F C and the density product
                             C diag(n) C^T run on the FP32 matrix cores with
                             FP32 accumulation (systems of more than 32 AOs
                             without cut bonds); the embedding-field passes
                             are FP32 while the monomer charges move by more
                             than 1e-6.  The basis, the eigensolver, the last
                             SCC iterations, the energies and the pair
                             differences stay FP64, so results keep the FP64
                             tolerances.  In both forms the Jacobi working
                             matrix of systems too large for an FP64 copy in
                             LDS (more than about 180 AOs) is stored in FP32
                             between FP64 rebuilds of C^T F C. */
  int32_t schedule;       /* FX_BATCHED (device-compacted active lists),
                             FX_BATCHED_HOST_SYNC, FX_BATCHED_GRAPH or
                             FX_PLAIN_LOOP (one fragment at a time) */
  int32_t guess;          /* initial monomer charges: superposition (zero),
                             the learned model (fx_mlp_load) or the charges
                             given with fx_set_guess */
  double guess_tau;       /* learned guess: a monomer whose first SCC
                             residual exceeds guess_tau restarts from
                             superposition charges (<= 0: never) */
  int32_t guess_max_iter; /* learned guess: a monomer not converged after this
                             many iterations of its first solve restarts from
                             superposition charges (<= 0: never) */
  double scc_tol;         /* SCC convergence: max |dq_out - dq_in| */
  double energy_tol;      /* SCC convergence: |E_k - E_(k-1)| */
  double macro_tol;       /* monomer loop: max change of any monomer charge */
  int32_t max_iter;       /* SCC iterations per fragment solve */
  int32_t max_macro;      /* monomer self-consistency sweeps */
  int32_t want_gradient;  /* compute the FMO2 or FMO3 analytic gradient
                             (FMO2 also with cut bonds: the derivative of
                             the energy plus the projector term sum_X w_X
                             Tr(P_X V^HOP_X), section "FMO-xTB HOP gradient";
                             FMO3 with cut bonds: FX_E_UNSUPPORTED) */
  int32_t want_response;  /* include the embedding response term */
  int32_t selection;      /* FX_SELECT_CUTOFF (default) or FX_SELECT_VDW */
  double vdw_dimer;       /* FX_SELECT_VDW: a pair is an SCC dimer when some
                             atom pair a in I, b in J is closer than
                             vdw_dimer * (r_a + r_b), r the element's van der
                             Waals radius (parameter file); default 2.0 */
  double vdw_trimer;      /* FX_SELECT_VDW: a trimer is computed when at least
                             two of its three pairs meet the same test with
                             vdw_trimer; default 1.5 */
  int32_t warm_clusters;  /* 1: an SCC dimer that was also solved in the last
                             fx_run on this system (same fragments, other
                             coordinates, e.g. the previous molecular-dynamics
                             step) starts from that run's converged charges
                             and orbitals (the orbitals re-orthonormalised in
                             the new overlap) instead of the monomers'; the
                             fixed point is the same.  Default 0; fx_md_verlet
                             sets it for its steps. */
  int32_t max_response;   /* sweeps of the adjoint response equation of the
                             gradient (default 400); a run whose response
                             has not reached its tolerance by then returns
                             FX_E_NOCONV (gradient still readable) */
  int32_t scc_retry;      /* 1 (default): an SCC dimer or trimer that has not
                             converged within max_iter is solved again from
                             where it stopped, first with plain Anderson
                             mixing without the Newton preconditioner and a
                             damping of 0.2 (FP64 products), then, if still
                             unconverged, at a tenfold electronic temperature
                             followed by a warm solve at the nominal one; each
                             stage allows max(max_iter, 200) iterations.  The
                             fixed point is the same.  0: none (the run then
                             returns FX_E_NOCONV). */
} fx_options;

typedef struct fx_counts {
  int64_t n_scc_pairs;
  int64_t n_esd_pairs;
  int64_t n_trimers;
  int32_t n_shells;       /* shells of the whole system */
  int32_t n_fragments;
} fx_counts;

/* Event-timed statistics of one kernel over a fx_run call: summed device
 * time of its launches (HIP events recorded on the context stream around each
 * launch), launch count and algorithmic work in GFLOP:
 *   fx::k_jacobi_lds<float|double>, fx::k_jacobi   6 n^2 (n - 1) per sweep
 *   fx::k_gemm_mfma, fx::k_gemm                      2 n^3 per product
 *   fx::k_field_sym,         8 per ordered inter-fragment shell pair (one
 *   fx::k_field_partial      rsqrt, the distance shared by an atom pair's
 *                            shells); the symmetric form evaluates each
 *                            unordered pair once and uses it both ways */
#define FX_MAX_KSTAT 8
typedef struct fx_kernel_stat {
  char name[48];          /* kernel name as rocprofv3 prints it, without arguments */
  double ms;
  int64_t launches;
  double gflop;
} fx_kernel_stat;

typedef struct fx_result {
  double e_total;         /* FMO2 or FMO3 energy */
  double e_fmo2;          /* FMO2 part of it */
  int32_t converged;      /* 1 if every solve and the monomer loop converged */
  int32_t macro_iter;     /* monomer self-consistency sweeps used */
  int64_t solves_mono, solves_dimer, solves_trimer;  /* fragment SCC solves */
  int64_t iters_mono, iters_dimer, iters_trimer;     /* SCC iterations, summed */
  double ms_lists, ms_monomer, ms_dimer, ms_trimer, ms_energy, ms_gradient, ms_response;
  int64_t guess_fallbacks;      /* monomers restarted from superposition charges */
  double first_residual_median; /* median over monomers of the first SCC
                                   residual max|dq_out - dq_in| of the first solve */
  /* device time of the hot kernels, largest first (see fx_kernel_stat) */
  int32_t n_kstat;
  fx_kernel_stat kstat[FX_MAX_KSTAT];
  int64_t warm_dimers;    /* SCC dimers started from the last run (warm_clusters) */
  int64_t device_allocs;  /* hipMalloc calls made by this fx_run (0 with a
                             workspace, and 0 without one once the buffers of
                             the same system and options already exist) */
  int64_t iters_fp32;     /* FX_MIXED: SCC iterations (summed over systems)
                             that ran the FP32 Fock build and products */
  int64_t scc_retries;    /* SCC dimers and trimers solved again by the
                             automatic retry (scc_retry) */
} fx_result;

/* Caller-owned device memory (the PyTorch wrapper passes a uint8 tensor).
 *
 * fx_workspace_size: *bytes = the workspace size that the calls made on this
 * context since its creation (or since its last fx_set_workspace) need: the
 * peak of the library's first-fit layout of its device buffers, tracked also
 * while the library allocates with hipMalloc, plus a margin of 1/32 of it and
 * 4 MiB (launch shapes chosen by timing can change a few buffer sizes between
 * otherwise identical calls).  Typical use: fx_set_system and fx_run once
 * without a workspace, query the size, allocate it, call fx_set_workspace,
 * then fx_set_system again and run; repeating the same calls fits.
 *
 * fx_set_workspace: dev_ptr is DEVICE memory on the context's device, at
 * least 256-byte aligned, `bytes` long; the caller keeps ownership and must
 * keep it alive until the context is destroyed or given another workspace.
 * The context is first reset to its state after fx_ctx_create (its system,
 * lists, results and learned-guess weights are dropped; options are kept),
 * then every device buffer it creates is carved from the workspace and the
 * library calls no hipMalloc or hipFree.  dev_ptr = NULL with bytes = 0
 * returns to library allocation (also a reset).  A call that needs more than
 * the workspace fails with FX_E_NOMEM and names the size reached.
 * Errors: FX_E_INVALID (misaligned or empty workspace), FX_E_DEVICE. */
int fx_workspace_size(fx_ctx* ctx, size_t* bytes);
int fx_set_workspace(fx_ctx* ctx, void* dev_ptr, size_t bytes);

/* Load element constants and STO-nG basis expansions from a JSON file.
 * *out is owned by the caller; release with fx_params_free.
 * Errors: FX_E_INVALID (unreadable or malformed file). */
int fx_params_load(const char* json_path, fx_params** out);
void fx_params_free(fx_params* p);

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * (NULL: the default stream); it must outlive the context.  The parameters
 * are copied.  Errors: FX_E_INVALID, FX_E_DEVICE. */
int fx_ctx_create(const fx_params* p, int device, void* hip_stream, fx_ctx** out);
void fx_ctx_destroy(fx_ctx* ctx);
/* Message of the last error on this context ("" if none); owned by the context. */
const char* fx_last_error(const fx_ctx* ctx);

/* Fill *o with defaults: order 2, cutoff 4 Angstrom, FP64, batched,
 * superposition guess, scc_tol 1e-10, energy_tol 1e-11, macro_tol 1e-10,
 * max_iter 200, max_macro 200, gradient and response on. */
int fx_default_options(fx_options* o);
int fx_set_options(fx_ctx* ctx, const fx_options* o);

/* Set the molecular system.  Z[n_atoms] atomic numbers, xyz_bohr[3*n_atoms]
 * Cartesian coordinates, atom_frag[n_atoms] fragment index of each atom
 * (0..n_frag-1, every fragment non-empty), frag_charge[n_frag] net charges.
 * Fragments are molecules (section "Energy accuracy") or pieces of a
 * covalent chain: bonds[2*n_bonds] lists the covalent bonds cut by the
 * fragmentation as (detached atom, attached atom) pairs (section "Covalent
 * bond fragmentation"): the detached atom keeps its fragment and gives one
 * electron to the bond; a ghost copy of it joins the attached atom's fragment
 * with one electron; hybrid-orbital projectors (V_HOP) constrain both sides.
 * n_bonds = 0 (bonds may be NULL) for molecular fragments.  The detached atom
 * must have one s and one p shell.  Inputs are copied.
 * With cut bonds the shell vectors of fx_get_charges / fx_set_guess hold the
 * ghost shells after those of the real atoms (one ghost per bond, in bond
 * order); the FMO2 gradient acts on real atoms only (a ghost's forces go to
 * its detached atom); the FMO3 gradient and molecular dynamics with cut bonds
 * return FX_E_UNSUPPORTED.
 * Errors: FX_E_INVALID (bad sizes, NaN, atoms closer than 0.3 bohr, empty
 * fragment, bond index out of range or inside one fragment),
 * FX_E_UNSUPPORTED (element without parameters, detached atom without s and
 * p shells). */
int fx_set_system(fx_ctx* ctx, int32_t n_atoms, const int32_t* Z, const double* xyz_bohr,
                  int32_t n_frag, const int32_t* atom_frag, const int32_t* frag_charge,
                  int32_t n_bonds, const int32_t* bonds);

/* Classify fragment pairs (and trimers for order 3) by closest contact
 * (section "Computational Details" selection rule, fixed cutoff reading) on
 * the GPU and report the counts.  Distances are compared as squared FP64
 * values formed as (dx*dx + dy*dy) + dz*dz without fused multiply-add.
 * Errors: FX_E_STATE (no system). */
int fx_build_lists(fx_ctx* ctx, fx_counts* out);
/* Counts of the current lists (built by fx_build_lists or by fx_run); no
 * GPU work.  Errors: FX_E_STATE if no lists exist yet. */
int fx_get_counts(fx_ctx* ctx, fx_counts* out);
/* Copy the lists into caller buffers sized from fx_counts: scc_pairs[2*n_scc],
 * esd_pairs[2*n_esd], trimers[3*n_tri] (any pointer may be NULL to skip). */
int fx_get_lists(fx_ctx* ctx, int32_t* scc_pairs, int32_t* esd_pairs, int32_t* trimers);

/* Initial monomer shell charges dq_shell[n_shells] (host, n_shells from
 * fx_counts; copied) used with FX_GUESS_USER, e.g. the previous step's
 * fx_get_charges in molecular dynamics (the fixed point of the monomer loop
 * does not depend on the start; section "FMO-xTB").  fx_set_system resets the guess to
 * zero.  FX_E_STATE without a system, FX_E_INVALID for a non-finite value. */
int fx_set_guess(fx_ctx* ctx, const double* dq_shell);

/* New atomic positions xyz_bohr[3*n_atoms] (host, copied) for the system of
 * the last fx_set_system: same atoms, fragments and cut bonds.  Lists and all
 * geometry-dependent tables are rebuilt; the charges given with fx_set_guess
 * are kept.  Errors as fx_set_system for the coordinates, FX_E_STATE without a
 * system. */
int fx_set_coordinates(fx_ctx* ctx, const double* xyz_bohr);

/* Molecular dynamics with the analytic gradient (the paper's motivation for
 * it, sections "Analytic energy gradients" and "Conclusion"): n_steps steps
 * of velocity Verlet of length dt, in atomic units throughout (bohr, electron
 * masses mass[n_atoms], time in hbar/Eh = 0.0241888 fs, velocities in
 * bohr per hbar/Eh):
 *   x <- x + v dt - grad E / (2 m) dt^2;  v <- v - (grad E_old + grad E_new) / (2 m) dt.
 * xyz_bohr and vel [3*n_atoms] hold the start on entry and the end on return
 * (host).  e_pot and e_kin [n_steps + 1] (host, may be NULL) receive the
 * FMO energy and the kinetic energy at every step, the start included.  The
 * energy and gradient use the current options (order, selection, precision,
 * response; the gradient is always computed); the first step starts from the
 * option's guess, every later step from the previous step's converged monomer
 * charges.  Lists are rebuilt at every step.  On return the context holds the
 * last geometry and its results (fx_get_energies, fx_get_gradient).  Errors:
 * FX_E_INVALID (n_steps < 0, dt <= 0, masses <= 0, non-finite input),
 * FX_E_STATE (no system), FX_E_UNSUPPORTED (cut bonds), FX_E_NOCONV (a step
 * did not converge; xyz_bohr and vel are then unchanged). */
int fx_md_verlet(fx_ctx* ctx, int32_t n_steps, double dt, const double* mass, double* xyz_bohr, double* vel,
                 double* e_pot, double* e_kin);

/* Run the FMO calculation: lists (if not built), supersystem CN, the monomer
 * self-consistency loop, dimer (and trimer) SCC solves in the converged
 * embedding, ES-DIM pairs, the energy and, if requested, the FMO2 or FMO3
 * gradient.
 * Blocks until done.  Returns FX_E_NOCONV (results still readable) when a
 * solve hit max_iter or the monomer loop hit max_macro. */
int fx_run(fx_ctx* ctx, fx_result* out);

/* Per-fragment energies of the last run: E_mono[n_frag] internal monomer
 * energies (embedding acts in the Fock matrix only), dE_scc[n_scc] SCC pair
 * interaction energies Delta E_IJ (eq. fmo2-energy-components), dE_esd[n_esd]
 * ES-DIM pair energies (eq. esdimer-energy), dE_tri[n_tri] trimer corrections
 * Delta E_IJK - Delta E_IJ - Delta E_IK - Delta E_JK (eq. fmo3_energy).
 * Buffers are sized from fx_get_counts after the run; NULL pointers are
 * skipped. */
int fx_get_energies(fx_ctx* ctx, double* E_mono, double* dE_scc, double* dE_esd, double* dE_tri);
/* Converged monomer shell charges dq_shell[n_shells]. */
int fx_get_charges(fx_ctx* ctx, double* dq_shell);
/* FMO2 / FMO3 gradient grad[3*n_atoms] (Eh/bohr) of the last run.
 * Errors: FX_E_STATE if the last run did not compute it. */
int fx_get_gradient(fx_ctx* ctx, double* grad);

/* ---- component entry points (single hot-path steps, for validation) ---- */

/* Supersystem coordination numbers cn[n_atoms] (eq. cn_def, no cutoff). */
int fx_compute_cn(fx_ctx* ctx, double* cn);

/* Overlap S and zeroth-order Hamiltonian H0 (eq. h0_hamiltonian with
 * eqs. xtb1_polynomial_correction, xtb1_diagonal_h0) of the cluster made of
 * fragments frags[0..nfrag-1] (1 to 3, basis in that fragment order, atoms of
 * a fragment in ascending global order).  S and H0 are row-major nao x nao,
 * nao written to *nao_out; pass S = H0 = NULL to query nao only. */
int fx_cluster_matrices(fx_ctx* ctx, int32_t nfrag, const int32_t* frags, int32_t* nao_out,
                        double* S, double* H0);

/* Electrostatic embedding field of eq. v_esp_matrix on every shell:
 * phi[s] = sum over shells t of other fragments of gamma_st * dq[t], for the
 * given shell charges dq[n_shells].  With precision FX_MIXED in the options
 * the pass of the mixed-precision form runs (FP32 distances, reciprocal
 * square roots and sums within a source chunk, chunk sums added in FP64);
 * otherwise the FP64 pass. */
int fx_embedding_field(fx_ctx* ctx, const double* dq, double* phi);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the field
 * of fx_embedding_field (FP64) with DEVICE pointers d_dq[n_shells] (input
 * shell charges) and d_phi[n_shells] (output), both owned by the caller.  It
 * calls no hipMalloc, hipFree or allocating routine: its partial sums live in
 * a static device array of FX_NOALLOC_SCRATCH_DOUBLES doubles (8 MiB) that
 * every GPU the library runs on holds until the process ends.  The work is
 * enqueued on the context's stream and the call returns without waiting;
 * d_phi is complete when that stream reaches this point.  Calls that overlap
 * on one GPU (other threads or streams, any context) share the array and
 * race.  Errors: FX_E_STATE (no system), FX_E_INVALID (NULL pointer, or a
 * system with more than FX_NOALLOC_SCRATCH_DOUBLES shells), FX_E_DEVICE. */
#define FX_NOALLOC_SCRATCH_DOUBLES (1 << 20)
int fx_embedding_field_noalloc(fx_ctx* ctx, const double* d_dq, double* d_phi);

/* Batched symmetric eigensolver used by the SCC, as the SCC runs it: the
 * LDS-resident Jacobi of a cold solve (working matrix in FP64 where it fits
 * in LDS, else FP32 with FP64 angles and eigenvectors), run to convergence,
 * then one warm iteration (A' = V A V^T rebuilt in FP64 on the matrix cores,
 * the rotation kernel on the LDS working matrix, the apply kernel on V);
 * matrices smaller than 8 (no SCC system is) and sizes without an LDS plan
 * use a global-memory Jacobi.  nmat matrices of
 * sizes n[k] (each <= 512), packed one after another row-major in A (sum
 * n[k]^2 doubles).  Writes eigenvalues w (sum n[k], unsorted) and
 * eigenvectors as rows of V (same packing as A: row i of matrix k is
 * eigenvector i). */
int fx_eigh_batched(fx_ctx* ctx, int32_t nmat, const int32_t* n, const double* A, double* w,
                    double* V);

/* ------------------------------------------------------------------------
 * Learned initial monomer charges (not part of the paper; its SCC starts
 * from superposition charges).  Per real atom: 20 features (one-hot H, C, N,
 * O and 16 radial symmetry functions sum_j exp(-eta (R_ij - Rs_k)^2) fc(R_ij)
 * over atoms within 6 Angstrom, Rs_k = 0.5 .. 6 Angstrom evenly spaced,
 * eta = 1/(2 * 0.35^2) Angstrom^-2, fc = (cos(pi R / 6 A) + 1) / 2), and a
 * 20 -> 64 -> 64 -> 2 perceptron (tanh hidden units) giving the atom's two
 * shell charges.  The forward pass rounds weights and features to bfloat16
 * (nearest even) and accumulates in FP32.  Each fragment's guess is shifted
 * uniformly over its real shells to sum to minus its net charge; ghost
 * shells start at zero.  Weight vector (FX_MLP_NW values): W1[64][20], b1[64],
 * W2[64][64], b2[64], W3[2][64], b3[2].  Training keeps FP32 master weights
 * and Adam moments in the context (beta1 0.9, beta2 0.999, eps 1e-8); the
 * loss is the mean squared error over atoms and both shells, its gradient is
 * taken with respect to the bfloat16-rounded weights.
 * ------------------------------------------------------------------------ */
#define FX_MLP_NW 5634
#define FX_MLP_NFEAT 20

/* Load bfloat16 weights (host, n = FX_MLP_NW raw bfloat16 bit patterns) as
 * the master weights; resets the Adam state.  Errors: FX_E_INVALID. */
int fx_mlp_load(fx_ctx* ctx, const uint16_t* bf16_weights, int64_t n);
/* The master weights rounded to bfloat16 (host, n = FX_MLP_NW). */
int fx_mlp_save(fx_ctx* ctx, uint16_t* bf16_out, int64_t n);
/* FP32 master weights in / out (host, n = FX_MLP_NW); set resets Adam. */
int fx_mlp_set_master(fx_ctx* ctx, const float* w, int64_t n);
int fx_mlp_get_master(fx_ctx* ctx, float* w, int64_t n);
/* Features of the real atoms of the current system into DEVICE memory
 * d_features[n_atoms][FX_MLP_NFEAT] (FP32, computed in FP64).  Errors:
 * FX_E_STATE (no system). */
int fx_mlp_features(fx_ctx* ctx, float* d_features);
/* Forward pass on n feature rows (DEVICE pointers): d_out[n][2].  Errors:
 * FX_E_STATE (no weights loaded). */
int fx_mlp_infer(fx_ctx* ctx, const float* d_features, float* d_out, int64_t n);
/* Loss and its gradient on n rows (DEVICE features and labels [n][2]);
 * loss and grad[FX_MLP_NW] returned to host memory (grad may be NULL). */
int fx_mlp_grad(fx_ctx* ctx, const float* d_features, const float* d_labels, int64_t n, double* loss,
                float* grad);
/* One Adam step of learning rate lr on n rows (DEVICE pointers); *loss
 * (host, may be NULL) is the loss before the step. */
int fx_mlp_train_step(fx_ctx* ctx, const float* d_features, const float* d_labels, int64_t n, float lr,
                      double* loss);

#ifdef __cplusplus
}
#endif

#endif /* FMOXTB_H */
