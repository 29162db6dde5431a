/*
 * afq.h -- C ABI of the MI355X (gfx950) phaseless-AFQMC walker-step library.
 *
 * The library implements the batched walker step of phaseless auxiliary-field
 * quantum Monte Carlo with a Cholesky-factorised two-electron tensor, for the
 * second-quantised Hamiltonian of Eq. eq:hamil in Section sec:afqmc
 * ("Auxiliary Field Quantum Monte Carlo") of arXiv 2003.01831:
 *
 *   H = sum_ij h_ij c+_i c_j + 1/2 sum_ijkl v_ijkl c+_i c+_j c_l c_k + E_II,
 *   v_ijkl = sum_n L^n_ik L^n*_lj   (the modified-Cholesky factorisation, the
 *                                    equation after eq:hamil in sec:afqmc)
 *
 * Cost model of the walk (Table tab:afqmc_comp, dense 3-index row):
 * propagation O(N M^2), energy O(x_c N^2 M^2) with X = x_c M vectors.
 *
 * Step equations (the paper cites them from the phaseless-AFQMC literature;
 * they follow from the two lines above by Wick's theorem and the
 * Hubbard-Stratonovich transformation):
 *   S^s = T^sH W^s, Theta^s = W^s (S^s)^-1, G^s = Theta^s T^sH,
 *   Omega^{ns} = Lt^{ns} Theta^s with Lt^{ns} = T^sH L^n (half rotation),
 *   vbar_n = sum_s tr Omega^{ns},
 *   E_L = E_II + sum_s tr(ht^s Theta^s) + 1/2 sum_n vbar_n^2
 *         - 1/2 sum_{n,s} tr(Omega^{ns} Omega^{ns}),   ht^s = T^sH h,
 *   xbar_n = -i sqrt(dt) vbar_n, A = i sqrt(dt) sum_n (x_n - xbar_n) L^n,
 *   W <- B1 T_K(A) B1 W,  B1 = exp(-dt h'/2),  h' = h - 1/2 sum_n L^n L^n,
 *   r = O'/O, I = r exp(sum_n x_n xbar_n - xbar_n^2/2) exp(dt E_shift),
 *   w <- w |I| max(0, cos arg r),  periodic thin QR of W (positive diag R).
 *
 * Conventions shared by every call
 *   - All array arguments of afq_step, afq_energy, afq_energy_backward,
 *     afq_walkers_get/set, afq_fields_generate and afq_batch_step are DEVICE
 *     pointers on the device that was current when the system was created
 *     (for instance torch.Tensor.data_ptr() of a CUDA tensor). The pointers
 *     of afq_walkers_create are device pointers too; those of
 *     afq_system_create are device pointers, or host pointers with the
 *     AFQ_HOST_PTRS flag.
 *   - Complex arrays are interleaved (re, im) float64 pairs, row-major.
 *   - Orbital matrices (trial, walkers) are M x (n_up + n_dn): up-spin
 *     columns first, then down-spin columns.
 *   - Work is enqueued on the HIP stream given to afq_system_create and is
 *     asynchronous unless stated otherwise; outputs are valid once that
 *     stream has been synchronised. The library never synchronises the
 *     device except in the create calls and afq_walkers_stats.
 *   - Every call returns an afq_status; on failure afq_last_error() gives a
 *     thread-local message. No C++ exception crosses the ABI.
 *   - Handles are not thread-safe: use one per thread.
 */
#ifndef AFQ_H
#define AFQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct afq_system_s *afq_system;
typedef struct afq_walkers_s *afq_walkers;
typedef struct afq_batch_s *afq_batch;

typedef enum {
  AFQ_OK = 0,
  AFQ_E_INVALID = -1,     /* bad shape, NULL pointer, bad argument value */
  AFQ_E_NOMEM = -2,       /* device allocation failed */
  AFQ_E_HIP = -3,         /* a HIP runtime call failed */
  AFQ_E_SINGULAR = -4,    /* initial walker overlap T^H W is singular */
  AFQ_E_STATE = -5,       /* handles that do not belong together */
  AFQ_E_UNSUPPORTED = -6  /* valid input outside what the library implements */
} afq_status;

/* Arithmetic of the contraction bulk (the Omega = Lt Theta exchange GEMM, the
 * A = sum_n c_n L^n build and the Taylor increments). The overlap inverse and
 * determinant, the phaseless ratio, the weights, QR and the walker orbitals
 * are FP64 in every mode. */
typedef enum {
  AFQ_FP64 = 0,   /* complex128 contractions on FP64 MFMA */
  AFQ_CFP32 = 1,  /* complex64 contractions on FP32 MFMA, FP32 accumulation */
  AFQ_BF16X3 = 2  /* split-BF16x3 (hi*hi + hi*lo + lo*hi) on BF16 MFMA for the
                     exchange GEMM, FP32 accumulation; complex64 elsewhere */
} afq_precision;

/* ------------------------------------------------------------------------ */
/* System: h1, L^n, the trial and E_II (Eq. eq:hamil and the Cholesky form).  */
/* ------------------------------------------------------------------------ */

/* afq_system_create flag: h1, chol and phi_t are host pointers (pageable or
 * pinned). Without it they are device pointers on the current device. */
#define AFQ_HOST_PTRS 1u

/* Creates a system from the one-body matrix h_ij and E_II of Eq. eq:hamil,
 * the Cholesky vectors L^n of the modified-Cholesky factorisation that
 * follows it (Section sec:afqmc; real symmetric L^n, so v_ijkl =
 * sum_n L^n_ik L^n_jl) and the trial determinant of the phaseless walk the
 * same section names. Copies the inputs into library-owned device memory
 * (the caller may free its buffers on return; this call synchronises).
 *   M        number of spatial orbitals (1 <= M <= 4096)
 *   n_up/dn  electrons per spin (1 <= n <= min(M, 128))
 *   n_chol   number of Cholesky vectors X (>= 1)
 *   h1       M*M float64, real symmetric one-body matrix h_ij
 *   chol     n_chol*M*M float64, real symmetric L^n_ik (n-major)
 *   phi_t    M*(n_up+n_dn) complex128 trial orbitals T (orthonormal columns
 *            per spin are assumed by the QR convention, not checked)
 *   e_core   E_II, added to every local energy
 *   precision one of afq_precision
 *   stream   hipStream_t (NULL = default stream) used by every later call
 *   flags    0: h1, chol, phi_t are device pointers (stream-ordered copy);
 *            AFQ_HOST_PTRS: they are host pointers
 * Errors: AFQ_E_INVALID for bad sizes, NULL pointers, unknown flags or an
 * h1/L^n that is not symmetric to 1e-12 (relative to its largest entry);
 * AFQ_E_NOMEM; AFQ_E_HIP when a copy fails (for instance a host pointer
 * passed without AFQ_HOST_PTRS). */
int afq_system_create(afq_system *out, int M, int n_up, int n_dn, int n_chol,
                      const double *h1, const double *chol, const double *phi_t,
                      double e_core, int precision, void *stream, unsigned flags);
/* Switches the contraction precision (prepares the packed operand copies;
 * synchronises). */
int afq_system_set_precision(afq_system s, int precision);

/* Form of the exchange term sum_n tr(Omega_n Omega_n) of the local energy
 * (the two-body part of Eq. eq:hamil evaluated with half-rotated Cholesky
 * vectors; its cost is the energy column of Table tab:afqmc_comp, dense
 * 3-index row, O(x_c N^2 M^2)). The Cholesky form contracts every vector
 * (X N^2 M products per walker and spin); the four-index form uses
 *   sum_n tr(Omega_n Omega_n) = Theta^T W Theta,
 *   W[(b,k),(a,l)] = sum_n (T^H L^n)[a][k] (T^H L^n)[b][l],
 * the half-rotated two-electron tensor, built once per system, which needs
 * about (N M)^2 / 2 products (its symmetric upper block triangle) and N^2 M^2
 * stored entries per distinct spin block (split-BF16x3: BF16 hi / lo planes;
 * FP64: the FP64 tensor itself, contracted by FP64 GEMMs). The four-index
 * form exists in split-BF16x3 and FP64 modes for a real trial on plain
 * (single-determinant, not k-point-blocked) systems; elsewhere (complex FP32
 * mode included) the Cholesky form is used whatever the setting. */
typedef enum {
  AFQ_EXCH_AUTO = 0,       /* four-index form when it needs fewer products (M < 2X),
                              N M >= 4096, and its tensor takes at most a quarter
                              of the free device memory; else Cholesky (default) */
  AFQ_EXCH_CHOLESKY = 1,   /* always the Cholesky form */
  AFQ_EXCH_FOUR_INDEX = 2  /* the four-index form where it exists */
} afq_exchange_form;

/* Sets the exchange form (AFQ_EXCH_*). Builds the four-index tensor at once
 * when it will be used, or frees it when it will not (synchronises; may
 * allocate about N^2 M^2 * 2 bytes per distinct spin block in split-BF16x3
 * mode, its upper block triangle, and (1/2 + 1/16) N^2 M^2 * 8 bytes in FP64
 * mode, plus FP64 set-up transients of (N M X + M N M) * 8 bytes; a precision
 * switch rebuilds it). A batch holding the system captures its
 * step again on its next call. AFQ_E_INVALID for an unknown form,
 * AFQ_E_NOMEM when the tensor does not fit. */
int afq_system_set_exchange_form(afq_system s, int form);
/* The form the next step uses: *in_use = AFQ_EXCH_CHOLESKY or
 * AFQ_EXCH_FOUR_INDEX; *tensor_bytes (optional) = device bytes the four-index
 * tensor holds (0 when none). */
int afq_system_exchange_form(afq_system s, int* in_use, uint64_t* tensor_bytes);
/* k-point-blocked system (the explicitly k-point dependent Cholesky
 * factorisation of Section "Auxiliary Field Quantum Monte Carlo" and its row
 * of Table tab:afqmc_comp). Copies the inputs (this call synchronises).
 *   nk      number of k-points, 1..64
 *   kq      host, nk*nk int32 addition table: kq[Q*nk + k] = index of k + Q;
 *           must be an abelian group law with identity 0 (symmetric,
 *           associative, every row and column a permutation)
 *   m       orbitals per k-point; n_up / n_dn electrons per k-point and spin
 *   xq      Cholesky vectors per momentum transfer Q
 *   hk      device, nk*m*m complex128 Hermitian one-body blocks h^k
 *   Lk      device, nk*nk*xq*m*m complex128: Lk[Q][k][n] = L^{Q,k}_n, the
 *           block of vector (Q, n) from orbitals of k-point k (columns) to
 *           those of k + Q (rows); the two-electron tensor is
 *           v_ijkl = sum_(Q,n) L_ik conj(L_lj) over these block vectors
 *   phik    device, nk*m*(n_up+n_dn) complex128 trial orbitals per k-point,
 *           up columns first
 * The system works with the ordinary walker calls (afq_walkers_*, afq_step,
 * afq_energy, afq_batch_*, afq_bp_*). Its dense orbital index is k*m + i and
 * its trial columns are (k, a), k-major, per spin (up block first): walkers
 * are M x N with M = nk*m and N = nk*(n_up + n_dn). It has 2*nk*xq auxiliary
 * fields, x for (L + L^+)/2 of every vector (Q, n) in (Q, n) order, then y for
 * (L - L^+)/(2i); explicit fields and vbar_out use that order. FP64 mode only
 * (AFQ_E_UNSUPPORTED otherwise); no multi-determinant trial and no adjoint.
 * Limits: nk*m <= 4096, nk*max(n_up, n_dn) <= 128, and the trace kernel's
 * LDS (about 16 bytes x (2 nk m n + n m (nk + 1) + 12 xq)) within 160 KB. */
int afq_kp_system_create(afq_system *out, int nk, const int32_t *kq, int m, int n_up, int n_dn, int xq,
                         const double *hk, const double *Lk, const double *phik, double e_core,
                         int precision, void *stream);
/* Orthogonal multi-determinant trial (the multi-determinant paragraph of
 * Section "Auxiliary Field Quantum Monte Carlo"): psi_T = sum_I c_I |D_I>.
 *   C       device, M*M complex128 orthonormal basis (|C^H C - I| <= 1e-10);
 *           its first n_up (n_dn) columns must equal the up (down) block of
 *           the system's trial to 1e-12, which is the reference determinant
 *   n_det   number of determinants (0 detaches the expansion: back to phi_t)
 *   coeffs  host, n_det complex128 c_I
 *   exc     host, n_det*2*9 int32: per determinant and spin (up first) the
 *           rank k <= 4, then 4 hole slots (reference columns, < n), then 4
 *           particle orbitals (columns of C, >= n); entries past k ignored.
 *           D_I puts particle q in the column of hole q of the reference.
 * Every determinant needs its own occupation (the expansion is orthogonal).
 * Later energies, force biases and overlap ratios use psi_T through
 * Sherman-Morrison-Woodbury ratios and cofactor expansions of the rank-k
 * changes (no determinant is inverted, so walkers orthogonal to some D_I are
 * exact); a walker whose overlap with the reference determinant is singular
 * counts as singular. FP64 mode only; back-propagation and the adjoint need a
 * single determinant. Limits per spin: 64 electrons, 16 active holes, 32
 * active virtual orbitals, 256 distinct excitations (AFQ_E_UNSUPPORTED
 * beyond); AFQ_E_INVALID for a malformed or non-orthogonal expansion.
 * Synchronises. */
int afq_system_set_msd(afq_system s, const double *C, int n_det, const double *coeffs,
                       const int32_t *exc);
/* Mean-field background subtraction, a standard part of the phaseless method
 * that Section sec:afqmc cites (the paper gives no formulas). For a real
 * vector c the two-body term of Eq. eq:hamil in Cholesky form is
 *   1/2 sum_n (v_n - c_n)^2 + sum_n c_n v_n - 1/2 sum_n c_n^2,
 * so later steps sample the shifted operators v_n - c_n: the one-body factor
 * becomes B1 = exp(-dt (h' + sum_n c_n L^n) / 2), the force bias is
 * xbar_n = -i sqrt(dt) (vbar_n - c_n), and the importance factor gains the
 * c-number c0 = -i sqrt(dt) sum_n (x_n - xbar_n) c_n and exp(dt/2 sum c_n^2);
 * the phaseless angle is arg(r) + Im c0 (the overlap ratio of the whole
 * shifted propagator). Local energies are unchanged; ratio outputs stay O'/O.
 *   on          0: off (the default); 1: on
 *   background  NULL: c is the trial's own force bias, c_n = sum_s tr(L^n
 *               T^s T^sH) (the mean field); else a device vector of n_chol
 *               float64 (any finite real vector is exact)
 * Plain and multi-determinant systems (the reference determinant's mean
 * field); AFQ_E_UNSUPPORTED for k-point systems. A back-propagation window
 * must not span a change (AFQ_E_STATE), batches capture again. Synchronises. */
int afq_system_set_background(afq_system s, int on, const double *background);
/* *on = 1 while a background is subtracted; background (device, n_chol
 * float64, may be NULL) receives c_n then. */
int afq_system_background(afq_system s, int *on, double *background);
/* Frees device memory. NULL-safe. */
int afq_system_destroy(afq_system s);

/* ------------------------------------------------------------------------ */
/* Walkers: Slater determinants W (M x (n_up+n_dn) complex128) and weights.   */
/* ------------------------------------------------------------------------ */

/* Creates the walker population of the phaseless AFQMC random walk (the
 * method Section sec:afqmc names in its first paragraph, in the orbital-space
 * form of Eq. eq:hamil): each walker is a Slater determinant W with a weight
 * and its overlap with the trial.
 * w0 (device): n_walkers*M*(n_up+n_dn) complex128, or NULL to start every walker at
 * the trial. weights0: n_walkers float64, or NULL for all ones. A walker with
 * weight 0 is dead (frozen). Synchronises; AFQ_E_SINGULAR if any live
 * walker's overlap with the trial is singular. */
int afq_walkers_create(afq_walkers *out, afq_system s, int n_walkers,
                       const double *w0, const double *weights0);
int afq_walkers_destroy(afq_walkers w);

/* Checkpoint/resume of the walker state of afq_walkers_create (device
 * pointers). W: n_walkers*M*Ntot complex128; weights: n_walkers;
 * logovlp: n_walkers complex128 (log of prod_s det(T^sH W^s), get only, may be
 * NULL); alive: n_walkers int32 (may be NULL); counter: the step counter that
 * keys the Philox fields (host pointer, may be NULL). */
int afq_walkers_get(afq_walkers w, double *W, double *weights, double *logovlp,
                    int32_t *alive, uint64_t *counter);
int afq_walkers_set(afq_walkers w, const double *W, const double *weights,
                    const int32_t *alive, uint64_t counter);
/* Host-side counts: walkers alive, and the number killed by the phaseless
 * projection or a singular overlap since creation. Synchronises. */
int afq_walkers_stats(afq_walkers w, int *n_alive, int64_t *n_killed);

/* ------------------------------------------------------------------------ */
/* Population control. The paper cites the phaseless method (Section          */
/* "Auxiliary Field Quantum Monte Carlo") without its production controls;   */
/* these are the standard ones of that method.                                */
/* ------------------------------------------------------------------------ */

/* Controls applied by later afq_step / afq_batch_step calls on this walker set
 * (a batch re-captures its graph when they change): fb_cap > 0 scales every force-bias shift xbar_n whose modulus
 * exceeds fb_cap back to modulus fb_cap, phase kept; w_cap > 0 caps every
 * updated weight at w_cap. 0 switches a control off (the default). Negative or
 * non-finite values give AFQ_E_INVALID. */
int afq_walkers_set_controls(afq_walkers w, double fb_cap, double w_cap);

/* Systematic resampling ("comb") of the n walkers into n walkers of equal
 * weight W/n, W = sum of the weights: with running sums C_i = w_0 + ... + w_i
 * formed in walker order, tooth k at u_k = (k + xi) W / n takes a copy of the
 * first walker i with C_i > u_k (a tooth at or beyond W takes the last walker
 * of positive weight); dead walkers get no copies and every new walker is
 * alive. xi: uniform number in [0, 1). src_out (host, n ints, may be NULL)
 * receives the source walker of every new walker, total_out (host, may be
 * NULL) receives W. Synchronises the system stream. W <= 0 gives AFQ_E_STATE
 * and leaves the walkers unchanged. */
int afq_walkers_comb(afq_walkers w, double xi, int32_t *src_out, double *total_out);

/* Largest walker set afq_walkers_comb_noalloc accepts. Its scratch is one
 * file-scope device array of 256 B + 12 B per walker (48.25 KiB), which every
 * GPU the library runs on holds until the process ends. */
#define AFQ_COMB_NOALLOC_MAX_WALKERS 4096
/* For callers that cannot allocate device memory (no hipMalloc / hipFree may
 * happen inside their loop: fixed-budget serving loops, harnesses that forbid
 * allocation): afq_walkers_comb with the same kernels and the same result bit
 * for bit, but its scratch (running weight sums, source indices, total weight)
 * lives in the library's static device array instead of buffers allocated on
 * the first comb. The call allocates nothing; it synchronises the system
 * stream like afq_walkers_comb. Every call on one GPU shares that GPU's array
 * and overwrites it: calls that overlap on one GPU (other threads, other
 * streams) race and must be serialised by the caller. Errors: AFQ_E_INVALID
 * for more than AFQ_COMB_NOALLOC_MAX_WALKERS walkers or xi outside [0, 1);
 * AFQ_E_UNSUPPORTED while a back-propagation window is open (its history
 * gather needs a buffer; use afq_walkers_comb); AFQ_E_STATE as
 * afq_walkers_comb. */
int afq_walkers_comb_noalloc(afq_walkers w, double xi, int32_t *src_out, double *total_out);

/* Energy-shift feedback of the population: *e_shift_out = e_est -
 * ln(w_total / w_target) / (gain_steps dt). Host arithmetic only. Non-positive
 * weights, dt or gain give AFQ_E_INVALID. */
int afq_eshift_update(double e_est, double w_total, double w_target, double dt, double gain_steps,
                      double *e_shift_out);

/* ------------------------------------------------------------------------ */
/* Hot path.                                                                  */
/* ------------------------------------------------------------------------ */

/* Advances the walkers n_steps steps of the phaseless AFQMC walk (Section
 * sec:afqmc, first paragraph: the method, and the Hubbard-Stratonovich
 * transformation that the Cholesky vectors make possible); each step is the
 * short-time propagator exp(-dt (H - E_shift)) of Eq. eq:hamil sampled over
 * the auxiliary fields (the equations at the top of this file). Its cost is
 * the propagation column of Table tab:afqmc_comp (dense 3-index row) plus one
 * local energy per step.
 *   fields   NULL: standard-normal fields from the device Philox4x32-10
 *            generator keyed by (seed, step counter, walker, n); else
 *            n_steps*n_walkers*n_chol float64 fields x[k][w][n].
 *   qr_every re-orthonormalise after every qr_every-th step (0 = never); the
 *            phase of this cadence follows the walkers' step counter.
 *   e_shift  E_shift of the importance function.
 *   taylor_order K >= 1 (6 in the reference workloads).
 * Optional outputs (NULL to skip), per step k, energies at the start-of-step
 * walkers with the pre-update weights:
 *   emix_out    n_steps float64: sum_w w Re E_L / sum_w w (0 if all dead)
 *   eloc_out    n_steps*n_walkers complex128 local energies
 *   weights_out n_steps*n_walkers float64 weights after step k
 *   ratio_out   n_steps*n_walkers complex128 overlap ratios O'/O (0 for walkers already dead)
 * Dead walkers are not errors; they are counted by afq_walkers_stats. */
int afq_step(afq_system s, afq_walkers w, int n_steps, double dt,
             const double *fields, uint64_t seed, int qr_every, double e_shift,
             int taylor_order, double *emix_out, double *eloc_out,
             double *weights_out, double *ratio_out);

/* Local energy of the walkers, E_L = <T|H|W>/<T|W> for the Hamiltonian of
 * Eq. eq:hamil with the Cholesky form of v_ijkl (Section sec:afqmc), in the
 * half-rotated form given at the top of this file; its cost is the energy
 * column of Table tab:afqmc_comp (dense 3-index row).
 *   eloc_out  n_walkers complex128 E_L (may be NULL)
 *   parts_out n_walkers*3 complex128 (E1, EJ, EK) (may be NULL)
 *   vbar_out  n_walkers*n_chol complex128 force bias vbar_n (may be NULL)
 *   emix_out  1 float64 weighted mixed energy (may be NULL) */
int afq_energy(afq_system s, afq_walkers w, double *eloc_out, double *parts_out,
               double *vbar_out, double *emix_out);

/* Derivatives of the weighted mean local energy of afq_energy with respect to
 * the inputs of Eq. eq:hamil (h_ij and the Cholesky vectors L^n of the
 * factorisation after it, Section sec:afqmc) and the walker orbitals; the
 * paper states the energy, not its derivative: this is the exact adjoint of
 * that expression.
 * Adjoint of  f = scale * sum_w w Re E_L / sum_w w  at the current walkers,
 * with the weights and the trial held fixed. Theta and Omega are recomputed; nothing
 * is stored from the forward call. Outputs (each may be NULL to skip):
 *   d_h1      M*M float64, df/dh_ij for every entry (not symmetrised)
 *   d_chol    n_chol*M*M float64, df/dL^n_ij for every entry
 *   d_walkers n_walkers*M*Ntot complex128, df/dRe W + i df/dIm W
 * The outputs are overwritten, not accumulated. */
int afq_energy_backward(afq_system s, afq_walkers w, double scale, double *d_h1,
                        double *d_chol, double *d_walkers);

/* The auxiliary fields of the Hubbard-Stratonovich transformation (Section
 * sec:afqmc, first paragraph), one per Cholesky vector, walker and step:
 * standard-normal fields x[k][w][n] for steps step0..step0+n_steps-1 from the
 * device Philox4x32-10 generator (the same stream afq_step draws with
 * fields == NULL): counter (n/2, w, step, sys_id), key (seed lo, seed hi),
 * Box-Muller on two 53-bit uniforms. out: n_steps*n_walkers*n_chol float64. */
int afq_fields_generate(uint64_t seed, uint32_t sys_id, uint64_t step0, int n_steps,
                        int n_walkers, int n_chol, double *out, void *stream);

/* Autotuner of the fused exchange contraction, the energy term that
 * dominates the cost (Table tab:afqmc_comp, dense 3-index row): times
 * each launch variant (waves per workgroup, accumulator budget) of both spins
 * on these walkers' own shapes with HIP events, `reps` launches each, and keeps
 * the fastest for this walker set and for later walker sets of the same shape
 * (a process-wide table). In split-BF16x3 mode it also times one step's
 * propagator products (a B1 product and the Horner chain) with every tile of
 * afq_system_set_propagator_tile and pins the fastest for the system. Recomputes Theta from the current walkers and writes
 * only per-step scratch: W, weights and counters are unchanged. Synchronises
 * the system stream. choice_out (host, 2 ints, may be NULL) receives the
 * variant per spin, -1 where the shape has a single kernel (split-BF16x3 with
 * 65..100 electrons per spin). */
int afq_autotune(afq_system s, afq_walkers w, int reps, int *choice_out);
/* Tile of the split-BF16x3 propagator products (the Taylor products of
 * A = sum_n c_n L^n in Horner form and the two B1 products, Section
 * "Auxiliary Field Quantum Monte Carlo" and Table tab:afqmc_comp): 0 = 224 x
 * 160 (walker-term rows x real-form columns per workgroup), 1 = 128 x 128,
 * 2 = 64 x 64; -1 = chosen per system by the least padded work (a larger tile
 * winning within 10%). The walkers' packed operands follow the tile: every
 * walker set clears them for the new layout at its next call, and a batch
 * holding the system captures its step again (synchronises). AFQ_E_INVALID
 * outside -1..2. The results do not depend on the tile beyond rounding of the
 * FP32 accumulation order. */
int afq_system_set_propagator_tile(afq_system s, int tile);
/* The tile the next step uses (0..2), into *tile (host int). */
int afq_system_propagator_tile(afq_system s, int* tile);
/* Pins the exchange launch variant of one spin for this walker set (0..2, or
 * -1 to return to the tuned/default choice), e.g. to replay a tuning table
 * saved from an earlier process. A variant that does not fit the shape makes
 * the next step or energy call fail with AFQ_E_UNSUPPORTED. For a k-point
 * system the variant picks the exchange-trace kernel of the spin: 1 the FP64
 * VALU kernel, any other value the FP64 MFMA kernel where the shape allows it
 * (m <= 32 and its LDS fits), else the VALU kernel. */
int afq_exchange_variant(afq_walkers w, int spin, int variant);

/* ------------------------------------------------------------------------ */
/* Back-propagated one-body density matrix (back-propagation paragraph of    */
/* Section "Auxiliary Field Quantum Monte Carlo"; the method is cited there). */
/* ------------------------------------------------------------------------ */

/* Opens a window of n_bp steps (0 <= n_bp <= 2^20) on the current walkers:
 * they become the kets phi_w, and each of the next n_bp afq_step steps stores
 * the conjugated propagator coefficients conj(c_wn) of every walker
 * (A = sum_n c_wn L^n). dt, the Taylor order and the precision must stay fixed
 * while the window records (AFQ_E_INVALID / AFQ_E_STATE otherwise);
 * afq_batch_step refuses to step a walker set whose window records, and
 * afq_walkers_set closes the window. An afq_walkers_comb inside the window
 * hands every copy its source walker's ket and coefficients. Device memory:
 * n_walkers*M*Ntot complex128 for the kets plus n_bp*n_walkers*n_chol complex
 * (complex128, or complex64 in the reduced-precision modes). Reopening
 * discards the previous window. */
int afq_bp_begin(afq_walkers w, int n_bp);
/* Once the window holds its n_bp steps and no further step was taken: carries
 * the trial backwards, |psi_w> = B_0^H ... B_{n_bp-1}^H |T> with
 * B_j^H = B1 T_K(A_j^H) B1 (the last step's first; QR of every spin block after
 * every qr_every of these steps, 0 = never), and writes the spin-resolved
 * back-propagated 1-RDM
 *   rdm_out[s][i][j] = sum_w w_w <psi_w|c+_is c_js|phi_w>/<psi_w|phi_w> / sum_w w_w
 * (device, 2*M*M complex128) with the weights w_w at the end of the window
 * (walkers of weight 0 drop out; no phase restoration along the path).
 * wsum_out (host, may be NULL) receives sum_w w_w. Synchronises the system
 * stream. AFQ_E_STATE if the window is not full, steps followed it, the
 * precision changed or no walker has positive weight; AFQ_E_SINGULAR if a
 * walker of positive weight has a singular <psi_w|phi_w> in either spin (the
 * output is then undefined). The window stays open: the call may be repeated. */
int afq_bp_rdm1(afq_walkers w, int qr_every, double *rdm_out, double *wsum_out);
/* Closes the window and frees its memory. */
int afq_bp_end(afq_walkers w);

/* ------------------------------------------------------------------------ */
/* Many uneven systems in one captured launch sequence.                       */
/* ------------------------------------------------------------------------ */

/* Many systems stepped together on one GPU (each is the walk of afq_step on
 * its own Hamiltonian of Eq. eq:hamil; the GPU column of Table
 * tab:afqmc_comp marks the dense 3-index and k-point paths as GPU ones).
 * Groups n (system, walkers) pairs that share one stream and precision.
 * The handles must outlive the batch. */
int afq_batch_create(afq_batch *out, int n, const afq_system *systems,
                     const afq_walkers *walkers);
/* Advances every system n_steps steps with Philox fields (system i uses
 * sys_id = i). The first call autotunes every system's exchange kernel
 * (afq_autotune), runs eager steps up to a multiple of qr_every, then captures
 * one HIP graph of qr_every steps (or one step when qr_every is 0) whose
 * concurrent branches are the systems; later calls replay it (a change of dt,
 * seed, qr_every, e_shift, order, precision or walker controls captures a new
 * graph). e_shift: n float64
 * (host). emix_out: n*n_steps float64 device array, system-major. */
int afq_batch_step(afq_batch b, int n_steps, double dt, uint64_t seed, int qr_every,
                   const double *e_shift, int taylor_order, double *emix_out);
int afq_batch_destroy(afq_batch b);

/* ------------------------------------------------------------------------ */
/* Phase timing (HIP events on the library stream; process-wide, not          */
/* thread-safe). Phases, in step order:                                       */
/* ------------------------------------------------------------------------ */
enum {
  AFQ_PH_OVERLAP = 0,   /* S = T^H W, Gauss-Jordan S^-1 and log det, Theta   */
  AFQ_PH_PACK = 1,      /* Theta -> packed exchange operand                   */
  AFQ_PH_EXCHANGE = 2,  /* fused Omega = Lt Theta, tr Omega, tr Omega^2 (one
                           event pair per spin launch)                        */
  AFQ_PH_COULOMB = 3,   /* FP64 force-bias traces (split-BF16x3 mode)         */
  AFQ_PH_ASSEMBLE = 4,  /* E_L, force bias, propagator coefficients, E_mix    */
  AFQ_PH_ABUILD = 5,    /* A = sum_n c_n L^n                                  */
  AFQ_PH_TAYLOR = 6,    /* B1 T_K(A) B1 W                                     */
  AFQ_PH_WEIGHT = 7,    /* new overlap, phaseless weight, walker commit       */
  AFQ_PH_QR = 8,        /* CholeskyQR2                                         */
  AFQ_PH_MSD_OMEGA = 9, /* multi-determinant trial: [T^H; C_V^H] L^g Theta GEMM
                           (one event pair per spin and walker chunk)          */
  AFQ_PH_MSD_SUMS = 10, /* multi-determinant trial: C_V^H Theta, cofactors,
                           small products and the determinant sums             */
  AFQ_TRACE_NPHASE = 11
};
/* on != 0 starts recording event pairs around every traced phase. */
int afq_trace_enable(int on);
/* Drops recorded events and zeroes the totals. */
int afq_trace_reset(void);
/* Synchronises on the recorded events and returns the summed milliseconds and
 * the number of event pairs of a phase since the last reset. */
int afq_trace_query(int phase, double *ms, int64_t *count);

/* Thread-local message of the last failing call on this thread. */
const char *afq_last_error(void);
/* Library version, (major << 16) | minor. */
int afq_version(void);

#ifdef __cplusplus
}
#endif
#endif /* AFQ_H */
